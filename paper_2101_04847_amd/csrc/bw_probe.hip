// Achievable HBM bandwidth on the current GPU: plain streaming kernels
// (copy = read + write, read-only, write-only) over caller buffers.  The
// measured denominator next to the published HBM peak; not part of the
// lattice Boltzmann library.
//
// Built as libbwprobe.so (C entry points, used in-process by the benchmark on
// the benchmark's own stream and buffers) and as the stand-alone program
// bw_probe (allocates its own buffers):
//
//     bw_probe [gigabytes=7.2]
//
// Copy variants:
//   0  grid-stride loop, 16 B per lane, 4 loads in flight per lane,
//      non-temporal stores;
//   1  each workgroup streams one contiguous chunk, 16 B per lane, 8 loads
//      in flight per lane, non-temporal stores;
//   2  as 1 with ordinary stores;
//   3  as 1 with buffer loads and stores through 128-bit resources (the
//      access form of the step kernels), non-temporal stores.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef unsigned uvec4 __attribute__((ext_vector_type(4)));

namespace {

template <int U>
__global__ void __launch_bounds__(256) copy_stride(const dvec2 *__restrict__ a, dvec2 *__restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = blockIdx.x * (size_t)blockDim.x + threadIdx.x; base < n; base += stride * U) {
        dvec2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + u * stride;
            if (i < n) v[u] = a[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + u * stride;
            if (i < n) __builtin_nontemporal_store(v[u], b + i);
        }
    }
}

// Workgroup k copies elements [k * chunk, (k + 1) * chunk): U passes of 256
// lanes x 16 B in flight at a time.
template <int U, bool NT>
__global__ void __launch_bounds__(256) copy_chunk(const dvec2 *__restrict__ a, dvec2 *__restrict__ b, size_t n,
                                                  size_t chunk)
{
    for (size_t c0 = (size_t)blockIdx.x * chunk; c0 < n; c0 += (size_t)gridDim.x * chunk) {
        const size_t c1 = c0 + chunk < n ? c0 + chunk : n;
        for (size_t base = c0 + threadIdx.x; base < c1; base += 256 * U) {
            dvec2 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t i = base + (size_t)u * 256;
                if (i < c1) v[u] = a[i];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t i = base + (size_t)u * 256;
                if (i < c1) {
                    if (NT) __builtin_nontemporal_store(v[u], b + i);
                    else b[i] = v[u];
                }
            }
        }
    }
}

constexpr int BUF_RAW_DWORD3 = 0x00020000;
constexpr int CPOL_NT = 2;

// As copy_chunk<8, true> through buffer resources of one chunk each
// (chunk * 16 B must stay below 2^31).
__global__ void __launch_bounds__(256) copy_chunk_buf(const dvec2 *__restrict__ a, dvec2 *__restrict__ b, size_t n,
                                                      size_t chunk)
{
    constexpr int U = 8;
    for (size_t c0 = (size_t)blockIdx.x * chunk; c0 < n; c0 += (size_t)gridDim.x * chunk) {
        const size_t len = (c0 + chunk < n ? chunk : n - c0) * sizeof(dvec2);
        const auto ra = __builtin_amdgcn_make_buffer_rsrc((void *)(a + c0), 0, (int)len, BUF_RAW_DWORD3);
        const auto rb = __builtin_amdgcn_make_buffer_rsrc((void *)(b + c0), 0, (int)len, BUF_RAW_DWORD3);
        for (unsigned off = threadIdx.x * 16u; off < len; off += 256u * 16u * U) {
            uvec4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = __builtin_amdgcn_raw_buffer_load_b128(ra, off + u * 4096u, 0, 0);
#pragma unroll
            for (int u = 0; u < U; ++u) __builtin_amdgcn_raw_buffer_store_b128(v[u], rb, off + u * 4096u, 0, CPOL_NT);
        }
    }
}

__global__ void __launch_bounds__(256) read_u(const dvec2 *__restrict__ a, double *__restrict__ out, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    double s = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        const dvec2 v = a[i];
        s += v.x + v.y;
    }
    if (s == 1234.5678) out[0] = s;   // keeps the loads; never true for zeroed input
}

__global__ void __launch_bounds__(256) fill(dvec2 *__restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const dvec2 w = {1.0, 2.0};
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) __builtin_nontemporal_store(w, b + i);
}

}  // namespace

extern "C" {

// Number of copy variants.
int bw_copy_variants(void) { return 4; }

// Enqueue one copy of `bytes` (a multiple of 16) from a to b (device, 16-byte
// aligned) on stream with the given variant and grid (workgroups of 256).
// Returns 0, or -1 for invalid arguments, -2 if the launch failed.
int bw_copy(const void *a, void *b, size_t bytes, int variant, int grid, void *stream)
{
    if (!a || !b || bytes % 16 || grid < 1 || ((uintptr_t)a | (uintptr_t)b) % 16) return -1;
    const size_t n = bytes / 16;
    const size_t chunk = (n + grid - 1) / grid;
    hipStream_t s = (hipStream_t)stream;
    const dvec2 *src = (const dvec2 *)a;
    dvec2 *dst = (dvec2 *)b;
    switch (variant) {
        case 0: hipLaunchKernelGGL(copy_stride<4>, dim3(grid), dim3(256), 0, s, src, dst, n); break;
        case 1: hipLaunchKernelGGL((copy_chunk<8, true>), dim3(grid), dim3(256), 0, s, src, dst, n, chunk); break;
        case 2: hipLaunchKernelGGL((copy_chunk<8, false>), dim3(grid), dim3(256), 0, s, src, dst, n, chunk); break;
        case 3:
            if (chunk * 16 >= ((size_t)1 << 31)) return -1;
            hipLaunchKernelGGL(copy_chunk_buf, dim3(grid), dim3(256), 0, s, src, dst, n, chunk);
            break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"

#ifdef BW_PROBE_MAIN
#define CHECK(x)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));          \
            return 1;                                                                     \
        }                                                                                 \
    } while (0)

int main(int argc, char **argv)
{
    const double gb = argc > 1 ? std::atof(argv[1]) : 7.2;
    const size_t n = (size_t)(gb * 1e9 / sizeof(dvec2));
    dvec2 *a = nullptr, *b = nullptr;
    double *o = nullptr;
    CHECK(hipMalloc(&a, n * sizeof(dvec2)));
    CHECK(hipMalloc(&b, n * sizeof(dvec2)));
    CHECK(hipMalloc(&o, 64));
    CHECK(hipMemset(a, 0, n * sizeof(dvec2)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    auto timed = [&](auto &&run, double bytes, const char *name, int grid) -> double {
        run();
        if (hipDeviceSynchronize() != hipSuccess) return -1.0;
        (void)hipEventRecord(e0);
        for (int r = 0; r < 10; ++r) run();
        (void)hipEventRecord(e1);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= 10;
        const double gbs = bytes / ms / 1e6;
        std::printf("%-10s grid=%-6d buffer %.2f GB: %.3f ms  %.1f GB/s\n", name, grid, gb, ms, gbs);
        return gbs;
    };
    double best_copy = 0, best_read = 0, best_fill = 0;
    const char *vname[] = {"copy-v0", "copy-v1", "copy-v2", "copy-v3"};
    for (int v = 0; v < bw_copy_variants(); ++v)
        for (int grid : {2048, 8192, 32768, 65536}) {
            const double g = timed([&]() { bw_copy(a, b, n * sizeof(dvec2), v, grid, nullptr); },
                                   2.0 * n * sizeof(dvec2), vname[v], grid);
            if (g > best_copy) best_copy = g;
        }
    for (int grid : {2048, 8192, 32768, 65536}) {
        const double r = timed([&]() { read_u<<<grid, 256>>>(a, o, n); }, 1.0 * n * sizeof(dvec2), "read", grid);
        const double f = timed([&]() { fill<<<grid, 256>>>(b, n); }, 1.0 * n * sizeof(dvec2), "fill", grid);
        if (r > best_read) best_read = r;
        if (f > best_fill) best_fill = f;
    }
    CHECK(hipGetLastError());
    std::printf("best GB/s: copy %.1f read %.1f fill %.1f\n", best_copy, best_read, best_fill);
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    CHECK(hipFree(o));
    return 0;
}
#endif
