// gfx950 kernels of the three-dimensional (D3Q19) two-component Shan-Chen
// step: the method of Sec. 2 (Eq. 1-7) with the D2Q9 set replaced by D3Q19.
//
// Storage: two buffers of row blocks [z][y][s][i][pitch] (the 38 row
// segments of one lattice row adjacent, x fastest) holding post-collision
// populations; f(t) is pulled: f_i(x) = f*_i(x - c_i), or f*_opp(i)(x) where
// x - c_i lies beyond a y wall.  Two ways to run a step, both HBM-bound:
//   k3_fused     one pass (the default): a block owns a tile of the x-y plane
//                and marches through a band of planes in z, keeping the
//                densities of four planes in an LDS ring and the pulled
//                populations of two planes in registers, so each population
//                crosses HBM about once per read and once per write;
//   k3_density + k3_collide
//                two passes with one thread per site: the densities go to a
//                [z][y][2][pitch] FP64 buffer, then the populations are pulled
//                again, the 18 neighbour densities of the other component read
//                (cache-resident: 16 B per site), and the Shan-Chen + body
//                acceleration, the 1/tau-weighted velocity, the shifted
//                equilibrium and the BGK relaxation applied; with FIELDS
//                k3_collide writes rho_A, rho_B and the hydrodynamic velocity
//                instead (the field pass).
// All arithmetic is FP64 in both storage modes, every expression in the
// order of its definition (sums over i in index order, no contraction), so
// the FP64 mode is reproducible bit for bit by a plain implementation.
#pragma once

#include "lb_memory.hpp"

namespace lbk3 {

using lbk::bload;
using lbk::bstore;
using lbk::row_rsrc;
using lbk::rsrc_t;
using lbk::Tr;

constexpr int NQ3 = 19;

// D3Q19: 0 rest; 1..6 axis links +x -x +y -y +z -z; 7..18 edge links in
// reversed pairs (+x+y, -x-y), (+x-y, -x+y), (+x+z, -x-z), (+x-z, -x+z),
// (+y+z, -y-z), (+y-z, -y+z).  Weights from the isotropy conditions of Eq. 4.
__host__ __device__ constexpr int c3x(int i)
{
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1 : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int c3y(int i)
{
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1 : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int c3z(int i)
{
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1 : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
__host__ __device__ constexpr int opp3(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double w3(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

static_assert(c3x(opp3(13)) == -1 && c3z(opp3(13)) == 1, "edge opposites");
static_assert(c3y(opp3(17)) == -1 && c3z(opp3(17)) == 1, "edge opposites");

// One lattice as the kernels see it (passed by value).
struct Lat3 {
    int32_t nx, ny, nz, pitch;   // pitch: elements per row segment (nx rounded up to 64)
    int64_t rstride;             // elements per population row block (2 * 19 * pitch)
    void *f[2];                  // ping-pong population buffers
    double *rho;                 // [nz][ny][2][pitch] densities of the current pull
    double tau[2], itau[2];      // relaxation times and their reciprocals
    double G;                    // Shan-Chen coupling
    double g[2][3];              // body acceleration per component
};

struct Fields3 {
    double *rhoA, *rhoB, *ux, *uy, *uz;   // [nz][ny][nx], any may be null
};

// Column offset of a lane that pulls nothing: beyond every row's extent, so
// its buffer loads return zero without a memory access.
constexpr unsigned NO_COLUMN = 0x80000000u;

// Pull the 38 populations of site (x, y, z) from the post-collision buffer.
// The values land in f as V: the storage type itself (kept in registers by
// the fused pass) or double (converted on load; the conversion is exact).
// A lane with live false loads nothing and gets zeros.
template <int ST, int BCY, class V>
__device__ __forceinline__ void pull3(const void *src, const Lat3 &L, int z, int y, int x, V (&f)[2][NQ3],
                                      bool live = true)
{
    using T = typename Tr<ST>::T;
    const int64_t row_bytes = L.rstride * (int64_t)sizeof(T);
    const unsigned is = (unsigned)L.pitch * (unsigned)sizeof(T);
    const unsigned ss = (unsigned)NQ3 * is;
    const unsigned oc = live ? (unsigned)x * (unsigned)sizeof(T) : NO_COLUMN;
    const unsigned om = live ? (unsigned)(x == 0 ? L.nx - 1 : x - 1) * (unsigned)sizeof(T) : NO_COLUMN;   // c_x = +1
    const unsigned op = live ? (unsigned)(x == L.nx - 1 ? 0 : x + 1) * (unsigned)sizeof(T) : NO_COLUMN;   // c_x = -1
#pragma unroll
    for (int i = 0; i < NQ3; ++i) {
        int ys = y - c3y(i), zs = z - c3z(i);
        unsigned col = c3x(i) > 0 ? om : (c3x(i) < 0 ? op : oc);
        int seg = i;
        if (BCY == lbk::BC_PERIODIC) {
            if (ys < 0) ys += L.ny;
            if (ys >= L.ny) ys -= L.ny;
        } else if (ys < 0 || ys >= L.ny) {
            // halfway bounce-back: the reversed population of the site itself
            ys = y;
            zs = z;
            col = oc;
            seg = opp3(i);
        }
        if (zs < 0) zs += L.nz;
        if (zs >= L.nz) zs -= L.nz;
        const rsrc_t r = row_rsrc(src, zs * L.ny + ys, row_bytes);
#pragma unroll
        for (int s = 0; s < 2; ++s)
            f[s][i] = (V)bload<T>(r, col, (unsigned)s * ss + (unsigned)seg * is);
    }
}

// Eq. 1: rho_s = sum_i f_i in index order.
template <class V>
__device__ __forceinline__ double density3(const V (&f)[NQ3])
{
    double r = (double)f[0];
#pragma unroll
    for (int i = 1; i < NQ3; ++i) r += (double)f[i];
    return r;
}

// j_s = sum_i f_i c_i in index order (terms with a zero component add nothing).
template <class V>
__device__ __forceinline__ void momentum3(const V (&f)[NQ3], double &jx, double &jy, double &jz)
{
    double mx = 0.0, my = 0.0, mz = 0.0;
    bool fx = true, fy = true, fz = true;
#pragma unroll
    for (int i = 1; i < NQ3; ++i) {
        if (c3x(i) != 0) {
            mx = fx ? (c3x(i) > 0 ? (double)f[i] : -(double)f[i]) : (c3x(i) > 0 ? mx + (double)f[i] : mx - (double)f[i]);
            fx = false;
        }
        if (c3y(i) != 0) {
            my = fy ? (c3y(i) > 0 ? (double)f[i] : -(double)f[i]) : (c3y(i) > 0 ? my + (double)f[i] : my - (double)f[i]);
            fy = false;
        }
        if (c3z(i) != 0) {
            mz = fz ? (c3z(i) > 0 ? (double)f[i] : -(double)f[i]) : (c3z(i) > 0 ? mz + (double)f[i] : mz - (double)f[i]);
            fz = false;
        }
    }
    jx = mx;
    jy = my;
    jz = mz;
}

// Density of component s at the neighbour x + c_i: x and z wrap; y wraps
// (periodic) or, beyond a wall, takes the wall row (mirror).
template <int BCY>
__device__ __forceinline__ double rho_nb(const Lat3 &L, int z, int y, int x, int s, int i)
{
    int xn = x + c3x(i), yn = y + c3y(i), zn = z + c3z(i);
    if (xn < 0) xn += L.nx;
    if (xn >= L.nx) xn -= L.nx;
    if (zn < 0) zn += L.nz;
    if (zn >= L.nz) zn -= L.nz;
    if (BCY == lbk::BC_PERIODIC) {
        if (yn < 0) yn += L.ny;
        if (yn >= L.ny) yn -= L.ny;
    } else {
        if (yn < 0) yn = 0;
        if (yn >= L.ny) yn = L.ny - 1;
    }
    return L.rho[((int64_t)(zn * L.ny + yn) * 2 + s) * L.pitch + xn];
}

// Eq. 5 sum S = sum_i w_i rho(x + c_i) c_i of one component, in index order
// (each component sums only the links with a nonzero entry); nb(i) is the
// component's density at x + c_i.
template <class NB>
__device__ __forceinline__ void sc_sum3_nb(NB &&nb, double (&S)[3])
{
    double sx = 0.0, sy = 0.0, sz = 0.0;
    bool fx = true, fy = true, fz = true;
#pragma unroll
    for (int i = 1; i < NQ3; ++i) {
        const double wp = w3(i) * nb(i);
        if (c3x(i) != 0) {
            sx = fx ? (c3x(i) > 0 ? wp : -wp) : (c3x(i) > 0 ? sx + wp : sx - wp);
            fx = false;
        }
        if (c3y(i) != 0) {
            sy = fy ? (c3y(i) > 0 ? wp : -wp) : (c3y(i) > 0 ? sy + wp : sy - wp);
            fy = false;
        }
        if (c3z(i) != 0) {
            sz = fz ? (c3z(i) > 0 ? wp : -wp) : (c3z(i) > 0 ? sz + wp : sz - wp);
            fz = false;
        }
    }
    S[0] = sx;
    S[1] = sy;
    S[2] = sz;
}

// Shan-Chen + body acceleration a_s = -G S_sbar + g_s (Eq. 5 with psi = rho,
// plus Eq. 7) of both components from the sums S[s] of each component.
__device__ __forceinline__ void accel3(const Lat3 &L, const double (&S)[2][3], double (&a)[2][3])
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int d = 0; d < 3; ++d) a[s][d] = -L.G * S[1 - s][d] + L.g[s][d];
}

// Collision of one site (Eq. 1-3 and the BGK relaxation of Eq. 2, velocity
// shift) and the store of f*(t) at the site into buffer cur ^ 1.
template <int ST, class V>
__device__ __forceinline__ void collide_store3(const Lat3 &L, const V (&f)[2][NQ3], const double (&rho)[2],
                                               const double (&a)[2][3], int cur, int z, int y, int x)
{
    using T = typename Tr<ST>::T;
    double j[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s) momentum3(f[s], j[s][0], j[s][1], j[s][2]);
    // Eq. 1: velocity weighted by 1/tau_s
    const double den = rho[0] * L.itau[0] + rho[1] * L.itau[1];
    const double ux = (j[0][0] * L.itau[0] + j[1][0] * L.itau[1]) / den;
    const double uy = (j[0][1] * L.itau[0] + j[1][1] * L.itau[1]) / den;
    const double uz = (j[0][2] * L.itau[0] + j[1][2] * L.itau[1]) / den;
    const rsrc_t wr = row_rsrc(L.f[cur ^ 1], z * L.ny + y, L.rstride * (int64_t)sizeof(T));
    const unsigned ox = (unsigned)x * (unsigned)sizeof(T);
    const unsigned is = (unsigned)L.pitch * (unsigned)sizeof(T);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        // Eq. 3 at the shifted velocity u + tau_s a_s
        const double vx = ux + L.tau[s] * a[s][0];
        const double vy = uy + L.tau[s] * a[s][1];
        const double vz = uz + L.tau[s] * a[s][2];
        const double vv = vx * vx + vy * vy + vz * vz;
        const double om = L.itau[s];
#pragma unroll
        for (int i = 0; i < NQ3; ++i) {
            // c_i . v, summed over the nonzero components in the order x, y, z
            double cv = 0.0;
            bool first = true;
            if (c3x(i) != 0) {
                cv = c3x(i) > 0 ? vx : -vx;
                first = false;
            }
            if (c3y(i) != 0) {
                cv = first ? (c3y(i) > 0 ? vy : -vy) : (c3y(i) > 0 ? cv + vy : cv - vy);
                first = false;
            }
            if (c3z(i) != 0) cv = first ? (c3z(i) > 0 ? vz : -vz) : (c3z(i) > 0 ? cv + vz : cv - vz);
            const double feq = rho[s] * w3(i) * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
            const double fi = (double)f[s][i];
            const double post = fi - om * (fi - feq);   // Eq. 2
            bstore<LBK_NT_STORE ? lbk::CPOL_NT : 0>((T)post, wr, ox, (unsigned)(s * NQ3 + i) * is);
        }
    }
}

constexpr int WX = 64, WY = 4;   // threads per block: one wave per row segment, four rows

template <int ST, int BCY>
__global__ void __launch_bounds__(WX * WY) k3_density(Lat3 L, int cur)
{
    const int x = blockIdx.x * WX + threadIdx.x;
    const int y = blockIdx.y * WY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= L.nx || y >= L.ny) return;
    double f[2][NQ3];
    pull3<ST, BCY>(L.f[cur], L, z, y, x, f);
    const int64_t base = (int64_t)(z * L.ny + y) * 2 * L.pitch + x;
    L.rho[base] = density3(f[0]);
    L.rho[base + L.pitch] = density3(f[1]);
}

template <int ST, int BCY, bool FIELDS>
__global__ void __launch_bounds__(WX * WY) k3_collide(Lat3 L, int cur, Fields3 fo)
{
    const int x = blockIdx.x * WX + threadIdx.x;
    const int y = blockIdx.y * WY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= L.nx || y >= L.ny) return;
    double f[2][NQ3];
    pull3<ST, BCY>(L.f[cur], L, z, y, x, f);
    double rho[2], S[2][3], a[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        rho[s] = density3(f[s]);
        sc_sum3_nb([&](int i) { return rho_nb<BCY>(L, z, y, x, s, i); }, S[s]);
    }
    accel3(L, S, a);
    if constexpr (FIELDS) {
        double j[2][3];
#pragma unroll
        for (int s = 0; s < 2; ++s) momentum3(f[s], j[s][0], j[s][1], j[s][2]);
        const double Fx = rho[0] * a[0][0] + rho[1] * a[1][0];
        const double Fy = rho[0] * a[0][1] + rho[1] * a[1][1];
        const double Fz = rho[0] * a[0][2] + rho[1] * a[1][2];
        const double rt = rho[0] + rho[1];
        const int64_t k = ((int64_t)z * L.ny + y) * L.nx + x;
        if (fo.rhoA) fo.rhoA[k] = rho[0];
        if (fo.rhoB) fo.rhoB[k] = rho[1];
        if (fo.ux) fo.ux[k] = (j[0][0] + j[1][0] + 0.5 * Fx) / rt;
        if (fo.uy) fo.uy[k] = (j[0][1] + j[1][1] + 0.5 * Fy) / rt;
        if (fo.uz) fo.uz[k] = (j[0][2] + j[1][2] + 0.5 * Fz) / rt;
    } else {
        collide_store3<ST>(L, f, rho, a, cur, z, y, x);
    }
}

// The fused step: one pass per time step.  A block of FX x FY threads owns
// an (FX - 2) x (FY - 2) tile of the x-y plane plus a one-site halo and
// marches through a band of planes in z.  Per plane every thread pulls its
// site of the plane ahead into registers and puts its densities into a ring
// of four density planes in LDS; after one barrier the interior threads
// collide the site they pulled one plane earlier (still in registers), with
// the 18 neighbour densities from the ring.  Two register sets alternate
// (the march is unrolled by two), so no population is read twice.
// The register sets hold the populations in the storage type (converted,
// exactly, where they are used).  Two sets of FP64 populations plus the
// collision need about 220 VGPRs, so a block of 512 threads (two waves per
// SIMD) is the largest that fits; taller blocks spill and run slower.
constexpr int FX = 64, FY = 8;

template <int ST, int BCY>
__global__ void __launch_bounds__(FX * FY) k3_fused(Lat3 L, int cur, int nzb)
{
    using V = typename Tr<ST>::T;
    __shared__ double ring[4][2][FY][FX];
    static_assert(FX == 64, "one wave per thread row: y is uniform across a wave");
    const int lane = threadIdx.x;
    const int ty = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    const int xu = bx * (FX - 2) - 1 + lane;    // unwrapped column of this thread
    const int yu = by * (FY - 2) - 1 + ty;      // unwrapped row (wave-uniform)
    const int z0 = bz * nzb;
    const int nplanes = min(nzb, L.nz - z0);
    // the site this thread pulls: x wraps; beyond a wall the wall row
    // (mirror), or y wraps.  For interior threads it is (xu, yu) itself.
    int xs = xu % L.nx;
    if (xs < 0) xs += L.nx;
    int ys = yu;
    if (BCY == lbk::BC_PERIODIC) {
        ys %= L.ny;
        if (ys < 0) ys += L.ny;
    } else {
        ys = ys < 0 ? 0 : (ys >= L.ny ? L.ny - 1 : ys);
    }
    const bool interior = lane >= 1 && lane <= FX - 2 && ty >= 1 && ty <= FY - 2 && xu < L.nx && yu < L.ny;
    // lanes beyond the one-site halo of the lattice's last column or row
    // (the spare width of the last tile) pull nothing
    const bool live = xu <= L.nx && yu <= L.ny;
    const void *src = L.f[cur];
    // pull plane zp of this thread's site into f and its densities into a ring slot
    auto pull_plane = [&](int zp, V (&f)[2][NQ3], int slot) {
        zp %= L.nz;
        if (zp < 0) zp += L.nz;
        pull3<ST, BCY>(src, L, zp, ys, xs, f, live);
        ring[slot][0][ty][lane] = density3(f[0]);
        ring[slot][1][ty][lane] = density3(f[1]);
    };
    V fa[2][NQ3], fb[2][NQ3];
    // ring slot of plane z0 + k is (k + 1) & 3
    pull_plane(z0 - 1, fb, 0);
    pull_plane(z0, fa, 1);
    // cf: plane z (pulled one plane earlier), nf: receives plane z + 1
    auto plane = [&](int k, V (&cf)[2][NQ3], V (&nf)[2][NQ3]) {
        const int z = z0 + k;
        pull_plane(z + 1, nf, (k + 2) & 3);
        __syncthreads();
        if (interior) {
            double rho[2], S[2][3], a[2][3];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                rho[s] = density3(cf[s]);
                sc_sum3_nb([&](int i) { return ring[(k + 1 + c3z(i)) & 3][s][ty + c3y(i)][lane + c3x(i)]; }, S[s]);
            }
            accel3(L, S, a);
            collide_store3<ST>(L, cf, rho, a, cur, z, yu, xu);
        }
    };
    int k = 0;
    for (; k + 2 <= nplanes; k += 2) {
        plane(k, fa, fb);
        plane(k + 1, fb, fa);
    }
    if (k < nplanes) plane(k, fa, fb);
}

// Canonical f(t) [s][i][z][y][x] (or the rest equilibrium w_i rho_s of the
// density fields when fcan is null) into the stored post-collision form:
// f*_i(x) = f_i(x + c_i), or f_opp(i)(x) where x + c_i lies beyond a wall.
template <int ST, int BCY>
__global__ void __launch_bounds__(WX * WY)
k3_scatter(Lat3 L, int cur, const double *__restrict__ fcan, const double *__restrict__ rhoA,
           const double *__restrict__ rhoB)
{
    using T = typename Tr<ST>::T;
    const int x = blockIdx.x * WX + threadIdx.x;
    const int y = blockIdx.y * WY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= L.nx || y >= L.ny) return;
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    const rsrc_t wr = row_rsrc(L.f[cur], z * L.ny + y, L.rstride * (int64_t)sizeof(T));
    const unsigned is = (unsigned)L.pitch * (unsigned)sizeof(T);
#pragma unroll
    for (int i = 0; i < NQ3; ++i) {
        int xs = x + c3x(i), ys = y + c3y(i), zs = z + c3z(i), src_i = i;
        if (xs < 0) xs += L.nx;
        if (xs >= L.nx) xs -= L.nx;
        if (zs < 0) zs += L.nz;
        if (zs >= L.nz) zs -= L.nz;
        if (BCY == lbk::BC_PERIODIC) {
            if (ys < 0) ys += L.ny;
            if (ys >= L.ny) ys -= L.ny;
        } else if (ys < 0 || ys >= L.ny) {
            xs = x;
            ys = y;
            zs = z;
            src_i = opp3(i);
        }
        const int64_t k = ((int64_t)zs * L.ny + ys) * L.nx + xs;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double v = fcan ? fcan[(int64_t)(s * NQ3 + src_i) * n + k] : w3(src_i) * (s == 0 ? rhoA[k] : rhoB[k]);
            bstore<0>((T)v, wr, (unsigned)x * (unsigned)sizeof(T), (unsigned)(s * NQ3 + i) * is);
        }
    }
}

// Stored form -> canonical f(t) (the pull).
template <int ST, int BCY>
__global__ void __launch_bounds__(WX * WY) k3_gather(Lat3 L, int cur, double *__restrict__ fcan)
{
    const int x = blockIdx.x * WX + threadIdx.x;
    const int y = blockIdx.y * WY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= L.nx || y >= L.ny) return;
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    double f[2][NQ3];
    pull3<ST, BCY>(L.f[cur], L, z, y, x, f);
    const int64_t k = ((int64_t)z * L.ny + y) * L.nx + x;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < NQ3; ++i) fcan[(int64_t)(s * NQ3 + i) * n + k] = f[s][i];
}

// Per-row partial sums of the fields: mass_A, mass_B, E_k (trimmed rows
// only), max |u|^2, count of non-finite values.  One block per (z, y) row.
constexpr int RED3_NQ = 5;
constexpr int RED3_THREADS = 256;

__global__ void __launch_bounds__(RED3_THREADS)
k3_reduce_rows(const double *__restrict__ rA, const double *__restrict__ rB, const double *__restrict__ ux,
               const double *__restrict__ uy, const double *__restrict__ uz, int nx, int ny, int trim,
               double *__restrict__ part)
{
    __shared__ double sh[RED3_NQ][RED3_THREADS];
    const int row = blockIdx.x;
    const int y = row % ny;
    const bool in_d = y >= trim && y < ny - trim;
    double acc[RED3_NQ] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int x = threadIdx.x; x < nx; x += RED3_THREADS) {
        const int64_t k = (int64_t)row * nx + x;
        const double a = rA[k], b = rB[k], u = ux[k], v = uy[k], w = uz[k];
        const double u2 = u * u + v * v + w * w;
        acc[0] += a;
        acc[1] += b;
        if (in_d) acc[2] += 0.5 * (a + b) * u2;
        acc[3] = fmax(acc[3], u2);
        const bool fin = isfinite(a) && isfinite(b) && isfinite(u) && isfinite(v) && isfinite(w);
        acc[4] += fin ? 0.0 : 1.0;
    }
#pragma unroll
    for (int q = 0; q < RED3_NQ; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = RED3_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int q = 0; q < RED3_NQ; ++q)
                sh[q][threadIdx.x] = q == 3 ? fmax(sh[q][threadIdx.x], sh[q][threadIdx.x + h])
                                            : sh[q][threadIdx.x] + sh[q][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x < RED3_NQ) part[(int64_t)row * RED3_NQ + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(RED3_THREADS) k3_reduce_final(const double *__restrict__ part, int rows, double *out)
{
    __shared__ double sh[RED3_NQ][RED3_THREADS];
    double acc[RED3_NQ] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int r = threadIdx.x; r < rows; r += RED3_THREADS) {
#pragma unroll
        for (int q = 0; q < RED3_NQ; ++q) {
            const double v = part[(int64_t)r * RED3_NQ + q];
            acc[q] = q == 3 ? fmax(acc[q], v) : acc[q] + v;
        }
    }
#pragma unroll
    for (int q = 0; q < RED3_NQ; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = RED3_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int q = 0; q < RED3_NQ; ++q)
                sh[q][threadIdx.x] = q == 3 ? fmax(sh[q][threadIdx.x], sh[q][threadIdx.x + h])
                                            : sh[q][threadIdx.x] + sh[q][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x < RED3_NQ) out[threadIdx.x] = sh[threadIdx.x][0];
}

}  // namespace lbk3
