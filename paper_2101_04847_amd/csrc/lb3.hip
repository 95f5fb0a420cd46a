// Host runtime of the 3D (D3Q19) entry points declared in include/lb3.h:
// validation, workspace layout, initial state, the step (one fused pass, or
// two passes), the field pass, reductions and state conversion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <vector>

#include "lb3.h"
#include "lb3_kernels.hpp"

using namespace lbk3;
using lbrt::fail;

namespace {

constexpr size_t ALIGN3 = 256;
inline size_t up(size_t v) { return (v + ALIGN3 - 1) / ALIGN3 * ALIGN3; }

struct Layout3 {
    size_t fbuf[2];     // population buffers
    size_t rho;         // [nz][ny][2][pitch] densities
    size_t fields;      // [5][n] FP64 fields (diagnostics)
    size_t part;        // [rows][RED3_NQ]
    size_t red;         // RED3_NQ
    size_t total;
};

int32_t validate3(const lb3_config *c)
{
    if (!c) return fail(LB_EINVAL, "config is NULL");
    if (c->nx < 3 || c->ny < 3 || c->nz < 3)
        return fail(LB_EINVAL, "nx = %d, ny = %d, nz = %d must each be >= 3", c->nx, c->ny, c->nz);
    if ((int64_t)c->nx * c->ny * c->nz >= ((int64_t)1 << 31))
        return fail(LB_EINVAL, "%d x %d x %d sites reach 2^31", c->nx, c->ny, c->nz);
    if (c->nz > 65535) return fail(LB_EINVAL, "nz = %d exceeds 65535", c->nz);
    if ((int64_t)2 * NQ3 * ((c->nx + 63) / 64 * 64) * (c->storage == LB_F32 ? 4 : 8) > (int64_t)INT32_MAX)
        return fail(LB_EINVAL, "a row block of nx = %d exceeds 2^31 bytes", c->nx);
    if (c->bc_y != LB_WALLS && c->bc_y != LB_PERIODIC_Y) return fail(LB_EINVAL, "bc_y = %d out of range", c->bc_y);
    if (c->storage != LB_F64 && c->storage != LB_F32)
        return fail(LB_EINVAL, "storage = %d: the 3D step supports LB_F64 and LB_F32", c->storage);
    if (c->diag_trim < 0 || c->ny <= 2 * c->diag_trim)
        return fail(LB_EINVAL, "diag_trim = %d must be >= 0 and leave rows of ny = %d", c->diag_trim, c->ny);
    for (int s = 0; s < 2; ++s)
        if (!(c->tau[s] > 0.5) || !std::isfinite(c->tau[s]))
            return fail(LB_EINVAL, "tau[%d] = %g must be finite and > 1/2", s, c->tau[s]);
    if (!std::isfinite(c->G_AB)) return fail(LB_EINVAL, "G_AB is not finite");
    for (int s = 0; s < 2; ++s)
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(c->g[s][a])) return fail(LB_EINVAL, "g[%d][%d] is not finite", s, a);
    if (!c->rhoA0 || !c->rhoB0) return fail(LB_EINVAL, "initial densities are NULL");
    if (c->two_pass != 0 && c->two_pass != 1) return fail(LB_EINVAL, "two_pass = %d must be 0 or 1", c->two_pass);
    if (c->reserved != 0) return fail(LB_EINVAL, "reserved = %d must be 0", c->reserved);
    return LB_OK;
}

Layout3 layout3(const lb3_config *c)
{
    Layout3 L{};
    const size_t pitch = (size_t)(c->nx + 63) / 64 * 64;
    const size_t rows = (size_t)c->ny * c->nz;
    const size_t n = (size_t)c->nx * c->ny * c->nz;
    const size_t es = c->storage == LB_F64 ? 8 : 4;
    size_t off = 0;
    for (int b = 0; b < 2; ++b) {
        L.fbuf[b] = off;
        off = up(off + rows * 2 * NQ3 * pitch * es);
    }
    L.rho = off;
    off = up(off + rows * 2 * pitch * sizeof(double));
    L.fields = off;
    off = up(off + 5 * n * sizeof(double));
    L.part = off;
    off = up(off + rows * RED3_NQ * sizeof(double));
    L.red = off;
    off = up(off + RED3_NQ * sizeof(double));
    L.total = off;
    return L;
}

}  // namespace

struct lb3_handle {
    lb3_config cfg{};
    Lat3 L{};
    Layout3 lay{};
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    int64_t t = 0;
    int cur = 0;
};

namespace {

std::mutex g3_mu;
std::set<const lb3_handle *> g3_live;

bool live3(const lb3_handle *h)
{
    std::lock_guard<std::mutex> lk(g3_mu);
    return h && g3_live.count(h) > 0;
}

dim3 grid3(const lb3_handle *h)
{
    return dim3((unsigned)((h->cfg.nx + WX - 1) / WX), (unsigned)((h->cfg.ny + WY - 1) / WY), (unsigned)h->cfg.nz);
}

// Planes per band of the fused pass.  Short bands measure fastest at 384^3
// (8: 6.31 / 10.35 GLUPS FP64 / FP32; 32: 6.18 / 9.36; 4: 6.08 / 10.07)
// although each band re-pulls two halo planes.
constexpr int FUSED_NZB = 8;

dim3 grid_fused(const lb3_handle *h)
{
    return dim3((unsigned)((h->cfg.nx + FX - 3) / (FX - 2)), (unsigned)((h->cfg.ny + FY - 3) / (FY - 2)),
                (unsigned)((h->cfg.nz + FUSED_NZB - 1) / FUSED_NZB));
}

using FusedFn = void (*)(Lat3, int, int);
template <int ST>
FusedFn fused_st(int bc) { return bc == LB_WALLS ? k3_fused<ST, lbk::BC_WALLS> : k3_fused<ST, lbk::BC_PERIODIC>; }
FusedFn pick_fused(int st, int bc) { return st == LB_F64 ? fused_st<lbk::ST_F64>(bc) : fused_st<lbk::ST_F32>(bc); }

using DensFn = void (*)(Lat3, int);
using CollFn = void (*)(Lat3, int, Fields3);
using ScatFn = void (*)(Lat3, int, const double *, const double *, const double *);
using GathFn = void (*)(Lat3, int, double *);

template <int ST>
DensFn dens_st(int bc) { return bc == LB_WALLS ? k3_density<ST, lbk::BC_WALLS> : k3_density<ST, lbk::BC_PERIODIC>; }
DensFn pick_dens(int st, int bc) { return st == LB_F64 ? dens_st<lbk::ST_F64>(bc) : dens_st<lbk::ST_F32>(bc); }

template <int ST, bool FIELDS>
CollFn coll_st(int bc)
{
    return bc == LB_WALLS ? k3_collide<ST, lbk::BC_WALLS, FIELDS> : k3_collide<ST, lbk::BC_PERIODIC, FIELDS>;
}
CollFn pick_coll(int st, int bc, bool fields)
{
    if (fields) return st == LB_F64 ? coll_st<lbk::ST_F64, true>(bc) : coll_st<lbk::ST_F32, true>(bc);
    return st == LB_F64 ? coll_st<lbk::ST_F64, false>(bc) : coll_st<lbk::ST_F32, false>(bc);
}

template <int ST>
ScatFn scat_st(int bc) { return bc == LB_WALLS ? k3_scatter<ST, lbk::BC_WALLS> : k3_scatter<ST, lbk::BC_PERIODIC>; }
ScatFn pick_scat(int st, int bc) { return st == LB_F64 ? scat_st<lbk::ST_F64>(bc) : scat_st<lbk::ST_F32>(bc); }

template <int ST>
GathFn gath_st(int bc) { return bc == LB_WALLS ? k3_gather<ST, lbk::BC_WALLS> : k3_gather<ST, lbk::BC_PERIODIC>; }
GathFn pick_gath(int st, int bc) { return st == LB_F64 ? gath_st<lbk::ST_F64>(bc) : gath_st<lbk::ST_F32>(bc); }

// Fields of f(t): the density pass, then the collide kernel in field mode.
int32_t fields3(lb3_handle *h, Fields3 fo)
{
    hipLaunchKernelGGL(pick_dens(h->cfg.storage, h->cfg.bc_y), grid3(h), dim3(WX, WY), 0, h->stream, h->L, h->cur);
    hipLaunchKernelGGL(pick_coll(h->cfg.storage, h->cfg.bc_y, true), grid3(h), dim3(WX, WY), 0, h->stream, h->L,
                       h->cur, fo);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

}  // namespace

extern "C" {

size_t lb3_workspace_bytes(const lb3_config *cfg)
{
    if (validate3(cfg) != LB_OK) return 0;
    return layout3(cfg).total;
}

int32_t lb3_init(const lb3_config *cfg, void *d_workspace, size_t bytes, void *hip_stream, lb3_handle **out)
{
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    int32_t rc = validate3(cfg);
    if (rc) return rc;
    if (!d_workspace) return fail(LB_EINVAL, "workspace is NULL");
    if ((uintptr_t)d_workspace % ALIGN3) return fail(LB_EINVAL, "workspace is not 256-byte aligned");
    const Layout3 lay = layout3(cfg);
    if (bytes < lay.total) return fail(LB_ENOMEM, "workspace of %zu bytes < %zu needed", bytes, lay.total);

    lb3_handle *h = new (std::nothrow) lb3_handle;
    if (!h) return fail(LB_ENOMEM, "host allocation failed");
    h->cfg = *cfg;
    h->cfg.rhoA0 = h->cfg.rhoB0 = nullptr;
    h->lay = lay;
    h->ws = (char *)d_workspace;
    h->stream = (hipStream_t)hip_stream;
    Lat3 &L = h->L;
    L.nx = cfg->nx;
    L.ny = cfg->ny;
    L.nz = cfg->nz;
    L.pitch = (cfg->nx + 63) / 64 * 64;
    L.rstride = (int64_t)2 * NQ3 * L.pitch;
    L.f[0] = h->ws + lay.fbuf[0];
    L.f[1] = h->ws + lay.fbuf[1];
    L.rho = (double *)(h->ws + lay.rho);
    L.G = cfg->G_AB;
    for (int s = 0; s < 2; ++s) {
        L.tau[s] = cfg->tau[s];
        L.itau[s] = 1.0 / cfg->tau[s];
        for (int a = 0; a < 3; ++a) L.g[s][a] = cfg->g[s][a];
    }
    // initial state: the rest equilibrium of the densities (staged in the field buffer)
    const size_t n = (size_t)cfg->nx * cfg->ny * cfg->nz;
    double *stage = (double *)(h->ws + lay.fields);
    auto bail = [&](int32_t code) {
        delete h;
        return code;
    };
    if (hipMemcpyAsync(stage, cfg->rhoA0, n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(stage + n, cfg->rhoB0, n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return bail(fail(LB_EHIP, "copy of initial densities failed"));
    hipLaunchKernelGGL(pick_scat(cfg->storage, cfg->bc_y), grid3(h), dim3(WX, WY), 0, h->stream, h->L, 0,
                       (const double *)nullptr, (const double *)stage, (const double *)(stage + n));
    if (hipGetLastError() != hipSuccess) return bail(fail(LB_EHIP, "initial scatter launch failed"));
    if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(LB_EHIP, "stream synchronisation failed"));
    {
        std::lock_guard<std::mutex> lk(g3_mu);
        g3_live.insert(h);
    }
    *out = h;
    return LB_OK;
}

int32_t lb3_step(lb3_handle *h, int64_t n)
{
    if (!live3(h)) return fail(LB_ESTATE, "handle is not live");
    if (n < 0) return fail(LB_EINVAL, "n = %lld is negative", (long long)n);
    if (h->cfg.two_pass) {
        const DensFn fd = pick_dens(h->cfg.storage, h->cfg.bc_y);
        const CollFn fc = pick_coll(h->cfg.storage, h->cfg.bc_y, false);
        const dim3 g = grid3(h);
        for (int64_t k = 0; k < n; ++k) {
            hipLaunchKernelGGL(fd, g, dim3(WX, WY), 0, h->stream, h->L, h->cur);
            hipLaunchKernelGGL(fc, g, dim3(WX, WY), 0, h->stream, h->L, h->cur, Fields3{});
            h->cur ^= 1;
            h->t += 1;
        }
    } else {
        const FusedFn ff = pick_fused(h->cfg.storage, h->cfg.bc_y);
        const dim3 g = grid_fused(h);
        for (int64_t k = 0; k < n; ++k) {
            hipLaunchKernelGGL(ff, g, dim3(FX, FY), 0, h->stream, h->L, h->cur, FUSED_NZB);
            h->cur ^= 1;
            h->t += 1;
        }
    }
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

int32_t lb3_fields(lb3_handle *h, double *d_rhoA, double *d_rhoB, double *d_ux, double *d_uy, double *d_uz)
{
    if (!live3(h)) return fail(LB_ESTATE, "handle is not live");
    return fields3(h, Fields3{d_rhoA, d_rhoB, d_ux, d_uy, d_uz});
}

int32_t lb3_diagnostics(lb3_handle *h, lb3_diag *out)
{
    if (!live3(h)) return fail(LB_ESTATE, "handle is not live");
    if (!out) return fail(LB_EINVAL, "out is NULL");
    const size_t n = (size_t)h->cfg.nx * h->cfg.ny * h->cfg.nz;
    double *fld = (double *)(h->ws + h->lay.fields);
    int32_t rc = fields3(h, Fields3{fld, fld + n, fld + 2 * n, fld + 3 * n, fld + 4 * n});
    if (rc) return rc;
    const int rows = h->cfg.ny * h->cfg.nz;
    double *part = (double *)(h->ws + h->lay.part);
    double *red = (double *)(h->ws + h->lay.red);
    hipLaunchKernelGGL(k3_reduce_rows, dim3(rows), dim3(RED3_THREADS), 0, h->stream, (const double *)fld,
                       (const double *)(fld + n), (const double *)(fld + 2 * n), (const double *)(fld + 3 * n),
                       (const double *)(fld + 4 * n), h->cfg.nx, h->cfg.ny, h->cfg.diag_trim, part);
    hipLaunchKernelGGL(k3_reduce_final, dim3(1), dim3(RED3_THREADS), 0, h->stream, (const double *)part, rows, red);
    HIP_TRY(hipGetLastError());
    double host[RED3_NQ];
    HIP_TRY(hipMemcpyAsync(host, red, sizeof host, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const double nd = (double)h->cfg.nx * (double)(h->cfg.ny - 2 * h->cfg.diag_trim) * (double)h->cfg.nz;
    out->t = h->t;
    out->mass[0] = host[0];
    out->mass[1] = host[1];
    out->Ek = host[2] / nd;
    out->umax = std::sqrt(host[3]);
    out->finite = host[4] == 0.0 ? 1 : 0;
    out->reserved = 0;
    return out->finite ? LB_OK : fail(LB_ENONFINITE, "non-finite density or velocity at t = %lld", (long long)h->t);
}

int32_t lb3_get_populations(lb3_handle *h, double *d_f)
{
    if (!live3(h)) return fail(LB_ESTATE, "handle is not live");
    if (!d_f) return fail(LB_EINVAL, "d_f is NULL");
    hipLaunchKernelGGL(pick_gath(h->cfg.storage, h->cfg.bc_y), grid3(h), dim3(WX, WY), 0, h->stream, h->L, h->cur,
                       d_f);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

int32_t lb3_set_populations(lb3_handle *h, const double *d_f)
{
    if (!live3(h)) return fail(LB_ESTATE, "handle is not live");
    if (!d_f) return fail(LB_EINVAL, "d_f is NULL");
    hipLaunchKernelGGL(pick_scat(h->cfg.storage, h->cfg.bc_y), grid3(h), dim3(WX, WY), 0, h->stream, h->L, h->cur,
                       d_f, (const double *)nullptr, (const double *)nullptr);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

int64_t lb3_time(const lb3_handle *h) { return live3(h) ? h->t : -1; }

int32_t lb3_destroy(lb3_handle *h)
{
    {
        std::lock_guard<std::mutex> lk(g3_mu);
        if (!h || !g3_live.count(h)) return fail(LB_ESTATE, "handle is not live");
        g3_live.erase(h);
    }
    const hipError_t e = hipStreamSynchronize(h->stream);
    delete h;
    if (e != hipSuccess) return fail(LB_EHIP, "stream synchronisation failed: %s", hipGetErrorString(e));
    return LB_OK;
}

}  // extern "C"
