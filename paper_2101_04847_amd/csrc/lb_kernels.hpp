// gfx950 kernels of the two-component D2Q9 Shan-Chen lattice Boltzmann step
// and of the analysis of its fields.
//
// Method (paper Sec. 2): per component s, rho_s = sum_i f_i^s (Eq. 1);
// Shan-Chen force F_s = -G rho_s sum_i w_i rho_sbar(x + c_i) c_i (Eq. 5) plus
// buoyancy rho_s g_s (Eq. 7), i.e. rho_s a_s with the acceleration
// a_s = -G sum_i w_i rho_sbar(x + c_i) c_i + g_s, on the two wall rows plus
// the fluid-boundary term of Eq. 6; common velocity weighted by 1/tau_s
// (Eq. 1); BGK relaxation towards f^eq(rho_s, u + tau_s a_s) (Eq. 2-3) or Guo
// forcing; streaming with periodic x and halfway bounce-back walls.  Beyond a
// wall psi is that of the wall row (mirror) or zero.
//
// Storage: per member two buffers of row blocks [y][s][i][pitch] (the 18
// row segments of one lattice row adjacent, x fastest, pitch a multiple of
// 64 elements).  A buffer holds post-collision populations f*(t-1); the
// pre-collision state f(t) is obtained by PULLING: f_i(x) = f*_i(x - c_i),
// or f*_opp(i)(x) where x - c_i lies beyond a wall.
//
// Two step passes, both HBM-bound (no dense contraction, so no MFMA):
//   k_step   one step per pass: a workgroup owns TX columns and marches
//            through a band of rows; each row's densities go to a 4-row LDS
//            ring (with two halo columns) from which, after one barrier, the
//            previous row's force is evaluated, collided and stored.
//   k_step2  two steps per pass (temporal blocking): a single wave marches a
//            band computing step t -> t+1 in registers and, two rows behind,
//            step t+1 -> t+2 from the neighbouring lanes' results (DPP
//            shifts); populations cross HBM once per two steps.
//   k_step3  three steps per pass, the same march with a third stage.
// All evaluate every site through collide_site, so they agree bit for bit.
//
// In the FP64 mode every expression is evaluated in the order of the
// definitions (sums over i in index order, no contraction), so the step is
// reproducible bit for bit by a plain CPU implementation of the same
// equations.
//
// Analysis kernels (Sec. 3): the field pass (k_step with FIELDS), energy
// averages (k_reduce_rows / k_reduce_final), the kinetic-energy budget
// (k_budget_rows), the interface crossings (k_interface_rows) and the
// connected components of the two phases (k_cc_*).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lb_internal.hpp"
#include "lb_memory.hpp"

namespace lbk {

// ---------------------------------------------------------------------------
// D2Q9 lattice (Sec. 2): velocities in the order
// 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
// and the weights fixed by the isotropy conditions of Eq. 4.
__host__ __device__ constexpr int cx(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0; }
__host__ __device__ constexpr int cy(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0; }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 5 + 2) % 4) + 5); }
__host__ __device__ constexpr double wgt(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }

static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "axis opposites");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "diagonal opposites");

// ---------------------------------------------------------------------------
// Sources of the pull of row y for column c (streaming with periodic x, and
// either halfway bounce-back walls or periodic y): f_i(x) = f*_i(x - c_i), or
// f*_opp(i)(x) where x - c_i lies beyond a wall.  Holds the buffer resources
// of rows y, y - 1 and y + 1 (row y itself where that row lies beyond a
// wall) and the per-lane byte offsets of the three source columns.
template <int ST, int BCY>
struct RowPull {
    using T = typename Tr<ST>::T;
    rsrc_t r0, rm, rp;
    unsigned oc, om, op;    // source columns c, c - 1 (c_x = +1), c + 1 (c_x = -1)
    unsigned is, ss;        // bytes between populations, between components
    int cc, cm, cp;         // the three source columns
    bool bb_lo, bb_hi;      // row y - 1 / y + 1 lies beyond a wall

    __device__ __forceinline__ RowPull(const void *src, const Member &M, int y, int c)
    {
        const int nx = M.nx, ny = M.ny;
        const int64_t row_bytes = M.ystride * (int64_t)sizeof(T);
        is = (unsigned)M.istride * (unsigned)sizeof(T);
        ss = (unsigned)M.sstride * (unsigned)sizeof(T);
        cc = c;
        cm = (c == 0) ? nx - 1 : c - 1;
        cp = (c == nx - 1) ? 0 : c + 1;
        oc = (unsigned)cc * (unsigned)sizeof(T);
        om = (unsigned)cm * (unsigned)sizeof(T);
        op = (unsigned)cp * (unsigned)sizeof(T);
        int ym = y - 1, yp = y + 1;   // source rows for c_y = +1 / -1
        bb_lo = bb_hi = false;
        if (BCY == BC_PERIODIC) {
            if (ym < 0) ym = ny - 1;
            if (yp >= ny) yp = 0;
        } else {
            bb_lo = ym < 0;
            bb_hi = yp >= ny;
            if (bb_lo) ym = y;   // bounce-back sources lie in row y
            if (bb_hi) yp = y;
        }
        r0 = row_rsrc(src, y, row_bytes);
        rm = row_rsrc(src, ym, row_bytes);
        rp = row_rsrc(src, yp, row_bytes);
    }

    // The stored source of population i of component s; beyond a wall
    // (bounce-back) the population comes from the same site with the
    // reversed velocity.  i is a constant after unrolling.
    __device__ __forceinline__ T load(int s, int i) const
    {
        const unsigned b = (unsigned)s * ss;
        switch (i) {
            case 0: return bload<T>(r0, oc, b + 0 * is);
            case 1: return bload<T>(r0, om, b + 1 * is);
            case 3: return bload<T>(r0, op, b + 3 * is);
            case 2: return bload<T>(rm, oc, b + (bb_lo ? 4 : 2) * is);
            case 5: return bload<T>(rm, bb_lo ? oc : om, b + (bb_lo ? 7 : 5) * is);
            case 6: return bload<T>(rm, bb_lo ? oc : op, b + (bb_lo ? 8 : 6) * is);
            case 4: return bload<T>(rp, oc, b + (bb_hi ? 2 : 4) * is);
            case 7: return bload<T>(rp, bb_hi ? oc : op, b + (bb_hi ? 5 : 7) * is);
            default: return bload<T>(rp, bb_hi ? oc : om, b + (bb_hi ? 6 : 8) * is);
        }
    }

    // 16-bit modes: the stored density of component s at the site that
    // population i is pulled from (the same site as load(s, i)).
    __device__ __forceinline__ float load_rho(const Member &M, int s, int i) const
    {
        const unsigned b = (unsigned)M.rho_off + (unsigned)s * (unsigned)M.rho_sstride;
        const unsigned fc = (unsigned)cc * 4u, fm = (unsigned)cm * 4u, fp = (unsigned)cp * 4u;
        switch (i) {
            case 0: return bload<float>(r0, fc, b);
            case 1: return bload<float>(r0, fm, b);
            case 3: return bload<float>(r0, fp, b);
            case 2: return bload<float>(rm, fc, b);
            case 5: return bload<float>(rm, bb_lo ? fc : fm, b);
            case 6: return bload<float>(rm, bb_lo ? fc : fp, b);
            case 4: return bload<float>(rp, fc, b);
            case 7: return bload<float>(rp, bb_hi ? fc : fp, b);
            default: return bload<float>(rp, bb_hi ? fc : fm, b);
        }
    }
};

// Weight class of population i (0: rest, 1: axis, 2: diagonal); the code
// scales S_i of the 16-bit modes depend on w_i only.
__host__ __device__ constexpr int wclass(int i) { return i == 0 ? 0 : (i <= 4 ? 1 : 2); }

// x S_i and v / S_i + b in the 16-bit modes.  bfloat16 codes are unscaled
// (S_i = 1): x * 1 and fma(v, 1, b) = v + b are exact, so skipping them gives
// the same results.
template <int ST>
__device__ __forceinline__ float code_scaled(const Member &M, int i, float x)
{
    if constexpr (ST == ST_BF16S) return x;
    else return x * M.cscale[wclass(i)];
}
template <int ST>
__device__ __forceinline__ float code_unscaled(const Member &M, int i, float v)
{
    if constexpr (ST == ST_BF16S) return v;
    else return v * M.ciscale[wclass(i)];
}

// 16-bit modes: population i decoded from its code q and the stored density
// rhat of the site it was stored at, f = w_i rhat + q / S_i.
template <int ST>
__device__ __forceinline__ float site_decode(const Member &M, typename Tr<ST>::T q, float rhat, int i)
{
    if constexpr (ST == ST_BF16S) return Tr<ST>::value(q) + (float)wgt(i) * rhat;
    else return fmaf(Tr<ST>::value(q), M.ciscale[wclass(i)], (float)wgt(i) * rhat);
}

// 16-bit modes: codes of the post-collision populations of component s at
// one site of density rho, q_i = code((post_i - w_i r) S_i) with r = rho
// rounded to FP32, and the stored density rhat = rho - sum_i q_i / S_i: the
// decoded populations w_i rhat + q_i / S_i then sum to rho up to FP32
// rounding (sum_i w_i = 1), whatever the rounding of the codes, so the codes
// carry no systematic mass error.
template <int ST>
__device__ __forceinline__ void site_encode(const Member &M, double rho, const float (&post)[NQ],
                                            typename Tr<ST>::T (&q)[NQ], float &rhat)
{
    const float r = (float)rho;
    float e = 0.0f;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const float d = fmaf(-(float)wgt(i), r, post[i]);
        q[i] = Tr<ST>::code(code_scaled<ST>(M, i, d));
        e += code_unscaled<ST>(M, i, Tr<ST>::value(q[i]));
    }
    rhat = (float)(rho - (double)e);
}

// Pull the 18 pre-collision populations f(t) of column c, row y from the
// post-collision buffer src, the loads grouped by source row.
template <int ST, int BCY>
__device__ __forceinline__ void pull_site(const void *src, const Member &M, int y, int c,
                                          typename Tr<ST>::C (&f)[2][NQ])
{
    using Q = Tr<ST>;
    const RowPull<ST, BCY> pr(src, M, y, c);
    constexpr int ORDER[NQ] = {0, 1, 3, 2, 5, 6, 4, 7, 8};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        typename Q::T v[NQ];
#pragma unroll
        for (int j = 0; j < NQ; ++j) v[ORDER[j]] = pr.load(s, ORDER[j]);
        if constexpr (Q::SITE) {
            float rh[NQ];
#pragma unroll
            for (int j = 0; j < NQ; ++j) rh[ORDER[j]] = pr.load_rho(M, s, ORDER[j]);
#pragma unroll
            for (int i = 0; i < NQ; ++i) f[s][i] = site_decode<ST>(M, v[i], rh[i], i);
        } else {
#pragma unroll
            for (int i = 0; i < NQ; ++i) f[s][i] = Q::dec(v[i]);
        }
    }
}

// Store the post-collision populations of one site (column byte offset ox
// of row resource wr) in the storage mode; post[s][i] in the arithmetic type.
// x is the site's column (for the 16-bit modes' density segment).
template <int ST>
__device__ __forceinline__ void store_site(const Member &M, rsrc_t wr, unsigned ox, int x, unsigned wis, unsigned wss,
                                           const double (&rho)[2], const typename Tr<ST>::C (&post)[2][NQ])
{
    using Q = Tr<ST>;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        if constexpr (Q::SITE) {
            typename Q::T q[NQ];
            float rhat;
            site_encode<ST>(M, rho[s], post[s], q, rhat);
#pragma unroll
            for (int i = 0; i < NQ; ++i)
                bstore<LBK_NT_STORE ? CPOL_NT : 0>(q[i], wr, ox, (unsigned)s * wss + (unsigned)i * wis);
            bstore<LBK_NT_STORE ? CPOL_NT : 0>(rhat, wr, (unsigned)x * 4u,
                                                (unsigned)M.rho_off + (unsigned)s * (unsigned)M.rho_sstride);
        } else {
#pragma unroll
            for (int i = 0; i < NQ; ++i)
                bstore<LBK_NT_STORE ? CPOL_NT : 0>(Q::enc(post[s][i]), wr, ox, (unsigned)s * wss + (unsigned)i * wis);
        }
    }
}

// Eq. 1: rho_s = sum_i f_i^s in index order, in FP64.
template <class C>
__device__ __forceinline__ double density(const C (&f)[NQ])
{
    double r = (double)f[0];
#pragma unroll
    for (int i = 1; i < NQ; ++i) r += (double)f[i];
    return r;
}

// j_s = sum_i f_i^s c_i in index order (terms with c = 0 add nothing).
template <class C>
__device__ __forceinline__ void momentum(const C (&f)[NQ], double &jx, double &jy)
{
    jx = (double)f[1];
    jx -= (double)f[3];
    jx += (double)f[5];
    jx -= (double)f[6];
    jx -= (double)f[7];
    jx += (double)f[8];
    jy = (double)f[2];
    jy -= (double)f[4];
    jy += (double)f[5];
    jy += (double)f[6];
    jy -= (double)f[7];
    jy -= (double)f[8];
}

// j_s = sum_i f_i^s c_i in the arithmetic type of the reduced-precision
// collision (FP32), same term order.
__device__ __forceinline__ void momentum_f(const float (&f)[NQ], float &jx, float &jy)
{
    jx = ((f[1] - f[3]) + (f[5] - f[6])) + (f[8] - f[7]);
    jy = ((f[2] - f[4]) + (f[5] + f[6])) - (f[7] + f[8]);
}

// ---------------------------------------------------------------------------
// Eq. 5 neighbour sum S = sum_i w_i psi(x + c_i) c_i of one component, in
// index order (i = 1..8), from its eight neighbour densities p1..p8 (p_i at
// x + c_i).
// FACTORED selects the form w_1 (p1 - p3) + w_5 ((p5 - p7) + (p8 - p6)) (and
// likewise for y), 12 instead of 22 FP64 operations: the reduced-precision
// modes use it (in both passes, so they still agree bit for bit); the FP64
// mode and the field pass keep the index order of the definition.
template <bool FACTORED = false>
__device__ __forceinline__ void sc_sum(double p1, double p2, double p3, double p4, double p5, double p6, double p7,
                                       double p8, double &Sx, double &Sy)
{
    if constexpr (FACTORED) {
        const double w1 = wgt(1), w5 = wgt(5);
        const double d57 = p5 - p7, d86 = p8 - p6;
        Sx = w1 * (p1 - p3) + w5 * (d57 + d86);
        Sy = w1 * (p2 - p4) + w5 * (d57 - d86);
        return;
    }

    const double w1 = wgt(1), w5 = wgt(5);
    double sx = w1 * p1;
    sx -= w1 * p3;
    sx += w5 * p5;
    sx -= w5 * p6;
    sx -= w5 * p7;
    sx += w5 * p8;
    double sy = w1 * p2;
    sy -= w1 * p4;
    sy += w5 * p5;
    sy += w5 * p6;
    sy -= w5 * p7;
    sy -= w5 * p8;
    Sx = sx;
    Sy = sy;
}

// Which Eq. 6 wall acceleration row y takes: 0 (row 0), 1 (row ny - 1), or
// -1 (none: an interior row, periodic y, or G_Ab = G_Bb = 0).  The boundary
// nodes are the rows just outside the lattice, so only the wall rows see them.
template <int BCY>
__device__ __forceinline__ int wall_row(const Member &M, int y)
{
    if (BCY != BC_WALLS_WET || !M.wall_force) return -1;
    return y == 0 ? 0 : (y == M.ny - 1 ? 1 : -1);
}

// Collision of one site (Eq. 1-3 and the BGK relaxation of Eq. 2, or Guo
// forcing) given the pulled populations cur_f, the densities rho_c and the
// Shan-Chen sums S of the other component (S[s] belongs to component s, so
// component s feels S[1 - s]); wrow selects the wall acceleration of Eq. 6
// (wall_row).  Each post-collision value is handed to emit(s, i, post) in
// the arithmetic type of the storage mode.
template <int ST, int FORCING, class Emit>
__device__ __forceinline__ void collide_site(const Member &M, const typename Tr<ST>::C (&cur_f)[2][NQ],
                                             const double (&rho_c)[2], const double (&Sx)[2], const double (&Sy)[2],
                                             int wrow, Emit &&emit)
{
    using C = typename Tr<ST>::C;
    if constexpr (ST == ST_F64) {
        double jx[2], jy[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) momentum(cur_f[s], jx[s], jy[s]);
        // FP64: the definitions evaluated in their written order.  With
        // psi_s = rho_s, Eq. 5 + Eq. 7 (+ Eq. 6 on a wall row) give
        // F_s = rho_s a_s with the acceleration a_s = -G S_sbar + g_s (+ a^w_s).
        double ax[2], ay[2], Fx[2], Fy[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            ax[s] = -M.G * Sx[1 - s] + M.g[s][0];
            ay[s] = -M.G * Sy[1 - s] + M.g[s][1];
            if (wrow >= 0) ay[s] += M.aw[s][wrow];
            Fx[s] = rho_c[s] * ax[s];
            Fy[s] = rho_c[s] * ay[s];
        }
        const double rt = rho_c[0] + rho_c[1];
        double ux, uy;
        if (FORCING == FORCE_SHIFT) {
            // Eq. 1: velocity weighted by 1/tau_s
            const double nxv = jx[0] * M.itau[0] + jx[1] * M.itau[1];
            const double nyv = jy[0] * M.itau[0] + jy[1] * M.itau[1];
            const double den = rho_c[0] * M.itau[0] + rho_c[1] * M.itau[1];
            ux = nxv / den;
            uy = nyv / den;
        } else {
            ux = (jx[0] + jx[1] + 0.5 * (Fx[0] + Fx[1])) / rt;
            uy = (jy[0] + jy[1] + 0.5 * (Fy[0] + Fy[1])) / rt;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            double vxd = ux, vyd = uy;
            if (FORCING == FORCE_SHIFT) {
                // Eq. 3: shifted velocity u + tau_s F_s / rho_s = u + tau_s a_s
                vxd = ux + M.tau[s] * ax[s];
                vyd = uy + M.tau[s] * ay[s];
            }
            C vx = (C)vxd, vy = (C)vyd;
            const C rho = (C)rho_c[s];
            // Under Guo forcing both components see the same velocity, so
            // every per-population term of the equilibrium and the source is
            // the same for both; kept from the first component for the
            // second they hold ~30 registers across the loop and the fused
            // pass spills.  The empty asm makes the values opaque per
            // component so that they are recomputed (same expressions, same
            // results); with it the FP64 fused Guo pass fits 256 VGPRs.
            if (FORCING == FORCE_GUO) asm volatile("" : "+v"(vx), "+v"(vy));
            const C omega = (C)M.itau[s];
            const C vv = vx * vx + vy * vy;
            C gcoef = (C)0, fx = (C)0, fy = (C)0, gux = (C)0, guy = (C)0;
            if (FORCING == FORCE_GUO) {
                gcoef = (C)(1.0 - 0.5 * M.itau[s]);
                fx = (C)Fx[s];
                fy = (C)Fy[s];
                gux = (C)ux;
                guy = (C)uy;
                asm volatile("" : "+v"(gux), "+v"(guy));
            }
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                // c_i . v with the same operand order as sum_a c_ia v_a
                C cv;
                if (cx(i) == 0 && cy(i) == 0) cv = (C)0;
                else if (cy(i) == 0) cv = cx(i) > 0 ? vx : -vx;
                else if (cx(i) == 0) cv = cy(i) > 0 ? vy : -vy;
                else cv = (cx(i) > 0 ? vx : -vx) + (cy(i) > 0 ? vy : -vy);
                // Eq. 3
                const C feq = rho * (C)wgt(i) * ((C)1 + (C)3 * cv + (C)4.5 * cv * cv - (C)1.5 * vv);
                const C fi = cur_f[s][i];
                // Eq. 2
                C post = fi - omega * (fi - feq);
                if (FORCING == FORCE_GUO) {
                    C cu;
                    if (cx(i) == 0 && cy(i) == 0) cu = (C)0;
                    else if (cy(i) == 0) cu = cx(i) > 0 ? gux : -gux;
                    else if (cx(i) == 0) cu = cy(i) > 0 ? guy : -guy;
                    else cu = (cx(i) > 0 ? gux : -gux) + (cy(i) > 0 ? guy : -guy);
                    const C ex = (C)3 * ((C)cx(i) - gux) + (C)9 * cu * (C)cx(i);
                    const C ey = (C)3 * ((C)cy(i) - guy) + (C)9 * cu * (C)cy(i);
                    post += gcoef * (C)wgt(i) * (ex * fx + ey * fy);
                }
                emit(s, i, post);
            }
        }
    } else {
        // Reduced-precision modes: momenta and the collision in FP32 with
        // fused multiply-adds.  Densities, the Shan-Chen sums and the
        // accelerations a_s = -G S_sbar + g_s (+ a^w_s) stay FP64.
        float jx[2], jy[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) momentum_f(cur_f[s], jx[s], jy[s]);
        float rf[2], ax[2], ay[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            rf[s] = (float)rho_c[s];
            ax[s] = (float)(-M.G * Sx[1 - s] + M.g[s][0]);
            double ays = -M.G * Sy[1 - s] + M.g[s][1];
            if (wrow >= 0) ays += M.aw[s][wrow];
            ay[s] = (float)ays;
        }
        float ux, uy;
        if (FORCING == FORCE_SHIFT) {
            // Eq. 1: velocity weighted by 1/tau_s
            const float itA = (float)M.itau[0], itB = (float)M.itau[1];
            const float iden = __builtin_amdgcn_rcpf(fmaf(rf[0], itA, rf[1] * itB));
            ux = fmaf(jx[0], itA, jx[1] * itB) * iden;
            uy = fmaf(jy[0], itA, jy[1] * itB) * iden;
        } else {
            // Guo: (sum_s j_s + F / 2) / rho
            const float irt = __builtin_amdgcn_rcpf(rf[0] + rf[1]);
            ux = fmaf(0.5f, fmaf(rf[0], ax[0], rf[1] * ax[1]), jx[0] + jx[1]) * irt;
            uy = fmaf(0.5f, fmaf(rf[0], ay[0], rf[1] * ay[1]), jy[0] + jy[1]) * irt;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            float vx = ux, vy = uy;
            if (FORCING == FORCE_SHIFT) {
                // Eq. 3: shifted velocity u + tau_s a_s
                vx = fmaf((float)M.tau[s], ax[s], ux);
                vy = fmaf((float)M.tau[s], ay[s], uy);
            }
            const float r = rf[s];
            const float om = (float)M.itau[s];
            const float base = fmaf(-1.5f, fmaf(vx, vx, vy * vy), 1.0f);   // 1 - 3/2 v.v
            // Guo source (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F
            // = coef w_i [9 (c.u)(c.F) - 3 u.F] +- coef w_i 3 c.F for +-c_i
            float coef = 0.f, fx = 0.f, fy = 0.f, uF = 0.f;
            if (FORCING == FORCE_GUO) {
                coef = 1.0f - 0.5f * om;
                fx = r * ax[s];
                fy = r * ay[s];
                uF = fmaf(ux, fx, uy * fy);
            }
            auto put = [&](int i, float fe, float src) {
                const float fi = cur_f[s][i];
                float post = fmaf(om, fe - fi, fi);          // Eq. 2
                if (FORCING == FORCE_GUO) post += src;
                emit(s, i, post);
            };
            // rest population
            {
                const float w = (float)wgt(0);
                put(0, (w * r) * base, FORCING == FORCE_GUO ? coef * w * (-3.0f * uF) : 0.f);
            }
            // pairs (i, opp(i)) sharing |c . v|: equilibria A +- B of Eq. 3
            auto pair = [&](int i, int o, float cu, float cvv, float cF) {
                const float w = (float)wgt(i);
                const float wr_ = w * r;
                const float A = wr_ * fmaf(4.5f * cvv, cvv, base);
                const float B = wr_ * (3.0f * cvv);
                float Ga = 0.f, Gb = 0.f;
                if (FORCING == FORCE_GUO) {
                    Ga = coef * w * fmaf(9.0f * cu, cF, -3.0f * uF);
                    Gb = coef * w * (3.0f * cF);
                }
                put(i, A + B, Ga + Gb);
                put(o, A - B, Ga - Gb);
            };
            pair(1, 3, ux, vx, fx);                         // c = (1, 0)
            pair(2, 4, uy, vy, fy);                         // c = (0, 1)
            pair(5, 7, ux + uy, vx + vy, fx + fy);          // c = (1, 1)
            pair(8, 6, ux - uy, vx - vy, fx - fy);          // c = (1, -1)
        }
    }
}

// ---------------------------------------------------------------------------
// The fused step.  FIELDS = false: collide and store f*(t) into the other
// buffer.  FIELDS = true: write rho_A, rho_B and the hydrodynamic velocity of
// f(t) instead (no state change).  Work items are tiles of TX columns by
// tile_h rows, numbered per member; a launch covers items [item0, item0 + n).
// Force, collision and store (or field output) of one row for one lane:
// Eq. 5 and 7 from the density ring, then collide_site.  s0, sp, sm are the
// ring slots of rows y, y + 1 and y - 1; e is this lane's ring column.
template <int ST, int FORCING, bool FIELDS, int LW>
__device__ __forceinline__ void row_update(const Member &M, const double (&ring)[4][2][LW], int s0, int sp, int sm,
                                           int e, int x, int y, int wrow, const typename Tr<ST>::C (&cur_f)[2][NQ],
                                           const double (&rho_c)[2], void *dst, const FieldOut &fo)
{
    using Q = Tr<ST>;
    using T = typename Q::T;
    using C = typename Q::C;
    double Sx[2], Sy[2];
#pragma unroll
    for (int o = 0; o < 2; ++o)
        sc_sum<!FIELDS && ST != ST_F64>(ring[s0][o][e + 1], ring[sp][o][e], ring[s0][o][e - 1], ring[sm][o][e], ring[sp][o][e + 1],
               ring[sp][o][e - 1], ring[sm][o][e - 1], ring[sm][o][e + 1], Sx[o], Sy[o]);
    if constexpr (FIELDS) {
        double jx[2], jy[2], Fx[2], Fy[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            momentum(cur_f[s], jx[s], jy[s]);
            // F_s = rho_s a_s, a_s = -G S_sbar + g_s (+ a^w_s)   (Eq. 5 + Eq. 7 + Eq. 6, psi_s = rho_s)
            Fx[s] = rho_c[s] * (-M.G * Sx[1 - s] + M.g[s][0]);
            double ay = -M.G * Sy[1 - s] + M.g[s][1];
            if (wrow >= 0) ay += M.aw[s][wrow];
            Fy[s] = rho_c[s] * ay;
        }
        const double rt = rho_c[0] + rho_c[1];
        // hydrodynamic velocity (sum_s j_s + sum_s F_s / 2) / rho
        const double ux = (jx[0] + jx[1] + 0.5 * (Fx[0] + Fx[1])) / rt;
        const double uy = (jy[0] + jy[1] + 0.5 * (Fy[0] + Fy[1])) / rt;
        const int64_t k = (int64_t)y * M.nx + x;
        if (fo.rhoA) fo.rhoA[k] = rho_c[0];
        if (fo.rhoB) fo.rhoB[k] = rho_c[1];
        if (fo.ux) fo.ux[k] = ux;
        if (fo.uy) fo.uy[k] = uy;
    } else {
        const rsrc_t wr = row_rsrc(dst, y, M.ystride * (int64_t)sizeof(T));
        const unsigned ox = (unsigned)x * (unsigned)sizeof(T);
        const unsigned wis = (unsigned)M.istride * (unsigned)sizeof(T);
        const unsigned wss = (unsigned)M.sstride * (unsigned)sizeof(T);
        if constexpr (Q::SITE) {
            C post[2][NQ];
            collide_site<ST, FORCING>(M, cur_f, rho_c, Sx, Sy, wrow, [&](int s, int i, C p) { post[s][i] = p; });
            store_site<ST>(M, wr, ox, x, wis, wss, rho_c, post);
        } else {
            collide_site<ST, FORCING>(M, cur_f, rho_c, Sx, Sy, wrow, [&](int s, int i, C post) {
                bstore<LBK_NT_STORE ? CPOL_NT : 0>(Q::enc(post), wr, ox, (unsigned)s * wss + (unsigned)i * wis);
            });
        }
    }
}

template <int ST, int FORCING, int BCY, int TX, bool FIELDS>
__global__ void __launch_bounds__(TX)
k_step(const Member *__restrict__ members, int n_members, int64_t item0, int64_t n_items, int cur,
       FieldOut fo)
{
    using Q = Tr<ST>;
    using C = typename Q::C;
    constexpr int LW = TX + 2;                  // ring row: TX columns plus two halo columns
    __shared__ double ring[4][2][LW];           // rho_A, rho_B of four consecutive rows

    const int lane = threadIdx.x;
    for (int64_t item = item0 + blockIdx.x; item < item0 + n_items; item += gridDim.x) {
        int m = 0;
        while (m + 1 < n_members && members[m].item_end <= item) ++m;
        const Member &M = members[m];
        const int nx = M.nx, ny = M.ny;
        // work item -> tile, row-major over the member's tiles
        const int64_t t = item - M.item_begin;
        const int tx = (int)(t % M.tiles_x);
        const int ty = (int)(t / M.tiles_x);
        const int x0 = tx * TX;
        const int y0 = ty * M.tile_h;
        const int nrows = min(M.tile_h, ny - y0);
        const void *src = M.f[cur];
        void *dst = M.f[cur ^ 1];
#if LBK_ALT_DIR
        // odd bands march down, so that two vertically adjacent bands read
        // the rows they share at the same time (both at their start or both
        // at their end): the second read then hits the cache
        const int dir = (ty & 1) ? -1 : 1;
#else
        const int dir = 1;
#endif
        const int yfirst = dir > 0 ? y0 : y0 + nrows - 1;
        // psi beyond a wall: that of the wall row (mirror) or zero
        const bool pz = BCY == BC_WALLS_WET && M.psi_zero;

        const int x = x0 + lane;
        const bool active = x < nx;
        // column pulled by this lane: its own, or column 0 (periodic image)
        // for the first lane past the right edge of the lattice
        const int col = active ? x : (x == nx ? 0 : -1);
        // halo columns of the ring: x0 - 1 and x0 + TX (the latter only when
        // the tile's last column is inside the lattice)
#if LBK_HALO_SPLIT
        constexpr int HL = 0, HR = TX - 1;      // first lane of the first wave, last lane of the last wave
#else
        constexpr int HL = 0, HR = 1;
#endif
        int hcol = -1;
        if (lane == HL) hcol = (x0 == 0) ? nx - 1 : x0 - 1;
        if (lane == HR && x0 + TX <= nx) hcol = (x0 + TX == nx) ? 0 : x0 + TX;
        const int hent = (lane == HL) ? 0 : LW - 1;

        // The software-pipelined march keeps three rows of populations in
        // registers; it pays off for the FP64 velocity-shift step (three waves
        // per SIMD, two rows of loads in flight each) and is not used where
        // the extra registers would cost occupancy.
        constexpr bool PIPE = LBK_PIPE && ST == ST_F64 && FORCING == FORCE_SHIFT && !FIELDS;
        if constexpr (PIPE) {
        // Software-pipelined march: the populations of the row two ahead are
        // requested before the barrier and the collision of the current row,
        // so one row of loads is always in flight behind the arithmetic.  The
        // loop is unrolled three times with rotating register sets so that no
        // register holding an outstanding load is ever copied.
        // Every lane issues every load (idle lanes read column 0), so that
        // the only branches around loads are uniform ones.
        const int lcol = col >= 0 ? col : 0;
        C fa[2][NQ], fb[2][NQ], fc[2][NQ];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < NQ; ++i) fa[s][i] = fb[s][i] = fc[s][i] = (C)0;
        double rho_c[2] = {0.0, 0.0};   // rho of this lane's column at the current row
        double rho_h[2] = {0.0, 0.0};   // rho of the halo column at the last row fetched

        // --- prologue: the first row of the march (full) and the row behind
        // it (densities only).  Ring slot of march index k is (k + 1) & 3.
        pull_site<ST, BCY>(src, M, yfirst, lcol, fa);
        rho_c[0] = density(fa[0]);
        rho_c[1] = density(fa[1]);
        ring[1][0][lane + 1] = rho_c[0];
        ring[1][1][lane + 1] = rho_c[1];
        if (hcol >= 0) {
            C hf[2][NQ];
            pull_site<ST, BCY>(src, M, yfirst, hcol, hf);
            rho_h[0] = density(hf[0]);
            rho_h[1] = density(hf[1]);
            ring[1][0][hent] = rho_h[0];
            ring[1][1][hent] = rho_h[1];
        }
        {
            int yb = yfirst - dir;
            const bool mirror = ((yb < 0) || (yb >= ny)) && (BCY != BC_PERIODIC);
            if (yb < 0) yb += ny;
            if (yb >= ny) yb -= ny;
            {
                double r0 = pz ? 0.0 : rho_c[0], r1 = pz ? 0.0 : rho_c[1];
                if (!mirror) {
                    C hf[2][NQ];
                    pull_site<ST, BCY>(src, M, yb, lcol, hf);
                    r0 = density(hf[0]);
                    r1 = density(hf[1]);
                }
                ring[0][0][lane + 1] = r0;
                ring[0][1][lane + 1] = r1;
            }
            if (hcol >= 0) {
                double r0 = pz ? 0.0 : rho_h[0], r1 = pz ? 0.0 : rho_h[1];
                if (!mirror) {
                    C hf[2][NQ];
                    pull_site<ST, BCY>(src, M, yb, hcol, hf);
                    r0 = density(hf[0]);
                    r1 = density(hf[1]);
                }
                ring[0][0][hent] = r0;
                ring[0][1][hent] = r1;
            }
        }
        // request the row ahead of the first one (march index 1)
        {
            int y1 = yfirst + dir;
            const bool mirror = ((y1 < 0) || (y1 >= ny)) && (BCY != BC_PERIODIC);
            if (y1 < 0) y1 += ny;
            if (y1 >= ny) y1 -= ny;
            if (!mirror) pull_site<ST, BCY>(src, M, y1, lcol, fb);
        }

        // one march step: cf holds row r, nf the (requested) row r + 1; the
        // row r + 2 is requested into pf
        auto march = [&](int r, C (&cf)[2][NQ], C (&nf)[2][NQ], C (&pf)[2][NQ]) {
            const int y = yfirst + dir * r;
            int yn = y + dir;                   // the row ahead
            const int sn = (r + 2) & 3;         // its ring slot
            const bool mirror = ((yn < 0) || (yn >= ny)) && (BCY != BC_PERIODIC);
            if (yn < 0) yn += ny;
            if (yn >= ny) yn -= ny;
            // evaluated on every path (mirror rows then discard it) so that
            // nf's loads are known to have landed before nf becomes current
            double rn[2] = {density(nf[0]), density(nf[1])};
            if (mirror) {
                rn[0] = pz ? 0.0 : rho_c[0];
                rn[1] = pz ? 0.0 : rho_c[1];
            }
            ring[sn][0][lane + 1] = rn[0];
            ring[sn][1][lane + 1] = rn[1];
            if (hcol >= 0) {
                if (!mirror) {
                    C hf[2][NQ];
                    pull_site<ST, BCY>(src, M, yn, hcol, hf);
                    rho_h[0] = density(hf[0]);
                    rho_h[1] = density(hf[1]);
                }
                ring[sn][0][hent] = (mirror && pz) ? 0.0 : rho_h[0];
                ring[sn][1][hent] = (mirror && pz) ? 0.0 : rho_h[1];
            }
            if (r + 2 <= nrows) {
                // the row after next: inside the band, or the halo row beyond it
                int y2 = y + 2 * dir;
                const bool mirror2 = ((y2 < 0) || (y2 >= ny)) && (BCY != BC_PERIODIC);
                if (y2 < 0) y2 += ny;
                if (y2 >= ny) y2 -= ny;
                if (!mirror2) pull_site<ST, BCY>(src, M, y2, lcol, pf);
            }
            __syncthreads();
            if (active) {
                const int s0 = (r + 1) & 3;
                const int sp = dir > 0 ? sn : (r & 3);
                const int sm = dir > 0 ? (r & 3) : sn;
                row_update<ST, FORCING, FIELDS, LW>(M, ring, s0, sp, sm, lane + 1, x, y, wall_row<BCY>(M, y), cf, rho_c, dst, fo);
            }
            rho_c[0] = rn[0];
            rho_c[1] = rn[1];
        };
        // whole triples without branches inside (keeps the compiler's
        // tracking of outstanding loads exact), then the remainder
        int r = 0;
        for (; r + 3 <= nrows; r += 3) {
            march(r, fa, fb, fc);
            march(r + 1, fb, fc, fa);
            march(r + 2, fc, fa, fb);
        }
        if (r < nrows) {
            march(r, fa, fb, fc);
            if (r + 1 < nrows) march(r + 1, fb, fc, fa);
        }
        } else {
        C cur_f[2][NQ], nxt_f[2][NQ];
        double rho_c[2] = {0.0, 0.0};   // rho of this lane's column at the current row
        double rho_h[2] = {0.0, 0.0};   // rho of the halo column at the last row fetched

        // --- prologue: the first row of the march (full) and the row behind
        // it (densities only).  Ring slot of march index k is (k + 1) & 3.
        if (col >= 0) {
            pull_site<ST, BCY>(src, M, yfirst, col, cur_f);
            rho_c[0] = density(cur_f[0]);
            rho_c[1] = density(cur_f[1]);
            ring[1][0][lane + 1] = rho_c[0];
            ring[1][1][lane + 1] = rho_c[1];
        }
        if (hcol >= 0) {
            C hf[2][NQ];
            pull_site<ST, BCY>(src, M, yfirst, hcol, hf);
            rho_h[0] = density(hf[0]);
            rho_h[1] = density(hf[1]);
            ring[1][0][hent] = rho_h[0];
            ring[1][1][hent] = rho_h[1];
        }
        {
            // the row behind: a real row, a periodic image, or (walls) the
            // mirror of the first row
            int yb = yfirst - dir;
            const bool outside = (yb < 0) || (yb >= ny);
            const bool mirror = outside && (BCY != BC_PERIODIC);
            if (yb < 0) yb += ny;
            if (yb >= ny) yb -= ny;
            if (col >= 0) {
                double r0 = pz ? 0.0 : rho_c[0], r1 = pz ? 0.0 : rho_c[1];
                if (!mirror) {
                    C hf[2][NQ];
                    pull_site<ST, BCY>(src, M, yb, col, hf);
                    r0 = density(hf[0]);
                    r1 = density(hf[1]);
                }
                ring[0][0][lane + 1] = r0;
                ring[0][1][lane + 1] = r1;
            }
            if (hcol >= 0) {
                double r0 = pz ? 0.0 : rho_h[0], r1 = pz ? 0.0 : rho_h[1];
                if (!mirror) {
                    C hf[2][NQ];
                    pull_site<ST, BCY>(src, M, yb, hcol, hf);
                    r0 = density(hf[0]);
                    r1 = density(hf[1]);
                }
                ring[0][0][hent] = r0;
                ring[0][1][hent] = r1;
            }
        }

        // --- march through the band
        for (int r = 0; r < nrows; ++r) {
            const int y = yfirst + dir * r;
            int yn = y + dir;                   // the row ahead
            const int sn = (r + 2) & 3;         // its ring slot
            const bool outside = (yn < 0) || (yn >= ny);
            const bool mirror = outside && (BCY != BC_PERIODIC);
            if (yn < 0) yn += ny;
            if (yn >= ny) yn -= ny;
            double rn[2] = {pz ? 0.0 : rho_c[0], pz ? 0.0 : rho_c[1]};
            if (col >= 0 && !mirror) {
                pull_site<ST, BCY>(src, M, yn, col, nxt_f);
                rn[0] = density(nxt_f[0]);
                rn[1] = density(nxt_f[1]);
            }
            if (col >= 0) {
                ring[sn][0][lane + 1] = rn[0];
                ring[sn][1][lane + 1] = rn[1];
            }
            if (hcol >= 0) {
                if (!mirror) {
                    C hf[2][NQ];
                    pull_site<ST, BCY>(src, M, yn, hcol, hf);
                    rho_h[0] = density(hf[0]);
                    rho_h[1] = density(hf[1]);
                }
                ring[sn][0][hent] = (mirror && pz) ? 0.0 : rho_h[0];
                ring[sn][1][hent] = (mirror && pz) ? 0.0 : rho_h[1];
            }
            __syncthreads();

            if (active) {
                // ring slots of rows y - 1, y, y + 1
                const int s0 = (r + 1) & 3;
                const int sp = dir > 0 ? sn : (r & 3);
                const int sm = dir > 0 ? (r & 3) : sn;
                row_update<ST, FORCING, FIELDS, LW>(M, ring, s0, sp, sm, lane + 1, x, y, wall_row<BCY>(M, y), cur_f, rho_c, dst, fo);
            }
            // rotate: the row ahead becomes current
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                rho_c[s] = rn[s];
#pragma unroll
                for (int i = 0; i < NQ; ++i) cur_f[s][i] = nxt_f[s][i];
            }
        }
        }
        __syncthreads();   // the ring is reused by the next item
    }
}

// ---------------------------------------------------------------------------
// Two steps per pass (temporal blocking).
//
// A work item is one wave of 64 lanes; lane l holds column x0 - 3 + l (mod
// nx).  It marches through a band of rows evaluating, per row, step t -> t+1
// for all 64 columns (kept in registers, never stored) and, two rows behind,
// step t+1 -> t+2, whose pulled populations come from the neighbouring
// lanes' step-1 results.  Column neighbours (densities of both steps and the
// x-streaming of step 2) move between lanes with DPP wavefront shifts, so the
// pass needs no LDS and no barrier.  Lane l's step-1 result is valid for
// l in [1, 62], its step-2 pull and density for [2, 61] and its step-2
// result for [3, 60]: 58 output columns per item.  Every site goes through
// collide_site exactly as in k_step (step-1 results pass through the storage
// encoding), so one pass of two steps equals two passes of one step bit for
// bit.  Populations are read once and written once per two steps; the price
// is 4 extra step-1 rows per band and 6 extra step-1 columns per 58.
constexpr int TX2 = 58;                 // output columns per work item
#ifndef LBK_NW2
#define LBK_NW2 4
#endif
constexpr int NW2 = LBK_NW2;            // waves (work items) per workgroup of the two-step pass

// Resident waves per SIMD the two-step pass is held to, per storage mode (0:
// as many as its registers allow).  The FP64 pass needs 249 VGPRs (two
// waves); the FP32 pass needs about 150 and would run three waves, which
// keep more rows in flight per CU than its caches hold (measured 12 %
// slower at 10000 x 5000); the 16-bit passes are fastest at three.
template <int ST>
constexpr int fused_waves_per_simd()
{
    return ST == ST_F32 ? 2 : ((ST == ST_F16S || ST == ST_BF16S) ? 3 : 0);
}
// LDS a workgroup of the two-step pass reserves (unused) so that no more
// than fused_waves_per_simd waves per SIMD are resident: one byte more per
// workgroup than fits one extra workgroup into the 160 KB of a CU.
constexpr int LDS_PER_CU = 160 * 1024;
template <int ST>
constexpr int fused_lds_cap_floats()
{
    return fused_waves_per_simd<ST>() == 0 ? 0
                                           : (LDS_PER_CU / (4 * fused_waves_per_simd<ST>() / NW2 + 1) + 256) / 4;
}
constexpr int DPP_WAVE_SHL1 = 0x130;    // lane l receives lane l + 1 (column x + 1)
constexpr int DPP_WAVE_SHR1 = 0x138;    // lane l receives lane l - 1 (column x - 1)

// Lane shifts across the whole wave.  The two edge lanes have no source
// lane: they keep their own value (ZF = false) or receive 0 (ZF = true, the
// DPP move's bound control; the compiler then need not copy the source into
// the destination first).  Edge-lane values never reach an output column
// (three lanes of halo on either side), so both forms give the same results;
// the zero fill is what the 16-bit passes run faster with (fewer VALU
// instructions where VALU is the limit), the keeping form what the FP64 and
// FP32 passes do.
template <int CTRL, bool ZF = false>
__device__ __forceinline__ int lane_shift_b32(int b)
{
    if constexpr (ZF) return __builtin_amdgcn_update_dpp(0, b, CTRL, 0xF, 0xF, true);
    else return __builtin_amdgcn_update_dpp(b, b, CTRL, 0xF, 0xF, false);
}
template <int CTRL, bool ZF = false>
__device__ __forceinline__ double lane_shift(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t nlo = (uint32_t)lane_shift_b32<CTRL, ZF>((int)(uint32_t)u);
    const uint32_t nhi = (uint32_t)lane_shift_b32<CTRL, ZF>((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)nhi << 32) | nlo);
}
template <int CTRL, bool ZF = false>
__device__ __forceinline__ float lane_shift(float v)
{
    return __builtin_bit_cast(float, lane_shift_b32<CTRL, ZF>(__builtin_bit_cast(int, v)));
}
// value of the column to the left (x - 1) / right (x + 1)
template <bool ZF = false, class V> __device__ __forceinline__ V from_left(V v) { return lane_shift<DPP_WAVE_SHR1, ZF>(v); }
template <bool ZF = false, class V> __device__ __forceinline__ V from_right(V v) { return lane_shift<DPP_WAVE_SHL1, ZF>(v); }

// Eq. 5 sums of both components from the densities of rows y - 1, y, y + 1
// of this lane's column; the other columns come from the neighbouring lanes.
template <bool FACTORED, bool ZF = false>
__device__ __forceinline__ void sc_sums_lanes(const double (&lo)[2], const double (&mid)[2], const double (&hi)[2],
                                              double (&Sx)[2], double (&Sy)[2])
{
#pragma unroll
    for (int o = 0; o < 2; ++o)
        sc_sum<FACTORED>(from_right<ZF>(mid[o]), hi[o], from_left<ZF>(mid[o]), lo[o], from_right<ZF>(hi[o]),
                         from_left<ZF>(hi[o]), from_left<ZF>(lo[o]), from_right<ZF>(lo[o]), Sx[o], Sy[o]);
}

// Streamed value of population i for this lane's column from the same row
// of step-1 results: shifted by c_x (bounce-back values are not shifted).
template <int I, bool ZF = false, class V>
__device__ __forceinline__ V shift_x(V v)
{
    if constexpr (cx(I) > 0) return from_left<ZF>(v);
    else if constexpr (cx(I) < 0) return from_right<ZF>(v);
    else return v;
}

// One band of a pass of NS fused steps (NS = 2 or 3), marching in direction
// DIR (+1: up).  Per march index k (step-1 row a = first - 2 (NS - 1) DIR +
// k DIR) and stage j = 1 .. NS:
//   stage 1 collides row a from the pulled f(t) (rho(t) of a - DIR, a, a + DIR);
//   stage j > 1 pulls row p_j = a - (2 j - 3) DIR from the results of stage
//   j - 1 (rows p_j - DIR: its c_y = DIR populations, p_j: c_y = 0, and
//   p_j + DIR: c_y = -DIR), whose densities are then known, and collides row
//   q_j = a - 2 (j - 1) DIR, whose neighbours' densities are known from this
//   and the two previous pulls.  The results of every stage but the last stay
//   in registers, in the stored form (encoded and decoded as the next pass
//   would pull them), so the pass equals NS single steps bit for bit; the
//   last stage's are stored.
// Stage j collides rows from k = 4 (j - 1) on: the last stage covers the band,
// each earlier stage the rows the next one needs (two more on either side).
// The populations of row a + 2 DIR are requested right after the stage-1
// collision of row a, into the registers it has just consumed (two rotating
// sets); the last step-1 row requests none.  Only one pulled input row per
// stage is held: row p_j's densities are summed from its sources, and its
// populations are rebuilt (the same DPP moves again) after the collision of
// row q_j.  This keeps the FP64 two-step pass within 256 VGPRs, two waves per
// SIMD.
// A work item covers 66 - 4 NS output columns (2 NS - 1 lanes of halo on
// either side: each step's pull and Eq. 5 sums reach one lane further, and
// the first step's pull comes from memory) and a band whose f(t) rows extend
// 2 NS - 1 rows beyond it on either side.
template <int NS> constexpr int tx_of_pass() { return 66 - 4 * NS; }
static_assert(tx_of_pass<2>() == TX2, "the two-step window");

template <int ST, int FORCING, int BCY, int DIR, int NS>
__device__ __forceinline__ void marchN(const Member &M, int cur, int y0, int nrows, int c, bool store_ok)
{
    static_assert(NS == 2 || NS == 3, "two or three fused steps");
    using Q = Tr<ST>;
    using T = typename Q::T;
    using C = typename Q::C;
    // zero-filling lane shifts (no copy of each shifted value first): the
    // 16-bit two-step passes and every three-step pass are bound by their
    // instruction issue (FP64 three-step 33.8 -> 37.1 GLUPS, FP32 66.9 ->
    // 68.7 at 10000 x 5000); the memory-bound FP64 and FP32 two-step passes
    // measured no faster with it
    constexpr bool ZF = NS >= 3 || Q::SITE;
    constexpr int NK = NS - 1;              // stages whose results stay in registers
    const int ny = M.ny;
    const void *src = M.f[cur];
    void *dst = M.f[cur ^ 1];
    const int64_t row_bytes = M.ystride * (int64_t)sizeof(T);
    const unsigned ox = (unsigned)c * (unsigned)sizeof(T);
    const unsigned wis = (unsigned)M.istride * (unsigned)sizeof(T);
    const unsigned wss = (unsigned)M.sstride * (unsigned)sizeof(T);
    auto inside = [&](int v) { return BCY == BC_PERIODIC || (v >= 0 && v < ny); };
    const bool pz = BCY == BC_WALLS_WET && M.psi_zero;
    auto wrap = [&](int v) {
        if (BCY == BC_PERIODIC) {
            v %= ny;
            if (v < 0) v += ny;
        }
        return v;
    };
    constexpr int FW[3] = {DIR > 0 ? 2 : 4, DIR > 0 ? 5 : 7, DIR > 0 ? 6 : 8};
    constexpr int BW[3] = {DIR > 0 ? 4 : 2, DIR > 0 ? 7 : 5, DIR > 0 ? 8 : 6};

    C fa[2][NQ], fb[2][NQ];     // pulled f(t) of rows a and a + DIR
    C g[NK][2][NQ];             // g[j]: pulled input of stage j + 2 (row q_{j+2}, then the row it pulls next)
    C P[NK][2][NQ], Qv[NK][2][NQ];   // results of stage j + 1: the row behind its latest (c_y = 0, DIR) and the one before (c_y = DIR)
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            fa[s][i] = fb[s][i] = (C)0;
#pragma unroll
            for (int j = 0; j < NK; ++j) g[j][s][i] = P[j][s][i] = Qv[j][s][i] = (C)0;
        }
    // rm[j], rc[j]: densities after j steps of the rows behind and at the
    // row stage j + 1 collides next
    double rm[NS][2], rc[NS][2];
#pragma unroll
    for (int j = 0; j < NS; ++j) rm[j][0] = rm[j][1] = rc[j][0] = rc[j][1] = 0.0;

    const int first = DIR > 0 ? y0 : y0 + nrows - 1;
    const int a0 = first - 2 * (NS - 1) * DIR;
    if (inside(a0 - DIR)) {
        C hf[2][NQ];
        pull_site<ST, BCY>(src, M, wrap(a0 - DIR), c, hf);
        rm[0][0] = density(hf[0]);
        rm[0][1] = density(hf[1]);
    }
    if (inside(a0)) {
        pull_site<ST, BCY>(src, M, wrap(a0), c, fa);
        rc[0][0] = density(fa[0]);
        rc[0][1] = density(fa[1]);
    }
    if (inside(a0 + DIR)) pull_site<ST, BCY>(src, M, wrap(a0 + DIR), c, fb);
    const int K = nrows + 4 * (NS - 1);

    auto sums = [&](const double (&rb)[2], const double (&rcur)[2], const double (&rf)[2], double (&Sx)[2],
                    double (&Sy)[2]) {
        if constexpr (DIR > 0) sc_sums_lanes<ST != ST_F64, ZF>(rb, rcur, rf, Sx, Sy);
        else sc_sums_lanes<ST != ST_F64, ZF>(rf, rcur, rb, Sx, Sy);
    };
    auto collide_keep = [&](const C (&f)[2][NQ], const double (&rho)[2], const double (&Sx)[2], const double (&Sy)[2],
                            int row, C (&out)[2][NQ]) {
        collide_site<ST, FORCING>(M, f, rho, Sx, Sy, wall_row<BCY>(M, row), [&](int s, int i, C post) {
            if constexpr (Q::SITE) out[s][i] = post;
            else out[s][i] = Q::dec(Q::enc(post));
        });
        if constexpr (Q::SITE) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                typename Q::T qc[NQ];
                float rhat;
                site_encode<ST>(M, rho[s], out[s], qc, rhat);
#pragma unroll
                for (int i = 0; i < NQ; ++i) out[s][i] = site_decode<ST>(M, qc[i], rhat, i);
            }
        }
    };
    auto pull_rows = [&](int s, const C (&Qr)[2][NQ], const C (&Pr)[2][NQ], const C (&Or)[2][NQ], bool bbf, bool bbb,
                         C (&v)[NQ]) {
        v[0] = Pr[s][0];
        v[1] = shift_x<1, ZF>(Pr[s][1]);
        v[3] = shift_x<3, ZF>(Pr[s][3]);
        v[FW[0]] = Qr[s][FW[0]];
        v[FW[1]] = bbf ? Qr[s][FW[1]] : shift_x<FW[1], ZF>(Qr[s][FW[1]]);
        v[FW[2]] = bbf ? Qr[s][FW[2]] : shift_x<FW[2], ZF>(Qr[s][FW[2]]);
        v[BW[0]] = Or[s][BW[0]];
        v[BW[1]] = bbb ? Or[s][BW[1]] : shift_x<BW[1], ZF>(Or[s][BW[1]]);
        v[BW[2]] = bbb ? Or[s][BW[2]] : shift_x<BW[2], ZF>(Or[s][BW[2]]);
    };
    auto beyond = [&](bool in, const double (&r)[2], const double (&wall)[2], double (&out)[2]) {
#pragma unroll
        for (int s = 0; s < 2; ++s) out[s] = in ? r[s] : (pz ? 0.0 : wall[s]);
    };
    auto rotate = [&](C (&Pr)[2][NQ], C (&Qr)[2][NQ], const C (&out)[2][NQ], bool bb_next) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int j = 0; j < 3; ++j) Qr[s][FW[j]] = bb_next ? out[s][opp(FW[j])] : Pr[s][FW[j]];
            Pr[s][0] = out[s][0];
            Pr[s][1] = out[s][1];
            Pr[s][3] = out[s][3];
#pragma unroll
            for (int j = 0; j < 3; ++j) Pr[s][FW[j]] = out[s][FW[j]];
        }
    };

    auto iter = [&](int k, C (&f1c)[2][NQ], C (&f1n)[2][NQ]) {
        const int a = a0 + k * DIR;
        const bool load_next = k + 1 < K && inside(a + 2 * DIR);
        double rn[NS][2];           // densities after j steps of the row stage j + 1 pulls now
        rn[0][0] = density(f1n[0]);
        rn[0][1] = density(f1n[1]);
        C out[NK][2][NQ];           // this iteration's results of the kept stages
#pragma unroll
        for (int j = 0; j < NK; ++j)
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int i = 0; i < NQ; ++i) out[j][s][i] = (C)0;
        // --- stage 1 at row a
        if (inside(a)) {
            double rb[2], rf[2], Sx[2], Sy[2];
            beyond(inside(a - DIR), rm[0], rc[0], rb);
            beyond(inside(a + DIR), rn[0], rc[0], rf);
            sums(rb, rc[0], rf, Sx, Sy);
            collide_keep(f1c, rc[0], Sx, Sy, a, out[0]);
        } else if (BCY != BC_PERIODIC) {
            // beyond a wall: the pull of the row behind takes its c_y = -DIR
            // populations from its own reversed ones (bounce-back)
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int j = 0; j < 3; ++j) out[0][s][BW[j]] = P[0][s][opp(BW[j])];
        }
        if (load_next) pull_site<ST, BCY>(src, M, wrap(a + 2 * DIR), c, f1c);
        // --- stages 2 .. NS
#pragma unroll
        for (int j = 2; j <= NS; ++j) {
            const int p = a - (2 * j - 3) * DIR;     // the row stage j pulls now
            const int q = a - 2 * (j - 1) * DIR;     // the row stage j collides now
            const bool pull = k >= 4 * j - 6 && inside(p);
            const bool bbf = (BCY != BC_PERIODIC) && !inside(p - DIR);
            const bool bbb = (BCY != BC_PERIODIC) && !inside(p + DIR);
            rn[j - 1][0] = rn[j - 1][1] = 0.0;
            if (pull) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    C v[NQ];
                    pull_rows(s, Qv[j - 2], P[j - 2], out[j - 2], bbf, bbb, v);
                    rn[j - 1][s] = density(v);
                }
            }
            if (k >= 4 * (j - 1)) {
                if (j < NS) {
                    if (inside(q)) {
                        double rb[2], rf[2], Sx[2], Sy[2];
                        beyond(inside(q - DIR), rm[j - 1], rc[j - 1], rb);
                        beyond(inside(p), rn[j - 1], rc[j - 1], rf);
                        sums(rb, rc[j - 1], rf, Sx, Sy);
                        collide_keep(g[j - 2], rc[j - 1], Sx, Sy, q, out[j - 1]);
                    } else if (BCY != BC_PERIODIC) {
#pragma unroll
                        for (int s = 0; s < 2; ++s)
#pragma unroll
                            for (int i = 0; i < 3; ++i) out[j - 1][s][BW[i]] = P[j - 1][s][opp(BW[i])];
                    }
                } else {
                    // the last stage: row q lies inside the band
                    double rb[2], rf[2], Sx[2], Sy[2];
                    beyond(inside(q - DIR), rm[j - 1], rc[j - 1], rb);
                    beyond(inside(p), rn[j - 1], rc[j - 1], rf);
                    sums(rb, rc[j - 1], rf, Sx, Sy);
                    const rsrc_t wr = row_rsrc(dst, wrap(q), row_bytes);
                    if constexpr (Q::SITE) {
                        C post[2][NQ];
                        collide_site<ST, FORCING>(M, g[j - 2], rc[j - 1], Sx, Sy, wall_row<BCY>(M, q),
                                                  [&](int s, int i, C pv) { post[s][i] = pv; });
                        if (store_ok) store_site<ST>(M, wr, ox, c, wis, wss, rc[j - 1], post);
                    } else {
                        collide_site<ST, FORCING>(M, g[j - 2], rc[j - 1], Sx, Sy, wall_row<BCY>(M, q),
                                                  [&](int s, int i, C post) {
                            if (store_ok)
                                bstore<LBK_NT_STORE ? CPOL_NT : 0>(Q::enc(post), wr, ox,
                                                                    (unsigned)s * wss + (unsigned)i * wis);
                        });
                    }
                }
            }
            if (pull) {
#pragma unroll
                for (int s = 0; s < 2; ++s) pull_rows(s, Qv[j - 2], P[j - 2], out[j - 2], bbf, bbb, g[j - 2][s]);
            }
        }
        // --- rotate the kept stages' results and the densities
#pragma unroll
        for (int j = 1; j <= NK; ++j) {
            const int q = a - 2 * (j - 1) * DIR;
            rotate(P[j - 1], Qv[j - 1], out[j - 1], (BCY != BC_PERIODIC) && inside(q) && !inside(q - DIR));
        }
#pragma unroll
        for (int j = 0; j < NS; ++j)
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                rm[j][s] = rc[j][s];
                rc[j][s] = rn[j][s];
            }
    };
    int k = 0;
    for (; k + 2 <= K; k += 2) {
        iter(k, fa, fb);
        iter(k + 1, fb, fa);
    }
    if (k < K) iter(k, fa, fb);
}

// Two waves per SIMD: the FP64 pass then fits in 256 VGPRs without spills
// (left alone the compiler takes a few more and drops to one wave); three
// waves would need spills and measure much slower.
template <int ST, int FORCING, int BCY>
__global__ void __launch_bounds__(64 * NW2) __attribute__((amdgpu_waves_per_eu(2)))
k_step2(const Member *__restrict__ members, int n_members, int64_t item0, int64_t n_items, int cur)
{
    // NW2 waves per workgroup take NW2 consecutive items (neighbouring
    // column windows of a band, row-major over the members' bands), so that
    // waves that share cache lines start together on one CU.  Blocks of two
    // windows by two bands, or four bands, measured slower.
    const int lane = threadIdx.x & 63;
    // the wave index is uniform across the wave: keep it (and with it the
    // work item and everything derived from it) in scalar registers
    const int wave = NW2 == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if constexpr (fused_lds_cap_floats<ST>() > 0) {
        // reserved to cap the workgroups resident per CU; never read
        __shared__ float cap[fused_lds_cap_floats<ST>()];
        if (n_members < 0) cap[threadIdx.x] = 0.0f;
    }
    for (int64_t item = item0 + (int64_t)blockIdx.x * NW2 + wave; item < item0 + n_items;
         item += (int64_t)gridDim.x * NW2) {
        int m = 0;
        while (m + 1 < n_members && members[m].item2_end <= item) ++m;
        const Member &M = members[m];
        const int64_t t = item - M.item2_begin;
        const int tx = (int)(t % M.tiles_x2);
        const int ty = (int)(t / M.tiles_x2);
        const int x0 = tx * TX2;
        const int y0 = ty * M.tile_h2;
        const int nrows = min(M.tile_h2, M.ny - y0);
        const int xl = x0 - 3 + lane;
        int c = xl % M.nx;
        if (c < 0) c += M.nx;
        const bool store_ok = lane >= 3 && lane < 3 + TX2 && xl < M.nx;
#if LBK_ALT_DIR
        const bool down = (ty & 1) != 0;
#else
        const bool down = false;
#endif
        if (down) marchN<ST, FORCING, BCY, -1, 2>(M, cur, y0, nrows, c, store_ok);
        else marchN<ST, FORCING, BCY, 1, 2>(M, cur, y0, nrows, c, store_ok);
    }
}

// ---------------------------------------------------------------------------
// Three steps per pass: the march with a third stage (54 output columns per
// wave, ten extra f(t) rows per band).
constexpr int TX3 = tx_of_pass<3>();

// FP32 arithmetic: about 210 VGPRs, two waves per SIMD.  FP64: the two sets
// of pulled rows and two stages of results need about 350 registers, so the
// pass runs one wave per SIMD (256 VGPRs and the rest in AGPRs, no scratch);
// with taller bands it is still faster per step than the two-step pass at two
// waves.
template <int ST, int FORCING, int BCY>
__global__ void __launch_bounds__(64 * NW2) __attribute__((amdgpu_waves_per_eu(ST == ST_F64 ? 1 : 2)))
k_step3(const Member *__restrict__ members, int n_members, int64_t item0, int64_t n_items, int cur)
{
    // work items and their order as in k_step2
    const int lane = threadIdx.x & 63;
    const int wave = NW2 == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t item = item0 + (int64_t)blockIdx.x * NW2 + wave; item < item0 + n_items;
         item += (int64_t)gridDim.x * NW2) {
        int m = 0;
        while (m + 1 < n_members && members[m].item3_end <= item) ++m;
        const Member &M = members[m];
        const int64_t t = item - M.item3_begin;
        const int tx = (int)(t % M.tiles_x3);
        const int ty = (int)(t / M.tiles_x3);
        const int x0 = tx * TX3;
        const int y0 = ty * M.tile_h3;
        const int nrows = min(M.tile_h3, M.ny - y0);
        const int xl = x0 - 5 + lane;
        int c = xl % M.nx;
        if (c < 0) c += M.nx;
        const bool store_ok = lane >= 5 && lane < 5 + TX3 && xl < M.nx;
        if constexpr (ST == ST_F64) {
            // one march direction: the FP64 pass is bound by its instruction
            // issue, and with both directions its code (75 KB) overflows the
            // instruction cache; with tall bands the alternation that lets
            // neighbouring bands share halo rows in the caches gains less
            // (measured 3 % faster without it at 10000 x 5000)
            (void)ty;
            marchN<ST, FORCING, BCY, 1, 3>(M, cur, y0, nrows, c, store_ok);
        } else {
            if ((ty & 1) != 0) marchN<ST, FORCING, BCY, -1, 3>(M, cur, y0, nrows, c, store_ok);
            else marchN<ST, FORCING, BCY, 1, 3>(M, cur, y0, nrows, c, store_ok);
        }
    }
}

// ---------------------------------------------------------------------------
// State conversion between the canonical FP64 pre-collision populations
// f(t)[s][i][y][x] and the stored post-collision representation.
//
// Scatter (inverse of the pull): stored f*_i(z) = f_i(z + c_i) when z + c_i
// is a lattice site, else f_opp(i)(z) (the population that bounces back at z).
// With from_rho, the canonical populations are the rest equilibrium
// f_i = w_i rho_s (Eq. 3 with u = 0) of the given densities.
template <int ST, int BCY>
__global__ void k_scatter(const Member *__restrict__ members, int mi, const double *__restrict__ fcan,
                          const double *__restrict__ rhoA, const double *__restrict__ rhoB, int from_rho, int cur)
{
    const Member &M = members[mi];
    using Q = Tr<ST>;
    using T = typename Q::T;
    const int64_t n = (int64_t)M.nx * M.ny;
    LBK_GLOBAL T *dst = gp<T>(M.f[cur]);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / M.nx), x = (int)(k % M.nx);
        double v[2][NQ];   // the stored (post-collision) values of this site
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            int xs = x + cx(i), ys = y + cy(i);
            if (xs < 0) xs += M.nx;
            if (xs >= M.nx) xs -= M.nx;
            int isrc = i;
            if (BCY == BC_PERIODIC) {
                if (ys < 0) ys += M.ny;
                if (ys >= M.ny) ys -= M.ny;
            } else if (ys < 0 || ys >= M.ny) {
                xs = x;
                ys = y;
                isrc = opp(i);
            }
            const int64_t ks = (int64_t)ys * M.nx + xs;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (from_rho) v[s][i] = wgt(isrc) * (s == 0 ? rhoA[ks] : rhoB[ks]);
                else v[s][i] = fcan[((int64_t)s * NQ + isrc) * n + ks];
            }
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if constexpr (Q::SITE) {
                // the site's stored density: the sum of its stored populations
                double rho = v[s][0];
#pragma unroll
                for (int i = 1; i < NQ; ++i) rho += v[s][i];
                float post[NQ];
#pragma unroll
                for (int i = 0; i < NQ; ++i) post[i] = (float)v[s][i];
                T q[NQ];
                float rhat;
                site_encode<ST>(M, rho, post, q, rhat);
#pragma unroll
                for (int i = 0; i < NQ; ++i) dst[(int64_t)s * M.sstride + (int64_t)i * M.istride + (int64_t)y * M.ystride + x] = q[i];
                LBK_GLOBAL char *row = (LBK_GLOBAL char *)dst + (int64_t)y * M.ystride * (int64_t)sizeof(T);
                *(LBK_GLOBAL float *)(row + M.rho_off + (int64_t)s * M.rho_sstride + 4 * (int64_t)x) = rhat;
            } else {
#pragma unroll
                for (int i = 0; i < NQ; ++i)
                    dst[(int64_t)s * M.sstride + (int64_t)i * M.istride + (int64_t)y * M.ystride + x] =
                        Q::enc((typename Q::C)v[s][i]);
            }
        }
    }
}

// Gather: canonical f(t) = pull of the stored buffer, decoded to FP64.
template <int ST, int BCY>
__global__ void k_gather(const Member *__restrict__ members, int mi, double *__restrict__ fcan, int cur)
{
    const Member &M = members[mi];
    using Q = Tr<ST>;
    const int64_t n = (int64_t)M.nx * M.ny;
    const void *src = M.f[cur];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / M.nx), x = (int)(k % M.nx);
        typename Q::C f[2][NQ];
        pull_site<ST, BCY>(src, M, y, x, f);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < NQ; ++i) fcan[((int64_t)s * NQ + i) * n + k] = (double)f[s][i];
    }
}

// ---------------------------------------------------------------------------
// Energy-budget reductions (Sec. 3, Eq. 15-18 and Eq. 22) over the field
// buffer [rho_A | rho_B | u_x | u_y], each [ny][nx] FP64.  Pass 1: one
// workgroup per row writes that row's partial sums; every workgroup uses the
// same thread count and the same combining tree, so the result does not
// depend on the tile shape of the step.  Pass 2: one workgroup combines the
// rows in a fixed order.
//
// part[row][0..8] = sum rho_A, sum rho_B, sum phi (all columns),
//                   sum rho |u|^2 / 2, sum -y (rho_A gA_y + rho_B gB_y),
//                   sum -u . (rho_A gA + rho_B gB), sum omega^2   (rows of D only),
//                   max |u|, number of non-finite values.
constexpr int RED_THREADS = 256;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Combine one value per thread of a RED_THREADS block: wave shuffles, then
// the four wave results in order.  Result valid in thread 0.
template <bool MAX>
__device__ __forceinline__ double block_combine(double v, double *sh)
{
    v = MAX ? wave_max(v) : wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int k = 1; k < RED_THREADS / 64; ++k) r = MAX ? fmax(r, sh[k]) : r + sh[k];
    return r;
}

__global__ void __launch_bounds__(RED_THREADS)
k_reduce_rows(const double *__restrict__ rA, const double *__restrict__ rB, const double *__restrict__ ux,
              const double *__restrict__ uy, int nx, int ny, int trim, double gAx, double gAy, double gBx,
              double gBy, double *__restrict__ part)
{
    __shared__ double sh[RED_THREADS / 64];
    const int y = blockIdx.x;
    const bool inD = (y >= trim) && (y < ny - trim);
    const double yj = (double)y - 0.5 * (double)(ny - 1);
    double a[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int x = threadIdx.x; x < nx; x += RED_THREADS) {
        const int64_t k = (int64_t)y * nx + x;
        const double ra = rA[k], rb = rB[k], vx = ux[k], vy = uy[k];
        a[0] += ra;
        a[1] += rb;
        a[2] += ra - rb;
        const double um = sqrt(vx * vx + vy * vy);
        a[7] = fmax(a[7], um);
        if (!(isfinite(ra) && isfinite(rb) && isfinite(vx) && isfinite(vy))) a[8] += 1.0;
        if (inD) {
            const double rt = ra + rb;
            a[3] += 0.5 * rt * (vx * vx + vy * vy);
            const double fy = ra * gAy + rb * gBy;
            const double fx = ra * gAx + rb * gBx;
            a[4] += -yj * fy;
            a[5] += -(vx * fx + vy * fy);
            const int xp = (x + 1 == nx) ? 0 : x + 1, xm = (x == 0) ? nx - 1 : x - 1;
            const double dvy_dx = 0.5 * (uy[(int64_t)y * nx + xp] - uy[(int64_t)y * nx + xm]);
            const double dux_dy = 0.5 * (ux[(int64_t)(y + 1) * nx + x] - ux[(int64_t)(y - 1) * nx + x]);
            const double om = dvy_dx - dux_dy;
            a[6] += om * om;
        }
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const double r = (q == 7) ? block_combine<true>(a[q], sh) : block_combine<false>(a[q], sh);
        if (threadIdx.x == 0) part[(int64_t)y * RED_NQ + q] = r;
    }
}

// ---------------------------------------------------------------------------
// Kinetic-energy budget of Sec. 3 (Eq. 11-14, 17-19) from the field buffer
// by centred differences: d_x q = (q(x+1) - q(x-1)) / 2 (x periodic), d_y
// likewise, the five-point Laplacian, and the divergence of a tensor
// (div T)_b = d_x T_xb + d_y T_yb with the tensor formed at each site.  The
// terms reach two rows and columns away (trim >= 2).  Each site's
// expressions are evaluated in a fixed order:
//   pb    u . grad p_b,  p_b = c_s^2 rho + (G c_s^2 / 4)(rho^2 - phi^2)         (Eq. 12)
//   kort  u . div P^K,   P^K = [-kappa phi lap phi - (kappa/2)|grad phi|^2] I
//                              + kappa grad phi (x) grad phi                    (Eq. 13)
//   ktau  u . div K,     K = c_s^4 (rho_A rho_B / rho)(tau - 1/2)^2 h (x) h,
//                        h = grad rho_A / rho_A - grad rho_B / rho_B           (Eq. 14)
//   V     u . div(grad u + grad u^T)   (the viscous term of Eq. 17 over eta)
// Per band of rows: sum rho, then over the sites of D: sum pb, sum kort,
// sum ktau, sum V, sum -u . (rho_A gA + rho_B gB).
struct BudgetConst {
    double cs2;     // c_s^2
    double gc;      // G c_s^2 / 4
    double kappa;   // c_s^4 G / 4
    double c0;      // c_s^4
    double tf;      // (tau - 1/2)^2
    double gA[2], gB[2];
};
constexpr int BUDGET_NQ = 6;
constexpr int BT_W = 64;        // output columns of a tile
constexpr int BT_R = 4;         // output rows of a tile (BT_W * BT_R = RED_THREADS)
static_assert(BT_W * BT_R == RED_THREADS, "one thread per output site of a tile");

// One workgroup per band of BT_R rows of D; it walks the band in tiles of
// BT_W columns.  Per tile: (1) the four fields on the tile plus two halo rows
// and columns go to LDS; (2) the tensors p_b, P^K, K and grad u + grad u^T
// are formed once at every point of the tile plus one halo row and column;
// (3) each thread takes the divergences at its site.  part[band][q] as for
// the row kernel: [0] sums rho over the band's rows (the first and last
// bands also cover the trimmed rows), [1..5] the budget terms over D.
__global__ void __launch_bounds__(RED_THREADS)
k_budget_rows(const double *__restrict__ fld, int nx, int ny, int trim, BudgetConst K, double *__restrict__ part)
{
    constexpr int FW = BT_W + 4, FR = BT_R + 4;   // field tile with two halo columns / rows per side
    constexpr int TW = BT_W + 2, TR = BT_R + 2;   // tensor tile with one halo
    __shared__ double sf[4][FR][FW];              // rho_A, rho_B, u_x, u_y
    __shared__ double st[10][TR][TW];             // p_b, Pxx, Pxy, Pyy, Kxx, Kxy, Kyy, Sxx, Sxy, Syy
    __shared__ double sh[RED_THREADS / 64];
    const int64_t n = (int64_t)nx * ny;
    const int nD = ny - 2 * trim;
    const int nb = (nD + BT_R - 1) / BT_R;
    const int b = blockIdx.x;
    const int y0 = trim + b * BT_R;               // first output row of the band
    const int tid = threadIdx.x;
    double a[BUDGET_NQ] = {0, 0, 0, 0, 0, 0};

    // [0]: total density over the band's rows (whole lattice over all bands)
    {
        const int lo = b == 0 ? 0 : y0, hi = b == nb - 1 ? ny : min(y0 + BT_R, ny - trim);
        for (int64_t k = (int64_t)lo * nx + tid; k < (int64_t)hi * nx; k += RED_THREADS) a[0] += fld[k] + fld[n + k];
    }
    const int ty = tid / BT_W, tx = tid % BT_W;
    for (int x0 = 0; x0 < nx; x0 += BT_W) {
        // (1) fields of rows y0-2 .. y0+BT_R+1 and columns x0-2 .. x0+BT_W+1;
        // rows beyond the lattice only feed non-output rows and are clamped
        for (int e = tid; e < FR * FW; e += RED_THREADS) {
            const int r = e / FW, cc = e % FW;
            const int yy = min(max(y0 - 2 + r, 0), ny - 1);
            int xx = (x0 - 2 + cc) % nx;
            if (xx < 0) xx += nx;
            const int64_t k = (int64_t)yy * nx + xx;
#pragma unroll
            for (int q = 0; q < 4; ++q) sf[q][r][cc] = fld[q * n + k];
        }
        __syncthreads();
        // (2) tensors at tile rows -1 .. BT_R and columns -1 .. BT_W
        for (int e = tid; e < TR * TW; e += RED_THREADS) {
            const int r = e / TW + 1, cc = e % TW + 1;    // position in the field tile
            auto A = [&](int dr, int dc) { return sf[0][r + dr][cc + dc]; };
            auto B = [&](int dr, int dc) { return sf[1][r + dr][cc + dc]; };
            auto phi = [&](int dr, int dc) { return A(dr, dc) - B(dr, dc); };
            auto rho = [&](int dr, int dc) { return A(dr, dc) + B(dr, dc); };
            const int o = e / TW, w = e % TW;
            {
                const double rr = rho(0, 0), pp = phi(0, 0);
                st[0][o][w] = K.cs2 * rr + K.gc * (rr * rr - pp * pp);
            }
            {
                const double gx = 0.5 * (phi(0, 1) - phi(0, -1)), gy = 0.5 * (phi(1, 0) - phi(-1, 0));
                const double lap = phi(0, 1) + phi(0, -1) + phi(1, 0) + phi(-1, 0) - 4.0 * phi(0, 0);
                const double iso = -K.kappa * phi(0, 0) * lap - 0.5 * K.kappa * (gx * gx + gy * gy);
                st[1][o][w] = iso + K.kappa * gx * gx;
                st[2][o][w] = K.kappa * gx * gy;
                st[3][o][w] = iso + K.kappa * gy * gy;
            }
            {
                const double ra = A(0, 0), rb = B(0, 0);
                const double hx = 0.5 * (A(0, 1) - A(0, -1)) / ra - 0.5 * (B(0, 1) - B(0, -1)) / rb;
                const double hy = 0.5 * (A(1, 0) - A(-1, 0)) / ra - 0.5 * (B(1, 0) - B(-1, 0)) / rb;
                const double c = K.c0 * (ra * rb / (ra + rb)) * K.tf;
                st[4][o][w] = c * hx * hx;
                st[5][o][w] = c * hx * hy;
                st[6][o][w] = c * hy * hy;
            }
            {
                auto U = [&](int dr, int dc) { return sf[2][r + dr][cc + dc]; };
                auto V = [&](int dr, int dc) { return sf[3][r + dr][cc + dc]; };
                st[7][o][w] = 2.0 * (0.5 * (U(0, 1) - U(0, -1)));
                st[9][o][w] = 2.0 * (0.5 * (V(1, 0) - V(-1, 0)));
                st[8][o][w] = 0.5 * (V(0, 1) - V(0, -1)) + 0.5 * (U(1, 0) - U(-1, 0));
            }
        }
        __syncthreads();
        // (3) divergences at this thread's site
        const int y = y0 + ty, x = x0 + tx;
        if (y < ny - trim && x < nx) {
            const int o = ty + 1, w = tx + 1;
            const double u = sf[2][ty + 2][tx + 2], v = sf[3][ty + 2][tx + 2];
            auto div = [&](int cxx, int cxy, int cyy, double &dvx, double &dvy) {
                dvx = 0.5 * (st[cxx][o][w + 1] - st[cxx][o][w - 1]) + 0.5 * (st[cxy][o + 1][w] - st[cxy][o - 1][w]);
                dvy = 0.5 * (st[cxy][o][w + 1] - st[cxy][o][w - 1]) + 0.5 * (st[cyy][o + 1][w] - st[cyy][o - 1][w]);
            };
            a[1] += u * (0.5 * (st[0][o][w + 1] - st[0][o][w - 1])) + v * (0.5 * (st[0][o + 1][w] - st[0][o - 1][w]));
            double dvx, dvy;
            div(1, 2, 3, dvx, dvy);
            a[2] += u * dvx + v * dvy;
            div(4, 5, 6, dvx, dvy);
            a[3] += u * dvx + v * dvy;
            div(7, 8, 9, dvx, dvy);
            a[4] += u * dvx + v * dvy;
            const double ra = sf[0][ty + 2][tx + 2], rb = sf[1][ty + 2][tx + 2];
            const double fy = ra * K.gA[1] + rb * K.gB[1];
            const double fx = ra * K.gA[0] + rb * K.gB[0];
            a[5] += -(u * fx + v * fy);
        }
        __syncthreads();   // the tiles are rewritten for the next x0
    }
#pragma unroll
    for (int q = 0; q < BUDGET_NQ; ++q) {
        const double r = block_combine<false>(a[q], sh);
        if (tid == 0) part[(int64_t)b * RED_NQ + q] = r;
    }
}

// out[q] = sum over rows r < nr of part[r][q], q < NQV, in a fixed order.
template <int NQV>
__global__ void __launch_bounds__(RED_THREADS)
k_sum_rows(const double *__restrict__ part, int nr, double *__restrict__ out)
{
    __shared__ double sh[RED_THREADS / 64];
    double a[NQV];
#pragma unroll
    for (int q = 0; q < NQV; ++q) a[q] = 0.0;
    for (int y = threadIdx.x; y < nr; y += RED_THREADS) {
#pragma unroll
        for (int q = 0; q < NQV; ++q) a[q] += part[(int64_t)y * RED_NQ + q];
    }
#pragma unroll
    for (int q = 0; q < NQV; ++q) {
        const double r = block_combine<false>(a[q], sh);
        if (threadIdx.x == 0) out[q] = r;
    }
}

// ---------------------------------------------------------------------------
// Interface phi = rho_A - rho_B = 0 (Sec. 3, Eq. 20-21): crossings of the
// lattice lines in four directions, for the Cauchy-Crofton length.  A
// crossing is a pair of neighbouring sites with phi > 0 at exactly one of
// them; pairs count when both sites lie in D (rows [trim, ny - trim)), x is
// periodic.  Row r = y - trim of part holds the pairs (x, y)-(x+1, y),
// (x, y)-(x, y+1), (x, y)-(x+1, y+1) and (x+1, y)-(x, y+1) as integers in
// doubles (exact below 2^53).
constexpr int IFACE_NQ = 4;

__global__ void __launch_bounds__(RED_THREADS)
k_interface_rows(const double *__restrict__ fld, int nx, int ny, int trim, double *__restrict__ part)
{
    __shared__ double sh[RED_THREADS / 64];
    const int y = trim + blockIdx.x;
    const int64_t n = (int64_t)nx * ny;
    const double *rA = fld, *rB = fld + n;
    auto pos = [&](int yy, int xx) {
        const int64_t k = (int64_t)yy * nx + xx;
        return rA[k] - rB[k] > 0.0;
    };
    const bool next = y + 1 < ny - trim;
    double a[IFACE_NQ] = {0, 0, 0, 0};
    for (int x = threadIdx.x; x < nx; x += RED_THREADS) {
        const int xp = (x + 1 == nx) ? 0 : x + 1;
        const bool p00 = pos(y, x), p10 = pos(y, xp);
        a[0] += (p00 != p10) ? 1.0 : 0.0;
        if (next) {
            const bool p01 = pos(y + 1, x), p11 = pos(y + 1, xp);
            a[1] += (p00 != p01) ? 1.0 : 0.0;
            a[2] += (p00 != p11) ? 1.0 : 0.0;
            a[3] += (p10 != p01) ? 1.0 : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < IFACE_NQ; ++q) {
        const double r = block_combine<false>(a[q], sh);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * RED_NQ + q] = r;
    }
}

// ---------------------------------------------------------------------------
// Connected components of the two phases (Sec. 3, the topology change of the
// interface): the A-rich set phi > 0 and its complement inside D, sites
// joined to their row and column neighbours of the same phase (x periodic).
// Sites of D are numbered s = (y - trim) nx + x.  Union-find on parent[]:
// every root points to itself and every other entry to a smaller index.
// k_cc_hook joins the two ends of each same-phase edge by a compare-and-swap
// that re-parents a root only while it is still a root, so concurrent joins
// lose no link and one pass over the edges suffices.  Finds halve the path
// they walk (a non-root entry may always be replaced by its grandparent: an
// ancestor in the same tree with a smaller index), which keeps the trees
// shallow; k_cc_compress then points every entry at its root.

__device__ __forceinline__ int cc_load(const int *parent, int a)
{
    return __hip_atomic_load(parent + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int cc_find(const int *parent, int a)
{
    int p;
    while ((p = cc_load(parent, a)) != a) a = p;
    return a;
}

__device__ __forceinline__ int cc_find_halve(int *parent, int a)
{
    while (true) {
        const int p = cc_load(parent, a);
        if (p == a) return a;
        const int gp = cc_load(parent, p);
        if (gp != p) __hip_atomic_store(parent + a, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a = gp;
    }
}

__device__ __forceinline__ bool cc_phase(const double *rA, const double *rB, int64_t k) { return rA[k] - rB[k] > 0.0; }

__global__ void k_cc_init(int *__restrict__ parent, int64_t nsites)
{
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nsites; s += (int64_t)gridDim.x * blockDim.x)
        parent[s] = (int)s;
}

__global__ void k_cc_hook(const double *__restrict__ fld, int nx, int ny, int trim, int *parent)
{
    const int64_t n = (int64_t)nx * ny;
    const double *rA = fld, *rB = fld + n;
    const int nD = ny - 2 * trim;
    const int64_t nsites = (int64_t)nD * nx;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nsites; s += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(s / nx), x = (int)(s % nx);
        const int64_t k = (int64_t)(r + trim) * nx + x;
        const bool ph = cc_phase(rA, rB, k);
        int nb[2];
        int cnt = 0;
        const int xr = (x + 1 == nx) ? 0 : x + 1;
        if (cc_phase(rA, rB, (int64_t)(r + trim) * nx + xr) == ph) nb[cnt++] = r * nx + xr;
        if (r + 1 < nD && cc_phase(rA, rB, k + nx) == ph) nb[cnt++] = (r + 1) * nx + x;
        for (int e = 0; e < cnt; ++e) {
            int a = (int)s, b = nb[e];
            while (true) {
                a = cc_find_halve(parent, a);
                b = cc_find_halve(parent, b);
                if (a == b) break;
                if (a < b) {
                    const int t = a;
                    a = b;
                    b = t;
                }
                // hook root a under b if a is still a root
                int expected = a;
                if (__hip_atomic_compare_exchange_strong(parent + a, &expected, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT))
                    break;
            }
        }
    }
}

__global__ void k_cc_compress(int *parent, int64_t nsites)
{
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nsites; s += (int64_t)gridDim.x * blockDim.x) {
        const int r = cc_find_halve(parent, (int)s);
        __hip_atomic_store(parent + s, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Per row r of D: part[r][0] roots of phase A, [1] roots of phase B, [2]
// same-phase edges whose ends have different roots (0 when the union is
// complete).
__global__ void __launch_bounds__(RED_THREADS)
k_cc_rows(const double *__restrict__ fld, int nx, int ny, int trim, const int *__restrict__ parent,
          double *__restrict__ part)
{
    __shared__ double sh[RED_THREADS / 64];
    const int64_t n = (int64_t)nx * ny;
    const double *rA = fld, *rB = fld + n;
    const int nD = ny - 2 * trim;
    const int r = blockIdx.x;
    double a[3] = {0, 0, 0};
    for (int x = threadIdx.x; x < nx; x += RED_THREADS) {
        const int s = r * nx + x;
        const int64_t k = (int64_t)(r + trim) * nx + x;
        const bool ph = cc_phase(rA, rB, k);
        if (parent[s] == s) a[ph ? 0 : 1] += 1.0;
        const int root = cc_find(parent, s);
        const int xr = (x + 1 == nx) ? 0 : x + 1;
        if (cc_phase(rA, rB, (int64_t)(r + trim) * nx + xr) == ph && cc_find(parent, r * nx + xr) != root) a[2] += 1.0;
        if (r + 1 < nD && cc_phase(rA, rB, k + nx) == ph && cc_find(parent, s + nx) != root) a[2] += 1.0;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double v = block_combine<false>(a[q], sh);
        if (threadIdx.x == 0) part[(int64_t)r * RED_NQ + q] = v;
    }
}

// out[0..8] as part[] summed over rows (max for [7]); prof[y] = row mean of phi.
__global__ void __launch_bounds__(RED_THREADS)
k_reduce_final(const double *__restrict__ part, int nx, int ny, double *__restrict__ out, double *__restrict__ prof)
{
    __shared__ double sh[RED_THREADS / 64];
    double a[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int y = threadIdx.x; y < ny; y += RED_THREADS) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const double v = part[(int64_t)y * RED_NQ + q];
            a[q] = (q == 7) ? fmax(a[q], v) : a[q] + v;
        }
        if (prof) prof[y] = part[(int64_t)y * RED_NQ + 2] / (double)nx;
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const double r = (q == 7) ? block_combine<true>(a[q], sh) : block_combine<false>(a[q], sh);
        if (threadIdx.x == 0) out[q] = r;
    }
}

// Integral width of the mixing layer from the row profile of phi (Sec. 3
// follows the layer's growth; the width is read as the integral measure):
// c_j = clamp((phibar_j - lo) / (hi - lo), 0, 1) is the fraction of the
// phase that starts at the top, with lo, hi the bulk values of phibar, and
// out[0] = sum over the rows of D of 6 c_j (1 - c_j).  One workgroup.
__global__ void __launch_bounds__(RED_THREADS)
k_mixing_width(const double *__restrict__ prof, int ny, int trim, double lo, double hi, double *__restrict__ out)
{
    __shared__ double sh[RED_THREADS / 64];
    double a = 0.0;
    for (int y = trim + (int)threadIdx.x; y < ny - trim; y += RED_THREADS) {
        double c = (prof[y] - lo) / (hi - lo);
        if (c < 0.0) c = 0.0;            // comparisons, so that a NaN row stays NaN
        else if (c > 1.0) c = 1.0;
        a += 6.0 * c * (1.0 - c);
    }
    const double r = block_combine<false>(a, sh);
    if (threadIdx.x == 0) out[0] = r;
}

}  // namespace lbk
