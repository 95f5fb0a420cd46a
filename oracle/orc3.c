/*
 * Reference oracle for the three-dimensional extension of the two-component
 * Shan-Chen lattice Boltzmann step (Tavares, Biferale, Sbragaglia, Mailybaev,
 * Sec. 2, Eq. 1-7, on the D3Q19 lattice that the paper's closing section
 * names as the next step).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: tests compare the GPU library's 3D step with it.  It
 * shares no source with the GPU library.
 *
 * The method is the one of the two-dimensional oracle with the D2Q9 set
 * replaced by D3Q19: moments (Eq. 1), Shan-Chen acceleration
 * a_s = -G sum_i w_i rho_sbar(x + c_i) c_i + g_s (Eq. 5 with psi_s = rho_s,
 * plus Eq. 7), the common velocity weighted by 1/tau_s (Eq. 1), equilibrium
 * (Eq. 3, unchanged in form since c_s^2 = 1/3) at the shifted velocity
 * u + tau_s a_s, BGK relaxation (Eq. 2), then streaming in PUSH form.
 * FP64, -ffp-contract=off, phases over the whole lattice in turn.
 *
 * Readings (the paper gives no 3D details):
 *   - velocity order: 0 rest; 1..6 the axis links (+x, -x, +y, -y, +z, -z);
 *     7..18 the edge links in the pairs (+x+y, -x-y), (+x-y, -x+y),
 *     (+x+z, -x-z), (+x-z, -x+z), (+y+z, -y-z), (+y-z, -y+z); the weights
 *     1/3, 1/18, 1/36 are the solution of the isotropy conditions of Eq. 4
 *     with c_s^2 = 1/3;
 *   - gravity along y as in 2D; x and z periodic; y either periodic or
 *     closed by halfway bounce-back walls half a link outside rows 0 and
 *     ny-1, with psi across a wall taken from the adjacent fluid row;
 *   - the hydrodynamic velocity reported is (sum_s j_s + sum_s F_s / 2)/rho.
 *
 * State: f[s][i][z][y][x], s in {A, B}, i = 0..18; fields [z][y][x].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ3 19

static const int CX[NQ3] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[NQ3] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[NQ3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const int OPP[NQ3] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
static const double W[NQ3] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                              1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

typedef struct {
    int32_t nx, ny, nz;
    int32_t periodic_y; /* 0: bounce-back walls below row 0 and above row ny-1 */
    double tau[2];      /* tau_A, tau_B (Eq. 2) */
    double G;           /* G_AB of Eq. 5 */
    double g[6];        /* body acceleration: gA (x, y, z), gB (x, y, z) */
} orc3_params;

static inline size_t sid(const orc3_params *p, int z, int y, int x)
{
    return ((size_t)z * (size_t)p->ny + (size_t)y) * (size_t)p->nx + (size_t)x;
}

static inline size_t fid(const orc3_params *p, int s, int i, int z, int y, int x)
{
    const size_t n = (size_t)p->nx * (size_t)p->ny * (size_t)p->nz;
    return ((size_t)s * NQ3 + (size_t)i) * n + sid(p, z, y, x);
}

static inline int wrap(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

void orc3_constants(int32_t *cx, int32_t *cy, int32_t *cz, int32_t *opp, double *w)
{
    for (int i = 0; i < NQ3; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        cz[i] = CZ[i];
        opp[i] = OPP[i];
        w[i] = W[i];
    }
}

/* Eq. 3 on D3Q19: f_i^eq = rho w_i (1 + 3 c.v + 9/2 (c.v)^2 - 3/2 v.v). */
static void equilibrium(double rho, double vx, double vy, double vz, double *feq)
{
    double vv = vx * vx + vy * vy + vz * vz;
    for (int i = 0; i < NQ3; ++i) {
        double cv = CX[i] * vx + CY[i] * vy + CZ[i] * vz;
        feq[i] = rho * W[i] * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
    }
}

/* f = equilibrium of the given densities at rest. */
void orc3_fill_equilibrium(const orc3_params *p, const double *rhoA, const double *rhoB, double *f)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; ++k) {
        double feq[NQ3];
        for (int s = 0; s < 2; ++s) {
            equilibrium(s == 0 ? rhoA[k] : rhoB[k], 0.0, 0.0, 0.0, feq);
            for (int i = 0; i < NQ3; ++i) f[(size_t)(s * NQ3 + i) * n + k] = feq[i];
        }
    }
}

/* Eq. 1: rho_s and j_s, sums over i in index order. Arrays [2][n] (j: 3 arrays). */
static void moments(const orc3_params *p, const double *f, double *rho, double *jx, double *jy, double *jz)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; ++k)
        for (int s = 0; s < 2; ++s) {
            double r = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
            for (int i = 0; i < NQ3; ++i) {
                double v = f[(size_t)(s * NQ3 + i) * n + k];
                r += v;
                mx += v * CX[i];
                my += v * CY[i];
                mz += v * CZ[i];
            }
            rho[s * n + k] = r;
            jx[s * n + k] = mx;
            jy[s * n + k] = my;
            jz[s * n + k] = mz;
        }
}

/* psi_s = rho_s at a neighbour: x and z wrap; y wraps or mirrors onto the
 * adjacent fluid row. */
static inline double psi_at(const orc3_params *p, const double *rho_s, int z, int y, int x)
{
    x = wrap(x, p->nx);
    z = wrap(z, p->nz);
    if (p->periodic_y)
        y = wrap(y, p->ny);
    else if (y < 0)
        y = 0;
    else if (y >= p->ny)
        y = p->ny - 1;
    return rho_s[sid(p, z, y, x)];
}

/* Eq. 5 + Eq. 7 per unit mass: a_s = -G sum_i w_i rho_sbar(x + c_i) c_i + g_s. */
static void accelerations(const orc3_params *p, const double *rho, double *a)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x)
                for (int s = 0; s < 2; ++s) {
                    const double *other = rho + (size_t)(1 - s) * n;
                    double sx = 0.0, sy = 0.0, sz = 0.0;
                    for (int i = 0; i < NQ3; ++i) {
                        double ps = psi_at(p, other, z + CZ[i], y + CY[i], x + CX[i]);
                        sx += W[i] * ps * CX[i];
                        sy += W[i] * ps * CY[i];
                        sz += W[i] * ps * CZ[i];
                    }
                    const size_t k = sid(p, z, y, x);
                    a[(size_t)(3 * s + 0) * n + k] = -p->G * sx + p->g[3 * s + 0];
                    a[(size_t)(3 * s + 1) * n + k] = -p->G * sy + p->g[3 * s + 1];
                    a[(size_t)(3 * s + 2) * n + k] = -p->G * sz + p->g[3 * s + 2];
                }
}

/* Scratch: rho[2], j[2][3], a[2][3] per site. */
size_t orc3_scratch_doubles(const orc3_params *p)
{
    return (size_t)14 * (size_t)p->nx * p->ny * p->nz;
}

/* One time step: fout = f(t + 1).  fout must not alias f. */
void orc3_step(const orc3_params *p, const double *f, double *fout, double *scratch)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t n = (size_t)nx * ny * nz;
    double *rho = scratch, *jx = scratch + 2 * n, *jy = scratch + 4 * n, *jz = scratch + 6 * n;
    double *a = scratch + 8 * n;
    const double itau[2] = {1.0 / p->tau[0], 1.0 / p->tau[1]};

    moments(p, f, rho, jx, jy, jz);
    accelerations(p, rho, a);

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t k = sid(p, z, y, x);
                /* Eq. 1: common velocity weighted by 1/tau_s */
                const double den = rho[k] * itau[0] + rho[n + k] * itau[1];
                const double ux = (jx[k] * itau[0] + jx[n + k] * itau[1]) / den;
                const double uy = (jy[k] * itau[0] + jy[n + k] * itau[1]) / den;
                const double uz = (jz[k] * itau[0] + jz[n + k] * itau[1]) / den;
                for (int s = 0; s < 2; ++s) {
                    /* Eq. 3: shifted velocity u + tau_s a_s */
                    const double vx = ux + p->tau[s] * a[(size_t)(3 * s + 0) * n + k];
                    const double vy = uy + p->tau[s] * a[(size_t)(3 * s + 1) * n + k];
                    const double vz = uz + p->tau[s] * a[(size_t)(3 * s + 2) * n + k];
                    double feq[NQ3];
                    equilibrium(rho[s * n + k], vx, vy, vz, feq);
                    for (int i = 0; i < NQ3; ++i) {
                        const double fi = f[fid(p, s, i, z, y, x)];
                        /* Eq. 2 */
                        const double post = fi - itau[s] * (fi - feq[i]);
                        /* streaming, push form */
                        const int xd = wrap(x + CX[i], nx), zd = wrap(z + CZ[i], nz);
                        const int yd = y + CY[i];
                        if (p->periodic_y)
                            fout[fid(p, s, i, zd, wrap(yd, ny), xd)] = post;
                        else if (yd < 0 || yd >= ny)
                            fout[fid(p, s, OPP[i], z, y, x)] = post;   /* halfway bounce-back */
                        else
                            fout[fid(p, s, i, zd, yd, xd)] = post;
                    }
                }
            }
}

int orc3_run(const orc3_params *p, double *f, int64_t nsteps)
{
    if (nsteps <= 0) return 0;
    const size_t nf = (size_t)2 * NQ3 * (size_t)p->nx * p->ny * p->nz;
    double *g = (double *)malloc(nf * sizeof(double));
    double *scratch = (double *)malloc(orc3_scratch_doubles(p) * sizeof(double));
    if (!g || !scratch) {
        free(g);
        free(scratch);
        return -1;
    }
    double *cur = f, *nxt = g;
    for (int64_t t = 0; t < nsteps; ++t) {
        orc3_step(p, cur, nxt, scratch);
        double *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    if (cur != f) memcpy(f, cur, nf * sizeof(double));
    free(g);
    free(scratch);
    return 0;
}

/* Fields of f: rhoA, rhoB, hydrodynamic velocity (sum j + sum F / 2)/rho and
 * the total force sum_s rho_s a_s.  Any output may be NULL. */
int orc3_macro(const orc3_params *p, const double *f, double *rhoA, double *rhoB, double *ux, double *uy,
               double *uz, double *Fx, double *Fy, double *Fz)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    double *scratch = (double *)malloc(orc3_scratch_doubles(p) * sizeof(double));
    if (!scratch) return -1;
    double *rho = scratch, *jx = scratch + 2 * n, *jy = scratch + 4 * n, *jz = scratch + 6 * n;
    double *a = scratch + 8 * n;
    moments(p, f, rho, jx, jy, jz);
    accelerations(p, rho, a);
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; ++k) {
        const double rA = rho[k], rB = rho[n + k];
        const double fx = rA * a[k] + rB * a[3 * n + k];
        const double fy = rA * a[n + k] + rB * a[4 * n + k];
        const double fz = rA * a[2 * n + k] + rB * a[5 * n + k];
        const double rt = rA + rB;
        if (rhoA) rhoA[k] = rA;
        if (rhoB) rhoB[k] = rB;
        if (ux) ux[k] = (jx[k] + jx[n + k] + 0.5 * fx) / rt;
        if (uy) uy[k] = (jy[k] + jy[n + k] + 0.5 * fy) / rt;
        if (uz) uz[k] = (jz[k] + jz[n + k] + 0.5 * fz) / rt;
        if (Fx) Fx[k] = fx;
        if (Fy) Fy[k] = fy;
        if (Fz) Fz[k] = fz;
    }
    free(scratch);
    return 0;
}
