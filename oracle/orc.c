/*
 * Reference oracle for the two-component D2Q9 Shan-Chen lattice Boltzmann
 * step (Tavares, Biferale, Sbragaglia, Mailybaev, "Validation and application
 * of the lattice Boltzmann algorithm for a turbulent immiscible
 * Rayleigh-Taylor system", Sec. 2 and Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU kernels against a plain,
 * slow, obviously correct FP64 implementation.  It shares no source with the
 * GPU library.
 *
 * Design rules of this file
 *   - FP64 everywhere, IEEE round-to-nearest, built with -ffp-contract=off and
 *     without -ffast-math.
 *   - The method is an iteration with no cheaper closed form, so the oracle
 *     takes the paper's steps in order: moments (Eq. 1), Shan-Chen force
 *     (Eq. 5) plus buoyancy (Eq. 7), velocity (Eq. 1), equilibrium (Eq. 3),
 *     BGK relaxation (Eq. 2), then streaming written in PUSH form
 *     f_i(x + c_i, t + 1) = f*_i(x, t), so that the GPU's pull indexing is
 *     checked by an independent formulation.
 *   - Each phase runs over the whole lattice before the next one starts.
 *     OpenMP splits rows; results do not depend on the thread count.
 *   - Reductions are serial, in row-major order, with Neumaier compensation.
 *
 * State: f[s][i][y][x], s in {0 = A, 1 = B}, i = 0..8, y = 0..ny-1,
 * x = 0..nx-1, contiguous.  f is the pre-collision population at time t,
 * i.e. the left-hand side of Eq. 2 after streaming.
 *
 * Readings of points the paper leaves open (each is also listed in the
 * design notes of the repository):
 *   - velocity order 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1)
 *     6:(-1,1) 7:(-1,-1) 8:(1,-1); the weights 4/9, 1/9, 1/36 are the unique
 *     solution of the isotropy conditions of Eq. 4 with c_s^2 = 1/3;
 *   - solid top and bottom use halfway bounce-back (walls half a link
 *     outside rows 0 and ny-1, zero wall velocity);
 *   - the neighbour density in Eq. 5 across a wall is by default the
 *     density of the adjacent fluid row (mirror), so that a uniform fluid
 *     feels no wall force, consistent with the neutral wetting
 *     G_Ab = G_Bb = 0 of Sec. 2; psi = 0 on the boundary nodes is the
 *     alternative (psi_wall = 1);
 *   - the boundary nodes S = 1 of Eq. 6 are the rows y = -1 and y = ny, so
 *     the fluid-boundary force acts on rows 0 and ny-1 only;
 *   - the sign of Eq. 5 is kept (G > 0 repels A from B);
 *   - besides the paper's velocity-shift forcing (Eq. 2-3) the oracle offers
 *     Guo forcing (Guo, Zheng and Shi 2002) with the common velocity
 *     u = (sum_s j_s + F/2) / rho in the equilibrium;
 *   - the hydrodynamic velocity reported by the diagnostics is
 *     u_phys = (sum_s j_s + sum_s F_s / 2) / rho under both schemes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 9

/* D2Q9 velocity set (Sec. 2: (0,0), (+-c,0), (0,+-c), (+-c,+-c), c = 1). */
static const int CX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Index of the reversed velocity, -c_i = c_opp[i]. */
static const int OPP[NQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* Weights from the isotropy conditions of Eq. 4 (c_s^2 = 1/3, sum w = 1). */
static const double W[NQ] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

typedef struct {
    int32_t nx, ny;
    int32_t forcing;    /* 0: velocity shift of Eq. 2-3; 1: Guo forcing */
    int32_t periodic_y; /* 0: bounce-back walls top and bottom; 1: periodic */
    double tau[2];      /* relaxation times tau_A, tau_B (Eq. 2) */
    double G;           /* coupling G_AB of Eq. 5 */
    double g[4];        /* body acceleration per component: gA_x, gA_y, gB_x, gB_y;
                           Eq. 7 is gA = (0, -g~), gB = (0, +g~) */
    double Gw[2];       /* fluid-boundary couplings G_Ab, G_Bb of Eq. 6 */
    int32_t psi_wall;   /* psi on boundary nodes in Eq. 5: 0 = the adjacent
                           fluid row (mirror), 1 = zero */
    int32_t pad_;
} orc_params;

static inline size_t fidx(const orc_params *p, int s, int i, int y, int x)
{
    return (((size_t)s * NQ + (size_t)i) * (size_t)p->ny + (size_t)y) * (size_t)p->nx + (size_t)x;
}

static inline size_t sidx(const orc_params *p, int y, int x)
{
    return (size_t)y * (size_t)p->nx + (size_t)x;
}

static inline int wrap(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void orc_constants(int32_t *cx, int32_t *cy, int32_t *opp, double *w)
{
    for (int i = 0; i < NQ; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        opp[i] = OPP[i];
        w[i] = W[i];
    }
}

/* Eq. 3: f_i^eq(rho, v) = rho w_i (1 + 3 c.v + 9/2 (c.v)^2 - 3/2 v.v), c = 1. */
void orc_equilibrium(double rho, double vx, double vy, double *feq)
{
    double vv = vx * vx + vy * vy;
    for (int i = 0; i < NQ; ++i) {
        double cv = CX[i] * vx + CY[i] * vy;
        feq[i] = rho * W[i] * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
    }
}

/* Fill f with the equilibrium of the given densities and a common velocity
 * (ux, uy may be NULL for a fluid at rest). */
void orc_fill_equilibrium(const orc_params *p, const double *rhoA, const double *rhoB,
                          const double *ux, const double *uy, double *f)
{
    const int nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        double feq[NQ];
        for (int x = 0; x < nx; ++x) {
            size_t k = sidx(p, y, x);
            double vx = ux ? ux[k] : 0.0, vy = uy ? uy[k] : 0.0;
            for (int s = 0; s < 2; ++s) {
                orc_equilibrium(s == 0 ? rhoA[k] : rhoB[k], vx, vy, feq);
                for (int i = 0; i < NQ; ++i) f[fidx(p, s, i, y, x)] = feq[i];
            }
        }
    }
}

/* Eq. 1: component densities rho_s = sum_i f_i^s and momenta j_s = sum_i f_i^s c_i,
 * summed in index order 0..8.  Arrays rho, jx, jy are [2][ny][nx]. */
static void moments(const orc_params *p, const double *f, double *rho, double *jx, double *jy)
{
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int s = 0; s < 2; ++s) {
                double r = 0.0, mx = 0.0, my = 0.0;
                for (int i = 0; i < NQ; ++i) {
                    double v = f[fidx(p, s, i, y, x)];
                    r += v;
                    mx += v * CX[i];
                    my += v * CY[i];
                }
                rho[s * n + sidx(p, y, x)] = r;
                jx[s * n + sidx(p, y, x)] = mx;
                jy[s * n + sidx(p, y, x)] = my;
            }
}

/* Solid indicator S of Eq. 6: with walls, the boundary nodes are the rows
 * y = -1 and y = ny just outside the fluid. */
static inline int solid_row(const orc_params *p, int y)
{
    return !p->periodic_y && (y < 0 || y >= p->ny);
}

/* Pseudopotential psi_s = rho_s (the choice stated under Eq. 5) at a lattice
 * point that may lie one row beyond a wall: x wraps; y either wraps
 * (periodic), or on a boundary node psi is that of the adjacent fluid row
 * (mirror) or zero, as p->psi_wall selects. */
static inline double psi_at(const orc_params *p, const double *rho_s, int y, int x)
{
    x = wrap(x, p->nx);
    if (p->periodic_y) {
        y = wrap(y, p->ny);
    } else if (solid_row(p, y)) {
        if (p->psi_wall) return 0.0;
        y = y < 0 ? 0 : p->ny - 1;
    }
    return rho_s[sidx(p, y, x)];
}

/* Eq. 5 + Eq. 7 + Eq. 6 per unit mass: with psi_s = rho_s the force
 * F_s = -G rho_s sum_i w_i psi_sbar(x + c_i) c_i + rho_s g_s
 *       - G_sb rho_s sum_i w_i S(x + c_i) c_i
 * is rho_s a_s with the acceleration
 * a_s = (-G sum_i w_i psi_sbar(x + c_i) c_i + g_s) - G_sb sum_i w_i S(x + c_i) c_i.
 * This writes a_s; F_s = rho_s a_s where the force itself is needed. */
static void accelerations(const orc_params *p, const double *rho, double *ax, double *ay)
{
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int s = 0; s < 2; ++s) {
                const double *other = rho + (size_t)(1 - s) * n;
                double sx = 0.0, sy = 0.0;
                for (int i = 0; i < NQ; ++i) {
                    double ps = psi_at(p, other, y + CY[i], x + CX[i]);
                    sx += W[i] * ps * CX[i];
                    sy += W[i] * ps * CY[i];
                }
                /* Eq. 6: boundary nodes among the neighbours */
                double wx = 0.0, wy = 0.0;
                for (int i = 0; i < NQ; ++i) {
                    double S = solid_row(p, y + CY[i]) ? 1.0 : 0.0;
                    wx += W[i] * S * CX[i];
                    wy += W[i] * S * CY[i];
                }
                ax[s * n + sidx(p, y, x)] = (-p->G * sx + p->g[2 * s + 0]) - p->Gw[s] * wx;
                ay[s * n + sidx(p, y, x)] = (-p->G * sy + p->g[2 * s + 1]) - p->Gw[s] * wy;
            }
}

/* Scratch layout used by one step: rho, jx, jy, ax, ay, each [2][ny][nx]. */
size_t orc_scratch_doubles(const orc_params *p)
{
    return (size_t)10 * (size_t)p->nx * (size_t)p->ny;
}

/* One time step t -> t+1: fout receives f(t+1).  scratch holds at least
 * orc_scratch_doubles(p) doubles.  fout must not alias f. */
void orc_step(const orc_params *p, const double *f, double *fout, double *scratch)
{
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    double *rho = scratch, *jx = scratch + 2 * n, *jy = scratch + 4 * n;
    double *ax = scratch + 6 * n, *ay = scratch + 8 * n;
    /* the factors 1/tau_s of Eq. 1 and Eq. 2 */
    const double itau[2] = {1.0 / p->tau[0], 1.0 / p->tau[1]};

    moments(p, f, rho, jx, jy);
    accelerations(p, rho, ax, ay);

#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const size_t k = sidx(p, y, x);
            const double rA = rho[k], rB = rho[n + k];
            /* Velocities entering the equilibrium. */
            double ux, uy;
            /* F_s = rho_s a_s */
            const double FxA = rA * ax[k], FxB = rB * ax[n + k];
            const double FyA = rA * ay[k], FyB = rB * ay[n + k];
            if (p->forcing == 0) {
                /* Eq. 1: common velocity weighted by 1/tau_s. */
                double num_x = jx[k] * itau[0] + jx[n + k] * itau[1];
                double num_y = jy[k] * itau[0] + jy[n + k] * itau[1];
                double den = rA * itau[0] + rB * itau[1];
                ux = num_x / den;
                uy = num_y / den;
            } else {
                /* Guo: common velocity including half the total force. */
                double rt = rA + rB;
                ux = (jx[k] + jx[n + k] + 0.5 * (FxA + FxB)) / rt;
                uy = (jy[k] + jy[n + k] + 0.5 * (FyA + FyB)) / rt;
            }
            for (int s = 0; s < 2; ++s) {
                const double r = rho[s * n + k];
                const double fx = s == 0 ? FxA : FxB, fy = s == 0 ? FyA : FyB;
                const double tau = p->tau[s];
                const double omega = itau[s];
                double vx = ux, vy = uy;
                if (p->forcing == 0) {
                    /* Eq. 3: shifted velocity u' = u + tau_s F_s / rho_s
                     * = u + tau_s a_s. */
                    vx = ux + tau * ax[s * n + k];
                    vy = uy + tau * ay[s * n + k];
                }
                double feq[NQ];
                orc_equilibrium(r, vx, vy, feq);
                for (int i = 0; i < NQ; ++i) {
                    const double fi = f[fidx(p, s, i, y, x)];
                    /* Eq. 2: BGK relaxation towards the equilibrium. */
                    double post = fi - omega * (fi - feq[i]);
                    if (p->forcing == 1) {
                        /* Guo source (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F_s */
                        double cu = CX[i] * ux + CY[i] * uy;
                        double ex = 3.0 * (CX[i] - ux) + 9.0 * cu * CX[i];
                        double ey = 3.0 * (CY[i] - uy) + 9.0 * cu * CY[i];
                        post += (1.0 - 0.5 / tau) * W[i] * (ex * fx + ey * fy);
                    }
                    /* Streaming, push form: f_i(x + c_i, t+1) = f*_i(x, t). */
                    int xd = wrap(x + CX[i], nx);
                    int yd = y + CY[i];
                    if (p->periodic_y) {
                        fout[fidx(p, s, i, wrap(yd, ny), xd)] = post;
                    } else if (yd < 0 || yd >= ny) {
                        /* Halfway bounce-back: the population returns to its
                         * own site with the reversed velocity. */
                        fout[fidx(p, s, OPP[i], y, x)] = post;
                    } else {
                        fout[fidx(p, s, i, yd, xd)] = post;
                    }
                }
            }
        }
    }
}

/* Advance f in place by nsteps.  Returns 0, or -1 on allocation failure. */
int orc_run(const orc_params *p, double *f, int64_t nsteps)
{
    if (nsteps <= 0) return 0;
    const size_t nf = (size_t)2 * NQ * (size_t)p->nx * (size_t)p->ny;
    double *g = (double *)malloc(nf * sizeof(double));
    double *scratch = (double *)malloc(orc_scratch_doubles(p) * sizeof(double));
    if (!g || !scratch) {
        free(g);
        free(scratch);
        return -1;
    }
    double *cur = f, *nxt = g;
    for (int64_t t = 0; t < nsteps; ++t) {
        orc_step(p, cur, nxt, scratch);
        double *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    if (cur != f) memcpy(f, cur, nf * sizeof(double));
    free(g);
    free(scratch);
    return 0;
}

/* Macroscopic fields at time t: rhoA, rhoB, hydrodynamic velocity
 * u_phys = (j_A + j_B + (F_A + F_B)/2) / rho, and the total force
 * F_A + F_B.  Any output pointer may be NULL.  Returns -1 on allocation
 * failure. */
int orc_macro(const orc_params *p, const double *f, double *rhoA, double *rhoB, double *ux,
              double *uy, double *Ftx, double *Fty)
{
    const size_t n = (size_t)p->nx * p->ny;
    double *scratch = (double *)malloc(orc_scratch_doubles(p) * sizeof(double));
    if (!scratch) return -1;
    double *rho = scratch, *jx = scratch + 2 * n, *jy = scratch + 4 * n;
    double *ax = scratch + 6 * n, *ay = scratch + 8 * n;
    moments(p, f, rho, jx, jy);
    accelerations(p, rho, ax, ay);
    for (size_t k = 0; k < n; ++k) {
        double rt = rho[k] + rho[n + k];
        /* F_s = rho_s a_s */
        const double FxA = rho[k] * ax[k], FxB = rho[n + k] * ax[n + k];
        const double FyA = rho[k] * ay[k], FyB = rho[n + k] * ay[n + k];
        if (rhoA) rhoA[k] = rho[k];
        if (rhoB) rhoB[k] = rho[n + k];
        if (ux) ux[k] = (jx[k] + jx[n + k] + 0.5 * (FxA + FxB)) / rt;
        if (uy) uy[k] = (jy[k] + jy[n + k] + 0.5 * (FyA + FyB)) / rt;
        if (Ftx) Ftx[k] = FxA + FxB;
        if (Fty) Fty[k] = FyA + FyB;
    }
    free(scratch);
    return 0;
}

/* Neumaier-compensated running sum. */
typedef struct {
    double s, c;
} nsum;

static inline void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static inline double nsum_get(const nsum *a) { return a->s + a->c; }

/*
 * Energy-budget diagnostics at time t (Sec. 3, Eq. 15-18 and Eq. 22).
 * Averages <.> run over the trimmed subdomain D made of rows
 * [trim, ny - trim) and all columns (the paper drops the 10 rows nearest to
 * each wall).  Derivatives are centred differences with x wrapping.
 *
 * out[0..7] = M_A, M_B (sums over the whole lattice),
 *             E_k = <rho |u|^2 / 2>,
 *             E_p = -<y sum_s rho_s g_s,y>   (= g~ <y phi> for Eq. 7),
 *             B   = -<u . sum_s rho_s g_s>   (= g~ <phi u_y>, the rate of E_p),
 *             Z   = <omega^2>, omega = d_x u_y - d_y u_x,
 *             max |u| over the whole lattice,
 *             1.0 if every density and velocity is finite, else 0.0.
 * y is measured from the centre line: y_j = j - (ny - 1)/2.
 * phi_profile (may be NULL) receives the row means of phi = rho_A - rho_B
 * for every row j = 0..ny-1.
 * Returns 0, -1 on allocation failure, -2 if D is empty.
 */
int orc_diagnostics(const orc_params *p, const double *f, int32_t trim, double *out,
                    double *phi_profile)
{
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    if (trim < 1 || ny - 2 * trim <= 0) return -2;
    double *buf = (double *)malloc(4 * n * sizeof(double));
    if (!buf) return -1;
    double *rA = buf, *rB = buf + n, *ux = buf + 2 * n, *uy = buf + 3 * n;
    if (orc_macro(p, f, rA, rB, ux, uy, NULL, NULL)) {
        free(buf);
        return -1;
    }
    nsum mA = {0, 0}, mB = {0, 0}, ek = {0, 0}, ep = {0, 0}, bu = {0, 0}, z = {0, 0};
    double umax = 0.0;
    int finite = 1;
    for (int y = 0; y < ny; ++y) {
        nsum prof = {0, 0};
        for (int x = 0; x < nx; ++x) {
            size_t k = sidx(p, y, x);
            nsum_add(&mA, rA[k]);
            nsum_add(&mB, rB[k]);
            nsum_add(&prof, rA[k] - rB[k]);
            if (!isfinite(rA[k]) || !isfinite(rB[k]) || !isfinite(ux[k]) || !isfinite(uy[k]))
                finite = 0;
            double um = sqrt(ux[k] * ux[k] + uy[k] * uy[k]);
            if (um > umax) umax = um;
        }
        if (phi_profile) phi_profile[y] = nsum_get(&prof) / nx;
    }
    const double yc = 0.5 * (ny - 1);
    for (int y = trim; y < ny - trim; ++y) {
        const double yj = (double)y - yc;
        for (int x = 0; x < nx; ++x) {
            size_t k = sidx(p, y, x);
            double rt = rA[k] + rB[k];
            nsum_add(&ek, 0.5 * rt * (ux[k] * ux[k] + uy[k] * uy[k]));
            double fy_ext = rA[k] * p->g[1] + rB[k] * p->g[3];
            double fx_ext = rA[k] * p->g[0] + rB[k] * p->g[2];
            nsum_add(&ep, -yj * fy_ext);
            nsum_add(&bu, -(ux[k] * fx_ext + uy[k] * fy_ext));
            double dvy_dx = 0.5 * (uy[sidx(p, y, wrap(x + 1, nx))] - uy[sidx(p, y, wrap(x - 1, nx))]);
            double dux_dy = 0.5 * (ux[sidx(p, y + 1, x)] - ux[sidx(p, y - 1, x)]);
            double om = dvy_dx - dux_dy;
            nsum_add(&z, om * om);
        }
    }
    const double nd = (double)nx * (double)(ny - 2 * trim);
    out[0] = nsum_get(&mA);
    out[1] = nsum_get(&mB);
    out[2] = nsum_get(&ek) / nd;
    out[3] = nsum_get(&ep) / nd;
    out[4] = nsum_get(&bu) / nd;
    out[5] = nsum_get(&z) / nd;
    out[6] = umax;
    out[7] = finite ? 1.0 : 0.0;
    free(buf);
    return 0;
}
