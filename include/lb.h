/*
 * lb.h - C ABI of liblb.so, a gfx950 (MI355X) implementation of the
 * two-component D2Q9 Shan-Chen lattice Boltzmann time step used by Tavares,
 * Biferale, Sbragaglia and Mailybaev for 2D Rayleigh-Taylor turbulence
 * ("Validation and application of the lattice Boltzmann algorithm for a
 * turbulent immiscible Rayleigh-Taylor system"), with the energy-budget
 * averages of its Sec. 3.
 *
 * Model (Sec. 2 of the paper)
 *   populations f_i^s(x, t), s in {A, B}, D2Q9 velocities c_i, i = 0..8 in
 *   the order (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1),
 *   weights 4/9, 1/9 (axes), 1/36 (diagonals);
 *   rho_s = sum_i f_i^s, common velocity weighted by 1/tau_s       (Eq. 1)
 *   BGK relaxation towards f^eq(rho_s, u + tau_s F_s / rho_s)     (Eq. 2-3)
 *   F_s = -G_AB rho_s sum_i w_i rho_sbar(x + c_i) c_i + rho_s g_s  (Eq. 5, 7)
 *   periodic in x; bounce-back walls below row 0 and above row ny-1 (or
 *   periodic in y for validation runs).
 *
 * Conventions
 *   - Every function returns an int32 status: LB_OK (0) or a negative
 *     LB_E* code; lb_last_error() then holds a message for the calling
 *     thread.  No C++ exception crosses this interface.
 *   - Device pointers are HIP device addresses on the current device;
 *     host pointers are ordinary process memory.  Fields are [ny][nx]
 *     row-major doubles (x fastest), populations [s][i][y][x] doubles.
 *   - Time t counts completed steps.  Every output describes the
 *     pre-collision state f(t) (after streaming), i.e. the left-hand side of
 *     Eq. 2 at time t.
 *   - Ownership: the caller owns the workspace (device memory of
 *     lb_workspace_bytes bytes) and the HIP stream; both must outlive the
 *     handle.  The library owns the host-side handle and any HIP graphs it
 *     builds; lb_destroy releases them.  Inputs are copied during the call
 *     that receives them.
 *   - All work is enqueued on the handle's stream.  lb_step, lb_fields,
 *     lb_get_populations and lb_set_populations never synchronise;
 *     lb_diagnostics synchronises the stream before returning.
 *   - A handle may be used from one host thread at a time.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define LB_OK 0
#define LB_EINVAL (-1)      /* invalid argument (message names it) */
#define LB_ENOMEM (-2)      /* workspace smaller than lb_workspace_bytes */
#define LB_EHIP (-3)        /* a HIP runtime call failed (message holds its error string) */
#define LB_ESTATE (-4)      /* handle unknown or already destroyed */
#define LB_ENONFINITE (-5)  /* lb_diagnostics found a NaN or Inf density or velocity */
#define LB_EINTERNAL (-6)   /* an algorithm of the library did not complete (message says
                               which); no HIP call failed */

/* Forcing scheme.  LB_FORCE_SHIFT is the paper's velocity shift inside the
 * equilibrium (Eq. 2-3).  LB_FORCE_GUO is Guo's forcing (Guo, Zheng and Shi,
 * 2002) with the common velocity (sum_s j_s + F/2)/rho in the equilibrium and
 * the source (1 - 1/(2 tau_s)) w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F_s;
 * it requires tau_A == tau_B. */
#define LB_FORCE_SHIFT 0
#define LB_FORCE_GUO 1

/* Storage of the populations between steps.  Densities, the Shan-Chen force
 * and every diagnostic sum are computed in FP64 in all modes.
 *   LB_F64   FP64 storage, FP64 arithmetic throughout (144 B per site).
 *   LB_F32   FP32 storage, FP32 collision (72 B per site).
 *   LB_F16S  per site and component, the FP32 density rhat_s(x) and IEEE
 *            binary16 codes q_i = (f*_i - w_i rhat_s) * scale_{s,i} of the
 *            populations, FP32 collision (44 B per site).
 *   LB_BF16S the same with bfloat16 codes.
 * A stored population decodes as f*_i = w_i rhat_s(x) + q_i / scale_{s,i}: the
 * codes hold only each population's departure from w_i times its own site's
 * density (the velocity and non-equilibrium parts), and rhat_s is set when
 * the codes are written so that the decoded populations of a site sum to its
 * density, so rounding the codes changes no component's mass.
 * scale_{s,i} is a power of two chosen at lb_init (lb_storage_scale). */
#define LB_F64 0
#define LB_F32 1
#define LB_F16S 2
#define LB_BF16S 3

/* Top/bottom boundary.  LB_WALLS: halfway bounce-back, no slip, walls half a
 * link outside rows 0 and ny-1; the boundary nodes (S = 1 in Eq. 6) are the
 * rows y = -1 and y = ny.  LB_PERIODIC_Y: periodic in y (validation runs
 * only; no boundary nodes). */
#define LB_WALLS 0
#define LB_PERIODIC_Y 1

/* psi of the other component on boundary nodes in the Shan-Chen sum of
 * Eq. 5.  LB_PSI_MIRROR: the density of the adjacent fluid row, so that a
 * uniform fluid feels no wall force (the neutral wetting of Sec. 2 with
 * G_Ab = G_Bb = 0).  LB_PSI_ZERO: zero (the solid holds no fluid); wetting is
 * then set by G_Ab, G_Bb of Eq. 6. */
#define LB_PSI_MIRROR 0
#define LB_PSI_ZERO 1

#define LB_MAX_MEMBERS 64

/* One independent realisation (ensemble member). */
typedef struct lb_member {
    int32_t nx, ny;          /* lattice size; nx >= 3, ny >= 3 */
    double tau[2];           /* relaxation times tau_A, tau_B > 1/2 (Eq. 2) */
    double G_AB;             /* Shan-Chen coupling of Eq. 5 (G > 0 repels A from B) */
    double g[2][2];          /* body acceleration of each component, g[s] = {x, y};
                                Eq. 7 is g[0] = {0, -g~}, g[1] = {0, +g~} */
    const double *rhoA0;     /* host, [ny][nx]: initial densities; f(0) = w_i rho_s */
    const double *rhoB0;
    double reserved2[2];     /* must be 0 */
    double G_wall[2];        /* fluid-boundary couplings G_Ab, G_Bb of Eq. 6 (finite;
                                used with LB_WALLS): row 0 gets the acceleration
                                +G_sb/6 and row ny-1 -G_sb/6 along y (exactly
                                -G_sb sum_i w_i S(x + c_i) c_i); G > 0 repels */
    int32_t wall_psi;        /* LB_PSI_MIRROR (0) or LB_PSI_ZERO */
    int32_t reserved;        /* must be 0 */
} lb_member;

typedef struct lb_config {
    int32_t n_members;       /* 1 .. LB_MAX_MEMBERS */
    const lb_member *members;
    int32_t forcing;         /* LB_FORCE_* */
    int32_t storage;         /* LB_F64 .. LB_BF16S, shared by all members */
    int32_t bc_y;            /* LB_WALLS or LB_PERIODIC_Y */
    int32_t diag_trim;       /* rows dropped at top and bottom for the averages of
                                lb_diagnostics (the paper drops 10); >= 1 */
    int32_t tile_x;          /* workgroup width in columns: 64, 128, 256 or 512;
                                0 chooses by timing candidates at lb_init */
    int32_t tile_h;          /* rows per tile (>= 1); 0 chooses with tile_x */
    int32_t graph_chunk;     /* steps per captured HIP graph (even, >= 2);
                                0 selects 100; negative disables graphs */
    int32_t steps_per_pass;  /* time steps per kernel pass over the lattice:
                                1, 2 (two steps fused in registers, so the
                                populations cross HBM once per two steps) or 3
                                (three steps).  A remainder of lb_step
                                shorter than a pass takes a two-step pass and
                                single steps; bit for bit the same result.  0
                                chooses by timing when tile_x == 0, else 1.
                                With 2 or 3, tile_x is ignored and tile_h (0 =
                                timed) is the band height of the fused pass */
} lb_config;

/* Energy-budget averages at time t (Sec. 3, Eq. 15-18 and Eq. 22).  <.> is
 * the mean over the trimmed domain D: rows [diag_trim, ny - diag_trim), all
 * columns.  u is the hydrodynamic velocity (sum_s j_s + sum_s F_s / 2)/rho,
 * y_j = j - (ny - 1)/2, derivatives are centred differences (x wraps). */
typedef struct lb_diag {
    int64_t t;
    double mass[2];          /* sum of rho_A, rho_B over the whole lattice */
    double Ek;               /* <rho |u|^2 / 2> */
    double Ep;               /* -<y sum_s rho_s g_s,y>, equal to g~ <y phi> for Eq. 7 */
    double buoyancy;         /* -<u . sum_s rho_s g_s>, equal to g~ <phi u_y>: dE_p/dt of Eq. 16 */
    double omega2;           /* <omega^2>, omega = d_x u_y - d_y u_x; the viscous
                                term of Eq. 22 is -eta * omega2 */
    double umax;             /* max |u| over the whole lattice */
    int32_t finite;          /* 1 if every density and velocity is finite */
} lb_diag;

typedef struct lb_handle lb_handle;

/* Bytes of device workspace lb_init needs for cfg (0 if cfg is invalid;
 * lb_last_error says why).  Every member's two population buffers, one
 * [4][ny][nx] FP64 field buffer of the largest member and small tables. */
size_t lb_workspace_bytes(const lb_config *cfg);

/* Create a handle.  Copies the member table and the initial densities,
 * lays out d_workspace (caller-owned, >= lb_workspace_bytes(cfg) bytes,
 * 256-byte aligned), writes f(0) = w_i rho_s(0) for every member (Eq. 3 at
 * rest), picks tile shapes (from the tile cache, see lb_tiles_cached, or by
 * timing candidates if tile_x or tile_h is 0, which advances no state) and
 * returns the handle in *out at t = 0.  hip_stream is a hipStream_t (NULL =
 * the null stream).  Synchronises the stream once. */
int32_t lb_init(const lb_config *cfg, void *d_workspace, size_t bytes, void *hip_stream,
                lb_handle **out);

/* Advance every member by n >= 0 time steps (Eq. 2), asynchronously on the
 * handle's stream.  Full chunks of graph_chunk steps replay a HIP graph. */
int32_t lb_step(lb_handle *h, int64_t n);

/* Macroscopic fields of member m at the current time into caller device
 * buffers of ny*nx doubles each: rho_A, rho_B and the hydrodynamic velocity
 * (u_x, u_y).  Any pointer may be NULL to skip that field.  Asynchronous. */
int32_t lb_fields(lb_handle *h, int32_t m, double *d_rhoA, double *d_rhoB, double *d_ux,
                  double *d_uy);

/* Energy-budget averages of member m (see lb_diag) into *out (host), and,
 * if phi_profile (host, ny doubles) is not NULL, the row means of
 * phi = rho_A - rho_B.  Synchronises the stream.  Returns LB_ENONFINITE
 * (after filling *out) if a density or velocity is not finite. */
int32_t lb_diagnostics(lb_handle *h, int32_t m, lb_diag *out, double *phi_profile);

/* Width of the mixing layer of member m at time t.  Sec. 3 follows the
 * growth of the layer between the two pure phases; its width is taken here
 * as the integral measure over the rows j of the trimmed domain D
 *   h = sum_j 6 c_j (1 - c_j),  c_j = clamp((phibar_j - lo) / (hi - lo), 0, 1),
 * with phibar_j the mean of phi = rho_A - rho_B over row j (the profile of
 * lb_diagnostics) and lo, hi the bulk references: phibar at the first and the
 * last row of D (rows diag_trim and ny - diag_trim - 1).  c_j is the fraction
 * of the phase that starts at the top; a pure row adds 0, a linear ramp of c
 * over m rows m + 1/(2m), a tanh profile of width w about 3w. */
typedef struct lb_mixing {
    int64_t t;
    double width;            /* h */
    double bulk_ref[2];      /* the lo, hi used */
} lb_mixing;

/* Mixing width of member m (see lb_mixing) into *out (host).  ref (host, two
 * doubles lo, hi) gives the bulk references; NULL takes those recorded by
 * lb_init from the initial state (t = 0).  LB_EINVAL if they are not finite
 * or equal.  Uses the workspace field buffer.  Synchronises the stream. */
int32_t lb_mixing_width(lb_handle *h, int32_t m, const double *ref, lb_mixing *out);

/* Largest ny accepted by lb_diagnostics_noalloc. */
#define LB_NOALLOC_MAX_NY 16384

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * averages of lb_diagnostics computed from caller fields, with no handle, no
 * workspace and no allocation of any kind.  d_rhoA, d_rhoB, d_ux, d_uy are
 * device [ny][nx] doubles as lb_fields writes them (u the hydrodynamic
 * velocity); g[4] = {gA_x, gA_y, gB_x, gB_y} are the body accelerations of
 * Eq. 7 (host); trim as lb_config.diag_trim; hip_stream a hipStream_t (NULL =
 * the null stream).  *out (host) receives the lb_diag averages with t = 0,
 * phi_profile (host, ny doubles, or NULL) the row means of phi.
 * The per-row partial sums live in a fixed scratch area inside the library
 * (about 1.3 MB per GPU, held until the process ends): ny above
 * LB_NOALLOC_MAX_NY returns LB_EINVAL.  All calls on one GPU share that
 * area, so calls that overlap on one GPU (other host threads, other
 * streams) race; calls in sequence on one stream do not.  Synchronises the
 * stream.  Returns LB_ENONFINITE (after filling *out) if a value is not
 * finite. */
int32_t lb_diagnostics_noalloc(const double *d_rhoA, const double *d_rhoB, const double *d_ux, const double *d_uy,
                               int32_t nx, int32_t ny, int32_t trim, const double *g, void *hip_stream,
                               lb_diag *out, double *phi_profile);

/* Terms of the kinetic-energy balance (Sec. 3, Eq. 17) of member m at time t,
 * averaged like lb_diag over the trimmed domain D, from the fields of
 * lb_fields by centred differences (d_x q = (q(x+1) - q(x-1))/2, x periodic;
 * five-point Laplacian; (div T)_b = d_x T_xb + d_y T_yb):
 *   dE_k/dt = -(pb + korteweg + ktau) + viscous - buoyancy,
 * the momentum-flux split of Eq. 19 with P = p_b I + P^K + K^(tau) (Eq. 11). */
typedef struct lb_budget {
    int64_t t;
    double pb;               /* <u . grad p_b>, p_b = c_s^2 rho + (G c_s^2/4)(rho^2 - phi^2) (Eq. 12) */
    double korteweg;         /* <u . div P^K>, P^K = [-kappa phi lap phi - (kappa/2)|grad phi|^2] I
                                + kappa grad phi (x) grad phi, kappa = c_s^4 G / 4 (Eq. 13) */
    double ktau;             /* <u . div K^(tau)>, K^(tau) = c_s^4 (rho_A rho_B / rho)(tau - 1/2)^2 h (x) h,
                                h = grad rho_A / rho_A - grad rho_B / rho_B (Eq. 14) */
    double viscous;          /* <u . div(eta grad u + eta grad u^T)> (Eq. 17) */
    double eta;              /* eta = mean(rho) c_s^2 (tau - 1/2), tau = (tau_A + tau_B)/2 */
    double buoyancy;         /* as lb_diag.buoyancy */
} lb_budget;

/* Energy-budget terms of member m (see lb_budget) into *out (host).  Needs
 * diag_trim >= 2 (the stencils reach two rows; LB_EINVAL otherwise).  Uses
 * the same workspace field buffer as lb_diagnostics.  Synchronises the
 * stream. */
int32_t lb_energy_budget(lb_handle *h, int32_t m, lb_budget *out);

/* Interface phi = rho_A - rho_B = 0 of member m at time t (Sec. 3, Eq. 20-21):
 * crossings of the lattice lines, counted as neighbouring site pairs with
 * phi > 0 at exactly one site, both sites in the trimmed domain D (x
 * periodic), and the Cauchy-Crofton length of the interface inside D. */
typedef struct lb_interface {
    int64_t t;
    int64_t crossings[4];    /* along rows (x, x+1), columns (y, y+1), and the
                                diagonals (x, y)-(x+1, y+1) and (x+1, y)-(x, y+1) */
    double length;           /* (pi/8) [N_rows + N_cols + (N_diag1 + N_diag2) / sqrt(2)] */
} lb_interface;

/* Interface crossings and length of member m (see lb_interface) into *out
 * (host).  Uses the workspace field buffer.  Synchronises the stream. */
int32_t lb_interface_length(lb_handle *h, int32_t m, lb_interface *out);

/* Topology of the two phases of member m at time t (Sec. 3): the numbers of
 * connected components of the A-rich set phi > 0 and of its complement
 * phi <= 0 inside the trimmed domain D, sites joined to their row and column
 * neighbours of the same phase, x periodic. */
typedef struct lb_topology {
    int64_t t;
    int64_t components[2];   /* [0]: phi > 0, [1]: phi <= 0 */
} lb_topology;

/* Component counts of member m (see lb_topology) into *out (host).  Uses
 * the workspace field buffer (the densities and 4 B per site of D for the
 * union-find parents).  Synchronises the stream.  LB_EINTERNAL if the
 * labelling left neighbouring sites of one phase in different components. */
int32_t lb_components(lb_handle *h, int32_t m, lb_topology *out);

/* Populations f(t) of member m, decoded to FP64, into a caller device buffer
 * of 2*9*ny*nx doubles, layout [s][i][y][x].  Asynchronous. */
int32_t lb_get_populations(lb_handle *h, int32_t m, double *d_f);

/* Replace the state of member m by the populations d_f (device, layout as
 * above) taken as f(t) at the current time.  Encoded to the storage mode.
 * Asynchronous; d_f may be reused once the stream has passed this call. */
int32_t lb_set_populations(lb_handle *h, int32_t m, const double *d_f);

/* Completed steps (-1 if h is not a live handle). */
int64_t lb_time(const lb_handle *h);

/* Tile shape of member m in the pass lb_step runs: columns per workgroup
 * (shared by all members: one launch covers them all; 58 / 54 output columns
 * per 64-lane wave for two- / three-step passes) and rows per tile (chosen per
 * member size class when tuned). */
int32_t lb_tile_shape(const lb_handle *h, int32_t m, int32_t *tile_x, int32_t *tile_h);

/* Time steps per kernel pass of lb_step: 1, 2 or 3 (negative: error code). */
int32_t lb_steps_per_pass(const lb_handle *h);

/* 1 if lb_init took the pass and tile shapes from the persisted tile cache,
 * 0 if it timed them (or they were given), negative: error code.  The cache
 * is a JSON file keyed by the device (architecture, compute units), the
 * version of the search, storage, forcing, boundary variant, the requested
 * steps_per_pass / tile_x / tile_h and every member's nx, ny: the
 * environment variable LB_TILE_CACHE names
 * it ("off" or empty: no cache), by default $XDG_CACHE_HOME/liblb/tiles.json
 * or $HOME/.cache/liblb/tiles.json.  A choice that is timed is recorded
 * there; a cached choice gives the same results bit for bit (tile shapes
 * never change results). */
int32_t lb_tiles_cached(const lb_handle *h);

/* Storage scale of member m for the 16-bit modes: scale[s*9 + i] receives
 * scale_{s,i} and weight[s*9 + i] the factor w_i (rounded to FP32) of the
 * per-site shift w_i rhat_s(x) (host arrays of 18; either may be NULL).  In
 * LB_F64 / LB_F32 the scales are 1 and the weights 0. */
int32_t lb_storage_scale(const lb_handle *h, int32_t m, double *scale, double *weight);

/* Destroy a handle: waits for its stream, frees graphs and host state.  The
 * workspace stays with the caller.  Later calls with h return LB_ESTATE. */
int32_t lb_destroy(lb_handle *h);

/* Message of the last failed call on this thread ("" if none). */
const char *lb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
