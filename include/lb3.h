/*
 * lb3.h - C ABI of the three-dimensional (D3Q19) extension in liblb.so: the
 * two-component Shan-Chen lattice Boltzmann step of Tavares, Biferale,
 * Sbragaglia and Mailybaev (Sec. 2, Eq. 1-7) on the D3Q19 lattice, the
 * extension their closing section proposes.
 *
 * Model
 *   populations f_i^s(x, t), s in {A, B}, D3Q19 velocities c_i, i = 0..18:
 *   0 rest; 1..6 the axis links +x, -x, +y, -y, +z, -z; 7..18 the edge links
 *   (+x+y, -x-y), (+x-y, -x+y), (+x+z, -x-z), (+x-z, -x+z), (+y+z, -y-z),
 *   (+y-z, -y+z); weights 1/3, 1/18 (axes), 1/36 (edges), the isotropic set
 *   with c_s^2 = 1/3 (Eq. 4);
 *   rho_s = sum_i f_i^s, common velocity weighted by 1/tau_s       (Eq. 1)
 *   BGK relaxation towards f^eq(rho_s, u + tau_s F_s / rho_s)     (Eq. 2-3)
 *   F_s = -G_AB rho_s sum_i w_i rho_sbar(x + c_i) c_i + rho_s g_s  (Eq. 5, 7)
 *   (the velocity-shift forcing of the paper); x and z periodic; y closed by
 *   halfway bounce-back walls below row 0 and above row ny-1, with the
 *   neighbour density across a wall taken from the adjacent row (neutral
 *   wetting), or periodic.
 *
 * Conventions are those of lb.h: int32 status codes (LB_OK, LB_E*), messages
 * from lb_last_error(), caller-owned workspace and stream, asynchronous calls
 * unless stated.  Fields are [nz][ny][nx] doubles (x fastest), populations
 * [s][i][z][y][x] doubles, both describing the pre-collision state f(t).
 */
#ifndef LB3_H
#define LB3_H

#include <stddef.h>
#include <stdint.h>

#include "lb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb3_config {
    int32_t nx, ny, nz;      /* lattice; each >= 3, nx * ny * nz < 2^31 */
    int32_t bc_y;            /* LB_WALLS or LB_PERIODIC_Y */
    int32_t storage;         /* LB_F64 or LB_F32 (the arithmetic is FP64 in both) */
    int32_t diag_trim;       /* rows dropped next to each wall for the E_k average of
                                lb3_diagnostics (>= 0, ny > 2 * diag_trim) */
    int32_t two_pass;        /* 0 (default): one fused pass per step (a plane march
                                with the densities of four planes in LDS); 1: two
                                passes (densities, then force and collision); bit for
                                bit the same result */
    int32_t reserved;        /* must be 0 */
    double tau[2];           /* tau_A, tau_B > 1/2 (Eq. 2) */
    double G_AB;             /* Shan-Chen coupling of Eq. 5 */
    double g[2][3];          /* body acceleration of each component, {x, y, z} */
    const double *rhoA0;     /* host, [nz][ny][nx]: initial densities; f(0) = w_i rho_s */
    const double *rhoB0;
} lb3_config;

/* Averages at time t: masses over the whole lattice; E_k = <rho |u|^2 / 2>
 * over the rows [diag_trim, ny - diag_trim) of every plane, u the
 * hydrodynamic velocity (sum_s j_s + sum_s F_s / 2)/rho. */
typedef struct lb3_diag {
    int64_t t;
    double mass[2];          /* sum of rho_A, rho_B */
    double Ek;
    double umax;             /* max |u| over the whole lattice */
    int32_t finite;          /* 1 if every density and velocity is finite */
    int32_t reserved;
} lb3_diag;

typedef struct lb3_handle lb3_handle;

/* Bytes of device workspace lb3_init needs (0 if cfg is invalid): two
 * population buffers, a [nz][ny][2] FP64 density buffer and small tables. */
size_t lb3_workspace_bytes(const lb3_config *cfg);

/* Create a handle: copies the initial densities (host), writes
 * f(0) = w_i rho_s(0) (Eq. 3 at rest) into d_workspace (>= lb3_workspace_bytes
 * bytes, 256-byte aligned) and returns the handle at t = 0.  Synchronises the
 * stream once. */
int32_t lb3_init(const lb3_config *cfg, void *d_workspace, size_t bytes, void *hip_stream, lb3_handle **out);

/* Advance by n >= 0 time steps (Eq. 2).  Fused (default): one kernel pass
 * per step, a plane march that keeps the densities of four planes in LDS and
 * the pulled populations in registers.  Two passes: densities of the pulled
 * populations, then force, collision and store. */
int32_t lb3_step(lb3_handle *h, int64_t n);

/* rho_A, rho_B and the hydrodynamic velocity (u_x, u_y, u_z) of f(t) into
 * caller device buffers of nz*ny*nx doubles; any pointer may be NULL. */
int32_t lb3_fields(lb3_handle *h, double *d_rhoA, double *d_rhoB, double *d_ux, double *d_uy, double *d_uz);

/* Averages of lb3_diag into *out (host).  Synchronises the stream; returns
 * LB_ENONFINITE (after filling *out) if a density or velocity is not finite. */
int32_t lb3_diagnostics(lb3_handle *h, lb3_diag *out);

/* f(t) decoded to FP64 into a device buffer of 2*19*nz*ny*nx doubles. */
int32_t lb3_get_populations(lb3_handle *h, double *d_f);

/* Replace the state by d_f (device, layout as above) taken as f(t). */
int32_t lb3_set_populations(lb3_handle *h, const double *d_f);

/* Completed steps (-1 if h is not a live handle). */
int64_t lb3_time(const lb3_handle *h);

/* Waits for the stream and frees the handle; later calls return LB_ESTATE. */
int32_t lb3_destroy(lb3_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* LB3_H */
