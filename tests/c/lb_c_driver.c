/*
 * Drives liblb.so through its C ABI from a plain C program: no Python, no
 * PyTorch.  The program allocates the workspace and a stream with the HIP
 * runtime, creates a one-member lattice from the densities in an input
 * file, advances it, and writes the canonical populations f(t), the fields
 * and the lb_diag averages to an output file for the test to compare with
 * the oracle.
 *
 * usage: lb_c_driver IN OUT STEPS FORCING BC_Y STEPS_PER_PASS
 *   IN:  int32 nx, ny; double tau[2], G_AB, g[2][2]; double rhoA[ny][nx], rhoB[ny][nx]
 *   OUT: int32 status of each call (7 of them: workspace, init, step, populations,
 *        fields, diagnostics, destroy); lb_diag as t (int64), mass[2], Ek, Ep,
 *        buoyancy, omega2, umax (doubles), finite (int32); then
 *        f[2][9][ny][nx] and rhoA, rhoB, ux, uy [ny][nx] (doubles)
 * Exit status 0 when every call returned LB_OK, 1 otherwise (the message of
 * lb_last_error goes to stderr), 2 on a usage, file or HIP runtime error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "lb.h"

static int read_all(FILE *fp, void *p, size_t n)
{
    return fread(p, 1, n, fp) == n;
}

int main(int argc, char **argv)
{
    if (argc != 7) {
        fprintf(stderr, "usage: %s IN OUT STEPS FORCING BC_Y STEPS_PER_PASS\n", argv[0]);
        return 2;
    }
    const long steps = strtol(argv[3], NULL, 10);
    FILE *in = fopen(argv[1], "rb");
    if (!in) {
        fprintf(stderr, "cannot open %s\n", argv[1]);
        return 2;
    }
    int32_t dims[2];
    double par[7];
    if (!read_all(in, dims, sizeof dims) || !read_all(in, par, sizeof par) || dims[0] < 1 || dims[1] < 1) {
        fprintf(stderr, "bad header in %s\n", argv[1]);
        fclose(in);
        return 2;
    }
    const size_t nsite = (size_t)dims[0] * (size_t)dims[1];
    double *rho = malloc(2 * nsite * sizeof(double));
    double *f = malloc(18 * nsite * sizeof(double));
    double *fld = malloc(4 * nsite * sizeof(double));
    if (!rho || !f || !fld || !read_all(in, rho, 2 * nsite * sizeof(double))) {
        fprintf(stderr, "cannot read the densities\n");
        fclose(in);
        return 2;
    }
    fclose(in);

    lb_member m = {0};
    m.nx = dims[0];
    m.ny = dims[1];
    m.tau[0] = par[0];
    m.tau[1] = par[1];
    m.G_AB = par[2];
    m.g[0][0] = par[3];
    m.g[0][1] = par[4];
    m.g[1][0] = par[5];
    m.g[1][1] = par[6];
    m.rhoA0 = rho;
    m.rhoB0 = rho + nsite;

    lb_config c = {0};
    c.n_members = 1;
    c.members = &m;
    c.forcing = (int32_t)strtol(argv[4], NULL, 10);
    c.storage = LB_F64;
    c.bc_y = (int32_t)strtol(argv[5], NULL, 10);
    c.diag_trim = 1;
    c.steps_per_pass = (int32_t)strtol(argv[6], NULL, 10);

    int32_t rc[7] = {LB_EINVAL, LB_EINVAL, LB_EINVAL, LB_EINVAL, LB_EINVAL, LB_EINVAL, LB_EINVAL};
    lb_diag d = {0};
    void *ws = NULL;
    double *d_f = NULL, *d_fld = NULL;
    hipStream_t st = NULL;
    lb_handle *h = NULL;

    const size_t bytes = lb_workspace_bytes(&c);
    rc[0] = bytes ? LB_OK : LB_EINVAL;
    if (bytes == 0) {
        fprintf(stderr, "lb_workspace_bytes: %s\n", lb_last_error());
    } else {
        if (hipMalloc(&ws, bytes) != hipSuccess || hipMalloc((void **)&d_f, 18 * nsite * sizeof(double)) != hipSuccess ||
            hipMalloc((void **)&d_fld, 4 * nsite * sizeof(double)) != hipSuccess || hipStreamCreate(&st) != hipSuccess) {
            fprintf(stderr, "HIP allocation failed\n");
            return 2;
        }
        rc[1] = lb_init(&c, ws, bytes, (void *)st, &h);
        if (rc[1] == LB_OK) {
            rc[2] = lb_step(h, steps);
            rc[3] = lb_get_populations(h, 0, d_f);
            rc[4] = lb_fields(h, 0, d_fld, d_fld + nsite, d_fld + 2 * nsite, d_fld + 3 * nsite);
            rc[5] = lb_diagnostics(h, 0, &d, NULL);   /* synchronises the stream */
            rc[6] = lb_destroy(h);
        }
        for (int k = 0; k < 7; ++k)
            if (rc[k] != LB_OK) fprintf(stderr, "call %d returned %d: %s\n", k, rc[k], lb_last_error());
        if (hipMemcpy(f, d_f, 18 * nsite * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(fld, d_fld, 4 * nsite * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
            fprintf(stderr, "HIP copy failed\n");
            return 2;
        }
        (void)hipStreamDestroy(st);
        (void)hipFree(d_fld);
        (void)hipFree(d_f);
        (void)hipFree(ws);
    }

    FILE *out = fopen(argv[2], "wb");
    if (!out) {
        fprintf(stderr, "cannot open %s\n", argv[2]);
        return 2;
    }
    const double dv[7] = {d.mass[0], d.mass[1], d.Ek, d.Ep, d.buoyancy, d.omega2, d.umax};
    int ok = fwrite(rc, sizeof rc, 1, out) == 1 && fwrite(&d.t, sizeof d.t, 1, out) == 1 &&
             fwrite(dv, sizeof dv, 1, out) == 1 && fwrite(&d.finite, sizeof d.finite, 1, out) == 1 &&
             fwrite(f, 18 * nsite * sizeof(double), 1, out) == 1 && fwrite(fld, 4 * nsite * sizeof(double), 1, out) == 1;
    ok = (fclose(out) == 0) && ok;
    free(fld);
    free(f);
    free(rho);
    if (!ok) return 2;
    for (int k = 0; k < 7; ++k)
        if (rc[k] != LB_OK) return 1;
    return 0;
}
