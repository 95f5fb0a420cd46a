/*
 * Drives the D3Q19 entry points of liblb.so (include/lb3.h) from a plain C
 * program: no Python, no PyTorch.  Creates one lattice from the densities in
 * an input file, advances it, and writes f(t), the fields and the lb3_diag
 * averages to an output file for the test to compare with the 3D oracle.
 *
 * usage: lb3_c_driver IN OUT STEPS BC_Y STORAGE TWO_PASS
 *   IN:  int32 nx, ny, nz; double tau[2], G_AB, g[2][3];
 *        double rhoA[nz][ny][nx], rhoB[nz][ny][nx]
 *   OUT: int32 status of each call (7: workspace, init, step, populations,
 *        fields, diagnostics, destroy); lb3_diag as t (int64), mass[2], Ek,
 *        umax (doubles), finite (int32); then f[2][19][nz][ny][nx] and
 *        rhoA, rhoB, ux, uy, uz [nz][ny][nx] (doubles)
 * Exit status 0 when every call returned LB_OK, 1 otherwise (the message of
 * lb_last_error goes to stderr), 2 on a usage, file or HIP runtime error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "lb3.h"

static int read_all(FILE *fp, void *p, size_t n)
{
    return fread(p, 1, n, fp) == n;
}

int main(int argc, char **argv)
{
    if (argc != 7) {
        fprintf(stderr, "usage: %s IN OUT STEPS BC_Y STORAGE TWO_PASS\n", argv[0]);
        return 2;
    }
    const long steps = strtol(argv[3], NULL, 10);
    FILE *in = fopen(argv[1], "rb");
    if (!in) {
        fprintf(stderr, "cannot open %s\n", argv[1]);
        return 2;
    }
    int32_t dims[3];
    double par[9];
    if (!read_all(in, dims, sizeof dims) || !read_all(in, par, sizeof par) || dims[0] < 1 || dims[1] < 1 ||
        dims[2] < 1) {
        fprintf(stderr, "bad header in %s\n", argv[1]);
        fclose(in);
        return 2;
    }
    const size_t nsite = (size_t)dims[0] * (size_t)dims[1] * (size_t)dims[2];
    double *rho = malloc(2 * nsite * sizeof(double));
    double *f = malloc(38 * nsite * sizeof(double));
    double *fld = malloc(5 * nsite * sizeof(double));
    if (!rho || !f || !fld || !read_all(in, rho, 2 * nsite * sizeof(double))) {
        fprintf(stderr, "cannot read the densities\n");
        fclose(in);
        return 2;
    }
    fclose(in);

    lb3_config c = {0};
    c.nx = dims[0];
    c.ny = dims[1];
    c.nz = dims[2];
    c.bc_y = (int32_t)strtol(argv[4], NULL, 10);
    c.storage = (int32_t)strtol(argv[5], NULL, 10);
    c.diag_trim = 0;
    c.two_pass = (int32_t)strtol(argv[6], NULL, 10);
    c.tau[0] = par[0];
    c.tau[1] = par[1];
    c.G_AB = par[2];
    for (int s = 0; s < 2; ++s)
        for (int d = 0; d < 3; ++d) c.g[s][d] = par[3 + 3 * s + d];
    c.rhoA0 = rho;
    c.rhoB0 = rho + nsite;

    int32_t rc[7] = {LB_EINVAL, LB_EINVAL, LB_EINVAL, LB_EINVAL, LB_EINVAL, LB_EINVAL, LB_EINVAL};
    lb3_diag d = {0};
    void *ws = NULL;
    double *d_f = NULL, *d_fld = NULL;
    hipStream_t st = NULL;
    lb3_handle *h = NULL;

    const size_t bytes = lb3_workspace_bytes(&c);
    rc[0] = bytes ? LB_OK : LB_EINVAL;
    if (bytes == 0) {
        fprintf(stderr, "lb3_workspace_bytes: %s\n", lb_last_error());
    } else {
        if (hipMalloc(&ws, bytes) != hipSuccess || hipMalloc((void **)&d_f, 38 * nsite * sizeof(double)) != hipSuccess ||
            hipMalloc((void **)&d_fld, 5 * nsite * sizeof(double)) != hipSuccess || hipStreamCreate(&st) != hipSuccess) {
            fprintf(stderr, "HIP allocation failed\n");
            return 2;
        }
        rc[1] = lb3_init(&c, ws, bytes, (void *)st, &h);
        if (rc[1] == LB_OK) {
            rc[2] = lb3_step(h, steps);
            rc[3] = lb3_get_populations(h, d_f);
            rc[4] = lb3_fields(h, d_fld, d_fld + nsite, d_fld + 2 * nsite, d_fld + 3 * nsite, d_fld + 4 * nsite);
            rc[5] = lb3_diagnostics(h, &d);   /* synchronises the stream */
            rc[6] = lb3_destroy(h);
        }
        for (int k = 0; k < 7; ++k)
            if (rc[k] != LB_OK) fprintf(stderr, "call %d returned %d: %s\n", k, rc[k], lb_last_error());
        if (hipMemcpy(f, d_f, 38 * nsite * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(fld, d_fld, 5 * nsite * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
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
    const double dv[4] = {d.mass[0], d.mass[1], d.Ek, d.umax};
    int ok = fwrite(rc, sizeof rc, 1, out) == 1 && fwrite(&d.t, sizeof d.t, 1, out) == 1 &&
             fwrite(dv, sizeof dv, 1, out) == 1 && fwrite(&d.finite, sizeof d.finite, 1, out) == 1 &&
             fwrite(f, 38 * nsite * sizeof(double), 1, out) == 1 && fwrite(fld, 5 * nsite * sizeof(double), 1, out) == 1;
    ok = (fclose(out) == 0) && ok;
    free(fld);
    free(f);
    free(rho);
    if (!ok) return 2;
    for (int k = 0; k < 7; ++k)
        if (rc[k] != LB_OK) return 1;
    return 0;
}
