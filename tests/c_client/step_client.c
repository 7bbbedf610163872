/* step_client.c -- a plain C caller of libipibm (no Python, no torch): one
 * explicit step of a closed mesh at its reference shape in a uniform velocity
 * field u0.  At the reference every potential is at its minimum, so the
 * internal force vanishes, and the 3-point delta weights sum to one, so the
 * interpolated velocity is u0: every node moves by dt u0 (Section 2.3 update
 * with F = 0).  Test infrastructure, run by tests/test_gpu_c_client.py.
 *
 * usage: step_client MESH_FILE
 * MESH_FILE (text): "N E F", then N lines of x y z, F lines of three node
 * ids, E lines of four node ids (edges4, -1 for a missing wing).
 * The new position is rounded to the spacing of |X|, so each coordinate must
 * match X + dt u0 within 1e-12 |dt u0| plus two ulps of |X|.  Prints the
 * worst error as a fraction of that bar and exits 0 if it is at most 1 and
 * the plan's status is clean. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "ipibm.h"

#define HIP_OK(x)                                                              \
    do {                                                                       \
        if ((x) != hipSuccess) {                                               \
            fprintf(stderr, "HIP error at %s:%d\n", __FILE__, __LINE__);      \
            return 2;                                                          \
        }                                                                      \
    } while (0)
#define IP_OK_(x)                                                              \
    do {                                                                       \
        ip_status s_ = (x);                                                    \
        if (s_ != IP_OK) {                                                     \
            fprintf(stderr, "ipibm error %d: %s\n", (int)s_, ip_last_error()); \
            return 3;                                                          \
        }                                                                      \
    } while (0)

static void *dalloc(size_t bytes) {
    void *p = NULL;
    return hipMalloc(&p, bytes ? bytes : 8) == hipSuccess ? p : NULL;
}

int main(int argc, char **argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s MESH_FILE\n", argv[0]);
        return 1;
    }
    FILE *fh = fopen(argv[1], "r");
    if (!fh) return 1;
    long n, e, f;
    if (fscanf(fh, "%ld %ld %ld", &n, &e, &f) != 3 || n <= 0 || e <= 0 || f <= 0) return 1;
    double *X = malloc(sizeof(double) * 3 * n);
    int32_t *faces = malloc(sizeof(int32_t) * 3 * f);
    int32_t *edges4 = malloc(sizeof(int32_t) * 4 * e);
    for (long i = 0; i < 3 * n; ++i)
        if (fscanf(fh, "%lf", &X[i]) != 1) return 1;
    for (long i = 0; i < 3 * f; ++i)
        if (fscanf(fh, "%d", &faces[i]) != 1) return 1;
    for (long i = 0; i < 4 * e; ++i)
        if (fscanf(fh, "%d", &edges4[i]) != 1) return 1;
    fclose(fh);

    /* one closed body on a 16^3 periodic grid of spacing 1/16 */
    const int64_t node_off[2] = {0, n}, edge_off[2] = {0, e}, face_off[2] = {0, f};
    const uint8_t closed[1] = {1};
    ip_mesh mesh = {1, node_off, edge_off, face_off, faces, edges4, closed, NULL};
    ip_grid grid = {16, 16, 16, 1.0 / 16};
    ip_plan *plan = NULL;
    IP_OK_(ip_plan_create(&plan, &mesh, &grid, IP_F64));

    const size_t xb = sizeof(double) * 3 * n, field = (size_t)16 * 16 * 16;
    double *dX = dalloc(xb), *dXref = dalloc(xb);
    double *l0 = dalloc(sizeof(double) * e), *cs0 = dalloc(sizeof(double) * 2 * e);
    double *A0 = dalloc(sizeof(double) * f), *V0 = dalloc(sizeof(double));
    double *u = dalloc(sizeof(double) * 3 * field), *fgrid = dalloc(sizeof(double) * 3 * field);
    double *kconst = dalloc(sizeof(double) * 5);
    if (!dX || !dXref || !l0 || !cs0 || !A0 || !V0 || !u || !fgrid || !kconst) return 2;
    HIP_OK(hipMemcpy(dX, X, xb, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dXref, X, xb, hipMemcpyHostToDevice));

    /* uniform velocity u0 on every lattice, constants ks kb kA kV m */
    const double u0[3] = {0.3, -0.2, 0.1}, dt = 1e-3;
    double *hu = malloc(sizeof(double) * 3 * field);
    for (int d = 0; d < 3; ++d)
        for (size_t i = 0; i < field; ++i) hu[d * field + i] = u0[d];
    HIP_OK(hipMemcpy(u, hu, sizeof(double) * 3 * field, hipMemcpyHostToDevice));
    HIP_OK(hipMemset(fgrid, 0, sizeof(double) * 3 * field));
    const double hk[5] = {1.0, 0.01, 0.1, 1.0, 1.0};
    HIP_OK(hipMemcpy(kconst, hk, sizeof hk, hipMemcpyHostToDevice));
    ip_constants k = {kconst, kconst + 1, kconst + 2, kconst + 3, kconst + 4};

    IP_OK_(ip_reference_from(plan, dXref, l0, cs0, A0, V0, NULL));
    ip_reference ref = {l0, cs0, A0, V0};
    IP_OK_(ip_step(plan, dX, &ref, &k, u, fgrid, dt, NULL, NULL, NULL));
    uint32_t flags = 0;
    IP_OK_(ip_plan_status(plan, NULL, &flags));

    double *Xn = malloc(xb);
    HIP_OK(hipMemcpy(Xn, dX, xb, hipMemcpyDeviceToHost));
    const double scale = dt * sqrt(u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2]);
    double worst = 0.0;
    for (long i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            const double x = fabs(X[3 * i + d]);
            const double bar = 1e-12 * scale + 2.0 * (nextafter(x, INFINITY) - x);
            const double err = fabs(Xn[3 * i + d] - (X[3 * i + d] + dt * u0[d])) / bar;
            if (!(err <= worst)) worst = err;
        }
    printf("nodes %ld, worst error / bar = %.3f, status flags %u\n", n, worst, (unsigned)flags);
    IP_OK_(ip_plan_destroy(plan));
    void *bufs[] = {dX, dXref, l0, cs0, A0, V0, u, fgrid, kconst};
    for (size_t i = 0; i < sizeof bufs / sizeof bufs[0]; ++i) HIP_OK(hipFree(bufs[i]));
    free(X);
    free(faces);
    free(edges4);
    free(hu);
    free(Xn);
    return worst <= 1.0 && flags == 0 ? 0 : 4;
}
