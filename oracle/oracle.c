/* oracle.c -- plain, slow FP64 reference of the interaction-potential +
 * immersed-boundary Lagrangian step (Spandan et al., "A parallel interaction
 * potential approach coupled with the immersed boundary method ...",
 * Section 2.2 transfer, Section 2.3 potentials and Newton update).
 *
 * TEST INFRASTRUCTURE ONLY: this library is loaded by the tests, by the smoke
 * check and by the CPU-baseline leg of the benchmark, never by the product
 * path.  It shares no code, header, table or helper with the GPU library.
 *
 * The core (oracle_core.inc) is compiled twice: once over double for values,
 * once over double complex for exact directional derivatives by the complex
 * step (Squire & Trapp 1998; Martins, Sturdza & Alonso 2003).
 *
 * Parity status of each exported function is recorded beside it.  All of them
 * are pinned by the CPU tests (closed forms, invariants, finite differences,
 * brute force); none is "parity unpinned".
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------- real instantiation ---------------- */
#define S double
#define FN(n) r_##n
#define RE(x) (x)
#define SQRT(x) sqrt(x)
#define SIN(x) sin(x)
#define COS(x) cos(x)
#define ATAN2(y, x) atan2((y), (x))
#include "oracle_core.inc"
#undef S
#undef FN
#undef RE
#undef SQRT
#undef SIN
#undef COS
#undef ATAN2

/* ---------------- complex-step instantiation ---------------- */
/* atan2 is not analytic as a library call; its complex-step extension is the
 * first-order expansion, exact to O(h^2) for the tiny imaginary steps used. */
static inline double complex cs_atan2(double complex y, double complex x)
{
    double yr = creal(y), xr = creal(x);
    return atan2(yr, xr) + I * ((xr * cimag(y) - yr * cimag(x)) / (xr * xr + yr * yr));
}
#define S double complex
#define FN(n) c_##n
#define RE(x) creal(x)
#define SQRT(x) csqrt(x)
#define SIN(x) csin(x)
#define COS(x) ccos(x)
#define ATAN2(y, x) cs_atan2((y), (x))
#include "oracle_core.inc"
#undef S
#undef FN
#undef RE
#undef SQRT
#undef SIN
#undef COS
#undef ATAN2

/* Imaginary step used by every complex-step derivative. */
#define CS_H 1e-30

/* ========================= exported C-ABI ========================= */

double orc_phi(double r) { return r_phi(r); }

void orc_geometry(int B, const int64_t *node_off, const int64_t *face_off,
                  const int32_t *faces, const double *X, double *V, double *A)
{
    r_geometry(B, node_off, face_off, faces, X, V, A);
}

void orc_reference(int B, const int64_t *node_off, const int64_t *edge_off,
                   const int64_t *face_off, const int32_t *faces, const int32_t *edges4,
                   const double *Xref, double *l0, double *theta0, double *A0, double *V0)
{
    r_reference(B, node_off, edge_off, face_off, faces, edges4, Xref, l0, theta0, A0, V0);
}

/* k = [4][B] (ks, kb, kA, kV); ew = [E][2] per-edge weights on ks and kb, or
 * NULL (all 1).  Ffam, V, A, W may be NULL. */
void orc_forces(int B, const int64_t *node_off, const int64_t *edge_off,
                const int64_t *face_off, const int32_t *faces, const int32_t *edges4,
                const uint8_t *closed, const double *X, const double *l0,
                const double *theta0, const double *A0, const double *V0,
                const double *k, const double *ew, double *F, double *Ffam, double *V,
                double *A, double *W)
{
    double *Vt = V ? V : (double *)malloc(sizeof(double) * (B > 0 ? B : 1));
    double *At = A ? A : (double *)malloc(sizeof(double) * (B > 0 ? B : 1));
    r_forces(B, node_off, edge_off, face_off, faces, edges4, closed, X, l0, theta0, A0, V0,
             k, k + B, k + 2 * B, k + 3 * B, ew, F, Ffam, Vt, At, W);
    if (!V) free(Vt);
    if (!A) free(At);
}

/* Directional derivative of the forces: dF = (dF/dX) dX (complex step).
 * Since F = -grad W, dF/dX is symmetric and this is also the VJP. */
void orc_forces_jvp(int B, const int64_t *node_off, const int64_t *edge_off,
                    const int64_t *face_off, const int32_t *faces, const int32_t *edges4,
                    const uint8_t *closed, const double *X, const double *dX,
                    const double *l0, const double *theta0, const double *A0,
                    const double *V0, const double *k, const double *ew, double *dF)
{
    int64_t N = node_off[B];
    double complex *Xc = malloc(sizeof(double complex) * 3 * N);
    double complex *Fc = malloc(sizeof(double complex) * 3 * N);
    double complex *kc = malloc(sizeof(double complex) * 4 * (B > 0 ? B : 1));
    double complex *Vc = malloc(sizeof(double complex) * (B > 0 ? B : 1));
    double complex *Ac = malloc(sizeof(double complex) * (B > 0 ? B : 1));
    for (int64_t i = 0; i < 3 * N; ++i) Xc[i] = X[i] + I * (CS_H * dX[i]);
    for (int64_t i = 0; i < 4 * B; ++i) kc[i] = k[i];
    c_forces(B, node_off, edge_off, face_off, faces, edges4, closed, Xc, l0, theta0, A0, V0,
             kc, kc + B, kc + 2 * B, kc + 3 * B, ew, Fc, NULL, Vc, Ac, NULL);
    for (int64_t i = 0; i < 3 * N; ++i) dF[i] = cimag(Fc[i]) / CS_H;
    free(Xc);
    free(Fc);
    free(kc);
    free(Vc);
    free(Ac);
}

void orc_interp(int64_t N, const double *X, int nx, int ny, int nz, double h,
                const double *u, double *U)
{
    r_interp(N, X, nx, ny, nz, h, u, U);
}

/* J[l][d][e] = dU_d(X_l)/dX_{l,e} by three complex steps (U_l depends only on
 * X_l, so one step along axis e for all nodes at once gives column e). */
void orc_interp_jac(int64_t N, const double *X, int nx, int ny, int nz, double h,
                    const double *u, double *J)
{
    double complex *Xc = malloc(sizeof(double complex) * 3 * N);
    double complex *Uc = malloc(sizeof(double complex) * 3 * N);
    for (int e = 0; e < 3; ++e) {
        for (int64_t i = 0; i < 3 * N; ++i) Xc[i] = X[i];
        for (int64_t l = 0; l < N; ++l) Xc[3 * l + e] += I * CS_H;
        c_interp(N, Xc, nx, ny, nz, h, u, Uc);
        for (int64_t l = 0; l < N; ++l)
            for (int d = 0; d < 3; ++d) J[9 * l + 3 * d + e] = cimag(Uc[3 * l + d]) / CS_H;
    }
    free(Xc);
    free(Uc);
}

void orc_spread(int64_t N, const double *X, const double *Fn, int nx, int ny, int nz,
                double h, double *f)
{
    r_spread(N, X, Fn, nx, ny, nz, h, f);
}

/* One explicit step (Section 2.3 Newton update with the immersed-boundary
 * direct-forcing reaction as external load; see the reading in the design
 * notes):  X <- X + dt U(X) + (dt^2 / m) F(X) for nodes not pinned, and
 * f += spread(F).  F, U, V, A receive the quantities at the old positions. */
void orc_step(int B, const int64_t *node_off, const int64_t *edge_off,
              const int64_t *face_off, const int32_t *faces, const int32_t *edges4,
              const uint8_t *closed, const uint8_t *pinned, const double *mass,
              double *X, const double *l0, const double *theta0, const double *A0,
              const double *V0, const double *k, const double *ew, int nx, int ny, int nz,
              double h, const double *u, double *f, double dt, double *F, double *U,
              double *V, double *A)
{
    int64_t N = node_off[B];
    orc_forces(B, node_off, edge_off, face_off, faces, edges4, closed, X, l0, theta0, A0, V0,
               k, ew, F, NULL, V, A, NULL);
    r_interp(N, X, nx, ny, nz, h, u, U);
    if (f) r_spread(N, X, F, nx, ny, nz, h, f);
    for (int b = 0; b < B; ++b) {
        double c = dt * dt / mass[b];
        for (int64_t l = node_off[b]; l < node_off[b + 1]; ++l) {
            if (pinned && pinned[l]) continue;
            for (int d = 0; d < 3; ++d) X[3 * l + d] += dt * U[3 * l + d] + c * F[3 * l + d];
        }
    }
}

/* ---------------- Taylor deformation of each body ----------------
 * C = (1/N) sum (x - c)(x - c)^T over the body's nodes, c the node mean;
 * eigenvalues by cyclic Jacobi rotations; L = sqrt(lambda_max),
 * B = sqrt(lambda_min), D = (L - B)/(L + B) (Section 3.1 deformation measure
 * built from the semi-axes; the node covariance is our reading). */
static void jacobi3(double a[3][3], double w[3], double v[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) v[i][j] = (i == j);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        double diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off <= 1e-34 * diag || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < 3; ++r) {      /* A <- A J */
                    double arp = a[r][p], arq = a[r][q];
                    a[r][p] = c * arp - s * arq;
                    a[r][q] = s * arp + c * arq;
                }
                for (int r = 0; r < 3; ++r) {      /* A <- J^T A */
                    double apr = a[p][r], aqr = a[q][r];
                    a[p][r] = c * apr - s * aqr;
                    a[q][r] = s * apr + c * aqr;
                }
                for (int r = 0; r < 3; ++r) {      /* V <- V J */
                    double vrp = v[r][p], vrq = v[r][q];
                    v[r][p] = c * vrp - s * vrq;
                    v[r][q] = s * vrp + c * vrq;
                }
            }
    }
    for (int i = 0; i < 3; ++i) w[i] = a[i][i];
}

static void body_cov(const double *X, int64_t n0, int64_t n1, double c[3], double C[3][3])
{
    int64_t n = n1 - n0;
    c[0] = c[1] = c[2] = 0.0;
    for (int64_t l = n0; l < n1; ++l)
        for (int d = 0; d < 3; ++d) c[d] += X[3 * l + d];
    for (int d = 0; d < 3; ++d) c[d] /= (double)n;
    memset(C, 0, sizeof(double) * 9);
    for (int64_t l = n0; l < n1; ++l)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                C[i][j] += (X[3 * l + i] - c[i]) * (X[3 * l + j] - c[j]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[i][j] /= (double)n;
}

/* D[b]; evals[b][3] sorted descending (optional). */
void orc_taylor(int B, const int64_t *node_off, const double *X, double *D, double *evals)
{
    for (int b = 0; b < B; ++b) {
        double c[3], C[3][3], w[3], v[3][3];
        body_cov(X, node_off[b], node_off[b + 1], c, C);
        jacobi3(C, w, v);
        double lmax = fmax(w[0], fmax(w[1], w[2])), lmin = fmin(w[0], fmin(w[1], w[2]));
        double L = sqrt(lmax), Bs = sqrt(lmin);
        D[b] = (L - Bs) / (L + Bs);
        if (evals) {
            double mid = w[0] + w[1] + w[2] - lmax - lmin;
            evals[3 * b + 0] = lmax;
            evals[3 * b + 1] = mid;
            evals[3 * b + 2] = lmin;
        }
    }
}

/* Loss sum_b (D_b - Dstar_b)^2 and its gradient gX[N][3] (overwritten).
 * dlambda_k = v_k^T dC v_k, and dC = (1/n) sum_m [dx_m r_m^T + r_m dx_m^T]
 * with r_m = x_m - c (the mean's variation cancels since sum r_m = 0), so
 * dlambda_k/dx_m = (2/n)(v_k . r_m) v_k. */
double orc_taylor_loss_grad(int B, const int64_t *node_off, const double *X,
                            const double *Dstar, double *gX)
{
    double loss = 0.0;
    for (int b = 0; b < B; ++b) {
        int64_t n0 = node_off[b], n1 = node_off[b + 1], n = n1 - n0;
        double c[3], C[3][3], w[3], v[3][3];
        body_cov(X, n0, n1, c, C);
        jacobi3(C, w, v);
        int imax = 0, imin = 0;
        for (int i = 1; i < 3; ++i) {
            if (w[i] > w[imax]) imax = i;
            if (w[i] < w[imin]) imin = i;
        }
        double L = sqrt(w[imax]), Bs = sqrt(w[imin]);
        double D = (L - Bs) / (L + Bs);
        double r = D - Dstar[b];
        loss += r * r;
        double dD_dL = 2.0 * Bs / ((L + Bs) * (L + Bs));
        double dD_dB = -2.0 * L / ((L + Bs) * (L + Bs));
        double g_lmax = 2.0 * r * dD_dL / (2.0 * L);   /* dloss/dlambda_max */
        double g_lmin = 2.0 * r * dD_dB / (2.0 * Bs);  /* dloss/dlambda_min */
        double vmax[3] = {v[0][imax], v[1][imax], v[2][imax]};
        double vmin[3] = {v[0][imin], v[1][imin], v[2][imin]};
        for (int64_t m = n0; m < n1; ++m) {
            double rm[3] = {X[3 * m] - c[0], X[3 * m + 1] - c[1], X[3 * m + 2] - c[2]};
            double pmax = vmax[0] * rm[0] + vmax[1] * rm[1] + vmax[2] * rm[2];
            double pmin = vmin[0] * rm[0] + vmin[1] * rm[1] + vmin[2] * rm[2];
            for (int d = 0; d < 3; ++d)
                gX[3 * m + d] = (2.0 / (double)n) * (g_lmax * pmax * vmax[d] + g_lmin * pmin * vmin[d]);
        }
    }
    return loss;
}

/* ---------------- MLS transfer at the triangle centroids ---------------- */
#include "oracle_mls.inc"
