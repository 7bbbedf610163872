// k_mls.hip -- moving-least-squares (MLS) transfer between the triangle
// centroids (the Lagrangian markers) and the staggered lattices (Section 2.2
// of Spandan et al.: the MLS equations with a linear basis, the exponential
// weight on a 3x3x3 support of threshold 1.5 h, and the force-conserving
// spreading factor c_l), and the transfer of centroid forces to the triangle
// vertices (one third per vertex, Section 2.3).
//
// One thread per marker.  The weight is a product over axes, W_k =
// wx_i wy_j wz_k with w(r) = exp(-(r/alpha)^2), r = |x_a - x^k_a| / 1.5 h, so
// every entry of the moment matrix A = sum_k W_k p_k p_k^T (p_k = [1, dx_i,
// dy_j, dz_k], offsets about the marker in units of h) is a product of three
// per-axis sums S0 = sum w, S1 = sum w d, S2 = sum w d^2.  A is symmetric
// positive definite (all 27 weights are positive inside the support); its
// Cholesky factor gives z = A^{-1} e_0 and phi_ijk = W_ijk (z0 + z1 dx_i +
// z2 dy_j + z3 dz_k).  All MLS arithmetic is FP64; the fields are R.
//
// The per-axis parts are shared: along any axis the three MAC lattices sit at
// only two offsets (integer or half cells), so a marker computes six axes for
// all three lattices (the probe kernel excepted, see there); the three weights of an axis take two exponentials
// (w_{c-1,c+1} = w_c exp(-q^2) exp(+-2 d_c q^2)); and the Cholesky factor keeps
// the reciprocals of its diagonal, so each solve is four divisions.
//
// Interpolation runs one thread per marker (its gathers of u hit in L2: the
// faces of a body are consecutive).  Spreading on plans with work units runs
// one workgroup per unit: the unit's positions go to LDS, each face whose
// first corner the unit owns adds its 27 weighted values per lattice into an
// FP64 LDS tile over the cell box of the unit's markers (ds_add_f64), and the
// tile's non-zero points are added to f once.  A unit whose tile does not fit
// adds into f directly.  (Measured on 1000 level-4 drops: per-marker global
// atomics 18.5 ms, the tiled form 0.8 ms; a tiled interpolation was slower
// than the per-marker one, 0.69 against 0.61 ms.)
#include <algorithm>
#include <cmath>

#include "step_common.h"

namespace {

struct MlsGrid {
    int nx, ny, nz;
    double h, inv_h;
    int64_t plane, field;
    // weight w(d) = exp(-(|d| q)^2), q = 1 / (1.5 alpha), d in cells
    double inv_alpha;
    double q2, cq;       // q^2 and exp(-q^2)
    int fast;            // q^2 small enough for the two-exponential form
};

// One axis of a marker's MLS shape on lattices with a given offset along
// that axis: the three support points c - 1, c, c + 1 around the marker.
struct MlsAxis {
    double w[3];         // weights
    double dk[3];        // offsets (x^k - x) / h
    int idx[3];          // wrapped lattice indices
    int c;               // unwrapped index of the middle point
    double s0, s1, s2;   // sum w, sum w d, sum w d^2
};

__device__ __forceinline__ void mls_axis(double xa, double off, int n, const MlsGrid &g,
                                         MlsAxis &A) {
    const double s = xa * g.inv_h - off;
    double c = floor(s + 0.5);
    if (!(fabs(c) < 1.0e9)) c = 0.0;           // non-finite or absurd position
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        A.dk[j] = (c - 1.0 + j) - s;
        A.idx[j] = wrapi((int)c - 1 + j, n);
    }
    A.c = (int)c;
    const double r1 = fabs(A.dk[1]) * (1.0 / 1.5) * g.inv_alpha;
    const double w1 = exp(-r1 * r1);
    double w0, w2;
    if (g.fast) {
        // (d1 -+ 1)^2 q^2 = d1^2 q^2 -+ 2 d1 q^2 + q^2, so the outer weights
        // are w1 exp(-q^2) exp(+-2 d1 q^2): two exponentials per axis
        const double E = exp(2.0 * A.dk[1] * g.q2);
        w0 = w1 * g.cq * E;
        w2 = w1 * g.cq / E;
    } else {
        const double r0 = fabs(A.dk[0]) * (1.0 / 1.5) * g.inv_alpha;
        const double r2 = fabs(A.dk[2]) * (1.0 / 1.5) * g.inv_alpha;
        w0 = exp(-r0 * r0);
        w2 = exp(-r2 * r2);
    }
    A.w[0] = fabs(A.dk[0]) <= 1.5 ? w0 : 0.0;
    A.w[1] = fabs(A.dk[1]) <= 1.5 ? w1 : 0.0;
    A.w[2] = fabs(A.dk[2]) <= 1.5 ? w2 : 0.0;
    A.s0 = A.s1 = A.s2 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        A.s0 += A.w[j];
        A.s1 += A.w[j] * A.dk[j];
        A.s2 += A.w[j] * A.dk[j] * A.dk[j];
    }
}

// Both offsets of every axis for one marker: o0 (lattice points at integer
// cells along the axis) and o5 (at half cells).  MAC lattice d is offset 0
// along axis d and 1/2 along the others; the cell-centred lattice is 1/2
// along all three.
struct MlsAxes {
    MlsAxis o0[3], o5[3];
};

__device__ __forceinline__ void mls_axes(const vec3<double> &x, const MlsGrid &g, MlsAxes &M) {
    const double xs[3] = {x.x, x.y, x.z};
    const int n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mls_axis(xs[a], 0.0, n[a], g, M.o0[a]);
        mls_axis(xs[a], 0.5, n[a], g, M.o5[a]);
    }
}

// Cholesky factor of the moment matrix A (symmetric, entries products of the
// per-axis sums: A_00 = X0 Y0 Z0, A_01 = X1 Y0 Z0, ...) with the reciprocals
// of its diagonal, and the solve of A x = b with it.
struct MlsChol {
    double l10, l20, l30, l21, l31, l32;
    double r0, r1, r2, r3;   // 1 / l_ii
};

__device__ __forceinline__ void mls_factor(const MlsAxis &X, const MlsAxis &Y, const MlsAxis &Z,
                                           MlsChol &L) {
    const double a00 = X.s0 * Y.s0 * Z.s0;
    const double a01 = X.s1 * Y.s0 * Z.s0, a02 = X.s0 * Y.s1 * Z.s0, a03 = X.s0 * Y.s0 * Z.s1;
    const double a11 = X.s2 * Y.s0 * Z.s0, a22 = X.s0 * Y.s2 * Z.s0, a33 = X.s0 * Y.s0 * Z.s2;
    const double a12 = X.s1 * Y.s1 * Z.s0, a13 = X.s1 * Y.s0 * Z.s1, a23 = X.s0 * Y.s1 * Z.s1;
    L.r0 = 1.0 / sqrt(a00);
    L.l10 = a01 * L.r0;
    L.l20 = a02 * L.r0;
    L.l30 = a03 * L.r0;
    L.r1 = 1.0 / sqrt(a11 - L.l10 * L.l10);
    L.l21 = (a12 - L.l20 * L.l10) * L.r1;
    L.l31 = (a13 - L.l30 * L.l10) * L.r1;
    L.r2 = 1.0 / sqrt(a22 - L.l20 * L.l20 - L.l21 * L.l21);
    L.l32 = (a23 - L.l30 * L.l20 - L.l31 * L.l21) * L.r2;
    L.r3 = 1.0 / sqrt(a33 - L.l30 * L.l30 - L.l31 * L.l31 - L.l32 * L.l32);
}

__device__ __forceinline__ bool mls_solve(const MlsChol &L, const double b[4], double x[4]) {
    const double y0 = b[0] * L.r0;
    const double y1 = (b[1] - L.l10 * y0) * L.r1;
    const double y2 = (b[2] - L.l20 * y0 - L.l21 * y1) * L.r2;
    const double y3 = (b[3] - L.l30 * y0 - L.l31 * y1 - L.l32 * y2) * L.r3;
    x[3] = y3 * L.r3;
    x[2] = (y2 - L.l32 * x[3]) * L.r2;
    x[1] = (y1 - L.l21 * x[2] - L.l31 * x[3]) * L.r1;
    x[0] = (y0 - L.l10 * x[1] - L.l20 * x[2] - L.l30 * x[3]) * L.r0;
    return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(x[3]);
}

// The shape of one marker on one lattice: per-axis parts and z = A^{-1} e_0.
struct MlsShape {
    double w[3][3];      // per-axis weights of the 3 support points
    double dk[3][3];     // per-axis offsets (x^k - x) / h
    double z[4];         // A^{-1} e_0
    int idx[3][3];       // wrapped lattice indices per axis
    int c[3];            // unwrapped index of the middle support point per axis
};

__device__ __forceinline__ bool mls_shape(const MlsAxis &X, const MlsAxis &Y, const MlsAxis &Z,
                                          MlsShape &S) {
    const MlsAxis *ax[3] = {&X, &Y, &Z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            S.w[a][j] = ax[a]->w[j];
            S.dk[a][j] = ax[a]->dk[j];
            S.idx[a][j] = ax[a]->idx[j];
        }
        S.c[a] = ax[a]->c;
    }
    MlsChol L;
    mls_factor(X, Y, Z, L);
    const double e0[4] = {1.0, 0.0, 0.0, 0.0};
    return mls_solve(L, e0, S.z);
}

// Shape on MAC lattice d from a marker's shared axes (d a compile-time
// constant after unrolling, so the axes stay in registers).
__device__ __forceinline__ bool mls_shape(const MlsAxes &M, int d, MlsShape &S) {
    return mls_shape(d == 0 ? M.o0[0] : M.o5[0], d == 1 ? M.o0[1] : M.o5[1],
                     d == 2 ? M.o0[2] : M.o5[2], S);
}

// Shape on MAC lattice d at x, every axis computed here.
__device__ __forceinline__ bool mls_shape(const vec3<double> &x, int d, const MlsGrid &g,
                                          MlsShape &S) {
    MlsAxis X, Y, Z;
    mls_axis(x.x, mac_off(d, 0), g.nx, g, X);
    mls_axis(x.y, mac_off(d, 1), g.ny, g, Y);
    mls_axis(x.z, mac_off(d, 2), g.nz, g, Z);
    return mls_shape(X, Y, Z, S);
}

__device__ __forceinline__ double mls_phi(const MlsShape &S, int i, int j, int k) {
    return S.w[0][i] * S.w[1][j] * S.w[2][k] *
           (S.z[0] + S.z[1] * S.dk[0][i] + S.z[2] * S.dk[1][j] + S.z[3] * S.dk[2][k]);
}

// Centroid and area of face f.
__device__ __forceinline__ vec3<double> centroid(const double *X, const int32_t *faces, int64_t f,
                                                 double &area) {
    const vec3<double> a = ldX(X, faces[3 * f]), b = ldX(X, faces[3 * f + 1]),
                       c = ldX(X, faces[3 * f + 2]);
    const vec3<double> n = cross(b - a, c - a);
    area = 0.5 * sqrt(dot(n, n));
    return vec3<double>{(a.x + b.x + c.x) * (1.0 / 3.0), (a.y + b.y + c.y) * (1.0 / 3.0),
                        (a.z + b.z + c.z) * (1.0 / 3.0)};
}

// U[f][d] = sum_k phi_k u_d[k] at the centroid of face f.
template <typename R>
__global__ __launch_bounds__(256) void k_interp_mls(const double *__restrict__ X,
                                                    const int32_t *__restrict__ faces, int64_t F,
                                                    const R *__restrict__ u, MlsGrid g,
                                                    R *__restrict__ U, uint32_t *status) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double area;
    const vec3<double> x = centroid(X, faces, f, area);
    MlsAxes M;
    mls_axes(x, g, M);
    bool bad = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        MlsShape S;
        bad |= !mls_shape(M, d, S);
        const R *ud = u + d * g.field;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const R *row = ud + (int64_t)S.idx[2][k] * g.plane + (int64_t)S.idx[1][j] * g.nx;
#pragma unroll
                for (int i = 0; i < 3; ++i) acc += mls_phi(S, i, j, k) * (double)row[S.idx[0][i]];
            }
        U[3 * f + d] = (R)acc;
    }
    if (bad) atomicOr(status, IP_STATUS_NONFINITE);
}

// f_d[k] += c_l phi_k Fm[f][d], c_l = dV_l / (sum_k phi_k dV^k), dV_l = A_l h_l,
// h_l = (1/3) sum_k phi_k (dx + dy + dz), dV^k = h^3 (device atomics).
template <typename R>
__global__ __launch_bounds__(256) void k_spread_mls(const double *__restrict__ X,
                                                    const int32_t *__restrict__ faces, int64_t F,
                                                    const R *__restrict__ Fm, MlsGrid g,
                                                    R *__restrict__ fld, uint32_t *status) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double area;
    const vec3<double> x = centroid(X, faces, f, area);
    MlsAxes M;
    mls_axes(x, g, M);
    bool bad = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        MlsShape S;
        bad |= !mls_shape(M, d, S);
        // sum_k phi_k (1 up to rounding, since A z = e_0), as the paper writes c_l
        double sphi = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int i = 0; i < 3; ++i) sphi += mls_phi(S, i, j, k);
        const double hl = (1.0 / 3.0) * sphi * (3.0 * g.h);
        const double cl = area * hl / (sphi * g.h * g.h * g.h);
        const double Fd = (double)Fm[3 * f + d] * cl;
        R *fd = fld + d * g.field;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                R *row = fd + (int64_t)S.idx[2][k] * g.plane + (int64_t)S.idx[1][j] * g.nx;
#pragma unroll
                for (int i = 0; i < 3; ++i) unsafeAtomicAdd(row + S.idx[0][i], (R)(mls_phi(S, i, j, k) * Fd));
            }
    }
    if (bad) atomicOr(status, IP_STATUS_NONFINITE);
}

// Direct forcing, one thread per marker (plans without work units):
// F = (V^b - U) / dt at the centroid, stored to Fout when given, spread with
// device atomics.
template <typename R>
__global__ __launch_bounds__(256) void k_direct_forcing_mls(
    const double *__restrict__ X, const int32_t *__restrict__ faces, int64_t F,
    const R *__restrict__ u, const R *__restrict__ Vb, MlsGrid g, double inv_dt, R *__restrict__ Fout, R *__restrict__ fld, uint32_t *status) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double area;
    const vec3<double> x = centroid(X, faces, f, area);
    MlsAxes M;
    mls_axes(x, g, M);
    bool bad = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        MlsShape S;
        bad |= !mls_shape(M, d, S);
        const R *ud = u + d * g.field;
        double U = 0.0, sphi = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const R *row = ud + (int64_t)S.idx[2][k] * g.plane + (int64_t)S.idx[1][j] * g.nx;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double ph = mls_phi(S, i, j, k);
                    U += ph * (double)row[S.idx[0][i]];
                    sphi += ph;
                }
            }
        const double Fl = ((double)Vb[3 * f + d] - U) * inv_dt;
        if (Fout != nullptr) Fout[3 * f + d] = (R)Fl;
        const double hl = (1.0 / 3.0) * sphi * (3.0 * g.h);
        const double Fd = Fl * area * hl / (sphi * g.h * g.h * g.h);
        R *fd = fld + d * g.field;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                R *row = fd + (int64_t)S.idx[2][k] * g.plane + (int64_t)S.idx[1][j] * g.nx;
#pragma unroll
                for (int i = 0; i < 3; ++i) unsafeAtomicAdd(row + S.idx[0][i], (R)(mls_phi(S, i, j, k) * Fd));
            }
    }
    if (bad) atomicOr(status, IP_STATUS_NONFINITE);
}

// MLS fit about a point on one lattice, from its per-axis shape parts:
// a = A^{-1} B q, the linear fit q ~ a0 + a1 dx + a2 dy + a3 dz (offsets in
// units of h); a0 is the MLS value at the point and a1..a3 / h its gradient.
// Returns false if the solve is not finite.
template <typename R>
__device__ __forceinline__ bool mls_fit(const MlsAxis &X, const MlsAxis &Y, const MlsAxis &Z,
                                        const MlsGrid &g, const R *__restrict__ q, double a[4]) {
    // B q: weighted moments of the 27 values
    double m[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const R *row = q + (int64_t)Z.idx[k] * g.plane + (int64_t)Y.idx[j] * g.nx;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double wq = X.w[i] * Y.w[j] * Z.w[k] * (double)row[X.idx[i]];
                m[0] += wq;
                m[1] += wq * X.dk[i];
                m[2] += wq * Y.dk[j];
                m[3] += wq * Z.dk[k];
            }
        }
    MlsChol L;
    mls_factor(X, Y, Z, L);
    return mls_solve(L, m, a);
}

// External loads on face f from probes of length h along its unit normal:
// one outward probe on closed bodies, both sides on open ones.  At a probe
// end y = x_c + s h n: p = (MLS value of the cell-centred pressure) +
// s h (Du/Dt).n, G_ij = du_i/dx_j (gradient of the MLS fit of lattice i),
// tau = mu (G + G^T); the load is sum_s s (-p n + tau n) A.
template <typename R>
__global__ __launch_bounds__(256) void k_probe_loads(
    const double *__restrict__ X, const int32_t *__restrict__ faces,
    const int64_t *__restrict__ face_off, const uint8_t *__restrict__ closed, int B, int64_t F,
    const R *__restrict__ u, const R *__restrict__ pr, const R *__restrict__ acc, MlsGrid g,
    double mu, R *__restrict__ Fext, uint32_t *status) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    // body of face f: the last b with face_off[b] <= f
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (face_off[mid] <= f)
            lo = mid;
        else
            hi = mid - 1;
    }
    const vec3<double> xa = ldX(X, faces[3 * f]), xb = ldX(X, faces[3 * f + 1]),
                       xc3 = ldX(X, faces[3 * f + 2]);
    const vec3<double> nn = cross(xb - xa, xc3 - xa);
    const double nlen = sqrt(dot(nn, nn));
    if (!(nlen > 0.0)) {
        // a zero-area face has no normal: no probe, no load
        Fext[3 * f] = (R)0.0;
        Fext[3 * f + 1] = (R)0.0;
        Fext[3 * f + 2] = (R)0.0;
        atomicOr(status, nlen == 0.0 ? IP_STATUS_DEGENERATE : IP_STATUS_NONFINITE);
        return;
    }
    const double area = 0.5 * nlen;
    const vec3<double> nu{nn.x / nlen, nn.y / nlen, nn.z / nlen};
    const vec3<double> xc{(xa.x + xb.x + xc3.x) * (1.0 / 3.0), (xa.y + xb.y + xc3.y) * (1.0 / 3.0),
                          (xa.z + xb.z + xc3.z) * (1.0 / 3.0)};
    const double an = acc == nullptr ? 0.0
                                     : (double)acc[3 * f] * nu.x + (double)acc[3 * f + 1] * nu.y +
                                           (double)acc[3 * f + 2] * nu.z;
    const int sides = closed[lo] ? 1 : 2;
    double F0 = 0.0, F1 = 0.0, F2 = 0.0;
    bool bad = false;
#pragma unroll 1
    for (int side = 0; side < sides; ++side) {
        const double sg = side == 0 ? 1.0 : -1.0;
        const vec3<double> y{xc.x + sg * g.h * nu.x, xc.y + sg * g.h * nu.y, xc.z + sg * g.h * nu.z};
        // the pressure lattice (cell centres) takes the half-cell axes on
        // all three axes; velocity lattice i the integer one along axis i
        // each fit computes its own axes: their exponentials overlap that
        // fit's 27 gathers (sharing the half-cell axes across the four fits
        // leaves the gathers exposed and measured slower)
        double ap[4], G[3][3];
        {
            MlsAxis X, Y, Z;
            mls_axis(y.x, 0.5, g.nx, g, X);
            mls_axis(y.y, 0.5, g.ny, g, Y);
            mls_axis(y.z, 0.5, g.nz, g, Z);
            bad |= !mls_fit<R>(X, Y, Z, g, pr, ap);
        }
#pragma unroll 1
        for (int i = 0; i < 3; ++i) {
            double ai[4];
            MlsAxis X, Y, Z;
            mls_axis(y.x, mac_off(i, 0), g.nx, g, X);
            mls_axis(y.y, mac_off(i, 1), g.ny, g, Y);
            mls_axis(y.z, mac_off(i, 2), g.nz, g, Z);
            bad |= !mls_fit<R>(X, Y, Z, g, u + i * g.field, ai);
            G[i][0] = ai[1] * g.inv_h;
            G[i][1] = ai[2] * g.inv_h;
            G[i][2] = ai[3] * g.inv_h;
        }
        const double pl = ap[0] + sg * g.h * an;
        const double n3[3] = {nu.x, nu.y, nu.z};
        double Fs[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double tn = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) tn += mu * (G[i][j] + G[j][i]) * n3[j];
            Fs[i] = sg * (-pl * n3[i] + tn) * area;
        }
        F0 += Fs[0];
        F1 += Fs[1];
        F2 += Fs[2];
    }
    Fext[3 * f] = (R)F0;
    Fext[3 * f + 1] = (R)F1;
    Fext[3 * f + 2] = (R)F2;
    if (bad) atomicOr(status, IP_STATUS_NONFINITE);
}

// The centroid's cell (the stencil centre of the lattices staggered by half a
// cell, as the fused step's tile uses): the supports of all three lattices lie
// in points cell - 1 .. cell + 2 per axis.
__device__ __forceinline__ int mls_cell(double x, double inv_h) {
    double c = floor((x * inv_h - 0.5) + 0.5);      // the expression mls_shape uses
    if (!(fabs(c) < 1.0e9)) c = 0.0;
    return (int)c;
}

// Centroid of the face with unit-local corners q (positions in LDS).
__device__ __forceinline__ vec3<double> marker_of(const double *xs, const uint16_t *q) {
    const vec3<double> s = ldx(xs, q[0]) + ldx(xs, q[1]) + ldx(xs, q[2]);
    return vec3<double>{s.x * (1.0 / 3.0), s.y * (1.0 / 3.0), s.z * (1.0 / 3.0)};
}

struct MlsUnitArgs {
    const double *X;
    const void *Fm;          // marker forces (spreading)
    const void *u, *Vb;      // velocity field and desired marker velocity (direct forcing)
    void *Fout;              // marker forces written by direct forcing (may be NULL)
    double inv_dt;
    void *f;
    MlsGrid g;
    uint32_t *status;
    const int64_t *node_off;
    const int32_t *wu_body, *wu_owned, *wu_nodes, *frec_perm;
    const int64_t *wu_noff, *wu_foff;
    const uint16_t *frec_lid;
    int nmax, tile_bytes;
};

// Spreading of the faces owned by one work unit (one workgroup per unit).
// DF (direct forcing): the marker force is F = (V^b - U) / dt with U
// interpolated from u with the same shape functions, stored to Fout when
// given, then spread.
template <typename R, int NT, bool DF>
__global__ __launch_bounds__(NT) void k_spread_mls_units(MlsUnitArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ double red[NT / 64];
    __shared__ int ired[6 * (NT / 64)];
    const int tid = threadIdx.x;
    const int w = blockIdx.x;
    const int b = a.wu_body[w];
    const int64_t nl0 = a.wu_noff[2 * w], nl1 = a.wu_noff[2 * w + 1];
    const bool whole = nl1 == nl0;
    const int64_t n0 = a.node_off[b];
    const int NL = whole ? (int)(a.node_off[b + 1] - n0) : (int)(nl1 - nl0);
    const int N = whole ? NL : a.wu_owned[w];
    const int32_t *gid = a.wu_nodes + nl0;
    const int64_t f0 = a.wu_foff[2 * w];
    const int F = (int)(a.wu_foff[2 * w + 1] - f0);
    if (NL == 0 || F == 0) return;     // uniform over the block
    double *xs = (double *)lds;                                  // [nmax][3]
    double *tile = xs + 3 * a.nmax;                              // tile_bytes
    const R *Fm = (const R *)a.Fm;
    R *fld = (R *)a.f;
    const MlsGrid &g = a.g;

    int lo[3], hi[3];
    load_positions<NT>(xs, a.X, whole, n0, gid, NL, N, g.inv_h, lo, hi);
    // cell box of the owned markers
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = INT_MAX;
        hi[c] = INT_MIN;
    }
    for (int t = tid; t < F; t += NT) {
        const uint16_t *q = a.frec_lid + 4 * (f0 + t);
        if (q[0] >= N) continue;                   // first corner not owned here
        const vec3<double> p = marker_of(xs, q);
        const int cc[3] = {mls_cell(p.x, g.inv_h), mls_cell(p.y, g.inv_h), mls_cell(p.z, g.inv_h)};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = min(lo[c], cc[c]);
            hi[c] = max(hi[c], cc[c]);
        }
    }
    double none[1] = {0.0};
    block_box_sums<NT, 1>(lo, hi, none, ired, red);
    if (lo[0] > hi[0]) return;                     // no owned marker (uniform)
    // tile points lo - 1 .. hi + 2 per axis
    const long long Lx = (long long)hi[0] - lo[0] + 4, Ly = (long long)hi[1] - lo[1] + 4,
                    Lz = (long long)hi[2] - lo[2] + 4;
    const bool use_tile = Lx <= g.nx && Ly <= g.ny && Lz <= g.nz && Lx * Ly * Lz * 8 <= a.tile_bytes;
    const int Tx = use_tile ? (int)Lx : 1, Ty = use_tile ? (int)Ly : 1, Tz = use_tile ? (int)Lz : 1;
    const long long Tl = (long long)Tx * Ty * Tz;
    TileGeom tg{{lo[0], lo[1], lo[2]}, Tx, Ty, Tz, (int)(use_tile ? Tl : 0), g.nx, g.ny, g.nz,
                g.plane, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if (use_tile) {
        tg.g0[0] = wrapi(lo[0] - 1, g.nx);
        tg.g0[1] = wrapi(lo[1] - 1, g.ny);
        tg.g0[2] = wrapi(lo[2] - 1, g.nz);
        const int qn = NT / Tx, r = tid / Tx;
        tg.s[0] = NT % Tx;
        tg.s[1] = qn % Ty;
        tg.s[2] = qn / Ty;
        tg.c0[0] = tid % Tx;
        tg.c0[1] = r % Ty;
        tg.c0[2] = r / Ty;
    }
    bool bad = false;
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        R *fd = fld + d * g.field;
        if (use_tile) {
            for (int t = tid; t < tg.T; t += NT) tile[t] = 0.0;
            lds_barrier();
        }
        for (int t = tid; t < F; t += NT) {
            const uint16_t *q = a.frec_lid + 4 * (f0 + t);
            if (q[0] >= N) continue;
            const vec3<double> xa = ldx(xs, q[0]), xb = ldx(xs, q[1]), xc = ldx(xs, q[2]);
            const vec3<double> n = cross(xb - xa, xc - xa);
            const double area = 0.5 * sqrt(dot(n, n));
            const vec3<double> p = marker_of(xs, q);
            MlsShape S;
            bad |= !mls_shape(p, d, g, S);
            double sphi = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int i = 0; i < 3; ++i) sphi += mls_phi(S, i, j, k);
            const double hl = (1.0 / 3.0) * sphi * (3.0 * g.h);
            const double cl = area * hl / (sphi * g.h * g.h * g.h);
            const int64_t pf = a.frec_perm[f0 + t];
            double Fl;
            if constexpr (DF) {
                const R *ud = (const R *)a.u + d * g.field;
                double U = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const R *row = ud + (int64_t)S.idx[2][k] * g.plane + (int64_t)S.idx[1][j] * g.nx;
#pragma unroll
                        for (int i = 0; i < 3; ++i) U += mls_phi(S, i, j, k) * (double)row[S.idx[0][i]];
                    }
                Fl = ((double)((const R *)a.Vb)[3 * pf + d] - U) * a.inv_dt;
                if (a.Fout != nullptr) ((R *)a.Fout)[3 * pf + d] = (R)Fl;
            } else {
                Fl = (double)Fm[3 * pf + d];
            }
            const double Fd = Fl * cl;
            // support point c - 1 + j is tile point c + j - lo (inside the tile
            // for every marker the box was taken from; checked all the same)
            const int ox = S.c[0] - lo[0], oy = S.c[1] - lo[1], oz = S.c[2] - lo[2];
            const bool in_tile = use_tile && ox >= 0 && oy >= 0 && oz >= 0 && ox + 2 < Tx &&
                                 oy + 2 < Ty && oz + 2 < Tz;
            if (in_tile) {
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int j = 0; j < 3; ++j)
#pragma unroll
                        for (int i = 0; i < 3; ++i)
                            lds_add(tile + ((oz + k) * Ty + (oy + j)) * Tx + (ox + i),
                                    mls_phi(S, i, j, k) * Fd);
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        R *row = fd + (int64_t)S.idx[2][k] * g.plane + (int64_t)S.idx[1][j] * g.nx;
#pragma unroll
                        for (int i = 0; i < 3; ++i)
                            unsafeAtomicAdd(row + S.idx[0][i], (R)(mls_phi(S, i, j, k) * Fd));
                    }
            }
        }
        if (use_tile) {
            lds_barrier();
            for (TileCursor c = TileCursor::first(tg); c.t < tg.T; c.template next<NT>(tg)) {
                const double v = tile[c.t];
                if (v != 0.0) unsafeAtomicAdd(fd + c.grid_index(tg), (R)v);
            }
            lds_barrier();
        }
    }
    if (bad) atomicOr(a.status, IP_STATUS_NONFINITE);
}

// Fn[n] = (1/3) sum of Fc over the faces of node n (deterministic gather over
// the node's face-corner slots, slot = 4 E + 3 f + corner).
template <typename R>
__global__ __launch_bounds__(256) void k_centroid_to_nodes(const int32_t *__restrict__ ptr,
                                                           const int32_t *__restrict__ slot,
                                                           int64_t N, int64_t E4,
                                                           const R *__restrict__ Fc,
                                                           R *__restrict__ Fn) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int q = ptr[n]; q < ptr[n + 1]; ++q) {
        const int64_t sl = slot[q];
        if (sl < E4) continue;
        const int64_t f = (sl - E4) / 3;
        s0 += (double)Fc[3 * f];
        s1 += (double)Fc[3 * f + 1];
        s2 += (double)Fc[3 * f + 2];
    }
    Fn[3 * n] = (R)(s0 * (1.0 / 3.0));
    Fn[3 * n + 1] = (R)(s1 * (1.0 / 3.0));
    Fn[3 * n + 2] = (R)(s2 * (1.0 / 3.0));
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

MlsGrid mls_grid(const ip_plan *p, double alpha) {
    MlsGrid g;
    g.nx = p->grid.nx;
    g.ny = p->grid.ny;
    g.nz = p->grid.nz;
    g.h = p->grid.h;
    g.inv_h = 1.0 / p->grid.h;
    g.plane = (int64_t)g.nx * g.ny;
    g.field = g.plane * g.nz;
    g.inv_alpha = 1.0 / alpha;
    const double q = (1.0 / 1.5) * g.inv_alpha;
    g.q2 = q * q;
    g.cq = std::exp(-g.q2);
    // with q^2 <= 200 the factors exp(+-2 d q^2), |d| <= 1/2, and exp(-q^2)
    // stay far inside the double range; beyond, each weight takes its own
    // exponential
    g.fast = g.q2 <= 200.0 ? 1 : 0;
    return g;
}

}  // namespace

// Arguments and LDS size of the per-unit kernels: positions [nmax][3] and the
// largest tile that fits beside them (1 KB kept for the static LDS).
static ip_status unit_args(ip_plan *p, const double *X, double alpha, MlsUnitArgs &a,
                           size_t &lds) {
    const int lds_optin = p->lds_optin;
    a.X = X;
    a.g = mls_grid(p, alpha);
    a.status = p->status;
    a.node_off = p->node_off;
    a.wu_body = p->wu_body;
    a.wu_owned = p->wu_owned;
    a.wu_nodes = p->wu_nodes;
    a.frec_perm = p->frec_perm;
    a.wu_noff = p->wu_noff;
    a.wu_foff = p->wu_foff;
    a.frec_lid = p->frec_lid;
    a.nmax = p->fused_nmax;
    a.tile_bytes = (int)std::max<long long>((lds_optin - 1024 - 24LL * a.nmax) / 16 * 16, 0);
    lds = (size_t)24 * a.nmax + (size_t)a.tile_bytes;
    return IP_OK;
}

// One workgroup per unit fills the LDS with its tile, so the workgroup size
// sets the waves per SIMD: 768 threads give 3 (512 gave 2 and were slower).
constexpr int kMlsThreads = 768;

// Launch attributes of the per-unit kernels (their dynamic LDS), set once when
// the plan is built, so that the launches themselves can be captured.
template <typename R>
static ip_status set_unit_attributes(size_t lds) {
    const void *fns[2] = {(const void *)k_spread_mls_units<R, kMlsThreads, false>,
                          (const void *)k_spread_mls_units<R, kMlsThreads, true>};
    for (const void *fn : fns)
        IP_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return IP_OK;
}

ip_status prepare_mls_units(ip_plan *p) {
    if (!p->fused_all || p->n_units == 0) return IP_OK;
    MlsUnitArgs a{};
    size_t lds = 0;
    IP_TRY(unit_args(p, nullptr, 1.0, a, lds));
    return p->prec == IP_F64 ? set_unit_attributes<double>(lds) : set_unit_attributes<float>(lds);
}

ip_status launch_interp_mls(ip_plan *p, const double *X, const void *u, double alpha, void *U,
                            hipStream_t s) {
    if (p->F == 0) return IP_OK;
    const MlsGrid g = mls_grid(p, alpha);
    const dim3 grid(nblocks(p->F, 256)), block(256);
    if (p->prec == IP_F64)
        hipLaunchKernelGGL(k_interp_mls<double>, grid, block, 0, s, X, p->faces, p->F,
                           (const double *)u, g, (double *)U, p->status);
    else
        hipLaunchKernelGGL(k_interp_mls<float>, grid, block, 0, s, X, p->faces, p->F,
                           (const float *)u, g, (float *)U, p->status);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

ip_status launch_spread_mls(ip_plan *p, const double *X, const void *Fm, double alpha, void *f,
                            hipStream_t s) {
    if (p->F == 0) return IP_OK;
    const MlsGrid g = mls_grid(p, alpha);
    if (p->fused_all && p->n_units > 0) {
        MlsUnitArgs a{};
        size_t lds = 0;
        IP_TRY(unit_args(p, X, alpha, a, lds));
        a.Fm = Fm;
        a.f = f;
        if (p->prec == IP_F64)
            hipLaunchKernelGGL((k_spread_mls_units<double, kMlsThreads, false>), dim3(p->n_units),
                               dim3(kMlsThreads), lds, s, a);
        else
            hipLaunchKernelGGL((k_spread_mls_units<float, kMlsThreads, false>), dim3(p->n_units),
                               dim3(kMlsThreads), lds, s, a);
        IP_HIP_CHECK(hipGetLastError());
        return IP_OK;
    }
    const dim3 grid(nblocks(p->F, 256)), block(256);
    if (p->prec == IP_F64)
        hipLaunchKernelGGL(k_spread_mls<double>, grid, block, 0, s, X, p->faces, p->F,
                           (const double *)Fm, g, (double *)f, p->status);
    else
        hipLaunchKernelGGL(k_spread_mls<float>, grid, block, 0, s, X, p->faces, p->F,
                           (const float *)Fm, g, (float *)f, p->status);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

ip_status launch_direct_forcing_mls(ip_plan *p, const double *X, const void *Vb, const void *u,
                                    double alpha, double dt, void *Fout, void *f, hipStream_t s) {
    if (p->F == 0) return IP_OK;
    const MlsGrid g = mls_grid(p, alpha);
    if (p->fused_all && p->n_units > 0) {
        MlsUnitArgs a{};
        size_t lds = 0;
        IP_TRY(unit_args(p, X, alpha, a, lds));
        a.u = u;
        a.Vb = Vb;
        a.Fout = Fout;
        a.inv_dt = 1.0 / dt;
        a.f = f;
        if (p->prec == IP_F64)
            hipLaunchKernelGGL((k_spread_mls_units<double, kMlsThreads, true>), dim3(p->n_units),
                               dim3(kMlsThreads), lds, s, a);
        else
            hipLaunchKernelGGL((k_spread_mls_units<float, kMlsThreads, true>), dim3(p->n_units),
                               dim3(kMlsThreads), lds, s, a);
        IP_HIP_CHECK(hipGetLastError());
        return IP_OK;
    }
    const dim3 grid(nblocks(p->F, 256)), block(256);
    if (p->prec == IP_F64)
        hipLaunchKernelGGL(k_direct_forcing_mls<double>, grid, block, 0, s, X, p->faces, p->F,
                           (const double *)u, (const double *)Vb, g, 1.0 / dt,
                           (double *)Fout, (double *)f, p->status);
    else
        hipLaunchKernelGGL(k_direct_forcing_mls<float>, grid, block, 0, s, X, p->faces, p->F,
                           (const float *)u, (const float *)Vb, g, 1.0 / dt,
                           (float *)Fout, (float *)f, p->status);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

ip_status launch_probe_loads(ip_plan *p, const double *X, const void *u, const void *pr,
                             const void *acc, double alpha, double mu, void *Fext, hipStream_t s) {
    if (p->F == 0) return IP_OK;
    const MlsGrid g = mls_grid(p, alpha);
    const dim3 grid(nblocks(p->F, 256)), block(256);
    if (p->prec == IP_F64)
        hipLaunchKernelGGL(k_probe_loads<double>, grid, block, 0, s, X, p->faces, p->face_off,
                           p->closed, p->B, p->F, (const double *)u, (const double *)pr,
                           (const double *)acc, g, mu, (double *)Fext, p->status);
    else
        hipLaunchKernelGGL(k_probe_loads<float>, grid, block, 0, s, X, p->faces, p->face_off,
                           p->closed, p->B, p->F, (const float *)u, (const float *)pr,
                           (const float *)acc, g, mu, (float *)Fext, p->status);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

ip_status launch_centroid_to_nodes(ip_plan *p, const void *Fc, void *Fn, hipStream_t s) {
    if (p->N == 0) return IP_OK;
    const dim3 grid(nblocks(p->N, 256)), block(256);
    if (p->prec == IP_F64)
        hipLaunchKernelGGL(k_centroid_to_nodes<double>, grid, block, 0, s, p->csr_ptr,
                           p->csr_slot, p->N, 4 * p->E, (const double *)Fc, (double *)Fn);
    else
        hipLaunchKernelGGL(k_centroid_to_nodes<float>, grid, block, 0, s, p->csr_ptr,
                           p->csr_slot, p->N, 4 * p->E, (const float *)Fc, (float *)Fn);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}
