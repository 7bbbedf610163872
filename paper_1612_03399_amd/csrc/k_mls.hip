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
#include "ipibm_internal.h"

namespace {

struct MlsGrid {
    int nx, ny, nz;
    double h, inv_h;
    int64_t plane, field;
};

struct MlsShape {
    double w[3][3];      // per-axis weights of the 3 support points
    double dk[3][3];     // per-axis offsets (x^k - x) / h
    double z[4];         // A^{-1} e_0
    int idx[3][3];       // wrapped lattice indices per axis
};

__device__ __forceinline__ bool mls_shape(const vec3<double> &x, int d, const MlsGrid &g,
                                          double inv_alpha, MlsShape &S) {
    const double xs[3] = {x.x, x.y, x.z};
    const int n[3] = {g.nx, g.ny, g.nz};
    double s0[3], s1[3], s2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double s = xs[a] * g.inv_h - mac_off(d, a);
        double c = floor(s + 0.5);
        if (!(fabs(c) < 1.0e9)) c = 0.0;           // non-finite or absurd position
        s0[a] = s1[a] = s2[a] = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double dk = (c - 1.0 + j) - s;
            const double r = fabs(dk) * (1.0 / 1.5) * inv_alpha;   // (r_k / alpha)
            const double w = fabs(dk) <= 1.5 ? exp(-r * r) : 0.0;
            S.w[a][j] = w;
            S.dk[a][j] = dk;
            S.idx[a][j] = wrapi((int)c - 1 + j, n[a]);
            s0[a] += w;
            s1[a] += w * dk;
            s2[a] += w * dk * dk;
        }
    }
    // moment matrix (symmetric): A_00 = X0 Y0 Z0, A_01 = X1 Y0 Z0, ...
    const double a00 = s0[0] * s0[1] * s0[2];
    const double a01 = s1[0] * s0[1] * s0[2], a02 = s0[0] * s1[1] * s0[2], a03 = s0[0] * s0[1] * s1[2];
    const double a11 = s2[0] * s0[1] * s0[2], a22 = s0[0] * s2[1] * s0[2], a33 = s0[0] * s0[1] * s2[2];
    const double a12 = s1[0] * s1[1] * s0[2], a13 = s1[0] * s0[1] * s1[2], a23 = s0[0] * s1[1] * s1[2];
    // Cholesky A = L L^T
    const double l00 = sqrt(a00);
    const double l10 = a01 / l00, l20 = a02 / l00, l30 = a03 / l00;
    const double l11 = sqrt(a11 - l10 * l10);
    const double l21 = (a12 - l20 * l10) / l11, l31 = (a13 - l30 * l10) / l11;
    const double l22 = sqrt(a22 - l20 * l20 - l21 * l21);
    const double l32 = (a23 - l30 * l20 - l31 * l21) / l22;
    const double l33 = sqrt(a33 - l30 * l30 - l31 * l31 - l32 * l32);
    // L y = e_0, L^T z = y
    const double y0 = 1.0 / l00;
    const double y1 = -l10 * y0 / l11;
    const double y2 = -(l20 * y0 + l21 * y1) / l22;
    const double y3 = -(l30 * y0 + l31 * y1 + l32 * y2) / l33;
    S.z[3] = y3 / l33;
    S.z[2] = (y2 - l32 * S.z[3]) / l22;
    S.z[1] = (y1 - l21 * S.z[2] - l31 * S.z[3]) / l11;
    S.z[0] = (y0 - l10 * S.z[1] - l20 * S.z[2] - l30 * S.z[3]) / l00;
    return isfinite(S.z[0]) && isfinite(S.z[1]) && isfinite(S.z[2]) && isfinite(S.z[3]);
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
                                                    double inv_alpha, R *__restrict__ U,
                                                    uint32_t *status) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double area;
    const vec3<double> x = centroid(X, faces, f, area);
    bool bad = false;
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        MlsShape S;
        bad |= !mls_shape(x, d, g, inv_alpha, S);
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
                                                    double inv_alpha, R *__restrict__ fld,
                                                    uint32_t *status) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double area;
    const vec3<double> x = centroid(X, faces, f, area);
    bool bad = false;
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        MlsShape S;
        bad |= !mls_shape(x, d, g, inv_alpha, S);
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

MlsGrid mls_grid(const ip_plan *p) {
    MlsGrid g;
    g.nx = p->grid.nx;
    g.ny = p->grid.ny;
    g.nz = p->grid.nz;
    g.h = p->grid.h;
    g.inv_h = 1.0 / p->grid.h;
    g.plane = (int64_t)g.nx * g.ny;
    g.field = g.plane * g.nz;
    return g;
}

}  // namespace

ip_status launch_interp_mls(ip_plan *p, const double *X, const void *u, double alpha, void *U,
                            hipStream_t s) {
    if (p->F == 0) return IP_OK;
    const MlsGrid g = mls_grid(p);
    const dim3 grid(nblocks(p->F, 256)), block(256);
    if (p->prec == IP_F64)
        hipLaunchKernelGGL(k_interp_mls<double>, grid, block, 0, s, X, p->faces, p->F,
                           (const double *)u, g, 1.0 / alpha, (double *)U, p->status);
    else
        hipLaunchKernelGGL(k_interp_mls<float>, grid, block, 0, s, X, p->faces, p->F,
                           (const float *)u, g, 1.0 / alpha, (float *)U, p->status);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

ip_status launch_spread_mls(ip_plan *p, const double *X, const void *Fm, double alpha, void *f,
                            hipStream_t s) {
    if (p->F == 0) return IP_OK;
    const MlsGrid g = mls_grid(p);
    const dim3 grid(nblocks(p->F, 256)), block(256);
    if (p->prec == IP_F64)
        hipLaunchKernelGGL(k_spread_mls<double>, grid, block, 0, s, X, p->faces, p->F,
                           (const double *)Fm, g, 1.0 / alpha, (double *)f, p->status);
    else
        hipLaunchKernelGGL(k_spread_mls<float>, grid, block, 0, s, X, p->faces, p->F,
                           (const float *)Fm, g, 1.0 / alpha, (float *)f, p->status);
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
