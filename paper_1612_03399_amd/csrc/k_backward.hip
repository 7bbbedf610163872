// k_backward.hip -- derivatives of the explicit step (FP64 plans).
//
// Forces: F = -grad W, so dF/dX is symmetric and its product with a vector is
// both the JVP and the VJP.  It is evaluated in forward mode: positions carry a
// tangent (dual numbers) through the same element code as the forward pass,
// and the body volume's tangent dV = sum_i dV/dx_i . dx_i (the rank-one part of
// the volume term's Hessian) comes from the dual-valued volume reduction.
//
// Reverse step (explicit update X' = X + M (dt U(X) + dt^2/m F(X; k)), M the
// not-pinned mask), for an adjoint lam' = dL/dX' and P = M lam':
//   lam = lam' + dt J_U(X)^T P + (dt^2/m) (dF/dX) P
//   dL/dk_s (body b) += (dt^2/m_b) sum_{l in b} (F_s,l / k_s) . P_l
//   dL/du += dt h^3 spread(P)        (interpolation's adjoint is spreading)
// F_s is linear in k_s, so F_s/k_s is the family's force at unit constant.
#include "step_common.h"
#include "xcd.h"

namespace {

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

__device__ __forceinline__ vec3<dual> ldXd(const double *X, const double *T, int64_t i) {
    return {dual(X[3 * i], T[3 * i]), dual(X[3 * i + 1], T[3 * i + 1]),
            dual(X[3 * i + 2], T[3 * i + 2])};
}

__device__ __forceinline__ double block_sum_any(double v, double *sh) { return block_sum(v, sh); }

// Volume of each body with its tangent along T (anchor = first node).
__global__ __launch_bounds__(256) void k_volume_dual(const double *__restrict__ X,
                                                     const double *__restrict__ T,
                                                     const int32_t *__restrict__ faces,
                                                     const int64_t *__restrict__ node_off,
                                                     const int64_t *__restrict__ face_off,
                                                     double *__restrict__ V,
                                                     double *__restrict__ dV) {
    __shared__ double sh[4];
    const int b = blockIdx.x;
    if (face_off[b] == face_off[b + 1]) {
        if (threadIdx.x == 0) V[b] = dV[b] = 0.0;
        return;
    }
    const vec3<dual> a = ldXd(X, T, node_off[b]);
    double v = 0.0, dv = 0.0;
    for (int64_t f = face_off[b] + threadIdx.x; f < face_off[b + 1]; f += blockDim.x) {
        const int32_t *t = faces + 3 * f;
        dual v6;
        double a2;
        face_geometry<dual, double>(ldXd(X, T, t[0]), ldXd(X, T, t[1]), ldXd(X, T, t[2]), a, v6,
                                    a2);
        v += v6.v;
        dv += v6.d;
    }
    v = block_sum_any(v, sh);
    dv = block_sum_any(dv, sh);
    if (threadIdx.x == 0) {
        V[b] = v / 6.0;
        dV[b] = dv / 6.0;
    }
}

// Edge elements along tangent T: 4 slot vectors (tangents of the node forces)
// and, when P is given, the dot products of the spring and hinge forces with P
// at their nodes (dotE[e][0..1]).
__global__ __launch_bounds__(256) void k_edges_jvp(
    const double *__restrict__ X, const double *__restrict__ T, const int4 *__restrict__ e4,
    const int64_t *__restrict__ edge_off, int B, int64_t E, const double *__restrict__ l0,
    const double *__restrict__ cs0, const double *__restrict__ ks, const double *__restrict__ kb,
    const double *__restrict__ ew, const double *__restrict__ P, double *__restrict__ slots,
    double *__restrict__ dotE) {
    const int64_t e = xcd_block() * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int b = body_of(edge_off, B, e);
    const double ws = ew ? ew[2 * e] : 1.0, wb = ew ? ew[2 * e + 1] : 1.0;
    const int4 q = e4[e];
    const bool hinge = q.z >= 0 && q.w >= 0;
    const vec3<dual> x1 = ldXd(X, T, q.x), x2 = ldXd(X, T, q.y);
    vec3<dual> x3 = x1, x4 = x1;
    if (hinge) {
        x3 = ldXd(X, T, q.z);
        x4 = ldXd(X, T, q.w);
    }
    vec3<dual> fsp, h1, h2, h3, h4;
    edge_parts<dual, dual>(x1, x2, x3, x4, hinge, dual(l0[e]),
                           dual(cs0[2 * e]), dual(cs0[2 * e + 1]), ks[b] * ws, kb[b] * wb, fsp, h1,
                           h2, h3, h4);
    const vec3<dual> f1 = fsp + h1, f2 = h2 - fsp;
    double *o = slots + 12 * e;
    o[0] = f1.x.d; o[1] = f1.y.d; o[2] = f1.z.d;
    o[3] = f2.x.d; o[4] = f2.y.d; o[5] = f2.z.d;
    o[6] = h3.x.d; o[7] = h3.y.d; o[8] = h3.z.d;
    o[9] = h4.x.d; o[10] = h4.y.d; o[11] = h4.z.d;
    if (dotE) {
        // family forces at unit constants (F_s is linear in k_s), dotted with P
        const vec3<double> y1 = {x1.x.v, x1.y.v, x1.z.v}, y2 = {x2.x.v, x2.y.v, x2.z.v},
                           y3 = {x3.x.v, x3.y.v, x3.z.v}, y4 = {x4.x.v, x4.y.v, x4.z.v};
        vec3<double> u0, u1, u2, u3, u4;
        edge_parts<double, double>(y1, y2, y3, y4, hinge, l0[e],
                                   cs0[2 * e], cs0[2 * e + 1], 1.0, 1.0, u0, u1, u2, u3, u4);
        const vec3<double> p1 = ldX(P, q.x), p2 = ldX(P, q.y);
        double bend = 0.0;
        if (hinge) {
            const vec3<double> p3 = ldX(P, q.z), p4 = ldX(P, q.w);
            bend = dot(u1, p1) + dot(u2, p2) + dot(u3, p3) + dot(u4, p4);
        }
        dotE[2 * e] = ws * dot(u0, p1 - p2);
        dotE[2 * e + 1] = wb * bend;
    }
}

// Face elements along tangent T (the volume coefficient's tangent comes from
// dV); dot products of the area and volume forces with P (dotF[f][0..1]).
__global__ __launch_bounds__(256) void k_faces_jvp(
    const double *__restrict__ X, const double *__restrict__ T,
    const int32_t *__restrict__ faces, const int64_t *__restrict__ face_off, int B, int64_t F,
    const double *__restrict__ A0, const double *__restrict__ V0, const double *__restrict__ V,
    const double *__restrict__ dV, const uint8_t *__restrict__ closed,
    const double *__restrict__ kA, const double *__restrict__ kV, const double *__restrict__ P,
    double *__restrict__ slots, double *__restrict__ dotF) {
    const int64_t f = xcd_block() * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int b = body_of(face_off, B, f);
    const int32_t *t = faces + 3 * f;
    const dual sV = volume_coefficient<dual>(closed[b] != 0, kV[b], dual(V[b], dV[b]), V0[b]);
    const vec3<dual> xi = ldXd(X, T, t[0]), xj = ldXd(X, T, t[1]), xk = ldXd(X, T, t[2]);
    vec3<dual> gi, gj, gk, gv;
    face_parts<dual, dual>(xi, xj, xk, dual(A0[f]), kA[b], sV, gi, gj, gk, gv);
    double *o = slots + 9 * f;
    o[0] = gi.x.d + gv.x.d; o[1] = gi.y.d + gv.y.d; o[2] = gi.z.d + gv.z.d;
    o[3] = gj.x.d + gv.x.d; o[4] = gj.y.d + gv.y.d; o[5] = gj.z.d + gv.z.d;
    o[6] = gk.x.d + gv.x.d; o[7] = gk.y.d + gv.y.d; o[8] = gk.z.d + gv.z.d;
    if (dotF) {
        // family forces at unit constants, dotted with P
        const vec3<double> yi = {xi.x.v, xi.y.v, xi.z.v}, yj = {xj.x.v, xj.y.v, xj.z.v},
                           yk = {xk.x.v, xk.y.v, xk.z.v};
        const double sV1 = volume_coefficient<double>(closed[b] != 0, 1.0, V[b], V0[b]);
        vec3<double> ai, aj, ak, av;
        face_parts<double, double>(yi, yj, yk, A0[f], 1.0, sV1, ai, aj, ak, av);
        const vec3<double> pi = ldX(P, t[0]), pj = ldX(P, t[1]), pk = ldX(P, t[2]);
        dotF[2 * f] = dot(ai, pi) + dot(aj, pj) + dot(ak, pk);
        dotF[2 * f + 1] = dot(av, pi + pj + pk);
    }
}

// Node gather of the tangent slots (same lists as the forward gather).
__global__ void k_gather_f64(const int32_t *__restrict__ ptr, const int32_t *__restrict__ ids,
                             const double *__restrict__ slots, int64_t N, double *__restrict__ out) {
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double fx = 0, fy = 0, fz = 0;
    for (int32_t s = ptr[i]; s < ptr[i + 1]; ++s) {
        const double *v = slots + 3 * (int64_t)ids[s];
        fx += v[0];
        fy += v[1];
        fz += v[2];
    }
    out[3 * i] = fx;
    out[3 * i + 1] = fy;
    out[3 * i + 2] = fz;
}

// P = M lam' (pinned rows zeroed)
__global__ void k_mask(const double *__restrict__ lam, const uint8_t *__restrict__ pinned,
                       int64_t N, double *__restrict__ P) {
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= 3 * N) return;
    P[i] = pinned[i / 3] ? 0.0 : lam[i];
}

// dL/dk_s for body b: (dt^2/m_b) times the sum of the body's unit-constant dots.
__global__ __launch_bounds__(256) void k_gk(const double *__restrict__ dotE,
                                            const double *__restrict__ dotF,
                                            const int64_t *__restrict__ edge_off,
                                            const int64_t *__restrict__ face_off,
                                            const double *__restrict__ mass, double dt, int B,
                                            double *__restrict__ gk) {
    __shared__ double sh[4];
    const int b = blockIdx.x;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int64_t e = edge_off[b] + threadIdx.x; e < edge_off[b + 1]; e += blockDim.x) {
        s0 += dotE[2 * e];
        s1 += dotE[2 * e + 1];
    }
    for (int64_t f = face_off[b] + threadIdx.x; f < face_off[b + 1]; f += blockDim.x) {
        s2 += dotF[2 * f];
        s3 += dotF[2 * f + 1];
    }
    s0 = block_sum(s0, sh);
    s1 = block_sum(s1, sh);
    s2 = block_sum(s2, sh);
    s3 = block_sum(s3, sh);
    if (threadIdx.x == 0) {
        const double c = dt * dt / mass[b];
        gk[b] += c * s0;
        gk[B + b] += c * s1;
        gk[2 * B + b] += c * s2;
        gk[3 * B + b] += c * s3;
    }
}

// Weights of the 3-point delta and their derivatives with respect to the
// fractional coordinate s at the points c-1, c, c+1 (r = s - c, q = sqrt(1-3r^2)):
//   dw/ds = ((r/q - 1)/2, -r/q, (1 + r/q)/2).
__device__ __forceinline__ int delta3_d(double s, double w[3], double dw[3]) {
    double c = floor(s + 0.5);
    if (!(fabs(c) < 1.0e9)) c = 0.0;
    const double r = s - c;
    const double v = 1.0 - 3.0 * r * r;
    const double iq = rsq_nr(v);
    const double q = v * iq;
    w[0] = (2.0 - 3.0 * r - q) * (1.0 / 6.0);
    w[1] = (1.0 + q) * (1.0 / 3.0);
    w[2] = (2.0 + 3.0 * r - q) * (1.0 / 6.0);
    const double rq = r * iq;
    dw[0] = 0.5 * (rq - 1.0);
    dw[1] = -rq;
    dw[2] = 0.5 * (1.0 + rq);
    return (int)c;
}

// lam = lam' + dt J_U^T P + c_b dF  (and X-independent pinned rows: lam = lam')
// J_U[d][e] = dU_d/dX_e = sum over lattice d's 27 points of u_d * dw/dX_e.
// g = J_U(x)^T p = sum_d p_d dU_d/dx: the gradient of the interpolated
// velocity at x (3-point delta and its derivative per axis) dotted with p.
__device__ __forceinline__ void interp_grad_dot(const vec3<double> &x, const vec3<double> &p,
                                                const double *__restrict__ u, int nx, int ny,
                                                int nz, double inv_h, double g[3]) {
    const double pd[3] = {p.x, p.y, p.z};
    const double xv[3] = {x.x, x.y, x.z};
    const int64_t plane = (int64_t)nx * ny, field = plane * nz;
    g[0] = g[1] = g[2] = 0.0;
    for (int d = 0; d < 3; ++d) {
        double w[3][3], dw[3][3];
        int cc[3];
        for (int ax = 0; ax < 3; ++ax)
            cc[ax] = delta3_d(xv[ax] * inv_h - mac_off(d, ax), w[ax], dw[ax]);
        const double *ud = u + d * field;
        const int ix[3] = {wrapi(cc[0] - 1, nx), wrapi(cc[0], nx), wrapi(cc[0] + 1, nx)};
        double gx = 0.0, gy = 0.0, gz = 0.0;
        // separable: per (y, z) row the x-sums with w and dw, then the row's
        // weights for each component
        for (int kz = 0; kz < 3; ++kz)
            for (int ky = 0; ky < 3; ++ky) {
                const double *row = ud + wrapi(cc[2] - 1 + kz, nz) * plane +
                                    (int64_t)wrapi(cc[1] - 1 + ky, ny) * nx;
                const double u0 = row[ix[0]], u1 = row[ix[1]], u2 = row[ix[2]];
                const double rw = u0 * w[0][0] + u1 * w[0][1] + u2 * w[0][2];
                const double rd = u0 * dw[0][0] + u1 * dw[0][1] + u2 * dw[0][2];
                gx += rd * (w[1][ky] * w[2][kz]);
                gy += rw * (dw[1][ky] * w[2][kz]);
                gz += rw * (w[1][ky] * dw[2][kz]);
            }
        g[0] += pd[d] * gx * inv_h;
        g[1] += pd[d] * gy * inv_h;
        g[2] += pd[d] * gz * inv_h;
    }
}

__global__ __launch_bounds__(256) void k_lambda(const double *__restrict__ X,
                                                const double *__restrict__ u,
                                                const double *__restrict__ lam_in,
                                                const double *__restrict__ P,
                                                const double *__restrict__ dF,
                                                const int64_t *__restrict__ node_off, int B,
                                                const double *__restrict__ mass, int64_t N, int nx,
                                                int ny, int nz, double inv_h, double dt,
                                                double *__restrict__ lam_out) {
    const int64_t l = xcd_block() * blockDim.x + threadIdx.x;
    if (l >= N) return;
    const int b = body_of(node_off, B, l);
    const double c = dt * dt / mass[b];
    double g[3];
    interp_grad_dot(ldX(X, l), ldX(P, l), u, nx, ny, nz, inv_h, g);
    for (int e = 0; e < 3; ++e)
        lam_out[3 * l + e] = lam_in[3 * l + e] + dt * g[e] + c * dF[3 * l + e];
}

// gX = J_U^T dU per node (the adjoint of interpolation with respect to X).
__global__ __launch_bounds__(256) void k_interp_vjp_x(const double *__restrict__ X,
                                                      const double *__restrict__ u,
                                                      const double *__restrict__ dU, int64_t N,
                                                      int nx, int ny, int nz, double inv_h,
                                                      double *__restrict__ gX) {
    const int64_t l = xcd_block() * blockDim.x + threadIdx.x;
    if (l >= N) return;
    double g[3];
    interp_grad_dot(ldX(X, l), ldX(dU, l), u, nx, ny, nz, inv_h, g);
    for (int e = 0; e < 3; ++e) gX[3 * l + e] = g[e];
}

// F := s P (spreading source for the u-gradient)
__global__ void k_scale(const double *__restrict__ P, double s, int64_t n, double *__restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = s * P[i];
}

// ---------------------------------------------------------------------------
// Taylor deformation: C = (1/n) sum (x - c)(x - c)^T over the body's nodes;
// eigenvalues and eigenvectors of the symmetric 3x3 C by Jacobi rotations,
// L = sqrt(lambda_max), B = sqrt(lambda_min), D = (L - B)/(L + B).
// ---------------------------------------------------------------------------
struct Sym3 {
    double xx, yy, zz, xy, xz, yz;
};

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations
// (each rotation annihilates one off-diagonal entry; sweeps until every
// off-diagonal entry is negligible against its diagonal pair, which keeps the
// small eigenvalues of a nearly flat body accurate relative to themselves).
// lam[k] with eigenvector column vec[.][k].
__device__ void sym3_jacobi(const Sym3 &C, double lam[3], double vec[3][3]) {
    double m[3][3] = {{C.xx, C.xy, C.xz}, {C.xy, C.yy, C.yz}, {C.xz, C.yz, C.zz}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) vec[i][j] = i == j ? 1.0 : 0.0;
    const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
    for (int sweep = 0; sweep < 32; ++sweep) {
        bool rotated = false;
        for (int k = 0; k < 3; ++k) {
            const int p = P[k], q = Q[k];
            const double apq = m[p][q];
            if (apq == 0.0 || fabs(apq) <= 1e-18 * sqrt(fabs(m[p][p] * m[q][q]))) {
                m[p][q] = m[q][p] = 0.0;
                continue;
            }
            rotated = true;
            const double theta = (m[q][q] - m[p][p]) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
            m[p][p] -= t * apq;
            m[q][q] += t * apq;
            m[p][q] = m[q][p] = 0.0;
            const int r = 3 - p - q;
            const double arp = m[r][p], arq = m[r][q];
            m[r][p] = m[p][r] = c * arp - sn * arq;
            m[r][q] = m[q][r] = sn * arp + c * arq;
            for (int i = 0; i < 3; ++i) {
                const double vp = vec[i][p], vq = vec[i][q];
                vec[i][p] = c * vp - sn * vq;
                vec[i][q] = sn * vp + c * vq;
            }
        }
        if (!rotated) break;
    }
    for (int k = 0; k < 3; ++k) lam[k] = m[k][k];
}

// Per body: D[b]; with Dstar, also loss[b] = (D - D*)^2 and gX = dloss/dX.
// dlambda_k/dx_m = (2/n)(v_k . r_m) v_k (the mean's variation cancels).
__global__ __launch_bounds__(256) void k_taylor(const double *__restrict__ X,
                                                const int64_t *__restrict__ node_off,
                                                const double *__restrict__ Dstar,
                                                double *__restrict__ D,
                                                double *__restrict__ loss,
                                                double *__restrict__ gX) {
    __shared__ double sh[4];
    __shared__ double bc[12];
    const int b = blockIdx.x;
    const int64_t n0 = node_off[b], n1 = node_off[b + 1];
    const double n = (double)(n1 - n0);
    if (n1 == n0) {           // empty body: no deformation, no gradient
        if (threadIdx.x == 0) {
            if (D) D[b] = 0.0;
            if (Dstar) loss[b] = 0.0;
        }
        return;
    }
    double s[3] = {0, 0, 0};
    for (int64_t m = n0 + threadIdx.x; m < n1; m += blockDim.x)
        for (int c = 0; c < 3; ++c) s[c] += X[3 * m + c];
    for (int c = 0; c < 3; ++c) s[c] = block_sum(s[c], sh);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) bc[c] = s[c] / n;
    __syncthreads();
    const vec3<double> cm = {bc[0], bc[1], bc[2]};
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t m = n0 + threadIdx.x; m < n1; m += blockDim.x) {
        const vec3<double> r = ldX(X, m) - cm;
        acc[0] += r.x * r.x;
        acc[1] += r.y * r.y;
        acc[2] += r.z * r.z;
        acc[3] += r.x * r.y;
        acc[4] += r.x * r.z;
        acc[5] += r.y * r.z;
    }
    for (int c = 0; c < 6; ++c) acc[c] = block_sum(acc[c], sh);
    if (threadIdx.x == 0) {
        const Sym3 C = {acc[0] / n, acc[1] / n, acc[2] / n, acc[3] / n, acc[4] / n, acc[5] / n};
        double lam[3], vec[3][3];
        sym3_jacobi(C, lam, vec);
        int kx = 0, kn = 0;
        for (int q = 1; q < 3; ++q) {
            if (lam[q] > lam[kx]) kx = q;
            if (lam[q] < lam[kn]) kn = q;
        }
        const double L = sqrt(lam[kx]), Bs = sqrt(fmax(lam[kn], 0.0));
        const double Db = (L - Bs) / (L + Bs);
        if (D) D[b] = Db;
        if (Dstar) {
            const double r = Db - Dstar[b];
            loss[b] = r * r;
            const double dDdL = 2.0 * Bs / ((L + Bs) * (L + Bs));
            const double dDdB = -2.0 * L / ((L + Bs) * (L + Bs));
            const vec3<double> vmax = {vec[0][kx], vec[1][kx], vec[2][kx]};
            const vec3<double> vmin = {vec[0][kn], vec[1][kn], vec[2][kn]};
            bc[3] = 2.0 * r * dDdL / (2.0 * L);       // dloss/dlambda_max
            bc[4] = 2.0 * r * dDdB / (2.0 * Bs);      // dloss/dlambda_min
            bc[5] = vmax.x; bc[6] = vmax.y; bc[7] = vmax.z;
            bc[8] = vmin.x; bc[9] = vmin.y; bc[10] = vmin.z;
        }
    }
    __syncthreads();
    if (!Dstar || !gX) return;
    const double gmax = bc[3], gmin = bc[4];
    const vec3<double> vmax = {bc[5], bc[6], bc[7]}, vmin = {bc[8], bc[9], bc[10]};
    for (int64_t m = n0 + threadIdx.x; m < n1; m += blockDim.x) {
        const vec3<double> r = ldX(X, m) - cm;
        const double a = (2.0 / n) * gmax * dot(vmax, r), c = (2.0 / n) * gmin * dot(vmin, r);
        gX[3 * m] = a * vmax.x + c * vmin.x;
        gX[3 * m + 1] = a * vmax.y + c * vmin.y;
        gX[3 * m + 2] = a * vmax.z + c * vmin.z;
    }
}

// ---------------------------------------------------------------------------
// Fused reverse step: one workgroup per work unit, the same units, packed
// records and LDS layout as the fused forward step.  With P = M lam' (the
// adjoint of the new positions, pinned rows zeroed) read from memory:
//  P0  positions -> LDS, accumulators dF zeroed, cell box of the owned nodes.
//  P1  volume V and its tangent dV along P (a whole body; patched bodies'
//      come from a pass before this kernel).
//  P2  every element in dual numbers at unit constants, tangent P: the
//      tangents scaled by k_s go into dF = (dF/dX) P, the values dotted with
//      P give the constants' gradients (each element counted by the unit that
//      owns its first node).
//  P2b lam = lam' + dt^2/m dF for the owned nodes, held in registers.
//  P3  P' = dt h^3 P of the owned nodes replaces dF in LDS; counting sort by
//      cell as in the forward step.
//  P4  gu += spread(P') = dt sum P w (the adjoint of interpolation).
//  P5  per lattice: the velocity tile is staged, every owned node adds
//      sum_d P'_d dU_d/dX = dt h^3 (J_U^T P); lam += that / h^3 is written.
// ---------------------------------------------------------------------------
struct VjpArgs {
    const double *X, *lam_in;
    double *lam_out;           // whole units; patched units write lam_stage
    double *lam_stage;
    const int64_t *node_off;
    const uint8_t *closed, *pinned;
    const double *V0, *ks, *kb, *kA, *kV, *mass;
    const double *u;
    double *gu, *gk;
    int B;
    int nx, ny, nz;
    double inv_h, inv_h3;
    int64_t plane, field;
    double dt;
    const double *Vpre, *dVpre;   // patched bodies: volume and its tangent
    uint32_t *status;
    const int32_t *wu_body, *wu_owned, *wu_nodes;
    const uint8_t *wu_pinned;     // [n_units] some node of the unit pinned
    const int64_t *wu_noff, *wu_eoff, *wu_foff;
    const void *erec, *frec;
    const double *ew;             // [n_erec][2] per-edge weights on ks, kb (EW only)
    int unit_base, nmax, tile_bytes;
};

// EW: the edges carry per-edge weights on ks and kb (record order).
template <int NT, bool EW>
__global__ __launch_bounds__(NT, NT <= 256 ? 3 : 1) void k_step_vjp_fused(VjpArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ double red[4 * (NT / 64)];
    __shared__ int ired[6 * (NT / 64)];
    __shared__ int n_occ_sh;
    __shared__ int cnt_bins[kCountBins + 1];

    const int tid = threadIdx.x;
    const int w = a.unit_base + xcd_unit((int)blockIdx.x, (int)gridDim.x);
    const int b = a.wu_body[w];
    const int64_t nl0 = a.wu_noff[2 * w], nl1 = a.wu_noff[2 * w + 1];
    const bool whole = nl1 == nl0;
    const int64_t n0 = a.node_off[b];
    const int NL = whole ? (int)(a.node_off[b + 1] - n0) : (int)(nl1 - nl0);
    const int N = whole ? NL : a.wu_owned[w];
    const int32_t *gid = a.wu_nodes + nl0;
    const int64_t e0 = a.wu_eoff[2 * w];
    const int E = (int)(a.wu_eoff[2 * w + 1] - e0);
    const int64_t f0 = a.wu_foff[2 * w];
    const int F = (int)(a.wu_foff[2 * w + 1] - f0);
    if (NL == 0) return;

    double *xs = (double *)lds;
    double *dF = xs + 3 * a.nmax;                     // dF, then P' (P3 onwards)
    unsigned char *tile_region = (unsigned char *)(dF + 3 * a.nmax);
    double *ftile = (double *)tile_region;
    double *utile = (double *)tile_region;
    uint16_t *occ_start = (uint16_t *)(tile_region + a.tile_bytes);
    uint16_t *occ_cnt = occ_start + a.nmax;
    bool bad = false;
    const double c2 = a.dt * a.dt / a.mass[b];
    const auto gnode = [&](int l) -> int64_t { return whole ? n0 + l : (int64_t)gid[l]; };
    // units without pinned nodes skip the flag's load in every tangent
    const bool any_pin = a.wu_pinned[w] != 0;
    const auto tangent = [&](int l) -> vec3<double> {   // P of unit node l
        const int64_t g = gnode(l);
        if (any_pin && a.pinned[g]) return {0.0, 0.0, 0.0};
        return {a.lam_in[3 * g], a.lam_in[3 * g + 1], a.lam_in[3 * g + 2]};
    };
    const auto dualx = [&](int l, const vec3<double> &t) -> vec3<dual> {
        return {dual(xs[3 * l], t.x), dual(xs[3 * l + 1], t.y), dual(xs[3 * l + 2], t.z)};
    };
    const auto addd = [&](int l, double k, const vec3<dual> &v) {
        lds_add(dF + 3 * l, k * v.x.d);
        lds_add(dF + 3 * l + 1, k * v.y.d);
        lds_add(dF + 3 * l + 2, k * v.z.d);
    };
    // k1 v1 + k2 v2 in one addition per component
    const auto addd2 = [&](int l, double k1, const vec3<dual> &v1, double k2,
                           const vec3<dual> &v2) {
        lds_add(dF + 3 * l, k1 * v1.x.d + k2 * v2.x.d);
        lds_add(dF + 3 * l + 1, k1 * v1.y.d + k2 * v2.y.d);
        lds_add(dF + 3 * l + 2, k1 * v1.z.d + k2 * v2.z.d);
    };

    int fi[FK][3];
    double fa0[FK];
    unsigned fmask = 0;
#pragma unroll
    for (int s = 0; s < FK; ++s) {
        const int t = tid + s * NT;
        fi[s][0] = fi[s][1] = fi[s][2] = 0;
        fa0[s] = 1.0;
        if (t < F) {
            fmask |= 1u << s;
            const int4 r = ((const int4 *)a.frec)[f0 + t];
            fi[s][0] = r.x & 0xFFFF;
            fi[s][1] = (int)((unsigned)r.x >> 16);
            fi[s][2] = r.y & 0xFFFF;
            fa0[s] = face_a0(r, 0.0);
        }
    }

    // ---- P0 ----
    for (int i = tid; i < 3 * NL; i += NT) dF[i] = 0.0;
    int kmin[3], kmax[3];
    load_positions<NT>(xs, a.X, whole, n0, gid, NL, N, a.inv_h, kmin, kmax);

    // ---- P1: V and dV, reduced together with the bounding box ----
    double sums[2] = {0.0, 0.0};
    if (whole) {
        const vec3<dual> anchor = dualx(0, tangent(0));
#pragma unroll
        for (int s = 0; s < FK; ++s) {
            if (fmask & (1u << s)) {
                // 6 V contribution of the face about the anchor (the area is
                // not needed here)
                const vec3<dual> xi = dualx(fi[s][0], tangent(fi[s][0])) - anchor,
                                 xj = dualx(fi[s][1], tangent(fi[s][1])) - anchor,
                                 xk = dualx(fi[s][2], tangent(fi[s][2])) - anchor;
                const dual v = dot(xi, cross(xj, xk));
                sums[0] += v.v;
                sums[1] += v.d;
            }
        }
    }
    block_box_sums<NT, 2>(kmin, kmax, sums, ired, red);
    double Vb, dVb;
    if (whole) {
        Vb = sums[0] * (1.0 / 6.0);
        dVb = sums[1] * (1.0 / 6.0);
    } else {
        Vb = a.Vpre[b];
        dVb = a.dVpre[b];
    }

    // ---- P2: elements (dual numbers, unit constants) ----
    double dot_s = 0.0, dot_b = 0.0, dot_a = 0.0, dot_v = 0.0;
    {
        const double kA = a.kA[b], kV = a.kV[b], ks = a.ks[b], kb = a.kb[b];
        const dual sV1 = volume_coefficient<dual>(a.closed[b] != 0, 1.0, dual(Vb, dVb), a.V0[b]);
#pragma unroll
        for (int s = 0; s < FK; ++s) {
            if (fmask & (1u << s)) {
                const int i = fi[s][0], j = fi[s][1], k = fi[s][2];
                const vec3<double> pi = tangent(i), pj = tangent(j), pk = tangent(k);
                vec3<dual> gi, gj, gk, gv;
                bad |= face_parts<dual, dual>(dualx(i, pi), dualx(j, pj), dualx(k, pk),
                                              dual(fa0[s]), 1.0, sV1, gi, gj, gk, gv);
                addd2(i, kA, gi, kV, gv);
                addd2(j, kA, gj, kV, gv);
                addd2(k, kA, gk, kV, gv);
                if (whole || i < N) {
                    dot_a += gi.x.v * pi.x + gi.y.v * pi.y + gi.z.v * pi.z + gj.x.v * pj.x +
                             gj.y.v * pj.y + gj.z.v * pj.z + gk.x.v * pk.x + gk.y.v * pk.y +
                             gk.z.v * pk.z;
                    dot_v += gv.x.v * (pi.x + pj.x + pk.x) + gv.y.v * (pi.y + pj.y + pk.y) +
                             gv.z.v * (pi.z + pj.z + pk.z);
                }
            }
        }
        using Raw = RawEdge<double>;
        for (int t = tid; t < E; t += NT) {
            const Raw r = Raw::load(a.erec, (int)e0 + t);
            const int4 q = r.ids();
            const bool hinge = q.z != kNoNode && q.w != kNoNode;
            const vec3<double> p1 = tangent(q.x), p2 = tangent(q.y);
            const vec3<double> p3 = hinge ? tangent(q.z) : vec3<double>{0.0, 0.0, 0.0};
            const vec3<double> p4 = hinge ? tangent(q.w) : vec3<double>{0.0, 0.0, 0.0};
            const vec3<dual> x1 = dualx(q.x, p1), x2 = dualx(q.y, p2);
            const vec3<dual> x3 = dualx(hinge ? q.z : 0, p3), x4 = dualx(hinge ? q.w : 0, p4);
            vec3<dual> fsp, h1, h2, h3, h4;
            bad |= edge_parts<dual, dual>(x1, x2, x3, x4, hinge, dual(r.l0()), dual(r.c0()),
                                          dual(r.s0()), 1.0, 1.0, fsp, h1, h2, h3, h4);
            double ws = 1.0, wb = 1.0;
            if constexpr (EW) {
                const double2 wt = reinterpret_cast<const double2 *>(a.ew)[e0 + t];
                ws = wt.x;
                wb = wt.y;
            }
            const double kse = ks * ws, kbe = kb * wb;
            if (hinge) {
                addd2(q.x, kse, fsp, kbe, h1);
                addd2(q.y, -kse, fsp, kbe, h2);
                addd(q.z, kbe, h3);
                addd(q.w, kbe, h4);
            } else {
                addd(q.x, kse, fsp);
                addd(q.y, -kse, fsp);
            }
            if (whole || q.x < N) {
                dot_s += ws * (fsp.x.v * (p1.x - p2.x) + fsp.y.v * (p1.y - p2.y) +
                               fsp.z.v * (p1.z - p2.z));
                if (hinge)
                    dot_b += wb * (h1.x.v * p1.x + h1.y.v * p1.y + h1.z.v * p1.z + h2.x.v * p2.x +
                                   h2.y.v * p2.y + h2.z.v * p2.z + h3.x.v * p3.x + h3.y.v * p3.y +
                                   h3.z.v * p3.z + h4.x.v * p4.x + h4.y.v * p4.y + h4.z.v * p4.z);
            }
        }
    }
    double dots[4] = {dot_s, dot_b, dot_a, dot_v};
    block_sums<NT, 4>(dots, red);      // its barriers also complete dF
    if (tid == 0 && a.gk) {
#pragma unroll
        for (int f = 0; f < 4; ++f) atomicAdd(a.gk + f * a.B + b, c2 * dots[f]);
    }

    // ---- P2b + P3: lam = lam' + dt^2/m dF written for the owned nodes, and
    // their dF replaced in place by P' = dt h^3 P (each thread its own nodes).
    // A whole unit may update lam' in place: no other unit reads its nodes,
    // and this unit reads no tangent after this point. ----
    double *dst = whole ? a.lam_out : a.lam_stage;
    const double sc = a.dt / a.inv_h3;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int j = tid + s * NT;
        if (j < N) {
            const int64_t g = gnode(j);
            const bool pin = a.pinned[g] != 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double l = a.lam_in[3 * g + c];
                dst[3 * g + c] = l + c2 * dF[3 * j + c];
                dF[3 * j + c] = pin ? 0.0 : sc * l;
            }
        }
    }
    __syncthreads();
    int pos[K];
    const CellSort cs = cell_sort<NT>(xs, dF, N, kmin, kmax, a.inv_h, tile_region, a.tile_bytes,
                                      occ_start, occ_cnt, ired, &n_occ_sh, cnt_bins, pos, a.nx,
                                      a.ny, a.nz, a.plane);
    const TileGeom &tg = cs.tg;

    // ---- P4: gu += spread(P'); the velocity tile of lattice 0 is fetched
    // into registers before the last flush ----
    constexpr int PF = NT >= 768 ? 5 : 8;
    TilePrefetch<NT, double, PF> pf;
    const bool pf_ok = cs.use_tile && TilePrefetch<NT, double, PF>::covers(tg);
    bool have0 = false;
    if (a.gu != nullptr)
        spread_to_grid<double, NT>(xs, dF, N, cs, occ_start, occ_cnt, ftile, a.gu, a.field,
                                   a.inv_h, a.inv_h3, bad, [&] {
                                       if (pf_ok) {
                                           pf.load(a.u, tg);
                                           have0 = true;
                                       }
                                   });

    // ---- P5: J_U^T P' per owned node, one lattice at a time; the velocity
    // tile of lattice d + 1 is loaded into registers while lattice d is used ----
    double gacc[K][3];
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) gacc[s][c] = 0.0;
    if (pf_ok && !have0) pf.load(a.u, tg);
    lds_barrier();
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double *ud = a.u + d * a.field;
        if (cs.use_tile) {
            if (pf_ok)
                pf.store(utile, tg);
            else
                stage_tile<NT>(utile, ud, tg);
            lds_barrier();
            if (pf_ok && d < 2) pf.load(ud + a.field, tg);
        }
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int j = tid + s * NT;
            if (j >= N) continue;
            const int p = pos[s];
            double w[3][3], dw[3][3];
            int cc[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
                cc[ax] = delta3_d(xs[3 * p + ax] * a.inv_h - mac_off(d, ax), w[ax], dw[ax]);
            double gx = 0.0, gy = 0.0, gz = 0.0;
            if (cs.use_tile) {
                const int lx = cc[0] - tg.kmin[0], ly = cc[1] - tg.kmin[1], lz = cc[2] - tg.kmin[2];
                if (lx < 0 || ly < 0 || lz < 0 || lx + 2 >= tg.Tx || ly + 2 >= tg.Ty ||
                    lz + 2 >= tg.Tz) {
                    bad = true;
                } else {
                    // separable: per (y, z) row the x-sums with w and dw,
                    // then the row's weights for each component
#pragma unroll
                    for (int z = 0; z < 3; ++z)
#pragma unroll
                        for (int y = 0; y < 3; ++y) {
                            const double *row = utile + ((lz + z) * tg.Ty + (ly + y)) * tg.Tx + lx;
                            const double rw = row[0] * w[0][0] + row[1] * w[0][1] + row[2] * w[0][2];
                            const double rd = row[0] * dw[0][0] + row[1] * dw[0][1] + row[2] * dw[0][2];
                            gx += rd * (w[1][y] * w[2][z]);
                            gy += rw * (dw[1][y] * w[2][z]);
                            gz += rw * (w[1][y] * dw[2][z]);
                        }
                }
            } else {
                const int ix[3] = {wrapi(cc[0] - 1, a.nx), wrapi(cc[0], a.nx), wrapi(cc[0] + 1, a.nx)};
#pragma unroll
                for (int z = 0; z < 3; ++z)
#pragma unroll
                    for (int y = 0; y < 3; ++y) {
                        const double *row = ud + wrapi(cc[2] - 1 + z, a.nz) * a.plane +
                                            (int64_t)wrapi(cc[1] - 1 + y, a.ny) * a.nx;
                        const double u0 = row[ix[0]], u1 = row[ix[1]], u2 = row[ix[2]];
                        const double rw = u0 * w[0][0] + u1 * w[0][1] + u2 * w[0][2];
                        const double rd = u0 * dw[0][0] + u1 * dw[0][1] + u2 * dw[0][2];
                        gx += rd * (w[1][y] * w[2][z]);
                        gy += rw * (dw[1][y] * w[2][z]);
                        gz += rw * (w[1][y] * dw[2][z]);
                    }
            }
            const double pd = dF[3 * p + d] * a.inv_h;    // P'_d d/dX = P'_d (1/h) d/ds
            gacc[s][0] += pd * gx;
            gacc[s][1] += pd * gy;
            gacc[s][2] += pd * gz;
        }
        if (cs.use_tile) lds_barrier();
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int j = tid + s * NT;
        if (j < N) {
            const int64_t g = gnode(j);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double v = dst[3 * g + c] + gacc[s][c] * a.inv_h3;
                if (!isfinite(v)) atomicOr(a.status, IP_STATUS_NONFINITE);
                dst[3 * g + c] = v;
            }
        }
    }
    if (bad) atomicOr(a.status, IP_STATUS_DEGENERATE);
}

// Volume and its tangent along P = M lam' of the listed bodies.
__global__ __launch_bounds__(256) void k_volume_dual_masked(
    const double *__restrict__ X, const double *__restrict__ lam, const uint8_t *__restrict__ pinned,
    const int32_t *__restrict__ faces, const int64_t *__restrict__ node_off,
    const int64_t *__restrict__ face_off, const int32_t *__restrict__ bodies,
    double *__restrict__ V, double *__restrict__ dV) {
    __shared__ double sh[4];
    const int b = bodies[blockIdx.x];
    if (face_off[b] == face_off[b + 1]) {
        if (threadIdx.x == 0) V[b] = dV[b] = 0.0;
        return;
    }
    const auto xd = [&](int64_t i) -> vec3<dual> {
        const bool pin = pinned[i] != 0;
        return {dual(X[3 * i], pin ? 0.0 : lam[3 * i]), dual(X[3 * i + 1], pin ? 0.0 : lam[3 * i + 1]),
                dual(X[3 * i + 2], pin ? 0.0 : lam[3 * i + 2])};
    };
    const vec3<dual> anchor = xd(node_off[b]);
    double v = 0.0, dv = 0.0;
    for (int64_t f = face_off[b] + threadIdx.x; f < face_off[b + 1]; f += blockDim.x) {
        const int32_t *t = faces + 3 * f;
        dual v6;
        double a2;
        face_geometry<dual, double>(xd(t[0]), xd(t[1]), xd(t[2]), anchor, v6, a2);
        v += v6.v;
        dv += v6.d;
    }
    v = block_sum(v, sh);
    dv = block_sum(dv, sh);
    if (threadIdx.x == 0) {
        V[b] = v / 6.0;
        dV[b] = dv / 6.0;
    }
}

}  // namespace

ip_status launch_forces_jvp(ip_plan *p, const double *X, const double *T, const ip_reference *ref,
                            const ip_constants *k, const double *P, double *dF, double *dotE,
                            double *dotF, hipStream_t s) {
    double *slots = (double *)p->slots;
    double *V = p->Vbuf, *dV = p->Abuf;
    if (p->B > 0)
        hipLaunchKernelGGL(k_volume_dual, dim3(p->B), dim3(256), 0, s, X, T, p->faces, p->node_off,
                           p->face_off, V, dV);
    if (p->E > 0)
        hipLaunchKernelGGL(k_edges_jvp, dim3(nblocks(p->E, 256)), dim3(256), 0, s, X, T,
                           (const int4 *)p->edges4, p->edge_off, p->B, p->E,
                           (const double *)ref->l0, (const double *)ref->cs0, k->ks, k->kb, p->ew,
                           P, slots, dotE);
    if (p->F > 0)
        hipLaunchKernelGGL(k_faces_jvp, dim3(nblocks(p->F, 256)), dim3(256), 0, s, X, T, p->faces,
                           p->face_off, p->B, p->F, (const double *)ref->A0, ref->V0, V, dV,
                           p->closed, k->kA, k->kV, P, slots + 12 * p->E, dotF);
    if (p->N > 0)
        hipLaunchKernelGGL(k_gather_f64, dim3(nblocks(p->N, 256)), dim3(256), 0, s, p->csr_ptr,
                           p->csr_slot, slots, p->N, dF);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

ip_status launch_step_vjp(ip_plan *p, const double *X, const ip_reference *ref,
                          const ip_constants *k, const double *u, double dt,
                          const double *lam_in, double *lam_out, double *gk, double *gu,
                          hipStream_t s) {
    double *P = (double *)p->Ubuf;        // [N][3] workspace (FP64 plans)
    double *dF = (double *)p->Fbuf;       // [N][3]
    if (p->N > 0)
        hipLaunchKernelGGL(k_mask, dim3(nblocks(3 * p->N, 256)), dim3(256), 0, s, lam_in,
                           p->pinned, p->N, P);
    double *dotE = p->bwd_dots, *dotF = p->bwd_dots + 2 * p->E;
    ip_status st = launch_forces_jvp(p, X, P, ref, k, P, dF, dotE, dotF, s);
    if (st != IP_OK) return st;
    if (gk && p->B > 0)
        hipLaunchKernelGGL(k_gk, dim3(p->B), dim3(256), 0, s, dotE, dotF, p->edge_off, p->face_off,
                           k->mass, dt, p->B, gk);
    if (p->N > 0)
        hipLaunchKernelGGL(k_lambda, dim3(nblocks(p->N, 256)), dim3(256), 0, s, X, u, lam_in, P,
                           dF, p->node_off, p->B, k->mass, p->N, p->grid.nx, p->grid.ny,
                           p->grid.nz, 1.0 / p->grid.h, dt, lam_out);
    IP_HIP_CHECK(hipGetLastError());
    if (gu && p->N > 0) {
        // dL/du = dt sum_l P_l w_l = spread(dt h^3 P) (spreading divides by h^3)
        const double h = p->grid.h;
        hipLaunchKernelGGL(k_scale, dim3(nblocks(3 * p->N, 256)), dim3(256), 0, s, P,
                           dt * h * h * h, 3 * p->N, dF);
        IP_HIP_CHECK(hipGetLastError());
        return launch_spread(p, X, dF, gu, s);
    }
    return IP_OK;
}

ip_status launch_interp_vjp(ip_plan *p, const double *X, const double *u, const double *dU,
                            double *gX, double *gu, hipStream_t s) {
    if (p->N == 0) return IP_OK;
    if (gX) {
        hipLaunchKernelGGL(k_interp_vjp_x, dim3(nblocks(p->N, 256)), dim3(256), 0, s, X, u, dU,
                           p->N, p->grid.nx, p->grid.ny, p->grid.nz, 1.0 / p->grid.h, gX);
        IP_HIP_CHECK(hipGetLastError());
    }
    if (gu) {
        // gu_d[k] += sum_l dU_l,d w_k(X_l) = spread(h^3 dU) (spreading divides by h^3)
        const double h = p->grid.h;
        double *tmp = (double *)p->Fbuf;
        hipLaunchKernelGGL(k_scale, dim3(nblocks(3 * p->N, 256)), dim3(256), 0, s, dU, h * h * h,
                           3 * p->N, tmp);
        IP_HIP_CHECK(hipGetLastError());
        return launch_spread(p, X, tmp, gu, s);
    }
    return IP_OK;
}

ip_status launch_taylor(ip_plan *p, const double *X, const double *Dstar, double *D, double *loss,
                        double *gX, hipStream_t s) {
    if (p->B == 0) return IP_OK;
    hipLaunchKernelGGL(k_taylor, dim3(p->B), dim3(256), 0, s, X, p->node_off, Dstar, D, loss, gX);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

ip_status prepare_step_vjp_fused(ip_plan *p) {
    for (int c = 0; c < p->n_step_classes; ++c) {
        const auto &sc = p->step_class[c];
        const int lds = (int)step_fused_lds_bytes(sc.nmax, sc.tile_bytes);
        const void *fns[2] = {
            sc.threads == 128   ? (const void *)k_step_vjp_fused<128, false>
            : sc.threads == 256 ? (const void *)k_step_vjp_fused<256, false>
            : sc.threads == 384 ? (const void *)k_step_vjp_fused<384, false>
                                : (const void *)k_step_vjp_fused<768, false>,
            sc.threads == 128   ? (const void *)k_step_vjp_fused<128, true>
            : sc.threads == 256 ? (const void *)k_step_vjp_fused<256, true>
            : sc.threads == 384 ? (const void *)k_step_vjp_fused<384, true>
                                : (const void *)k_step_vjp_fused<768, true>};
        for (const void *fn : fns)
            IP_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    }
    return IP_OK;
}

ip_status launch_step_vjp_fused(ip_plan *p, const double *X, const ip_reference *ref,
                                const ip_constants *k, const double *u, double dt,
                                const double *lam_in, double *lam_out, double *gk, double *gu,
                                hipStream_t s) {
    if (p->B == 0) return IP_OK;
    VjpArgs a{};
    a.X = X;
    a.lam_in = lam_in;
    a.lam_out = lam_out;
    a.lam_stage = p->Xstage;
    a.node_off = p->node_off;
    a.closed = p->closed;
    a.pinned = p->pinned;
    a.V0 = ref->V0;
    a.ks = k->ks;
    a.kb = k->kb;
    a.kA = k->kA;
    a.kV = k->kV;
    a.mass = k->mass;
    a.u = u;
    a.gu = gu;
    a.gk = gk;
    a.B = p->B;
    a.nx = p->grid.nx;
    a.ny = p->grid.ny;
    a.nz = p->grid.nz;
    a.inv_h = 1.0 / p->grid.h;
    a.inv_h3 = 1.0 / (p->grid.h * p->grid.h * p->grid.h);
    a.plane = (int64_t)a.nx * a.ny;
    a.field = a.plane * a.nz;
    a.dt = dt;
    a.Vpre = p->Vbuf;
    a.dVpre = p->Abuf;
    a.status = p->status;
    a.wu_body = p->wu_body;
    a.wu_owned = p->wu_owned;
    a.wu_pinned = p->wu_pinned;
    a.wu_nodes = p->wu_nodes;
    a.wu_noff = p->wu_noff;
    a.wu_eoff = p->wu_eoff;
    a.wu_foff = p->wu_foff;
    a.erec = p->edge_rec;
    a.frec = p->face_rec;
    a.ew = p->ew_rec;
    if (p->n_patched_bodies > 0) {
        hipLaunchKernelGGL(k_volume_dual_masked, dim3(p->n_patched_bodies), dim3(256), 0, s, X,
                           lam_in, p->pinned, p->faces, p->node_off, p->face_off,
                           p->patched_bodies, p->Vbuf, p->Abuf);
        IP_HIP_CHECK(hipGetLastError());
    }
    for (int c = 0; c < p->n_step_classes; ++c) {
        const auto &sc = p->step_class[c];
        a.unit_base = sc.unit_begin;
        a.nmax = sc.nmax;
        a.tile_bytes = sc.tile_bytes;
        const size_t lds = step_fused_lds_bytes(sc.nmax, sc.tile_bytes);
        const dim3 grid(sc.unit_end - sc.unit_begin), block(sc.threads);
        if (sc.threads == 128) {
            if (a.ew)
                hipLaunchKernelGGL((k_step_vjp_fused<128, true>), grid, block, lds, s, a);
            else
                hipLaunchKernelGGL((k_step_vjp_fused<128, false>), grid, block, lds, s, a);
        } else if (sc.threads == 256) {
            if (a.ew)
                hipLaunchKernelGGL((k_step_vjp_fused<256, true>), grid, block, lds, s, a);
            else
                hipLaunchKernelGGL((k_step_vjp_fused<256, false>), grid, block, lds, s, a);
        } else if (sc.threads == 384) {
            if (a.ew)
                hipLaunchKernelGGL((k_step_vjp_fused<384, true>), grid, block, lds, s, a);
            else
                hipLaunchKernelGGL((k_step_vjp_fused<384, false>), grid, block, lds, s, a);
        } else {
            if (a.ew)
                hipLaunchKernelGGL((k_step_vjp_fused<768, true>), grid, block, lds, s, a);
            else
                hipLaunchKernelGGL((k_step_vjp_fused<768, false>), grid, block, lds, s, a);
        }
        IP_HIP_CHECK(hipGetLastError());
    }
    return launch_commit(p, p->Xstage, lam_out, s);
}
