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
#include "elements.h"
#include "ipibm_internal.h"

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
    const double *__restrict__ P, double *__restrict__ slots, double *__restrict__ dotE) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int b = body_of(edge_off, B, e);
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
                           dual(cs0[2 * e]), dual(cs0[2 * e + 1]), ks[b], kb[b], fsp, h1, h2, h3,
                           h4);
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
        dotE[2 * e] = dot(u0, p1 - p2);
        dotE[2 * e + 1] = bend;
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
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
__global__ __launch_bounds__(256) void k_lambda(const double *__restrict__ X,
                                                const double *__restrict__ u,
                                                const double *__restrict__ lam_in,
                                                const double *__restrict__ P,
                                                const double *__restrict__ dF,
                                                const int64_t *__restrict__ node_off, int B,
                                                const double *__restrict__ mass, int64_t N, int nx,
                                                int ny, int nz, double inv_h, double dt,
                                                double *__restrict__ lam_out) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= N) return;
    const int b = body_of(node_off, B, l);
    const double c = dt * dt / mass[b];
    const vec3<double> x = ldX(X, l), p = ldX(P, l);
    const double pd[3] = {p.x, p.y, p.z};
    const double xv[3] = {x.x, x.y, x.z};
    const int64_t plane = (int64_t)nx * ny, field = plane * nz;
    double g[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
        double w[3][3], dw[3][3];
        int cc[3];
        for (int ax = 0; ax < 3; ++ax)
            cc[ax] = delta3_d(xv[ax] * inv_h - mac_off(d, ax), w[ax], dw[ax]);
        const double *ud = u + d * field;
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int kz = 0; kz < 3; ++kz)
            for (int ky = 0; ky < 3; ++ky) {
                const double *row = ud + wrapi(cc[2] - 1 + kz, nz) * plane +
                                    (int64_t)wrapi(cc[1] - 1 + ky, ny) * nx;
                for (int kx = 0; kx < 3; ++kx) {
                    const double uv = row[wrapi(cc[0] - 1 + kx, nx)];
                    gx += uv * dw[0][kx] * w[1][ky] * w[2][kz];
                    gy += uv * w[0][kx] * dw[1][ky] * w[2][kz];
                    gz += uv * w[0][kx] * w[1][ky] * dw[2][kz];
                }
            }
        g[0] += pd[d] * gx * inv_h;
        g[1] += pd[d] * gy * inv_h;
        g[2] += pd[d] * gz * inv_h;
    }
    for (int e = 0; e < 3; ++e)
        lam_out[3 * l + e] = lam_in[3 * l + e] + dt * g[e] + c * dF[3 * l + e];
}

// F := s P (spreading source for the u-gradient)
__global__ void k_scale(const double *__restrict__ P, double s, int64_t n, double *__restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = s * P[i];
}

// ---------------------------------------------------------------------------
// Taylor deformation: C = (1/n) sum (x - c)(x - c)^T over the body's nodes;
// eigenvalues of the symmetric 3x3 C in closed form (trigonometric solution
// of the characteristic cubic), L = sqrt(lambda_max), B = sqrt(lambda_min),
// D = (L - B)/(L + B).  Eigenvectors from cross products of rows of C - lambda I.
// ---------------------------------------------------------------------------
struct Sym3 {
    double xx, yy, zz, xy, xz, yz;
};

__device__ void sym3_eigs(const Sym3 &A, double lam[3]) {
    const double p1 = A.xy * A.xy + A.xz * A.xz + A.yz * A.yz;
    const double q = (A.xx + A.yy + A.zz) / 3.0;
    const double dx = A.xx - q, dy = A.yy - q, dz = A.zz - q;
    const double p2 = dx * dx + dy * dy + dz * dz + 2.0 * p1;
    const double p = sqrt(p2 / 6.0);
    if (p == 0.0) {
        lam[0] = lam[1] = lam[2] = q;
        return;
    }
    const double ip = 1.0 / p;
    const double bxx = dx * ip, byy = dy * ip, bzz = dz * ip, bxy = A.xy * ip, bxz = A.xz * ip,
                 byz = A.yz * ip;
    const double detB = bxx * (byy * bzz - byz * byz) - bxy * (bxy * bzz - byz * bxz) +
                        bxz * (bxy * byz - byy * bxz);
    double r = detB / 2.0;
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    const double phi = acos(r) / 3.0;
    lam[0] = q + 2.0 * p * cos(phi);                              // largest
    lam[2] = q + 2.0 * p * cos(phi + 2.0 * 3.14159265358979323846 / 3.0);   // smallest
    lam[1] = 3.0 * q - lam[0] - lam[2];
}

__device__ vec3<double> sym3_eigvec(const Sym3 &A, double l) {
    const vec3<double> r0 = {A.xx - l, A.xy, A.xz}, r1 = {A.xy, A.yy - l, A.yz},
                       r2 = {A.xz, A.yz, A.zz - l};
    vec3<double> c0 = cross(r0, r1), c1 = cross(r0, r2), c2 = cross(r1, r2);
    const double n0 = dot(c0, c0), n1 = dot(c1, c1), n2 = dot(c2, c2);
    vec3<double> v = n0 >= n1 && n0 >= n2 ? c0 : (n1 >= n2 ? c1 : c2);
    const double n = sqrt(dot(v, v));
    return (1.0 / n) * v;
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
        double lam[3];
        sym3_eigs(C, lam);
        const double L = sqrt(lam[0]), Bs = sqrt(lam[2]);
        const double Db = (L - Bs) / (L + Bs);
        if (D) D[b] = Db;
        if (Dstar) {
            const double r = Db - Dstar[b];
            loss[b] = r * r;
            const double dDdL = 2.0 * Bs / ((L + Bs) * (L + Bs));
            const double dDdB = -2.0 * L / ((L + Bs) * (L + Bs));
            const vec3<double> vmax = sym3_eigvec(C, lam[0]), vmin = sym3_eigvec(C, lam[2]);
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
                           (const double *)ref->l0, (const double *)ref->cs0, k->ks, k->kb, P,
                           slots, dotE);
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

ip_status launch_taylor(ip_plan *p, const double *X, const double *Dstar, double *D, double *loss,
                        double *gX, hipStream_t s) {
    if (p->B == 0) return IP_OK;
    hipLaunchKernelGGL(k_taylor, dim3(p->B), dim3(256), 0, s, X, p->node_off, Dstar, D, loss, gX);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}
