// elements.h -- per-element interaction-potential forces (Section 2.3 of
// Spandan et al.), shared by the element kernels, the fused step and the
// forward-mode (dual-number) derivative kernels.
//
// Two scalar types: P carries positions, the hinge angle and the volume (FP64,
// or a dual number for directional derivatives); R carries the force vectors
// (FP64 or FP32, or the dual type).
#pragma once

#include "ipibm_internal.h"

// Dual number a + b eps (eps^2 = 0): forward-mode derivative along a tangent.
struct dual {
    double v, d;
    __host__ __device__ dual() : v(0.0), d(0.0) {}
    __host__ __device__ dual(double a) : v(a), d(0.0) {}
    __host__ __device__ dual(double a, double b) : v(a), d(b) {}
    __host__ __device__ explicit operator double() const { return v; }   // drops the tangent
};
__device__ __forceinline__ dual operator+(dual a, dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ dual operator-(dual a, dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ dual operator-(dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ dual operator*(dual a, dual b) {
    return {a.v * b.v, fma(a.v, b.d, a.d * b.v)};
}
__device__ __forceinline__ dual &operator+=(dual &a, dual b) { return a = a + b; }
__device__ __forceinline__ bool operator>(dual a, dual b) { return a.v > b.v; }
__device__ __forceinline__ dual rcp_nr(dual x) {
    const double r = rcp_nr(x.v);
    return {r, -r * r * x.d};
}
__device__ __forceinline__ dual rsq_nr(dual x) {
    const double q = rsq_nr(x.v);
    return {q, -0.5 * q * q * q * x.d};
}
__device__ __forceinline__ double value_of(double x) { return x; }
__device__ __forceinline__ double value_of(float x) { return x; }
__device__ __forceinline__ double value_of(dual x) { return x.v; }

template <typename T, typename S>
__device__ __forceinline__ vec3<T> to(const vec3<S> &a) {
    return {(T)a.x, (T)a.y, (T)a.z};
}

// Edge element (see edge_forces for the combination into node forces).
//
// Spring W_e = 1/2 ks (l - l0)^2: fsp is the force on v1 (v2 receives -fsp).
// Bending hinge W_b = kb (1 - cos(theta - theta0)) on (v1, v2 | v3, v4),
// e = x2 - x1, nA = e x (x3 - x1), nB = (x4 - x1) x e, with
// |nA||nB| cos(theta) = nA.nB and |nA||nB| sin(theta) = (nA x nB).e / |e| (a
// convex fold has theta > 0); dW/dtheta = kb sin(theta - theta0)
// = kb (sin c0 - cos s0) with (c0, s0) = (cos theta0, sin theta0).
// Gradient of theta: the wings move along their face normals,
//   dtheta/dx3 = -|e| nA/|nA|^2,  dtheta/dx4 = -|e| nB/|nB|^2,
// and the edge nodes take the unique combination that keeps theta invariant
// under translation and rotation: with s3 = (x3-x1).e/|e|^2, s4 likewise,
//   dtheta/dx1 = -(1-s3) dtheta/dx3 - (1-s4) dtheta/dx4,
//   dtheta/dx2 = -s3 dtheta/dx3 - s4 dtheta/dx4.
// h1..h4 are the hinge forces on v1..v4.  The angle (normals, cos, sin,
// dW/dtheta) is evaluated in P: with FP32 edge vectors sin(theta) would carry
// ~1e-7 absolute error while theta - theta0 is ~1e-3 on fine smooth meshes.
// x3 and x4 are read only when `hinge` (an edge on the open boundary of a
// membrane has no hinge).  Returns true if the element is degenerate (zero
// length or zero-area wing).
template <typename P, typename R>
__device__ __forceinline__ bool edge_parts(const vec3<P> &x1, const vec3<P> &x2,
                                           const vec3<P> &x3, const vec3<P> &x4, bool hinge, R l0,
                                           R c0, R s0, double ks, double kb, vec3<R> &fsp,
                                           vec3<R> &h1, vec3<R> &h2, vec3<R> &h3, vec3<R> &h4) {
    const vec3<R> ev = to<R>(x2 - x1);
    const R le2 = dot(ev, ev);
    const R inv_le = rsq_nr(le2);
    const R le = le2 * inv_le;
    fsp = ((R)ks * (le - l0) * inv_le) * ev;
    h1 = h2 = h3 = h4 = vec3<R>{(R)0, (R)0, (R)0};
    bool bad = !(le2 > (R)0);
    if (hinge) {
        const vec3<P> evd = x2 - x1, d3d = x3 - x1, d4d = x4 - x1;
        const vec3<P> nA = cross(evd, d3d);
        const vec3<P> nB = cross(d4d, evd);
        const P nA2 = dot(nA, nA), nB2 = dot(nB, nB);
        bad |= !(nA2 > (P)0.0) || !(nB2 > (P)0.0);
        const P le2d = dot(evd, evd);
        const P inv_led = rsq_nr(le2d);
        const P led = le2d * inv_led;
        const P inv = rsq_nr(nA2 * nB2);            // 1 / (|nA| |nB|)
        const P cth = dot(nA, nB) * inv;
        const P sth = dot(cross(nA, nB), evd) * inv * inv_led;
        const P dW = (P)kb * (sth * (P)c0 - cth * (P)s0);
        // F3 = -dW dtheta/dx3 = dW |e| nA/|nA|^2, F4 likewise;
        // 1/|nA|^2 = |nB|^2 / (|nA|^2 |nB|^2) = |nB|^2 inv^2
        const P g = dW * led * inv * inv;
        const R a3 = (R)(g * nB2), a4 = (R)(g * nA2);
        h3 = a3 * to<R>(nA);
        h4 = a4 * to<R>(nB);
        const vec3<R> d3 = to<R>(d3d), d4 = to<R>(d4d);
        const R inv_le2 = inv_le * inv_le;
        const R s3 = dot(d3, ev) * inv_le2, s4 = dot(d4, ev) * inv_le2;
        h1 = (R)-1 * (((R)1 - s3) * h3 + ((R)1 - s4) * h4);
        h2 = (R)-1 * (s3 * h3 + s4 * h4);
    }
    return bad;
}

// Node forces of an edge element: f1 = fsp + h1, f2 = -fsp + h2, f3 = h3, f4 = h4.
template <typename P, typename R>
__device__ __forceinline__ bool edge_forces(const vec3<P> &x1, const vec3<P> &x2,
                                            const vec3<P> &x3, const vec3<P> &x4, bool hinge, R l0,
                                            R c0, R s0, double ks, double kb, vec3<R> &f1,
                                            vec3<R> &f2, vec3<R> &f3, vec3<R> &f4) {
    vec3<R> fsp, h1, h2;
    const bool bad =
        edge_parts<P, R>(x1, x2, x3, x4, hinge, l0, c0, s0, ks, kb, fsp, h1, h2, f3, f4);
    f1 = fsp + h1;
    f2 = h2 - fsp;
    return bad;
}

// Face element: area W_a = 1/2 kA (A - A0)^2 / A0 with dA/dx_i = 1/2 nhat x
// (x_k - x_j) (cyclic) -> area forces gi, gj, gk; and, on closed bodies, the
// volume potential through sV = -dW_v/dV / 6 = -kV (V - V0) / (6 V0).
// Differentiating the divergence-theorem volume gives
// dV/dx_i = (1/6) sum_{f ni i} (x_j - a) x (x_k - a) for any anchor a; around
// the closed fan of node i the anchor terms cancel and taking a = x_i leaves
// (1/6) sum_{f ni i} n_f, so every face hands gv = sV n_f to each of its
// corners (no anchor cancellation: the anchored terms are ~|x - a| |edge|
// while their sum is ~|edge|^2).  Returns true if the face is degenerate.
// nn_out (optional) receives |n| = twice the face's area.
template <typename P, typename R>
__device__ __forceinline__ bool face_parts(const vec3<P> &xi, const vec3<P> &xj,
                                           const vec3<P> &xk, R a0, double kA, R sV,
                                           vec3<R> &gi, vec3<R> &gj, vec3<R> &gk, vec3<R> &gv,
                                           R *nn_out = nullptr) {
    const vec3<R> n = cross(to<R>(xj - xi), to<R>(xk - xi));
    const R nn2 = dot(n, n);
    const R inv_nn = rsq_nr(nn2);
    const R nn = nn2 * inv_nn;
    if (nn_out) *nn_out = nn;
    const R cA = (R)kA * ((R)0.5 * nn - a0) * rcp_nr(a0);    // dW_a/dA
    // -cA * 1/2 nhat x edge = (-cA / (2|n|)) n x edge
    const R sA = (R)-0.5 * cA * inv_nn;
    gv = sV * n;
    gi = sA * cross(n, to<R>(xk - xj));
    gj = sA * cross(n, to<R>(xi - xk));
    gk = sA * cross(n, to<R>(xj - xi));
    return !(nn2 > (R)0);
}

template <typename P, typename R>
__device__ __forceinline__ bool face_forces(const vec3<P> &xi, const vec3<P> &xj,
                                            const vec3<P> &xk, R a0, double kA, R sV,
                                            vec3<R> &gi, vec3<R> &gj, vec3<R> &gk,
                                            R *nn_out = nullptr) {
    vec3<R> gv;
    const bool bad = face_parts<P, R>(xi, xj, xk, a0, kA, sV, gi, gj, gk, gv, nn_out);
    gi = gi + gv;
    gj = gj + gv;
    gk = gk + gv;
    return bad;
}

// Contribution of one face to the body's enclosed volume (times 6) and area
// (times 2): (x_i - a).((x_j - a) x (x_k - a)) in P, |n| in R.
template <typename P, typename R>
__device__ __forceinline__ void face_geometry(const vec3<P> &xi, const vec3<P> &xj,
                                              const vec3<P> &xk, const vec3<P> &a, P &vol6,
                                              double &area2) {
    vol6 = dot(xi - a, cross(xj - a, xk - a));
    const vec3<R> n = cross(to<R>(xj - xi), to<R>(xk - xi));
    area2 = (double)sqrt(value_of(dot(n, n)));
}

// -dW_v/dV / 6 for a body (0 for open bodies); V may carry a tangent.
template <typename R, typename P>
__device__ __forceinline__ R volume_coefficient(bool closed, double kV, P V, double V0) {
    if (!closed) return (R)0;
    return (R)((P)(-kV / (6.0 * V0)) * (V - (P)V0));
}
