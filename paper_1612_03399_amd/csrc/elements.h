// elements.h -- per-element interaction-potential forces (Section 2.3 of
// Spandan et al.), shared by the unfused element kernels and the fused step.
#pragma once

#include "ipibm_internal.h"

// Edge element: spring W_e = 1/2 ks (l - l0)^2 on every edge and, when both
// wings exist, the bending hinge W_b = kb (1 - cos(theta - theta0)).
//
// Hinge (v1, v2 | v3, v4), e = x2 - x1, nA = e x (x3 - x1), nB = (x4 - x1) x e,
// |nA||nB| cos(theta) = nA.nB, |nA||nB| sin(theta) = (nA x nB).e / |e|, so a
// convex fold has theta > 0.  dW/dtheta = kb sin(theta - theta0)
// = kb (sin c0 - cos s0) with (c0, s0) = (cos theta0, sin theta0).
// Gradient of theta: the wings move along their face normals,
//   dtheta/dx3 = -|e| nA/|nA|^2,  dtheta/dx4 = -|e| nB/|nB|^2,
// and the edge nodes take the unique combination that keeps theta invariant
// under translation and rotation: with s3 = (x3-x1).e/|e|^2, s4 likewise,
//   dtheta/dx1 = -(1-s3) dtheta/dx3 - (1-s4) dtheta/dx4,
//   dtheta/dx2 = -s3 dtheta/dx3 - s4 dtheta/dx4.
// The angle (normals, cos, sin, dW/dtheta) is evaluated in FP64 for every R:
// on fine smooth meshes theta - theta0 is ~1e-3 while FP32 edge vectors leave
// ~1e-7 absolute error in sin(theta).  Force vectors are then formed in R.
// Returns true if the element is degenerate (zero length or zero-area wing).
template <typename R>
__device__ __forceinline__ bool edge_forces(const vec3<double> &x1, const vec3<double> &x2,
                                            const vec3<double> *x3, const vec3<double> *x4,
                                            R l0, R c0, R s0, double ks, double kb,
                                            vec3<R> &f1, vec3<R> &f2, vec3<R> &f3,
                                            vec3<R> &f4) {
    const vec3<R> ev = diffR<R>(x2, x1);
    const R le2 = dot(ev, ev);
    const R inv_le = rsq_nr(le2);
    const R le = le2 * inv_le;
    const R fs = (R)ks * (le - l0) * inv_le;
    f1 = fs * ev;
    f2 = (R)-1 * f1;
    f3 = {0, 0, 0};
    f4 = {0, 0, 0};
    bool bad = !(le2 > (R)0);
    if (x3 && x4) {
        const vec3<double> evd = x2 - x1, d3d = *x3 - x1, d4d = *x4 - x1;
        const vec3<double> nA = cross(evd, d3d);
        const vec3<double> nB = cross(d4d, evd);
        const double nA2 = dot(nA, nA), nB2 = dot(nB, nB);
        bad |= !(nA2 > 0.0) || !(nB2 > 0.0);
        const double le2d = dot(evd, evd);
        const double inv_led = rsq_nr(le2d);
        const double led = le2d * inv_led;
        const double inv = rsq_nr(nA2 * nB2);           // 1 / (|nA| |nB|)
        const double cth = dot(nA, nB) * inv;
        const double sth = dot(cross(nA, nB), evd) * inv * inv_led;
        const double dW = kb * (sth * (double)c0 - cth * (double)s0);
        // F3 = -dW dtheta/dx3 = dW |e| nA/|nA|^2, F4 likewise;
        // 1/|nA|^2 = |nB|^2 / (|nA|^2 |nB|^2) = |nB|^2 inv^2
        const double g = dW * led * inv * inv;
        const R a3 = (R)(g * nB2), a4 = (R)(g * nA2);
        f3 = a3 * vec3<R>{(R)nA.x, (R)nA.y, (R)nA.z};
        f4 = a4 * vec3<R>{(R)nB.x, (R)nB.y, (R)nB.z};
        const vec3<R> d3 = diffR<R>(*x3, x1), d4 = diffR<R>(*x4, x1);
        const R inv_le2 = inv_le * inv_le;
        const R s3 = dot(d3, ev) * inv_le2, s4 = dot(d4, ev) * inv_le2;
        f1 = f1 - ((R)1 - s3) * f3 - ((R)1 - s4) * f4;
        f2 = f2 - s3 * f3 - s4 * f4;
    }
    return bad;
}

// Face element: area W_a = 1/2 kA (A - A0)^2 / A0 with dA/dx_i = 1/2 nhat x
// (x_k - x_j) (cyclic), plus, on closed bodies, the volume potential through
// sV = -dW_v/dV / 6 = -kV (V - V0) / (6 V0).  Differentiating the
// divergence-theorem volume gives dV/dx_i = (1/6) sum_{f ni i} (x_j - a) x (x_k - a)
// for any anchor a; around the closed fan of node i the anchor terms cancel
// and taking a = x_i leaves (1/6) sum_{f ni i} n_f, so every face hands
// sV n_f to each of its corners (no anchor cancellation: the anchored terms
// are ~|x - a| |edge| while their sum is ~|edge|^2).
// Returns true if the face is degenerate.
template <typename R>
__device__ __forceinline__ bool face_forces(const vec3<double> &xi, const vec3<double> &xj,
                                            const vec3<double> &xk, R a0, double kA, R sV,
                                            vec3<R> &gi, vec3<R> &gj, vec3<R> &gk) {
    const vec3<R> n = cross(diffR<R>(xj, xi), diffR<R>(xk, xi));
    const R nn2 = dot(n, n);
    const R inv_nn = rsq_nr(nn2);
    const R nn = nn2 * inv_nn;
    const R cA = (R)kA * ((R)0.5 * nn - a0) * rcp_nr(a0);    // dW_a/dA
    // -cA * 1/2 nhat x edge = (-cA / (2|n|)) n x edge
    const R sA = (R)-0.5 * cA * inv_nn;
    const vec3<R> gv = sV * n;
    gi = sA * cross(n, diffR<R>(xk, xj)) + gv;
    gj = sA * cross(n, diffR<R>(xi, xk)) + gv;
    gk = sA * cross(n, diffR<R>(xj, xi)) + gv;
    return !(nn2 > (R)0);
}

// Contribution of one face to the body's enclosed volume (times 6) and area
// (times 2): (x_i - a).((x_j - a) x (x_k - a)) in FP64, |n| in R.
template <typename R>
__device__ __forceinline__ void face_geometry(const vec3<double> &xi, const vec3<double> &xj,
                                              const vec3<double> &xk, const vec3<double> &a,
                                              double &vol6, double &area2) {
    vol6 = dot(xi - a, cross(xj - a, xk - a));
    const vec3<R> n = cross(diffR<R>(xj, xi), diffR<R>(xk, xi));
    area2 = (double)sqrt(dot(n, n));
}

// -dW_v/dV / 6 for body b (0 for open bodies).
template <typename R>
__device__ __forceinline__ R volume_coefficient(bool closed, double kV, double V, double V0) {
    return closed ? (R)(-kV * (V - V0) / V0 * (1.0 / 6.0)) : (R)0;
}
