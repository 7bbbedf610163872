// k_mls.hip -- moving-least-squares (MLS) transfer between the triangle
// centroids (the Lagrangian markers) and the staggered lattices (Section 2.2
// of Spandan et al.: the MLS equations with a linear basis, the exponential
// weight on a 3x3x3 support of threshold 1.5 h, and the force-conserving
// spreading factor c_l), and the transfer of centroid forces to the triangle
// vertices (one third per vertex, Section 2.3).
//
// The weight is a product over axes, W_k = wx_i wy_j wz_k with w(r) =
// exp(-(r/alpha)^2), r = |x_a - x^k_a| / 1.5 h, and the shape functions do not
// change when the weights of one axis are scaled (A and A^{-1} B scale
// inversely), so each axis's three weights are normalised to sum one.  With
// the per-axis mean m_a and variance v_a of the offsets d_a = (x^k_a - x_a)/h
// under those weights, the moment matrix of the linear basis p = [1, dx, dy,
// dz] is A = S (pm pm^T + diag(0, v_x, v_y, v_z)), pm = [1, m_x, m_y, m_z],
// S the product of the weight sums, and its inverse is closed-form: the
// weighted linear fit of values q_k has gradient coefficients
//   a_a = sum_k Wn_k (d_a - m_a) q_k / v_a        (a = x, y, z)
// and value a_0 = sum_k Wn_k q_k - sum_a m_a a_a (Wn the normalised weight
// product), and the shape functions are
//   phi_ijk = Wn_ijk (1 - sum_a m_a (d_a - m_a) / v_a).
// Every sum over the 27 points is separable (rows of three along x, then y,
// then z), so no moment matrix is formed or solved.  All MLS arithmetic is
// FP64; the fields are R.
//
// The per-axis parts are shared: along any axis the three MAC lattices sit at
// only two offsets (integer or half cells), so a marker computes six axes for
// all three lattices (a probe end six for its four fits, the cell-centred
// pressure lattice taking the half-cell ones), and the three weights of an
// axis take one exponential (scaled by exp(2 d_c q^2) / w_c they
// are exp(-q^2) exp(2 d_c q^2)^2, exp(2 d_c q^2), exp(-q^2)).
//
// On plans with work units every transfer but the probes runs one workgroup
// per unit, with the unit's positions in LDS:
// * interpolation stages the three velocity lattices over the cell box of
//   the unit's markers in LDS (or one lattice per pass when three do not
//   fit) and fits each marker from there; a whole body takes its faces in
//   face order, so each wave writes its rows of U whole;
// * spreading adds each owned face's 27 weighted values per lattice into
//   FP64 LDS tiles over the box (ds_add_f64; the three lattices in one pass
//   when their tiles fit) and adds the tiles' non-zero points to f once;
// * direct forcing fits the marker velocity from the lattice's velocity
//   staged beside its force tile, then spreads as above.
// A marker whose support leaves the box, or a unit whose box does not fit,
// gathers from u and adds to f directly.  Plans without work units run one
// thread per marker with device atomics.  (Measured on 1000 level-4 drops:
// per-marker global atomics 18.5 ms for spreading, the tiled form 0.65 ms;
// per-marker interpolation 0.38 ms, from the staged tile 0.31 ms.)
#include <algorithm>
#include <cmath>

#include "step_common.h"
#include "xcd.h"

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
    double w[3];         // weights, normalised to sum one
    double e[3];         // gradient weights w_j (d_j - m) / v
    double m;            // mean offset sum_j w_j d_j (offsets d_j = (x^k - x) / h)
    int c;               // unwrapped index of the middle point
    bool ok;             // weights and variance finite, variance positive
};

__device__ __forceinline__ void mls_axis(double xa, double off, int n, const MlsGrid &g,
                                         MlsAxis &A) {
    const double s = xa * g.inv_h - off;
    double c = floor(s + 0.5);
    if (!(fabs(c) < 1.0e9)) c = 0.0;           // non-finite or absurd position
    double dk[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) dk[j] = (c - 1.0 + j) - s;
    A.c = (int)c;
    double w0, w1, w2;
    if (g.fast) {
        // (d1 -+ 1)^2 q^2 = d1^2 q^2 -+ 2 d1 q^2 + q^2: relative to the middle
        // weight the outer ones are exp(-q^2) exp(+-2 d1 q^2); scaled by
        // E = exp(2 d1 q^2) (|d1| <= 1/2, q^2 <= 200: all in range)
        const double E = exp(2.0 * dk[1] * g.q2);
        w0 = g.cq * E * E;
        w1 = E;
        w2 = g.cq;
    } else {
        const double r0 = fabs(dk[0]) * (1.0 / 1.5) * g.inv_alpha;
        const double r1 = fabs(dk[1]) * (1.0 / 1.5) * g.inv_alpha;
        const double r2 = fabs(dk[2]) * (1.0 / 1.5) * g.inv_alpha;
        w0 = exp(-r0 * r0);
        w1 = exp(-r1 * r1);
        w2 = exp(-r2 * r2);
    }
    w0 = fabs(dk[0]) <= 1.5 ? w0 : 0.0;
    w1 = fabs(dk[1]) <= 1.5 ? w1 : 0.0;
    w2 = fabs(dk[2]) <= 1.5 ? w2 : 0.0;
    const double inv_s = rcp_nr(w0 + w1 + w2);
    A.w[0] = w0 * inv_s;
    A.w[1] = w1 * inv_s;
    A.w[2] = w2 * inv_s;
    A.m = A.w[0] * dk[0] + A.w[1] * dk[1] + A.w[2] * dk[2];
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        dk[j] -= A.m;
        v += A.w[j] * dk[j] * dk[j];
    }
    const double inv_v = rcp_nr(v);
#pragma unroll
    for (int j = 0; j < 3; ++j) A.e[j] = A.w[j] * dk[j] * inv_v;
    A.ok = isfinite(inv_s) && isfinite(inv_v) && isfinite(A.m) && v > 0.0;
}

// The half-cell axes of a marker.  MAC lattice d sits at integer cells along
// axis d and at half cells along the other two (the cell-centred lattice at
// half cells along all three), so each half-cell axis serves two of the three
// MAC lattices; the integer-cell axis of lattice d is computed when lattice d
// is reached (fewer axes live at once).
struct MlsHalf {
    MlsAxis h[3];
};

__device__ __forceinline__ void mls_half_axes(const vec3<double> &x, const MlsGrid &g, MlsHalf &H) {
    mls_axis(x.x, 0.5, g.nx, g, H.h[0]);
    mls_axis(x.y, 0.5, g.ny, g, H.h[1]);
    mls_axis(x.z, 0.5, g.nz, g, H.h[2]);
}

__device__ __forceinline__ void mls_int_axis(const vec3<double> &x, int d, const MlsGrid &g,
                                             MlsAxis &I) {
    mls_axis(d == 0 ? x.x : d == 1 ? x.y : x.z, 0.0, d == 0 ? g.nx : d == 1 ? g.ny : g.nz, g, I);
}

// Axes of MAC lattice d from the half-cell axes and its integer-cell axis I
// (d a compile-time constant after unrolling, so the axes stay in registers).
__device__ __forceinline__ const MlsAxis &axis_x(const MlsHalf &H, const MlsAxis &I, int d) {
    return d == 0 ? I : H.h[0];
}
__device__ __forceinline__ const MlsAxis &axis_y(const MlsHalf &H, const MlsAxis &I, int d) {
    return d == 1 ? I : H.h[1];
}
__device__ __forceinline__ const MlsAxis &axis_z(const MlsHalf &H, const MlsAxis &I, int d) {
    return d == 2 ? I : H.h[2];
}

// The three axes of MAC lattice d at x, computed here.
__device__ __forceinline__ void mls_axes(const vec3<double> &x, int d, const MlsGrid &g,
                                         MlsAxis &X, MlsAxis &Y, MlsAxis &Z) {
    mls_axis(x.x, mac_off(d, 0), g.nx, g, X);
    mls_axis(x.y, mac_off(d, 1), g.ny, g, Y);
    mls_axis(x.z, mac_off(d, 2), g.nz, g, Z);
}

// MLS fit of the lattice values q over the 27 support points: a[0] the value
// at the marker, a[1..3] the gradient in units of 1/h.  Separable sums: rows
// along x, then y, then z (KZ: unroll count of the z planes; 1 keeps a
// plane's nine gathers in flight at a time).
// Wrapped lattice indices of an axis's three support points (c - 1, c, c + 1
// on a periodic lattice of n points); computed where a gather or an atomic
// to the grid needs them, so the axes carry only the unwrapped c.
struct Wrap3 {
    int i[3];
};
__device__ __forceinline__ Wrap3 wrap3(int c, int n) {
    const int m = wrapi(c, n);
    return {{m == 0 ? n - 1 : m - 1, m, m == n - 1 ? 0 : m + 1}};
}

// a[k] by selects: with k a loop counter that is not unrolled, indexing the
// array would place it in scratch memory
template <typename T>
__device__ __forceinline__ T pick3(const T (&a)[3], int k) {
    return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]);
}

// ld(i, j, k): the value at support point (i, j, k).
template <int KZ, typename Load>
__device__ __forceinline__ void mls_fit_with(const MlsAxis &X, const MlsAxis &Y, const MlsAxis &Z,
                                             double a[4], Load &&ld) {
    double t0 = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
#pragma unroll KZ
    for (int k = 0; k < 3; ++k) {
        double s0 = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double r0 = 0.0, rx = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double v = ld(i, j, k);
                r0 += X.w[i] * v;
                rx += X.e[i] * v;
            }
            s0 += Y.w[j] * r0;
            sx += Y.w[j] * rx;
            sy += Y.e[j] * r0;
        }
        const double wz = KZ == 1 ? pick3(Z.w, k) : Z.w[k];
        const double ez = KZ == 1 ? pick3(Z.e, k) : Z.e[k];
        t0 += wz * s0;
        tx += wz * sx;
        ty += wz * sy;
        tz += ez * s0;
    }
    a[1] = tx;
    a[2] = ty;
    a[3] = tz;
    a[0] = t0 - X.m * tx - Y.m * ty - Z.m * tz;
}

// The fit from a lattice field q in global memory (wrapped indices).
template <typename R, int KZ = 3>
__device__ __forceinline__ void mls_fit(const MlsAxis &X, const MlsAxis &Y, const MlsAxis &Z,
                                        const MlsGrid &g, const R *__restrict__ q, double a[4]) {
    const Wrap3 wx = wrap3(X.c, g.nx), wy = wrap3(Y.c, g.ny), wz = wrap3(Z.c, g.nz);
    mls_fit_with<KZ>(X, Y, Z, a, [&](int i, int j, int k) {
        const int zk = KZ == 1 ? pick3(wz.i, k) : wz.i[k];
        return (double)q[(int64_t)zk * g.plane + (int64_t)wy.i[j] * g.nx + wx.i[i]];
    });
}

// sum_k phi_k (1 up to rounding: the fit reproduces constants).
__device__ __forceinline__ double mls_phi_sum(const MlsAxis &X, const MlsAxis &Y,
                                              const MlsAxis &Z) {
    const double gx = X.w[0] + X.w[1] + X.w[2], gy = Y.w[0] + Y.w[1] + Y.w[2],
                 gz = Z.w[0] + Z.w[1] + Z.w[2];
    const double ex = X.e[0] + X.e[1] + X.e[2], ey = Y.e[0] + Y.e[1] + Y.e[2],
                 ez = Z.e[0] + Z.e[1] + Z.e[2];
    return gx * gy * gz - X.m * ex * gy * gz - Y.m * gx * ey * gz - Z.m * gx * gy * ez;
}

// fn(i, j, k, phi_ijk) at the 27 support points, in (k, j, i) order.
template <typename Fn>
__device__ __forceinline__ void mls_for_each_phi(const MlsAxis &X, const MlsAxis &Y,
                                                 const MlsAxis &Z, Fn &&fn) {
    double hx[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) hx[i] = X.m * X.e[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double hz = Z.m * Z.e[k];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double gyz = Y.w[j] * Z.w[k];
            const double t = gyz - (Y.m * Y.e[j] * Z.w[k] + Y.w[j] * hz);
#pragma unroll
            for (int i = 0; i < 3; ++i) fn(i, j, k, X.w[i] * t - hx[i] * gyz);
        }
    }
}

// out[3 f + c] = v[c] for the wave's consecutive faces f = f0 + lane (those
// below F), written as whole rows: lane l stores elements l, l + 64 and
// l + 128 of the wave's 192-value segment, exchanged across lanes, so each
// store instruction covers consecutive words rather than every third one (a
// stride-3 store leaves partial lines).  f0 is the face of lane 0; every lane
// of the wave calls it.
template <typename R>
__device__ __forceinline__ void store3_rows(R *__restrict__ out, int64_t f0, int64_t F,
                                            const double v[3]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int e = lane + 64 * k, src = e / 3, c = e - 3 * src;
        const double a0 = __shfl(v[0], src), a1 = __shfl(v[1], src), a2 = __shfl(v[2], src);
        const double val = c == 0 ? a0 : (c == 1 ? a1 : a2);
        if (f0 + src < F) out[3 * f0 + e] = (R)val;
    }
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
    const int64_t f = xcd_block() * blockDim.x + threadIdx.x;
    if (f >= F) return;
    bool bad = false;
    double area;
    const vec3<double> x = centroid(X, faces, f, area);
    MlsHalf H;
    mls_half_axes(x, g, H);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        MlsAxis I;
        mls_int_axis(x, d, g, I);
        const MlsAxis &AX = axis_x(H, I, d), &AY = axis_y(H, I, d), &AZ = axis_z(H, I, d);
        bad |= !(AX.ok && AY.ok && AZ.ok);
        double a[4];
        mls_fit<R>(AX, AY, AZ, g, u + d * g.field, a);
        U[3 * f + d] = (R)a[0];
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
    const int64_t f = xcd_block() * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double area;
    const vec3<double> x = centroid(X, faces, f, area);
    MlsHalf H;
    mls_half_axes(x, g, H);
    bool bad = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        MlsAxis I;
        mls_int_axis(x, d, g, I);
        const MlsAxis &AX = axis_x(H, I, d), &AY = axis_y(H, I, d), &AZ = axis_z(H, I, d);
        bad |= !(AX.ok && AY.ok && AZ.ok);
        // c_l as the paper writes it, with sum_k phi_k (1 up to rounding)
        const double sphi = mls_phi_sum(AX, AY, AZ);
        const double hl = (1.0 / 3.0) * sphi * (3.0 * g.h);
        const double cl = area * hl / (sphi * g.h * g.h * g.h);
        const double Fd = (double)Fm[3 * f + d] * cl;
        R *fd = fld + d * g.field;
        const Wrap3 wx = wrap3(AX.c, g.nx), wy = wrap3(AY.c, g.ny), wz = wrap3(AZ.c, g.nz);
        mls_for_each_phi(AX, AY, AZ, [&](int i, int j, int k, double ph) {
            unsafeAtomicAdd(fd + (int64_t)wz.i[k] * g.plane + (int64_t)wy.i[j] * g.nx + wx.i[i],
                            (R)(ph * Fd));
        });
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
    const int64_t f = xcd_block() * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double area;
    const vec3<double> x = centroid(X, faces, f, area);
    MlsHalf H;
    mls_half_axes(x, g, H);
    bool bad = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        MlsAxis I;
        mls_int_axis(x, d, g, I);
        const MlsAxis &AX = axis_x(H, I, d), &AY = axis_y(H, I, d), &AZ = axis_z(H, I, d);
        bad |= !(AX.ok && AY.ok && AZ.ok);
        double a[4];
        mls_fit<R>(AX, AY, AZ, g, u + d * g.field, a);
        const double Fl = ((double)Vb[3 * f + d] - a[0]) * inv_dt;
        if (Fout != nullptr) Fout[3 * f + d] = (R)Fl;
        const double sphi = mls_phi_sum(AX, AY, AZ);
        const double hl = (1.0 / 3.0) * sphi * (3.0 * g.h);
        const double Fd = Fl * area * hl / (sphi * g.h * g.h * g.h);
        R *fd = fld + d * g.field;
        const Wrap3 wx = wrap3(AX.c, g.nx), wy = wrap3(AY.c, g.ny), wz = wrap3(AZ.c, g.nz);
        mls_for_each_phi(AX, AY, AZ, [&](int i, int j, int k, double ph) {
            unsafeAtomicAdd(fd + (int64_t)wz.i[k] * g.plane + (int64_t)wy.i[j] * g.nx + wx.i[i],
                            (R)(ph * Fd));
        });
    }
    if (bad) atomicOr(status, IP_STATUS_NONFINITE);
}

// External loads on face f from probes of length h along its unit normal:
// one outward probe on closed bodies, both sides on open ones.  At a probe
// end y = x_c + s h n: p = (MLS value of the cell-centred pressure) +
// s h (Du/Dt).n, G_ij = du_i/dx_j (gradient of the MLS fit of lattice i),
// tau = mu (G + G^T); the load is sum_s s (-p n + tau n) A.
template <typename R>
__device__ __forceinline__ void probe_face(
    int64_t f, int lo, const double *__restrict__ X, const int32_t *__restrict__ faces,
    const uint8_t *__restrict__ closed, const R *__restrict__ u, const R *__restrict__ pr,
    const R *__restrict__ acc, const MlsGrid &g, double mu, double out[3], uint32_t *status) {
    const vec3<double> xa = ldX(X, faces[3 * f]), xb = ldX(X, faces[3 * f + 1]),
                       xc3 = ldX(X, faces[3 * f + 2]);
    const vec3<double> nn = cross(xb - xa, xc3 - xa);
    const double nlen = sqrt(dot(nn, nn));
    if (!(nlen > 0.0)) {
        // a zero-area face has no normal: no probe, no load
        out[0] = out[1] = out[2] = 0.0;
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
        // all three axes, velocity lattice i the integer one along axis i and
        // the same half-cell axes along the others: six axes for the four
        // fits.  (G + G^T) n is accumulated row by row as the fits give the
        // rows G_i. of the velocity gradient: component i takes (G n)_i,
        // every component j takes G_ij n_i; the loop over i is unrolled so
        // that each lattice's axes are chosen at compile time (a choice made
        // at run time would place the axes in scratch memory)
        double ap[4];
        MlsHalf H;
        mls_half_axes(y, g, H);
        bad |= !(H.h[0].ok && H.h[1].ok && H.h[2].ok);
        mls_fit<R, 1>(H.h[0], H.h[1], H.h[2], g, pr, ap);
        double tn0 = 0.0, tn1 = 0.0, tn2 = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double ai[4];
            MlsAxis I;
            mls_int_axis(y, i, g, I);
            bad |= !I.ok;
            mls_fit<R, 1>(axis_x(H, I, i), axis_y(H, I, i), axis_z(H, I, i), g, u + i * g.field, ai);
            const double gx = ai[1] * g.inv_h, gy = ai[2] * g.inv_h, gz = ai[3] * g.inv_h;
            const double ni = i == 0 ? nu.x : (i == 1 ? nu.y : nu.z);
            const double gn = gx * nu.x + gy * nu.y + gz * nu.z;
            tn0 += gx * ni + (i == 0 ? gn : 0.0);
            tn1 += gy * ni + (i == 1 ? gn : 0.0);
            tn2 += gz * ni + (i == 2 ? gn : 0.0);
        }
        const double pl = ap[0] + sg * g.h * an;
        const double Fs[3] = {sg * (-pl * nu.x + mu * tn0) * area,
                              sg * (-pl * nu.y + mu * tn1) * area,
                              sg * (-pl * nu.z + mu * tn2) * area};
        F0 += Fs[0];
        F1 += Fs[1];
        F2 += Fs[2];
    }
    out[0] = F0;
    out[1] = F1;
    out[2] = F2;
    if (bad) atomicOr(status, IP_STATUS_NONFINITE);
}

template <typename R>
__global__ __launch_bounds__(256, 2) void k_probe_loads(
    const double *__restrict__ X, const int32_t *__restrict__ faces,
    const int64_t *__restrict__ face_off, const uint8_t *__restrict__ closed, int B, int64_t F,
    const R *__restrict__ u, const R *__restrict__ pr, const R *__restrict__ acc, MlsGrid g,
    double mu, R *__restrict__ Fext, uint32_t *status) {
    // blocks in XCD-contiguous order: the faces of a body, whose probe ends
    // read the same grid points, share an L2
    const int64_t f = xcd_block() * blockDim.x + threadIdx.x;
    // body of face f, the last b with face_off[b] <= f: one binary search for
    // the wave's first face on scalar registers (the wave's faces are
    // consecutive), then each lane steps over the few body ends before its face
    const int64_t fl = f - (threadIdx.x & 63);
    const int64_t fw = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(fl >> 32))
                                  << 32) |
                                 (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)fl));
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (face_off[mid] <= fw)
            lo = mid;
        else
            hi = mid - 1;
    }
    while (lo + 1 < B && face_off[lo + 1] <= f) ++lo;
    double v[3] = {0.0, 0.0, 0.0};
    if (f < F) probe_face<R>(f, lo, X, faces, closed, u, pr, acc, g, mu, v, status);
    store3_rows(Fext, f - (threadIdx.x & 63), F, v);
}

// The centroid's cell (the stencil centre of the lattices staggered by half a
// cell, as the fused step's tile uses): the supports of all three lattices lie
// in points cell - 1 .. cell + 2 per axis.
__device__ __forceinline__ int mls_cell(double x, double inv_h) {
    double c = floor((x * inv_h - 0.5) + 0.5);      // the expression mls_axis uses
    if (!(fabs(c) < 1.0e9)) c = 0.0;
    return (int)c;
}

// Centroid of the face with unit-local corners q (positions in LDS).
__device__ __forceinline__ vec3<double> marker_of(const double *xs, const uint16_t *q) {
    const vec3<double> s = ldx(xs, q[0]) + ldx(xs, q[1]) + ldx(xs, q[2]);
    return vec3<double>{s.x * (1.0 / 3.0), s.y * (1.0 / 3.0), s.z * (1.0 / 3.0)};
}

// Centroid of the face with unit-local corners c (positions in LDS).
__device__ __forceinline__ vec3<double> marker_at(const double *xs, const int c[3]) {
    const vec3<double> s = ldx(xs, c[0]) + ldx(xs, c[1]) + ldx(xs, c[2]);
    return vec3<double>{s.x * (1.0 / 3.0), s.y * (1.0 / 3.0), s.z * (1.0 / 3.0)};
}

struct MlsUnitArgs {
    const double *X;
    const void *Fm;          // marker forces (spreading)
    const void *u, *Vb;      // velocity field and desired marker velocity (direct forcing)
    void *Fout;              // marker forces written by direct forcing (may be NULL)
    void *U;                 // interpolated marker velocities (interpolation)
    double inv_dt;
    void *f;
    MlsGrid g;
    uint32_t *status;
    const int64_t *node_off;
    const int32_t *wu_body, *wu_owned, *wu_nodes, *frec_perm;
    const int64_t *wu_noff, *wu_foff;
    const uint16_t *frec_lid;
    const int32_t *faces;        // [F][3] global corners (whole units take faces in face order)
    const int64_t *face_off;
    int nmax, tile_bytes;
};

// The unit's t-th face: unit-local corners c and the global face id, or -1
// for a patch's record whose first corner it does not own.  A whole unit
// (fb = its body's first face) takes its faces in face order, so that
// consecutive lanes read and write consecutive faces; a patch takes its
// records.
__device__ __forceinline__ int64_t unit_face(const MlsUnitArgs &a, bool whole, int64_t fb,
                                             int64_t n0, int64_t f0, int N, int t, int c[3]) {
    if (whole) {
        const int32_t *q = a.faces + 3 * (fb + t);
        c[0] = (int)(q[0] - n0);
        c[1] = (int)(q[1] - n0);
        c[2] = (int)(q[2] - n0);
        return fb + t;
    }
    const uint16_t *q = a.frec_lid + 4 * (f0 + t);
    c[0] = q[0];
    c[1] = q[1];
    c[2] = q[2];
    return c[0] < N ? (int64_t)a.frec_perm[f0 + t] : -1;
}

// Cell box (lo, hi per axis, reduced over the block) of the markers a unit
// owns: the faces whose first corner is one of its owned nodes.
template <int NT>
__device__ __forceinline__ void owned_marker_box(const double *xs, const uint16_t *frec, int F,
                                                 int N, double inv_h, int lo[3], int hi[3],
                                                 int *ired, double *red) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = INT_MAX;
        hi[c] = INT_MIN;
    }
    for (int t = threadIdx.x; t < F; t += NT) {
        const uint16_t *q = frec + 4 * t;
        if (q[0] >= N) continue;                   // first corner not owned here
        const vec3<double> p = marker_of(xs, q);
        const int cc[3] = {mls_cell(p.x, inv_h), mls_cell(p.y, inv_h), mls_cell(p.z, inv_h)};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = min(lo[c], cc[c]);
            hi[c] = max(hi[c], cc[c]);
        }
    }
    double none[1] = {0.0};
    block_box_sums<NT, 1>(lo, hi, none, ired, red);
}

// Tile over grid points lo - 1 .. lo + L - 2 per axis (L = hi - lo + 4), the
// threads' first points and strides (a tile no larger than the grid).
template <int NT>
__device__ __forceinline__ TileGeom mls_tile_geom(const int lo[3], int Tx, int Ty, int Tz,
                                                  const MlsGrid &g) {
    TileGeom tg{{lo[0], lo[1], lo[2]}, Tx, Ty, Tz, Tx * Ty * Tz, g.nx, g.ny, g.nz,
                g.plane, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    const int tid = threadIdx.x;
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
    return tg;
}

// The three lattices' tiles in one walk: three loads per tile point, U points
// per thread in flight.
template <int NT, typename R, int U = 8>
__device__ __forceinline__ void stage_tiles3(R *__restrict__ tile, const R *__restrict__ field,
                                             int64_t fstride, int Tl, const TileGeom &g) {
    TileCursor c = TileCursor::first(g);
    while (c.t < g.T) {
        R v0[U], v1[U], v2[U];
        int t[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            t[k] = c.t;
            if (c.t < g.T) {
                const int64_t i = c.grid_index(g);
                v0[k] = field[i];
                v1[k] = field[fstride + i];
                v2[k] = field[2 * fstride + i];
            } else {
                v0[k] = v1[k] = v2[k] = (R)0;
            }
            c.template next<NT>(g);
        }
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (t[k] < g.T) {
                tile[t[k]] = v0[k];
                tile[Tl + t[k]] = v1[k];
                tile[2 * Tl + t[k]] = v2[k];
            }
    }
}

// Interpolation at the faces owned by one work unit (one workgroup per unit).
// The velocity over the cell box of the unit's markers is staged in LDS,
// coalesced, so each marker's 81 reads come from LDS instead of scattered
// gathers (one cache line per lane and read).  All three lattices are staged
// at once when they fit, the marker then sharing its half-cell axes across
// them; otherwise one lattice per pass; a unit whose box does not fit at all,
// and any marker outside the box, gathers from u.
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_interp_mls_units(MlsUnitArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ double red[NT / 64];
    __shared__ int ired[6 * (NT / 64)];
    const int tid = threadIdx.x;
    const int w = xcd_unit((int)blockIdx.x, (int)gridDim.x);
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
    R *tile = (R *)(xs + 3 * a.nmax);                            // tile_bytes
    const R *u = (const R *)a.u;
    R *Uo = (R *)a.U;
    const MlsGrid &g = a.g;
    const uint16_t *frec = a.frec_lid + 4 * f0;

    int lo[3], hi[3];
    load_positions<NT>(xs, a.X, whole, n0, gid, NL, N, g.inv_h, lo, hi);
    if (whole) {
        // a centroid lies between its corners, so its cell lies in the box of
        // the body's node cells (the same monotone cell function; a marker a
        // rounding pushes outside is caught by the in-tile check): no pass
        // over the face records is needed to find the box
        double none[1] = {0.0};
        block_box_sums<NT, 1>(lo, hi, none, ired, red);
    } else {
        owned_marker_box<NT>(xs, frec, F, N, g.inv_h, lo, hi, ired, red);
    }
    if (lo[0] > hi[0]) return;                     // no owned marker (uniform)
    const long long Lx = (long long)hi[0] - lo[0] + 4, Ly = (long long)hi[1] - lo[1] + 4,
                    Lz = (long long)hi[2] - lo[2] + 4;
    const long long Tl = Lx * Ly * Lz;
    const bool box_ok = Lx <= g.nx && Ly <= g.ny && Lz <= g.nz;
    const int per_pass = !box_ok                                         ? 0
                         : 3 * Tl * (long long)sizeof(R) <= a.tile_bytes ? 3
                         : Tl * (long long)sizeof(R) <= a.tile_bytes     ? 1
                                                                         : 0;
    bool bad = false;
    // marker t's fit on lattice d from the tile T of that lattice, or from u
    // when a support point falls outside the tile
    auto fit = [&](const MlsAxis &X, const MlsAxis &Y, const MlsAxis &Z, int d, const R *T,
                   double out[4]) {
        const int ox = X.c - lo[0], oy = Y.c - lo[1], oz = Z.c - lo[2];
        if (T != nullptr && ox >= 0 && oy >= 0 && oz >= 0 && ox + 2 < Lx && oy + 2 < Ly &&
            oz + 2 < Lz) {
            const R *base = T + (oz * (int)Ly + oy) * (int)Lx + ox;
            // one z plane (nine LDS reads) at a time: fewer registers
            mls_fit_with<1>(X, Y, Z, out, [&](int i, int j, int k) {
                return (double)base[(k * (int)Ly + j) * (int)Lx + i];
            });
        } else {
            mls_fit<R>(X, Y, Z, g, u + d * g.field, out);
        }
    };
    // whole units take their faces in face order: rows of U written whole
    const int64_t fb = whole ? a.face_off[b] : 0;
    const auto face_of = [&](int t, int c[3]) -> int64_t {
        return unit_face(a, whole, fb, n0, f0, N, t, c);
    };
    const int lane = tid & 63;
    if (per_pass != 1) {
        // all three lattices per marker, from the tile (per_pass 3) or from u
        if (per_pass == 3) {
            const TileGeom tg = mls_tile_geom<NT>(lo, (int)Lx, (int)Ly, (int)Lz, g);
            stage_tiles3<NT, R>(tile, u, g.field, (int)Tl, tg);
            lds_barrier();
        }
        for (int t0 = tid - lane; t0 < F; t0 += NT) {          // wave-uniform bound
            // lanes past the last face repeat it (every lane takes part in
            // the row store); a patch's records it does not own are computed
            // and not stored
            const int t = min(t0 + lane, F - 1);
            int c[3];
            const int64_t pf = face_of(t, c);
            const vec3<double> x = marker_at(xs, c);
            MlsHalf H;
            mls_half_axes(x, g, H);
            double v[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                MlsAxis I;
                mls_int_axis(x, d, g, I);
                const MlsAxis &AX = axis_x(H, I, d), &AY = axis_y(H, I, d), &AZ = axis_z(H, I, d);
                if (pf >= 0) bad |= !(AX.ok && AY.ok && AZ.ok);
                double r[4];
                fit(AX, AY, AZ, d, per_pass == 3 ? tile + d * Tl : nullptr, r);
                v[d] = r[0];
            }
            if (whole) {
                store3_rows(Uo, fb + t0, fb + F, v);
            } else if (pf >= 0 && t0 + lane < F) {
                Uo[3 * pf] = (R)v[0];
                Uo[3 * pf + 1] = (R)v[1];
                Uo[3 * pf + 2] = (R)v[2];
            }
        }
    } else {
        // one lattice per pass
        const TileGeom tg = mls_tile_geom<NT>(lo, (int)Lx, (int)Ly, (int)Lz, g);
#pragma unroll 1
        for (int d0 = 0; d0 < 3; ++d0) {
            stage_tile<NT, R>(tile, u + d0 * g.field, tg);
            lds_barrier();
            for (int t = tid; t < F; t += NT) {
                int c[3];
                const int64_t pf = face_of(t, c);
                if (pf < 0) continue;
                const vec3<double> x = marker_at(xs, c);
                MlsAxis AX, AY, AZ;
                mls_axes(x, d0, g, AX, AY, AZ);
                bad |= !(AX.ok && AY.ok && AZ.ok);
                double r[4];
                fit(AX, AY, AZ, d0, tile, r);
                Uo[3 * pf + d0] = (R)r[0];
            }
            lds_barrier();                         // before the next pass restages
        }
    }
    if (bad) atomicOr(a.status, IP_STATUS_NONFINITE);
}

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
    const int w = xcd_unit((int)blockIdx.x, (int)gridDim.x);
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
    owned_marker_box<NT>(xs, a.frec_lid + 4 * f0, F, N, g.inv_h, lo, hi, ired, red);
    if (lo[0] > hi[0]) return;                     // no owned marker (uniform)
    // tile points lo - 1 .. hi + 2 per axis
    const long long Lx = (long long)hi[0] - lo[0] + 4, Ly = (long long)hi[1] - lo[1] + 4,
                    Lz = (long long)hi[2] - lo[2] + 4;
    const bool box_ok = Lx <= g.nx && Ly <= g.ny && Lz <= g.nz;
    const long long Tl = Lx * Ly * Lz;
    // all three lattices' tiles at once when they fit (each face then
    // computes its geometry and half-cell axes once), else one per pass.
    // Direct forcing keeps one lattice per pass: with its fits beside the
    // shared axes it spills (56 registers against 12).
    const bool all3 = !DF && box_ok && 3 * Tl * 8 <= a.tile_bytes;
    const bool use_tile = box_ok && Tl * 8 <= a.tile_bytes;
    const int Tx = (int)Lx, Ty = (int)Ly, Tz = (int)Lz;
    bool bad = false;
    // face pf (area, the axes of lattice d) into T, the lattice's tile, or,
    // without a tile or outside it, into f directly
    // UT: lattice d's velocity staged over the box (direct forcing), or null
    const auto spread_one = [&](int d, const MlsAxis &AX, const MlsAxis &AY, const MlsAxis &AZ,
                                double area, int64_t pf, double *T, const R *UT) {
        bad |= !(AX.ok && AY.ok && AZ.ok);
        const double sphi = mls_phi_sum(AX, AY, AZ);
        const double hl = (1.0 / 3.0) * sphi * (3.0 * g.h);
        const double cl = area * hl / (sphi * g.h * g.h * g.h);
        const int ox = AX.c - lo[0], oy = AY.c - lo[1], oz = AZ.c - lo[2];
        const bool inside = ox >= 0 && oy >= 0 && oz >= 0 && ox + 2 < Tx && oy + 2 < Ty &&
                            oz + 2 < Tz;
        double Fl;
        if constexpr (DF) {
            double fit[4];
            if (UT != nullptr && inside) {
                const R *base = UT + (oz * Ty + oy) * Tx + ox;
                mls_fit_with<1>(AX, AY, AZ, fit, [&](int i, int j, int k) {
                    return (double)base[(k * Ty + j) * Tx + i];
                });
            } else {
                mls_fit<R>(AX, AY, AZ, g, (const R *)a.u + d * g.field, fit);
            }
            Fl = ((double)((const R *)a.Vb)[3 * pf + d] - fit[0]) * a.inv_dt;
            if (a.Fout != nullptr) ((R *)a.Fout)[3 * pf + d] = (R)Fl;
        } else {
            Fl = (double)Fm[3 * pf + d];
        }
        const double Fd = Fl * cl;
        // support point c - 1 + j is tile point c + j - lo (inside the tile
        // for every marker the box was taken from; checked all the same)
        if (T != nullptr && inside) {
            double *base = T + (oz * Ty + oy) * Tx + ox;
            mls_for_each_phi(AX, AY, AZ, [&](int i, int j, int k, double ph) {
                lds_add(base + (k * Ty + j) * Tx + i, ph * Fd);
            });
        } else {
            R *fd = fld + d * g.field;
            const Wrap3 wx = wrap3(AX.c, g.nx), wy = wrap3(AY.c, g.ny), wz = wrap3(AZ.c, g.nz);
            mls_for_each_phi(AX, AY, AZ, [&](int i, int j, int k, double ph) {
                unsafeAtomicAdd(fd + (int64_t)wz.i[k] * g.plane + (int64_t)wy.i[j] * g.nx + wx.i[i],
                                (R)(ph * Fd));
            });
        }
    };
    // record order also for whole units: the records of a run of 64 touch
    // distinct nodes, so the lanes of a wave add into distinct tile points
    // (in face order neighbouring faces of the subdivided mesh collide: 1.30
    // against 0.72 ms on the 1000-drop batch)
    if (all3) {
        const TileGeom tg = mls_tile_geom<NT>(lo, Tx, Ty, Tz, g);
        for (int t = tid; t < 3 * tg.T; t += NT) tile[t] = 0.0;
        lds_barrier();
        for (int t = tid; t < F; t += NT) {
            int q[3];
            const int64_t pf = unit_face(a, false, 0, n0, f0, N, t, q);
            if (pf < 0) continue;
            const vec3<double> xa = ldx(xs, q[0]), xb = ldx(xs, q[1]), xc = ldx(xs, q[2]);
            const vec3<double> n = cross(xb - xa, xc - xa);
            const double area = 0.5 * sqrt(dot(n, n));
            const vec3<double> p = marker_at(xs, q);
            MlsHalf H;
            mls_half_axes(p, g, H);
            // one lattice at a time (unrolled, the three interleave and spill)
#pragma unroll 1
            for (int d = 0; d < 3; ++d) {
                MlsAxis I;
                mls_int_axis(p, d, g, I);
                spread_one(d, axis_x(H, I, d), axis_y(H, I, d), axis_z(H, I, d), area, pf,
                           tile + d * tg.T, nullptr);
            }
        }
        lds_barrier();
        for (TileCursor c = TileCursor::first(tg); c.t < tg.T; c.template next<NT>(tg)) {
            const int64_t gi = c.grid_index(tg);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double v = tile[d * tg.T + c.t];
                if (v != 0.0) unsafeAtomicAdd(fld + d * g.field + gi, (R)v);
            }
        }
    } else {
        TileGeom tg{{lo[0], lo[1], lo[2]}, 1, 1, 1, 0, g.nx, g.ny, g.nz, g.plane,
                    {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        if (use_tile) tg = mls_tile_geom<NT>(lo, Tx, Ty, Tz, g);
        // direct forcing: lattice d's velocity staged beside its force tile
        // when both fit, so the fits read LDS instead of gathering from u
        R *utile = DF && use_tile && Tl * (8 + (long long)sizeof(R)) <= a.tile_bytes
                       ? (R *)(tile + Tl)
                       : nullptr;
#pragma unroll 1
        for (int d = 0; d < 3; ++d) {
            if (use_tile) {
                for (int t = tid; t < tg.T; t += NT) tile[t] = 0.0;
                if (utile != nullptr) stage_tile<NT, R>(utile, (const R *)a.u + d * g.field, tg);
                lds_barrier();
            }
            for (int t = tid; t < F; t += NT) {
                int q[3];
                const int64_t pf = unit_face(a, false, 0, n0, f0, N, t, q);
                if (pf < 0) continue;
                const vec3<double> xa = ldx(xs, q[0]), xb = ldx(xs, q[1]), xc = ldx(xs, q[2]);
                const vec3<double> n = cross(xb - xa, xc - xa);
                const double area = 0.5 * sqrt(dot(n, n));
                const vec3<double> p = marker_at(xs, q);
                MlsAxis AX, AY, AZ;
                mls_axes(p, d, g, AX, AY, AZ);
                spread_one(d, AX, AY, AZ, area, pf, use_tile ? tile : nullptr, utile);
            }
            if (use_tile) {
                lds_barrier();
                R *fd = fld + d * g.field;
                for (TileCursor c = TileCursor::first(tg); c.t < tg.T; c.template next<NT>(tg)) {
                    const double v = tile[c.t];
                    if (v != 0.0) unsafeAtomicAdd(fd + c.grid_index(tg), (R)v);
                }
                lds_barrier();
            }
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
    const int64_t n = xcd_block() * blockDim.x + threadIdx.x;
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
    a.faces = p->faces;
    a.face_off = p->face_off;
    a.nmax = p->fused_nmax;
    a.tile_bytes = (int)std::max<long long>((lds_optin - 1024 - 24LL * a.nmax) / 16 * 16, 0);
    lds = (size_t)24 * a.nmax + (size_t)a.tile_bytes;
    return IP_OK;
}

// One workgroup per unit fills the LDS with its tile, so the workgroup size
// sets the waves per SIMD: 768 threads give 3 (512 gave 2 and were slower).
constexpr int kMlsThreads = 768;
// Interpolation on work units: the tile is read, not added to.
constexpr int kMlsInterpThreads = 768;

// Launch attributes of the per-unit kernels (their dynamic LDS), set once when
// the plan is built, so that the launches themselves can be captured.
template <typename R>
static ip_status set_unit_attributes(size_t lds) {
    const void *fns[3] = {(const void *)k_spread_mls_units<R, kMlsThreads, false>,
                          (const void *)k_spread_mls_units<R, kMlsThreads, true>,
                          (const void *)k_interp_mls_units<R, kMlsInterpThreads>};
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
    if (p->fused_all && p->n_units > 0) {
        MlsUnitArgs a{};
        size_t lds = 0;
        IP_TRY(unit_args(p, X, alpha, a, lds));
        a.u = u;
        a.U = U;
        if (p->prec == IP_F64)
            hipLaunchKernelGGL((k_interp_mls_units<double, kMlsInterpThreads>), dim3(p->n_units),
                               dim3(kMlsInterpThreads), lds, s, a);
        else
            hipLaunchKernelGGL((k_interp_mls_units<float, kMlsInterpThreads>), dim3(p->n_units),
                               dim3(kMlsInterpThreads), lds, s, a);
        IP_HIP_CHECK(hipGetLastError());
        return IP_OK;
    }
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
