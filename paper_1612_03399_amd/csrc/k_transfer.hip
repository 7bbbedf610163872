// k_transfer.hip -- Eulerian <-> Lagrangian transfer with the 3-point
// regularised delta (27-point support, Section 2.2 of Spandan et al.) and the
// explicit node update (Section 2.3).
#include "ipibm_internal.h"
#include "xcd.h"

namespace {

struct GridArgs {
    int nx, ny, nz;
    double inv_h;
    int64_t plane, field;
};

inline GridArgs grid_args(const ip_plan *p) {
    GridArgs g;
    g.nx = p->grid.nx;
    g.ny = p->grid.ny;
    g.nz = p->grid.nz;
    g.inv_h = 1.0 / p->grid.h;
    g.plane = (int64_t)g.nx * g.ny;
    g.field = g.plane * g.nz;
    return g;
}

// Stencil of one node on lattice d: wrapped indices and weights per axis.
template <typename R>
struct Stencil {
    int ix[3], iy[3], iz[3];
    R wx[3], wy[3], wz[3];
};

template <typename R>
__device__ __forceinline__ void stencil(const vec3<double> &x, int d, const GridArgs &g,
                                        Stencil<R> &st) {
    const int cx = delta3<R>(x.x * g.inv_h - mac_off(d, 0), st.wx);
    const int cy = delta3<R>(x.y * g.inv_h - mac_off(d, 1), st.wy);
    const int cz = delta3<R>(x.z * g.inv_h - mac_off(d, 2), st.wz);
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        st.ix[o] = wrapi(cx - 1 + o, g.nx);
        st.iy[o] = wrapi(cy - 1 + o, g.ny);
        st.iz[o] = wrapi(cz - 1 + o, g.nz);
    }
}

// U_d(X_l) = sum over the 27 points of lattice d of u_d * wx wy wz.
template <typename R>
__global__ __launch_bounds__(256) void k_interp(const double *__restrict__ X,
                                                const R *__restrict__ u, int64_t N, GridArgs g,
                                                R *__restrict__ U) {
    const int64_t l = xcd_block() * blockDim.x + threadIdx.x;
    if (l >= N) return;
    const vec3<double> x = ldX(X, l);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Stencil<R> st;
        stencil(x, d, g, st);
        const R *ud = u + d * g.field;
        R acc = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int bq = 0; bq < 3; ++bq) {
                const R *row = ud + st.iz[c] * g.plane + (int64_t)st.iy[bq] * g.nx;
                const R wzy = st.wz[c] * st.wy[bq];
                acc += wzy * (st.wx[0] * row[st.ix[0]] + st.wx[1] * row[st.ix[1]] +
                              st.wx[2] * row[st.ix[2]]);
            }
        }
        U[3 * l + d] = acc;
    }
}

// f_d += F_{l,d} wx wy wz / h^3 over the 27 points of lattice d (device atomics).
template <typename R>
__global__ __launch_bounds__(256) void k_spread(const double *__restrict__ X,
                                                const R *__restrict__ Fn, int64_t N, GridArgs g,
                                                R inv_h3, R *__restrict__ f) {
    const int64_t l = xcd_block() * blockDim.x + threadIdx.x;
    if (l >= N) return;
    const vec3<double> x = ldX(X, l);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Stencil<R> st;
        stencil(x, d, g, st);
        const R fd = Fn[3 * l + d] * inv_h3;
        R *fdp = f + d * g.field;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int bq = 0; bq < 3; ++bq) {
                R *row = fdp + st.iz[c] * g.plane + (int64_t)st.iy[bq] * g.nx;
                const R wzy = fd * st.wz[c] * st.wy[bq];
#pragma unroll
                for (int a = 0; a < 3; ++a) unsafeAtomicAdd(row + st.ix[a], wzy * st.wx[a]);
            }
        }
    }
}

// X <- X + dt U + (dt^2 / m_b) F for nodes that are not pinned (FP64).
template <typename R>
__global__ void k_update(double *__restrict__ X, const R *__restrict__ U,
                         const R *__restrict__ Fn, const uint8_t *__restrict__ pinned,
                         const int64_t *__restrict__ node_off, int B,
                         const double *__restrict__ mass, int64_t N, double dt) {
    const int64_t l = xcd_block() * blockDim.x + threadIdx.x;
    if (l >= N || pinned[l]) return;
    const int b = body_of(node_off, B, l);
    const double c = dt * dt / mass[b];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        X[3 * l + d] += dt * (double)U[3 * l + d] + c * (double)Fn[3 * l + d];
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

ip_status launch_interp(ip_plan *p, const double *X, const void *u, void *U, hipStream_t s) {
    if (p->N == 0) return IP_OK;
    const GridArgs g = grid_args(p);
    if (p->prec == IP_F64)
        hipLaunchKernelGGL(k_interp<double>, dim3(nblocks(p->N, 256)), dim3(256), 0, s, X,
                           (const double *)u, p->N, g, (double *)U);
    else
        hipLaunchKernelGGL(k_interp<float>, dim3(nblocks(p->N, 256)), dim3(256), 0, s, X,
                           (const float *)u, p->N, g, (float *)U);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

ip_status launch_spread(ip_plan *p, const double *X, const void *F, void *f, hipStream_t s) {
    if (p->N == 0) return IP_OK;
    const GridArgs g = grid_args(p);
    const double h = p->grid.h;
    const double inv_h3 = 1.0 / (h * h * h);
    if (p->prec == IP_F64)
        hipLaunchKernelGGL(k_spread<double>, dim3(nblocks(p->N, 256)), dim3(256), 0, s, X,
                           (const double *)F, p->N, g, inv_h3, (double *)f);
    else
        hipLaunchKernelGGL(k_spread<float>, dim3(nblocks(p->N, 256)), dim3(256), 0, s, X,
                           (const float *)F, p->N, g, (float)inv_h3, (float *)f);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

ip_status launch_update(ip_plan *p, double *X, const void *U, const void *F,
                        const ip_constants *k, double dt, hipStream_t s) {
    if (p->N == 0) return IP_OK;
    if (p->prec == IP_F64)
        hipLaunchKernelGGL(k_update<double>, dim3(nblocks(p->N, 256)), dim3(256), 0, s, X,
                           (const double *)U, (const double *)F, p->pinned, p->node_off, p->B,
                           k->mass, p->N, dt);
    else
        hipLaunchKernelGGL(k_update<float>, dim3(nblocks(p->N, 256)), dim3(256), 0, s, X,
                           (const float *)U, (const float *)F, p->pinned, p->node_off, p->B,
                           k->mass, p->N, dt);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}
