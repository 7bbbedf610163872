// k_forces.hip -- interaction-potential forces (Section 2.3 of Spandan et al.):
// per-body geometry reductions, per-edge spring + bending hinge, per-face area +
// volume-gradient, and the scatter-free gather of element results into nodes.
#include <cmath>
#include <mutex>
#include <string>

#include "elements.h"
#include "ipibm_internal.h"
#include "xcd.h"

namespace {

constexpr int kGeomThreads = 256;
constexpr int kElemThreads = 256;

// ----------------------------------------------------------------------------
// Per-body area A_b = sum |n_f|/2 and enclosed volume
// V_b = (1/6) sum_f (x_i - a).((x_j - a) x (x_k - a)), a = first node of the
// body (divergence theorem).  One workgroup per body; FP64 accumulation and a
// fixed-shape tree reduction (wave shuffles, then LDS), so the result does not
// depend on scheduling.
// ----------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kGeomThreads) void k_geometry(
    const double *__restrict__ X, const int32_t *__restrict__ faces,
    const int64_t *__restrict__ node_off, const int64_t *__restrict__ face_off,
    double *__restrict__ V, double *__restrict__ A, const int32_t *__restrict__ bodies) {
    __shared__ double sh[kGeomThreads / 64];
    const int b = bodies ? bodies[blockIdx.x] : (int)blockIdx.x;
    if (face_off[b] == face_off[b + 1]) {   // no faces: the body may own no node
        if (threadIdx.x == 0) V[b] = A[b] = 0.0;
        return;
    }
    const vec3<double> a = ldX(X, node_off[b]);
    double vs = 0.0, as = 0.0;
    for (int64_t f = face_off[b] + threadIdx.x; f < face_off[b + 1]; f += blockDim.x) {
        const int32_t *t = faces + 3 * f;
        double v6, a2;
        face_geometry<double, R>(ldX(X, t[0]), ldX(X, t[1]), ldX(X, t[2]), a, v6, a2);
        vs += v6;
        as += a2;
    }
    vs = block_sum(vs, sh);
    as = block_sum(as, sh);
    if (threadIdx.x == 0) {
        V[b] = vs * (1.0 / 6.0);
        A[b] = 0.5 * as;
    }
}

// ----------------------------------------------------------------------------
// Reference state: l0 per edge, (cos, sin) of the signed dihedral per edge,
// A0 per face.  Computed in FP64 and rounded once to R.
// ----------------------------------------------------------------------------
template <typename R>
__global__ void k_reference_edges(const double *__restrict__ X, const int4 *__restrict__ e4,
                                  int64_t E, R *__restrict__ l0, R *__restrict__ cs0) {
    const int64_t e = xcd_block() * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int4 q = e4[e];
    const vec3<double> x1 = ldX(X, q.x), x2 = ldX(X, q.y);
    const vec3<double> ev = x2 - x1;
    const double le = sqrt(dot(ev, ev));
    l0[e] = (R)le;
    double c = 1.0, s = 0.0;
    if (q.z >= 0 && q.w >= 0) {
        const vec3<double> nA = cross(ev, ldX(X, q.z) - x1);
        const vec3<double> nB = cross(ldX(X, q.w) - x1, ev);
        const double inv = 1.0 / sqrt(dot(nA, nA) * dot(nB, nB));
        c = dot(nA, nB) * inv;
        s = dot(cross(nA, nB), ev) * inv / le;
    }
    cs0[2 * e] = (R)c;
    cs0[2 * e + 1] = (R)s;
}

template <typename R>
__global__ void k_reference_faces(const double *__restrict__ X, const int32_t *__restrict__ faces,
                                  int64_t F, R *__restrict__ A0) {
    const int64_t f = xcd_block() * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int32_t *t = faces + 3 * f;
    const vec3<double> xi = ldX(X, t[0]);
    const vec3<double> n = cross(ldX(X, t[1]) - xi, ldX(X, t[2]) - xi);
    A0[f] = (R)(0.5 * sqrt(dot(n, n)));
}

// ----------------------------------------------------------------------------
// Edge elements (spring + bending hinge, see edge_forces): 4 slot vectors per
// edge, the forces on v1..v4.
// ----------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kElemThreads) void k_edges(
    const double *__restrict__ X, const int4 *__restrict__ e4,
    const int64_t *__restrict__ edge_off, int B, int64_t E, const R *__restrict__ l0,
    const R *__restrict__ cs0, const double *__restrict__ ks, const double *__restrict__ kb,
    const double *__restrict__ ew, R *__restrict__ slots, uint32_t *__restrict__ status) {
    const int64_t e = xcd_block() * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int b = body_of(edge_off, B, e);
    const double kse = ew ? ks[b] * ew[2 * e] : ks[b];
    const double kbe = ew ? kb[b] * ew[2 * e + 1] : kb[b];
    const int4 q = e4[e];
    const vec3<double> x1 = ldX(X, q.x), x2 = ldX(X, q.y);
    vec3<double> x3, x4;
    const bool hinge = q.z >= 0 && q.w >= 0;
    if (hinge) {
        x3 = ldX(X, q.z);
        x4 = ldX(X, q.w);
    }
    vec3<R> f1, f2, f3, f4;
    const bool bad = edge_forces<double, R>(x1, x2, x3, x4, hinge, l0[e],
                                    cs0[2 * e], cs0[2 * e + 1], kse, kbe, f1, f2, f3, f4);
    if (bad) atomicOr(status, IP_STATUS_DEGENERATE);
    R *o = slots + 12 * e;
    o[0] = f1.x; o[1] = f1.y; o[2] = f1.z;
    o[3] = f2.x; o[4] = f2.y; o[5] = f2.z;
    o[6] = f3.x; o[7] = f3.y; o[8] = f3.z;
    o[9] = f4.x; o[10] = f4.y; o[11] = f4.z;
}

// ----------------------------------------------------------------------------
// Face elements (area + volume, see face_forces): 3 slot vectors per face, the
// forces on its corners.  V from k_geometry.
// ----------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kElemThreads) void k_faces(
    const double *__restrict__ X, const int32_t *__restrict__ faces,
    const int64_t *__restrict__ face_off, int B, int64_t F, const R *__restrict__ A0,
    const double *__restrict__ V0, const double *__restrict__ Vcur,
    const uint8_t *__restrict__ closed, const double *__restrict__ kA,
    const double *__restrict__ kV, R *__restrict__ slots, uint32_t *__restrict__ status) {
    const int64_t f = xcd_block() * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int b = body_of(face_off, B, f);
    const int32_t *t = faces + 3 * f;
    const R sV = volume_coefficient<R>(closed[b] != 0, kV[b], Vcur[b], V0[b]);
    vec3<R> gi, gj, gk;
    if (face_forces<double, R>(ldX(X, t[0]), ldX(X, t[1]), ldX(X, t[2]), A0[f], kA[b], sV, gi, gj, gk))
        atomicOr(status, IP_STATUS_DEGENERATE);
    R *o = slots + 9 * f;
    o[0] = gi.x; o[1] = gi.y; o[2] = gi.z;
    o[3] = gj.x; o[4] = gj.y; o[5] = gj.z;
    o[6] = gk.x; o[7] = gk.y; o[8] = gk.z;
}

// ----------------------------------------------------------------------------
// Node gather: F_i = sum of the node's element slots, in ascending slot order
// (deterministic, no atomics).
// ----------------------------------------------------------------------------
template <typename R>
__global__ void k_gather(const int32_t *__restrict__ ptr, const int32_t *__restrict__ slot_ids,
                         const R *__restrict__ slots, int64_t N, R *__restrict__ F,
                         uint32_t *__restrict__ status) {
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= N) return;
    R fx = 0, fy = 0, fz = 0;
    for (int32_t s = ptr[i]; s < ptr[i + 1]; ++s) {
        const R *v = slots + 3 * (int64_t)slot_ids[s];
        fx += v[0];
        fy += v[1];
        fz += v[2];
    }
    if (!isfinite(fx) || !isfinite(fy) || !isfinite(fz)) atomicOr(status, IP_STATUS_NONFINITE);
    F[3 * i] = fx;
    F[3 * i + 1] = fy;
    F[3 * i + 2] = fz;
}

// ----------------------------------------------------------------------------
// Per-body energies W[b][4] = (spring, bending, area, volume); one workgroup
// per body, evaluated and accumulated in FP64 for every plan precision (the
// energies are diagnostics, off the step).  Only launched when W is requested.
// ----------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kGeomThreads) void k_energy(
    const double *__restrict__ X, const int4 *__restrict__ e4, const int32_t *__restrict__ faces,
    const int64_t *__restrict__ edge_off, const int64_t *__restrict__ face_off,
    const R *__restrict__ l0, const R *__restrict__ cs0, const R *__restrict__ A0,
    const double *__restrict__ V0, const double *__restrict__ Vcur,
    const uint8_t *__restrict__ closed, const double *__restrict__ ks,
    const double *__restrict__ kb, const double *__restrict__ kA,
    const double *__restrict__ kV, const double *__restrict__ ew, double *__restrict__ W) {
    __shared__ double sh[kGeomThreads / 64];
    const int b = blockIdx.x;
    double ws = 0.0, wb = 0.0, wa = 0.0;
    for (int64_t e = edge_off[b] + threadIdx.x; e < edge_off[b + 1]; e += blockDim.x) {
        const int4 q = e4[e];
        const vec3<double> x1 = ldX(X, q.x);
        const vec3<double> ev = ldX(X, q.y) - x1;
        const double dl = sqrt(dot(ev, ev)) - (double)l0[e];
        ws += (ew ? ew[2 * e] : 1.0) * dl * dl;
        if (q.z >= 0 && q.w >= 0) {
            const vec3<double> nA = cross(ev, ldX(X, q.z) - x1);
            const vec3<double> nB = cross(ldX(X, q.w) - x1, ev);
            const double inv = 1.0 / sqrt(dot(nA, nA) * dot(nB, nB));
            const double cth = dot(nA, nB) * inv;
            const double sth = dot(cross(nA, nB), ev) * inv / sqrt(dot(ev, ev));
            // cos and sin of theta - theta0 (the stored pair renormalised, which
            // matters once it has been rounded to FP32); 1 - cos d = sin^2 d /
            // (1 + cos d) avoids the cancellation near the reference state
            const double c0 = (double)cs0[2 * e], s0 = (double)cs0[2 * e + 1];
            const double r0 = 1.0 / sqrt(c0 * c0 + s0 * s0);
            const double cd = (cth * c0 + sth * s0) * r0, sd = (sth * c0 - cth * s0) * r0;
            wb += (ew ? ew[2 * e + 1] : 1.0) * (cd > 0.0 ? sd * sd / (1.0 + cd) : 1.0 - cd);
        }
    }
    for (int64_t f = face_off[b] + threadIdx.x; f < face_off[b + 1]; f += blockDim.x) {
        const int32_t *t = faces + 3 * f;
        const vec3<double> xi = ldX(X, t[0]);
        const vec3<double> n = cross(ldX(X, t[1]) - xi, ldX(X, t[2]) - xi);
        const double a0 = (double)A0[f];
        const double da = 0.5 * sqrt(dot(n, n)) - a0;
        wa += da * da / a0;
    }
    ws = block_sum(ws, sh);
    wb = block_sum(wb, sh);
    wa = block_sum(wa, sh);
    if (threadIdx.x == 0) {
        double wv = 0.0;
        if (closed[b]) {
            const double dv = Vcur[b] - V0[b];
            wv = 0.5 * kV[b] * dv * dv / V0[b];
        }
        W[4 * b + 0] = 0.5 * ks[b] * ws;
        W[4 * b + 1] = kb[b] * wb;
        W[4 * b + 2] = 0.5 * kA[b] * wa;
        W[4 * b + 3] = wv;
    }
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// slots: element-slot workspace, [(4E + 3F)][3] R; Vb, Ab: [B] doubles
template <typename R>
ip_status forces_impl(ip_plan *p, const double *X, const ip_reference *ref,
                      const ip_constants *k, void *Fv, double *Vb, double *Ab, double *W,
                      R *slots, hipStream_t s) {
    if (p->B > 0)
        hipLaunchKernelGGL(k_geometry<R>, dim3(p->B), dim3(kGeomThreads), 0, s, X, p->faces,
                           p->node_off, p->face_off, Vb, Ab, (const int32_t *)nullptr);
    if (p->E > 0)
        hipLaunchKernelGGL(k_edges<R>, dim3(nblocks(p->E, kElemThreads)), dim3(kElemThreads), 0,
                           s, X, (const int4 *)p->edges4, p->edge_off, p->B, p->E,
                           (const R *)ref->l0, (const R *)ref->cs0, k->ks, k->kb, p->ew, slots,
                           p->status);
    if (p->F > 0)
        hipLaunchKernelGGL(k_faces<R>, dim3(nblocks(p->F, kElemThreads)), dim3(kElemThreads), 0,
                           s, X, p->faces, p->face_off, p->B, p->F,
                           (const R *)ref->A0, ref->V0, Vb, p->closed, k->kA, k->kV,
                           slots + 12 * p->E, p->status);
    if (p->N > 0)
        hipLaunchKernelGGL(k_gather<R>, dim3(nblocks(p->N, 256)), dim3(256), 0, s, p->csr_ptr,
                           p->csr_slot, slots, p->N, (R *)Fv, p->status);
    if (W && p->B > 0)
        hipLaunchKernelGGL(k_energy<R>, dim3(p->B), dim3(kGeomThreads), 0, s, X,
                           (const int4 *)p->edges4, p->faces, p->edge_off, p->face_off,
                           (const R *)ref->l0, (const R *)ref->cs0, (const R *)ref->A0, ref->V0,
                           Vb, p->closed, k->ks, k->kb, k->kA, k->kV, p->ew, W);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

template <typename R>
ip_status reference_impl(ip_plan *p, const double *X, void *l0, void *cs0, void *A0,
                         hipStream_t s) {
    if (p->E > 0)
        hipLaunchKernelGGL(k_reference_edges<R>, dim3(nblocks(p->E, 256)), dim3(256), 0, s, X,
                           (const int4 *)p->edges4, p->E, (R *)l0, (R *)cs0);
    if (p->F > 0)
        hipLaunchKernelGGL(k_reference_faces<R>, dim3(nblocks(p->F, 256)), dim3(256), 0, s, X,
                           p->faces, p->F, (R *)A0);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

// Per-edge weights: checked (finite, non-negative), copied in the caller's
// edge order and gathered into the record order of the fused kernels.
__global__ void k_clear_flag(int32_t *flag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0;
}

__global__ __launch_bounds__(256) void k_copy_weights(const double *__restrict__ src, int64_t E,
                                                      double *__restrict__ dst,
                                                      int32_t *__restrict__ bad) {
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= 2 * E) return;
    const double w = src[i];
    if (!(w >= 0.0) || !isfinite(w)) atomicOr(bad, 1);
    dst[i] = w;
}

__global__ __launch_bounds__(256) void k_gather_weights(const double2 *__restrict__ ew,
                                                        const int32_t *__restrict__ perm,
                                                        int64_t n, double2 *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) out[r] = ew[perm[r]];
}

}  // namespace

ip_status launch_bind_edge_weights(ip_plan *p, const double *ew, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, s, p->ew_bad);
    if (p->E > 0)
        hipLaunchKernelGGL(k_copy_weights, dim3(nblocks(2 * p->E, 256)), dim3(256), 0, s, ew,
                           p->E, p->ew_store, p->ew_bad);
    if (p->n_erec > 0)
        hipLaunchKernelGGL(k_gather_weights, dim3(nblocks(p->n_erec, 256)), dim3(256), 0, s,
                           (const double2 *)p->ew_store, p->erec_perm, p->n_erec,
                           (double2 *)p->ew_rec_store);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

ip_status launch_geometry(ip_plan *p, const double *X, double *V, double *A, hipStream_t s,
                          const int32_t *bodies, int n_bodies) {
    const int nb = bodies ? n_bodies : p->B;
    if (nb <= 0) return IP_OK;
    if (p->prec == IP_F64)
        hipLaunchKernelGGL(k_geometry<double>, dim3(nb), dim3(kGeomThreads), 0, s, X, p->faces,
                           p->node_off, p->face_off, V, A, bodies);
    else
        hipLaunchKernelGGL(k_geometry<float>, dim3(nb), dim3(kGeomThreads), 0, s, X, p->faces,
                           p->node_off, p->face_off, V, A, bodies);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

ip_status launch_reference(ip_plan *p, const double *Xref, void *l0, void *cs0, void *A0,
                           hipStream_t s) {
    return p->prec == IP_F64 ? reference_impl<double>(p, Xref, l0, cs0, A0, s)
                             : reference_impl<float>(p, Xref, l0, cs0, A0, s);
}

ip_status launch_forces(ip_plan *p, const double *X, const ip_reference *ref,
                        const ip_constants *k, void *F, double *V, double *A, double *W,
                        hipStream_t s) {
    double *Vb = V ? V : p->Vbuf;
    double *Ab = A ? A : p->Abuf;
    return p->prec == IP_F64
               ? forces_impl<double>(p, X, ref, k, F, Vb, Ab, W, (double *)p->slots, s)
               : forces_impl<float>(p, X, ref, k, F, Vb, Ab, W, (float *)p->slots, s);
}

// ----------------------------------------------------------------------------
// ip_forces_noalloc: the same kernels with their workspace (the element slots,
// and V, A when the caller passes none) in a static device array instead of
// the plan's allocations, for callers that cannot allocate.  Each device holds
// its own copy of the array for the life of the process; its address on a
// device is looked up once, at the first plan creation on that device, and
// only that address reaches kernels.  Every slot, V and A entry is written
// before it is read, so nothing needs clearing between calls.
// ----------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

size_t align_up(size_t n, size_t a) { return (n + a - 1) / a * a; }
}  // namespace

ip_status prepare_noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) {
        ipibm_set_error("device id " + std::to_string(device) + " beyond the scratch table");
        return IP_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return IP_OK;
    void *ptr = nullptr;
    IP_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
        ipibm_set_error("hipGetSymbolAddress returned no address for the static scratch");
        return IP_ERR_HIP;
    }
    g_scratch_ptr[device] = ptr;
    return IP_OK;
}

size_t noalloc_scratch_need(const ip_plan *p) {
    return align_up((size_t)p->B * 2 * sizeof(double), 256) +
           (size_t)(4 * p->E + 3 * p->F) * 3 * p->real_size();
}

ip_status launch_forces_noalloc(ip_plan *p, const double *X, const ip_reference *ref,
                                const ip_constants *k, void *F, double *V, double *A,
                                double *W, hipStream_t s) {
    const size_t need = noalloc_scratch_need(p);
    if (need > (size_t)kNoAllocScratchBytes) {
        ipibm_set_error("ip_forces_noalloc: the plan needs " + std::to_string(need) +
                        " bytes of scratch, more than the " +
                        std::to_string((size_t)kNoAllocScratchBytes) +
                        " bytes of the static array (use ip_forces)");
        return IP_ERR_ARG;
    }
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (p->device >= 0 && p->device < kMaxDevices) base = g_scratch_ptr[p->device];
    }
    if (!base) {
        ipibm_set_error("ip_forces_noalloc: no static scratch address for device " +
                        std::to_string(p->device));
        return IP_ERR_UNSUPPORTED;
    }
    double *Vb = V ? V : (double *)base;
    double *Ab = A ? A : (double *)base + p->B;
    void *slots = (unsigned char *)base + align_up((size_t)p->B * 2 * sizeof(double), 256);
    return p->prec == IP_F64
               ? forces_impl<double>(p, X, ref, k, F, Vb, Ab, W, (double *)slots, s)
               : forces_impl<float>(p, X, ref, k, F, Vb, Ab, W, (float *)slots, s);
}
