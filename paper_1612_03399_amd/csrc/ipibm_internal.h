// ipibm_internal.h -- plan object and device helpers shared by the HIP sources
// of libipibm (gfx950).  Not part of the public C-ABI (include/ipibm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ipibm.h"

// ----------------------------------------------------------------------------
// error plumbing
// ----------------------------------------------------------------------------
void ipibm_set_error(const std::string &msg);

// Return the status of `expr` if it is not IP_OK.
#define IP_TRY(expr)                        \
    do {                                    \
        ip_status st_ = (expr);             \
        if (st_ != IP_OK) return st_;       \
    } while (0)

#define IP_HIP_CHECK(expr)                                                        \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ipibm_set_error(std::string(#expr) + ": " + hipGetErrorString(e_));   \
            return IP_ERR_HIP;                                                    \
        }                                                                         \
    } while (0)

// ----------------------------------------------------------------------------
// plan
// ----------------------------------------------------------------------------
struct ip_plan {
    int32_t B = 0;
    int64_t N = 0, E = 0, F = 0;
    ip_precision prec = IP_F64;
    bool has_grid = false;
    ip_grid grid{};
    int device = 0;

    std::vector<int64_t> h_node_off, h_edge_off, h_face_off;

    // device copies of the mesh
    int64_t *node_off = nullptr, *edge_off = nullptr, *face_off = nullptr;
    int32_t *faces = nullptr;    // [F][3]
    int32_t *edges4 = nullptr;   // [E][4]
    uint8_t *closed = nullptr;   // [B]
    uint8_t *pinned = nullptr;   // [N]

    // node <- element-slot gather lists (CSR), slot id = 4 e + role for edges,
    // 4 E + 3 f + corner for faces
    int32_t *csr_ptr = nullptr;   // [N+1]
    int32_t *csr_slot = nullptr;  // [csr_ptr[N]]

    // workspace
    void *slots = nullptr;        // [(4E + 3F)][3] real
    void *Fbuf = nullptr;         // [N][3] real
    void *Ubuf = nullptr;         // [N][3] real
    double *Vbuf = nullptr;       // [B]
    double *Abuf = nullptr;       // [B]
    uint32_t *status = nullptr;   // device status word

    // fused step: one workgroup per work unit (a whole body, or a patch of a
    // larger one: owned nodes plus the halo its elements reach)
    bool fused_all = false;
    int fused_nmax = 0;           // largest work unit (nodes, owned + halo)
    int fused_tile_bytes = 0;     // LDS bytes for the grid tile (first launch class)
    int lds_optin = 0;            // LDS bytes one workgroup may use on this device
    int step_threads = 768;       // threads per workgroup (first launch class)
    // launch classes of the fused step: consecutive ranges of the units
    // (largest first), each with its own workgroup size and LDS layout
    struct StepClass {
        int32_t unit_begin = 0, unit_end = 0;
        int threads = 768, nmax = 0, tile_bytes = 0;
    };
    StepClass step_class[2];
    int n_step_classes = 0;
    int32_t n_units = 0;
    int32_t *wu_body = nullptr;   // [n_units] body of each unit, largest unit first
    int32_t *wu_owned = nullptr;  // [n_units] owned nodes
    uint8_t *wu_pinned = nullptr; // [n_units] 1 = some node of the unit is pinned
    int64_t *wu_noff = nullptr;   // [n_units][2] node-list range (empty: whole body)
    int32_t *wu_nodes = nullptr;  // global ids of patch nodes, owned first
    int64_t *wu_eoff = nullptr;   // [n_units][2] edge-record range
    int64_t *wu_foff = nullptr;   // [n_units][2] face-record range
    int64_t n_erec = 0, n_frec = 0;
    int32_t *erec_perm = nullptr; // [n_erec] edge id of each record
    uint16_t *erec_lid = nullptr; // [n_erec][4] unit-local node ids (kNoNode: none)
    int32_t *frec_perm = nullptr; // [n_frec] face id of each record
    uint16_t *frec_lid = nullptr; // [n_frec][4] unit-local node ids, last unused
    void *edge_rec = nullptr;     // [n_erec] EdgeRec<real>
    void *face_rec = nullptr;     // [n_frec] FaceRec<real>
    int packed = 0;               // records hold: 0 nothing, 1 the bound reference,
                                  // 2 the last explicit reference
    int32_t n_patched_bodies = 0;
    int32_t *patched_bodies = nullptr;  // bodies split into patches
    int32_t n_patched_units = 0;
    int32_t *patched_units = nullptr;   // their units
    double *Xstage = nullptr;     // [N][3] new positions of patched bodies

    double *bwd_dots = nullptr;   // [2E + 2F] family dot products (reverse step)

    // per-edge weights on ks and kb (ip_plan_bind_edge_weights); NULL while
    // none are bound (every weight 1)
    double *ew = nullptr;         // [E][2] caller's edge order (element kernels)
    double *ew_rec = nullptr;     // [n_erec][2] record order (fused kernels)
    double *ew_store = nullptr;   // storage behind ew, kept across unbinding
    double *ew_rec_store = nullptr;
    int32_t *ew_bad = nullptr;    // device flag: an invalid weight was seen

    // bound reference (ip_plan_bind_reference): copies in the caller's
    // element order (element kernels; source of the packed records)
    bool ref_bound = false;
    void *bref_l0 = nullptr, *bref_cs0 = nullptr, *bref_A0 = nullptr;  // real, caller order
    double *bref_V0 = nullptr;
    ip_reference bref{};

    size_t real_size() const { return prec == IP_F64 ? sizeof(double) : sizeof(float); }
};

// Packed element records of a bound reference: node ids local to the body
// (0xFFFF = no wing) with the element's reference values, one or two vector
// loads per element.
constexpr uint16_t kNoNode = 0xFFFF;
template <typename R>
struct EdgeRec;
template <>
struct alignas(16) EdgeRec<double> {
    uint16_t v[4];
    double l0, c0, s0;
};
template <>
struct alignas(8) EdgeRec<float> {
    uint16_t v[4];
    float l0, c0, s0, pad;
};
template <typename R>
struct alignas(16) FaceRec {
    uint16_t v[3], pad;
    R a0;
};
static_assert(sizeof(EdgeRec<double>) == 32 && sizeof(EdgeRec<float>) == 24, "edge record");
static_assert(sizeof(FaceRec<double>) == 16 && sizeof(FaceRec<float>) == 16, "face record");

// Work units of the fused step (workunits.hip).
struct WorkUnitHost {
    int32_t body = 0, owned = 0, n_nodes = 0;
    int64_t node_begin = 0, node_end = 0, edge_begin = 0, edge_end = 0, face_begin = 0,
            face_end = 0;
};
struct WorkUnits {
    std::vector<WorkUnitHost> units;
    std::vector<int32_t> nodes, edge_perm, face_perm;
    std::vector<uint16_t> edge_lid, face_lid;
};
// Bodies of at most whole_max nodes and fmax_unit faces become one unit;
// larger bodies are split into patches of at most patch_owned owned nodes
// (further where a patch with its halo would exceed nmax_unit nodes or
// fmax_unit faces).  False if some body cannot be split to fit.
bool build_work_units(const ip_mesh *m, int whole_max, int nmax_unit, int fmax_unit,
                      int patch_owned, WorkUnits &out);

// launchers (k_forces.hip / k_transfer.hip); all asynchronous on `s`
ip_status launch_geometry(ip_plan *p, const double *X, double *V, double *A, hipStream_t s,
                          const int32_t *bodies = nullptr, int n_bodies = -1);
ip_status launch_reference(ip_plan *p, const double *Xref, void *l0, void *cs0, void *A0,
                           hipStream_t s);
ip_status launch_forces(ip_plan *p, const double *X, const ip_reference *ref,
                        const ip_constants *k, void *F, double *V, double *A, double *W,
                        hipStream_t s);
ip_status launch_interp(ip_plan *p, const double *X, const void *u, void *U, hipStream_t s);
// ip_forces with its workspace in the static scratch array (k_forces.hip)
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
ip_status prepare_noalloc_scratch(int device);   // once per device, device current
size_t noalloc_scratch_need(const ip_plan *p);
ip_status launch_forces_noalloc(ip_plan *p, const double *X, const ip_reference *ref,
                                const ip_constants *k, void *F, double *V, double *A,
                                double *W, hipStream_t s);
ip_status launch_spread(ip_plan *p, const double *X, const void *F, void *f, hipStream_t s);
// MLS transfer at the triangle centroids (k_mls.hip)
ip_status launch_interp_mls(ip_plan *p, const double *X, const void *u, double alpha, void *U,
                            hipStream_t s);
ip_status launch_spread_mls(ip_plan *p, const double *X, const void *Fm, double alpha, void *f,
                            hipStream_t s);
ip_status launch_centroid_to_nodes(ip_plan *p, const void *Fc, void *Fn, hipStream_t s);
ip_status launch_probe_loads(ip_plan *p, const double *X, const void *u, const void *pr,
                             const void *acc, double alpha, double mu, void *Fext, hipStream_t s);
ip_status launch_direct_forcing_mls(ip_plan *p, const double *X, const void *Vb, const void *u,
                                    double alpha, double dt, void *Fout, void *f, hipStream_t s);
ip_status launch_update(ip_plan *p, double *X, const void *U, const void *F,
                        const ip_constants *k, double dt, hipStream_t s);

// derivatives (k_backward.hip), FP64 plans
ip_status launch_forces_jvp(ip_plan *p, const double *X, const double *T, const ip_reference *ref,
                            const ip_constants *k, const double *P, double *dF, double *dotE,
                            double *dotF, hipStream_t s);
ip_status launch_step_vjp(ip_plan *p, const double *X, const ip_reference *ref,
                          const ip_constants *k, const double *u, double dt,
                          const double *lam_in, double *lam_out, double *gk, double *gu,
                          hipStream_t s);
ip_status launch_interp_vjp(ip_plan *p, const double *X, const double *u, const double *dU,
                            double *gX, double *gu, hipStream_t s);
ip_status launch_taylor(ip_plan *p, const double *X, const double *Dstar, double *D, double *loss,
                        double *gX, hipStream_t s);

// fused step (k_step.hip)
constexpr int kStepThreads = 768;         // default threads per workgroup (also 384)
constexpr int kStepNodesPerThread = 4;
constexpr int kStepFacesPerThread = 8;   // faces held in registers per thread
constexpr int kPatchOwned = 512;         // owned nodes per patch of a large body
size_t step_fused_lds_bytes(int nmax, int tile_bytes);
ip_status prepare_step_fused(ip_plan *p);   // one-time launch attributes
ip_status prepare_mls_units(ip_plan *p);    // one-time launch attributes
ip_status launch_bind_edge_weights(ip_plan *p, const double *ew, hipStream_t s);
ip_status launch_pack_reference(ip_plan *p, const ip_reference *ref, hipStream_t s);
// the nodes of patched bodies: src -> dst ([N][3] double each)
ip_status launch_commit(ip_plan *p, const double *src, double *dst, hipStream_t s);
// fused reverse step (k_backward.hip), FP64 fused plans; records hold `ref`
ip_status launch_step_vjp_fused(ip_plan *p, const double *X, const ip_reference *ref,
                                const ip_constants *k, const double *u, double dt,
                                const double *lam_in, double *lam_out, double *gk, double *gu,
                                hipStream_t s);
ip_status prepare_step_vjp_fused(ip_plan *p);
ip_status launch_step_fused(ip_plan *p, double *X, const ip_reference *ref,
                            const ip_constants *k, const void *u, void *f, double dt,
                            double *V, double *A, hipStream_t s);

// ----------------------------------------------------------------------------
// device helpers
// ----------------------------------------------------------------------------
template <typename R>
struct vec3 {
    R x, y, z;
};

template <typename R>
__device__ __forceinline__ vec3<R> operator-(vec3<R> a, vec3<R> b) {
    return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <typename R>
__device__ __forceinline__ vec3<R> operator+(vec3<R> a, vec3<R> b) {
    return {a.x + b.x, a.y + b.y, a.z + b.z};
}
template <typename R>
__device__ __forceinline__ vec3<R> operator*(R s, vec3<R> a) {
    return {s * a.x, s * a.y, s * a.z};
}
template <typename R>
__device__ __forceinline__ R dot(vec3<R> a, vec3<R> b) {
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename R>
__device__ __forceinline__ vec3<R> cross(vec3<R> a, vec3<R> b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// difference of two FP64 points, rounded once to R
template <typename R>
__device__ __forceinline__ vec3<R> diffR(const vec3<double> &a, const vec3<double> &b) {
    return {(R)(a.x - b.x), (R)(a.y - b.y), (R)(a.z - b.z)};
}
__device__ __forceinline__ vec3<double> ldX(const double *X, int64_t i) {
    const double *p = X + 3 * i;
    return {p[0], p[1], p[2]};
}

// Index of the body owning element/node i: the last b with off[b] <= i.
__device__ __forceinline__ int body_of(const int64_t *off, int B, int64_t i) {
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the block; the result is valid in thread 0.  `sh` holds
// blockDim.x / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x < (blockDim.x >> 6)) r = sh[threadIdx.x];
    if (w == 0) r = wave_sum(r);
    return r;
}

// Reciprocal and reciprocal square root from the hardware estimates (about
// 2^-24 relative) refined by two Newton-Raphson steps each (quadratic
// convergence: ~1e-16, i.e. 1-3 ulp; measured 2.2e-16 and 3.0e-16 over
// [1e-6, 1e6]).  Valid for positive normal inputs; zero, infinite or NaN
// inputs propagate to non-finite results, which the callers flag.
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double rsq_nr(double x) {
    double q = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    q = q * fma(-h * q, q, 1.5);
    q = q * fma(-h * q, q, 1.5);
    return q;
}
// FP32: the hardware estimates are already within ~1 ulp
__device__ __forceinline__ float rcp_nr(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq_nr(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ int wrapi(int i, int n) {
    int m = i % n;
    return m < 0 ? m + n : m;
}

// Weights of the 3-point regularised delta (Roma, Peskin & Berger) at the three
// lattice points nearest to the fractional lattice coordinate s: c = floor(s+1/2),
// r = s - c in [-1/2, 1/2], q = sqrt(1 - 3 r^2):
//   w[0] (point c-1) = (2 - 3r - q)/6, w[1] (point c) = (1 + q)/3,
//   w[2] (point c+1) = (2 + 3r - q)/6.
// Returns c.
template <typename R>
__device__ __forceinline__ int delta3(double s, R w[3]) {
    double c = floor(s + 0.5);
    if (!(fabs(c) < 1.0e9)) c = 0.0;   // non-finite or absurd position: stay in bounds
    const R r = (R)(s - c);
    const R v = (R)1 - (R)3 * r * r;          // in [1/4, 1]
    const R q = v * rsq_nr(v);
    w[0] = ((R)2 - (R)3 * r - q) * (R)(1.0 / 6.0);
    w[1] = ((R)1 + q) * (R)(1.0 / 3.0);
    w[2] = ((R)2 + (R)3 * r - q) * (R)(1.0 / 6.0);
    return (int)c;
}

// MAC lattice offsets (cells): lattice d has offset 0 along axis d, 1/2 along
// the two others.
__device__ __forceinline__ double mac_off(int d, int axis) { return d == axis ? 0.0 : 0.5; }
