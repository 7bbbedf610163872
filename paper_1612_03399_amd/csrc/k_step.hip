// k_step.hip -- the fused explicit step, one workgroup per body.
//
// LDS (per workgroup): positions xs[N][3] (FP64), force accumulators
// Fs[N][3] (FP64 for every plan precision: FP32 LDS atomics are an order of
// magnitude slower than FP64 ones on gfx950), a tile region for the cell
// histogram and the per-lattice grid tiles, and the occupied-cell list.
//
// Phases (every body is independent; no inter-workgroup communication except
// the additions into the grid force field):
//  P0  positions -> LDS and owner registers; cell bounding box (the per-marker
//      cell index and the body bounding box of Section 5).
//  P1  enclosed volume and area of the body (FP64 block reduction).
//  P2  face (area + volume) and edge (spring + hinge) elements, their forces
//      added into the node accumulators (ds_add_f64).  Element data for the
//      next iteration is loaded while the current one is computed.
//  P3  counting sort of the nodes by Eulerian cell; xs and Fs are permuted in
//      place into cell order so each occupied cell's nodes are contiguous.
//  P4  spreading, per lattice: each occupied cell sums its nodes' force-
//      weighted stencils in registers over the cell's 4x3x3 block, adds the
//      block to an FP64 LDS tile, and the tile's non-zero points are added to
//      the grid with device atomics.
//  P5  per lattice d: the velocity tile is staged in LDS, every node
//      interpolates U_d from its 27-point stencil and writes
//      X_d + dt U_d + dt^2/m F_d (nodes that are not pinned).
// Bodies whose tile does not fit the tile region interpolate and spread
// directly against the grid (same arithmetic, global atomics).
#include <climits>

#include "elements.h"
#include "ipibm_internal.h"

namespace {

constexpr int K = kStepNodesPerThread;
constexpr int kCountBins = 32;     // occupied cells are ordered by node count (capped)
constexpr int FK = kStepFacesPerThread;

struct StepArgs {
    double *X;
    double *Xstage;          // new positions of patched bodies
    const int64_t *node_off;
    const uint8_t *closed, *pinned;
    const double *V0, *ks, *kb, *kA, *kV, *mass;
    const void *u;
    void *f;
    int nx, ny, nz;
    double inv_h, inv_h3;
    int64_t plane, field;
    double dt;
    double *V, *A;
    uint32_t *status;
    // work units (one per workgroup, largest first)
    const int32_t *wu_body, *wu_owned, *wu_nodes;
    const int64_t *wu_noff, *wu_eoff, *wu_foff;
    const void *erec, *frec; // packed element records
    int unit_base;           // unit of workgroup 0 of this launch
    int nmax;                // node capacity of the LDS layout
    int tile_bytes;          // bytes of the tile region
};

__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ vec3<double> ldx(const double *xs, int i) {
    return {xs[3 * i], xs[3 * i + 1], xs[3 * i + 2]};
}

template <typename R>
__device__ __forceinline__ void add3(double *F, int i, const vec3<R> &v) {
    lds_add(F + 3 * i, (double)v.x);
    lds_add(F + 3 * i + 1, (double)v.y);
    lds_add(F + 3 * i + 2, (double)v.z);
}

// Cell of a coordinate: the stencil centre of the lattices staggered by half a
// cell along this axis, computed with exactly the expression delta3() uses.
__device__ __forceinline__ int cell_of(double x, double inv_h) {
    double c = floor((x * inv_h - 0.5) + 0.5);
    if (!(fabs(c) < 1.0e9)) c = 0.0;
    return (int)c;
}

// Block-wide minimum / maximum of an int (every thread gets the result).
template <int NT, bool MAX>
__device__ __forceinline__ int block_extreme_int(int v, int *sh) {
    const auto pick = [](int x, int y) { return MAX ? max(x, y) : min(x, y); };
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = pick(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = sh[0];
    for (int w = 1; w < NT / 64; ++w) r = pick(r, sh[w]);
    return r;
}

template <int NT>
__device__ __forceinline__ int block_min_int(int v, int *sh) { return block_extreme_int<NT, false>(v, sh); }
template <int NT>
__device__ __forceinline__ int block_max_int(int v, int *sh) { return block_extreme_int<NT, true>(v, sh); }

// In-place exclusive scan of a[0..n) by the whole block; returns the total.
template <int NT>
__device__ int block_exclusive_scan(int *a, int n, int *sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int chunk = (n + NT - 1) / NT;
    const int lo = min(tid * chunk, n), hi = min(lo + chunk, n);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += a[i];
    int incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    __syncthreads();
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < NT / 64; ++w) {
        if (w < wave) before += sh[w];
        total += sh[w];
    }
    int run = before + incl - s;
    for (int i = lo; i < hi; ++i) {
        const int v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

// Copy n values from global memory to LDS, U loads in flight per thread.
template <int NT, typename T, int U = 8>
__device__ __forceinline__ void copy_to_lds(T *__restrict__ dst, const T *__restrict__ src, int n) {
    for (int base = 0; base < n; base += NT * U) {
        T v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = base + k * NT + (int)threadIdx.x;
            v[k] = i < n ? src[i] : (T)0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = base + k * NT + (int)threadIdx.x;
            if (i < n) dst[i] = v[k];
        }
    }
}

struct TileGeom {
    int kmin[3];            // lowest occupied cell per axis
    int Tx, Ty, Tz, T;      // the tile spans points kmin-1 .. kmax+2
    int nx, ny, nz;
    int64_t plane;
    __device__ __forceinline__ int64_t grid_index(int t) const {
        const int tx = t % Tx, ty = (t / Tx) % Ty, tz = t / (Tx * Ty);
        return wrapi(kmin[2] - 1 + tz, nz) * plane + (int64_t)wrapi(kmin[1] - 1 + ty, ny) * nx +
               wrapi(kmin[0] - 1 + tx, nx);
    }
};

// Stage the tile of one grid field into LDS, U loads in flight per thread.
template <int NT, typename R, int U = 8>
__device__ __forceinline__ void stage_tile(R *__restrict__ tile, const R *__restrict__ field,
                                           const TileGeom &g) {
    for (int base = 0; base < g.T; base += NT * U) {
        R v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int t = base + k * NT + (int)threadIdx.x;
            v[k] = t < g.T ? field[g.grid_index(t)] : (R)0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int t = base + k * NT + (int)threadIdx.x;
            if (t < g.T) tile[t] = v[k];
        }
    }
}

template <int D>
struct BlockDims {
    static constexpr int LX = D == 0 ? 4 : 3;
    static constexpr int LY = D == 1 ? 4 : 3;
    static constexpr int LZ = D == 2 ? 4 : 3;
};

// Spread the (cell-contiguous) nodes p0..p1 of one cell on lattice D into the
// LDS tile: their force-weighted stencils are summed in registers over the
// cell's 4x3x3 block (4 points along the lattice's unstaggered axis, whose
// stencil centre may be the cell or the next one) and the block is added to
// the tile once.
template <typename R, int D>
__device__ __forceinline__ void spread_cell(const double *xs, const double *Fs, int p0, int p1,
                                            const int kc[3], const int kmin[3], int Tx, int Ty,
                                            int T, double inv_h, double inv_h3, double *tile,
                                            bool &bad) {
    using Dm = BlockDims<D>;
    R acc[Dm::LZ][Dm::LY][Dm::LX];
#pragma unroll
    for (int z = 0; z < Dm::LZ; ++z)
#pragma unroll
        for (int y = 0; y < Dm::LY; ++y)
#pragma unroll
            for (int x = 0; x < Dm::LX; ++x) acc[z][y][x] = 0;
    for (int p = p0; p < p1; ++p) {
        R wx[4], wy[4], wz[4];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            R w3[3];
            const int c = delta3<R>(xs[3 * p + ax] * inv_h - mac_off(D, ax), w3);
            const int sh = c - kc[ax];
            R *w = ax == 0 ? wx : (ax == 1 ? wy : wz);
            if (ax == D) {
                const bool s1 = sh == 1;
                w[0] = s1 ? (R)0 : w3[0];
                w[1] = s1 ? w3[0] : w3[1];
                w[2] = s1 ? w3[1] : w3[2];
                w[3] = s1 ? w3[2] : (R)0;
                if (sh != 0 && sh != 1) bad = true;
            } else {
                w[0] = w3[0];
                w[1] = w3[1];
                w[2] = w3[2];
                if (sh != 0) bad = true;
            }
        }
        const R fd = (R)(Fs[3 * p + D] * inv_h3);
#pragma unroll
        for (int z = 0; z < Dm::LZ; ++z) {
            const R fz = fd * wz[z];
#pragma unroll
            for (int y = 0; y < Dm::LY; ++y) {
                const R fzy = fz * wy[y];
#pragma unroll
                for (int x = 0; x < Dm::LX; ++x) acc[z][y][x] += fzy * wx[x];
            }
        }
    }
    // block origin in tile coordinates: point k - 1 is tile index k - kmin
    const int ox = kc[0] - kmin[0], oy = kc[1] - kmin[1], oz = kc[2] - kmin[2];
#pragma unroll
    for (int z = 0; z < Dm::LZ; ++z)
#pragma unroll
        for (int y = 0; y < Dm::LY; ++y)
#pragma unroll
            for (int x = 0; x < Dm::LX; ++x) {
                const int t = ((oz + z) * Ty + (oy + y)) * Tx + (ox + x);
                if (acc[z][y][x] != (R)0 && t >= 0 && t < T) lds_add(tile + t, (double)acc[z][y][x]);
            }
}

// Raw packed records (vector loads) and their fields.
template <typename R>
struct RawEdge;
template <>
struct RawEdge<double> {
    int4 a, b;
    __device__ static RawEdge load(const void *base, int t) {
        const int4 *p = (const int4 *)base + 2 * (int64_t)t;
        return {p[0], p[1]};
    }
    __device__ int4 ids() const {
        return {a.x & 0xFFFF, (int)((unsigned)a.x >> 16), a.y & 0xFFFF, (int)((unsigned)a.y >> 16)};
    }
    __device__ double l0() const { return __hiloint2double(a.w, a.z); }
    __device__ double c0() const { return __hiloint2double(b.y, b.x); }
    __device__ double s0() const { return __hiloint2double(b.w, b.z); }
};
template <>
struct RawEdge<float> {
    int2 a, b, c;
    __device__ static RawEdge load(const void *base, int t) {
        const int2 *p = (const int2 *)base + 3 * (int64_t)t;
        return {p[0], p[1], p[2]};
    }
    __device__ int4 ids() const {
        return {a.x & 0xFFFF, (int)((unsigned)a.x >> 16), a.y & 0xFFFF, (int)((unsigned)a.y >> 16)};
    }
    __device__ float l0() const { return __int_as_float(b.x); }
    __device__ float c0() const { return __int_as_float(b.y); }
    __device__ float s0() const { return __int_as_float(c.x); }
};
__device__ __forceinline__ double face_a0(const int4 &r, double) { return __hiloint2double(r.w, r.z); }
__device__ __forceinline__ float face_a0(const int4 &r, float) { return __int_as_float(r.z); }

template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_step_fused(StepArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ double red[NT / 64];
    __shared__ int ired[NT / 64];
    __shared__ double bcd[1];
    __shared__ int n_occ_sh;
    __shared__ int cnt_bins[kCountBins + 1];

    const int tid = threadIdx.x;
    const int w = a.unit_base + (int)blockIdx.x;
    const int b = a.wu_body[w];
    const int64_t nl0 = a.wu_noff[2 * w], nl1 = a.wu_noff[2 * w + 1];
    const bool whole = nl1 == nl0;                    // a whole body, nodes contiguous
    const int64_t n0 = a.node_off[b];
    const int NL = whole ? (int)(a.node_off[b + 1] - n0) : (int)(nl1 - nl0);   // unit nodes
    const int N = whole ? NL : a.wu_owned[w];         // owned nodes (the first N)
    const int32_t *gid = a.wu_nodes + nl0;            // patch: global node ids
    const int64_t e0 = a.wu_eoff[2 * w];
    const int E = (int)(a.wu_eoff[2 * w + 1] - e0);
    const int64_t f0 = a.wu_foff[2 * w];
    const int F = (int)(a.wu_foff[2 * w + 1] - f0);
    if (NL == 0) {     // uniform over the block
        if (tid == 0) {
            a.V[b] = 0.0;
            a.A[b] = 0.0;
        }
        return;
    }

    double *xs = (double *)lds;                       // [nmax][3]
    double *Fs = xs + 3 * a.nmax;                     // [nmax][3]
    unsigned char *tile_region = (unsigned char *)(Fs + 3 * a.nmax);
    int *hist = (int *)tile_region;                   // P3: cell counts, then flags
    double *ftile = (double *)tile_region;            // P4: force tile (FP64)
    R *utile = (R *)tile_region;                      // P5: velocity tile
    uint16_t *occ_start = (uint16_t *)(tile_region + a.tile_bytes);  // [nmax] first node
    uint16_t *occ_cnt = occ_start + a.nmax;                           // [nmax] node count
    bool bad = false;

    // ---- faces of this thread (packed records: unit-local node ids and A0),
    // loaded first so that their latency overlaps the position copy; kept in
    // registers for P1 and P2.  The records are ordered so that each run of
    // 64 touches distinct nodes, and lane t takes record t. ----
    int fi[FK][3];
    R fa0[FK];
    unsigned fmask = 0;
#pragma unroll
    for (int s = 0; s < FK; ++s) {
        const int t = tid + s * NT;
        fi[s][0] = fi[s][1] = fi[s][2] = 0;
        fa0[s] = (R)1;
        if (t < F) {
            fmask |= 1u << s;
            const int4 r = ((const int4 *)a.frec)[f0 + t];
            fi[s][0] = r.x & 0xFFFF;
            fi[s][1] = (int)((unsigned)r.x >> 16);
            fi[s][2] = r.y & 0xFFFF;
            fa0[s] = face_a0(r, (R)0);
        }
    }

    // ---- P0: positions (contiguous for a whole body, gathered for a patch) ----
    if (whole) {
        copy_to_lds<NT>(xs, a.X + 3 * n0, 3 * NL);
    } else {
        for (int i = tid; i < NL; i += NT) {
            const int64_t g = gid[i];
            xs[3 * i] = a.X[3 * g];
            xs[3 * i + 1] = a.X[3 * g + 1];
            xs[3 * i + 2] = a.X[3 * g + 2];
        }
    }
    for (int i = tid; i < 3 * NL; i += NT) Fs[i] = 0.0;
    __syncthreads();
    // cell bounding box of the owned nodes (the ones spread and interpolated)
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int j = tid + s * NT;
        if (j < N) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int kc = cell_of(xs[3 * j + c], a.inv_h);
                lo[c] = min(lo[c], kc);
                hi[c] = max(hi[c], kc);
            }
        }
    }
    int kmin[3], kmax[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        kmin[c] = block_min_int<NT>(lo[c], ired);
        kmax[c] = block_max_int<NT>(hi[c], ired);
    }

    // ---- P1: volume and area (a whole body; a patched body's come from the
    // geometry pass that precedes this kernel) ----
    double Vb;
    if (whole) {
        const vec3<double> anchor = ldx(xs, 0);
        double v6 = 0.0, a2 = 0.0;
#pragma unroll
        for (int s = 0; s < FK; ++s) {
            if (fmask & (1u << s)) {
                double v, ar;
                face_geometry<double, R>(ldx(xs, fi[s][0]), ldx(xs, fi[s][1]), ldx(xs, fi[s][2]),
                                         anchor, v, ar);
                v6 += v;
                a2 += ar;
            }
        }
        v6 = block_sum(v6, red);
        a2 = block_sum(a2, red);
        if (tid == 0) {
            bcd[0] = v6 * (1.0 / 6.0);
            a.V[b] = bcd[0];
            a.A[b] = 0.5 * a2;
        }
        __syncthreads();
        Vb = bcd[0];
    } else {
        Vb = a.V[b];
    }

    // ---- P2: elements -> node accumulators ----
    {
        const R sV = volume_coefficient<R>(a.closed[b] != 0, a.kV[b], Vb, a.V0[b]);
        const double kA = a.kA[b];
#pragma unroll
        for (int s = 0; s < FK; ++s) {
            if (fmask & (1u << s)) {
                const int i = fi[s][0], j = fi[s][1], k = fi[s][2];
                vec3<R> gi, gj, gk;
                bad |= face_forces<double, R>(ldx(xs, i), ldx(xs, j), ldx(xs, k), fa0[s], kA, sV,
                                              gi, gj, gk);
                add3(Fs, i, gi);
                add3(Fs, j, gj);
                add3(Fs, k, gk);
            }
        }
        const double ks = a.ks[b], kb = a.kb[b];
        // edge records two iterations ahead; the next edge's node positions
        // are read before the current edge's accumulator additions are issued
        // (waiting for those reads never waits for the additions)
        using Raw = RawEdge<R>;
        const auto fetch = [&](int t) {
            Raw r{};
            if (t < E) r = Raw::load(a.erec, (int)e0 + t);
            return r;
        };
        const auto read_nodes = [&](const int4 &q, vec3<double> &y1, vec3<double> &y2,
                                    vec3<double> &y3, vec3<double> &y4) {
            const bool h = q.z != kNoNode && q.w != kNoNode;
            y1 = ldx(xs, q.x);
            y2 = ldx(xs, q.y);
            y3 = ldx(xs, h ? q.z : 0);
            y4 = ldx(xs, h ? q.w : 0);
        };
        Raw rc = fetch(tid), rn = fetch(tid + NT);
        vec3<double> x1, x2, x3, x4;
        if (tid < E) read_nodes(rc.ids(), x1, x2, x3, x4);
        for (int t = tid; t < E; t += NT) {
            const Raw cur = rc;
            rc = rn;
            rn = fetch(t + 2 * NT);
            const int4 q = cur.ids();
            const bool hinge = q.z != kNoNode && q.w != kNoNode;
            vec3<R> f1, f2, f3, f4;
            bad |= edge_forces<double, R>(x1, x2, x3, x4, hinge, cur.l0(), cur.c0(), cur.s0(), ks,
                                          kb, f1, f2, f3, f4);
            if (t + NT < E) read_nodes(rc.ids(), x1, x2, x3, x4);
            add3(Fs, q.x, f1);
            add3(Fs, q.y, f2);
            if (hinge) {
                add3(Fs, q.z, f3);
                add3(Fs, q.w, f4);
            }
        }
    }
    __syncthreads();

    // ---- P3: counting sort by cell; permute xs and Fs into cell order ----
    const int Cx = kmax[0] - kmin[0] + 1, Cy = kmax[1] - kmin[1] + 1, Cz = kmax[2] - kmin[2] + 1;
    const int Tx = Cx + 3, Ty = Cy + 3, Tz = Cz + 3;    // points kmin-1 .. kmax+2
    const long long Cl = (long long)Cx * Cy * Cz, Tl = (long long)Tx * Ty * Tz;
    const bool use_tile = Cx >= 1 && Cy >= 1 && Cz >= 1 && Cl <= 65535 && Cl * 8 <= a.tile_bytes &&
                          Tl * 8 <= a.tile_bytes;
    const int C = use_tile ? (int)Cl : 0, T = use_tile ? (int)Tl : 0;
    int pos[K];
#pragma unroll
    for (int s = 0; s < K; ++s) pos[s] = tid + s * NT;     // identity unless sorted
    if (use_tile) {
        for (int c = tid; c < C; c += NT) hist[c] = 0;
        __syncthreads();
        int key[K];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int j = tid + s * NT;
            key[s] = 0;
            if (j < N) {
                key[s] = ((cell_of(xs[3 * j + 2], a.inv_h) - kmin[2]) * Cy +
                          (cell_of(xs[3 * j + 1], a.inv_h) - kmin[1])) * Cx +
                         (cell_of(xs[3 * j], a.inv_h) - kmin[0]);
                atomicAdd(hist + key[s], 1);
            }
        }
        __syncthreads();
        int *occ_idx = hist + C;
        for (int c = tid; c < C; c += NT) occ_idx[c] = hist[c] > 0 ? 1 : 0;
        __syncthreads();
        const int n_occ = block_exclusive_scan<NT>(occ_idx, C, ired);
        block_exclusive_scan<NT>(hist, C, ired);
        for (int c = tid; c < C; c += NT) {
            const int start = hist[c];
            const int next = c + 1 < C ? hist[c + 1] : N;
            if (next > start) {
                occ_start[occ_idx[c]] = (uint16_t)start;
                occ_cnt[occ_idx[c]] = (uint16_t)(next - start);
            }
        }
        if (tid == 0) n_occ_sh = n_occ;
        if (tid <= kCountBins) cnt_bins[tid] = 0;
        __syncthreads();
        // order the occupied cells by decreasing node count, so that the
        // threads of a wave spread cells of similar size (counting sort)
        int ost[K], ocn[K], obin[K];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int o = tid + s * NT;
            ost[s] = o < n_occ ? occ_start[o] : 0;
            ocn[s] = o < n_occ ? occ_cnt[o] : 0;
            obin[s] = kCountBins - min(ocn[s], kCountBins);
            if (o < n_occ) atomicAdd(cnt_bins + obin[s], 1);
        }
        __syncthreads();
        if (tid == 0) {
            int run = 0;
            for (int i = 0; i <= kCountBins; ++i) {
                const int v = cnt_bins[i];
                cnt_bins[i] = run;
                run += v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int o = tid + s * NT;
            if (o < n_occ) {
                const int r = atomicAdd(cnt_bins + obin[s], 1);
                occ_start[r] = (uint16_t)ost[s];
                occ_cnt[r] = (uint16_t)ocn[s];
            }
        }
        double xr[K][3], fr[K][3];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int j = tid + s * NT;
            if (j < N) {
                pos[s] = atomicAdd(hist + key[s], 1);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xr[s][c] = xs[3 * j + c];
                    fr[s][c] = Fs[3 * j + c];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int j = tid + s * NT;
            if (j < N) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xs[3 * pos[s] + c] = xr[s][c];
                    Fs[3 * pos[s] + c] = fr[s][c];
                }
            }
        }
        __syncthreads();
    }
    const TileGeom tg{{kmin[0], kmin[1], kmin[2]}, Tx, Ty, Tz, T, a.nx, a.ny, a.nz, a.plane};

    // ---- P4: spreading ----
    if (a.f != nullptr) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            R *fd = (R *)a.f + d * a.field;
            if (use_tile) {
                for (int t = tid; t < T; t += NT) ftile[t] = 0.0;
                __syncthreads();
                const int n_occ = n_occ_sh;
                for (int o = tid; o < n_occ; o += NT) {
                    const int p = occ_start[o], q = p + occ_cnt[o];
                    const int kcell[3] = {cell_of(xs[3 * p], a.inv_h), cell_of(xs[3 * p + 1], a.inv_h),
                                          cell_of(xs[3 * p + 2], a.inv_h)};
                    if (d == 0)
                        spread_cell<R, 0>(xs, Fs, p, q, kcell, kmin, Tx, Ty, T, a.inv_h, a.inv_h3,
                                          ftile, bad);
                    else if (d == 1)
                        spread_cell<R, 1>(xs, Fs, p, q, kcell, kmin, Tx, Ty, T, a.inv_h, a.inv_h3,
                                          ftile, bad);
                    else
                        spread_cell<R, 2>(xs, Fs, p, q, kcell, kmin, Tx, Ty, T, a.inv_h, a.inv_h3,
                                          ftile, bad);
                }
                __syncthreads();
                for (int t = tid; t < T; t += NT) {
                    const double v = ftile[t];
                    if (v != 0.0) unsafeAtomicAdd(fd + tg.grid_index(t), (R)v);
                }
                __syncthreads();
            } else {
                for (int p = tid; p < N; p += NT) {
                    R wx[3], wy[3], wz[3];
                    const int cx = delta3<R>(xs[3 * p] * a.inv_h - mac_off(d, 0), wx);
                    const int cy = delta3<R>(xs[3 * p + 1] * a.inv_h - mac_off(d, 1), wy);
                    const int cz = delta3<R>(xs[3 * p + 2] * a.inv_h - mac_off(d, 2), wz);
                    const R fv = (R)(Fs[3 * p + d] * a.inv_h3);
                    for (int z = 0; z < 3; ++z)
                        for (int y = 0; y < 3; ++y) {
                            R *row = fd + wrapi(cz - 1 + z, a.nz) * a.plane +
                                     (int64_t)wrapi(cy - 1 + y, a.ny) * a.nx;
                            const R fzy = fv * wz[z] * wy[y];
                            for (int x = 0; x < 3; ++x)
                                unsafeAtomicAdd(row + wrapi(cx - 1 + x, a.nx), fzy * wx[x]);
                        }
                }
            }
        }
    }

    // ---- P5: interpolation and update, one lattice (= one component) at a time ----
    // Nodes are visited in work order (cell order when sorted); the new
    // coordinate d replaces F_d in Fs, which nothing reads after this lattice.
    const double cm = a.dt * a.dt / a.mass[b];
    __syncthreads();      // every thread is done with spreading
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const R *ud = (const R *)a.u + d * a.field;
        if (use_tile) {
            stage_tile<NT>(utile, ud, tg);
            __syncthreads();
        }
        for (int p = tid; p < N; p += NT) {
            R wx[3], wy[3], wz[3];
            const double xd = xs[3 * p + d];
            const int cx = delta3<R>(xs[3 * p] * a.inv_h - mac_off(d, 0), wx);
            const int cy = delta3<R>(xs[3 * p + 1] * a.inv_h - mac_off(d, 1), wy);
            const int cz = delta3<R>(xs[3 * p + 2] * a.inv_h - mac_off(d, 2), wz);
            R acc = 0;
            if (use_tile) {
                const int lx = cx - kmin[0], ly = cy - kmin[1], lz = cz - kmin[2];
                if (lx < 0 || ly < 0 || lz < 0 || lx + 2 >= Tx || ly + 2 >= Ty || lz + 2 >= Tz) {
                    bad = true;
                } else {
#pragma unroll
                    for (int z = 0; z < 3; ++z)
#pragma unroll
                        for (int y = 0; y < 3; ++y) {
                            const R *row = utile + ((lz + z) * Ty + (ly + y)) * Tx + lx;
                            acc += wz[z] * wy[y] * (wx[0] * row[0] + wx[1] * row[1] + wx[2] * row[2]);
                        }
                }
            } else {
#pragma unroll
                for (int z = 0; z < 3; ++z)
#pragma unroll
                    for (int y = 0; y < 3; ++y) {
                        const R *row = ud + wrapi(cz - 1 + z, a.nz) * a.plane +
                                       (int64_t)wrapi(cy - 1 + y, a.ny) * a.nx;
                        acc += wz[z] * wy[y] *
                               (wx[0] * row[wrapi(cx - 1, a.nx)] + wx[1] * row[wrapi(cx, a.nx)] +
                                wx[2] * row[wrapi(cx + 1, a.nx)]);
                    }
            }
            const double fd = Fs[3 * p + d];
            if (!isfinite(fd) || !isfinite((double)acc)) atomicOr(a.status, IP_STATUS_NONFINITE);
            Fs[3 * p + d] = xd + a.dt * (double)acc + cm * (double)(R)fd;
        }
        if (use_tile) __syncthreads();
    }
    __syncthreads();
    // back to node order (pinned nodes keep their position), staged in xs;
    // a whole body is written in place, once and coalesced, a patch into the
    // staging array (its nodes are other patches' halo until the step ends)
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int j = tid + s * NT;
        if (j < N) {
            const int64_t g = whole ? n0 + j : (int64_t)gid[j];
            const bool pin = a.pinned[g] != 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) xs[3 * j + c] = pin ? a.X[3 * g + c] : Fs[3 * pos[s] + c];
        }
    }
    __syncthreads();
    if (whole) {
        for (int i = tid; i < 3 * N; i += NT) a.X[3 * n0 + i] = xs[i];
    } else {
        for (int j = tid; j < N; j += NT) {
            const int64_t g = gid[j];
            a.Xstage[3 * g] = xs[3 * j];
            a.Xstage[3 * g + 1] = xs[3 * j + 1];
            a.Xstage[3 * g + 2] = xs[3 * j + 2];
        }
    }
    if (bad) atomicOr(a.status, IP_STATUS_DEGENERATE);
}

// Packed records (the fused step's element input): reference values of the
// given reference gathered into the plan's record order, with the records'
// unit-local node ids.
template <typename R>
__global__ void k_pack_edges(const int32_t *__restrict__ perm, const ushort4 *__restrict__ lid,
                             int64_t n, const R *__restrict__ l0, const R *__restrict__ cs0,
                             EdgeRec<R> *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t e = perm[r];
    const ushort4 v = lid[r];
    EdgeRec<R> o{};
    o.v[0] = v.x;
    o.v[1] = v.y;
    o.v[2] = v.z;
    o.v[3] = v.w;
    o.l0 = l0[e];
    o.c0 = cs0[2 * e];
    o.s0 = cs0[2 * e + 1];
    out[r] = o;
}

template <typename R>
__global__ void k_pack_faces(const int32_t *__restrict__ perm, const ushort4 *__restrict__ lid,
                             int64_t n, const R *__restrict__ A0, FaceRec<R> *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const ushort4 v = lid[r];
    FaceRec<R> o{};
    o.v[0] = v.x;
    o.v[1] = v.y;
    o.v[2] = v.z;
    o.a0 = A0[perm[r]];
    out[r] = o;
}

template <typename R>
void pack_reference(ip_plan *p, const ip_reference *ref, hipStream_t s) {
    const int t = 256;
    if (p->n_erec > 0)
        hipLaunchKernelGGL(k_pack_edges<R>, dim3((unsigned)((p->n_erec + t - 1) / t)), dim3(t), 0,
                           s, p->erec_perm, (const ushort4 *)p->erec_lid, p->n_erec,
                           (const R *)ref->l0, (const R *)ref->cs0, (EdgeRec<R> *)p->edge_rec);
    if (p->n_frec > 0)
        hipLaunchKernelGGL(k_pack_faces<R>, dim3((unsigned)((p->n_frec + t - 1) / t)), dim3(t), 0,
                           s, p->frec_perm, (const ushort4 *)p->frec_lid, p->n_frec,
                           (const R *)ref->A0, (FaceRec<R> *)p->face_rec);
}

// New positions of patched bodies: staging array -> X (owned nodes of each
// patch unit; one workgroup per unit).
__global__ void k_commit(const int32_t *__restrict__ units, const int64_t *__restrict__ noff,
                         const int32_t *__restrict__ owned, const int32_t *__restrict__ nodes,
                         const double *__restrict__ Xstage, double *__restrict__ X) {
    const int w = units[blockIdx.x];
    const int32_t *gid = nodes + noff[2 * w];
    for (int j = threadIdx.x; j < owned[w]; j += blockDim.x) {
        const int64_t g = gid[j];
        X[3 * g] = Xstage[3 * g];
        X[3 * g + 1] = Xstage[3 * g + 1];
        X[3 * g + 2] = Xstage[3 * g + 2];
    }
}

}  // namespace

ip_status launch_pack_reference(ip_plan *p, const ip_reference *ref, hipStream_t s) {
    if (p->prec == IP_F64)
        pack_reference<double>(p, ref, s);
    else
        pack_reference<float>(p, ref, s);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

size_t step_fused_lds_bytes(int nmax, int tile_bytes) {
    // xs + Fs (FP64), the tile region, the occupied-cell list (start, count)
    return (size_t)nmax * 48 + (size_t)tile_bytes + (size_t)nmax * 2 * sizeof(uint16_t);
}

template <typename R>
const void *step_kernel(int threads) {
    return threads == 384 ? (const void *)k_step_fused<R, 384> : (const void *)k_step_fused<R, 768>;
}

ip_status prepare_step_fused(ip_plan *p) {
    for (int c = 0; c < p->n_step_classes; ++c) {
        const auto &sc = p->step_class[c];
        const int lds = (int)step_fused_lds_bytes(sc.nmax, sc.tile_bytes);
        const void *fn = p->prec == IP_F64 ? step_kernel<double>(sc.threads)
                                           : step_kernel<float>(sc.threads);
        IP_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    }
    return IP_OK;
}

// The records must hold `ref` (packed by the caller of this launcher).
ip_status launch_step_fused(ip_plan *p, double *X, const ip_reference *ref,
                            const ip_constants *k, const void *u, void *f, double dt,
                            double *V, double *A, hipStream_t s) {
    if (p->B == 0) return IP_OK;
    StepArgs a{};
    a.X = X;
    a.Xstage = p->Xstage;
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
    a.f = f;
    a.nx = p->grid.nx;
    a.ny = p->grid.ny;
    a.nz = p->grid.nz;
    a.inv_h = 1.0 / p->grid.h;
    a.inv_h3 = 1.0 / (p->grid.h * p->grid.h * p->grid.h);
    a.plane = (int64_t)a.nx * a.ny;
    a.field = a.plane * a.nz;
    a.dt = dt;
    a.V = V ? V : p->Vbuf;
    a.A = A ? A : p->Abuf;
    a.status = p->status;
    a.wu_body = p->wu_body;
    a.wu_owned = p->wu_owned;
    a.wu_nodes = p->wu_nodes;
    a.wu_noff = p->wu_noff;
    a.wu_eoff = p->wu_eoff;
    a.wu_foff = p->wu_foff;
    a.erec = p->edge_rec;
    a.frec = p->face_rec;
    // volume and area of patched bodies, before their patches need them
    if (p->n_patched_bodies > 0)
        IP_TRY(launch_geometry(p, X, a.V, a.A, s, p->patched_bodies, p->n_patched_bodies));
    for (int c = 0; c < p->n_step_classes; ++c) {
        const auto &sc = p->step_class[c];
        a.unit_base = sc.unit_begin;
        a.nmax = sc.nmax;
        a.tile_bytes = sc.tile_bytes;
        const size_t lds = step_fused_lds_bytes(sc.nmax, sc.tile_bytes);
        const dim3 grid(sc.unit_end - sc.unit_begin), block(sc.threads);
        if (p->prec == IP_F64) {
            if (sc.threads == 384)
                hipLaunchKernelGGL((k_step_fused<double, 384>), grid, block, lds, s, a);
            else
                hipLaunchKernelGGL((k_step_fused<double, 768>), grid, block, lds, s, a);
        } else {
            if (sc.threads == 384)
                hipLaunchKernelGGL((k_step_fused<float, 384>), grid, block, lds, s, a);
            else
                hipLaunchKernelGGL((k_step_fused<float, 768>), grid, block, lds, s, a);
        }
        IP_HIP_CHECK(hipGetLastError());
    }
    if (p->n_patched_units > 0) {
        hipLaunchKernelGGL(k_commit, dim3(p->n_patched_units), dim3(256), 0, s, p->patched_units,
                           p->wu_noff, p->wu_owned, p->wu_nodes, p->Xstage, X);
        IP_HIP_CHECK(hipGetLastError());
    }
    return IP_OK;
}
