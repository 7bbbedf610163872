// step_common.h -- device pieces shared by the fused forward step and the
// fused reverse step: LDS accumulation, block reductions and scans, the
// per-unit load of positions with the cell bounding box, the counting sort of
// a unit's nodes by Eulerian cell, spreading through an LDS tile, and the
// packed element records.  Every function is called by all threads of the
// workgroup (they contain barriers) unless stated otherwise.
#pragma once

#include <climits>

#include "elements.h"
#include "ipibm_internal.h"

namespace {

constexpr int K = kStepNodesPerThread;
constexpr int kCountBins = 32;     // occupied cells are ordered by node count (capped)
constexpr int FK = kStepFacesPerThread;


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


// ---------------------------------------------------------------------------
// Unit positions -> LDS (contiguous for a whole body, gathered for a patch),
// and the cell bounding box of the first N (owned) nodes.
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void load_positions(double *xs, const double *X, bool whole, int64_t n0,
                                               const int32_t *gid, int NL, int N, double inv_h,
                                               int *ired, int kmin[3], int kmax[3]) {
    const int tid = threadIdx.x;
    if (whole) {
        copy_to_lds<NT>(xs, X + 3 * n0, 3 * NL);
    } else {
        for (int i = tid; i < NL; i += NT) {
            const int64_t g = gid[i];
            xs[3 * i] = X[3 * g];
            xs[3 * i + 1] = X[3 * g + 1];
            xs[3 * i + 2] = X[3 * g + 2];
        }
    }
    __syncthreads();
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int j = tid + s * NT;
        if (j < N) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int kc = cell_of(xs[3 * j + c], inv_h);
                lo[c] = min(lo[c], kc);
                hi[c] = max(hi[c], kc);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        kmin[c] = block_min_int<NT>(lo[c], ired);
        kmax[c] = block_max_int<NT>(hi[c], ired);
    }
}

// ---------------------------------------------------------------------------
// Counting sort of the first N nodes by Eulerian cell (section 5's per-marker
// cell index): xs and vals ([N][3] each) are permuted in place into cell
// order, pos[s] receives the new index of node tid + s NT, and the occupied
// cells are listed (first node, count) ordered by decreasing count, so that
// the threads of a wave spread cells of similar size.  Skipped (use_tile =
// false, identity order) when the unit's cell box or grid tile does not fit
// the tile region.
// ---------------------------------------------------------------------------
struct CellSort {
    bool use_tile;
    int C, n_occ;
    TileGeom tg;
};

template <int NT>
__device__ CellSort cell_sort(double *xs, double *vals, int N, const int kmin[3], const int kmax[3],
                              double inv_h, unsigned char *tile_region, int tile_bytes,
                              uint16_t *occ_start, uint16_t *occ_cnt, int *ired, int *n_occ_sh,
                              int *cnt_bins, int pos[K], int nx, int ny, int nz, int64_t plane) {
    const int tid = threadIdx.x;
    int *hist = (int *)tile_region;
    const int Cx = kmax[0] - kmin[0] + 1, Cy = kmax[1] - kmin[1] + 1, Cz = kmax[2] - kmin[2] + 1;
    const int Tx = Cx + 3, Ty = Cy + 3, Tz = Cz + 3;    // points kmin-1 .. kmax+2
    const long long Cl = (long long)Cx * Cy * Cz, Tl = (long long)Tx * Ty * Tz;
    const bool use_tile = Cx >= 1 && Cy >= 1 && Cz >= 1 && Cl <= 65535 && Cl * 8 <= tile_bytes &&
                          Tl * 8 <= tile_bytes;
    const int C = use_tile ? (int)Cl : 0, T = use_tile ? (int)Tl : 0;
#pragma unroll
    for (int s = 0; s < K; ++s) pos[s] = tid + s * NT;     // identity unless sorted
    int n_occ = 0;
    if (use_tile) {
        for (int c = tid; c < C; c += NT) hist[c] = 0;
        __syncthreads();
        int key[K];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int j = tid + s * NT;
            key[s] = 0;
            if (j < N) {
                key[s] = ((cell_of(xs[3 * j + 2], inv_h) - kmin[2]) * Cy +
                          (cell_of(xs[3 * j + 1], inv_h) - kmin[1])) * Cx +
                         (cell_of(xs[3 * j], inv_h) - kmin[0]);
                atomicAdd(hist + key[s], 1);
            }
        }
        __syncthreads();
        int *occ_idx = hist + C;
        for (int c = tid; c < C; c += NT) occ_idx[c] = hist[c] > 0 ? 1 : 0;
        __syncthreads();
        n_occ = block_exclusive_scan<NT>(occ_idx, C, ired);
        block_exclusive_scan<NT>(hist, C, ired);
        for (int c = tid; c < C; c += NT) {
            const int start = hist[c];
            const int next = c + 1 < C ? hist[c + 1] : N;
            if (next > start) {
                occ_start[occ_idx[c]] = (uint16_t)start;
                occ_cnt[occ_idx[c]] = (uint16_t)(next - start);
            }
        }
        if (tid == 0) *n_occ_sh = n_occ;
        if (tid <= kCountBins) cnt_bins[tid] = 0;
        __syncthreads();
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
                    fr[s][c] = vals[3 * j + c];
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
                    vals[3 * pos[s] + c] = fr[s][c];
                }
            }
        }
        __syncthreads();
    }
    return {use_tile, C, n_occ, TileGeom{{kmin[0], kmin[1], kmin[2]}, Tx, Ty, Tz, T, nx, ny, nz, plane}};
}

// ---------------------------------------------------------------------------
// Spreading of vals ([N][3], cell order when sorted) onto the three lattices
// of the grid field f (real R, [3][nz][ny][nx], accumulated): per occupied
// cell a 4x3x3 register block, added once to the FP64 LDS tile whose non-zero
// points are then added to f with device atomics; without a tile, every node
// adds its 27 weights to f directly.
// ---------------------------------------------------------------------------
template <typename R, int NT>
__device__ void spread_to_grid(const double *xs, const double *vals, int N, const CellSort &cs,
                               const uint16_t *occ_start, const uint16_t *occ_cnt, double *ftile,
                               R *f, int64_t field, double inv_h, double inv_h3, bool &bad) {
    const int tid = threadIdx.x;
    const TileGeom &tg = cs.tg;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R *fd = f + d * field;
        if (cs.use_tile) {
            for (int t = tid; t < tg.T; t += NT) ftile[t] = 0.0;
            __syncthreads();
            for (int o = tid; o < cs.n_occ; o += NT) {
                const int p = occ_start[o], q = p + occ_cnt[o];
                const int kcell[3] = {cell_of(xs[3 * p], inv_h), cell_of(xs[3 * p + 1], inv_h),
                                      cell_of(xs[3 * p + 2], inv_h)};
                if (d == 0)
                    spread_cell<R, 0>(xs, vals, p, q, kcell, tg.kmin, tg.Tx, tg.Ty, tg.T, inv_h,
                                      inv_h3, ftile, bad);
                else if (d == 1)
                    spread_cell<R, 1>(xs, vals, p, q, kcell, tg.kmin, tg.Tx, tg.Ty, tg.T, inv_h,
                                      inv_h3, ftile, bad);
                else
                    spread_cell<R, 2>(xs, vals, p, q, kcell, tg.kmin, tg.Tx, tg.Ty, tg.T, inv_h,
                                      inv_h3, ftile, bad);
            }
            __syncthreads();
            for (int t = tid; t < tg.T; t += NT) {
                const double v = ftile[t];
                if (v != 0.0) unsafeAtomicAdd(fd + tg.grid_index(t), (R)v);
            }
            __syncthreads();
        } else {
            for (int p = tid; p < N; p += NT) {
                R wx[3], wy[3], wz[3];
                const int cx = delta3<R>(xs[3 * p] * inv_h - mac_off(d, 0), wx);
                const int cy = delta3<R>(xs[3 * p + 1] * inv_h - mac_off(d, 1), wy);
                const int cz = delta3<R>(xs[3 * p + 2] * inv_h - mac_off(d, 2), wz);
                const R fv = (R)(vals[3 * p + d] * inv_h3);
                for (int z = 0; z < 3; ++z)
                    for (int y = 0; y < 3; ++y) {
                        R *row = fd + wrapi(cz - 1 + z, tg.nz) * tg.plane +
                                 (int64_t)wrapi(cy - 1 + y, tg.ny) * tg.nx;
                        const R fzy = fv * wz[z] * wy[y];
                        for (int x = 0; x < 3; ++x)
                            unsafeAtomicAdd(row + wrapi(cx - 1 + x, tg.nx), fzy * wx[x]);
                    }
            }
        }
    }
}

}  // namespace
