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
constexpr int kCellChunk = 8;      // nodes of a cell spread by one thread, at most
constexpr int FK = kStepFacesPerThread;


__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Values equal in every lane, moved to scalar registers (the compiler cannot
// see that a value reduced over the block is uniform).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xFFFFFFFFll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Unit of workgroup i among n.  Workgroup i runs on XCD i mod 8, each XCD
// with its own L2.  The units are dealt to the XCDs in chunks of 16
// consecutive ones, so that neighbouring units (the patches of one body,
// which share grid lines) share an L2, while every XCD still takes units of
// every size class; the last partial round of 128 units keeps the plain
// order.  A bijection of 0 .. n - 1.
__device__ __forceinline__ int xcd_unit(int i, int n) {
    constexpr int C = 16, G = 8 * C;
    if (i >= n / G * G) return i;
    const int x = i % 8, k = i / 8;
    return (k / C) * G + x * C + (k % C);
}

// Workgroup barrier that orders LDS accesses only: outstanding global memory
// operations (the grid atomics of a tile flush, prefetch loads) stay in
// flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

// The cell bounding box of a unit (minimum of lo[3], maximum of hi[3]) and D
// double sums s[D], reduced over the block in one pass (two barriers); every
// thread receives every result, the sums added in a fixed order.  ish holds
// 6 NT/64 ints, dsh D NT/64 doubles.
template <int NT, int D>
__device__ __forceinline__ void block_box_sums(int lo[3], int hi[3], double s[D], int *ish,
                                               double *dsh) {
    constexpr int W = NT / 64;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = min(lo[c], __shfl_xor(lo[c], o, 64));
            hi[c] = max(hi[c], __shfl_xor(hi[c], o, 64));
        }
#pragma unroll
        for (int j = 0; j < D; ++j) s[j] += __shfl_xor(s[j], o, 64);
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ish[6 * w + c] = lo[c];
            ish[6 * w + 3 + c] = hi[c];
        }
#pragma unroll
        for (int j = 0; j < D; ++j) dsh[D * w + j] = s[j];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = ish[c];
        hi[c] = ish[3 + c];
    }
#pragma unroll
    for (int j = 0; j < D; ++j) s[j] = dsh[j];
    for (int v = 1; v < W; ++v) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = min(lo[c], ish[6 * v + c]);
            hi[c] = max(hi[c], ish[6 * v + 3 + c]);
        }
#pragma unroll
        for (int j = 0; j < D; ++j) s[j] += dsh[D * v + j];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = uniform(lo[c]);
        hi[c] = uniform(hi[c]);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) s[j] = uniform(s[j]);
}

// D double sums over the block in one pass (two barriers); every thread
// receives them, added in a fixed order.  dsh holds D NT/64 doubles.
template <int NT, int D>
__device__ __forceinline__ void block_sums(double s[D], double *dsh) {
    constexpr int W = NT / 64;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int j = 0; j < D; ++j) s[j] += __shfl_xor(s[j], o, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int j = 0; j < D; ++j) dsh[D * w + j] = s[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < D; ++j) s[j] = dsh[j];
    for (int v = 1; v < W; ++v)
#pragma unroll
        for (int j = 0; j < D; ++j) s[j] += dsh[D * v + j];
#pragma unroll
    for (int j = 0; j < D; ++j) s[j] = uniform(s[j]);
}

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

// The grid tile of a unit: points kmin-1 .. kmax+2 per axis, t = (z Ty + y) Tx
// + x.  Threads walk it as t = threadIdx.x + k NT; each keeps its point's tile
// coordinates and advances them by the step NT (s, in tile coordinates) with
// at most one carry per axis, so no point needs a division.  The tile is no
// larger than the grid along any axis, so a coordinate g0 + x wraps at most
// once.
struct TileGeom {
    int kmin[3];            // lowest occupied cell per axis
    int Tx, Ty, Tz, T;
    int nx, ny, nz;
    int64_t plane;
    int g0[3];              // wrapped grid coordinates of tile point 0
    int s[3];               // NT in tile coordinates (s[0] < Tx, s[1] < Ty)
    int c0[3];              // this thread's first point
};

struct TileCursor {
    int t, x, y, z;
    __device__ __forceinline__ static TileCursor first(const TileGeom &g) {
        return {(int)threadIdx.x, g.c0[0], g.c0[1], g.c0[2]};
    }
    template <int NT>
    __device__ __forceinline__ void next(const TileGeom &g) {
        t += NT;
        x += g.s[0];
        y += g.s[1];
        z += g.s[2];
        if (x >= g.Tx) {
            x -= g.Tx;
            ++y;
        }
        if (y >= g.Ty) {
            y -= g.Ty;
            ++z;
        }
    }
    __device__ __forceinline__ int64_t grid_index(const TileGeom &g) const {
        int gx = g.g0[0] + x, gy = g.g0[1] + y, gz = g.g0[2] + z;
        gx -= gx >= g.nx ? g.nx : 0;
        gy -= gy >= g.ny ? g.ny : 0;
        gz -= gz >= g.nz ? g.nz : 0;
        return (int64_t)gz * g.plane + (int64_t)gy * g.nx + gx;
    }
};

// Stage the tile of one grid field into LDS, U loads in flight per thread.
template <int NT, typename R, int U = 8>
__device__ __forceinline__ void stage_tile(R *__restrict__ tile, const R *__restrict__ field,
                                           const TileGeom &g) {
    TileCursor c = TileCursor::first(g);
    while (c.t < g.T) {
        R v[U];
        int t[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            t[k] = c.t;
            v[k] = c.t < g.T ? field[c.grid_index(g)] : (R)0;
            c.template next<NT>(g);
        }
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (t[k] < g.T) tile[t[k]] = v[k];
    }
}

// A grid tile held in registers, PF values per thread: loaded while the
// previous tile is in use (the loads stay in flight), stored to LDS once that
// tile is free.  Covers tiles of at most PF NT points.
template <int NT, typename R, int PF>
struct TilePrefetch {
    R v[PF];
    __device__ __forceinline__ static bool covers(const TileGeom &g) { return g.T <= PF * NT; }
    __device__ __forceinline__ void load(const R *__restrict__ field, const TileGeom &g) {
        TileCursor c = TileCursor::first(g);
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            v[k] = c.t < g.T ? field[c.grid_index(g)] : (R)0;
            c.template next<NT>(g);
        }
    }
    __device__ __forceinline__ void store(R *__restrict__ tile, const TileGeom &g) const {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int t = (int)threadIdx.x + k * NT;
            if (t < g.T) tile[t] = v[k];
        }
    }
};

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
                                            int Tz, double inv_h, double inv_h3, double *tile,
                                            bool &bad) {
    using Dm = BlockDims<D>;
    R acc[Dm::LZ][Dm::LY][Dm::LX];
#pragma unroll
    for (int z = 0; z < Dm::LZ; ++z)
#pragma unroll
        for (int y = 0; y < Dm::LY; ++y)
#pragma unroll
            for (int x = 0; x < Dm::LX; ++x) acc[z][y][x] = 0;
    // the block's first and last planes along the lattice's unstaggered axis
    // carry weight only from nodes whose stencil centre is the cell (first)
    // or the next one (last)
    bool used0 = false, used3 = false;
    // weights of node p on this lattice, with its stencil shifted into the
    // block along the unstaggered axis
    const auto weights = [&](int p, R wx[4], R wy[4], R wz[4], bool &u0, bool &u3, bool &bd) {
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
                u0 = !s1;
                u3 = s1;
                bd = bd || (sh != 0 && sh != 1);
            } else {
                w[0] = w3[0];
                w[1] = w3[1];
                w[2] = w3[2];
                bd = bd || sh != 0;
            }
        }
    };
    const auto accumulate = [&](R fd, const R wx[4], const R wy[4], const R wz[4]) {
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
    };
    for (int p = p0; p < p1; ++p) {
        R wx[4], wy[4], wz[4];
        bool u0 = false, u3 = false, bd = false;
        weights(p, wx, wy, wz, u0, u3, bd);
        used0 |= u0;
        used3 |= u3;
        bad |= bd;
        accumulate((R)(Fs[3 * p + D] * inv_h3), wx, wy, wz);
    }
    // block origin in tile coordinates: point k - 1 is tile index k - kmin.
    // The tile spans the cells' box with one point below and two above, so
    // the block lies inside it; one check for the whole block.
    const int ox = kc[0] - kmin[0], oy = kc[1] - kmin[1], oz = kc[2] - kmin[2];
    if (!(ox >= 0 && oy >= 0 && oz >= 0 && ox + Dm::LX <= Tx && oy + Dm::LY <= Ty &&
          oz + Dm::LZ <= Tz)) {
        bad = true;
        return;
    }
    double *base = tile + (oz * Ty + oy) * Tx + ox;
    const int sz = Tx * Ty;
    // plane by plane along the unstaggered axis, so that the optional first
    // and last planes are one branch each
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if ((q == 0 && !used0) || (q == 3 && !used3)) continue;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int x = D == 0 ? q : a, y = D == 1 ? q : (D == 0 ? a : b),
                          z = D == 2 ? q : b;
                lds_add(base + z * sz + y * Tx + x, (double)acc[z][y][x]);
            }
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
// and this thread's share of the cell bounding box of the first N (owned)
// nodes (lo, hi: to be reduced over the block with block_box_sums).
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void load_positions(double *xs, const double *X, bool whole, int64_t n0,
                                               const int32_t *gid, int NL, int N, double inv_h,
                                               int lo[3], int hi[3]) {
    const int tid = threadIdx.x;
    if (whole) {
        // one round of loads in flight for the largest unit (4 NT nodes)
        copy_to_lds<NT, double, 12>(xs, X + 3 * n0, 3 * NL);
    } else {
        for (int i = tid; i < NL; i += NT) {
            const int64_t g = gid[i];
            xs[3 * i] = X[3 * g];
            xs[3 * i + 1] = X[3 * g + 1];
            xs[3 * i + 2] = X[3 * g + 2];
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = INT_MAX;
        hi[c] = INT_MIN;
    }
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
}

// ---------------------------------------------------------------------------
// Counting sort of the first N nodes by Eulerian cell (section 5's per-marker
// cell index): xs and vals ([N][3] each) are permuted in place into cell
// order, pos[s] receives the new index of node tid + s NT, and the occupied
// cells are listed as work items (first node, count) of at most kCellChunk
// nodes (a crowded cell gives several), ordered by decreasing count, so that
// the threads of a wave spread items of similar size.  Skipped (use_tile =
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
                          Tl * 8 <= tile_bytes && Tx <= nx && Ty <= ny && Tz <= nz;
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
        // a cell's nodes form ceil(n / kCellChunk) work items of at most
        // kCellChunk consecutive nodes (each item at least one node, so at most
        // N items)
        for (int c = tid; c < C; c += NT) occ_idx[c] = (hist[c] + kCellChunk - 1) / kCellChunk;
        __syncthreads();
        n_occ = uniform(block_exclusive_scan<NT>(occ_idx, C, ired));
        block_exclusive_scan<NT>(hist, C, ired);
        for (int c = tid; c < C; c += NT) {
            const int start = hist[c];
            const int next = c + 1 < C ? hist[c + 1] : N;
            for (int p = start, o = occ_idx[c]; p < next; p += kCellChunk, ++o) {
                occ_start[o] = (uint16_t)p;
                occ_cnt[o] = (uint16_t)min(kCellChunk, next - p);
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
    TileGeom tg{{kmin[0], kmin[1], kmin[2]}, Tx, Ty, Tz, T, nx, ny, nz, plane, {0, 0, 0}, {0, 0, 0},
                {0, 0, 0}};
    if (use_tile) {
        tg.g0[0] = wrapi(kmin[0] - 1, nx);
        tg.g0[1] = wrapi(kmin[1] - 1, ny);
        tg.g0[2] = wrapi(kmin[2] - 1, nz);
        const int q = NT / Tx, r = tid / Tx;
        tg.s[0] = NT % Tx;
        tg.s[1] = q % Ty;
        tg.s[2] = q / Ty;
        tg.c0[0] = tid % Tx;
        tg.c0[1] = r % Ty;
        tg.c0[2] = r / Ty;
    }
    return {use_tile, C, n_occ, tg};
}

// ---------------------------------------------------------------------------
// Spreading of vals ([N][3], cell order when sorted) onto the three lattices
// of the grid field f (real R, [3][nz][ny][nx], accumulated): per occupied
// cell a 4x3x3 register block, added once to the FP64 LDS tile whose non-zero
// points are then added to f with device atomics; without a tile, every node
// adds its 27 weights to f directly.  The atomics are not waited for (the
// barriers here order LDS only).  before_last_flush() is called by every
// thread once the last lattice's tile is complete (tile path only), so that a
// caller can issue loads that overlap the last flush.
// ---------------------------------------------------------------------------
template <typename R, int NT, typename BeforeLastFlush>
__device__ void spread_to_grid(const double *xs, const double *vals, int N, const CellSort &cs,
                               const uint16_t *occ_start, const uint16_t *occ_cnt, double *ftile,
                               R *f, int64_t field, double inv_h, double inv_h3, bool &bad,
                               BeforeLastFlush before_last_flush) {
    const int tid = threadIdx.x;
    const TileGeom &tg = cs.tg;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R *fd = f + d * field;
        if (cs.use_tile) {
            for (int t = tid; t < tg.T; t += NT) ftile[t] = 0.0;
            lds_barrier();
            for (int o = tid; o < cs.n_occ; o += NT) {
                const int p = occ_start[o], q = p + occ_cnt[o];
                const int kcell[3] = {cell_of(xs[3 * p], inv_h), cell_of(xs[3 * p + 1], inv_h),
                                      cell_of(xs[3 * p + 2], inv_h)};
                if (d == 0)
                    spread_cell<R, 0>(xs, vals, p, q, kcell, tg.kmin, tg.Tx, tg.Ty, tg.Tz, inv_h,
                                      inv_h3, ftile, bad);
                else if (d == 1)
                    spread_cell<R, 1>(xs, vals, p, q, kcell, tg.kmin, tg.Tx, tg.Ty, tg.Tz, inv_h,
                                      inv_h3, ftile, bad);
                else
                    spread_cell<R, 2>(xs, vals, p, q, kcell, tg.kmin, tg.Tx, tg.Ty, tg.Tz, inv_h,
                                      inv_h3, ftile, bad);
            }
            lds_barrier();
            if (d == 2) before_last_flush();
            // the grid atomics stay in flight across the following barriers
            for (TileCursor c = TileCursor::first(tg); c.t < tg.T; c.template next<NT>(tg)) {
                const double v = ftile[c.t];
                if (v != 0.0) unsafeAtomicAdd(fd + c.grid_index(tg), (R)v);
            }
            lds_barrier();
        } else {
            // three lanes per node, lane j adding the stencil's column x = j
            // of every (y, z) row: the three additions to one row fall in
            // one cache line and travel as one atomic request, where a lane
            // per node sends one request per point (21 nodes per wave)
            const int lane = tid & 63, j = lane % 3;
            if (lane < 63)
                for (int p = (tid >> 6) * 21 + lane / 3; p < N; p += (NT / 64) * 21) {
                    R wx[3], wy[3], wz[3];
                    const int cx = delta3<R>(xs[3 * p] * inv_h - mac_off(d, 0), wx);
                    const int cy = delta3<R>(xs[3 * p + 1] * inv_h - mac_off(d, 1), wy);
                    const int cz = delta3<R>(xs[3 * p + 2] * inv_h - mac_off(d, 2), wz);
                    const R fvx = (R)(vals[3 * p + d] * inv_h3) * (j == 0 ? wx[0] : (j == 1 ? wx[1] : wx[2]));
                    const int64_t ix = wrapi(cx - 1 + j, tg.nx);
                    int64_t iy[3], iz[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        iy[k] = (int64_t)wrapi(cy - 1 + k, tg.ny) * tg.nx;
                        iz[k] = (int64_t)wrapi(cz - 1 + k, tg.nz) * tg.plane;
                    }
#pragma unroll
                    for (int z = 0; z < 3; ++z)
#pragma unroll
                        for (int y = 0; y < 3; ++y)
                            unsafeAtomicAdd(fd + iz[z] + iy[y] + ix, fvx * wz[z] * wy[y]);
                }
        }
    }
}

}  // namespace
