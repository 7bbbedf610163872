// k_step.hip -- the fused explicit step, one workgroup per work unit (a whole
// body, or a patch of a larger body: its owned nodes plus the halo its
// elements reach).
//
// LDS (per workgroup): positions xs[n][3] (FP64), force accumulators
// Fs[n][3] (FP64 for every plan precision: FP32 LDS atomics are an order of
// magnitude slower than FP64 ones on gfx950), a tile region for the cell
// histogram and the per-lattice grid tiles, and the occupied-cell list.
//
// Phases (units are independent; no inter-workgroup communication except the
// additions into the grid force field):
//  P0  positions -> LDS; cell bounding box of the owned nodes (the per-marker
//      cell index and the body bounding box of Section 5).
//  P1  enclosed volume of a whole body (FP64 block reduction); a patched
//      body's comes from a geometry pass before this kernel.  The area is
//      summed from the face loop of P2 and reduced at the end.
//  P2  face (area + volume) and edge (spring + hinge) elements from the packed
//      records, their forces added into the node accumulators (ds_add_f64).
//  P3  counting sort of the owned nodes by Eulerian cell; xs and Fs are
//      permuted in place into cell order.
//  P4  spreading, per lattice, through an FP64 LDS tile (step_common.h).
//  P5  per lattice d: the velocity tile is staged in LDS, every owned node
//      interpolates U_d from its 27-point stencil and gets the new coordinate
//      X_d + dt U_d + dt^2/m F_d (nodes that are not pinned).
// Units whose tile does not fit the tile region interpolate and spread
// directly against the grid (same arithmetic, global atomics).
#include "step_common.h"

namespace {

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
    const double *ew;        // [n_erec][2] per-edge weights on ks, kb (EW only)
    int unit_base;           // unit of workgroup 0 of this launch
    int nmax;                // node capacity of the LDS layout
    int tile_bytes;          // bytes of the tile region
};

// EW: the edges carry per-edge weights on ks and kb (record order).
// NT = 256 and 128 workgroups are meant to share a compute unit three to six
// at a time, which caps their registers at 168.
template <typename R, int NT, bool EW>
__global__ __launch_bounds__(NT, NT <= 256 ? 3 : 1) void k_step_fused(StepArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ double red[2 * (NT / 64)];
    __shared__ int ired[6 * (NT / 64)];
    __shared__ int n_occ_sh;
    __shared__ int cnt_bins[kCountBins + 1];

    const int tid = threadIdx.x;
    const int w = a.unit_base + xcd_unit((int)blockIdx.x, (int)gridDim.x);
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

    // ---- P0: positions (contiguous for a whole body, gathered for a patch),
    // this thread's share of the cell bounding box of the owned nodes (the
    // ones spread and interpolated) ----
    for (int i = tid; i < 3 * NL; i += NT) Fs[i] = 0.0;
    int kmin[3], kmax[3];
    load_positions<NT>(xs, a.X, whole, n0, gid, NL, N, a.inv_h, kmin, kmax);

    // ---- P1: volume (a whole body; a patched body's comes from the geometry
    // pass that precedes this kernel), reduced together with the bounding box ----
    double sums[1] = {0.0};
    if (whole) {
        const vec3<double> anchor = ldx(xs, 0);
#pragma unroll
        for (int s = 0; s < FK; ++s) {
            if (fmask & (1u << s)) {
                const vec3<double> xi = ldx(xs, fi[s][0]), xj = ldx(xs, fi[s][1]),
                                   xk = ldx(xs, fi[s][2]);
                sums[0] += dot(xi - anchor, cross(xj - anchor, xk - anchor));
            }
        }
    }
    block_box_sums<NT, 1>(kmin, kmax, sums, ired, red);
    double Vb;
    if (whole) {
        Vb = sums[0] * (1.0 / 6.0);
        if (tid == 0) a.V[b] = Vb;
    } else {
        Vb = a.V[b];
    }
    // twice the area of this thread's faces, from the face forces below
    double area2 = 0.0;

    // ---- P2: elements -> node accumulators ----
    {
        const R sV = volume_coefficient<R>(a.closed[b] != 0, a.kV[b], Vb, a.V0[b]);
        const double kA = a.kA[b];
#pragma unroll
        for (int s = 0; s < FK; ++s) {
            if (fmask & (1u << s)) {
                const int i = fi[s][0], j = fi[s][1], k = fi[s][2];
                vec3<R> gi, gj, gk;
                R nn;
                bad |= face_forces<double, R>(ldx(xs, i), ldx(xs, j), ldx(xs, k), fa0[s], kA, sV,
                                              gi, gj, gk, &nn);
                area2 += (double)nn;
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
            double kse = ks, kbe = kb;
            if constexpr (EW) {
                const double2 wt = reinterpret_cast<const double2 *>(a.ew)[e0 + t];
                kse *= wt.x;
                kbe *= wt.y;
            }
            bad |= edge_forces<double, R>(x1, x2, x3, x4, hinge, cur.l0(), cur.c0(), cur.s0(), kse,
                                          kbe, f1, f2, f3, f4);
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
    int pos[K];
    const CellSort cs = cell_sort<NT>(xs, Fs, N, kmin, kmax, a.inv_h, tile_region, a.tile_bytes,
                                      occ_start, occ_cnt, ired, &n_occ_sh, cnt_bins, pos, a.nx,
                                      a.ny, a.nz, a.plane);
    const bool use_tile = cs.use_tile;
    const TileGeom &tg = cs.tg;
    const int Tx = tg.Tx, Ty = tg.Ty, Tz = tg.Tz;

    // ---- P4: spreading; the velocity tile of lattice 0 is fetched into
    // registers before the last flush ----
    constexpr int PF = NT >= 768 ? 5 : 8;
    TilePrefetch<NT, R, PF> pf;
    const bool pf_ok = use_tile && TilePrefetch<NT, R, PF>::covers(tg);
    bool have0 = false;
    if (a.f != nullptr)
        spread_to_grid<R, NT>(xs, Fs, N, cs, occ_start, occ_cnt, ftile, (R *)a.f, a.field, a.inv_h,
                              a.inv_h3, bad, [&] {
                                  if (pf_ok) {
                                      pf.load((const R *)a.u, tg);
                                      have0 = true;
                                  }
                              });

    // ---- P5: interpolation and update, one lattice (= one component) at a time ----
    // Nodes are visited in work order (cell order when sorted); the new
    // coordinate d replaces F_d in Fs, which nothing reads after this lattice.
    // The velocity tile of lattice d + 1 is loaded into registers while
    // lattice d is interpolated.
    const double cm = a.dt * a.dt / a.mass[b];
    if (pf_ok && !have0) pf.load((const R *)a.u, tg);
    lds_barrier();      // every thread is done with spreading
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const R *ud = (const R *)a.u + d * a.field;
        if (use_tile) {
            if (pf_ok)
                pf.store(utile, tg);
            else
                stage_tile<NT>(utile, ud, tg);
            lds_barrier();
            if (pf_ok && d < 2) pf.load(ud + a.field, tg);
        }
        if (use_tile) {
            // interpolation of node p from the tile (bounds-checked)
            const auto interp = [&](int p) {
                R wx[3], wy[3], wz[3];
                const int cx = delta3<R>(xs[3 * p] * a.inv_h - mac_off(d, 0), wx);
                const int cy = delta3<R>(xs[3 * p + 1] * a.inv_h - mac_off(d, 1), wy);
                const int cz = delta3<R>(xs[3 * p + 2] * a.inv_h - mac_off(d, 2), wz);
                R acc = 0;
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
                return acc;
            };
            const auto update = [&](int p, R acc) {
                const double fd = Fs[3 * p + d];
                if (!isfinite(fd) || !isfinite((double)acc)) atomicOr(a.status, IP_STATUS_NONFINITE);
                Fs[3 * p + d] = xs[3 * p + d] + a.dt * (double)acc + cm * (double)(R)fd;
            };
            for (int p = tid; p < N; p += NT) update(p, interp(p));
        } else {
            // directly from the grid, three lanes per node (21 nodes per
            // wave): lane j reads column x = j of the stencil's nine rows,
            // so the three reads of a row share a cache line, and the node's
            // value is the sum over its three lanes
            const int lane = tid & 63, j = lane % 3;
            for (int pb = (tid >> 6) * 21; pb < N; pb += (NT / 64) * 21) {
                const int p = pb + lane / 3;
                const bool act = lane < 63 && p < N;
                R acc = 0;
                if (act) {
                    R wx[3], wy[3], wz[3];
                    const int cx = delta3<R>(xs[3 * p] * a.inv_h - mac_off(d, 0), wx);
                    const int cy = delta3<R>(xs[3 * p + 1] * a.inv_h - mac_off(d, 1), wy);
                    const int cz = delta3<R>(xs[3 * p + 2] * a.inv_h - mac_off(d, 2), wz);
                    const R *col = ud + wrapi(cx - 1 + j, a.nx);
                    int64_t iy[3], iz[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        iy[k] = (int64_t)wrapi(cy - 1 + k, a.ny) * a.nx;
                        iz[k] = (int64_t)wrapi(cz - 1 + k, a.nz) * a.plane;
                    }
                    R v[3][3];
#pragma unroll
                    for (int z = 0; z < 3; ++z)
#pragma unroll
                        for (int y = 0; y < 3; ++y) v[z][y] = col[iz[z] + iy[y]];
#pragma unroll
                    for (int z = 0; z < 3; ++z)
#pragma unroll
                        for (int y = 0; y < 3; ++y) acc += wz[z] * wy[y] * v[z][y];
                    acc *= j == 0 ? wx[0] : (j == 1 ? wx[1] : wx[2]);
                }
                // every lane of the wave takes part in the exchange
                const R s1 = __shfl_down(acc, 1, 64), s2 = __shfl_down(acc, 2, 64);
                if (act && j == 0) {
                    const R tot = acc + s1 + s2;
                    const double xd = xs[3 * p + d];
                    const double fd = Fs[3 * p + d];
                    if (!isfinite(fd) || !isfinite((double)tot)) atomicOr(a.status, IP_STATUS_NONFINITE);
                    Fs[3 * p + d] = xd + a.dt * (double)tot + cm * (double)(R)fd;
                }
            }
        }
        if (use_tile) lds_barrier();
    }
    // the body's area (whole bodies; a patched body's comes from the geometry
    // pass): per-wave sums of the face loop's |n|, added in wave order below
    area2 = wave_sum(area2);
    if ((tid & 63) == 0) red[tid >> 6] = area2;
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
    if (whole && tid == 0) {
        double ar = 0.0;
        for (int v = 0; v < NT / 64; ++v) ar += red[v];
        a.A[b] = 0.5 * ar;
    }
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

// Results of patched bodies: staging array -> destination.  The patches of
// a body own each of its nodes exactly once, so a patched body's whole node
// range is copied, contiguous and coalesced (one workgroup per body).
__global__ __launch_bounds__(256) void k_commit(const int32_t *__restrict__ bodies,
                                                const int64_t *__restrict__ node_off,
                                                const double *__restrict__ Xstage,
                                                double *__restrict__ X) {
    const int b = bodies[blockIdx.x];
    const int64_t i0 = 3 * node_off[b], i1 = 3 * node_off[b + 1];
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) X[i] = Xstage[i];
}

}  // namespace

ip_status launch_commit(ip_plan *p, const double *src, double *dst, hipStream_t s) {
    if (p->n_patched_bodies == 0) return IP_OK;
    hipLaunchKernelGGL(k_commit, dim3(p->n_patched_bodies), dim3(256), 0, s, p->patched_bodies,
                       p->node_off, src, dst);
    IP_HIP_CHECK(hipGetLastError());
    return IP_OK;
}

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

template <typename R, bool EW>
const void *step_kernel(int threads) {
    return threads == 128   ? (const void *)k_step_fused<R, 128, EW>
           : threads == 256 ? (const void *)k_step_fused<R, 256, EW>
           : threads == 384 ? (const void *)k_step_fused<R, 384, EW>
                            : (const void *)k_step_fused<R, 768, EW>;
}

ip_status prepare_step_fused(ip_plan *p) {
    for (int c = 0; c < p->n_step_classes; ++c) {
        const auto &sc = p->step_class[c];
        const int lds = (int)step_fused_lds_bytes(sc.nmax, sc.tile_bytes);
        const void *fns[2] = {
            p->prec == IP_F64 ? step_kernel<double, false>(sc.threads)
                              : step_kernel<float, false>(sc.threads),
            p->prec == IP_F64 ? step_kernel<double, true>(sc.threads)
                              : step_kernel<float, true>(sc.threads)};
        for (const void *fn : fns)
            IP_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    }
    return IP_OK;
}

template <typename R, int NT>
void launch_step_variant(dim3 grid, dim3 block, size_t lds, hipStream_t s, const StepArgs &a) {
    if (a.ew)
        hipLaunchKernelGGL((k_step_fused<R, NT, true>), grid, block, lds, s, a);
    else
        hipLaunchKernelGGL((k_step_fused<R, NT, false>), grid, block, lds, s, a);
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
    a.ew = p->ew_rec;
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
            if (sc.threads == 128)
                launch_step_variant<double, 128>(grid, block, lds, s, a);
            else if (sc.threads == 256)
                launch_step_variant<double, 256>(grid, block, lds, s, a);
            else if (sc.threads == 384)
                launch_step_variant<double, 384>(grid, block, lds, s, a);
            else
                launch_step_variant<double, 768>(grid, block, lds, s, a);
        } else {
            if (sc.threads == 128)
                launch_step_variant<float, 128>(grid, block, lds, s, a);
            else if (sc.threads == 256)
                launch_step_variant<float, 256>(grid, block, lds, s, a);
            else if (sc.threads == 384)
                launch_step_variant<float, 384>(grid, block, lds, s, a);
            else
                launch_step_variant<float, 768>(grid, block, lds, s, a);
        }
        IP_HIP_CHECK(hipGetLastError());
    }
    return launch_commit(p, p->Xstage, X, s);
}
