// api.hip -- the C-ABI of libipibm: plan construction (validation, device copies
// of the mesh, node gather lists, workspace) and the entry points declared in
// include/ipibm.h.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include <cmath>

#include "ipibm_internal.h"

namespace {
thread_local std::string g_last_error;

template <typename T>
ip_status upload(T **dst, const T *src, size_t n) {
    *dst = nullptr;
    if (n == 0) return IP_OK;
    hipError_t e = hipMalloc((void **)dst, n * sizeof(T));
    if (e != hipSuccess) {
        *dst = nullptr;
        ipibm_set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        return IP_ERR_OOM;
    }
    if (src) IP_HIP_CHECK(hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice));
    return IP_OK;
}

ip_status alloc_bytes(void **dst, size_t n) {
    *dst = nullptr;
    if (n == 0) return IP_OK;
    hipError_t e = hipMalloc(dst, n);
    if (e != hipSuccess) {
        *dst = nullptr;
        ipibm_set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        return IP_ERR_OOM;
    }
    return IP_OK;
}

ip_status arg_error(const std::string &m) {
    ipibm_set_error(m);
    return IP_ERR_ARG;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

ip_status check_offsets(const int64_t *off, int B, const char *name) {
    if (!off) return arg_error(std::string(name) + " is NULL");
    if (off[0] != 0) return arg_error(std::string(name) + "[0] != 0");
    for (int b = 0; b < B; ++b)
        if (off[b + 1] < off[b]) return arg_error(std::string(name) + " decreases");
    return IP_OK;
}

void free_plan(ip_plan *p) {
    if (!p) return;
    void *ptrs[] = {p->node_off, p->edge_off, p->face_off, p->faces, p->edges4, p->closed,
                    p->pinned, p->csr_ptr, p->csr_slot, p->slots, p->Fbuf, p->Ubuf,
                    p->Vbuf, p->Abuf, p->status, p->bwd_dots, p->bref_l0, p->bref_cs0,
                    p->bref_A0, p->bref_V0, p->wu_body, p->wu_owned, p->wu_pinned, p->wu_noff,
                    p->wu_nodes,
                    p->wu_eoff, p->wu_foff, p->erec_perm, p->erec_lid, p->frec_perm,
                    p->frec_lid, p->edge_rec, p->face_rec, p->patched_bodies,
                    p->patched_units, p->Xstage, p->ew_store, p->ew_rec_store, p->ew_bad};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete p;
}

ip_status build_plan(ip_plan *p, const ip_mesh *m, const ip_grid *grid, ip_precision prec,
                     const ip_plan_options &opt) {
    const int B = m->n_bodies;
    if (B < 0) return arg_error("n_bodies < 0");
    if (prec != IP_F64 && prec != IP_F32) return arg_error("unknown precision");
    IP_TRY(check_offsets(m->node_off, B, "node_off"));
    IP_TRY(check_offsets(m->edge_off, B, "edge_off"));
    IP_TRY(check_offsets(m->face_off, B, "face_off"));
    const int64_t N = m->node_off[B], E = m->edge_off[B], F = m->face_off[B];
    if (N >= INT32_MAX) return arg_error("more than 2^31-1 nodes");
    if ((E > 0 && !m->edges4) || (F > 0 && !m->faces) || (B > 0 && !m->closed))
        return arg_error("mesh array is NULL");
    if (4 * E + 3 * F >= (int64_t)INT32_MAX)
        return (ipibm_set_error("element slot count exceeds int32"), IP_ERR_UNSUPPORTED);
    if (grid) {
        if (grid->nx < 3 || grid->ny < 3 || grid->nz < 3 || !(grid->h > 0.0))
            return arg_error("grid needs nx, ny, nz >= 3 and h > 0");
        p->grid = *grid;
        p->has_grid = true;
    }
    // element nodes must lie in their body
    for (int b = 0; b < B; ++b) {
        const int64_t n0 = m->node_off[b], n1 = m->node_off[b + 1];
        if (m->closed[b] && n1 == n0) return arg_error("closed body without nodes");
        auto inb = [&](int32_t v) { return v >= n0 && v < n1; };
        for (int64_t e = m->edge_off[b]; e < m->edge_off[b + 1]; ++e) {
            const int32_t *q = m->edges4 + 4 * e;
            if (!inb(q[0]) || !inb(q[1]) || q[0] == q[1])
                return arg_error("edges4 row " + std::to_string(e) + ": bad edge nodes");
            for (int r = 2; r < 4; ++r)
                if (q[r] != -1 && !inb(q[r]))
                    return arg_error("edges4 row " + std::to_string(e) + ": bad wing");
            if (m->closed[b] && (q[2] < 0 || q[3] < 0))
                return arg_error("edges4 row " + std::to_string(e) +
                                 ": boundary edge in a body marked closed");
        }
        for (int64_t f = m->face_off[b]; f < m->face_off[b + 1]; ++f) {
            const int32_t *t = m->faces + 3 * f;
            if (!inb(t[0]) || !inb(t[1]) || !inb(t[2]) || t[0] == t[1] || t[1] == t[2] ||
                t[0] == t[2])
                return arg_error("faces row " + std::to_string(f) + ": bad nodes");
        }
    }
    p->B = B;
    p->N = N;
    p->E = E;
    p->F = F;
    p->prec = prec;
    IP_HIP_CHECK(hipGetDevice(&p->device));
    IP_TRY(prepare_noalloc_scratch(p->device));
    p->h_node_off.assign(m->node_off, m->node_off + B + 1);
    p->h_edge_off.assign(m->edge_off, m->edge_off + B + 1);
    p->h_face_off.assign(m->face_off, m->face_off + B + 1);

    // node <- slot gather lists, slots ascending within each node
    std::vector<int32_t> cnt(N + 1, 0);
    for (int64_t e = 0; e < E; ++e) {
        const int32_t *q = m->edges4 + 4 * e;
        const bool hinge = q[2] >= 0 && q[3] >= 0;
        for (int r = 0; r < (hinge ? 4 : 2); ++r) ++cnt[q[r] + 1];
    }
    for (int64_t f = 0; f < F; ++f)
        for (int c = 0; c < 3; ++c) ++cnt[m->faces[3 * f + c] + 1];
    for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> slot_ids(cnt[N]);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
        const int32_t *q = m->edges4 + 4 * e;
        const bool hinge = q[2] >= 0 && q[3] >= 0;
        for (int r = 0; r < (hinge ? 4 : 2); ++r) slot_ids[fill[q[r]]++] = (int32_t)(4 * e + r);
    }
    for (int64_t f = 0; f < F; ++f)
        for (int c = 0; c < 3; ++c)
            slot_ids[fill[m->faces[3 * f + c]]++] = (int32_t)(4 * E + 3 * f + c);

    std::vector<uint8_t> pin(N, 0);
    if (m->pinned) std::copy(m->pinned, m->pinned + N, pin.begin());

    IP_TRY(upload(&p->node_off, m->node_off, B + 1));
    IP_TRY(upload(&p->edge_off, m->edge_off, B + 1));
    IP_TRY(upload(&p->face_off, m->face_off, B + 1));
    IP_TRY(upload(&p->faces, m->faces, 3 * F));
    IP_TRY(upload(&p->edges4, m->edges4, 4 * E));
    IP_TRY(upload(&p->closed, m->closed, B));
    IP_TRY(upload(&p->pinned, pin.data(), N));
    IP_TRY(upload(&p->csr_ptr, cnt.data(), N + 1));
    IP_TRY(upload(&p->csr_slot, slot_ids.data(), slot_ids.size()));
    const size_t rs = p->real_size();
    IP_TRY(alloc_bytes(&p->slots, (size_t)(4 * E + 3 * F) * 3 * rs));
    IP_TRY(alloc_bytes(&p->Fbuf, (size_t)N * 3 * rs));
    IP_TRY(alloc_bytes(&p->Ubuf, (size_t)N * 3 * rs));
    IP_TRY(upload(&p->Vbuf, (const double *)nullptr, B));
    IP_TRY(upload(&p->Abuf, (const double *)nullptr, B));
    IP_TRY(upload(&p->status, (const uint32_t *)nullptr, 1));
    IP_HIP_CHECK(hipMemset(p->status, 0, sizeof(uint32_t)));

    // fused step: work units (whole bodies, patches of larger ones) that fit
    // one workgroup's registers and LDS
    int lds_optin = 0;
    IP_HIP_CHECK(hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin,
                                       p->device));
    if (lds_optin <= 0) IP_HIP_CHECK(hipDeviceGetAttribute(&lds_optin,
                                     hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
    p->lds_optin = lds_optin;
    // threads: 0 = large units on 768-thread workgroups and units of at most
    // 384 x 4 nodes on 384-thread ones (two per compute unit); 768 or 384 =
    // every unit on that size
    const int big = opt.threads > 0 ? opt.threads : 768;
    const int unit_max = big * kStepNodesPerThread;
    const int unit_nodes = opt.unit_nodes > 0 ? std::min(opt.unit_nodes, unit_max) : unit_max;
    const int unit_faces = big * kStepFacesPerThread;
    const int patch_owned = opt.patch_owned > 0 ? opt.patch_owned : kPatchOwned;
    WorkUnits wu;
    if (B > 0 && build_work_units(m, unit_nodes, unit_max, unit_faces, patch_owned, wu)) {
        const int W = (int)wu.units.size();
        // units are sorted by size: the longest suffix of units that fit a
        // 384-thread workgroup forms the second class
        int split = W;
        if (opt.threads == 0)
            while (split > 0 && wu.units[split - 1].n_nodes <= 384 * kStepNodesPerThread &&
                   wu.units[split - 1].face_end - wu.units[split - 1].face_begin <=
                       384 * kStepFacesPerThread)
                --split;
        const auto tile_for = [&](int nmax, int share) {
            // LDS left for the grid tile once positions, accumulators and the
            // cell list are placed (1 KB kept for the kernel's static LDS),
            // for `share` workgroups per compute unit
            long long t = ((long long)lds_optin / share - 1024 - (long long)step_fused_lds_bytes(nmax, 0)) / 16 * 16;
            if (opt.tile_bytes > 0) t = std::min<long long>(t, opt.tile_bytes / 16 * 16);
            return std::min<long long>(t, 1 << 20);
        };
        bool ok = true;
        p->n_step_classes = 0;
        const int bounds[3] = {0, split, W};
        for (int c = 0; c < 2; ++c) {
            if (bounds[c + 1] <= bounds[c]) continue;
            ip_plan::StepClass sc;
            sc.unit_begin = bounds[c];
            sc.unit_end = bounds[c + 1];
            sc.threads = c == 0 ? big : 384;
            sc.nmax = 1;
            for (int w = sc.unit_begin; w < sc.unit_end; ++w)
                sc.nmax = std::max(sc.nmax, wu.units[w].n_nodes);
            // the last launch (the smaller units, or the only one) is sized
            // for wg_per_cu workgroups per compute unit when that is set, the
            // 384-thread launch of the default split for two
            const bool last = bounds[c + 1] == W;
            const int share = last && opt.wg_per_cu > 0 ? opt.wg_per_cu : (c == 1 ? 2 : 1);
            long long t = share > 1 ? tile_for(sc.nmax, share) : -1;
            if (t < 4096) t = tile_for(sc.nmax, 1);
            ok = ok && t >= 4096;
            sc.tile_bytes = (int)std::max<long long>(t, 0);
            p->step_class[p->n_step_classes++] = sc;
        }
        if (ok) {
            p->fused_all = true;
            p->fused_nmax = p->step_class[0].nmax;
            p->fused_tile_bytes = p->step_class[0].tile_bytes;
            p->step_threads = p->step_class[0].threads;
            p->n_units = W;
            // ranges as (begin, end) pairs: units are stored largest first,
            // their lists in build order
            std::vector<int32_t> body(W), owned(W), pb, pu;
            std::vector<uint8_t> upin(W, 0);
            std::vector<int64_t> n2(2 * W), e2(2 * W), f2(2 * W);
            std::vector<char> patched(B, 0);
            for (int w = 0; w < W; ++w) {
                const auto &u = wu.units[w];
                body[w] = u.body;
                owned[w] = u.owned;
                n2[2 * w] = u.node_begin;
                n2[2 * w + 1] = u.node_end;
                e2[2 * w] = u.edge_begin;
                e2[2 * w + 1] = u.edge_end;
                f2[2 * w] = u.face_begin;
                f2[2 * w + 1] = u.face_end;
                if (u.node_end > u.node_begin) {
                    for (int64_t i = u.node_begin; i < u.node_end; ++i) upin[w] |= pin[wu.nodes[i]];
                } else {
                    for (int64_t i = m->node_off[u.body]; i < m->node_off[u.body + 1]; ++i)
                        upin[w] |= pin[i];
                }
                if (u.node_end > u.node_begin) {
                    pu.push_back(w);
                    if (!patched[u.body]) pb.push_back(u.body);
                    patched[u.body] = 1;
                }
            }
            IP_TRY(upload(&p->wu_body, body.data(), W));
            IP_TRY(upload(&p->wu_owned, owned.data(), W));
            IP_TRY(upload(&p->wu_pinned, upin.data(), W));
            IP_TRY(upload(&p->wu_noff, n2.data(), 2 * W));
            IP_TRY(upload(&p->wu_eoff, e2.data(), 2 * W));
            IP_TRY(upload(&p->wu_foff, f2.data(), 2 * W));
            IP_TRY(upload(&p->wu_nodes, wu.nodes.data(), wu.nodes.size()));
            p->n_erec = (int64_t)wu.edge_perm.size();
            p->n_frec = (int64_t)wu.face_perm.size();
            IP_TRY(upload(&p->erec_perm, wu.edge_perm.data(), wu.edge_perm.size()));
            IP_TRY(upload(&p->erec_lid, wu.edge_lid.data(), wu.edge_lid.size()));
            IP_TRY(upload(&p->frec_perm, wu.face_perm.data(), wu.face_perm.size()));
            IP_TRY(upload(&p->frec_lid, wu.face_lid.data(), wu.face_lid.size()));
            const size_t er = p->prec == IP_F64 ? sizeof(EdgeRec<double>) : sizeof(EdgeRec<float>);
            IP_TRY(alloc_bytes(&p->edge_rec, (size_t)p->n_erec * er));
            IP_TRY(alloc_bytes(&p->face_rec, (size_t)p->n_frec * sizeof(FaceRec<double>)));
            p->n_patched_bodies = (int32_t)pb.size();
            p->n_patched_units = (int32_t)pu.size();
            IP_TRY(upload(&p->patched_bodies, pb.data(), pb.size()));
            IP_TRY(upload(&p->patched_units, pu.data(), pu.size()));
            if (!pb.empty()) IP_TRY(alloc_bytes((void **)&p->Xstage, (size_t)N * 3 * sizeof(double)));
            IP_TRY(prepare_step_fused(p));
            if (p->prec == IP_F64) IP_TRY(prepare_step_vjp_fused(p));
            if (p->has_grid) IP_TRY(prepare_mls_units(p));
        }
    }
    IP_HIP_CHECK(hipDeviceSynchronize());
    return IP_OK;
}

ip_status check_plan(const ip_plan *p) {
    if (!p) return arg_error("plan is NULL");
    int dev = -1;
    IP_HIP_CHECK(hipGetDevice(&dev));
    if (dev != p->device) return arg_error("current device differs from the plan's device");
    return IP_OK;
}

// A NULL reference means the one bound to the plan; `ref` is resolved in place.
ip_status check_ref_k(const ip_plan *p, const ip_reference *&ref, const ip_constants *k,
                      bool need_mass) {
    if (!ref) {
        if (!p->ref_bound) return arg_error("reference is NULL and none is bound to the plan");
        ref = &p->bref;
    }
    if (!k) return arg_error("constants is NULL");
    if ((p->E > 0 && (!ref->l0 || !ref->cs0)) || (p->F > 0 && !ref->A0) ||
        (p->B > 0 && !ref->V0))
        return arg_error("reference array is NULL");
    if (p->B > 0 && (!k->ks || !k->kb || !k->kA || !k->kV || (need_mass && !k->mass)))
        return arg_error("constant array is NULL");
    const size_t rs = p->real_size();
    if (!aligned(ref->l0, rs) || !aligned(ref->cs0, rs) || !aligned(ref->A0, rs) ||
        !aligned(ref->V0, 8))
        return arg_error("misaligned reference array");
    return IP_OK;
}

}  // namespace

void ipibm_set_error(const std::string &msg) { g_last_error = msg; }

extern "C" {

const char *ip_last_error(void) { return g_last_error.c_str(); }

ip_status ip_plan_create(ip_plan **plan, const ip_mesh *mesh, const ip_grid *grid,
                         ip_precision precision) {
    return ip_plan_create_ex(plan, mesh, grid, precision, nullptr);
}

ip_status ip_plan_create_ex(ip_plan **plan, const ip_mesh *mesh, const ip_grid *grid,
                            ip_precision precision, const ip_plan_options *options) {
    if (!plan) return arg_error("plan out-pointer is NULL");
    *plan = nullptr;
    if (!mesh) return arg_error("mesh is NULL");
    ip_plan_options opt{};
    if (options) {
        opt = *options;
        if (opt.unit_nodes < 0 || opt.patch_owned < 0 || opt.tile_bytes < 0 ||
            (opt.patch_owned > 0 && opt.patch_owned < 16) ||
            (opt.tile_bytes > 0 && opt.tile_bytes < 4096) ||
            (opt.threads != 0 && opt.threads != 128 && opt.threads != 256 &&
             opt.threads != 384 && opt.threads != 768) ||
            opt.wg_per_cu < 0 || opt.wg_per_cu > 8)
            return arg_error("invalid plan options");
    }
    ip_plan *p = new ip_plan();
    ip_status st = build_plan(p, mesh, grid, precision, opt);
    if (st != IP_OK) {
        free_plan(p);
        return st;
    }
    *plan = p;
    return IP_OK;
}

ip_status ip_plan_destroy(ip_plan *plan) {
    if (!plan) return IP_OK;
    (void)hipDeviceSynchronize();
    free_plan(plan);
    return IP_OK;
}

ip_status ip_plan_sizes(const ip_plan *plan, int64_t counts[4]) {
    if (!plan || !counts) return arg_error("NULL argument");
    counts[0] = plan->B;
    counts[1] = plan->N;
    counts[2] = plan->E;
    counts[3] = plan->F;
    return IP_OK;
}

ip_status ip_plan_properties(const ip_plan *plan, int64_t props[6]) {
    if (!plan || !props) return arg_error("NULL argument");
    props[0] = plan->fused_all ? 1 : 0;
    props[1] = plan->fused_nmax;
    props[2] = plan->fused_tile_bytes;
    props[3] = plan->step_threads;
    props[4] = plan->n_units;
    props[5] = plan->n_patched_bodies;
    return IP_OK;
}

ip_status ip_reference_from(ip_plan *plan, const double *Xref, void *l0, void *cs0, void *A0,
                            double *V0, void *stream) {
    IP_TRY(check_plan(plan));
    if ((plan->N > 0 && !Xref) || (plan->E > 0 && (!l0 || !cs0)) || (plan->F > 0 && !A0) ||
        (plan->B > 0 && !V0))
        return arg_error("NULL array");
    if (!aligned(Xref, 8)) return arg_error("misaligned X");
    hipStream_t s = (hipStream_t)stream;
    IP_TRY(launch_geometry(plan, Xref, V0, plan->Abuf, s));
    return launch_reference(plan, Xref, l0, cs0, A0, s);
}

ip_status ip_plan_bind_reference(ip_plan *plan, const ip_reference *ref, void *stream) {
    IP_TRY(check_plan(plan));
    if (!ref) return arg_error("reference is NULL");
    if ((plan->E > 0 && (!ref->l0 || !ref->cs0)) || (plan->F > 0 && !ref->A0) ||
        (plan->B > 0 && !ref->V0))
        return arg_error("reference array is NULL");
    const size_t rs = plan->real_size();
    if (!aligned(ref->l0, rs) || !aligned(ref->cs0, rs) || !aligned(ref->A0, rs) ||
        !aligned(ref->V0, 8))
        return arg_error("misaligned reference array");
    if (!plan->bref_V0 && plan->B > 0) {
        IP_TRY(alloc_bytes(&plan->bref_l0, (size_t)plan->E * rs));
        IP_TRY(alloc_bytes(&plan->bref_cs0, (size_t)plan->E * 2 * rs));
        IP_TRY(alloc_bytes(&plan->bref_A0, (size_t)plan->F * rs));
        IP_TRY(upload(&plan->bref_V0, (const double *)nullptr, plan->B));
    }
    hipStream_t s = (hipStream_t)stream;
    if (plan->E > 0) {
        IP_HIP_CHECK(hipMemcpyAsync(plan->bref_l0, ref->l0, (size_t)plan->E * rs,
                                    hipMemcpyDeviceToDevice, s));
        IP_HIP_CHECK(hipMemcpyAsync(plan->bref_cs0, ref->cs0, (size_t)plan->E * 2 * rs,
                                    hipMemcpyDeviceToDevice, s));
    }
    if (plan->F > 0)
        IP_HIP_CHECK(hipMemcpyAsync(plan->bref_A0, ref->A0, (size_t)plan->F * rs,
                                    hipMemcpyDeviceToDevice, s));
    if (plan->B > 0)
        IP_HIP_CHECK(hipMemcpyAsync(plan->bref_V0, ref->V0, (size_t)plan->B * sizeof(double),
                                    hipMemcpyDeviceToDevice, s));
    plan->bref = ip_reference{plan->bref_l0, plan->bref_cs0, plan->bref_A0, plan->bref_V0};
    plan->ref_bound = true;
    if (plan->fused_all) {
        IP_TRY(launch_pack_reference(plan, &plan->bref, s));
        plan->packed = 1;
    }
    return IP_OK;
}

ip_status ip_plan_bind_edge_weights(ip_plan *plan, const double *ew, void *stream) {
    IP_TRY(check_plan(plan));
    if (!ew) {
        plan->ew = nullptr;
        plan->ew_rec = nullptr;
        return IP_OK;
    }
    if (!aligned(ew, 16)) return arg_error("misaligned weights");
    if (!plan->ew_store) {
        IP_TRY(alloc_bytes((void **)&plan->ew_store, (size_t)std::max<int64_t>(plan->E, 1) * 16));
        IP_TRY(alloc_bytes((void **)&plan->ew_rec_store,
                           (size_t)std::max<int64_t>(plan->n_erec, 1) * 16));
        IP_TRY(upload(&plan->ew_bad, (const int32_t *)nullptr, 1));
    }
    // the weights are checked before they replace the bound ones
    plan->ew = nullptr;
    plan->ew_rec = nullptr;
    IP_TRY(launch_bind_edge_weights(plan, ew, (hipStream_t)stream));
    int32_t bad = 0;
    IP_HIP_CHECK(hipMemcpyAsync(&bad, plan->ew_bad, sizeof(bad), hipMemcpyDeviceToHost,
                                (hipStream_t)stream));
    IP_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
    if (bad) return arg_error("edge weights must be finite and non-negative");
    plan->ew = plan->ew_store;
    plan->ew_rec = plan->n_erec > 0 ? plan->ew_rec_store : nullptr;
    return IP_OK;
}

ip_status ip_forces(ip_plan *plan, const double *X, const ip_reference *ref,
                    const ip_constants *k, void *F, double *V, double *A, double *W,
                    void *stream) {
    IP_TRY(check_plan(plan));
    IP_TRY(check_ref_k(plan, ref, k, false));
    if (plan->N > 0 && (!X || !F)) return arg_error("X or F is NULL");
    if (!aligned(X, 8) || !aligned(F, plan->real_size())) return arg_error("misaligned X or F");
    return launch_forces(plan, X, ref, k, F, V, A, W, (hipStream_t)stream);
}

ip_status ip_forces_noalloc(ip_plan *plan, const double *X, const ip_reference *ref,
                            const ip_constants *k, void *F, double *V, double *A, double *W,
                            void *stream) {
    IP_TRY(check_plan(plan));
    IP_TRY(check_ref_k(plan, ref, k, false));
    if (plan->N > 0 && (!X || !F)) return arg_error("X or F is NULL");
    if (!aligned(X, 8) || !aligned(F, plan->real_size())) return arg_error("misaligned X or F");
    return launch_forces_noalloc(plan, X, ref, k, F, V, A, W, (hipStream_t)stream);
}

ip_status ibm_interp(ip_plan *plan, const double *X, const void *u, void *U, void *stream) {
    IP_TRY(check_plan(plan));
    if (!plan->has_grid) return arg_error("plan has no grid");
    if (plan->N > 0 && (!X || !u || !U)) return arg_error("NULL array");
    if (!aligned(X, 8) || !aligned(u, plan->real_size()) || !aligned(U, plan->real_size()))
        return arg_error("misaligned array");
    return launch_interp(plan, X, u, U, (hipStream_t)stream);
}

ip_status ibm_spread(ip_plan *plan, const double *X, const void *F, void *f, void *stream) {
    IP_TRY(check_plan(plan));
    if (!plan->has_grid) return arg_error("plan has no grid");
    if (plan->N > 0 && (!X || !F || !f)) return arg_error("NULL array");
    if (!aligned(X, 8) || !aligned(F, plan->real_size()) || !aligned(f, plan->real_size()))
        return arg_error("misaligned array");
    return launch_spread(plan, X, F, f, (hipStream_t)stream);
}

ip_status ibm_interp_mls(ip_plan *plan, const double *X, const void *u, double alpha, void *U,
                         void *stream) {
    IP_TRY(check_plan(plan));
    if (!plan->has_grid) return arg_error("plan has no grid");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return arg_error("alpha must be positive and finite");
    if (plan->F > 0 && (!X || !u || !U)) return arg_error("NULL array");
    if (!aligned(X, 8) || !aligned(u, plan->real_size()) || !aligned(U, plan->real_size()))
        return arg_error("misaligned array");
    return launch_interp_mls(plan, X, u, alpha, U, (hipStream_t)stream);
}

ip_status ibm_spread_mls(ip_plan *plan, const double *X, const void *Fm, double alpha, void *f,
                         void *stream) {
    IP_TRY(check_plan(plan));
    if (!plan->has_grid) return arg_error("plan has no grid");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return arg_error("alpha must be positive and finite");
    if (plan->F > 0 && (!X || !Fm || !f)) return arg_error("NULL array");
    if (!aligned(X, 8) || !aligned(Fm, plan->real_size()) || !aligned(f, plan->real_size()))
        return arg_error("misaligned array");
    return launch_spread_mls(plan, X, Fm, alpha, f, (hipStream_t)stream);
}

ip_status ibm_direct_forcing_mls(ip_plan *plan, const double *X, const void *Vb, const void *u,
                                 double alpha, double dt, void *Fm, void *f, void *stream) {
    IP_TRY(check_plan(plan));
    if (!plan->has_grid) return arg_error("plan has no grid");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return arg_error("alpha must be positive and finite");
    if (!(dt > 0.0) || !std::isfinite(dt)) return arg_error("dt must be positive and finite");
    if (plan->F > 0 && (!X || !Vb || !u || !f)) return arg_error("NULL array");
    if (!aligned(X, 8) || !aligned(Vb, plan->real_size()) || !aligned(u, plan->real_size()) ||
        !aligned(Fm, plan->real_size()) || !aligned(f, plan->real_size()))
        return arg_error("misaligned array");
    return launch_direct_forcing_mls(plan, X, Vb, u, alpha, dt, Fm, f, (hipStream_t)stream);
}

ip_status ibm_probe_loads(ip_plan *plan, const double *X, const void *u, const void *p,
                          const void *acc, double alpha, double mu, void *Fext, void *stream) {
    IP_TRY(check_plan(plan));
    if (!plan->has_grid) return arg_error("plan has no grid");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return arg_error("alpha must be positive and finite");
    if (!(mu >= 0.0) || !std::isfinite(mu)) return arg_error("mu must be non-negative and finite");
    if (plan->F > 0 && (!X || !u || !p || !Fext)) return arg_error("NULL array");
    if (!aligned(X, 8) || !aligned(u, plan->real_size()) || !aligned(p, plan->real_size()) ||
        !aligned(acc, plan->real_size()) || !aligned(Fext, plan->real_size()))
        return arg_error("misaligned array");
    return launch_probe_loads(plan, X, u, p, acc, alpha, mu, Fext, (hipStream_t)stream);
}

ip_status ip_centroid_to_nodes(ip_plan *plan, const void *Fc, void *Fn, void *stream) {
    IP_TRY(check_plan(plan));
    if (plan->N > 0 && (!Fn || (plan->F > 0 && !Fc))) return arg_error("NULL array");
    if (!aligned(Fc, plan->real_size()) || !aligned(Fn, plan->real_size()))
        return arg_error("misaligned array");
    return launch_centroid_to_nodes(plan, Fc, Fn, (hipStream_t)stream);
}

ip_status ip_step(ip_plan *plan, double *X, const ip_reference *ref, const ip_constants *k,
                  const void *u, void *f, double dt, double *V, double *A, void *stream) {
    IP_TRY(check_plan(plan));
    if (!plan->has_grid) return arg_error("plan has no grid");
    IP_TRY(check_ref_k(plan, ref, k, true));
    if (plan->N > 0 && (!X || !u)) return arg_error("X or u is NULL");
    if (!aligned(X, 8) || !aligned(u, plan->real_size()) || !aligned(f, plan->real_size()))
        return arg_error("misaligned array");
    if (!(dt == dt)) return arg_error("dt is NaN");
    hipStream_t s = (hipStream_t)stream;
    if (plan->fused_all) {
        // the records hold the reference the step reads: the bound one, or
        // this call's explicit one (packed afresh: its contents may change)
        const bool bound = ref == &plan->bref;
        if (!bound || plan->packed != 1) {
            IP_TRY(launch_pack_reference(plan, ref, s));
            plan->packed = bound ? 1 : 2;
        }
        return launch_step_fused(plan, X, ref, k, u, f, dt, V, A, s);
    }
    IP_TRY(launch_forces(plan, X, ref, k, plan->Fbuf, V, A, nullptr, s));
    IP_TRY(launch_interp(plan, X, u, plan->Ubuf, s));
    if (f) IP_TRY(launch_spread(plan, X, plan->Fbuf, f, s));
    return launch_update(plan, X, plan->Ubuf, plan->Fbuf, k, dt, s);
}

ip_status ip_forces_jvp(ip_plan *plan, const double *X, const double *dX,
                        const ip_reference *ref, const ip_constants *k, double *dF,
                        void *stream) {
    IP_TRY(check_plan(plan));
    if (plan->prec != IP_F64)
        return (ipibm_set_error("derivatives need an IP_F64 plan"), IP_ERR_UNSUPPORTED);
    IP_TRY(check_ref_k(plan, ref, k, false));
    if (plan->N > 0 && (!X || !dX || !dF)) return arg_error("NULL array");
    if (!aligned(X, 8) || !aligned(dX, 8) || !aligned(dF, 8)) return arg_error("misaligned array");
    return launch_forces_jvp(plan, X, dX, ref, k, nullptr, dF, nullptr, nullptr,
                             (hipStream_t)stream);
}

ip_status ip_step_vjp(ip_plan *plan, const double *X, const ip_reference *ref,
                      const ip_constants *k, const double *u, double dt, const double *lam_next,
                      double *lam, double *gk, double *gu, void *stream) {
    IP_TRY(check_plan(plan));
    if (plan->prec != IP_F64)
        return (ipibm_set_error("derivatives need an IP_F64 plan"), IP_ERR_UNSUPPORTED);
    if (!plan->has_grid) return arg_error("plan has no grid");
    IP_TRY(check_ref_k(plan, ref, k, true));
    if (plan->N > 0 && (!X || !u || !lam_next || !lam)) return arg_error("NULL array");
    if (!aligned(X, 8) || !aligned(u, 8) || !aligned(lam_next, 8) || !aligned(lam, 8) ||
        !aligned(gk, 8) || !aligned(gu, 8))
        return arg_error("misaligned array");
    hipStream_t s = (hipStream_t)stream;
    if (plan->fused_all) {
        // the fused reverse step reads the same packed records as the step
        const bool bound = ref == &plan->bref;
        if (!bound || plan->packed != 1) {
            IP_TRY(launch_pack_reference(plan, ref, s));
            plan->packed = bound ? 1 : 2;
        }
        return launch_step_vjp_fused(plan, X, ref, k, (const double *)u, dt, lam_next, lam, gk,
                                     (double *)gu, s);
    }
    if (!plan->bwd_dots && plan->E + plan->F > 0)
        IP_TRY(alloc_bytes((void **)&plan->bwd_dots, (size_t)(plan->E + plan->F) * 2 * sizeof(double)));
    return launch_step_vjp(plan, X, ref, k, (const double *)u, dt, lam_next, lam, gk,
                           (double *)gu, s);
}

ip_status ibm_interp_vjp(ip_plan *plan, const double *X, const double *u, const double *dU,
                         double *gX, double *gu, void *stream) {
    IP_TRY(check_plan(plan));
    if (plan->prec != IP_F64)
        return (ipibm_set_error("derivatives need an IP_F64 plan"), IP_ERR_UNSUPPORTED);
    if (!plan->has_grid) return arg_error("plan has no grid");
    if (plan->N > 0 && (!X || !u || !dU)) return arg_error("NULL array");
    if (!aligned(X, 8) || !aligned(u, 8) || !aligned(dU, 8) || !aligned(gX, 8) || !aligned(gu, 8))
        return arg_error("misaligned array");
    return launch_interp_vjp(plan, X, u, dU, gX, gu, (hipStream_t)stream);
}

ip_status ip_taylor(ip_plan *plan, const double *X, const double *Dstar, double *D,
                    double *loss, double *gX, void *stream) {
    IP_TRY(check_plan(plan));
    if (plan->N > 0 && !X) return arg_error("X is NULL");
    if (Dstar && (!loss || !gX)) return arg_error("loss and gX are required with Dstar");
    if (!aligned(X, 8)) return arg_error("misaligned X");
    return launch_taylor(plan, X, Dstar, D, loss, gX, (hipStream_t)stream);
}

ip_status ip_plan_status(ip_plan *plan, void *stream, uint32_t *flags) {
    IP_TRY(check_plan(plan));
    uint32_t v = 0;
    hipStream_t s = (hipStream_t)stream;
    IP_HIP_CHECK(hipMemcpyAsync(&v, plan->status, sizeof(v), hipMemcpyDeviceToHost, s));
    IP_HIP_CHECK(hipStreamSynchronize(s));
    IP_HIP_CHECK(hipMemsetAsync(plan->status, 0, sizeof(uint32_t), s));
    IP_HIP_CHECK(hipStreamSynchronize(s));
    if (flags) *flags = v;
    if (v & IP_STATUS_NONFINITE) return IP_ERR_NONFINITE;
    if (v & IP_STATUS_DEGENERATE) return IP_ERR_DEGENERATE;
    return IP_OK;
}

}  // extern "C"
