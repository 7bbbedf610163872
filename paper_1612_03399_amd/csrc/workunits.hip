// workunits.hip -- host-side construction of the fused step's work units.
//
// A work unit is what one workgroup of the fused step processes: a whole body
// when its nodes, elements and LDS layout fit one workgroup, otherwise a patch
// of a larger body.  A patch owns a compact set of the body's nodes (recursive
// bisection of the mesh graph by breadth-first order from a peripheral node)
// and carries every element that touches an owned node, plus the halo of the
// non-owned nodes those elements reach; its forces are exact on the owned
// nodes, which are the only ones it spreads, interpolates and moves.  The
// element records of every unit use node ids local to the unit (owned nodes
// first) and are ordered so that each run of 64 elements touches distinct
// nodes where the mesh allows (the 64 lanes of one instruction then never add
// into the same node accumulator).
#include <algorithm>
#include <numeric>
#include <thread>
#include <vector>

#include "ipibm_internal.h"

namespace {

// Greedy first fit of the elements into groups of 64 with pairwise distinct
// nodes (local ids, -1 = none): element e goes to the lowest group that is not
// full and holds none of its nodes.  The candidate groups are examined 64 at a
// time as a bit mask (the window starts at the lowest group that is not full),
// so one pass over the element's nodes' group lists finds the group.
void conflict_free_order(int count, int width, const int32_t *elem, int n_nodes,
                         std::vector<std::vector<int32_t>> &node_groups,
                         std::vector<int32_t> &group_of, std::vector<int32_t> &order) {
    constexpr int G = 64;
    if ((int)node_groups.size() < n_nodes) node_groups.resize(n_nodes);
    for (int v = 0; v < n_nodes; ++v) node_groups[v].clear();
    std::vector<int32_t> size;          // elements per group
    group_of.resize(count);
    size_t g0 = 0;                      // lowest group that is not full
    uint64_t fullw = 0;                 // bit i: group g0 + i is full
    for (int e = 0; e < count; ++e) {
        size_t base = g0;
        uint64_t full = fullw;
        size_t g;
        for (;;) {
            uint64_t busy = full;
            for (int r = 0; r < width; ++r) {
                const int v = elem[e * width + r];
                if (v < 0) continue;
                for (int32_t gg : node_groups[v]) {
                    const size_t d = (size_t)gg - base;   // wraps for gg < base
                    if (d < 64) busy |= 1ull << d;
                }
            }
            if (busy != ~0ull) {
                g = base + (size_t)__builtin_ctzll(~busy);
                break;
            }
            base += 64;                 // every group of this window is taken
            full = 0;
            for (int i = 0; i < 64 && base + i < size.size(); ++i)
                if (size[base + i] >= G) full |= 1ull << i;
        }
        if (g >= size.size()) size.resize(g + 1, 0);
        group_of[e] = (int32_t)g;
        ++size[g];
        for (int r = 0; r < width; ++r) {
            const int v = elem[e * width + r];
            if (v >= 0) node_groups[v].push_back((int32_t)g);
        }
        if (size[g] >= G && g - g0 < 64) fullw |= 1ull << (g - g0);
        while (g0 < size.size() && size[g0] >= G) {
            ++g0;
            fullw >>= 1;
            if (g0 + 63 < size.size() && size[g0 + 63] >= G) fullw |= 1ull << 63;
        }
    }
    // elements by group, in element order within a group
    std::vector<int32_t> start(size.size() + 1, 0);
    for (size_t i = 0; i < size.size(); ++i) start[i + 1] = start[i] + size[i];
    order.resize(count);
    for (int e = 0; e < count; ++e) order[start[group_of[e]]++] = e;
}

struct Builder {
    const ip_mesh *m;
    WorkUnits &out;
    int whole_max, nmax_unit, fmax_unit, patch_owned;
    std::vector<std::vector<int32_t>> node_groups;
    std::vector<int32_t> loc, order, group_of;

    // Append one unit: `nodes` = global ids (owned first) or empty for a whole
    // body; `edges`, `faces` = global element ids; `local` maps global node
    // id - n0 to the unit's local id.
    void emit(int b, bool whole, const std::vector<int32_t> &nodes, int owned,
              const std::vector<int32_t> &edges, const std::vector<int32_t> &faces,
              const std::vector<int32_t> &local, int64_t n0, int n_unit) {
        WorkUnitHost u;
        u.body = b;
        u.owned = owned;
        u.n_nodes = n_unit;
        u.node_begin = (int64_t)out.nodes.size();
        if (!whole) out.nodes.insert(out.nodes.end(), nodes.begin(), nodes.end());
        u.node_end = (int64_t)out.nodes.size();
        // edges
        loc.resize(4 * edges.size());
        for (size_t i = 0; i < edges.size(); ++i)
            for (int r = 0; r < 4; ++r) {
                const int32_t v = m->edges4[4 * (int64_t)edges[i] + r];
                loc[4 * i + r] = v < 0 ? -1 : local[v - n0];
            }
        conflict_free_order((int)edges.size(), 4, loc.data(), n_unit, node_groups, group_of, order);
        u.edge_begin = (int64_t)out.edge_perm.size();
        for (int32_t i : order) {
            out.edge_perm.push_back(edges[i]);
            for (int r = 0; r < 4; ++r)
                out.edge_lid.push_back(loc[4 * i + r] < 0 ? kNoNode : (uint16_t)loc[4 * i + r]);
        }
        u.edge_end = (int64_t)out.edge_perm.size();
        // faces
        loc.resize(3 * faces.size());
        for (size_t i = 0; i < faces.size(); ++i)
            for (int r = 0; r < 3; ++r) loc[3 * i + r] = local[m->faces[3 * (int64_t)faces[i] + r] - n0];
        conflict_free_order((int)faces.size(), 3, loc.data(), n_unit, node_groups, group_of, order);
        u.face_begin = (int64_t)out.face_perm.size();
        for (int32_t i : order) {
            out.face_perm.push_back(faces[i]);
            for (int r = 0; r < 3; ++r) out.face_lid.push_back((uint16_t)loc[3 * i + r]);
            out.face_lid.push_back(0);
        }
        u.face_end = (int64_t)out.face_perm.size();
        out.units.push_back(u);
    }

    // Breadth-first order of the nodes of `part` (local body ids) from
    // `seed`, over the body graph restricted to the part; nodes not reached
    // (another component) follow in their given order.
    void bfs_order(const std::vector<int32_t> &part, int seed, const std::vector<int32_t> &adj_ptr,
                   const std::vector<int32_t> &adj, std::vector<int32_t> &mark, int stamp,
                   std::vector<int32_t> &res) {
        // mark[v] == stamp: in part, not visited; stamp + 1: visited
        for (int v : part) mark[v] = stamp;
        res.clear();
        res.push_back(seed);
        mark[seed] = stamp + 1;
        for (size_t h = 0; h < res.size(); ++h) {
            const int v = res[h];
            for (int k = adj_ptr[v]; k < adj_ptr[v + 1]; ++k) {
                const int w = adj[k];
                if (mark[w] == stamp) {
                    mark[w] = stamp + 1;
                    res.push_back(w);
                }
            }
        }
        if (res.size() < part.size())
            for (int v : part)
                if (mark[v] == stamp) {
                    mark[v] = stamp + 1;
                    res.push_back(v);
                }
    }

    bool build_body(int b) {
        const int64_t n0 = m->node_off[b], n1 = m->node_off[b + 1];
        const int64_t e0 = m->edge_off[b], e1 = m->edge_off[b + 1];
        const int64_t f0 = m->face_off[b], f1 = m->face_off[b + 1];
        const int n = (int)(n1 - n0);
        std::vector<int32_t> edges(e1 - e0), faces(f1 - f0);
        std::iota(edges.begin(), edges.end(), (int32_t)e0);
        std::iota(faces.begin(), faces.end(), (int32_t)f0);
        if (n <= whole_max && (f1 - f0) <= fmax_unit) {
            std::vector<int32_t> local(n);
            std::iota(local.begin(), local.end(), 0);
            emit(b, true, {}, n, edges, faces, local, n0, n);
            return true;
        }
        // mesh graph of the body (local ids) and node -> element incidence
        std::vector<int32_t> deg(n + 1, 0);
        for (int64_t f = f0; f < f1; ++f)
            for (int r = 0; r < 3; ++r) deg[m->faces[3 * f + r] - n0] += 2;
        std::vector<int32_t> adj_ptr(n + 1, 0);
        for (int v = 0; v < n; ++v) adj_ptr[v + 1] = adj_ptr[v] + deg[v];
        std::vector<int32_t> adj(adj_ptr[n]), fill(adj_ptr.begin(), adj_ptr.end() - 1);
        for (int64_t f = f0; f < f1; ++f) {
            const int i = m->faces[3 * f] - (int)n0, j = m->faces[3 * f + 1] - (int)n0,
                      k = m->faces[3 * f + 2] - (int)n0;
            adj[fill[i]++] = j; adj[fill[i]++] = k;
            adj[fill[j]++] = k; adj[fill[j]++] = i;
            adj[fill[k]++] = i; adj[fill[k]++] = j;
        }
        std::vector<std::vector<int32_t>> node_edges(n), node_faces(n);
        for (int64_t e = e0; e < e1; ++e)
            for (int r = 0; r < 4; ++r) {
                const int32_t v = m->edges4[4 * e + r];
                if (v >= 0) node_edges[v - n0].push_back((int32_t)e);
            }
        for (int64_t f = f0; f < f1; ++f)
            for (int r = 0; r < 3; ++r) node_faces[m->faces[3 * f + r] - n0].push_back((int32_t)f);
        // recursive bisection
        std::vector<int32_t> mark(n, -1), ordr, emark_e(e1 - e0, -1), emark_f(f1 - f0, -1);
        std::vector<int32_t> local(n, -1);
        std::vector<std::vector<int32_t>> stack;
        stack.emplace_back(n);
        std::iota(stack.back().begin(), stack.back().end(), 0);
        int stamp = 0, unit_stamp = 0;
        while (!stack.empty()) {
            std::vector<int32_t> part = std::move(stack.back());
            stack.pop_back();
            if ((int)part.size() > patch_owned) {
                // split at half the breadth-first order from a peripheral node
                bfs_order(part, part[0], adj_ptr, adj, mark, stamp, ordr);
                stamp += 2;
                const int far = ordr.back();
                bfs_order(part, far, adj_ptr, adj, mark, stamp, ordr);
                stamp += 2;
                const size_t h = ordr.size() / 2;
                stack.emplace_back(ordr.begin() + h, ordr.end());
                stack.emplace_back(ordr.begin(), ordr.begin() + h);
                continue;
            }
            // unit: owned nodes, elements touching them, halo
            ++unit_stamp;
            std::vector<int32_t> nodes, ue, uf;
            for (size_t i = 0; i < part.size(); ++i) local[part[i]] = (int32_t)i;
            for (int v : part) nodes.push_back((int32_t)(n0 + v));
            const int owned = (int)part.size();
            for (int v : part) {
                for (int32_t e : node_edges[v])
                    if (emark_e[e - e0] != unit_stamp) {
                        emark_e[e - e0] = unit_stamp;
                        ue.push_back(e);
                    }
                for (int32_t f : node_faces[v])
                    if (emark_f[f - f0] != unit_stamp) {
                        emark_f[f - f0] = unit_stamp;
                        uf.push_back(f);
                    }
            }
            const auto add_halo = [&](int32_t g) {
                const int v = g - (int)n0;
                if (local[v] < 0) {
                    local[v] = (int32_t)nodes.size();
                    nodes.push_back(g);
                }
            };
            for (int32_t e : ue)
                for (int r = 0; r < 4; ++r)
                    if (m->edges4[4 * (int64_t)e + r] >= 0) add_halo(m->edges4[4 * (int64_t)e + r]);
            for (int32_t f : uf)
                for (int r = 0; r < 3; ++r) add_halo(m->faces[3 * (int64_t)f + r]);
            const bool fits = (int)nodes.size() <= nmax_unit && (int)uf.size() <= fmax_unit;
            if (!fits) {
                for (int32_t g : nodes) local[g - n0] = -1;
                if (owned <= 16) return false;       // cannot be made to fit
                // split this part further
                bfs_order(part, part[0], adj_ptr, adj, mark, stamp, ordr);
                stamp += 2;
                bfs_order(part, ordr.back(), adj_ptr, adj, mark, stamp, ordr);
                stamp += 2;
                const size_t h = ordr.size() / 2;
                stack.emplace_back(ordr.begin() + h, ordr.end());
                stack.emplace_back(ordr.begin(), ordr.begin() + h);
                continue;
            }
            emit(b, false, nodes, owned, ue, uf, local, n0, (int)nodes.size());
            for (int32_t g : nodes) local[g - n0] = -1;
        }
        return true;
    }
};

}  // namespace

bool build_work_units(const ip_mesh *m, int whole_max, int nmax_unit, int fmax_unit,
                      int patch_owned, WorkUnits &out) {
    out = WorkUnits{};
    const int B = m->n_bodies;
    // contiguous runs of bodies of about equal size (nodes + elements), one
    // per host thread; concatenated in body order, the result does not depend
    // on the thread count
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int T = std::max(1, std::min({(int)std::min(hw, 16u), B / 16, 16}));
    std::vector<int64_t> cost(B + 1, 0);
    for (int b = 0; b < B; ++b)
        cost[b + 1] = cost[b] + (m->node_off[b + 1] - m->node_off[b]) +
                      (m->edge_off[b + 1] - m->edge_off[b]) + (m->face_off[b + 1] - m->face_off[b]);
    std::vector<int> cut(T + 1, B);
    cut[0] = 0;
    for (int t = 1; t < T; ++t)
        cut[t] = (int)(std::lower_bound(cost.begin(), cost.end(), cost[B] * t / T) - cost.begin());
    for (int t = 1; t <= T; ++t) cut[t] = std::max(cut[t], cut[t - 1]);
    std::vector<WorkUnits> parts(T);
    std::vector<char> ok(T, 1);
    const auto run = [&](int t) {
        try {
            Builder bld{m, parts[t], whole_max, nmax_unit, fmax_unit, patch_owned, {}, {}, {}, {}};
            for (int b = cut[t]; b < cut[t + 1]; ++b)
                if (!bld.build_body(b)) {
                    ok[t] = 0;
                    return;
                }
        } catch (...) {
            ok[t] = 0;
        }
    };
    std::vector<std::thread> threads;
    for (int t = 1; t < T; ++t) threads.emplace_back(run, t);
    run(0);
    for (auto &th : threads) th.join();
    for (int t = 0; t < T; ++t)
        if (!ok[t]) return false;
    for (auto &p : parts) {
        const int64_t dn = (int64_t)out.nodes.size(), de = (int64_t)out.edge_perm.size(),
                      df = (int64_t)out.face_perm.size();
        for (auto u : p.units) {
            u.node_begin += dn;
            u.node_end += dn;
            u.edge_begin += de;
            u.edge_end += de;
            u.face_begin += df;
            u.face_end += df;
            out.units.push_back(u);
        }
        out.nodes.insert(out.nodes.end(), p.nodes.begin(), p.nodes.end());
        out.edge_perm.insert(out.edge_perm.end(), p.edge_perm.begin(), p.edge_perm.end());
        out.edge_lid.insert(out.edge_lid.end(), p.edge_lid.begin(), p.edge_lid.end());
        out.face_perm.insert(out.face_perm.end(), p.face_perm.begin(), p.face_perm.end());
        out.face_lid.insert(out.face_lid.end(), p.face_lid.begin(), p.face_lid.end());
        p = WorkUnits{};
    }
    // largest units first (the tail of the launch runs the small ones), in
    // size classes of 64 nodes; within a class the patches of a body stay
    // together, so that units running side by side share their grid lines
    // (the unit kernels deal consecutive units to one XCD in chunks, so
    // that such neighbours also share an L2)
    std::vector<int32_t> idx(out.units.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
        const int cx = out.units[x].n_nodes / 64, cy = out.units[y].n_nodes / 64;
        if (cx != cy) return cx > cy;
        return out.units[x].body < out.units[y].body;
    });
    std::vector<WorkUnitHost> sorted;
    sorted.reserve(idx.size());
    for (int i : idx) sorted.push_back(out.units[i]);
    out.units.swap(sorted);
    return true;
}
