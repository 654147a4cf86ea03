// Host preprocessing of a P2 surface mesh: topology validation, the double
// Morton permutation of Sec. 5, renumbering, node incidence, singular
// element-pair lists (Sec. 4.2) and the sparsity pattern of the mass matrix.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <unordered_map>

#include "mbem_internal.h"

namespace mbem {

namespace {

// Spread the low 21 bits of v so that bit b lands on bit 3b.
inline uint64_t spread_bits3(uint64_t v) {
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

inline uint64_t quantise(double x, double lo, double ext) {
    double q = std::floor((x - lo) / ext * 2097152.0);  // 2^21 cells per side
    if (q < 0.0) q = 0.0;
    if (q > 2097151.0) q = 2097151.0;
    return (uint64_t)q;
}

inline uint64_t zorder(const double p[3], const double lo[3], double ext) {
    return spread_bits3(quantise(p[0], lo[0], ext)) |
           (spread_bits3(quantise(p[1], lo[1], ext)) << 1) |
           (spread_bits3(quantise(p[2], lo[2], ext)) << 2);
}

std::vector<int64_t> stable_order(const std::vector<uint64_t> &key) {
    std::vector<int64_t> ord(key.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int64_t a, int64_t b) { return key[a] < key[b]; });
    return ord;
}

}  // namespace

int morton_order_host(const double *xyz, int64_t nn, const int64_t *tri6,
                      int64_t nt, std::vector<int64_t> &node_order,
                      std::vector<int64_t> &tri_order, std::vector<uint64_t> *node_keys) {
    for (int64_t i = 0; i < 3 * nn; ++i)
        if (!std::isfinite(xyz[i])) {
            set_error("node coordinate " + std::to_string(i) + " is not finite");
            return MBEM_EINVAL;
        }
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = xyz[d];
    for (int64_t v = 0; v < nn; ++v)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], xyz[3 * v + d]);
            hi[d] = std::max(hi[d], xyz[3 * v + d]);
        }
    double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    if (!(ext > 0.0)) {
        set_error("degenerate mesh bounding box");
        return MBEM_EMESH;
    }
    std::vector<uint64_t> key(nn);
    for (int64_t v = 0; v < nn; ++v) key[v] = zorder(xyz + 3 * v, lo, ext);
    node_order = stable_order(key);
    if (node_keys) {
        node_keys->resize(nn);
        for (int64_t k = 0; k < nn; ++k) (*node_keys)[k] = key[node_order[k]];
    }
    key.assign(nt, 0);
    for (int64_t t = 0; t < nt; ++t) {
        double c[3];
        for (int d = 0; d < 3; ++d) {
            double s = xyz[3 * tri6[6 * t] + d] + xyz[3 * tri6[6 * t + 1] + d];
            s = s + xyz[3 * tri6[6 * t + 2] + d];
            c[d] = s / 3.0;
        }
        key[t] = zorder(c, lo, ext);
    }
    tri_order = stable_order(key);
    return MBEM_OK;
}

// Legendre roots and weights on [-1, 1] by Newton iteration.
void gauss_legendre(int n, double *x, double *w) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));
        double pn = 0, dpn = 1;
        for (int it = 0; it < 200; ++it) {
            double pm = 1.0, pc = z;             // P_0, P_1
            for (int k = 2; k <= n; ++k) {
                double pk = ((2 * k - 1) * z * pc - (k - 1) * pm) / k;
                pm = pc;
                pc = pk;
            }
            pn = (n == 1) ? z : pc;
            double pprev = (n == 1) ? 1.0 : pm;
            dpn = n * (pprev - z * pn) / (1.0 - z * z);
            double dz = pn / dpn;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        {
            double pm = 1.0, pc = z;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2 * k - 1) * z * pc - (k - 1) * pm) / k;
                pm = pc;
                pc = pk;
            }
            pn = (n == 1) ? z : pc;
            double pprev = (n == 1) ? 1.0 : pm;
            dpn = n * (pprev - z * pn) / (1.0 - z * z);
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dpn * dpn);
    }
}

int build_mesh_host(const double *xyz_in, int64_t nn, const int64_t *tri_in,
                    int64_t nt, mbem_mesh *m) {
    if (nn < 4 || nt < 4 || nn > (1LL << 29) || nt > (1LL << 28)) {
        set_error("mesh sizes out of range");
        return MBEM_EINVAL;
    }
    // ---- index checks and vertex / mid-edge roles
    std::vector<int8_t> role(nn, 0);  // 1 vertex, 2 mid-edge
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 6; ++k) {
            int64_t v = tri_in[6 * t + k];
            if (v < 0 || v >= nn) {
                set_error("triangle node index out of range");
                return MBEM_EINVAL;
            }
            int8_t r = k < 3 ? 1 : 2;
            if (role[v] && role[v] != r) {
                set_error("node used both as a vertex and as a mid-edge node");
                return MBEM_EMESH;
            }
            role[v] = r;
            for (int l = 0; l < k; ++l)
                if (tri_in[6 * t + l] == v) {
                    set_error("repeated node inside a triangle");
                    return MBEM_EMESH;
                }
        }
    for (int64_t v = 0; v < nn; ++v)
        if (!role[v]) {
            set_error("node not referenced by any triangle");
            return MBEM_EMESH;
        }
    // ---- every edge in exactly two triangles, opposite directions, one mid
    struct EdgeUse { int64_t t; int a; bool fwd; int64_t mid; };
    std::unordered_map<uint64_t, std::vector<EdgeUse>> edges;
    edges.reserve(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int a = 0; a < 3; ++a) {
            int64_t u = tri_in[6 * t + a], v = tri_in[6 * t + (a + 1) % 3];
            uint64_t key = (uint64_t)std::min(u, v) << 32 | (uint64_t)std::max(u, v);
            edges[key].push_back({t, a, u < v, tri_in[6 * t + 3 + a]});
        }
    for (auto &kv : edges) {
        const auto &u = kv.second;
        if (u.size() != 2 || u[0].fwd == u[1].fwd || u[0].mid != u[1].mid) {
            set_error("mesh is not a closed, consistently oriented P2 surface");
            return MBEM_EMESH;
        }
    }
    // ---- Morton permutation and renumbering
    std::vector<int64_t> no, to;
    MBEM_TRY(morton_order_host(xyz_in, nn, tri_in, nt, no, to, &m->node_key));
    std::vector<int64_t> rank(nn);
    for (int64_t k = 0; k < nn; ++k) rank[no[k]] = k;
    m->nn = nn;
    m->nt = nt;
    m->node_order = no;
    m->tri_order = to;
    m->xyz.resize(3 * nn);
    m->amax = 0.0;
    for (int64_t k = 0; k < nn; ++k) {
        double r2 = 0;
        for (int d = 0; d < 3; ++d) {
            m->xyz[3 * k + d] = xyz_in[3 * no[k] + d];
            r2 += m->xyz[3 * k + d] * m->xyz[3 * k + d];
        }
        m->amax = std::max(m->amax, std::sqrt(r2));
    }
    m->tri.resize(6 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 6; ++k)
            m->tri[6 * t + k] = (int32_t)rank[tri_in[6 * to[t] + k]];
    return MBEM_OK;
}

}  // namespace mbem

// ------------------------------------------------------------------------
// incidence, singular pairs and mass pattern on the renumbered mesh
// ------------------------------------------------------------------------
namespace mbem {

// perm code: three 2-bit local vertex indices (re-indexed order)
static inline int32_t pack_perm(int a, int b, int c) { return a | (b << 2) | (c << 4); }

int build_tables(const mbem_mesh *m, MeshTables &T) {
    const int64_t nn = m->nn, nt = m->nt;
    const int32_t *tri = m->tri.data();
    // node incidence
    T.inc_ptr.assign(nn + 1, 0);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 6; ++k) T.inc_ptr[tri[6 * t + k] + 1]++;
    for (int64_t v = 0; v < nn; ++v) T.inc_ptr[v + 1] += T.inc_ptr[v];
    T.inc.assign(T.inc_ptr[nn], 0);
    {
        std::vector<int32_t> fill(T.inc_ptr.begin(), T.inc_ptr.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (int k = 0; k < 6; ++k) T.inc[fill[tri[6 * t + k]]++] = (int32_t)(t * 8 + k);
    }
    // singular pairs: for every test triangle e, all triangles f sharing at
    // least one vertex node, with both re-indexed so that the shared
    // vertices come first, ordered along e's counter-clockwise edge.
    for (int64_t e = 0; e < nt; ++e) {
        std::vector<int32_t> cand;
        for (int a = 0; a < 3; ++a) {
            int32_t v = tri[6 * e + a];
            for (int32_t s = T.inc_ptr[v]; s < T.inc_ptr[v + 1]; ++s)
                if ((T.inc[s] & 7) < 3) cand.push_back(T.inc[s] >> 3);
        }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        for (int32_t f : cand) {
            int pos_e[3], pos_f[3], ns = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    if (tri[6 * e + a] == tri[6 * f + b]) { pos_e[ns] = a; pos_f[ns] = b; ++ns; }
            int32_t pe, pf;
            if (ns == 3) {
                pe = pf = pack_perm(0, 1, 2);
            } else if (ns == 2) {
                // A -> B must be an edge of e in e's own orientation
                int i0 = 0, i1 = 1;
                if ((pos_e[0] + 1) % 3 != pos_e[1]) { i0 = 1; i1 = 0; }
                int ea = pos_e[i0], eb = pos_e[i1], fa = pos_f[i0], fb = pos_f[i1];
                pe = pack_perm(ea, eb, 3 - ea - eb);
                pf = pack_perm(fa, fb, 3 - fa - fb);
            } else {
                pe = pack_perm(pos_e[0], (pos_e[0] + 1) % 3, (pos_e[0] + 2) % 3);
                pf = pack_perm(pos_f[0], (pos_f[0] + 1) % 3, (pos_f[0] + 2) % 3);
            }
            T.spairs.push_back((int32_t)e);
            T.spairs.push_back(f);
            T.spairs.push_back(ns);
            T.spairs.push_back(pe | (pf << 6));
            T.n_single[ns]++;
        }
    }
    // mass pattern: nodes sharing a triangle
    std::vector<std::vector<int32_t>> rows(nn);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 6; ++k)
            for (int l = 0; l < 6; ++l) rows[tri[6 * t + k]].push_back(tri[6 * t + l]);
    T.m_ptr.assign(nn + 1, 0);
    for (int64_t v = 0; v < nn; ++v) {
        auto &r = rows[v];
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        T.m_ptr[v + 1] = T.m_ptr[v] + (int32_t)r.size();
    }
    T.m_col.resize(T.m_ptr[nn]);
    for (int64_t v = 0; v < nn; ++v)
        std::copy(rows[v].begin(), rows[v].end(), T.m_col.begin() + T.m_ptr[v]);
    T.m_slot.resize(36 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 6; ++k)
            for (int l = 0; l < 6; ++l) {
                int32_t i = tri[6 * t + k], j = tri[6 * t + l];
                auto b = T.m_col.begin() + T.m_ptr[i], en = T.m_col.begin() + T.m_ptr[i + 1];
                T.m_slot[36 * t + 6 * k + l] = (int32_t)(std::lower_bound(b, en, j) - T.m_col.begin());
            }
    // trial chunks: kChunk Morton-consecutive triangles, their distinct
    // nodes ("slots", ascending) and, per slot, the (triangle, local node)
    // pairs that touch it
    const int64_t nch = (nt + kChunk - 1) / kChunk;
    T.chunks.assign(nch * kChunkRec, 0);
    for (int64_t k = 0; k < nch; ++k) {
        int32_t *rec = T.chunks.data() + k * kChunkRec;
        std::vector<std::pair<int32_t, int32_t>> uses;   // (node, fs*8 + loc)
        for (int fs = 0; fs < kChunk; ++fs) {
            const int64_t f = k * kChunk + fs;
            if (f >= nt) break;
            for (int l = 0; l < 6; ++l) uses.push_back({tri[6 * f + l], fs * 8 + l});
        }
        std::sort(uses.begin(), uses.end());
        int ns = 0, ni = 0;
        for (size_t u = 0; u < uses.size(); ++u) {
            if (u == 0 || uses[u].first != uses[u - 1].first) {
                rec[1 + ns] = uses[u].first;
                rec[25 + ns] = ni;
                ++ns;
            }
            rec[50 + ni] = uses[u].second;
            ++ni;
        }
        rec[0] = ns;
        rec[25 + ns] = ni;
    }
    // column ranges: L.rng consecutive nodes; the triangles touching a
    // range (ascending) in batches of L.nb, and per batch the incidences of
    // the range's nodes grouped by node
    {
        constexpr RngLayout L = kRng;
        std::vector<int32_t> &off = T.rng_off, &recs = T.rng_rec;
        const int64_t nrng = (nn + L.rng - 1) / L.rng;
        off.assign(nrng + 1, 0);
        recs.clear();
        std::vector<int32_t> rtris;
        for (int64_t r = 0; r < nrng; ++r) {
            const int64_t j0 = r * L.rng, j1 = std::min<int64_t>(nn, j0 + L.rng);
            rtris.clear();
            for (int64_t j = j0; j < j1; ++j)
                for (int32_t q = T.inc_ptr[j]; q < T.inc_ptr[j + 1]; ++q) rtris.push_back(T.inc[q] >> 3);
            std::sort(rtris.begin(), rtris.end());
            rtris.erase(std::unique(rtris.begin(), rtris.end()), rtris.end());
            for (size_t b0 = 0; b0 < rtris.size(); b0 += L.nb) {
                const size_t base = recs.size();
                recs.resize(base + L.rec(), 0);
                int32_t *rec = recs.data() + base;
                const int nb = (int)std::min<size_t>(L.nb, rtris.size() - b0);
                std::vector<std::pair<int32_t, int32_t>> uses;   // (range-local node, fb*8 + loc)
                rec[0] = nb;
                for (int fb = 0; fb < nb; ++fb) {
                    const int32_t f = rtris[b0 + fb];
                    rec[1 + fb] = f;
                    for (int l = 0; l < 6; ++l) {
                        const int32_t v = tri[6 * (int64_t)f + l];
                        if (v >= j0 && v < j1) uses.push_back({(int32_t)(v - j0), fb * 8 + l});
                    }
                }
                std::sort(uses.begin(), uses.end());
                size_t u = 0;
                for (int jl = 0; jl <= L.rng; ++jl) {
                    while (u < uses.size() && uses[u].first < jl) ++u;
                    rec[L.off() + jl] = (int32_t)u;
                }
                for (size_t k = 0; k < uses.size(); ++k) rec[L.inc() + k] = uses[k].second;
            }
            off[r + 1] = (int32_t)(recs.size() / L.rec());
        }
    }
    // Colour classes (greedy in Morton order, then balanced) so that the
    // regular-pair fill can add to Z with plain read-modify-write: inside one
    // launch no two test triangles share a node (disjoint rows) and no two
    // trial chunks share a node (disjoint columns).  Balancing moves items from classes above the mean
    // size to smaller classes they do not conflict with, so that every
    // launch has about the same number of workgroups.
    auto colour = [&](int64_t nitems, auto nodes_of, std::vector<int32_t> &list,
                      std::vector<int32_t> &off) {
        std::vector<std::vector<int32_t>> users(nn);
        std::vector<std::vector<int32_t>> item_nodes(nitems);
        std::vector<int32_t> col(nitems, -1);
        int ncol = 0;
        for (int64_t it = 0; it < nitems; ++it) {
            nodes_of(it, item_nodes[it]);
            std::vector<char> used(ncol + 1, 0);
            for (int32_t v : item_nodes[it])
                for (int32_t o : users[v]) used[col[o]] = 1;
            int c = 0;
            while (c < ncol && used[c]) ++c;
            col[it] = c;
            ncol = std::max(ncol, c + 1);
            for (int32_t v : item_nodes[it]) users[v].push_back((int32_t)it);
        }
        std::vector<int64_t> size(ncol, 0);
        for (int64_t it = 0; it < nitems; ++it) size[col[it]]++;
        const int64_t target = (nitems + ncol - 1) / ncol;
        for (int round = 0; round < 8; ++round) {
            int64_t moved = 0;
            for (int64_t it = 0; it < nitems; ++it) {
                const int c = col[it];
                if (size[c] <= target) continue;
                std::vector<char> used(ncol, 0);
                for (int32_t v : item_nodes[it])
                    for (int32_t o : users[v])
                        if (o != it) used[col[o]] = 1;
                int best = -1;
                for (int d = 0; d < ncol; ++d)
                    if (!used[d] && size[d] < target && (best < 0 || size[d] < size[best])) best = d;
                if (best >= 0) { col[it] = best; --size[c]; ++size[best]; ++moved; }
            }
            if (!moved) break;
        }
        off.assign(ncol + 1, 0);
        for (int64_t it = 0; it < nitems; ++it) off[col[it] + 1]++;
        for (int c = 0; c < ncol; ++c) off[c + 1] += off[c];
        list.assign(nitems, 0);
        std::vector<int32_t> fill(off.begin(), off.end() - 1);
        for (int64_t it = 0; it < nitems; ++it) list[fill[col[it]]++] = (int32_t)it;
    };
    colour(nt, [&](int64_t e, std::vector<int32_t> &out) {
        for (int k = 0; k < 6; ++k) out.push_back(tri[6 * e + k]);
    }, T.tcol_list, T.tcol_off);
    {
        // the triangles of a node have distinct test colours: the lowest one
        // writes the node's rows first
        std::vector<int32_t> tcolour(nt), low(nn, INT32_MAX);
        for (size_t c = 0; c + 1 < T.tcol_off.size(); ++c)
            for (int32_t q = T.tcol_off[c]; q < T.tcol_off[c + 1]; ++q) tcolour[T.tcol_list[q]] = (int32_t)c;
        for (int64_t e = 0; e < nt; ++e)
            for (int k = 0; k < 6; ++k) low[tri[6 * e + k]] = std::min(low[tri[6 * e + k]], tcolour[e]);
        T.row_first.assign(nt, 0);
        for (int64_t e = 0; e < nt; ++e)
            for (int k = 0; k < 6; ++k)
                if (tcolour[e] == low[tri[6 * e + k]]) T.row_first[e] |= 1 << k;
    }
    colour(nch, [&](int64_t k, std::vector<int32_t> &out) {
        const int32_t *rec = T.chunks.data() + k * kChunkRec;
        for (int s2 = 0; s2 < rec[0]; ++s2) out.push_back(rec[1 + s2]);
    }, T.ccol_list, T.ccol_off);
    {
        // likewise the chunks of a node: the lowest chunk colour writes the
        // node's columns first
        std::vector<int32_t> ccolour(nch), low(nn, INT32_MAX);
        for (size_t c = 0; c + 1 < T.ccol_off.size(); ++c)
            for (int32_t q = T.ccol_off[c]; q < T.ccol_off[c + 1]; ++q) ccolour[T.ccol_list[q]] = (int32_t)c;
        for (int64_t k = 0; k < nch; ++k) {
            const int32_t *rec = T.chunks.data() + k * kChunkRec;
            for (int s2 = 0; s2 < rec[0]; ++s2) low[rec[1 + s2]] = std::min(low[rec[1 + s2]], ccolour[k]);
        }
        T.col_first.assign(nch, 0);
        for (int64_t k = 0; k < nch; ++k) {
            const int32_t *rec = T.chunks.data() + k * kChunkRec;
            for (int s2 = 0; s2 < rec[0]; ++s2)
                if (ccolour[k] == low[rec[1 + s2]]) T.col_first[k] |= 1 << s2;
        }
    }
    return MBEM_OK;
}

}  // namespace mbem
