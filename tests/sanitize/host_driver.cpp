// Host preprocessing under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Built with g++ (host code only, no device code) together with
// paper_2604_21181_amd/csrc/host_mesh.cpp by tests/test_sanitizers.py.
// Reads a P2 mesh (int64 nn, int64 nt, double xyz[3 nn], int64 tri[6 nt]),
// runs mesh validation, the double Morton permutation and the table build
// (incidence, singular pairs, mass pattern, trial chunks, colour classes),
// checks the invariants of the colour classes (every item in exactly one
// class; no two items of a class share a node) and of the column ranges of
// the regular-pair fill, runs the rejection paths
// on corrupted copies, and writes node_order[nn], tri_order[nt] (int64) and
// the four singular-pair counts to the output file.  Exit status 0 = every
// check held.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <limits>
#include <set>
#include <string>
#include <vector>

#include "mbem_internal.h"

namespace mbem {
static std::string g_last;
void set_error(const std::string &msg) { g_last = msg; }
}  // namespace mbem

using namespace mbem;

static int fail(const char *what) {
    std::fprintf(stderr, "host_driver: %s\n", what);
    return 1;
}

// every item in exactly one class, and the items of one class share no node
template <typename NodesOf>
static int check_classes(const std::vector<int32_t> &list, const std::vector<int32_t> &off, int64_t nitems,
                         NodesOf nodes_of, const char *what) {
    if (off.empty() || off.front() != 0 || off.back() != (int32_t)list.size()) return fail(what);
    std::vector<int> seen(nitems, 0);
    for (size_t c = 0; c + 1 < off.size(); ++c) {
        std::set<int32_t> used;
        for (int32_t q = off[c]; q < off[c + 1]; ++q) {
            const int32_t it = list[q];
            if (it < 0 || it >= nitems) return fail(what);
            seen[it]++;
            std::vector<int32_t> nodes;
            nodes_of(it, nodes);
            std::set<int32_t> own(nodes.begin(), nodes.end());
            for (int32_t v : own)
                if (!used.insert(v).second) return fail(what);
        }
    }
    for (int64_t i = 0; i < nitems; ++i)
        if (seen[i] != 1) return fail(what);
    return 0;
}

int main(int argc, char **argv) {
    if (argc != 3) return fail("usage: host_driver in.bin out.bin");
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return fail("cannot open input");
    int64_t nn = 0, nt = 0;
    if (std::fread(&nn, 8, 1, f) != 1 || std::fread(&nt, 8, 1, f) != 1 || nn < 1 || nt < 1) return fail("header");
    std::vector<double> xyz(3 * nn);
    std::vector<int64_t> tri(6 * nt);
    if (std::fread(xyz.data(), 8, xyz.size(), f) != xyz.size() ||
        std::fread(tri.data(), 8, tri.size(), f) != tri.size())
        return fail("body");
    std::fclose(f);

    mbem_mesh m;
    if (build_mesh_host(xyz.data(), nn, tri.data(), nt, &m) != MBEM_OK) return fail(g_last.c_str());
    MeshTables T;
    if (build_tables(&m, T) != MBEM_OK) return fail(g_last.c_str());

    // permutations are bijections
    std::vector<int> hit(nn, 0), hitt(nt, 0);
    for (int64_t k = 0; k < nn; ++k) hit[m.node_order[k]]++;
    for (int64_t k = 0; k < nt; ++k) hitt[m.tri_order[k]]++;
    for (int64_t k = 0; k < nn; ++k)
        if (hit[k] != 1) return fail("node permutation");
    for (int64_t k = 0; k < nt; ++k)
        if (hitt[k] != 1) return fail("triangle permutation");

    auto tri_nodes = [&](int32_t e, std::vector<int32_t> &out) {
        out.assign(m.tri.begin() + 6 * e, m.tri.begin() + 6 * e + 6);
    };
    if (check_classes(T.tcol_list, T.tcol_off, nt, tri_nodes, "test-triangle colour classes")) return 1;
    const int64_t nch = (nt + 3) / 4;
    auto chunk_nodes = [&](int32_t k, std::vector<int32_t> &out) {
        out.clear();
        for (int64_t t = 4 * (int64_t)k; t < std::min<int64_t>(nt, 4 * (int64_t)k + 4); ++t)
            for (int a = 0; a < 6; ++a) out.push_back(m.tri[6 * t + a]);
    };
    if (check_classes(T.ccol_list, T.ccol_off, nch, chunk_nodes, "trial-chunk colour classes")) return 1;
    // column ranges: the batches of a range hold exactly the triangles that
    // touch it, ascending, and every (triangle, local node) incidence of a
    // node of the range once, under that node
    {
        const RngLayout L = kRng;
        const int64_t nrng = (nn + L.rng - 1) / L.rng;
        if ((int64_t)T.rng_off.size() != nrng + 1 || T.rng_off[0] != 0 ||
            (int64_t)T.rng_rec.size() != (int64_t)T.rng_off.back() * L.rec())
            return fail("column-range offsets");
        for (int64_t r = 0; r < nrng; ++r) {
            const int64_t j0 = r * L.rng, j1 = std::min<int64_t>(nn, j0 + L.rng);
            std::set<int32_t> want;
            int64_t want_inc = 0;
            for (int64_t t = 0; t < nt; ++t)
                for (int k = 0; k < 6; ++k)
                    if (m.tri[6 * t + k] >= j0 && m.tri[6 * t + k] < j1) { want.insert((int32_t)t); ++want_inc; }
            std::vector<int32_t> got;
            int64_t got_inc = 0;
            for (int32_t b = T.rng_off[r]; b < T.rng_off[r + 1]; ++b) {
                const int32_t *rec = T.rng_rec.data() + (int64_t)b * L.rec();
                const int nb = rec[0];
                if (nb < 1 || nb > L.nb) return fail("column-range batch size");
                for (int fb = 0; fb < nb; ++fb) got.push_back(rec[1 + fb]);
                if (rec[L.off()] != 0) return fail("column-range incidence offsets");
                for (int jl = 0; jl < L.rng; ++jl) {
                    if (rec[L.off() + jl + 1] < rec[L.off() + jl] || rec[L.off() + jl + 1] > 6 * nb)
                        return fail("column-range incidence offsets");
                    for (int32_t u = rec[L.off() + jl]; u < rec[L.off() + jl + 1]; ++u) {
                        const int fl = rec[L.inc() + u], fb = fl >> 3, loc = fl & 7;
                        if (fb >= nb || loc > 5 || m.tri[6 * (int64_t)rec[1 + fb] + loc] != j0 + jl)
                            return fail("column-range incidence");
                        ++got_inc;
                    }
                }
            }
            if (!std::is_sorted(got.begin(), got.end()) || std::set<int32_t>(got.begin(), got.end()) != want ||
                got.size() != want.size() || got_inc != want_inc)
                return fail("column-range triangles");
        }
    }
    // every node's rows have exactly one first writer among its triangles
    {
        std::vector<int> firsts(nn, 0);
        if ((int64_t)T.row_first.size() != nt) return fail("row first writers");
        for (int64_t e = 0; e < nt; ++e)
            for (int k = 0; k < 6; ++k)
                if ((T.row_first[e] >> k) & 1) firsts[m.tri[6 * e + k]]++;
        for (int64_t v = 0; v < nn; ++v)
            if (firsts[v] != 1) return fail("row first writers");
        // and exactly one first chunk among the chunks of a node
        std::vector<int> cf(nn, 0);
        if ((int64_t)T.col_first.size() != nch) return fail("column first writers");
        for (int64_t k = 0; k < nch; ++k) {
            const int32_t *rec = T.chunks.data() + k * kChunkRec;
            for (int s2 = 0; s2 < rec[0]; ++s2)
                if ((T.col_first[k] >> s2) & 1) cf[rec[1 + s2]]++;
        }
        for (int64_t v = 0; v < nn; ++v)
            if (cf[v] != 1) return fail("column first writers");
    }
    // mass pattern: CSR rows sorted, every column in range
    if ((int64_t)T.m_ptr.size() != nn + 1) return fail("mass pattern rows");
    for (int64_t i = 0; i < nn; ++i)
        for (int32_t s = T.m_ptr[i]; s < T.m_ptr[i + 1]; ++s) {
            if (T.m_col[s] < 0 || T.m_col[s] >= nn) return fail("mass pattern column");
            if (s > T.m_ptr[i] && T.m_col[s] <= T.m_col[s - 1]) return fail("mass pattern order");
        }

    // rejection paths on corrupted copies: each must fail with its code
    {
        std::vector<double> bad = xyz;
        bad[3 * (nn / 2) + 1] = std::numeric_limits<double>::quiet_NaN();
        mbem_mesh b;
        if (build_mesh_host(bad.data(), nn, tri.data(), nt, &b) != MBEM_EINVAL) return fail("NaN coordinate");
    }
    {
        std::vector<int64_t> bad = tri;
        bad[6 * (nt - 1) + 4] = nn;
        mbem_mesh b;
        if (build_mesh_host(xyz.data(), nn, bad.data(), nt, &b) != MBEM_EINVAL) return fail("index out of range");
    }
    {
        std::vector<int64_t> bad = tri;
        std::swap(bad[6 * 0 + 1], bad[6 * 0 + 2]);   // one triangle turned over
        mbem_mesh b;
        if (build_mesh_host(xyz.data(), nn, bad.data(), nt, &b) != MBEM_EMESH) return fail("orientation");
    }
    {
        mbem_mesh b;   // the last triangle dropped: an open surface with unused nodes
        if (build_mesh_host(xyz.data(), nn, tri.data(), nt - 1, &b) != MBEM_EMESH) return fail("open surface");
    }
    {
        mbem_mesh b;
        if (build_mesh_host(xyz.data(), 3, tri.data(), nt, &b) != MBEM_EINVAL) return fail("tiny mesh");
    }

    FILE *o = std::fopen(argv[2], "wb");
    if (!o) return fail("cannot open output");
    std::fwrite(m.node_order.data(), 8, nn, o);
    std::fwrite(m.tri_order.data(), 8, nt, o);
    std::fwrite(T.n_single, 8, 4, o);
    std::fclose(o);
    return 0;
}
