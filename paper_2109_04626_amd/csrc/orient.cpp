// Phase II of Algorithms 1 and 2: orientation of the learned skeleton
// into a CPDAG from the separating sets (Sec. 2.2.1, Phase II listing; the
// reverse algorithm reuses it unchanged, Sec. 3.2.2).
//
// Marks: D[a*p + b] = 1 when the edge between a and b may point a -> b, so
// an undirected edge has both marks and a directed edge a -> b has
// D[a][b] = 1, D[b][a] = 0.
//
// 1. Unshielded triples i - k - j (i, j non-adjacent): if k is not in
//    S(i, j), orient i -> k <- j.  Triples are visited in lexicographic
//    (i, j, k) order and an arrowhead that would point back into an edge
//    already directed the other way is not placed (the first orientation
//    stands).
// 2. Until nothing changes, orient an undirected edge a - b as a -> b when
//    R1  some c -> a with c, b non-adjacent;
//    R2  some c with a -> c -> b;
//    R3  two non-adjacent c, d with a - c -> b and a - d -> b;
//    R4  some c, d with a - c, c -> d -> b, c and b non-adjacent, a and d
//        adjacent.
#include <algorithm>
#include <array>
#include <cstring>
#include <vector>

#include "fpc_internal.h"

namespace {

inline int64_t pair_index(int i, int j, int p)
{
    return (int64_t)i * p - (int64_t)i * (i + 1) / 2 + (j - i - 1);
}

}  // namespace

extern "C" int fpc_orient(int p, const uint8_t *adj, const int32_t *sep_level, const int8_t *sep_kind,
                          const int64_t *sep_off, const int32_t *sep_nodes, uint8_t *cpdag_out)
{
    if (p < 1 || !adj || !sep_kind || !sep_off || !cpdag_out) return FPC_EINVAL;
    (void)sep_level;
    const size_t pp = (size_t)p * p;
    std::vector<uint8_t> D(pp);
    auto A = [&](int a, int b) { return adj[(size_t)a * p + b] != 0; };
    std::vector<std::vector<int>> nb(p);
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b)
            if (a != b && A(a, b)) nb[a].push_back(b);
    for (size_t k = 0; k < pp; ++k) D[k] = adj[k] ? 1 : 0;
    auto directed = [&](int a, int b) { return D[(size_t)a * p + b] && !D[(size_t)b * p + a]; };
    auto undirected = [&](int a, int b) { return D[(size_t)a * p + b] && D[(size_t)b * p + a]; };
    // membership of k in S(i, j)
    auto in_sep = [&](int i, int j, int k) -> bool {
        const int64_t pr = pair_index(i, j, p);
        if (sep_kind[pr] == FPC_SEP_ALL_BUT) return true;  // every variable but i, j
        if (sep_kind[pr] != FPC_SEP_LIST) return false;
        for (int64_t t = sep_off[pr]; t < sep_off[pr + 1]; ++t)
            if (sep_nodes[t] == k) return true;
        return false;
    };
    // 1. v-structures, in lexicographic (i, j, k) order
    std::vector<std::array<int, 3>> tri;
    for (int k = 0; k < p; ++k)
        for (size_t x = 0; x < nb[k].size(); ++x)
            for (size_t y = x + 1; y < nb[k].size(); ++y) {
                const int i = nb[k][x], j = nb[k][y];  // i < j: lists are sorted
                if (!A(i, j) && !in_sep(i, j, k)) tri.push_back({i, j, k});
            }
    std::sort(tri.begin(), tri.end());
    for (const auto &t : tri) {
        const int i = t[0], j = t[1], k = t[2];
        // i -> k <- j unless an edge is already directed away from k
        if (!directed(k, i) && !directed(k, j)) {
            D[(size_t)k * p + i] = 0;
            D[(size_t)k * p + j] = 0;
        }
    }
    // 2. propagation: sweeps over (a, b) in row-major order until one sweep
    //    changes nothing; an orientation is visible to the rest of its sweep
    bool changed = true;
    while (changed) {
        changed = false;
        for (int a = 0; a < p; ++a)
            for (int b : nb[a]) {
                if (!undirected(a, b)) continue;
                bool orient = false;
                for (int c : nb[a]) {
                    if (c == b) continue;
                    if (directed(c, a) && !A(c, b)) orient = true;                 // R1
                    else if (directed(a, c) && directed(c, b)) orient = true;       // R2
                    if (orient) break;
                }
                for (size_t x = 0; x < nb[a].size() && !orient; ++x) {            // R3
                    const int c = nb[a][x];
                    if (c == b || !undirected(a, c) || !directed(c, b)) continue;
                    for (size_t y = x + 1; y < nb[a].size() && !orient; ++y) {
                        const int d = nb[a][y];
                        if (d == b || !undirected(a, d) || !directed(d, b)) continue;
                        if (!A(c, d)) orient = true;
                    }
                }
                for (size_t x = 0; x < nb[a].size() && !orient; ++x) {            // R4
                    const int c = nb[a][x];
                    if (c == b || !undirected(a, c) || A(c, b)) continue;
                    for (int d : nb[c]) {
                        if (d == a || d == b) continue;
                        if (directed(c, d) && directed(d, b) && A(a, d)) {
                            orient = true;
                            break;
                        }
                    }
                }
                if (orient) {
                    D[(size_t)b * p + a] = 0;
                    changed = true;
                }
            }
    }
    std::memcpy(cpdag_out, D.data(), pp);
    return FPC_OK;
}
