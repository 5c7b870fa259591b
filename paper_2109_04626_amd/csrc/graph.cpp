// Host graph logic: candidate sets adj(G,i,j) n path(G,i,j) (Sec. 2.1
// definitions; used by every level of Algorithm 2).
//
// For an edge (i,j) of G and a neighbour k of i (k != j), k lies on a simple
// path between i and j iff k reaches j in G - i, i.e. iff the edges (i,k)
// and (i,j) lie on a common simple cycle, i.e. iff they belong to the same
// biconnected component (block).  Symmetrically for neighbours of j.  One
// Hopcroft-Tarjan pass labels every edge with its block, after which each
// candidate set is a merge of two filtered neighbour lists: O(p + E) for
// the labelling plus O(deg i + deg j) per edge.
#include <algorithm>
#include <cstring>

#include "fpc_internal.h"

namespace fpc {

namespace {

struct Adjacency {
    std::vector<int32_t> off, nb, eid;  // CSR of neighbours and undirected edge ids
    std::vector<int32_t> eu, ev;        // endpoints of edge id (eu < ev)
};

void build_adjacency(const uint8_t *adj, int p, Adjacency &g)
{
    g.off.assign(p + 1, 0);
    for (int u = 0; u < p; ++u) {
        int d = 0;
        const uint8_t *row = adj + (size_t)u * p;
        for (int v = 0; v < p; ++v) d += (row[v] != 0 && v != u);
        g.off[u + 1] = g.off[u] + d;
    }
    g.nb.resize(g.off[p]);
    g.eid.resize(g.off[p]);
    g.eu.clear();
    g.ev.clear();
    std::vector<int32_t> fill(g.off.begin(), g.off.end() - 1);
    // edge ids in row-major (u < v) order
    for (int u = 0; u < p; ++u) {
        const uint8_t *row = adj + (size_t)u * p;
        for (int v = u + 1; v < p; ++v) {
            if (!row[v]) continue;
            int id = (int)g.eu.size();
            g.eu.push_back(u);
            g.ev.push_back(v);
            g.nb[fill[u]] = v;
            g.eid[fill[u]++] = id;
            g.nb[fill[v]] = u;
            g.eid[fill[v]++] = id;
        }
    }
    // neighbour lists sorted ascending (u's list gets smaller ids first from
    // the v-loop of earlier rows, then larger ones from its own row)
    for (int u = 0; u < p; ++u) {
        int a = g.off[u], b = g.off[u + 1];
        std::vector<std::pair<int32_t, int32_t>> tmp;
        tmp.reserve(b - a);
        for (int t = a; t < b; ++t) tmp.emplace_back(g.nb[t], g.eid[t]);
        std::sort(tmp.begin(), tmp.end());
        for (int t = a; t < b; ++t) {
            g.nb[t] = tmp[t - a].first;
            g.eid[t] = tmp[t - a].second;
        }
    }
}

// Block (biconnected component) label of every edge, iterative DFS.
void edge_blocks(const Adjacency &g, int p, std::vector<int32_t> &block)
{
    const int E = (int)g.eu.size();
    block.assign(E, -1);
    std::vector<int32_t> disc(p, -1), low(p, 0);
    struct Frame { int32_t v, pe, it; };
    std::vector<Frame> st;
    std::vector<int32_t> estack;
    int timer = 0, nblk = 0;
    for (int s = 0; s < p; ++s) {
        if (disc[s] != -1) continue;
        disc[s] = low[s] = timer++;
        st.push_back({s, -1, g.off[s]});
        while (!st.empty()) {
            Frame &f = st.back();
            const int v = f.v;
            if (f.it < g.off[v + 1]) {
                const int w = g.nb[f.it], id = g.eid[f.it];
                ++f.it;
                if (id == f.pe) continue;
                if (disc[w] == -1) {
                    estack.push_back(id);
                    disc[w] = low[w] = timer++;
                    st.push_back({w, id, g.off[w]});
                } else if (disc[w] < disc[v]) {
                    estack.push_back(id);
                    low[v] = std::min(low[v], disc[w]);
                }
            } else {
                const int pe = f.pe;
                st.pop_back();
                if (st.empty()) break;
                const int u = st.back().v;
                low[u] = std::min(low[u], low[v]);
                if (low[v] >= disc[u]) {
                    int id;
                    do {
                        id = estack.back();
                        estack.pop_back();
                        block[id] = nblk;
                    } while (id != pe);
                    ++nblk;
                }
            }
        }
    }
}

}  // namespace

void candidate_sets(const uint8_t *adj, int p, CandSets &out)
{
    Adjacency g;
    build_adjacency(adj, p, g);
    std::vector<int32_t> block;
    edge_blocks(g, p, block);
    const int E = (int)g.eu.size();
    out.ei.assign(g.eu.begin(), g.eu.end());
    out.ej.assign(g.ev.begin(), g.ev.end());
    out.off.assign(E + 1, 0);
    out.nodes.clear();
    out.nodes.reserve((size_t)E * 8);
    for (int e = 0; e < E; ++e) {
        const int i = g.eu[e], j = g.ev[e], b = block[e];
        int a = g.off[i], ae = g.off[i + 1], c = g.off[j], ce = g.off[j + 1];
        // merge the block-filtered neighbour lists of i and j
        while (a < ae || c < ce) {
            int ka = INT32_MAX, kc = INT32_MAX;
            while (a < ae && (g.nb[a] == j || block[g.eid[a]] != b)) ++a;
            while (c < ce && (g.nb[c] == i || block[g.eid[c]] != b)) ++c;
            if (a < ae) ka = g.nb[a];
            if (c < ce) kc = g.nb[c];
            if (ka == INT32_MAX && kc == INT32_MAX) break;
            if (ka < kc) { out.nodes.push_back(ka); ++a; }
            else if (kc < ka) { out.nodes.push_back(kc); ++c; }
            else { out.nodes.push_back(ka); ++a; ++c; }
        }
        out.off[e + 1] = (int64_t)out.nodes.size();
    }
}

}  // namespace fpc

extern "C" int fpc_candidates(const uint8_t *adj, int p, int64_t *n_edges, int64_t *n_nodes,
                              int32_t *edge_i, int32_t *edge_j, int64_t *off, int32_t *nodes)
{
    if (!adj || p < 1) return FPC_EINVAL;
    for (int u = 0; u < p; ++u) {
        if (adj[(size_t)u * p + u]) return FPC_EINVAL;
        for (int v = u + 1; v < p; ++v)
            if ((adj[(size_t)u * p + v] != 0) != (adj[(size_t)v * p + u] != 0)) return FPC_EINVAL;
    }
    fpc::CandSets cs;
    fpc::candidate_sets(adj, p, cs);
    const int64_t E = (int64_t)cs.ei.size();
    if (n_edges) *n_edges = E;
    if (n_nodes) *n_nodes = cs.off[E];
    if (edge_i) std::memcpy(edge_i, cs.ei.data(), sizeof(int32_t) * E);
    if (edge_j) std::memcpy(edge_j, cs.ej.data(), sizeof(int32_t) * E);
    if (off) std::memcpy(off, cs.off.data(), sizeof(int64_t) * (E + 1));
    if (nodes) std::memcpy(nodes, cs.nodes.data(), sizeof(int32_t) * cs.off[E]);
    return FPC_OK;
}
