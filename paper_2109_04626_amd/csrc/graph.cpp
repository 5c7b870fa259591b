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
#include <chrono>
#include <cstdio>
#include <cstring>
#include <thread>

#include "fpc_internal.h"

namespace fpc {

namespace {

struct Adjacency {
    std::vector<int32_t> off, nb, eid;  // CSR of neighbours and undirected edge ids
    std::vector<int32_t> eu, ev;        // endpoints of edge id (eu < ev)
};

// Edges (u < v) of rows [u0, u1), in row-major order.
void scan_rows(const uint8_t *adj, int p, int u0, int u1, std::vector<int32_t> &eu, std::vector<int32_t> &ev)
{
    for (int u = u0; u < u1; ++u) {
        const uint8_t *row = adj + (size_t)u * p;
        int v = u + 1;
        // eight entries at a time: nz has the top bit of every nonzero byte
        constexpr uint64_t lo7 = 0x7f7f7f7f7f7f7f7full;
        for (; v + 8 <= p; v += 8) {
            uint64_t word;
            std::memcpy(&word, row + v, 8);
            uint64_t nz = (((word & lo7) + lo7) | word) & ~lo7;
            while (nz) {
                eu.push_back(u);
                ev.push_back(v + (__builtin_ctzll(nz) >> 3));
                nz &= nz - 1;
            }
        }
        for (; v < p; ++v)
            if (row[v]) {
                eu.push_back(u);
                ev.push_back(v);
            }
    }
}

// Working storage of one candidate-set computation, kept per calling
// thread so that repeated calls reuse their memory.
struct Scratch {
    Adjacency g;
    std::vector<std::vector<int32_t>> parts;
    std::vector<std::vector<int64_t>> lens;
    std::vector<int32_t> block, nbblk, deg, fill, disc, low, estack;
};

// Nonzero bytes of row[a, b).
int count_nonzero(const uint8_t *row, int a, int b)
{
    constexpr uint64_t lo7 = 0x7f7f7f7f7f7f7f7full;
    int n = 0, v = a;
    for (; v + 8 <= b; v += 8) {
        uint64_t word;
        std::memcpy(&word, row + v, 8);
        n += __builtin_popcountll((((word & lo7) + lo7) | word) & ~lo7);
    }
    for (; v < b; ++v) n += row[v] != 0;
    return n;
}

// Calls fn(v) for the nonzero bytes of row[0, p) in increasing v.
template <class F>
void for_nonzero(const uint8_t *row, int p, F &&fn)
{
    constexpr uint64_t lo7 = 0x7f7f7f7f7f7f7f7full;
    int v = 0;
    for (; v + 8 <= p; v += 8) {
        uint64_t word;
        std::memcpy(&word, row + v, 8);
        uint64_t nz = (((word & lo7) + lo7) | word) & ~lo7;
        while (nz) {
            fn(v + (__builtin_ctzll(nz) >> 3));
            nz &= nz - 1;
        }
    }
    for (; v < p; ++v)
        if (row[v]) fn(v);
}

void build_adjacency(const uint8_t *adj, int p, Adjacency &g, int nth, Scratch &sc)
{
    // edge ids in row-major (u < v) order; every neighbour list sorted
    g.eu.clear();
    g.ev.clear();
    std::vector<int32_t> &deg = sc.deg;
    if (nth > 1 && p >= 512) {
        // blocks of rows on the host threads, three passes with no scatter:
        // the neighbour counts of each row (all, and above the diagonal);
        // each row's sorted list, with the ids of its edges to larger
        // neighbours; the id of each slot of a smaller neighbour u, found
        // by a binary search in u's list of larger neighbours
        std::vector<int32_t> &up = sc.fill;
        deg.assign(p, 0);
        up.assign(p, 0);
        const int nblk = std::min(p, 4 * nth);
        const auto rows = [&](int b, int &u0, int &u1) {
            u0 = (int)((int64_t)p * b / nblk);
            u1 = (int)((int64_t)p * (b + 1) / nblk);
        };
        host_parallel(nblk, [&](int b) {
            int u0, u1;
            rows(b, u0, u1);
            for (int u = u0; u < u1; ++u) {
                const uint8_t *row = adj + (size_t)u * p;
                up[u] = count_nonzero(row, u + 1, p);
                deg[u] = count_nonzero(row, 0, u) + up[u];
            }
        });
        std::vector<int32_t> upoff(p + 1, 0);
        g.off.assign(p + 1, 0);
        for (int u = 0; u < p; ++u) {
            g.off[u + 1] = g.off[u] + deg[u];
            upoff[u + 1] = upoff[u] + up[u];
        }
        const int E = upoff[p];
        g.nb.resize(g.off[p]);
        g.eid.resize(g.off[p]);
        g.eu.resize(E);
        g.ev.resize(E);
        host_parallel(nblk, [&](int b) {
            int u0, u1;
            rows(b, u0, u1);
            for (int u = u0; u < u1; ++u) {
                int k = g.off[u], id = upoff[u];
                for_nonzero(adj + (size_t)u * p, p, [&](int v) {
                    if (v == u) return;
                    g.nb[k] = v;
                    if (v > u) {
                        g.eid[k] = id;
                        g.eu[id] = u;
                        g.ev[id] = v;
                        ++id;
                    }
                    ++k;
                });
            }
        });
        host_parallel(nblk, [&](int b) {
            int v0, v1;
            rows(b, v0, v1);
            for (int v = v0; v < v1; ++v) {
                const int lo_n = deg[v] - up[v];
                for (int k = g.off[v]; k < g.off[v] + lo_n; ++k) {
                    const int u = g.nb[k];
                    const int32_t *a = g.nb.data() + g.off[u + 1] - up[u], *e = g.nb.data() + g.off[u + 1];
                    g.eid[k] = upoff[u] + (int)(std::lower_bound(a, e, v) - a);
                }
            }
        });
        return;
    }
    // one pass over the upper triangle, then the lists by a scatter
    scan_rows(adj, p, 0, p, g.eu, g.ev);
    deg.assign(p, 0);
    for (size_t id = 0; id < g.eu.size(); ++id) {
        ++deg[g.eu[id]];
        ++deg[g.ev[id]];
    }
    g.off.assign(p + 1, 0);
    for (int u = 0; u < p; ++u) g.off[u + 1] = g.off[u] + deg[u];
    g.nb.resize(g.off[p]);
    g.eid.resize(g.off[p]);
    std::vector<int32_t> &fill = sc.fill;
    fill.assign(g.off.begin(), g.off.end() - 1);
    // edges in (u, v) row-major order: every list receives its smaller
    // neighbours (as v) before its larger ones (as u), in increasing order
    const int E = (int)g.eu.size();
    for (int id = 0; id < E; ++id) {
        const int u = g.eu[id], v = g.ev[id];
        g.nb[fill[v]] = u;
        g.eid[fill[v]++] = id;
    }
    for (int id = 0; id < E; ++id) {
        const int u = g.eu[id], v = g.ev[id];
        g.nb[fill[u]] = v;
        g.eid[fill[u]++] = id;
    }
}

// Block (biconnected component) label of every edge, iterative DFS.
void edge_blocks(const Adjacency &g, int p, std::vector<int32_t> &block, Scratch &sc)
{
    const int E = (int)g.eu.size();
    block.assign(E, -1);
    std::vector<int32_t> &disc = sc.disc, &low = sc.low;
    disc.assign(p, -1);
    low.assign(p, 0);
    struct Frame { int32_t v, pe, it; };
    std::vector<Frame> st;
    std::vector<int32_t> &estack = sc.estack;
    estack.clear();
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

void candidate_sets(const uint8_t *adj, int p, CandSets &out, int threads)
{
    using clk = std::chrono::steady_clock;
    const auto ms = [](clk::time_point a, clk::time_point b) {
        return std::chrono::duration<double, std::milli>(b - a).count();
    };
    const auto t0 = clk::now();
    thread_local Scratch sc;
    Adjacency &g = sc.g;
    build_adjacency(adj, p, g, threads > 0 ? threads : host_threads(), sc);
    const auto t1 = clk::now();
    std::vector<int32_t> &block = sc.block;
    edge_blocks(g, p, block, sc);
    const auto t2 = clk::now();
    const int E = (int)g.eu.size();
    // block id of each adjacency slot, so the merge reads two flat arrays
    std::vector<int32_t> &nbblk = sc.nbblk;
    nbblk.resize(g.nb.size());
    for (size_t t = 0; t < g.nb.size(); ++t) nbblk[t] = block[g.eid[t]];
    out.ei.assign(g.eu.begin(), g.eu.end());
    out.ej.assign(g.ev.begin(), g.ev.end());
    out.off.resize(E + 1);
    out.off[0] = 0;
    // per edge: the neighbours of i in block b (other than j) and those of j
    // in block b (other than i), each filtered without branches, then their
    // sorted union by a branch-free merge (both lists are sorted); edges
    // are split into contiguous chunks handled by separate host threads
    int maxdeg = 0;
    for (int u = 0; u < p; ++u) maxdeg = std::max(maxdeg, g.off[u + 1] - g.off[u]);
    auto merge_range = [&](int e0, int e1, std::vector<int32_t> &dst, std::vector<int64_t> &len) {
        size_t bound = 0;
        for (int e = e0; e < e1; ++e)
            bound += (size_t)(g.off[g.eu[e] + 1] - g.off[g.eu[e]]) + (size_t)(g.off[g.ev[e] + 1] - g.off[g.ev[e]]);
        dst.resize(bound);
        len.resize((size_t)(e1 - e0));
        std::vector<int32_t> fa((size_t)maxdeg + 1), fc((size_t)maxdeg + 1);
        size_t o = 0;
        for (int e = e0; e < e1; ++e) {
            const int i = g.eu[e], j = g.ev[e], b = block[e];
            const int32_t *na = g.nb.data() + g.off[i], *ba = nbblk.data() + g.off[i];
            const int32_t *nc = g.nb.data() + g.off[j], *bc = nbblk.data() + g.off[j];
            const int da = g.off[i + 1] - g.off[i], dc = g.off[j + 1] - g.off[j];
            int la = 0, lc = 0;
            for (int t = 0; t < da; ++t) {
                fa[la] = na[t];
                la += (ba[t] == b) & (na[t] != j);
            }
            for (int t = 0; t < dc; ++t) {
                fc[lc] = nc[t];
                lc += (bc[t] == b) & (nc[t] != i);
            }
            int32_t *out = dst.data() + o;
            int a = 0, c = 0, k = 0;
            while (a < la && c < lc) {
                const int32_t x = fa[a], y = fc[c];
                out[k++] = x < y ? x : y;
                a += x <= y;
                c += y <= x;
            }
            while (a < la) out[k++] = fa[a++];
            while (c < lc) out[k++] = fc[c++];
            o += (size_t)k;
            len[e - e0] = k;
        }
        dst.resize(o);
    };
    int nth = threads > 0 ? threads : host_threads();
    if (E < 256) nth = 1;
    // chunks of about equal work (an edge costs deg i + deg j: the edges of
    // a hub are many and long, and sit together in the edge order), four per
    // thread, taken by the threads as they come free
    const int nck = nth == 1 ? 1 : std::min(E, 4 * nth);
    auto &parts = sc.parts;
    auto &lens = sc.lens;
    if ((int)parts.size() < nck) {
        parts.resize(nck);
        lens.resize(nck);
    }
    std::vector<int> bounds(nck + 1, E);
    bounds[0] = 0;
    if (nck > 1) {
        int64_t total = 0;
        for (int e = 0; e < E; ++e) total += (g.off[g.eu[e] + 1] - g.off[g.eu[e]]) + (g.off[g.ev[e] + 1] - g.off[g.ev[e]]);
        int64_t acc = 0;
        int c = 1;
        for (int e = 0; e < E && c < nck; ++e) {
            acc += (g.off[g.eu[e] + 1] - g.off[g.eu[e]]) + (g.off[g.ev[e] + 1] - g.off[g.ev[e]]);
            while (c < nck && acc * nck >= total * c) bounds[c++] = e + 1;
        }
    }
    if (nck == 1) {
        merge_range(0, E, parts[0], lens[0]);
    } else {
        host_parallel(nck, [&](int t) { merge_range(bounds[t], bounds[t + 1], parts[t], lens[t]); });
    }
    std::vector<size_t> at(nck + 1, 0);
    for (int t = 0; t < nck; ++t) at[t + 1] = at[t] + parts[t].size();
    out.nodes.resize(at[nck]);
    int e = 0;
    for (int t = 0; t < nck; ++t)
        for (int64_t L : lens[t]) {
            out.off[e + 1] = out.off[e] + L;
            ++e;
        }
    const auto t3 = clk::now();
    auto copy_part = [&](int t) {
        std::memcpy(out.nodes.data() + at[t], parts[t].data(), sizeof(int32_t) * parts[t].size());
    };
    if (nck == 1) copy_part(0);
    else host_parallel(nck, copy_part);
    if (trace_on())
        std::fprintf(stderr, "[fpc]   candidate sets: adjacency %.3f blocks %.3f merge %.3f concat %.3f ms (%d threads)\n",
                     ms(t0, t1), ms(t1, t2), ms(t2, t3), ms(t3, clk::now()), nth);
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
