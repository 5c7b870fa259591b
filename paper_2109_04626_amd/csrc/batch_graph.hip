// Many instances with the whole skeleton on the device, captured once per
// call as one HIP graph (FPC_FLAG_GRAPH in fpc_skeleton_batch).
//
// The graph holds, in stream order:
//   - every instance's correlation matrices (FP64, and the FP32 matrix of
//     the mixed form with its entry error);
//   - the first reverse level of every instance together (Algorithm 2's
//     first stage through Omega = C^{-1}: one sweep launch per panel step
//     for all instances), which writes each instance's adjacency bytes;
//   - the levels l = L .. 0 (L the largest cap over the instances).  Level
//     l of an instance runs when l <= its cap and its largest candidate set
//     has at least l nodes -- the same levels, in the same order, as a call
//     on the instance alone (next level = min(current, largest set)).  Each
//     level, on the device:
//       * compressed rows of every instance's graph;
//       * for every node v, its neighbours grouped by the connected
//         components of G - v (a breadth-first search in LDS per node):
//         k in adj(v) lies on a simple path from v to u in adj(v) exactly
//         when k and u fall in one component of G - v (Sec. 2.1
//         definitions: adj(G,i,j) n path(G,i,j));
//       * per edge (v < u) its candidate list, the sorted union of the
//         neighbours of v grouped with u and of u grouped with v;
//       * the edge table of the edges with |cand| >= l, bucketed by list
//         length into classes of fixed kernels and LDS (the order inside a
//         class is immaterial: every edge's result is its own);
//       * the level's test launches (the kernels of the host-driven path,
//         reading the class ranges from device memory), the FP64 re-runs;
//       * deletions at level end (stable variant), the separating set of
//         each deleted edge decoded from its lowest independent rank, and
//         the level's counts per instance.
// The host reads the results once after the graph.  A capacity that the
// work outgrows (recheck queue, candidate pool, separating-set store, a
// list of 1024 candidates or more, a level count that overflows) is
// reported and the call runs on the host-driven path instead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fpc_internal.h"

namespace fpc {

namespace {

constexpr int kNC = kMaxDeviceClasses;
constexpr int kScanThreads = 1024;

struct GInst {
    int p, cap;       // variables; highest subset level of the instance (-1: none)
    int64_t adj_off;  // byte offset of its p x p adjacency in the pool
    int64_t row0;     // its first row in the rows of all instances
};

struct GStat {  // one level of one instance
    unsigned long long eligible, possible, executed, rechecked, deleted, required;
    int max_cand;  // largest candidate set of the level's graph (-1: no edge)
    int pad;
};

struct GSep {  // one separating set
    int64_t pair;
    int64_t node_off;
    int inst, level;
};

struct GFlags {
    unsigned int overflow;  // a capacity was outgrown: the host-driven path runs instead
    unsigned int bad_rows;  // a resample row index out of range
    unsigned int pad0, pad1;
    unsigned long long cand_fill, sep_fill, node_fill;
};

struct GArgs {
    const GInst *I;
    const int *rowinst;
    int R;              // rows of all instances
    uint8_t *adj;
    int *deg, *up;      // per row: neighbours, neighbours after the node
    int64_t *rowoff;    // R+1: offsets of the rows in nbr
    int64_t *edgeoff;   // R+1: first edge index of each row
    int *nbr, *grp;     // neighbour ids (sorted per row), group label per neighbour
    int *em;            // per edge: |cand| (-1: instance not at this level)
    int64_t *eslot;     // per edge: its record in the level's table (-1: not eligible)
    int64_t emax;       // edge capacity
    int *row_mmax;      // per row: largest |cand| of its edges (-1: none)
    unsigned long long *row_cnt;  // per row: eligible, possible, deleted, required, (spare)
    unsigned long long *class_cnt, *class_fill;  // per class
    int64_t *class_range;                         // per class [begin, end)
    int cbound[kNC];    // this level's class bounds (device_class_bounds)
    int ncls;
    EdgeRec *rec;
    uint64_t *minhit;
    int32_t *cand;
    int64_t cand_cap;
    const int64_t *binom;
    GStat *stat;        // this level's row of the statistics (ni entries)
    unsigned long long *inst_cnt;  // per instance: tests run, tests re-run in FP64
    unsigned long long *counters;  // the level's counters ([3] queue overflow)
    GFlags *flags;
    GSep *sep;
    int64_t sep_cap;
    int32_t *nodes;
    int64_t node_cap;
    int ni, l;
};

__device__ __forceinline__ int64_t binom_dev(const int64_t *binom, int a, int b)
{
    if (b < 0 || b > a) return 0;
    const int bb = min(b, a - b);
    return bb < kBinomCols ? binom[a * kBinomCols + bb] : INT64_MAX;
}

__device__ __forceinline__ int lower_bound_dev(const int *a, int n, int x)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void g_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

// Counters of a level: classes, the candidate pool, the test counters.
__global__ void g_level_init(GArgs G, int n_cnt)
{
    const int t = threadIdx.x;
    if (t < kNC) {
        G.class_cnt[t] = 0;
        G.class_fill[t] = 0;
    }
    for (int k = t; k < n_cnt; k += blockDim.x) G.counters[k] = 0;
    if (t == 0) G.flags->cand_fill = 0;
}

// Row r: neighbours of node v of its instance, and those after v.
__global__ __launch_bounds__(64) void g_csr_count(GArgs G)
{
    const int r = blockIdx.x;
    const GInst g = G.I[G.rowinst[r]];
    const int v = (int)(r - g.row0);
    const uint8_t *row = G.adj + g.adj_off + (int64_t)v * g.p;
    int c = 0, cu = 0;
    for (int u = threadIdx.x; u < g.p; u += 64) {
        const bool a = row[u] != 0;
        c += a;
        cu += a && u > v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o);
        cu += __shfl_xor(cu, o);
    }
    if (threadIdx.x == 0) {
        G.deg[r] = c;
        G.up[r] = cu;
    }
}

// Exclusive prefix sums of deg and up over all rows (one workgroup, chunks
// of kScanThreads rows with a running carry).
__global__ __launch_bounds__(kScanThreads) void g_scan_rows(GArgs G)
{
    __shared__ int64_t wa[kScanThreads / 64], wb[kScanThreads / 64];
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    int64_t ca = 0, cb = 0;
    for (int base = 0; base < G.R; base += kScanThreads) {
        const int r = base + threadIdx.x;
        const int64_t a = r < G.R ? G.deg[r] : 0, b = r < G.R ? G.up[r] : 0;
        int64_t xa = a, xb = b;
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t ya = __shfl_up(xa, d), yb = __shfl_up(xb, d);
            if (lane >= d) {
                xa += ya;
                xb += yb;
            }
        }
        if (lane == 63) {
            wa[w] = xa;
            wb[w] = xb;
        }
        __syncthreads();
        int64_t pa = 0, pb = 0, ta = 0, tb = 0;
        for (int k = 0; k < kScanThreads / 64; ++k) {
            if (k < w) {
                pa += wa[k];
                pb += wb[k];
            }
            ta += wa[k];
            tb += wb[k];
        }
        if (r < G.R) {
            G.rowoff[r] = ca + pa + xa - a;
            G.edgeoff[r] = cb + pb + xb - b;
        }
        ca += ta;
        cb += tb;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        G.rowoff[G.R] = ca;
        G.edgeoff[G.R] = cb;
    }
}

// Row r's neighbour ids in increasing order.
__global__ __launch_bounds__(64) void g_csr_fill(GArgs G)
{
    const int r = blockIdx.x;
    const GInst g = G.I[G.rowinst[r]];
    const int v = (int)(r - g.row0);
    const uint8_t *row = G.adj + g.adj_off + (int64_t)v * g.p;
    int *out = G.nbr + G.rowoff[r];
    const int lane = threadIdx.x;
    int base = 0;
    for (int u0 = 0; u0 < g.p; u0 += 64) {
        const int u = u0 + lane;
        const bool a = u < g.p && row[u] != 0;
        const unsigned long long m = __ballot(a);
        if (a) out[base + __popcll(m & ((1ull << lane) - 1ull))] = u;
        base += __popcll(m);
    }
}

// Groups of row r's neighbours by the components of G - v: a breadth-first
// search from the first neighbour not yet grouped labels every neighbour it
// reaches with that neighbour's position; the search stops once every
// neighbour is grouped.  LDS: visited and neighbour bitsets, labels and two
// frontiers (maxp nodes).
__global__ __launch_bounds__(256) void g_groups(GArgs G, int maxp)
{
    extern __shared__ __align__(16) unsigned char sm[];
    const int r = blockIdx.x;
    const GInst g = G.I[G.rowinst[r]];
    if (g.cap < G.l) return;  // the instance is past this level (uniform)
    const int d = G.deg[r];
    if (d == 0) return;
    const int *nb = G.nbr + G.rowoff[r];
    int *out = G.grp + G.rowoff[r];
    if (d == 1) {
        if (threadIdx.x == 0) out[0] = 0;
        return;
    }
    const int v = (int)(r - g.row0);
    const int W = (maxp + 31) / 32;
    unsigned int *vis = reinterpret_cast<unsigned int *>(sm);
    unsigned int *isnb = vis + W;
    int *lab = reinterpret_cast<int *>(isnb + W);
    int *fa = lab + maxp, *fb = fa + maxp;
    __shared__ int remaining, nnext;
    for (int k = threadIdx.x; k < W; k += 256) {
        vis[k] = 0u;
        isnb[k] = 0u;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < d; s += 256) {
        lab[s] = -1;
        atomicOr(&isnb[nb[s] >> 5], 1u << (nb[s] & 31));
    }
    if (threadIdx.x == 0) {
        atomicOr(&vis[v >> 5], 1u << (v & 31));  // G - v
        remaining = d;
    }
    __syncthreads();
    for (int s = 0; s < d; ++s) {
        // every thread reads the shared state before thread 0 changes it
        const bool stop = remaining == 0, seen = lab[s] >= 0;
        __syncthreads();
        if (stop) break;   // uniform
        if (seen) continue;
        int *cur = fa, *nxt = fb;
        if (threadIdx.x == 0) {
            const int x = nb[s];
            lab[s] = s;
            remaining -= 1;
            atomicOr(&vis[x >> 5], 1u << (x & 31));
            cur[0] = x;
        }
        int ncur = 1;
        __syncthreads();
        while (ncur > 0 && remaining > 0) {
            if (threadIdx.x == 0) nnext = 0;
            __syncthreads();
            for (int idx = threadIdx.x; idx < ncur; idx += 256) {
                const int w = cur[idx];
                const int64_t rw = g.row0 + w;
                const int *nw = G.nbr + G.rowoff[rw];
                const int dw = G.deg[rw];
                for (int t = 0; t < dw; ++t) {
                    const int x = nw[t];
                    const unsigned int bit = 1u << (x & 31);
                    if (atomicOr(&vis[x >> 5], bit) & bit) continue;
                    nxt[atomicAdd(&nnext, 1)] = x;
                    if (isnb[x >> 5] & bit) {
                        lab[lower_bound_dev(nb, d, x)] = s;
                        atomicSub(&remaining, 1);
                    }
                }
            }
            __syncthreads();
            ncur = nnext;
            int *tmp = cur;
            cur = nxt;
            nxt = tmp;
            __syncthreads();  // nnext is read before the next reset
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < d; s += 256) out[s] = lab[s];
}

// The edge (v < u) at position pu of row r (instance g), and the position
// of v in u's row.
struct EdgeRef {
    int k, v, u;
    int64_t rv, ru;
    int pu, pv;
};

__device__ __forceinline__ EdgeRef edge_ref_row(const GArgs &G, int r, int k, const GInst &g, int pu)
{
    EdgeRef E;
    E.k = k;
    E.rv = r;
    E.v = (int)(r - g.row0);
    E.pu = pu;
    E.u = G.nbr[G.rowoff[r] + pu];
    E.ru = g.row0 + E.u;
    E.pv = lower_bound_dev(G.nbr + G.rowoff[E.ru], G.deg[E.ru], E.v);
    return E;
}

// The sorted union of the neighbours of v grouped with u and of u grouped
// with v (out NULL: count only).
__device__ int cand_merge(const GArgs &G, const EdgeRef &E, int32_t *out)
{
    const int *nv = G.nbr + G.rowoff[E.rv], *gv = G.grp + G.rowoff[E.rv];
    const int *nu = G.nbr + G.rowoff[E.ru], *gu = G.grp + G.rowoff[E.ru];
    const int dv = G.deg[E.rv], du = G.deg[E.ru];
    const int lu = gv[E.pu], lv = gu[E.pv];
    int a = 0, b = 0, m = 0;
    for (;;) {
        while (a < dv && (a == E.pu || gv[a] != lu)) ++a;
        while (b < du && (b == E.pv || gu[b] != lv)) ++b;
        if (a >= dv && b >= du) break;
        int x;
        if (b >= du || (a < dv && nv[a] < nu[b])) {
            x = nv[a++];
        } else if (a >= dv || nu[b] < nv[a]) {
            x = nu[b++];
        } else {
            x = nv[a];
            ++a;
            ++b;
        }
        if (out) out[m] = x;
        ++m;
    }
    return m;
}

__device__ __forceinline__ int class_of(const GArgs &G, int m)
{
    int c = 0;
    while (c < G.ncls - 1 && m > G.cbound[c]) ++c;
    return c;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// The edge kernels take one row per wave: row r's edges are (v, u) for the
// last up[r] neighbours u > v, edge indices edgeoff[r] + t.  A row's counts
// go to per-row slots, summed per instance by g_level_stats (no atomics on
// a per-instance word).

// Candidate-set sizes of row r's edges; the row's largest.
__global__ __launch_bounds__(64) void g_edge_count(GArgs G)
{
    const int r = blockIdx.x, lane = threadIdx.x;
    const int k = G.rowinst[r];
    const GInst g = G.I[k];
    const int up = G.up[r], d = G.deg[r];
    const int64_t e0 = G.edgeoff[r];
    const bool on = g.cap >= G.l;
    int mx = -1;
    for (int t = lane; t < up; t += 64) {
        int m = -1;
        if (on) {
            const EdgeRef R = edge_ref_row(G, r, k, g, d - up + t);
            m = cand_merge(G, R, nullptr);
        }
        G.em[e0 + t] = m;
        mx = max(mx, m);
    }
    mx = wave_max(mx);
    if (lane == 0) G.row_mmax[r] = mx;
}

// Edges with |cand| >= l counted per class (one atomic per wave and class).
__global__ __launch_bounds__(256) void g_edge_classes(GArgs G)
{
    const int64_t E = G.edgeoff[G.R];
    const int lane = threadIdx.x % 64;
    for (int64_t e0 = (int64_t)blockIdx.x * 256; e0 < E; e0 += (int64_t)gridDim.x * 256) {
        const int64_t e = e0 + threadIdx.x;
        const int m = e < E ? G.em[e] : -1;
        if (m >= G.l && m >= kBinomRows) atomicOr(&G.flags->overflow, 1u);
        const bool el = m >= G.l && m < kBinomRows;  // as g_edge_fill
        const int c = el ? class_of(G, m) : -1;
        for (int q = 0; q < G.ncls; ++q) {
            const unsigned long long b = __ballot(c == q);
            if (b && lane == __ffsll((long long)b) - 1) atomicAdd(&G.class_cnt[q], (unsigned long long)__popcll(b));
        }
    }
}

__global__ void g_class_ranges(GArgs G)
{
    if (threadIdx.x != 0) return;
    int64_t b = 0;
    for (int c = 0; c < G.ncls; ++c) {
        G.class_range[2 * c] = b;
        b += (int64_t)G.class_cnt[c];
        G.class_range[2 * c + 1] = b;
    }
}

// The level's edge table, row r's part: each eligible edge takes a slot in
// its class and room for its list in the candidate pool (one atomic per
// wave for each), and writes its record, its list and minhit = no hit;
// eslot[e] = its slot (-1: not eligible).
__global__ __launch_bounds__(64) void g_edge_fill(GArgs G)
{
    const int r = blockIdx.x, lane = threadIdx.x;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int k = G.rowinst[r];
    const GInst g = G.I[k];
    const int up = G.up[r], d = G.deg[r];
    const int64_t e0 = G.edgeoff[r];
    unsigned long long n_el = 0, n_poss = 0;
    for (int t0 = 0; t0 < up; t0 += 64) {  // uniform
        const int t = t0 + lane;
        const int m = t < up ? G.em[e0 + t] : -1;
        const bool el = m >= G.l && m < kBinomRows;  // em is -1 past the instance's cap
        const int c = el ? class_of(G, m) : -1;
        int64_t slot = -1;
        for (int q = 0; q < G.ncls; ++q) {
            const unsigned long long b = __ballot(c == q);
            if (!b) continue;
            const int lead = __ffsll((long long)b) - 1;
            unsigned long long base = 0;
            if (lane == lead) base = atomicAdd(&G.class_fill[q], (unsigned long long)__popcll(b));
            base = __shfl(base, lead);
            if (c == q) slot = G.class_range[2 * q] + (int64_t)(base + __popcll(b & below));
        }
        // room in the pool: a wave prefix sum of the lists
        const int64_t mm = el ? m : 0;
        int64_t x = mm;
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int64_t y = __shfl_up(x, dd);
            if (lane >= dd) x += y;
        }
        unsigned long long cbase = 0;
        if (lane == 63 && x > 0) cbase = atomicAdd(&G.flags->cand_fill, (unsigned long long)x);
        cbase = __shfl(cbase, 63);
        if (t < up) G.eslot[e0 + t] = slot;
        if (el) {
            const int64_t coff = (int64_t)cbase + x - mm;
            const EdgeRef R = edge_ref_row(G, r, k, g, d - up + t);
            G.minhit[slot] = ~0ull;
            const int64_t N = binom_dev(G.binom, m, G.l);
            if (coff + m > G.cand_cap || N == INT64_MAX) {
                // no room: a record without tests keeps the level's launches
                // in bounds, and the call is run again host-driven
                atomicOr(&G.flags->overflow, 1u);
                G.rec[slot] = EdgeRec{R.v, R.u, 0, 0, 0, k, 0};
            } else {
                cand_merge(G, R, G.cand + coff);
                G.rec[slot] = EdgeRec{R.v, R.u, m, (int32_t)coff, N, k, 0};
                n_el += 1;
                n_poss += (unsigned long long)N;
            }
        }
    }
    n_el = wave_sum(n_el);
    n_poss = wave_sum(n_poss);
    if (lane == 0) {
        G.row_cnt[5 * (int64_t)r] = n_el;
        G.row_cnt[5 * (int64_t)r + 1] = n_poss;
    }
}

// After the level's tests, row r's edges: deletions (stable variant: the
// graph the level read is changed only now), separating sets, tests
// required.
__global__ __launch_bounds__(64) void g_apply(GArgs G)
{
    const int r = blockIdx.x, lane = threadIdx.x;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int k = G.rowinst[r];
    const GInst g = G.I[k];
    const int up = G.up[r];
    const int64_t e0 = G.edgeoff[r];
    unsigned long long n_del = 0, n_req = 0;
    for (int t0 = 0; t0 < up; t0 += 64) {  // uniform
        const int t = t0 + lane;
        const int64_t slot = t < up ? G.eslot[e0 + t] : -1;
        bool del = false;
        EdgeRec E{};
        uint64_t mh = ~0ull;
        if (slot >= 0) {
            E = G.rec[slot];
            mh = G.minhit[slot];
            del = mh != ~0ull;
            n_req += del ? (unsigned long long)(mh + 1) : (unsigned long long)E.ntests;
            n_del += del;
        }
        const unsigned long long b = __ballot(del);
        if (!b) continue;  // uniform
        unsigned long long rs0 = 0, ro0 = 0;
        if (lane == 0) {
            rs0 = atomicAdd(&G.flags->sep_fill, (unsigned long long)__popcll(b));
            ro0 = atomicAdd(&G.flags->node_fill, (unsigned long long)__popcll(b) * (unsigned long long)G.l);
        }
        rs0 = __shfl(rs0, 0);
        ro0 = __shfl(ro0, 0);
        if (!del) continue;
        uint8_t *adj = G.adj + g.adj_off;
        adj[(int64_t)E.i * g.p + E.j] = 0;
        adj[(int64_t)E.j * g.p + E.i] = 0;
        const unsigned long long rank = __popcll(b & below);
        const unsigned long long rs = rs0 + rank, ro = ro0 + rank * (unsigned long long)G.l;
        if ((int64_t)rs >= G.sep_cap || (int64_t)(ro + G.l) > G.node_cap) {
            atomicOr(&G.flags->overflow, 1u);
            continue;
        }
        // lexicographic unranking of the lowest independent rank
        int64_t R = (int64_t)mh;
        int x = 0;
        const int32_t *cl = G.cand + E.cand_off;
        for (int s = 0; s < G.l; ++s) {
            for (;;) {
                const int64_t cnt = binom_dev(G.binom, E.m - 1 - x, G.l - 1 - s);
                if (R < cnt) break;
                R -= cnt;
                ++x;
            }
            G.nodes[ro + s] = cl[x];  // the list is sorted, so the set is too
            ++x;
        }
        const int64_t pair = (int64_t)E.i * g.p - (int64_t)E.i * (E.i + 1) / 2 + (E.j - E.i - 1);
        G.sep[rs] = GSep{pair, (int64_t)ro, E.inst, G.l};
    }
    n_del = wave_sum(n_del);
    n_req = wave_sum(n_req);
    if (lane == 0) {
        G.row_cnt[5 * (int64_t)r + 2] = n_del;
        G.row_cnt[5 * (int64_t)r + 3] = n_req;
    }
}

// The level's counts of instance blockIdx.x: its rows' counts and the
// tests' counters.
__global__ __launch_bounds__(256) void g_level_stats(GArgs G)
{
    const int k = blockIdx.x;
    const GInst g = G.I[k];
    unsigned long long v[4] = {0, 0, 0, 0};
    int mx = -1;
    for (int v0 = threadIdx.x; v0 < g.p; v0 += 256) {
        const int64_t r = g.row0 + v0;
        for (int f = 0; f < 4; ++f) v[f] += G.row_cnt[5 * r + f];
        mx = max(mx, G.row_mmax[r]);
    }
    __shared__ unsigned long long red[4][4];
    __shared__ int redm[4];
    for (int f = 0; f < 4; ++f) v[f] = wave_sum(v[f]);
    mx = wave_max(mx);
    const int w = threadIdx.x / 64;
    if (threadIdx.x % 64 == 0) {
        for (int f = 0; f < 4; ++f) red[w][f] = v[f];
        redm[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        GStat st{};
        st.max_cand = -1;
        for (int q = 0; q < 4; ++q) {
            st.eligible += red[q][0];
            st.possible += red[q][1];
            st.deleted += red[q][2];
            st.required += red[q][3];
            st.max_cand = max(st.max_cand, redm[q]);
        }
        st.executed = G.inst_cnt[2 * k];
        st.rechecked = G.inst_cnt[2 * k + 1];
        G.stat[k] = st;
        if (k == 0 && G.counters[3]) atomicOr(&G.flags->overflow, 1u);
    }
}

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

struct Carver {
    char *base = nullptr;
    size_t off = 0;
    template <class T> T *take(size_t n)
    {
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += align_up(sizeof(T) * std::max<size_t>(n, 1));
        return p;
    }
};

double now_ms_g()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

int skeleton_batch_graph(fpc_ctx *ctx, const fpc_params *P, int ni, const fpc_instance *inst, GraphBatchOut &out)
{
    const double t_start = now_ms_g();
    hipStream_t st = ctx->stream;
    const bool mixed = P->precision == FPC_PREC_MIXED;
    if (P->max_level < 0 || P->max_level > kMaxGraphLevel || P->max_tests > 0) return kGraphFallback;
    const int m32 = P->c32_method ? P->c32_method : FPC_CORR_BF16X6;
    const size_t esz = P->x_dtype == FPC_F64 ? 8 : 4;
    int maxp = 0, L0 = -1;
    int64_t R = 0, Sp2 = 0, Emax = 0, maxnx = 0;
    std::vector<GInst> gi(ni);
    std::vector<int> rowinst;
    std::vector<double> qk(ni);
    for (int k = 0; k < ni; ++k) {
        const int p = inst[k].p;
        if (p > kMaxGraphP) return kGraphFallback;
        maxp = std::max(maxp, p);
        gi[k].p = p;
        gi[k].cap = std::min(P->max_level, p - 3);
        gi[k].adj_off = Sp2;
        gi[k].row0 = R;
        L0 = std::max(L0, gi[k].cap);
        for (int v = 0; v < p; ++v) rowinst.push_back(k);
        R += p;
        Sp2 += (int64_t)p * p;
        Emax += (int64_t)p * (p - 1) / 2;
        maxnx = std::max<int64_t>(maxnx, (int64_t)inst[k].n * p);
        qk[k] = std::isnan(P->q_override) ? normal_quantile_upper(P->alpha) : P->q_override;
    }
    const int nsteps = L0 + 1;
    const int64_t cand_cap = std::min<int64_t>(Emax * 64 + 1024, int64_t(1) << 28);
    const int64_t sep_cap = std::min<int64_t>(Emax, int64_t(1) << 24);
    const int64_t node_cap = std::min<int64_t>(sep_cap * kMaxGraphLevel, int64_t(1) << 26);
    const int n_cnt = 8 + 2 * ni;
    const int64_t queue_cap = mixed ? std::max<int64_t>(ctx->queue_init,
                                                        (int64_t)(ctx->queue.bytes / (2 * sizeof(int64_t))))
                                    : 0;

    // ---- one device pool for the whole call
    auto carve = [&](Carver &c) {
        struct P_ {
            std::vector<double *> c64, buf0, buf1, pinv;
            std::vector<float *> c32;
        } ptrs;
        for (int k = 0; k < ni; ++k) {
            const size_t pp = (size_t)inst[k].p * inst[k].p;
            ptrs.c64.push_back(c.take<double>(pp));
            ptrs.c32.push_back(mixed ? c.take<float>(pp) : nullptr);
            ptrs.buf0.push_back(c.take<double>(pp));
            ptrs.buf1.push_back(c.take<double>(pp));
            ptrs.pinv.push_back(c.take<double>(7 * 32 * 32));
        }
        return ptrs;
    };
    Carver c0;
    (void)carve(c0);
    c0.take<int>(ni);                       // first-level flags
    c0.take<unsigned long long>(ni);        // first-level deletions
    c0.take<unsigned long long>(ni);        // entry errors (FP64 bits)
    c0.take<uint8_t>(Sp2);                  // adjacency
    c0.take<GInst>(ni);
    c0.take<int>(R);                        // rowinst
    c0.take<int>(R);
    c0.take<int>(R);                        // deg, up
    c0.take<int64_t>(R + 1);
    c0.take<int64_t>(R + 1);                // rowoff, edgeoff
    c0.take<int>(2 * Emax);
    c0.take<int>(2 * Emax);                 // nbr, grp
    c0.take<int>(Emax);                     // em
    c0.take<int64_t>(Emax);                 // eslot
    c0.take<int>(R);                        // row_mmax
    c0.take<unsigned long long>(5 * R);     // row_cnt
    c0.take<unsigned long long>(2 * kNC);
    c0.take<int64_t>(2 * kNC);
    c0.take<EdgeRec>(Emax);
    c0.take<uint64_t>(Emax);
    c0.take<int32_t>(cand_cap);
    c0.take<int64_t>(Emax + 3 * kNC);  // plan
    c0.take<unsigned long long>(n_cnt);
    c0.take<char>(inst_rec_bytes() * ni * std::max(nsteps, 1));
    c0.take<DevInstSrc>(ni);
    c0.take<GStat>((size_t)ni * std::max(nsteps, 1));
    c0.take<GFlags>(1);
    c0.take<GSep>(sep_cap);
    c0.take<int32_t>(node_cap);
    int rc = ctx->batch_c.ensure(c0.off);
    if (rc) return rc;
    Carver c;
    c.base = ctx->batch_c.as<char>();
    auto ptrs = carve(c);
    int *fl_bad = c.take<int>(ni);
    unsigned long long *fl_del = c.take<unsigned long long>(ni);
    unsigned long long *cerr_slot = c.take<unsigned long long>(ni);
    GArgs G{};
    G.adj = c.take<uint8_t>(Sp2);
    GInst *d_gi = c.take<GInst>(ni);
    int *d_rowinst = c.take<int>(R);
    G.deg = c.take<int>(R);
    G.up = c.take<int>(R);
    G.rowoff = c.take<int64_t>(R + 1);
    G.edgeoff = c.take<int64_t>(R + 1);
    G.nbr = c.take<int>(2 * Emax);
    G.grp = c.take<int>(2 * Emax);
    G.em = c.take<int>(Emax);
    G.eslot = c.take<int64_t>(Emax);
    G.row_mmax = c.take<int>(R);
    G.row_cnt = c.take<unsigned long long>(5 * R);
    G.class_cnt = c.take<unsigned long long>(2 * kNC);
    G.class_fill = G.class_cnt + kNC;
    G.class_range = c.take<int64_t>(2 * kNC);
    G.rec = c.take<EdgeRec>(Emax);
    G.minhit = c.take<uint64_t>(Emax);
    G.cand = c.take<int32_t>(cand_cap);
    int64_t *plan = c.take<int64_t>(Emax + 3 * kNC);
    G.counters = c.take<unsigned long long>(n_cnt);
    G.inst_cnt = G.counters + 8;
    char *insts = c.take<char>(inst_rec_bytes() * ni * std::max(nsteps, 1));
    DevInstSrc *d_src = c.take<DevInstSrc>(ni);
    GStat *stats = c.take<GStat>((size_t)ni * std::max(nsteps, 1));
    G.flags = c.take<GFlags>(1);
    G.sep = c.take<GSep>(sep_cap);
    G.nodes = c.take<int32_t>(node_cap);
    G.I = d_gi;
    G.rowinst = d_rowinst;
    G.R = (int)R;
    G.emax = Emax;
    G.cand_cap = cand_cap;
    G.binom = ctx->binom.as<int64_t>();
    G.sep_cap = sep_cap;
    G.node_cap = node_cap;
    G.ni = ni;

    // ---- other workspaces, grown before the capture
    for (int k = 0; k < ni; ++k) {
        if ((rc = corr_reserve(ctx, inst[k].n, inst[k].p, FPC_CORR_FP64))) return rc;
        if (mixed && m32 != FPC_CORR_FP32 && (rc = corr_reserve(ctx, inst[k].n, inst[k].p, m32))) return rc;
    }
    if ((rc = ctx->x_copy.ensure(esz * (size_t)maxnx))) return rc;
    if (mixed && (rc = ctx->queue.ensure(sizeof(int64_t) * 2 * queue_cap))) return rc;

    // ---- tables
    std::vector<DevInstSrc> src(ni);
    std::vector<FirstLevelInst> fli(ni);
    for (int k = 0; k < ni; ++k) {
        src[k] = DevInstSrc{ptrs.c32[k], ptrs.c64[k], inst[k].p, inst[k].n, qk[k],
                            mixed ? reinterpret_cast<const double *>(cerr_slot + k) : nullptr};
        fli[k] = FirstLevelInst{ptrs.c64[k], ptrs.buf0[k], ptrs.buf1[k], ptrs.pinv[k], fl_bad + k,
                                fl_del + k, G.adj + gi[k].adj_off, inst[k].p, inst[k].n, qk[k]};
    }
    std::vector<SweepJob> fj, pj;
    std::vector<DecideJob> dj;
    FirstLevelBatchBufs fb;
    first_level_batch_plan(fli, fj, pj, fb.panel_job0, fb.panel_njobs, fb.panel_tiles, dj, fb.decide_elems);
    if ((rc = ctx->batch_tmp.ensure(sizeof(SweepJob) * (fj.size() + pj.size()) + sizeof(DecideJob) * dj.size() + 256)))
        return rc;
    SweepJob *d_jobs = ctx->batch_tmp.as<SweepJob>();
    DecideJob *d_dj = reinterpret_cast<DecideJob *>(d_jobs + fj.size() + pj.size());
    FPC_HIP(hipMemcpy(d_jobs, fj.data(), sizeof(SweepJob) * fj.size(), hipMemcpyHostToDevice));
    if (!pj.empty())
        FPC_HIP(hipMemcpy(d_jobs + fj.size(), pj.data(), sizeof(SweepJob) * pj.size(), hipMemcpyHostToDevice));
    FPC_HIP(hipMemcpy(d_dj, dj.data(), sizeof(DecideJob) * dj.size(), hipMemcpyHostToDevice));
    fb.first_jobs = d_jobs;
    fb.panel_jobs = d_jobs + fj.size();
    fb.decide_jobs = d_dj;
    FPC_HIP(hipMemcpy(d_gi, gi.data(), sizeof(GInst) * ni, hipMemcpyHostToDevice));
    FPC_HIP(hipMemcpy(d_rowinst, rowinst.data(), sizeof(int) * R, hipMemcpyHostToDevice));
    FPC_HIP(hipMemcpy(d_src, src.data(), sizeof(DevInstSrc) * ni, hipMemcpyHostToDevice));
    // size classes of every level, fixed now (the graph is static)
    std::vector<std::vector<int>> bounds(std::max(nsteps, 1));
    for (int l = L0; l >= 0; --l) {
        bounds[L0 - l] = device_class_bounds(ctx, l, mixed && l <= kMaxTemplL);
        if (trace_on()) {
            std::fprintf(stderr, "[fpc] graph level %d: class bounds", l);
            for (int b : bounds[L0 - l]) std::fprintf(stderr, " %d", b);
            std::fprintf(stderr, "\n");
        }
    }
    const size_t groups_lds = (size_t)2 * ((maxp + 31) / 32) * 4 + (size_t)3 * maxp * 4;
    if (groups_lds > 65536) {
        FPC_HIP(hipFuncSetAttribute((const void *)g_groups, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)groups_lds));
    }
    FPC_HIP(hipStreamSynchronize(st));

    // ---- capture
    const unsigned edge_grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((Emax + 255) / 256, 8 * ctx->num_cus));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const double t_cap = now_ms_g();
    FPC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    auto body = [&]() -> int {
        int r;
        g_fill_u32<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t *>(G.flags), sizeof(GFlags) / 4, 0u);
        g_fill_u32<<<1, 256, 0, st>>>(reinterpret_cast<uint32_t *>(fl_bad), ni, 0u);
        g_fill_u32<<<1, 256, 0, st>>>(reinterpret_cast<uint32_t *>(fl_del), 2 * ni, 0u);
        g_fill_u32<<<64, 256, 0, st>>>(reinterpret_cast<uint32_t *>(stats),
                                       (int64_t)sizeof(GStat) / 4 * ni * std::max(nsteps, 1), 0u);
        g_fill_u32<<<1, 32, 0, st>>>(ctx->flag.as<uint32_t>(), 2, 0u);
        for (int k = 0; k < ni; ++k) {
            const void *X = inst[k].X;
            if (inst[k].rows) {
                if ((r = gather_rows_enqueue(ctx, inst[k].X, P->x_dtype, inst[k].x_rows, inst[k].p, inst[k].rows,
                                             inst[k].n, ctx->x_copy.ptr, reinterpret_cast<int *>(&G.flags->bad_rows))))
                    return r;
                X = ctx->x_copy.ptr;
            }
            if ((r = corr_compute(ctx, X, P->x_dtype, inst[k].n, inst[k].p, FPC_CORR_FP64, ptrs.c64[k], false, false,
                                  true)))
                return r;
            if (mixed) {
                if (m32 == FPC_CORR_FP32) {
                    if ((r = corr_round_enqueue(ctx, ptrs.c64[k], ptrs.c32[k], inst[k].p, false))) return r;
                } else if ((r = corr_compute(ctx, X, P->x_dtype, inst[k].n, inst[k].p, m32, ptrs.c32[k], true, false,
                                             true))) {
                    return r;
                }
                if ((r = corr_max_abs_diff_enqueue(ctx, ptrs.c64[k], ptrs.c32[k], inst[k].p, cerr_slot + k))) return r;
            }
        }
        if ((r = first_level_batch_enqueue(ctx, fli, fb))) return r;
        for (int l = L0; l >= 0; --l) {
            const int step = L0 - l;
            G.l = l;
            G.stat = stats + (size_t)step * ni;
            const std::vector<int> &bd = bounds[step];
            G.ncls = (int)bd.size();
            for (int q = 0; q < G.ncls; ++q) G.cbound[q] = bd[q];
            std::vector<DeviceLevelClass> dcls(G.ncls);
            for (int q = 0; q < G.ncls; ++q) dcls[q] = DeviceLevelClass{bd[q], G.class_range + 2 * q};
            g_level_init<<<1, 256, 0, st>>>(G, n_cnt);
            g_csr_count<<<(unsigned)R, 64, 0, st>>>(G);
            g_scan_rows<<<1, kScanThreads, 0, st>>>(G);
            g_csr_fill<<<(unsigned)R, 64, 0, st>>>(G);
            g_groups<<<(unsigned)R, 256, groups_lds, st>>>(G, maxp);
            g_edge_count<<<(unsigned)R, 64, 0, st>>>(G);
            g_edge_classes<<<edge_grid, 256, 0, st>>>(G);
            g_class_ranges<<<1, 64, 0, st>>>(G);
            g_edge_fill<<<(unsigned)R, 64, 0, st>>>(G);
            void *itab = insts + inst_rec_bytes() * ni * step;
            const bool fp32 = mixed && l <= kMaxTemplL;
            if ((r = level_inst_table_enqueue(ctx, d_src, ni, l, P->recheck_margin > 0 ? P->recheck_margin : 1e-3,
                                              P->ill_cond_tau, fp32, itab)))
                return r;
            DeviceLevel D{};
            D.l = l;
            D.fp32 = fp32;
            D.edges = G.rec;
            D.cand = G.cand;
            D.insts = itab;
            D.minhit = G.minhit;
            D.counters = G.counters;
            D.inst_cnt = G.inst_cnt;
            D.queue = fp32 ? ctx->queue.as<int64_t>() : nullptr;
            D.queue_cap = fp32 ? queue_cap : 0;
            D.plan = plan;
            D.max_m_all = bd.back();
            D.classes = dcls.data();
            D.n_classes = G.ncls;
            if ((r = level_tests_device(ctx, D))) return r;
            g_apply<<<(unsigned)R, 64, 0, st>>>(G);
            g_level_stats<<<(unsigned)ni, 256, 0, st>>>(G);
        }
        FPC_HIP(hipGetLastError());
        return FPC_OK;
    };
    rc = body();
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    FPC_HIP(ec);
    const double t_inst = now_ms_g();
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    const double t_run = now_ms_g();
    if (e == hipSuccess) e = hipEventRecord(ctx->ev0, st);
    if (e == hipSuccess) e = hipGraphLaunch(exec, st);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev1, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    FPC_HIP(e);
    out.prep_ms = t_cap - t_start;
    out.capture_ms = t_inst - t_cap;
    out.instantiate_ms = t_run - t_inst;
    out.run_ms = now_ms_g() - t_run;
    float gms = 0.f;
    FPC_HIP(hipEventElapsedTime(&gms, ctx->ev0, ctx->ev1));

    // ---- results
    GFlags hf{};
    FPC_HIP(hipMemcpy(&hf, G.flags, sizeof(GFlags), hipMemcpyDeviceToHost));
    int cflags[2] = {0, 0};
    FPC_HIP(hipMemcpy(cflags, ctx->flag.ptr, sizeof(cflags), hipMemcpyDeviceToHost));
    if (cflags[0]) return FPC_ENONFINITE;
    if (cflags[1]) return FPC_ESINGULAR;
    if (hf.bad_rows) return FPC_EINVAL;
    std::vector<int> hbad(ni);
    std::vector<unsigned long long> hdel(ni), hcerr(ni);
    FPC_HIP(hipMemcpy(hbad.data(), fl_bad, sizeof(int) * ni, hipMemcpyDeviceToHost));
    for (int k = 0; k < ni; ++k)
        if (hbad[k]) return FPC_ESINGULAR;
    if (hf.overflow) return kGraphFallback;
    FPC_HIP(hipMemcpy(hdel.data(), fl_del, sizeof(unsigned long long) * ni, hipMemcpyDeviceToHost));
    FPC_HIP(hipMemcpy(hcerr.data(), cerr_slot, sizeof(unsigned long long) * ni, hipMemcpyDeviceToHost));
    std::vector<GStat> hst((size_t)ni * std::max(nsteps, 1));
    FPC_HIP(hipMemcpy(hst.data(), stats, sizeof(GStat) * hst.size(), hipMemcpyDeviceToHost));
    const int64_t nsep = (int64_t)hf.sep_fill;
    std::vector<GSep> hsep((size_t)nsep);
    std::vector<int32_t> hnodes((size_t)hf.node_fill);
    if (nsep) FPC_HIP(hipMemcpy(hsep.data(), G.sep, sizeof(GSep) * nsep, hipMemcpyDeviceToHost));
    if (!hnodes.empty())
        FPC_HIP(hipMemcpy(hnodes.data(), G.nodes, sizeof(int32_t) * hnodes.size(), hipMemcpyDeviceToHost));
    out.inst.assign(ni, GraphBatchOut::Inst{});
    for (int k = 0; k < ni; ++k) {
        GraphBatchOut::Inst &o = out.inst[k];
        const int p = inst[k].p;
        o.adj.resize((size_t)p * p);
        FPC_HIP(hipMemcpy(o.adj.data(), G.adj + gi[k].adj_off, (size_t)p * p, hipMemcpyDeviceToHost));
        double ce = 0.0;
        std::memcpy(&ce, &hcerr[k], sizeof(ce));
        o.c_err = mixed ? ce : 0.0;
        o.q = qk[k];
        fpc_level_stats f{};
        f.level = p - 2;
        f.max_cand = p - 2;
        f.edges_eligible = f.tests_possible = f.tests_executed = f.tests_required = (int64_t)p * (p - 1) / 2;
        f.deleted = (int64_t)hdel[k];
        o.levels.push_back(f);
        for (int step = 0; step < nsteps; ++step) {
            const int l = L0 - step;
            const GStat &s = hst[(size_t)step * ni + k];
            if (l > gi[k].cap || s.max_cand < l) continue;  // the instance did not run this level
            fpc_level_stats x{};
            x.level = l;
            x.max_cand = s.max_cand;
            x.edges_eligible = (int64_t)s.eligible;
            x.tests_possible = (int64_t)s.possible;
            x.tests_executed = (int64_t)s.executed;
            x.tests_rechecked = (int64_t)s.rechecked;
            x.deleted = (int64_t)s.deleted;
            x.tests_required = (int64_t)s.required;
            o.levels.push_back(x);
        }
    }
    for (const GSep &s : hsep) {
        GraphBatchOut::Inst &o = out.inst[s.inst];
        o.sep_pair.push_back(s.pair);
        o.sep_level.push_back(s.level);
        o.sep_off.push_back((int64_t)o.sep_nodes.size());
        o.sep_nodes.insert(o.sep_nodes.end(), hnodes.begin() + s.node_off, hnodes.begin() + s.node_off + s.level);
    }
    out.graph_ms = gms;
    out.total_ms = now_ms_g() - t_start;
    return FPC_OK;
}

}  // namespace fpc
