// Level tests of Algorithm 2 (Sec. 3.2) with the Fisher-z CI test of
// Sec. 2.2.2 and the partial correlation of Sec. 5:
//     H = H0 - H1 H2^{-1} H1^T,  r = h12 / sqrt(h11 h22),
//     independent iff sqrt(n - l - 3) |atanh r| <= q.
// H is formed through a Cholesky factorisation H2 = L L^T:
//     u = L^{-1} C_Ki, v = L^{-1} C_Kj,
//     h11 = 1 - u.u,  h22 = 1 - v.v,  h12 = C_ij - u.v
// (the unit diagonal of a correlation matrix is used directly).
//
// Work layout.  One level enumerates, for every edge e with m_e = |cand|
// >= l, the C(m_e, l) l-subsets of its sorted candidate list in
// lexicographic order; rank r of edge e is the r-th subset.  A launch
// covers a window of ranks [lo, hi) of every edge; a workgroup owns
// kRanksPerBlock consecutive ranks of one edge and first stages that
// edge's correlation entries in LDS (strict upper triangle over the
// candidates plus the i and j rows: m(m-1)/2 + 2m + 1 values).  Each
// wave walks 64 consecutive ranks per step: neighbouring lanes then share
// the first l-1 elements of K (broadcast LDS reads) and differ in the last
// one (consecutive LDS addresses).  Each lane runs one test with the
// factor in registers (l <= kMaxTemplL, l a template parameter).
//
// Edge deletion: a hit (independent test) at rank r lowers the edge's
// minhit to r with one atomicMin per wave (ballot of the lanes, lowest
// lane).  A wave or workgroup whose ranks all lie above the current minhit
// stops, so each edge's final minhit is the lexicographically first
// separating set whatever the launch order.
//
// Mixed precision: FP32 tests whose z lies within band of q (band = the
// stated margin plus a bound on the FP32 error of this test) are appended
// to a queue (ballot + prefix sum per wave) and re-run in FP64 from the
// FP64 matrix by the recheck kernel after each window's launch; degenerate
// FP32 tests are re-run too.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <type_traits>
#include <vector>

#include "fpc_internal.h"

namespace fpc {

namespace {

constexpr int kWaves = 4;
constexpr size_t kStaticLds = 256;  // LDS kept free for the kernels' static words (dynamic LDS cap)
constexpr int kSteps = 8;
constexpr int kRanksPerWave = 64 * kSteps;               // default ranks per wave, per-test kernel
constexpr int kGenericRanks = 16;                        // ranks per workgroup, wide-level kernel
constexpr double kErrSafety = 4.0;                       // multiplier of the FP32 error bound
constexpr int kSplitMinRanksPerWave = 256;  // triple kernel: smallest work item after splitting, per wave
constexpr int kMinhitEvery = 512;  // shared-prefix kernels: tests between reads of an edge's minimum hit

enum : int { DEC_DEP = 0, DEC_INDEP = 1, DEC_RECHECK = 2 };

__device__ __forceinline__ uint64_t load_minhit(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float rsq(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

// ------------------------------------------------------------------ views
// Candidate positions 0..m-1 index the edge's candidate list; i and j are
// addressed separately.  kk(row(a), b) = C(cand[a], cand[b]).
template <typename T>
struct PackedTile {
    const T *tri, *ci, *cj;
    T cij;
    int m;
    __device__ __forceinline__ int row(int a) const { return a * (2 * m - a - 3) / 2 - 1; }
    __device__ __forceinline__ T kk(int rowa, int b) const { return tri[rowa + b]; }  // a < b
    __device__ __forceinline__ T ki(int b) const { return ci[b]; }
    __device__ __forceinline__ T kj(int b) const { return cj[b]; }
    __device__ __forceinline__ T ij() const { return cij; }
};

template <typename T>
struct GlobalRows {
    const T *C;
    int p;
    const int32_t *cand;
    int i, j;
    __device__ __forceinline__ int row(int a) const { return cand[a] * p; }
    __device__ __forceinline__ T kk(int rowa, int b) const { return C[(size_t)rowa + cand[b]]; }
    __device__ __forceinline__ T ki(int b) const { return C[(size_t)i * p + cand[b]]; }
    __device__ __forceinline__ T kj(int b) const { return C[(size_t)j * p + cand[b]]; }
    __device__ __forceinline__ T ij() const { return C[(size_t)i * p + j]; }
};

// Rows of the index matrix B: positions are variable ids, any order.
template <typename T>
struct DirectRows {
    const T *C;
    int p, i, j;
    __device__ __forceinline__ int row(int a) const { return a * p; }
    __device__ __forceinline__ T kk(int rowa, int b) const { return C[(size_t)rowa + b]; }
    __device__ __forceinline__ T ki(int b) const { return C[(size_t)i * p + b]; }
    __device__ __forceinline__ T kj(int b) const { return C[(size_t)j * p + b]; }
    __device__ __forceinline__ T ij() const { return C[(size_t)i * p + j]; }
};

// ------------------------------------------------------------------ one test
// r and the conditioning measure rho = (smallest pivot of C_KK) *
// min(h11, h22) of the factorisation; ok is false for a degenerate test
// (pivot <= 0, h11 or h22 <= 0, |r| >= 1).
template <typename T, int L, class View>
__device__ __forceinline__ void pcor_reg(const View &V, const int *k, T &r, T &rho, bool &ok)
{
    constexpr int LL = L > 0 ? L : 1;
    T Lf[L > 0 ? L * (L + 1) / 2 : 1];
    T u[LL], v[LL], inv[LL];
    int rw[LL];
    ok = true;
    T dmin = T(1);
    T h11 = T(1), h22 = T(1), h12 = V.ij();
#pragma unroll
    for (int t = 0; t < L; ++t) rw[t] = V.row(k[t]);
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const int kt = k[t];
        T *Lt = Lf + t * (t + 1) / 2;
#pragma unroll
        for (int s = 0; s < t; ++s) {
            T a = V.kk(rw[s], kt);
            const T *Ls = Lf + s * (s + 1) / 2;
#pragma unroll
            for (int c = 0; c < s; ++c) a -= Lt[c] * Ls[c];
            Lt[s] = a * inv[s];
        }
        T d = T(1);
#pragma unroll
        for (int c = 0; c < t; ++c) d -= Lt[c] * Lt[c];
        ok = ok && (d > T(0));
        dmin = d < dmin ? d : dmin;
        inv[t] = rsq(d);
        T ai = V.ki(kt), aj = V.kj(kt);
#pragma unroll
        for (int c = 0; c < t; ++c) {
            ai -= Lt[c] * u[c];
            aj -= Lt[c] * v[c];
        }
        u[t] = ai * inv[t];
        v[t] = aj * inv[t];
        h11 -= u[t] * u[t];
        h22 -= v[t] * v[t];
        h12 -= u[t] * v[t];
    }
    ok = ok && (h11 > T(0)) && (h22 > T(0));
    rho = dmin * (h11 < h22 ? h11 : h22);
    r = h12 * rsq(h11 * h22);
    ok = ok && (fabs(r) < T(1));
}

struct Thresholds {
    double q;       // Phi^{-1}(1 - alpha/2)
    double r_lo;    // below: surely z < q
    double r_hi;    // above: surely z > q
    double sqrt_nu; // sqrt(n - l - 3)
    double band_z;  // mixed: stated margin (z units)
    double c_eff;   // mixed: entry error bound of the FP32 matrix + FP32 rounding
    double rb_lo;   // mixed: tanh((q - band_z) / sqrt_nu)
    double rb_hi;   // mixed: tanh((q + band_z) / sqrt_nu)
    double tau;     // mixed: FP32 tests with rho below this are re-run in FP64
};

// Per-instance parameters of a level: the matrices, their row stride and
// the thresholds.  Every edge names its instance, so one launch can serve
// several independent problems.
struct InstRec {
    const void *C;       // matrix of the test precision
    const double *C64;   // FP64 matrix (recheck, wide levels)
    int64_t ld;          // row stride: the instance's p
    Thresholds th;
};

// FP64 decision identical in form to the reference rule z <= q.
__device__ __forceinline__ bool decide64(double r, bool ok, const Thresholds &th)
{
    if (!ok) return false;
    const double a = fabs(r);
    if (a < th.r_lo) return true;
    if (a > th.r_hi) return false;
    return th.sqrt_nu * fabs(atanh(r)) <= th.q;
}

// Mixed form, per-test kernel: decided in FP32 when z lies outside the
// band of q (stated margin plus the error bound of this test), else left to
// the FP64 re-run, as are ill-conditioned tests (rho below tau).  The bound:
// an absolute error e in the entries of the (l+2)x(l+2) matrix (FP32 matrix
// and arithmetic) moves H by at most about (l+2) e / dmin(C_KK) and r by at
// most twice that over min(h11, h22), i.e. 2 (l+2) e / rho; z by that times
// sqrt(n-l-3) / (1 - r^2).  kErrSafety covers the factor 2 and more.
template <int L>
__device__ __forceinline__ int decide32(float r, float rho, bool ok, const Thresholds &th)
{
    if (!ok || !(rho >= (float)th.tau)) return DEC_RECHECK;
    const float a = fabsf(r);
    const float snu = (float)th.sqrt_nu;
    const float z = snu * 0.5f * __logf((1.0f + a) / (1.0f - a));
    const float err = (float)kErrSafety * snu * (float)th.c_eff * (float)(L + 2) / (rho * (1.0f - a * a));
    const float band = (float)th.band_z + err;
    const float qf = (float)th.q;
    if (z < qf - band) return DEC_INDEP;
    if (z > qf + band) return DEC_DEP;
    return DEC_RECHECK;
}

// ------------------------------------------------------------------ enumeration
// C(a, b) from the table, through C(a, b) = C(a, a - b): every value the
// enumeration reads is at most C(m, l) < 2^63, which forces min(b, a-b) <= 33.
__device__ __forceinline__ int64_t binom_at(const int64_t *__restrict__ binom, int a, int b)
{
    if (b < 0 || b > a) return 0;
    const int bb = min(b, a - b);
    return bb < kBinomCols ? binom[a * kBinomCols + bb] : INT64_MAX;
}

// Lexicographic unranking of rank R among the L-subsets of m positions.
// It reads C(a, b) for b < L only; STRIDE = columns of the table.
template <int L, int STRIDE = kBinomCols>
__device__ __forceinline__ void unrank(int64_t R, int m, const int64_t *__restrict__ binom, int *c)
{
    int x = 0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        for (;;) {
            const int a = m - 1 - x;
            if (a < L - 1 - t) break;  // never taken for R < C(m, L)
            const int b = L - 1 - t, bb = min(b, a - b);
            const int64_t cnt = binom[a * STRIDE + bb];
            if (R < cnt) break;
            R -= cnt;
            ++x;
        }
        c[t] = x;
        ++x;
    }
}

// The same unranking by a whole wave (R and m uniform, every lane active),
// one coalesced load per element instead of a walk of up to m dependent
// loads.  Subsets of the positions >= x0 whose element t lies before x
// number C(m - x0, L - t) - C(m - x, L - t) (hockey-stick identity), so the
// element is the last x with C(m - x, L - t) >= C(m - x0, L - t) - R; those
// x form a prefix of the lanes, read off a ballot.  binT is column-major.
template <int L>
__device__ __forceinline__ void unrank_wave(int64_t R, int m, const int64_t *__restrict__ binT, int *c)
{
    const int lane = threadIdx.x % 64;
    int x0 = 0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const int k = L - t;
        const int64_t *col = binT + (size_t)k * kBinomRows;
        const int64_t top = col[m - x0];  // the subsets left: C(m - x0, L - t) > R
        const int64_t need = top - R;
        const int last = m - k;  // element t leaves room for the L - 1 - t after it
        int x = x0;
        for (int base = x0; base <= last; base += 64) {
            const int xl = base + lane;
            const bool ok = xl <= last && col[m - xl] >= need;
            const int n = __popcll(__ballot(ok));
            if (n > 0) x = base + n - 1;
            if (n < 64) break;  // uniform
        }
        R -= top - col[m - x];
        c[t] = x;
        x0 = x + 1;
    }
}

// Given c = the combination at some rank b (wave-uniform), set my = the
// combination at rank b + lane and advance c to rank b + 64.  Lanes past
// the last combination keep the (valid) initial my.  Returns false when no
// combination follows rank b + 63.
template <int L>
__device__ __forceinline__ bool walk64(int *c, int m, int lane, int *my)
{
    int cur[L];
#pragma unroll
    for (int s = 0; s < L; ++s) {
        cur[s] = c[s];
        my[s] = s;
    }
    int off = 0;
    for (int guard = 0; guard <= 64; ++guard) {
        const int leaves = m - cur[L - 1];
        const int t = lane - off;
        if (t >= 0 && t < leaves) {
#pragma unroll
            for (int s = 0; s < L - 1; ++s) my[s] = cur[s];
            my[L - 1] = cur[L - 1] + t;
        }
        if (off + leaves > 64) {
#pragma unroll
            for (int s = 0; s < L - 1; ++s) c[s] = cur[s];
            c[L - 1] = cur[L - 1] + (64 - off);
            return true;
        }
        off += leaves;
        int a = -1;
#pragma unroll
        for (int s = 0; s + 1 < L; ++s)
            if (cur[s] != m - L + s) a = s;
        if (a < 0) return false;
#pragma unroll
        for (int s = 0; s < L; ++s) {
            if (s == a) cur[s] += 1;
            else if (s > a) cur[s] = cur[s - 1] + 1;
        }
        if (off == 64) {
#pragma unroll
            for (int s = 0; s < L; ++s) c[s] = cur[s];
            return true;
        }
    }
    return false;
}

struct LevelArgs {
    const EdgeRec *edges;
    const int32_t *cand;
    const InstRec *inst;      // per-instance matrices and thresholds
    const int64_t *blockoff;  // n_edges + 1 prefix of work items per edge (this window)
    const int64_t *n_items;   // work items of this window (written on the device)
    unsigned long long *item_ctr;  // next work item (zeroed with the window's plan)
    const int64_t *binom;
    const int64_t *binomT;  // the binomial table column-major
    uint64_t *minhit;
    unsigned long long *counters;  // [1] recheck queue length, [3] queue overflow
    unsigned long long *inst_cnt;  // per instance: tests executed, tests re-run in FP64
    int64_t *queue;       // recheck queue: (level edge index, rank) pairs
    int64_t queue_cap;
    int64_t edge_base;    // level index of edges[0] (the launch's class starts there)
    int64_t n_edges;
    int64_t win_lo, win_hi;
    int ranks_per_block;
    int max_m;  // largest candidate set of the level
    int pdec_n;  // entries of the triple kernel's pair table
    // diagnostic run (fpc_level_series): r and the decision of every rank
    // of the window at [rank - diag_lo]; no early exit, no recheck queue
    double *diag_r;
    uint8_t *diag_dec;
    int64_t diag_lo;
    // device-built level (many instances, level loop on the device): the
    // class's edge range [dclass[0], dclass[1]) of the level's table, read
    // at launch instead of edges/minhit/n_edges/edge_base (then relative to
    // the level's table); blockoff then points at the class's plan region
    // less dclass[0]
    const int64_t *dclass;
};

// Moves the launch's view to its class when the class range lives on the
// device (the kernels take A by value).
__device__ __forceinline__ void apply_dclass(LevelArgs &A)
{
    if (A.dclass) {
        const int64_t b = A.dclass[0], e = A.dclass[1];
        A.edges += b;
        A.minhit += b;
        A.blockoff += b;
        A.n_edges = e - b;
        A.edge_base = b;
    }
}

__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A value equal in every lane, marked so for the compiler (kept in SGPRs)
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Persistent workgroups: each takes work items (a run of consecutive ranks
// of one edge) from the window's counter until none is left.  Item bodies
// may return early only uniformly over the workgroup or after their last
// block-wide barrier; the barrier after each item protects the LDS tile.
// A workgroup's first item is its own index; later ones come from the
// counter (offset by the grid size), which a launch with no more items than
// workgroups never touches: a counter that every workgroup hits at once
// serialises the launch's start.
template <class F>
__device__ __forceinline__ void for_each_item(const LevelArgs &A, F &&body)
{
    __shared__ int64_t next_item;
    const int64_t total = *A.n_items;
    int64_t blk = blockIdx.x;
    for (;;) {
        if (blk >= total) return;  // uniform
        body(blk);
        __syncthreads();
        if (total <= (int64_t)gridDim.x) return;  // every item had a workgroup of its own
        if (threadIdx.x == 0) next_item = (int64_t)gridDim.x + (int64_t)atomicAdd(A.item_ctr, 1ull);
        __syncthreads();
        blk = uniform_i64(next_item);
    }
}

// Tests run, per instance: each wave sums them in a register and adds the
// sum to the instance's shared counter when it moves on to an item of
// another instance and when it ends, so the counter takes a few atomics per
// wave instead of one per work item.
struct ExecCount {
    int inst = -1;
    unsigned long long n = 0;
    __device__ void add(const LevelArgs &A, int i, unsigned long long k)
    {
        if (i != inst) {
            flush(A);
            inst = i;
        }
        n += k;
    }
    __device__ void flush(const LevelArgs &A)
    {
        if (n && threadIdx.x % 64 == 0) atomicAdd(&A.inst_cnt[2 * inst], n);
        n = 0;
    }
};

// Persistent grid: as many workgroups as fit on the device at once, and no
// more than the window can possibly use.
// The register and wave limits come from the runtime's occupancy query;
// the LDS limit is applied here from the CU's LDS size, since the query
// does not account for workgroups that opt into more than 64 KiB.
thread_local int g_max_blocks_per_cu = 0;  // tuning cap of the launch being issued (0: none)
thread_local unsigned g_last_grid = 0;      // grid of the last launch sized here (for tracing)

unsigned resident_grid(const void *fn, int threads, size_t shm, int64_t ub, int cus, size_t lds_cu)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (shm > 0) per_cu = std::min<int>(per_cu, std::max<int>(1, (int)(lds_cu / (shm + 256))));
    if (g_max_blocks_per_cu > 0) per_cu = std::min(per_cu, g_max_blocks_per_cu);
    g_last_grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ub, (int64_t)per_cu * cus));
    return g_last_grid;
}

__device__ __forceinline__ int64_t find_edge(const int64_t *__restrict__ off, int64_t n, int64_t b)
{
    int64_t lo = 0, hi = n;  // off[lo] <= b < off[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// One row of the strict upper triangle per wave at a time, lanes along the
// row (coalesced reads of C, consecutive LDS writes).
template <typename T>
__device__ void stage_tile(const T *__restrict__ C, int p, const int32_t *__restrict__ cand, int m, int i, int j,
                           T *tri, T *ci, T *cj)
{
    const int lane = threadIdx.x % 64, nw = blockDim.x / 64;
    for (int a = threadIdx.x / 64; a < m - 1; a += nw) {
        const int base = a * (2 * m - a - 3) / 2 - 1;
        const T *Crow = C + (size_t)cand[a] * p;
        for (int b = a + 1 + lane; b < m; b += 64) tri[base + b] = Crow[cand[b]];
    }
    for (int b = threadIdx.x; b < m; b += blockDim.x) {
        ci[b] = C[(size_t)i * p + cand[b]];
        cj[b] = C[(size_t)j * p + cand[b]];
    }
}

// ------------------------------------------------------------------ level kernel
template <typename T, int L, bool TILE>
__device__ __forceinline__ void level_item(const LevelArgs &A, int64_t blk, unsigned char *smem, ExecCount &ec)
{
    const int64_t e = find_edge(A.blockoff, A.n_edges, blk);
    const EdgeRec E = A.edges[e];
    const int m = E.m;
    const int64_t rpb = A.ranks_per_block, rpw = rpb / kWaves;
    const int64_t r0 = A.win_lo + (blk - A.blockoff[e]) * rpb;
    const int64_t r1 = min(r0 + rpb, min(A.win_hi, E.ntests));
    if (r0 >= r1) return;  // uniform
    __shared__ int skip;
    if (threadIdx.x == 0) skip = load_minhit(&A.minhit[e]) < (uint64_t)r0;
    __syncthreads();
    if (skip) return;  // uniform
    const InstRec &I = A.inst[E.inst];
    const T *C = static_cast<const T *>(I.C);
    const int p = (int)I.ld;
    const Thresholds th = I.th;
    const int32_t *cand = A.cand + E.cand_off;

    PackedTile<T> tile{};
    GlobalRows<T> glob{C, p, cand, E.i, E.j};
    if constexpr (TILE) {
        T *tri = reinterpret_cast<T *>(smem);
        const int ntri = m * (m - 1) / 2;
        T *ci = tri + ntri, *cj = ci + m;
        stage_tile<T>(C, p, cand, m, E.i, E.j, tri, ci, cj);
        tile = PackedTile<T>{tri, ci, cj, C[(size_t)E.i * p + E.j], m};
        __syncthreads();
    }
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int64_t wlo = r0 + (int64_t)wave * rpw;
    const int64_t whi = min(wlo + rpw, r1);
    uint64_t executed = 0;
    if (wlo < whi) {
        constexpr int LL = L > 0 ? L : 1;
        int c[LL], my[LL];
        if constexpr (L > 0) unrank<L>(wlo, m, A.binom, c);
        // the edge's shared minimum is read one round ahead, so the wave
        // does not wait for the load (a hit elsewhere stops it one round later)
        uint64_t mh_ahead = load_minhit(&A.minhit[e]);
        for (int64_t base = wlo; base < whi; base += 64) {
            const unsigned long long mh = (unsigned long long)uniform_i64((int64_t)mh_ahead);
            mh_ahead = load_minhit(&A.minhit[e]);
            if (mh < (unsigned long long)base) break;
            bool more = true;
            if constexpr (L > 0) more = walk64<L>(c, m, lane, my);
            const bool valid = base + lane < whi;
            T r, rho;
            bool ok;
            if constexpr (TILE) pcor_reg<T, L>(tile, my, r, rho, ok);
            else pcor_reg<T, L>(glob, my, r, rho, ok);
            int dec;
            if constexpr (sizeof(T) == 8) dec = decide64((double)r, ok, th) ? DEC_INDEP : DEC_DEP;
            else dec = decide32<L>((float)r, (float)rho, ok, th);
            const uint64_t nvalid = (uint64_t)min((int64_t)64, whi - base);
            executed += nvalid;
            if (A.diag_r) {  // uniform
                if (valid) {
                    A.diag_r[base + lane - A.diag_lo] = ok ? (double)r : (double)NAN;
                    A.diag_dec[base + lane - A.diag_lo] = (uint8_t)dec;
                }
                if (!more) break;
                continue;
            }
            if constexpr (sizeof(T) == 4) {
                const bool rq = valid && dec == DEC_RECHECK;
                const unsigned long long qb = __ballot(rq);
                if (qb) {
                    unsigned long long slot = 0;
                    if (lane == 0) slot = atomicAdd(&A.counters[1], (unsigned long long)__popcll(qb));
                    slot = __shfl(slot, 0);
                    if (rq) {
                        const unsigned long long idx = slot + __popcll(qb & ((1ull << lane) - 1ull));
                        if ((int64_t)idx < A.queue_cap) {
                            A.queue[2 * idx] = e + A.edge_base;
                            A.queue[2 * idx + 1] = base + lane;
                        }
                    }
                }
            }
            const unsigned long long hb = __ballot(valid && dec == DEC_INDEP);
            if (hb) {
                if (lane == 0) atomicMin((unsigned long long *)&A.minhit[e], (unsigned long long)(base + __ffsll((long long)hb) - 1));
                break;
            }
            if (!more) break;
        }
    }
    ec.add(A, E.inst, (unsigned long long)executed);
}

template <typename T, int L, bool TILE>
__global__ __launch_bounds__(256) void level_kernel(LevelArgs A)
{
    apply_dclass(A);
    extern __shared__ __align__(16) unsigned char smem[];
    ExecCount ec;
    for_each_item(A, [&](int64_t blk) { level_item<T, L, TILE>(A, blk, smem, ec); });
    ec.flush(A);
}

// Binomial rows the recheck kernel stages in LDS: C(a, b), a < max_m,
// b < L, when they fit in kRecheckLds bytes (else it reads the global table).
constexpr size_t kRecheckLds = 32768;
__host__ __device__ inline size_t recheck_lds_bytes(int max_m, int L)
{
    const size_t b = sizeof(int64_t) * (size_t)max_m * (size_t)(L > 0 ? L : 1);
    return b <= kRecheckLds ? b : 0;
}

// FP64 re-run of queued FP32 tests (rank below the edge's current minhit).
template <int L>
__global__ __launch_bounds__(256) void recheck_kernel(LevelArgs A)
{
    extern __shared__ int64_t bl[];  // C(a, b) at a * L + b
    constexpr int LL = L > 0 ? L : 1;
    const bool staged = recheck_lds_bytes(A.max_m, L) > 0;
    if (staged) {
        for (int t = threadIdx.x; t < A.max_m * LL; t += blockDim.x) {
            const int a = t / LL, b = t % LL;
            bl[t] = binom_at(A.binom, a, b);
        }
        __syncthreads();
    }
    const unsigned long long queued = A.counters[1];
    const unsigned long long total = min((unsigned long long)A.queue_cap, queued);
    if (blockIdx.x == 0 && threadIdx.x == 0 && queued > (unsigned long long)A.queue_cap)
        atomicMax(&A.counters[3], 1ull);  // entries were dropped: the caller re-runs the level in FP64
    for (unsigned long long idx = (unsigned long long)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (unsigned long long)gridDim.x * 256) {
        const int64_t e = A.queue[2 * idx], R = A.queue[2 * idx + 1];
        const bool run = (uint64_t)R < load_minhit(&A.minhit[e]);
        int inst = -1;
        if (run) {
            const EdgeRec E = A.edges[e];
            inst = E.inst;
            int k[L > 0 ? L : 1];
            if constexpr (L > 0) {
                if (staged) unrank<L, L>(R, E.m, bl, k);
                else unrank<L>(R, E.m, A.binom, k);
            }
            const InstRec &I = A.inst[E.inst];
            GlobalRows<double> g{I.C64, (int)I.ld, A.cand + E.cand_off, E.i, E.j};
            double r, rho;
            bool ok;
            pcor_reg<double, L>(g, k, r, rho, ok);
            if (decide64(r, ok, I.th)) atomicMin((unsigned long long *)&A.minhit[e], (unsigned long long)R);
        }
        // re-run counts: one atomic per wave when the wave's re-runs share
        // an instance (the usual case), per lane otherwise; a single
        // counter hit by every lane would serialise the launch
        const unsigned long long mask = __ballot(run);
        if (mask) {
            const int lead = __ffsll((long long)mask) - 1;
            const int inst0 = __shfl(inst, lead);
            if (__all(!run || inst == inst0)) {
                if ((int)(threadIdx.x % 64) == lead)
                    atomicAdd(&A.inst_cnt[2 * inst0 + 1], (unsigned long long)__popcll(mask));
            } else if (run) {
                atomicAdd(&A.inst_cnt[2 * inst + 1], 1ull);
            }
        }
    }
}


// ------------------------------------------------------------------ pair kernel (l >= 2)
// Tests of one edge in lexicographic order are grouped by their first
// l-2 elements Q; the last two (a < b) range over the positions after
// max(Q).  With L_Q the Cholesky factor of C_QQ and, for every later
// position x, w_x = L_Q^{-1} C_Qx, the Schur complement of C_QQ is
//     S_xy = C_xy - w_x.w_y,   S_xi = C_xi - w_x.u_Q,   S_xj = C_xj - w_x.v_Q
// (u_Q = L_Q^{-1} C_Qi, v_Q = L_Q^{-1} C_Qj), and the test of K = Q + {a,b}
// eliminates a and b from it:
//     l1 = S_ab / sqrt(S_aa),  d2 = S_bb - l1^2,
//     ua = S_ai / sqrt(S_aa),  ub = (S_bi - l1 ua) / sqrt(d2)  (same for j)
//     h11 = H11_Q - ua^2 - ub^2, h22 = H22_Q - va^2 - vb^2, h12 = H12_Q - ua va - ub vb
// -- the same factorisation of [K, i, j] as a per-test Cholesky, with the
// Q part shared.  A wave walks kPairRanksPerWave consecutive ranks; per Q
// it builds a table of the per-position quantities in its LDS slice (one
// lane per position) and then runs 64 pairs per step, decoding the pair
// index in the triangle of the positions after max(Q).
constexpr int kPairRanksPerWave = 2048;  // default ranks per wave, shared-prefix kernels

template <typename T, int QL>
struct PairLayout {
    static constexpr int V = 16 / (int)sizeof(T);           // elements per 16-byte load
    static constexpr int nA = QL + 5;                        // w[QL], 1/sqrt(S_xx), S_xi/sqrt(S_xx), S_xj/sqrt(S_xx),
                                                             // S_xx, row offset of x in the packed tile
    static constexpr int nB = QL + 3;                        // w[QL], S_xx, S_xi, S_xj
    static constexpr int SA = (nA + V - 1) / V * V;
    static constexpr int SB = (nB + V - 1) / V * V;
    static constexpr int S = SA + SB;                        // elements per position
};

// Lane mask of a condition across the wave (a bool straight into the
// ballot, so the mask is not rebuilt from a 0/1 integer).
__device__ __forceinline__ unsigned long long wave_mask(bool c) { return __builtin_amdgcn_ballot_w64(c); }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reciprocal square root: the hardware approximation in FP32 (about 1 ulp;
// a denormal or zero argument gives +inf, which the positivity checks of
// the test then reject), the accurate library routine in FP64.
__device__ __forceinline__ float rsqv(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqv(double x) { return rsqrt(x); }

__device__ __forceinline__ void put_int(float &d, int v) { d = __int_as_float(v); }
__device__ __forceinline__ void put_int(double &d, int v) { d = (double)v; }
__device__ __forceinline__ int get_int(float d) { return __float_as_int(d); }
__device__ __forceinline__ int get_int(double d) { return (int)d; }

// Decision of one FP32 shared-prefix test in r space (band and error bound,
// as in decide32): independent when |r| < rlo - errk/rho, dependent when
// |r| > rhi + errk/rho, else re-run in FP64, as are tests with rho below
// tau (ill-conditioned); rho > 0 whenever ok, so the bounds are compared
// after multiplying through by rho.
__device__ __forceinline__ int decide32r(float r, float rho, bool ok, float rlo, float rhi, float errk, float tau)
{
    if (!ok || !(rho >= tau)) return DEC_RECHECK;
    const float a = fabsf(r);
    if ((rlo - a) * rho > errk) return DEC_INDEP;
    if ((a - rhi) * rho > errk) return DEC_DEP;
    return DEC_RECHECK;
}

// The same decision as two flags, without the band products: with
// t = |r| rho, independent when t < rho rlo - errk, dependent when
// t > rho rhi + errk (neither: the FP64 re-run).
__device__ __forceinline__ void decide32b(float r, float rho, bool ok, float rlo, float rhi, float errk, float tau,
                                          bool &indep, bool &dep)
{
    const bool live = ok && rho >= tau;
    const float t = fabsf(r) * rho;
    indep = live && t < fmaf(rho, rlo, -errk);
    dep = live && t > fmaf(rho, rhi, errk);
}

// Smaller of two positive floats through their bit patterns (positive
// floats order as integers); the result is used only when both are > 0.
__device__ __forceinline__ float pos_min(float a, float b)
{
    return __int_as_float(min(__float_as_int(a), __float_as_int(b)));
}

// Row of the reversed pair index u in a triangle: rr with
// rr(rr+1)/2 <= u < (rr+1)(rr+2)/2.  u < 2^19 (lists shorter than 1024), so
// the products fit the 24-bit multiplier.
__device__ __forceinline__ unsigned tri_root(unsigned u)
{
    unsigned rr = (unsigned)((__builtin_amdgcn_sqrtf(8.0f * (float)u + 1.0f) - 1.0f) * 0.5f);
    rr += (__umul24(rr + 1u, rr + 2u) >> 1) <= u ? 1u : 0u;
    rr -= (__umul24(rr, rr + 1u) >> 1) > u ? 1u : 0u;
    return rr;
}

template <typename T, int QL>
__device__ __forceinline__ void pair_item(const LevelArgs &A, int64_t blk, unsigned char *smem, ExecCount &ec)
{
    using Lay = PairLayout<T, QL>;
    constexpr int L = QL + 2;
    constexpr int QLL = QL > 0 ? QL : 1;
    const int64_t e = find_edge(A.blockoff, A.n_edges, blk);
    const EdgeRec E = A.edges[e];
    const int m = E.m;
    const int64_t rpb = A.ranks_per_block, rpw = rpb / kWaves;
    const int64_t r0 = A.win_lo + (blk - A.blockoff[e]) * rpb;
    const int64_t r1 = min(r0 + rpb, min(A.win_hi, E.ntests));
    if (r0 >= r1) return;  // uniform
    __shared__ int skip;
    if (threadIdx.x == 0) skip = load_minhit(&A.minhit[e]) < (uint64_t)r0;
    __syncthreads();
    if (skip) return;  // uniform
    const InstRec &I = A.inst[E.inst];
    const T *C = static_cast<const T *>(I.C);
    const int p = (int)I.ld;
    const Thresholds th = I.th;
    const int32_t *cand = A.cand + E.cand_off;
    T *tri = reinterpret_cast<T *>(smem);
    const int ntri = m * (m - 1) / 2;
    T *ci = tri + ntri, *cj = ci + m;
    stage_tile<T>(C, p, cand, m, E.i, E.j, tri, ci, cj);
    const T cij = C[(size_t)E.i * p + E.j];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    // per-wave table slice, 16-byte aligned after the tile
    const size_t tile_elems = ((size_t)ntri + 2 * (size_t)m + Lay::V - 1) / Lay::V * Lay::V;
    T *tab = tri + tile_elems + (size_t)wave * A.max_m * Lay::S;
    __syncthreads();

    const int64_t wlo = r0 + (int64_t)wave * rpw;
    const int64_t whi = min(wlo + rpw, r1);
    if (wlo >= whi) return;  // no later block-wide barrier
    const auto row = [&](int a) { return a * (2 * m - a - 3) / 2 - 1; };

    // first test of the range: K = Q + {a, b}
    int c[L];
    unrank_wave<L>(wlo, m, A.binomT, c);
    int Q[QLL];
#pragma unroll
    for (int t = 0; t < QL; ++t) Q[t] = c[t];
    int sQ = QL > 0 ? Q[QL - 1] + 1 : 0;  // first position after Q
    int n = m - sQ;
    int tau;
    {
        const int a0 = c[L - 2] - sQ, b0 = c[L - 1] - sQ;
        tau = a0 * (2 * n - a0 - 1) / 2 + (b0 - a0 - 1);
    }
    int64_t rank = wlo;
    int64_t remaining = whi - wlo;
    uint64_t executed = 0;
    const float errk = (float)(kErrSafety * th.c_eff * (L + 2));
    const float rlo32 = (float)th.rb_lo, rhi32 = (float)th.rb_hi, tau32 = (float)th.tau;
    while (remaining > 0) {
        const unsigned long long mh = (unsigned long long)uniform_i64((int64_t)load_minhit(&A.minhit[e]));
        if (mh < (unsigned long long)rank) break;
        // ---- Q state: L_Q, u_Q, v_Q, H_Q (identical in every lane)
        T LQ[QL > 0 ? QL * (QL + 1) / 2 : 1], invQ[QLL], uQ[QLL], vQ[QLL];
        int rwQ[QLL];
        T H11 = T(1), H22 = T(1), H12 = cij, dminQ = T(1);
        bool okQ = true;
#pragma unroll
        for (int t = 0; t < QL; ++t) rwQ[t] = row(Q[t]);
#pragma unroll
        for (int t = 0; t < QL; ++t) {
            T *Lt = LQ + t * (t + 1) / 2;
#pragma unroll
            for (int s2 = 0; s2 < t; ++s2) {
                T a = tri[rwQ[s2] + Q[t]];
                const T *Ls = LQ + s2 * (s2 + 1) / 2;
#pragma unroll
                for (int q = 0; q < s2; ++q) a -= Lt[q] * Ls[q];
                Lt[s2] = a * invQ[s2];
            }
            T d = T(1);
#pragma unroll
            for (int q = 0; q < t; ++q) d -= Lt[q] * Lt[q];
            okQ = okQ && d > T(0);
            dminQ = d < dminQ ? d : dminQ;
            invQ[t] = rsqv(d);
            T ai = ci[Q[t]], aj = cj[Q[t]];
#pragma unroll
            for (int q = 0; q < t; ++q) {
                ai -= Lt[q] * uQ[q];
                aj -= Lt[q] * vQ[q];
            }
            uQ[t] = ai * invQ[t];
            vQ[t] = aj * invQ[t];
            H11 -= uQ[t] * uQ[t];
            H22 -= vQ[t] * vQ[t];
            H12 -= uQ[t] * vQ[t];
        }
        // ---- per-position table for x in [sQ, m)
        wave_sync();  // previous Q's table fully read
        for (int xp = lane; xp < n; xp += 64) {
            const int x = sQ + xp;
            T w[QLL];
#pragma unroll
            for (int t = 0; t < QL; ++t) {
                T a = tri[rwQ[t] + x];
#pragma unroll
                for (int q = 0; q < t; ++q) a -= LQ[t * (t + 1) / 2 + q] * w[q];
                w[t] = a * invQ[t];
            }
            T sxx = T(1), sxi = ci[x], sxj = cj[x];
#pragma unroll
            for (int t = 0; t < QL; ++t) {
                sxx -= w[t] * w[t];
                sxi -= w[t] * uQ[t];
                sxj -= w[t] * vQ[t];
            }
            const T i1 = sxx > T(0) ? rsqv(sxx) : T(0);
            T *ea = tab + (size_t)xp * Lay::S, *eb = ea + Lay::SA;
#pragma unroll
            for (int t = 0; t < QL; ++t) {
                ea[t] = w[t];
                eb[t] = w[t];
            }
            ea[QL] = i1;
            ea[QL + 1] = sxi * i1;
            ea[QL + 2] = sxj * i1;
            ea[QL + 3] = sxx;
            put_int(ea[QL + 4], row(x));
            eb[QL] = sxx;
            eb[QL + 1] = sxi;
            eb[QL + 2] = sxj;
        }
        wave_sync();
        // ---- pairs tau .. tau + cnt - 1 of this Q
        const int P = n * (n - 1) / 2;
        const int cnt = (int)min((int64_t)(P - tau), remaining);
        bool hit_found = false;
        for (int it = 0; it < cnt; it += 64) {
            const bool valid = it + lane < cnt;
            // pair index t -> (a', b') in the triangle over n positions,
            // from the reversed index u = P-1-t: u = rr(rr+1)/2 + (n-1-b')
            const unsigned t = (unsigned)(tau + min(it + lane, cnt - 1));
            const unsigned u = (unsigned)P - 1u - t;
            const unsigned rr = tri_root(u);
            const int ap = n - 2 - (int)rr, bp = n - 1 - (int)(u - (__umul24(rr, rr + 1u) >> 1));
            const T *ea = tab + (size_t)ap * Lay::S;
            const T *eb = tab + (size_t)bp * Lay::S + Lay::SA;
            T sab = tri[get_int(ea[QL + 4]) + sQ + bp];
#pragma unroll
            for (int q = 0; q < QL; ++q) sab -= ea[q] * eb[q];
            const T i1 = ea[QL], ua = ea[QL + 1], va = ea[QL + 2], d1 = ea[QL + 3];
            const T sbb = eb[QL], sbi = eb[QL + 1], sbj = eb[QL + 2];
            const T l1 = sab * i1;
            const T d2 = sbb - l1 * l1;
            const T i2 = rsqv(d2);
            const T ub = (sbi - l1 * ua) * i2, vb = (sbj - l1 * va) * i2;
            const T h11 = H11 - ua * ua - ub * ub;
            const T h22 = H22 - va * va - vb * vb;
            const T h12 = H12 - ua * va - ub * vb;
            bool ok = okQ && d1 > T(0) && d2 > T(0) && h11 > T(0) && h22 > T(0);
            const T r = h12 * rsqv(h11 * h22);
            ok = ok && fabs(r) < T(1);
            int dec;
            if constexpr (sizeof(T) == 8) {
                dec = decide64((double)r, ok, th) ? DEC_INDEP : DEC_DEP;
            } else {
                const float rho = fminf((float)dminQ, fminf((float)d1, (float)d2)) * fminf((float)h11, (float)h22);
                dec = decide32r((float)r, rho, ok, rlo32, rhi32, errk, tau32);
            }
            executed += (uint64_t)min(64, cnt - it);
            if (A.diag_r) {  // uniform
                if (valid) {
                    A.diag_r[rank + it + lane - A.diag_lo] = ok ? (double)r : (double)NAN;
                    A.diag_dec[rank + it + lane - A.diag_lo] = (uint8_t)dec;
                }
                continue;
            }
            if constexpr (sizeof(T) == 4) {
                const bool rq = valid && dec == DEC_RECHECK;
                const unsigned long long qb = __ballot(rq);
                if (qb) {
                    unsigned long long slot = 0;
                    if (lane == 0) slot = atomicAdd(&A.counters[1], (unsigned long long)__popcll(qb));
                    slot = __shfl(slot, 0);
                    if (rq) {
                        const unsigned long long idx = slot + __popcll(qb & ((1ull << lane) - 1ull));
                        if ((int64_t)idx < A.queue_cap) {
                            A.queue[2 * idx] = e + A.edge_base;
                            A.queue[2 * idx + 1] = rank + it + lane;
                        }
                    }
                }
            }
            const unsigned long long hb = __ballot(valid && dec == DEC_INDEP);
            if (hb) {
                if (lane == 0)
                    atomicMin((unsigned long long *)&A.minhit[e],
                              (unsigned long long)(rank + it + __ffsll((long long)hb) - 1));
                hit_found = true;
                break;
            }
        }
        if (hit_found) break;
        rank += cnt;
        remaining -= cnt;
        if (remaining <= 0) break;
        // ---- next Q: next (L-2)-combination of positions [0, m-2)
        if constexpr (QL == 0) {
            break;
        } else {
            int a = -1;
#pragma unroll
            for (int t = 0; t < QL; ++t)
                if (Q[t] != (m - 2) - QL + t) a = t;
            if (a < 0) break;
#pragma unroll
            for (int t = 0; t < QL; ++t) {
                if (t == a) Q[t] += 1;
                else if (t > a) Q[t] = Q[t - 1] + 1;
            }
            sQ = Q[QL - 1] + 1;
            n = m - sQ;
            tau = 0;
        }
    }
    ec.add(A, E.inst, (unsigned long long)executed);
}

template <typename T, int QL>
__global__ __launch_bounds__(256) void pair_kernel(LevelArgs A)
{
    apply_dclass(A);
    extern __shared__ __align__(16) unsigned char smem[];
    ExecCount ec;
    for_each_item(A, [&](int64_t blk) { pair_item<T, QL>(A, blk, smem, ec); });
    ec.flush(A);
}

template <typename T, int QL = 0>
hipError_t launch_pair(int l, int64_t ub, int cus, size_t lds_cu, size_t shm, hipStream_t st, const LevelArgs &A)
{
    if constexpr (QL + 2 <= kMaxTemplL) {
        if (l == QL + 2) {
            const void *fn = (const void *)pair_kernel<T, QL>;
            if (shm > 65536) {
                // dynamic LDS beyond 64 KiB is opted into per kernel
                const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
                if (e != hipSuccess) return e;
            }
            pair_kernel<T, QL><<<resident_grid(fn, 256, shm, ub, cus, lds_cu), 256, shm, st>>>(A);
            return hipGetLastError();
        }
        return launch_pair<T, QL + 1>(l, ub, cus, lds_cu, shm, st, A);
    }
    return hipErrorInvalidValue;
}

template <typename T, int QL = 0>
const void *pair_fn(int l)
{
    if constexpr (QL + 2 <= kMaxTemplL) {
        if (l == QL + 2) return (const void *)pair_kernel<T, QL>;
        return pair_fn<T, QL + 1>(l);
    }
    return nullptr;
}

template <typename T>
size_t pair_lds_bytes(int l, int m)
{
    // tile (rounded to 16 bytes) + 4 wave tables of m positions
    const int QL = l - 2;
    const int V = 16 / (int)sizeof(T);
    const int SA = (QL + 5 + V - 1) / V * V, SB = (QL + 3 + V - 1) / V * V;
    const size_t tile = ((size_t)m * (m - 1) / 2 + 2 * (size_t)m + V - 1) / V * V;
    return sizeof(T) * (tile + (size_t)kWaves * m * (SA + SB));
}


// ------------------------------------------------------------------ triple kernel (l >= 3)
// As the pair kernel, with the shared prefix one shorter: Q holds the
// first l-3 elements, the next element a is uniform across the wave (its
// row of the Schur table is a broadcast read and its pivot is computed
// once), and the lanes run the pairs (b < c) after a.  Eliminating a from
// the Schur complement of Q is a rank-1 update applied on the fly:
//     l_x = S_ax / sqrt(S_aa),  S'_xy = S_xy - l_x l_y,  S'_xi = S_xi - l_x u_a
// and the pair (b, c) is then eliminated from S' as in the pair kernel.
// The table is built once per Q (C(n,3) tests) instead of once per
// (l-2)-prefix (C(n,2) tests).
// Entry stride (elements) of the per-wave Schur table.  Lanes read the
// entries of consecutive positions; a stride of an odd number of 8-byte
// words (FP32: read as 8-byte pairs) or of 16-byte words (FP64: read as
// double pairs) spreads such reads over all LDS banks.  Four FP32 values fit
// one 16-byte read, which is conflict free as it is.
__host__ __device__ constexpr int triple_stride(int nE, int elem_bytes)
{
    return elem_bytes == 4 && nE <= 4 ? 4 : ((nE + 1) / 2 | 1) * 2;
}

template <typename T, int QL>
struct TripleLayout {
    static constexpr int V = 16 / (int)sizeof(T);
    static constexpr int nE = QL + 4;  // w[QL], S_xx, S_xi, S_xj, row offset of x in the packed tile
    static constexpr int S = triple_stride(nE, (int)sizeof(T));
};

template <typename T, int QL>
__device__ __forceinline__ void triple_item(const LevelArgs &A, int64_t blk, unsigned char *smem,
                                            const uint8_t *__restrict__ pdec, ExecCount &ec)
{
    using Lay = TripleLayout<T, QL>;
    constexpr int L = QL + 3;
    constexpr int QLL = QL > 0 ? QL : 1;
    const int64_t e = find_edge(A.blockoff, A.n_edges, blk);
    const EdgeRec E = A.edges[e];
    const int m = uniform_i32(E.m);
    const int64_t rpb = A.ranks_per_block, rpw = rpb / kWaves;
    const int64_t r0 = A.win_lo + (blk - A.blockoff[e]) * rpb;
    const int64_t r1 = min(r0 + rpb, min(A.win_hi, E.ntests));
    if (r0 >= r1) return;  // uniform
    __shared__ int skip;
    if (threadIdx.x == 0) skip = load_minhit(&A.minhit[e]) < (uint64_t)r0;
    __syncthreads();
    if (skip) return;  // uniform
    const InstRec &I = A.inst[E.inst];
    const T *C = static_cast<const T *>(I.C);
    const int p = (int)I.ld;
    const Thresholds th = I.th;
    const int32_t *cand = A.cand + E.cand_off;
    T *tri = reinterpret_cast<T *>(smem);
    const int ntri = m * (m - 1) / 2;
    T *ci = tri + ntri, *cj = ci + m;
    stage_tile<T>(C, p, cand, m, E.i, E.j, tri, ci, cj);
    const T cij = C[(size_t)E.i * p + E.j];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const size_t tile_elems = ((size_t)ntri + 2 * (size_t)m + Lay::V - 1) / Lay::V * Lay::V;
    T *tab = tri + tile_elems + (size_t)wave * A.max_m * Lay::S;
    __syncthreads();

    const int64_t wlo = r0 + (int64_t)wave * rpw;
    const int64_t whi = min(wlo + rpw, r1);
    if (wlo >= whi) return;  // no later block-wide barrier
    const auto row = [&](int a) { return a * (2 * m - a - 3) / 2 - 1; };
    // tile entry at a row offset and a column offset, both in bytes
    const auto tri_at = [&](int row_bytes, int col_bytes) {
        return *reinterpret_cast<const T *>(reinterpret_cast<const unsigned char *>(tri) + row_bytes + col_bytes);
    };

    // the walk's position (Q, a, tau, rank) is the same in every lane
    int c[L];
    unrank_wave<L>(wlo, m, A.binomT, c);
    int Q[QLL];
#pragma unroll
    for (int t = 0; t < QL; ++t) Q[t] = uniform_i32(c[t]);
    int sQ = QL > 0 ? Q[QL - 1] + 1 : 0;
    int a = uniform_i32(c[QL]);
    int tau;
    {
        const int na = m - 1 - a, b0 = uniform_i32(c[QL + 1]) - (a + 1), c0 = uniform_i32(c[QL + 2]) - (a + 1);
        tau = b0 * (2 * na - b0 - 1) / 2 + (c0 - b0 - 1);
    }
    int64_t rank = uniform_i64(wlo);
    int64_t remaining = uniform_i64(whi - wlo);
    uint64_t executed = 0;
    const float errk = (float)(kErrSafety * th.c_eff * (L + 2));
    const float rlo32 = (float)th.rb_lo, rhi32 = (float)th.rb_hi, tau32 = (float)th.tau;
    bool stop = false;
    // The shared minimum is read one check ahead: each check compares with
    // the value read at the previous one and issues the next read, so the
    // wave never waits for the load (another wave's hit stops this one at
    // most one interval later; tests run past it are discarded).
    int since_check = 0;  // tests since the last check
    uint64_t mh_ahead = load_minhit(&A.minhit[e]);
    while (!stop) {
        // ---- Q state (identical in every lane)
        T LQ[QL > 0 ? QL * (QL + 1) / 2 : 1], invQ[QLL], uQ[QLL], vQ[QLL];
        int rwQ[QLL];
        T H11 = T(1), H22 = T(1), H12 = cij, dminQ = T(1);
        bool okQ = true;
#pragma unroll
        for (int t = 0; t < QL; ++t) rwQ[t] = row(Q[t]);
#pragma unroll
        for (int t = 0; t < QL; ++t) {
            T *Lt = LQ + t * (t + 1) / 2;
#pragma unroll
            for (int s2 = 0; s2 < t; ++s2) {
                T v = tri[rwQ[s2] + Q[t]];
                const T *Ls = LQ + s2 * (s2 + 1) / 2;
#pragma unroll
                for (int q = 0; q < s2; ++q) v -= Lt[q] * Ls[q];
                Lt[s2] = v * invQ[s2];
            }
            T d = T(1);
#pragma unroll
            for (int q = 0; q < t; ++q) d -= Lt[q] * Lt[q];
            okQ = okQ && d > T(0);
            dminQ = d < dminQ ? d : dminQ;
            invQ[t] = rsqv(d);
            T ai = ci[Q[t]], aj = cj[Q[t]];
#pragma unroll
            for (int q = 0; q < t; ++q) {
                ai -= Lt[q] * uQ[q];
                aj -= Lt[q] * vQ[q];
            }
            uQ[t] = ai * invQ[t];
            vQ[t] = aj * invQ[t];
            H11 -= uQ[t] * uQ[t];
            H22 -= vQ[t] * vQ[t];
            H12 -= uQ[t] * vQ[t];
        }
        // ---- Schur table of Q over the positions [sQ, m)
        const int n = m - sQ;
        wave_sync();
        for (int xp = lane; xp < n; xp += 64) {
            const int x = sQ + xp;
            T w[QLL];
#pragma unroll
            for (int t = 0; t < QL; ++t) {
                T v = tri[rwQ[t] + x];
#pragma unroll
                for (int q = 0; q < t; ++q) v -= LQ[t * (t + 1) / 2 + q] * w[q];
                w[t] = v * invQ[t];
            }
            T sxx = T(1), sxi = ci[x], sxj = cj[x];
#pragma unroll
            for (int t = 0; t < QL; ++t) {
                sxx -= w[t] * w[t];
                sxi -= w[t] * uQ[t];
                sxj -= w[t] * vQ[t];
            }
            // entries at their absolute positions (x < m), so the pair loop
            // addresses them without subtracting sQ; the row offset of x in
            // the packed tile is stored in bytes
            T *ex = tab + __umul24((unsigned)x, (unsigned)Lay::S);
#pragma unroll
            for (int t = 0; t < QL; ++t) ex[t] = w[t];
            ex[QL] = sxx;
            ex[QL + 1] = sxi;
            ex[QL + 2] = sxj;
            put_int(ex[QL + 3], row(x) * (int)sizeof(T));
        }
        wave_sync();
        // ---- a loop (uniform), pairs (b, c) after a across the lanes
        for (; a <= m - 3; ++a) {
            // another wave's hit below this rank ends the range; the shared
            // minimum is read once per kMinhitEvery tests run
            if (since_check >= kMinhitEvery) {
                since_check = 0;
                const unsigned long long mh = (unsigned long long)uniform_i64((int64_t)mh_ahead);
                mh_ahead = load_minhit(&A.minhit[e]);
                if (mh < (unsigned long long)rank) {
                    stop = true;
                    break;
                }
            }
            const T *eaP = tab + __umul24((unsigned)a, (unsigned)Lay::S);
            T wa[QLL];
#pragma unroll
            for (int t = 0; t < QL; ++t) wa[t] = eaP[t];
            const T saa = eaP[QL], sai = eaP[QL + 1], saj = eaP[QL + 2];
            const int rowa = get_int(eaP[QL + 3]);  // bytes
            const T i1 = saa > T(0) ? rsqv(saa) : T(0);
            const T ua = sai * i1, va = saj * i1;
            const T H11a = H11 - ua * ua, H22a = H22 - va * va, H12a = H12 - ua * va;
            const bool oka = okQ && saa > T(0);
            const T dmina = saa < dminQ ? saa : dminQ;
            const int na = m - 1 - a;
            const int P = na * (na - 1) / 2;
            const int cnt = (int)min((int64_t)(P - tau), remaining);
            bool hit_found = false;
            int done_tests = cnt;  // tests of this a run by the wave
            const int u0 = P - 1 - tau;  // reversed index of the first pair
            const int lane_u = u0 - lane;
            // pairs from the table when it covers u0 (and so every u below),
            // from tri_root otherwise
            auto pairs = [&](auto tabled, auto diag) {
            for (int it = 0; it < cnt; it += 64) {
                const bool valid = lane < cnt - it;
                const unsigned u = (unsigned)max(lane_u - it, u0 - (cnt - 1));  // u0 - min(it + lane, cnt - 1)
                unsigned rr;
                if constexpr (decltype(tabled)::value) rr = pdec[u];
                else rr = tri_root(u);
                const int b = m - 2 - (int)rr;
                const int cc = m - 1 - (int)(u - (__umul24(rr, rr + 1u) >> 1));
                // LDS offsets fit 24 bits
                const T *eb = tab + __umul24((unsigned)b, (unsigned)Lay::S);
                const T *ec = tab + __umul24((unsigned)cc, (unsigned)Lay::S);
                const int cb = cc * (int)sizeof(T);
                T sab = tri_at(rowa, b * (int)sizeof(T)), sac = tri_at(rowa, cb),
                  sbc = tri_at(get_int(eb[QL + 3]), cb);
#pragma unroll
                for (int q = 0; q < QL; ++q) {
                    sab -= wa[q] * eb[q];
                    sac -= wa[q] * ec[q];
                    sbc -= eb[q] * ec[q];
                }
                const T lb = sab * i1, lc = sac * i1;
                const T sbb = eb[QL] - lb * lb, scc = ec[QL] - lc * lc, sbc2 = sbc - lb * lc;
                const T sbi = eb[QL + 1] - lb * ua, sbj = eb[QL + 2] - lb * va;
                const T sci = ec[QL + 1] - lc * ua, scj = ec[QL + 2] - lc * va;
                const T i2 = rsqv(sbb);
                const T l2 = sbc2 * i2;
                const T d3 = scc - l2 * l2;
                const T i3 = rsqv(d3);
                const T ub = sbi * i2, vb = sbj * i2;
                const T uc = (sci - l2 * ub) * i3, vc = (scj - l2 * vb) * i3;
                const T h11 = H11a - ub * ub - uc * uc;
                const T h22 = H22a - vb * vb - vc * vc;
                const T h12 = H12a - ub * vb - uc * vc;
                const T r = h12 * rsqv(h11 * h22);
                bool ok, indep, dep;
                if constexpr (sizeof(T) == 8) {
                    ok = oka && sbb > T(0) && d3 > T(0) && h11 > T(0) && h22 > T(0) && fabs(r) < T(1);
                    indep = decide64((double)r, ok, th);
                    dep = !indep;
                } else {
                    // smallest pivots through the bit patterns: > 0 as an integer
                    // exactly when every pivot is a positive float (a negative
                    // one or a zero becomes the minimum).  A NaN needs a zero or
                    // denormal pivot upstream, which is then the minimum and
                    // makes rho tiny: the test goes to the FP64 re-run.
                    const float dK = pos_min(dmina, pos_min(sbb, d3)), hmin = pos_min(h11, h22);
                    ok = oka && __float_as_int(pos_min(dK, hmin)) > 0 && fabsf(r) < 1.0f;
                    decide32b(r, dK * hmin, ok, rlo32, rhi32, errk, tau32, indep, dep);
                }
                if constexpr (decltype(diag)::value) {
                    if (valid) {
                        A.diag_r[rank + it + lane - A.diag_lo] = ok ? (double)r : (double)NAN;
                        A.diag_dec[rank + it + lane - A.diag_lo] =
                            (uint8_t)(indep ? DEC_INDEP : dep ? DEC_DEP : DEC_RECHECK);
                    }
                } else {
                    const bool hit = valid && indep;
                    const bool rq = sizeof(T) == 4 && valid && !indep && !dep;
                    // the common round has neither an FP64 re-run nor a hit
                    if (wave_mask(rq || hit)) {
                        if constexpr (sizeof(T) == 4) {
                            const unsigned long long qb = wave_mask(rq);
                            if (qb) {
                                unsigned long long slot = 0;
                                if (lane == 0) slot = atomicAdd(&A.counters[1], (unsigned long long)__popcll(qb));
                                slot = __shfl(slot, 0);
                                if (rq) {
                                    const unsigned long long idx = slot + __popcll(qb & ((1ull << lane) - 1ull));
                                    if ((int64_t)idx < A.queue_cap) {
                                        A.queue[2 * idx] = e + A.edge_base;
                                        A.queue[2 * idx + 1] = rank + it + lane;
                                    }
                                }
                            }
                        }
                        const unsigned long long hb = wave_mask(hit);
                        if (hb) {
                            if (lane == 0)
                                atomicMin((unsigned long long *)&A.minhit[e],
                                          (unsigned long long)(rank + it + __ffsll((long long)hb) - 1));
                            hit_found = true;
                            done_tests = min(cnt, it + 64);
                            break;
                        }
                    }
                }
            }
            };
            // the diagnostic form (r and the decision of every test written
            // out) is a separate loop, so the search loop carries no branch
            // for it
            if (A.diag_r) {
                if (u0 < A.pdec_n) pairs(std::true_type{}, std::true_type{});
                else pairs(std::false_type{}, std::true_type{});
            } else {
                if (u0 < A.pdec_n) pairs(std::true_type{}, std::false_type{});
                else pairs(std::false_type{}, std::false_type{});
            }
            executed += (uint64_t)done_tests;
            since_check += done_tests;
            if (hit_found) {
                stop = true;
                break;
            }
            rank += cnt;
            remaining -= cnt;
            tau = 0;
            if (remaining <= 0) {
                stop = true;
                break;
            }
        }
        if (stop) break;
        // ---- next Q: next (l-3)-combination of positions [0, m-3)
        if constexpr (QL == 0) {
            break;
        } else {
            int k = -1;
#pragma unroll
            for (int t = 0; t < QL; ++t)
                if (Q[t] != (m - 3) - QL + t) k = t;
            if (k < 0) break;
#pragma unroll
            for (int t = 0; t < QL; ++t) {
                if (t == k) Q[t] += 1;
                else if (t > k) Q[t] = Q[t - 1] + 1;
            }
            sQ = Q[QL - 1] + 1;
            a = sQ;
            tau = 0;
        }
    }
    ec.add(A, E.inst, (unsigned long long)executed);
}

// Pairs (b < c) of the positions after a, in reversed order: the pair of
// reversed index u lies in row rr = tri_root(u) of the triangle, column
// s = u - rr(rr+1)/2, which puts it at b = m-2-rr, c = m-1-s whatever a is.
// The table holds the row rr (one byte) for each u below pdec_n; the
// column follows from it.  pdec_n <= C(256, 2) keeps rr below 255.  The
// host sizes it to the LDS a workgroup can take without fewer workgroups
// fitting on a CU (a byte per entry covers twice the pairs of a 16-bit
// entry holding both indices).
constexpr int kPdecCap = 256 * 255 / 2;
__host__ __device__ constexpr size_t pdec_bytes(int n) { return ((size_t)n + 15) / 16 * 16; }

template <typename T, int QL>
__global__ __launch_bounds__(256, (sizeof(T) == 4 && QL <= 2) ? 7 : 1) void triple_kernel(LevelArgs A)
{
    apply_dclass(A);
    extern __shared__ __align__(16) unsigned char smem[];
    // the pair table is built once per launch and read by every item; the
    // barrier at the start of each item orders these writes before the reads
    uint8_t *pdec = reinterpret_cast<uint8_t *>(smem);
    const unsigned np = (unsigned)A.pdec_n;
    for (unsigned u = threadIdx.x; u < np; u += blockDim.x) pdec[u] = (uint8_t)tri_root(u);
    unsigned char *rest = smem + pdec_bytes(A.pdec_n);
    ExecCount ec;
    for_each_item(A, [&](int64_t blk) { triple_item<T, QL>(A, blk, rest, pdec, ec); });
    ec.flush(A);
}

template <typename T, int QL = 0>
hipError_t launch_triple(int l, int64_t ub, int cus, size_t lds_cu, size_t shm, hipStream_t st, const LevelArgs &A)
{
    if constexpr (QL + 3 <= kMaxTemplL) {
        if (l == QL + 3) {
            const void *fn = (const void *)triple_kernel<T, QL>;
            if (shm > 65536) {
                const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
                if (e != hipSuccess) return e;
            }
            triple_kernel<T, QL><<<resident_grid(fn, 256, shm, ub, cus, lds_cu), 256, shm, st>>>(A);
            return hipGetLastError();
        }
        return launch_triple<T, QL + 1>(l, ub, cus, lds_cu, shm, st, A);
    }
    return hipErrorInvalidValue;
}

// LDS of the triple kernel without its pair table
template <typename T>
size_t triple_lds_bytes(int l, int m)
{
    const int QL = l - 3;
    const int V = 16 / (int)sizeof(T);
    const int S = triple_stride(QL + 4, (int)sizeof(T));
    const size_t tile = ((size_t)m * (m - 1) / 2 + 2 * (size_t)m + V - 1) / V * V;
    return sizeof(T) * (tile + (size_t)kWaves * m * S);
}

template <typename T, int QL = 0>
const void *triple_fn(int l)
{
    if constexpr (QL + 3 <= kMaxTemplL) {
        if (l == QL + 3) return (const void *)triple_kernel<T, QL>;
        return triple_fn<T, QL + 1>(l);
    }
    return nullptr;
}

// Entries of the pair table for a class whose other LDS is `base` bytes:
// as many as cover its largest list, within what leaves the workgroups per
// CU (by registers, LDS and the tuning cap) unchanged.
int triple_table_entries(int l, bool fp32, int max_m, size_t base, size_t lds_cu, size_t lds_cap, int cap_blocks)
{
    const size_t full = max_m > 2 ? std::min<size_t>((size_t)(max_m - 1) * (max_m - 2) / 2, kPdecCap) : 0;
    const void *fn = fp32 ? triple_fn<float>(l) : triple_fn<double>(l);
    int regs = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&regs, fn, 256, 0) != hipSuccess || regs < 1) regs = 1;
    int k0 = std::min<int>(regs, (int)(lds_cu / (base + 256)));
    if (cap_blocks > 0) k0 = std::min(k0, cap_blocks);
    k0 = std::max(k0, 1);
    const size_t room = std::min<size_t>(lds_cu / (size_t)k0 - 256, lds_cap);
    if (room <= base) return 0;
    return (int)std::min<size_t>(full, (room - base) / 16 * 16);
}

// Workgroups of the triple kernel resident on one CU (registers, LDS of
// `shm` bytes each and the tuning cap).
int triple_blocks_per_cu(int l, bool fp32, size_t shm, size_t lds_cu, int cap_blocks)
{
    const void *fn = fp32 ? triple_fn<float>(l) : triple_fn<double>(l);
    int k = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, fn, 256, 0) != hipSuccess || k < 1) k = 1;
    k = std::min<int>(k, (int)(lds_cu / (shm + 256)));
    if (cap_blocks > 0) k = std::min(k, cap_blocks);
    return std::max(k, 1);
}

// ------------------------------------------------------------------ wide levels
// One wave per test, the (l+2)x(l+2) matrix over [K, i, j] packed lower in
// LDS, right-looking Cholesky; after l steps the trailing 2x2 block is H.
template <typename T>
__device__ bool wave_pcor(T *M, int l, int lane, T &r)
{
    auto at = [&](int a, int b) -> T & { return M[a * (a + 1) / 2 + b]; };  // a >= b
    const int n2 = l + 2;
    for (int t = 0; t < l; ++t) {
        const T d = at(t, t);
        if (!(d > T(0))) return false;  // uniform: every lane reads the same value
        const T s = rsq(d);
        for (int a = t + 1 + lane; a < n2; a += 64) at(a, t) *= s;
        __syncthreads();
        const int rem = n2 - t - 1;
        for (int idx = lane; idx < rem * (rem + 1) / 2; idx += 64) {
            // idx -> (a, b) with t < b <= a
            int a = (int)((sqrtf(8.0f * idx + 1.0f) - 1.0f) * 0.5f);
            while ((a + 1) * (a + 2) / 2 <= idx) ++a;
            while (a * (a + 1) / 2 > idx) --a;
            const int b = idx - a * (a + 1) / 2;
            const int aa = t + 1 + a, bb = t + 1 + b;
            at(aa, bb) -= at(aa, t) * at(bb, t);
        }
        __syncthreads();
    }
    const T h11 = at(l, l), h22 = at(l + 1, l + 1), h12 = at(l + 1, l);
    if (!(h11 > T(0)) || !(h22 > T(0))) return false;
    r = h12 * rsq(h11 * h22);
    return fabs(r) < T(1);
}

template <typename T>
__device__ __forceinline__ void wide_item(const LevelArgs &A, int l, int64_t blk, unsigned char *smem, ExecCount &ec)
{
    T *M = reinterpret_cast<T *>(smem);
    int *k = reinterpret_cast<int *>(M + (size_t)(l + 2) * (l + 3) / 2 + 1);
    const int64_t e = find_edge(A.blockoff, A.n_edges, blk);
    const EdgeRec E = A.edges[e];
    const int m = E.m;
    const int64_t r0 = A.win_lo + (blk - A.blockoff[e]) * A.ranks_per_block;
    const int64_t r1 = min(r0 + (int64_t)A.ranks_per_block, min(A.win_hi, E.ntests));
    if (r0 >= r1) return;  // uniform
    const InstRec &I = A.inst[E.inst];
    const double *C = I.C64;  // wide levels run in FP64
    const int p = (int)I.ld;
    const Thresholds th = I.th;
    const int32_t *cand = A.cand + E.cand_off;
    const int lane = threadIdx.x;
    // unrank r0 into k (lane 0), shared through LDS
    if (lane == 0) {
        int64_t R = r0;
        int x = 0;
        for (int t = 0; t < l; ++t) {
            for (;;) {
                const int a = m - 1 - x;
                if (a < l - 1 - t) break;
                const int64_t cnt = binom_at(A.binom, a, l - 1 - t);
                if (R < cnt) break;
                R -= cnt;
                ++x;
            }
            k[t] = x++;
        }
    }
    __syncthreads();
    uint64_t executed = 0;
    for (int64_t R = r0; R < r1; ++R) {
        const unsigned long long mh = (unsigned long long)uniform_i64((int64_t)load_minhit(&A.minhit[e]));
        if (mh < (unsigned long long)R) break;  // wave-uniform
        __syncthreads();
        // gather [cand[k_0..k_{l-1}], i, j]
        const int n2 = l + 2;
        for (int idx = lane; idx < n2 * (n2 + 1) / 2; idx += 64) {
            int a = (int)((sqrtf(8.0f * idx + 1.0f) - 1.0f) * 0.5f);
            while ((a + 1) * (a + 2) / 2 <= idx) ++a;
            while (a * (a + 1) / 2 > idx) --a;
            const int b = idx - a * (a + 1) / 2;
            const int va = a < l ? cand[k[a]] : (a == l ? E.i : E.j);
            const int vb = b < l ? cand[k[b]] : (b == l ? E.i : E.j);
            M[idx] = (T)C[(size_t)va * p + vb];
        }
        __syncthreads();
        T r;
        const bool ok = wave_pcor<T>(M, l, lane, r);
        ++executed;
        bool indep = false;
        if (ok) {
            const double a = fabs((double)r);
            indep = a < th.r_lo ? true
                  : a > th.r_hi ? false
                  : th.sqrt_nu * fabs(atanh((double)r)) <= th.q;
        }
        if (A.diag_r) {
            if (lane == 0) {
                A.diag_r[R - A.diag_lo] = ok ? (double)r : (double)NAN;
                A.diag_dec[R - A.diag_lo] = indep ? DEC_INDEP : DEC_DEP;
            }
            indep = false;
        }
        if (indep) {
            if (lane == 0) atomicMin((unsigned long long *)&A.minhit[e], (unsigned long long)R);
            break;
        }
        __syncthreads();
        if (lane == 0) {  // next combination
            int a = l - 1;
            while (a >= 0 && k[a] == m - l + a) --a;
            if (a >= 0) {
                ++k[a];
                for (int b = a + 1; b < l; ++b) k[b] = k[b - 1] + 1;
            }
        }
        __syncthreads();
    }
    ec.add(A, E.inst, (unsigned long long)executed);
}

template <typename T>
__global__ __launch_bounds__(64) void level_kernel_wide(LevelArgs A, int l)
{
    apply_dclass(A);
    extern __shared__ __align__(16) unsigned char smem[];
    ExecCount ec;
    for_each_item(A, [&](int64_t blk) { wide_item<T>(A, l, blk, smem, ec); });
    ec.flush(A);
}

// ------------------------------------------------------------------ window plans
// Work items of window [lo, hi) of one edge: ceil(span / rpb) runs of
// ranks, none for an edge that already has a separating rank (filter).
// The plan is an exclusive prefix over the edges, built on the device from
// the current minhit, so windows follow each other with no host round trip.
struct PlanArgs {
    const EdgeRec *edges;
    const uint64_t *minhit;
    int64_t n_edges;
    int64_t lo, hi;
    int rpb;
    int filter;
    int64_t *sums;                  // per-workgroup totals, then their exclusive prefix
    int64_t *off;                   // n_edges + 1 exclusive prefix of items per edge
    int64_t *n_items;               // total items of the window
    unsigned long long *item_ctr;   // zeroed for the window's test kernel
    unsigned long long *queue_len;  // recheck queue of the previous window, emptied (null: kept)
    const int64_t *dclass;          // device class range (see LevelArgs::dclass), or null
};

constexpr int kPlanPer = 8;                 // edges per thread
constexpr int kPlanChunk = 256 * kPlanPer;  // edges per workgroup

__device__ __forceinline__ int64_t window_items(const EdgeRec &E, uint64_t mh, int64_t lo, int64_t hi, int rpb,
                                                int filter)
{
    if (filter && mh != ~0ull) return 0;
    const int64_t span = min(E.ntests, hi) - lo;
    return span > 0 ? (span + rpb - 1) / rpb : 0;
}

// Exclusive scan of one value per thread over a workgroup of NW waves;
// returns the workgroup total.
template <int NW = 4>
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t &excl)
{
    __shared__ int64_t wsum[NW];
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    int64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int64_t before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        if (k < w) before += wsum[k];
        total += wsum[k];
    }
    excl = before + x - v;
    __syncthreads();  // wsum is free again
    return total;
}

__global__ __launch_bounds__(256) void plan_reduce(PlanArgs P)
{
    const int64_t base = (int64_t)blockIdx.x * kPlanChunk;
    int64_t s = 0;
#pragma unroll
    for (int t = 0; t < kPlanPer; ++t) {
        const int64_t e = base + (int64_t)t * 256 + threadIdx.x;
        if (e < P.n_edges) s += window_items(P.edges[e], P.minhit[e], P.lo, P.hi, P.rpb, P.filter);
    }
    int64_t ex;
    const int64_t tot = block_exclusive_scan(s, ex);
    if (threadIdx.x == 0) P.sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void plan_sums(PlanArgs P, int nb)
{
    int64_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const int64_t v = b < nb ? P.sums[b] : 0;
        int64_t ex;
        const int64_t tot = block_exclusive_scan(v, ex);
        if (b < nb) P.sums[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        P.off[P.n_edges] = carry;
        *P.n_items = carry;
        *P.item_ctr = 0;
        if (P.queue_len) *P.queue_len = 0;
    }
}

__global__ __launch_bounds__(256) void plan_scan(PlanArgs P)
{
    const int64_t base = (int64_t)blockIdx.x * kPlanChunk + (int64_t)threadIdx.x * kPlanPer;
    int64_t v[kPlanPer];
    int64_t s = 0;
#pragma unroll
    for (int t = 0; t < kPlanPer; ++t) {
        const int64_t e = base + t;
        v[t] = e < P.n_edges ? window_items(P.edges[e], P.minhit[e], P.lo, P.hi, P.rpb, P.filter) : 0;
        s += v[t];
    }
    int64_t ex;
    block_exclusive_scan(s, ex);
    int64_t run = P.sums[blockIdx.x] + ex;
#pragma unroll
    for (int t = 0; t < kPlanPer; ++t) {
        const int64_t e = base + t;
        if (e < P.n_edges) P.off[e] = run;
        run += v[t];
    }
}

// The three plan passes in one 1024-thread workgroup, for classes of at
// most kPlanSingleEdges edges: chunks of 8192 edges are scanned one after
// the other with a running carry.
constexpr int kPlanSingleThreads = 1024;
constexpr int64_t kPlanSingleEdges = 65536;

__global__ __launch_bounds__(kPlanSingleThreads) void plan_single(PlanArgs P)
{
    if (P.dclass) {
        const int64_t b = P.dclass[0];
        P.edges += b;
        P.minhit += b;
        P.off += b;
        P.n_edges = P.dclass[1] - b;
    }
    constexpr int64_t chunk = (int64_t)kPlanSingleThreads * kPlanPer;
    int64_t carry = 0;
    for (int64_t base0 = 0; base0 < P.n_edges; base0 += chunk) {
        const int64_t base = base0 + (int64_t)threadIdx.x * kPlanPer;
        int64_t v[kPlanPer];
        int64_t s = 0;
#pragma unroll
        for (int t = 0; t < kPlanPer; ++t) {
            const int64_t e = base + t;
            v[t] = e < P.n_edges ? window_items(P.edges[e], P.minhit[e], P.lo, P.hi, P.rpb, P.filter) : 0;
            s += v[t];
        }
        int64_t ex;
        const int64_t tot = block_exclusive_scan<kPlanSingleThreads / 64>(s, ex);
        int64_t run = carry + ex;
#pragma unroll
        for (int t = 0; t < kPlanPer; ++t) {
            const int64_t e = base + t;
            if (e < P.n_edges) P.off[e] = run;
            run += v[t];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        P.off[P.n_edges] = carry;
        *P.n_items = carry;
        *P.item_ctr = 0;
        if (P.queue_len) *P.queue_len = 0;
    }
}

// ------------------------------------------------------------------ compaction
__global__ __launch_bounds__(256) void compact_kernel(const uint64_t *__restrict__ minhit, int64_t n,
                                                      int64_t *__restrict__ out, unsigned long long *__restrict__ cnt)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x % 64;
    const bool del = e < n && minhit[e] != ~0ull;
    const unsigned long long b = __ballot(del);
    if (!b) return;
    unsigned long long slot = 0;
    if (lane == 0) slot = atomicAdd(cnt, (unsigned long long)__popcll(b));
    slot = __shfl(slot, 0);
    if (del) {
        const unsigned long long idx = slot + __popcll(b & ((1ull << lane) - 1ull));
        out[2 * idx] = e;
        out[2 * idx + 1] = (int64_t)minhit[e];
    }
}

// ------------------------------------------------------------------ index-matrix batch
template <typename T, int L>
__global__ __launch_bounds__(256) void batch_kernel(const T *__restrict__ C, int p, const int32_t *__restrict__ B,
                                                    int64_t b, Thresholds th, double *__restrict__ z_out,
                                                    uint8_t *__restrict__ ind_out, int *__restrict__ bad)
{
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= b) return;
    const int32_t *Br = B + row * (2 + L);
    int k[L > 0 ? L : 1];
    bool inb = Br[0] >= 0 && Br[0] < p && Br[1] >= 0 && Br[1] < p;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        k[t] = Br[2 + t];
        inb = inb && k[t] >= 0 && k[t] < p;
    }
    if (!inb) {  // out-of-range index: flagged, nothing read
        if (z_out) z_out[row] = NAN;
        if (ind_out) ind_out[row] = 0;
        atomicOr(bad, 1);
        return;
    }
    DirectRows<T> V{C, p, Br[0], Br[1]};
    T r, rho;
    bool ok;
    pcor_reg<T, L>(V, k, r, rho, ok);
    double z = NAN;
    uint8_t ind = 0;
    if (ok) {
        if constexpr (sizeof(T) == 8) {
            z = th.sqrt_nu * fabs(atanh((double)r));
            ind = decide64((double)r, ok, th);
        } else {
            const float zf = (float)th.sqrt_nu * fabsf(atanhf((float)r));
            z = zf;
            ind = zf <= (float)th.q;
        }
    }
    if (z_out) z_out[row] = z;
    if (ind_out) ind_out[row] = ind;
}

template <typename T>
__global__ __launch_bounds__(64) void batch_kernel_wide(const T *__restrict__ C, int p, const int32_t *__restrict__ B,
                                                        int64_t b, int l, Thresholds th, double *__restrict__ z_out,
                                                        uint8_t *__restrict__ ind_out, int *__restrict__ bad)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T *M = reinterpret_cast<T *>(smem);
    const int64_t row = blockIdx.x;
    const int32_t *Br = B + row * (2 + l);
    const int n2 = l + 2;
    __shared__ int oob;
    if (threadIdx.x == 0) oob = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < n2; t += 64)
        if (Br[t] < 0 || Br[t] >= p) oob = 1;
    __syncthreads();
    if (oob) {  // uniform
        if (threadIdx.x == 0) {
            if (z_out) z_out[row] = NAN;
            if (ind_out) ind_out[row] = 0;
            atomicOr(bad, 1);
        }
        return;
    }
    for (int idx = threadIdx.x; idx < n2 * (n2 + 1) / 2; idx += 64) {
        int a = (int)((sqrtf(8.0f * idx + 1.0f) - 1.0f) * 0.5f);
        while ((a + 1) * (a + 2) / 2 <= idx) ++a;
        while (a * (a + 1) / 2 > idx) --a;
        const int bb = idx - a * (a + 1) / 2;
        const int va = a < l ? Br[2 + a] : (a == l ? Br[0] : Br[1]);
        const int vb = bb < l ? Br[2 + bb] : (bb == l ? Br[0] : Br[1]);
        M[idx] = C[(size_t)va * p + vb];
    }
    __syncthreads();
    T r;
    const bool ok = wave_pcor<T>(M, l, threadIdx.x, r);
    if (threadIdx.x == 0) {
        double z = NAN;
        uint8_t ind = 0;
        if (ok) {
            z = th.sqrt_nu * fabs(atanh((double)r));
            ind = z <= th.q;
        }
        if (z_out) z_out[row] = z;
        if (ind_out) ind_out[row] = ind;
    }
}

// ------------------------------------------------------------------ dispatch tables
template <typename T, bool TILE, int L = 0>
void launch_level(int l, int64_t ub, int cus, size_t lds_cu, size_t shm, hipStream_t st, const LevelArgs &A)
{
    if constexpr (L <= kMaxTemplL) {
        if (l == L) {
            const void *fn = (const void *)level_kernel<T, L, TILE>;
            level_kernel<T, L, TILE><<<resident_grid(fn, 256, shm, ub, cus, lds_cu), 256, shm, st>>>(A);
            return;
        }
        launch_level<T, TILE, L + 1>(l, ub, cus, lds_cu, shm, st, A);
    }
}

template <int L = 0>
void launch_recheck(int l, hipStream_t st, const LevelArgs &A)
{
    if constexpr (L <= kMaxTemplL) {
        if (l == L) {
            recheck_kernel<L><<<512, 256, recheck_lds_bytes(A.max_m, L), st>>>(A);
            return;
        }
        launch_recheck<L + 1>(l, st, A);
    }
}

template <typename T, int L = 0>
void launch_batch(int l, dim3 g, hipStream_t st, const T *C, int p, const int32_t *B, int64_t b,
                  const Thresholds &th, double *z, uint8_t *ind, int *bad)
{
    if constexpr (L <= kMaxTemplL) {
        if (l == L) {
            batch_kernel<T, L><<<g, 256, 0, st>>>(C, p, B, b, th, z, ind, bad);
            return;
        }
        launch_batch<T, L + 1>(l, g, st, C, p, B, b, th, z, ind, bad);
    }
}

Thresholds make_thresholds(double q, int n, int l, double band_z, double c_eff, double tau = 0.0)
{
    Thresholds th;
    th.tau = tau;
    th.q = q;
    th.sqrt_nu = std::sqrt((double)(n - l - 3));
    const double rt = std::tanh(q / th.sqrt_nu);
    th.r_lo = rt * (1.0 - 1e-9);
    th.r_hi = rt * (1.0 + 1e-9);
    if (!std::isfinite(q)) {  // q = +inf: every non-degenerate test is independent
        th.r_lo = 2.0;
        th.r_hi = 2.0;
    }
    th.band_z = band_z;
    th.c_eff = c_eff;
    th.rb_lo = std::tanh(std::max(0.0, q - band_z) / th.sqrt_nu);
    th.rb_hi = std::tanh((q + band_z) / th.sqrt_nu);
    if (!std::isfinite(q)) {
        th.rb_lo = 2.0;
        th.rb_hi = 2.0;
    }
    return th;
}

// Threshold of the ill-conditioning trigger: tau >= 0 as given; negative
// selects the default, the rho below which the FP32 error model of a test,
// sqrt(n-l-3) (l+2) (2^-24 + c_err) / rho in z units (FP32 arithmetic and
// the entry error of the FP32 matrix), exceeds kZModelCap.  Measured FP32 z
// errors stay below 0.04 of that model (level 5 of the p = 1000 benchmark
// graph on an FP32-rounded matrix, about 1e6 tests), so the FP32 z of every
// test left in FP32 is then within 1e-4.
constexpr double kZModelCap = 1e-4 / 0.04;
double resolve_tau(double tau, int n, int l, double c_err)
{
    if (tau >= 0.0) return tau;
    return std::sqrt((double)(n - l - 3)) * (l + 2) * (0x1p-24 + c_err) / kZModelCap;
}

size_t tile_bytes(int m, size_t elem) { return elem * ((size_t)m * (m - 1) / 2 + 2 * (size_t)m + 1) + 16; }

}  // namespace

// LDS of the shared-prefix kernel the tuning table picks for level l: the
// pair kernel (prefix l-2) or, from l = 3, the triple kernel (prefix l-3).
bool use_triple(const fpc_ctx *ctx, int l)
{
    return l >= 3 && ctx->tuning.shared_prefix_depth[std::min(l, FPC_TUNE_LEVELS - 1)] == 3;
}

size_t shared_lds_bytes(const fpc_ctx *ctx, int l, bool fp32, int m)
{
    if (l < 2) return 0;
    if (use_triple(ctx, l)) return fp32 ? triple_lds_bytes<float>(l, m) : triple_lds_bytes<double>(l, m);
    return fp32 ? pair_lds_bytes<float>(l, m) : pair_lds_bytes<double>(l, m);
}

int level_class_key(const fpc_ctx *ctx, int l, bool fp32, int m)
{
    if (l > kMaxTemplL) return 0;  // wide levels: one class
    const size_t cap = (size_t)ctx->lds_per_block - kStaticLds;
    const size_t ps = shared_lds_bytes(ctx, l, fp32, m);
    int kind;
    size_t shm;
    if (l >= 2 && ctx->use_pair_kernel && ps <= cap) {
        kind = 0;
        shm = ps;
    } else {
        const size_t ts = tile_bytes(m, fp32 ? 4 : 8);
        kind = ts <= std::min<size_t>(cap, 65536) ? 1 : 2;
        shm = kind == 1 ? ts : 0;
    }
    const int per_cu = shm ? std::max(1, std::min(8, (int)((size_t)ctx->lds_per_cu / (shm + 256)))) : 8;
    return kind * 16 + (8 - per_cu);
}

std::vector<int> device_class_bounds(const fpc_ctx *ctx, int l, bool fp32)
{
    const int lt = std::min(l, FPC_TUNE_LEVELS - 1);
    const int tcap = ctx->tuning.max_blocks_per_cu[lt] > 0 ? ctx->tuning.max_blocks_per_cu[lt] : 1 << 20;
    const size_t cap = (size_t)ctx->lds_per_block - kStaticLds;
    const size_t lds_cu = (size_t)ctx->lds_per_cu;
    const bool triple = use_triple(ctx, l);
    int regs = 1 << 20;
    if (l >= 2) {
        const void *fn = triple ? (fp32 ? triple_fn<float>(l) : triple_fn<double>(l))
                                : (fp32 ? pair_fn<float>(l) : pair_fn<double>(l));
        int k = 0;
        if (fn && hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, fn, 256, 0) == hipSuccess && k >= 1) regs = k;
    }
    auto key = [&](int m) {
        const size_t ps = shared_lds_bytes(ctx, l, fp32, m);
        if (l >= 2 && ps <= cap)
            return std::min({regs, tcap, std::max(1, (int)(lds_cu / (ps + 256)))});
        const size_t ts = tile_bytes(m, fp32 ? 4 : 8);
        if (ts <= std::min<size_t>(cap, 65536)) return 100 + std::min({8, tcap, std::max(1, (int)(lds_cu / (ts + 256)))});
        return 200;
    };
    std::vector<int> b;
    int prev = key(std::max(l, 1));
    for (int m = std::max(l, 1) + 1; m < kBinomRows; ++m) {
        const int k = key(m);
        if (k != prev) b.push_back(m - 1);
        prev = k;
    }
    b.push_back(kBinomRows - 1);
    // at most kMaxDeviceClasses: the longest runs merge into the last class
    if ((int)b.size() > kMaxDeviceClasses) {
        b.resize(kMaxDeviceClasses);
        b.back() = kBinomRows - 1;
    }
    return b;
}

namespace {

// InstRec of every instance for level l, on the device: the thresholds of
// make_thresholds with the FP32 matrix's entry error read from device
// memory (it is measured by the same captured work).
__global__ void inst_table_kernel(const DevInstSrc *__restrict__ src, int ni, int l, double band_z, double tau_param,
                                  int fp32, InstRec *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ni) return;
    const DevInstSrc S = src[k];
    const double c_err = S.c_err ? *S.c_err : 0.0;
    InstRec R;
    R.C = fp32 ? (const void *)S.C32 : (const void *)S.C64;
    R.C64 = S.C64;
    R.ld = S.p;
    Thresholds &th = R.th;
    const double q = S.q;
    th.q = q;
    th.sqrt_nu = sqrt((double)(S.n - l - 3));
    const bool inf = isinf(q);
    const double rt = tanh(q / th.sqrt_nu);
    th.r_lo = inf ? 2.0 : rt * (1.0 - 1e-9);
    th.r_hi = inf ? 2.0 : rt * (1.0 + 1e-9);
    th.band_z = band_z;
    th.c_eff = c_err + 4.0 * (l + 2) * 6.0e-8;
    th.rb_lo = inf ? 2.0 : tanh(fmax(0.0, q - band_z) / th.sqrt_nu);
    th.rb_hi = inf ? 2.0 : tanh((q + band_z) / th.sqrt_nu);
    th.tau = tau_param >= 0.0 ? tau_param : th.sqrt_nu * (l + 2) * (0x1p-24 + c_err) / kZModelCap;
    out[k] = R;
}

}  // namespace

size_t inst_rec_bytes() { return sizeof(InstRec); }

int level_inst_table_enqueue(fpc_ctx *ctx, const DevInstSrc *src, int ni, int l, double band_z, double tau, bool fp32,
                             void *out)
{
    if (ni < 1) return FPC_OK;
    inst_table_kernel<<<(ni + 63) / 64, 64, 0, ctx->stream>>>(src, ni, l, band_z, tau, fp32 ? 1 : 0,
                                                             static_cast<InstRec *>(out));
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

// The launches of one device-built level: for each size class (static
// bound of its lists, edge range on the device) its rank windows, each a
// plan and a persistent test launch, and the FP64 re-run of the window's
// queue.  Nothing is read back: launches past a class's work find no items.
int level_tests_device(fpc_ctx *ctx, const DeviceLevel &D)
{
    hipStream_t st = ctx->stream;
    const int l = D.l;
    if (l > kMaxTemplL) return FPC_EINVAL;
    const bool fp32 = D.fp32;
    const int lt = std::min(l, FPC_TUNE_LEVELS - 1);
    const size_t lds_cap = (size_t)ctx->lds_per_block - kStaticLds;
    const int cus = ctx->num_cus;
    const size_t lds_cu = (size_t)ctx->lds_per_cu;
    const fpc_tuning &tu = ctx->tuning;
    g_max_blocks_per_cu = tu.max_blocks_per_cu[lt];
    enum Kind { K_TRIPLE, K_PAIR, K_TILE, K_GLOBAL };
    struct Cls {
        Kind kind;
        size_t shm;
        int pdec_n, rpb, max_m;
        std::vector<int64_t> wins;
        const int64_t *range;
    };
    std::vector<Cls> cls;
    int max_nw = 0;
    for (int c = 0; c < D.n_classes; ++c) {
        Cls k{};
        k.max_m = D.classes[c].max_m;
        k.range = D.classes[c].range;
        const bool triple = use_triple(ctx, l);
        const size_t ps = l < 2 ? 0
                        : triple ? (fp32 ? triple_lds_bytes<float>(l, k.max_m) : triple_lds_bytes<double>(l, k.max_m))
                                 : (fp32 ? pair_lds_bytes<float>(l, k.max_m) : pair_lds_bytes<double>(l, k.max_m));
        if (l >= 2 && ps <= lds_cap) {
            k.kind = triple ? K_TRIPLE : K_PAIR;
            k.shm = ps;
            if (triple) {
                k.pdec_n = triple_table_entries(l, fp32, k.max_m, ps, lds_cu, lds_cap, tu.max_blocks_per_cu[lt]);
                k.shm += pdec_bytes(k.pdec_n);
            }
            k.rpb = kWaves * tu.shared_ranks_per_wave[lt];
        } else {
            const size_t ts = tile_bytes(k.max_m, fp32 ? 4 : 8);
            k.kind = ts <= std::min<size_t>(lds_cap, 65536) ? K_TILE : K_GLOBAL;
            k.shm = k.kind == K_TILE ? ts : 0;
            k.rpb = kWaves * tu.test_ranks_per_wave[lt];
        }
        // windows covering the most tests a list of the class can hold
        const int64_t maxN = binom_sat(k.max_m, l);
        if (maxN == INT64_MAX) return FPC_EBUDGET;
        k.wins.push_back(0);
        for (int64_t w = (int64_t)k.rpb * std::max(1, tu.first_window_items[lt]); k.wins.back() < maxN;
             w = w > INT64_MAX / 64 ? w : w * std::max(2, tu.window_growth[lt]))
            k.wins.push_back(k.wins.back() > maxN - w ? maxN : k.wins.back() + w);
        max_nw = std::max(max_nw, (int)k.wins.size() - 1);
        cls.push_back(std::move(k));
    }
    if (D.n_classes > kMaxDeviceClasses) return FPC_EINVAL;
    // plan buffer: per class [items, item counter], then the classes' item
    // offsets, class c at [begin_c + c, end_c + c] (disjoint for any ranges)
    int64_t *slots = D.plan;
    int64_t *offs = D.plan + 2 * D.n_classes;
    LevelArgs A{};
    A.cand = D.cand;
    A.inst = static_cast<const InstRec *>(D.insts);
    A.binom = ctx->binom.as<int64_t>();
    A.binomT = ctx->binomT.as<int64_t>();
    A.counters = D.counters;
    A.inst_cnt = D.inst_cnt;
    A.queue = D.queue;
    A.queue_cap = D.queue_cap;
    A.edges = D.edges;
    A.minhit = D.minhit;
    hipError_t err = hipSuccess;
    for (int w = 0; w < max_nw && err == hipSuccess; ++w) {
        // the classes of the window one after the other, each its plan and
        // its persistent launch (as concurrent graph branches they ran
        // slower: several classes with work then exceed the tuned
        // workgroups per CU)
        std::vector<int> act;
        for (int c = 0; c < (int)cls.size(); ++c)
            if (w + 1 < (int)cls[c].wins.size()) act.push_back(c);
        if (act.empty()) continue;
        for (size_t j = 0; j < act.size() && err == hipSuccess; ++j) {
            const Cls &k = cls[act[j]];
            const int c = act[j];
            PlanArgs P{};
            P.edges = D.edges;
            P.minhit = D.minhit;
            P.dclass = k.range;
            P.lo = k.wins[w];
            P.hi = k.wins[w + 1];
            P.rpb = k.rpb;
            P.filter = w > 0;
            P.off = offs + c;
            P.n_items = slots + 2 * c;
            P.item_ctr = reinterpret_cast<unsigned long long *>(slots + 2 * c + 1);
            // the first plan of the window empties the re-run queue that the
            // previous window's re-run has drained
            P.queue_len = j == 0 ? &D.counters[1] : nullptr;
            plan_single<<<1, kPlanSingleThreads, 0, st>>>(P);
            LevelArgs B = A;
            B.dclass = k.range;
            B.blockoff = P.off;
            B.n_items = P.n_items;
            B.item_ctr = P.item_ctr;
            B.win_lo = P.lo;
            B.win_hi = P.hi;
            B.ranks_per_block = k.rpb;
            B.max_m = k.max_m;
            B.pdec_n = k.pdec_n;
            const int64_t ub = INT64_MAX;
            switch (k.kind) {
            case K_TRIPLE:
                err = fp32 ? launch_triple<float>(l, ub, cus, lds_cu, k.shm, st, B)
                           : launch_triple<double>(l, ub, cus, lds_cu, k.shm, st, B);
                break;
            case K_PAIR:
                err = fp32 ? launch_pair<float>(l, ub, cus, lds_cu, k.shm, st, B)
                           : launch_pair<double>(l, ub, cus, lds_cu, k.shm, st, B);
                break;
            case K_TILE:
                if (fp32) launch_level<float, true>(l, ub, cus, lds_cu, k.shm, st, B);
                else launch_level<double, true>(l, ub, cus, lds_cu, k.shm, st, B);
                break;
            case K_GLOBAL:
                if (fp32) launch_level<float, false>(l, ub, cus, lds_cu, 0, st, B);
                else launch_level<double, false>(l, ub, cus, lds_cu, 0, st, B);
                break;
            }
            if (err == hipSuccess) err = hipGetLastError();
        }
        if (fp32 && err == hipSuccess) {
            LevelArgs Q = A;
            Q.dclass = nullptr;
            Q.edge_base = 0;
            Q.max_m = D.max_m_all;
            launch_recheck(l, st, Q);
            err = hipGetLastError();
        }
    }
    FPC_HIP(err);
    return FPC_OK;
}

int level_tests(fpc_ctx *ctx, const LevelLaunch &Lv, const std::vector<int64_t> &ntests, LevelTiming *timing)
{
    hipStream_t st = ctx->stream;
    const int l = Lv.l;
    const int64_t E = Lv.n_edges;
    *timing = LevelTiming{};
    if (E == 0) return FPC_OK;
    if (Lv.n_insts < 1 || !Lv.insts) return FPC_EINVAL;
    const bool wide = l > kMaxTemplL;
    const bool fp32 = Lv.fp32 && !wide;
    const int lt = std::min(l, FPC_TUNE_LEVELS - 1);  // row of the tuning table
    // dynamic LDS available next to the kernels' few static words
    const size_t lds_cap = (size_t)ctx->lds_per_block - kStaticLds;

    // per size class: kernel, LDS, ranks per work item, windows of ranks
    // ([0, rpb), then growing by 8x; the first window covers every edge,
    // later ones only the edges with no separating rank yet, so the ranks
    // past an edge's first hit are never handed out)
    enum Kind { K_WIDE, K_TRIPLE, K_PAIR, K_TILE, K_GLOBAL };
    struct Cls {
        int64_t begin, end;
        int max_m;
        Kind kind;
        size_t shm;
        int pdec_n;
        int rpb;
        std::vector<int64_t> wins;
    };
    std::vector<Cls> cls;
    const LevelClass all{0, E, Lv.max_m};
    const LevelClass *lc = Lv.classes ? Lv.classes : &all;
    const int nlc = Lv.classes ? Lv.n_classes : 1;
    int max_nw = 0;
    for (int c = 0; c < nlc; ++c) {
        Cls k{lc[c].begin, lc[c].end, lc[c].max_m, K_GLOBAL, 0, 0, 0, {}};
        if (k.begin < 0 || k.end > E || k.begin >= k.end) return FPC_EINVAL;
        const int fk = Lv.force_kernel;
        if (wide) {
            if (fk != 0) return FPC_EINVAL;  // levels above the register kernels have one kernel
            k.kind = K_WIDE;
            k.shm = 8 * ((size_t)(l + 2) * (l + 3) / 2 + 1) + sizeof(int) * (l + 1) + 16;
            if (k.shm > lds_cap) return FPC_EBUDGET;
        } else {
            // shared-prefix kernel: the triple form when the tuning table (or
            // the caller) asks for it, else the pair form
            const bool triple = fk ? fk == FPC_KERNEL_TRIPLE : use_triple(ctx, l);
            if ((fk == FPC_KERNEL_PAIR && l < 2) || (fk == FPC_KERNEL_TRIPLE && l < 3)) return FPC_EINVAL;
            const size_t ps = l < 2 ? 0
                            : triple ? (fp32 ? triple_lds_bytes<float>(l, k.max_m) : triple_lds_bytes<double>(l, k.max_m))
                                     : (fp32 ? pair_lds_bytes<float>(l, k.max_m) : pair_lds_bytes<double>(l, k.max_m));
            const bool shared = fk ? (fk == FPC_KERNEL_PAIR || fk == FPC_KERNEL_TRIPLE)
                                   : (l >= 2 && ctx->use_pair_kernel && ps <= lds_cap);
            if (shared) {
                if (ps > lds_cap) return FPC_EINVAL;
                k.kind = triple ? K_TRIPLE : K_PAIR;
                k.shm = ps;
                if (k.kind == K_TRIPLE) {
                    k.pdec_n = triple_table_entries(l, fp32, k.max_m, ps, (size_t)ctx->lds_per_cu, lds_cap,
                                                    ctx->tuning.max_blocks_per_cu[lt]);
                    if (Lv.force_pdec >= 0) {
                        const int full = k.max_m > 2 ? std::min((k.max_m - 1) * (k.max_m - 2) / 2, kPdecCap) : 0;
                        k.pdec_n = std::min(Lv.force_pdec, full);
                        if (ps + pdec_bytes(k.pdec_n) > lds_cap) return FPC_EINVAL;
                    }
                    k.shm += pdec_bytes(k.pdec_n);
                }
            } else {
                const size_t ts = tile_bytes(k.max_m, fp32 ? 4 : 8);
                k.kind = fk != FPC_KERNEL_GLOBAL && ts <= std::min<size_t>(lds_cap, 65536) ? K_TILE : K_GLOBAL;
                k.shm = k.kind == K_TILE ? ts : 0;
            }
        }
        // ranks per work item: the tuning table's value for this level and kernel
        const fpc_tuning &tu = ctx->tuning;
        k.rpb = k.kind == K_WIDE ? kGenericRanks
              : (k.kind == K_TRIPLE || k.kind == K_PAIR) ? kWaves * tu.shared_ranks_per_wave[lt]
                                                           : kWaves * tu.test_ranks_per_wave[lt];
        if (Lv.force_rpw > 0 && k.kind != K_WIDE) k.rpb = kWaves * Lv.force_rpw;
        if (Lv.diag_r) {  // one window: the requested ranks
            k.wins = {Lv.diag_lo, Lv.diag_hi};
        } else {
            int64_t maxN = 0;
            for (int64_t e = k.begin; e < k.end; ++e) maxN = std::max(maxN, ntests[e]);
            k.wins.push_back(0);
            for (int64_t w = (int64_t)k.rpb * std::max(1, ctx->tuning.first_window_items[lt]); k.wins.back() < maxN;
                 w *= std::max(2, ctx->tuning.window_growth[lt]))
                k.wins.push_back(std::min<int64_t>(maxN, k.wins.back() + w));
        }
        max_nw = std::max(max_nw, (int)k.wins.size() - 1);
        cls.push_back(std::move(k));
    }

    // instance table: matrices of the level's precision and thresholds
    const int ni = Lv.n_insts;
    int rc = ctx->insts.ensure(sizeof(InstRec) * (size_t)ni);
    if (rc) return rc;
    if ((rc = ctx->h_inst.ensure(Lv.inst_off + sizeof(InstRec) * (size_t)ni))) return rc;
    // the level's records in h_inst are free: the upload from them of the
    // last level that used them completed before a stream synchronisation
    // (levels queued back to back use records of their own)
    InstRec *hin = reinterpret_cast<InstRec *>(ctx->h_inst.as<char>() + Lv.inst_off);
    for (int k = 0; k < ni; ++k) {
        const LevelInst &I = Lv.insts[k];
        hin[k].C = fp32 ? (const void *)I.C32 : (const void *)I.C64;
        hin[k].C64 = I.C64;
        hin[k].ld = I.p;
        hin[k].th = make_thresholds(I.q, I.n, l, Lv.band_z, I.c_err + 4.0 * (l + 2) * 6.0e-8,
                                    resolve_tau(Lv.ill_cond_tau, I.n, l, I.c_err));
    }
    if ((rc = upload_enqueue(ctx, ctx->insts.ptr, ctx->h_inst, Lv.inst_off, sizeof(InstRec) * (size_t)ni)))
        return rc;

    // plan buffers, [n_items, item_ctr], workgroup sums, per-edge offsets:
    // one for the first class of each window (main stream), one for the
    // classes after it (second stream), each reused in its stream's order
    const int64_t nbmax = (E + kPlanChunk - 1) / kPlanChunk;
    const size_t plan_words = (size_t)(2 + nbmax + E + 1);
    if ((rc = ctx->blockoff.ensure(sizeof(int64_t) * 2 * plan_words))) return rc;
    int64_t *const plan_buf[2] = {ctx->blockoff.as<int64_t>(), ctx->blockoff.as<int64_t>() + plan_words};

    LevelArgs A{};
    A.cand = Lv.cand;
    A.inst = ctx->insts.as<InstRec>();
    A.binom = ctx->binom.as<int64_t>();
    A.binomT = ctx->binomT.as<int64_t>();
    A.counters = Lv.counters;
    A.inst_cnt = Lv.inst_cnt;
    A.queue = Lv.queue;
    A.queue_cap = Lv.queue_cap;
    A.diag_r = Lv.diag_r;
    A.diag_dec = Lv.diag_dec;
    A.diag_lo = Lv.diag_lo;

    const int cus = ctx->num_cus;
    const size_t lds_cu = (size_t)ctx->lds_per_cu;
    g_max_blocks_per_cu = ctx->tuning.max_blocks_per_cu[lt];
    const hipEvent_t ev0 = Lv.events ? Lv.events->ev0 : ctx->ev0;
    const hipEvent_t ev1 = Lv.events ? Lv.events->ev1 : ctx->ev1;
    const hipEvent_t *lev = Lv.events ? Lv.events->lev : ctx->lev;
    const int n_lev = Lv.events ? Lv.events->n_lev : fpc_ctx::kLaunchEvents;
    const bool graph = Lv.graph;
    hipGraph_t g = nullptr;
    if (graph) FPC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    else FPC_HIP(hipEventRecord(ev0, st));
    int nev = 0, nlaunch = 0;
    hipError_t err = hipSuccess;
    // the size classes of a window test disjoint edges: they are split over
    // the main stream and a second one, so that their launches (few long
    // items on the long lists) overlap instead of following one another; a
    // captured level keeps one stream
    const bool two = !graph && !Lv.diag_r && ctx->aux;
    for (int w = 0; w < max_nw && err == hipSuccess; ++w) {
        // the classes of a window share the recheck queue: the window's first
        // plan empties it and one FP64 re-run after its last launch drains it
        // (before any plan of the next window reads minhit)
        bool window_open = false, forked = false;
        // the window's launches: range, items (upper bound) and ranks per item
        struct WinLaunch {
            const Cls *k;
            int64_t lo, hi, ub;
            int rpb;
            bool aux;
        };
        std::vector<WinLaunch> wl;
        for (const Cls &k : cls) {
            if (w + 1 >= (int)k.wins.size()) continue;
            const int64_t lo = k.wins[w], hi = k.wins[w + 1];
            // upper bound of the items (every edge live) sizes the grid
            const auto items_ub = [&](int64_t rpb) {
                int64_t n = 0;
                for (int64_t e = k.begin; e < k.end; ++e) {
                    const int64_t span = std::min(ntests[e], hi) - lo;
                    if (span > 0) n += (span + rpb - 1) / rpb;
                }
                return n;
            };
            int rpb = k.rpb;
            int64_t ub = items_ub(rpb);
            if (ub == 0) continue;
            // A launch with fewer items than resident workgroups leaves CUs
            // idle and lasts as long as its longest item: the triple kernel
            // halves its items while they still fit one resident round (an
            // edge's result does not depend on how its ranks are cut; every
            // item stages its tile again, so more rounds would cost more).
            if (k.kind == K_TRIPLE && Lv.force_rpw == 0) {
                const int64_t slots =
                    (int64_t)cus * triple_blocks_per_cu(l, fp32, k.shm, lds_cu, ctx->tuning.max_blocks_per_cu[lt]);
                while (rpb / 2 >= kWaves * kSplitMinRanksPerWave) {
                    const int64_t n2 = items_ub(rpb / 2);
                    if (n2 > slots) break;
                    rpb /= 2;
                    ub = n2;
                }
            }
            wl.push_back({&k, lo, hi, ub, rpb, false});
        }
        // Two streams: the class with the most ranks (upper bound) leads on
        // the context's stream; each other class, in decreasing ranks, goes
        // to the stream with fewer ranks so far (longest first).
        if (two && wl.size() > 1) {
            std::stable_sort(wl.begin(), wl.end(), [](const WinLaunch &x, const WinLaunch &y) {
                return (double)x.ub * x.rpb > (double)y.ub * y.rpb;
            });
            double on_main = (double)wl[0].ub * wl[0].rpb, on_aux = 0.0;
            for (size_t i = 1; i < wl.size(); ++i) {
                const double r = (double)wl[i].ub * wl[i].rpb;
                wl[i].aux = on_aux <= on_main;
                (wl[i].aux ? on_aux : on_main) += r;
            }
        }
        for (const WinLaunch &wn : wl) {
            const Cls &k = *wn.k;
            const int64_t lo = wn.lo, hi = wn.hi, ub = wn.ub;
            const int rpb = wn.rpb;
            const int64_t Ek = k.end - k.begin, nb = (Ek + kPlanChunk - 1) / kPlanChunk;
            // on the second stream: after the first class's plan (which
            // empties the recheck queue)
            const bool on_aux = wn.aux;
            if (on_aux && !forked) {
                err = hipStreamWaitEvent(ctx->aux, ctx->ev_fork, 0);
                if (err != hipSuccess) break;
                forked = true;
            }
            const hipStream_t ls = on_aux ? ctx->aux : st;
            int64_t *const pl = plan_buf[on_aux ? 1 : 0];
            A.n_items = pl;
            A.item_ctr = reinterpret_cast<unsigned long long *>(pl + 1);
            PlanArgs P{};
            P.edges = Lv.edges + k.begin;
            P.minhit = Lv.minhit + k.begin;
            P.n_edges = Ek;
            P.lo = lo;
            P.hi = hi;
            P.rpb = rpb;
            P.filter = w > 0;
            P.sums = pl + 2;
            P.off = pl + 2 + nb;
            P.n_items = pl;
            P.item_ctr = A.item_ctr;
            P.queue_len = window_open ? nullptr : &Lv.counters[1];
            window_open = true;
            A.edges = P.edges;
            A.minhit = Lv.minhit + k.begin;
            A.n_edges = Ek;
            A.blockoff = P.off;
            A.win_lo = lo;
            A.win_hi = hi;
            A.ranks_per_block = rpb;
            A.edge_base = k.begin;
            A.max_m = k.max_m;
            A.pdec_n = k.pdec_n;
            if (Ek <= kPlanSingleEdges) {
                plan_single<<<1, kPlanSingleThreads, 0, ls>>>(P);
            } else {
                plan_reduce<<<(unsigned)nb, 256, 0, ls>>>(P);
                plan_sums<<<1, 256, 0, ls>>>(P, (int)nb);
                plan_scan<<<(unsigned)nb, 256, 0, ls>>>(P);
            }
            if (two && &wn == &wl[0]) {  // the point the window's other classes start from
                err = hipEventRecord(ctx->ev_fork, st);
                if (err != hipSuccess) break;
            }
            const bool timed = !graph && nev < n_lev;
            if (timed) (void)hipEventRecord(lev[2 * nev], ls);
            switch (k.kind) {
            case K_WIDE: {  // wide levels always run in FP64
                const void *fn = (const void *)level_kernel_wide<double>;
                level_kernel_wide<double><<<resident_grid(fn, 64, k.shm, ub, cus, lds_cu), 64, k.shm, ls>>>(A, l);
                break;
            }
            case K_TRIPLE:
                err = fp32 ? launch_triple<float>(l, ub, cus, lds_cu, k.shm, ls, A)
                           : launch_triple<double>(l, ub, cus, lds_cu, k.shm, ls, A);
                break;
            case K_PAIR:
                err = fp32 ? launch_pair<float>(l, ub, cus, lds_cu, k.shm, ls, A)
                           : launch_pair<double>(l, ub, cus, lds_cu, k.shm, ls, A);
                break;
            case K_TILE:
                if (fp32) launch_level<float, true>(l, ub, cus, lds_cu, k.shm, ls, A);
                else launch_level<double, true>(l, ub, cus, lds_cu, k.shm, ls, A);
                break;
            case K_GLOBAL:
                if (fp32) launch_level<float, false>(l, ub, cus, lds_cu, 0, ls, A);
                else launch_level<double, false>(l, ub, cus, lds_cu, 0, ls, A);
                break;
            }
            if (timed) {
                (void)hipEventRecord(lev[2 * nev + 1], ls);
                ++nev;
            }
            if (trace_on())
                std::fprintf(stderr, "[fpc]   l=%d window %d class %d: kind %d, lists <= %d, LDS %zu B (pair table %d), "
                             "grid %u, items <= %lld of %d ranks\n", l, w, (int)(&k - cls.data()), (int)k.kind, k.max_m, k.shm,
                             k.pdec_n, g_last_grid, (long long)ub, rpb);
            ++nlaunch;
            if (err == hipSuccess) err = hipGetLastError();
            if (err != hipSuccess) break;
        }
        // join: the re-run and the next window's plans follow every class
        if (forked) {
            const hipError_t e1 = hipEventRecord(ctx->ev_join, ctx->aux);
            const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(st, ctx->ev_join, 0) : e1;
            if (err == hipSuccess) err = e2;
        }
        // FP64 re-run of the window's queue (level edge indices)
        if (fp32 && window_open && err == hipSuccess && !Lv.diag_r) {
            LevelArgs Q = A;
            Q.edges = Lv.edges;
            Q.minhit = Lv.minhit;
            Q.n_edges = E;
            Q.edge_base = 0;
            Q.max_m = Lv.max_m;
            launch_recheck(l, st, Q);
            err = hipGetLastError();
        }
    }
    if (graph) {
        const hipError_t e2 = hipStreamEndCapture(st, &g);
        if (err == hipSuccess) err = e2;
        hipGraphExec_t ge = nullptr;
        if (err == hipSuccess) err = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (err == hipSuccess) err = hipEventRecord(ev0, st);
        if (err == hipSuccess) err = hipGraphLaunch(ge, st);
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
    }
    FPC_HIP(err);
    FPC_HIP(hipEventRecord(ev1, st));
    timing->test_launches = nlaunch;
    timing->n_events = nev;
    timing->graph = graph;
    timing->e0 = ev0;
    timing->e1 = ev1;
    timing->lev = lev;
    return FPC_OK;
}

int level_timing(fpc_ctx *ctx, LevelTiming *timing)
{
    (void)ctx;
    if (!timing->e1) return FPC_OK;  // nothing was launched
    FPC_HIP(hipEventSynchronize(timing->e1));
    FPC_HIP(hipEventElapsedTime(&timing->all_ms, timing->e0, timing->e1));
    // the launches of a window's size classes overlap (two streams): the
    // test time is the length of the union of the launch intervals
    timing->test_ms = 0.f;
    std::vector<std::pair<float, float>> iv(timing->n_events);
    for (int k = 0; k < timing->n_events; ++k) {
        FPC_HIP(hipEventElapsedTime(&iv[k].first, timing->e0, timing->lev[2 * k]));
        FPC_HIP(hipEventElapsedTime(&iv[k].second, timing->e0, timing->lev[2 * k + 1]));
    }
    std::sort(iv.begin(), iv.end());
    float lo = 0.f, hi = -1.f;
    for (const auto &x : iv) {
        if (x.first > hi) {
            if (hi > lo) timing->test_ms += hi - lo;
            lo = x.first;
            hi = x.second;
        } else {
            hi = std::max(hi, x.second);
        }
    }
    if (hi > lo) timing->test_ms += hi - lo;
    if (timing->graph) timing->test_ms = timing->all_ms;  // one graph: plans and rechecks included
    return FPC_OK;
}

int level_reserve(fpc_ctx *ctx, int64_t n_edges, int n_insts, int n_levels, size_t *inst_stride)
{
    if (n_edges < 0 || n_insts < 1 || n_levels < 1) return FPC_EINVAL;
    // the two plan buffers of level_tests at their size for n_edges
    const int64_t nbmax = (n_edges + kPlanChunk - 1) / kPlanChunk;
    int rc = ctx->blockoff.ensure(sizeof(int64_t) * 2 * (size_t)(2 + nbmax + n_edges + 1));
    if (!rc) rc = ctx->insts.ensure(sizeof(InstRec) * (size_t)n_insts);
    const size_t stride = (sizeof(InstRec) * (size_t)n_insts + 255) / 256 * 256;
    if (!rc) rc = ctx->h_inst.ensure(stride * (size_t)n_levels);
    if (rc) return rc;
    *inst_stride = stride;
    return FPC_OK;
}

// minhit[e] = no hit yet (all ones), counters zeroed: one small kernel in
// place of two memset commands.
__global__ __launch_bounds__(256) void level_init_kernel(uint64_t *__restrict__ minhit, int64_t n_edges,
                                                         unsigned long long *__restrict__ counters, int n_cnt)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n_edges) minhit[t] = ~0ull;
    if (t < n_cnt) counters[t] = 0ull;
}

int level_init(fpc_ctx *ctx, uint64_t *minhit, int64_t n_edges, unsigned long long *counters, int n_cnt)
{
    const int64_t n = std::max<int64_t>(n_edges, n_cnt);
    if (n > 0)
        level_init_kernel<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(minhit, n_edges, counters, n_cnt);
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

// Upload of 4-byte words from pinned host memory by a kernel that reads the
// host buffer through its device mapping with system-scope loads (coherent
// with the host's writes made before the launch).
__global__ __launch_bounds__(256) void upload_kernel(uint32_t *__restrict__ dst, const uint32_t *src, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += stride)
        dst[k] = __hip_atomic_load(src + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

int upload_enqueue(fpc_ctx *ctx, void *dst, const HostBuf &src, size_t offset, size_t bytes)
{
    if (bytes == 0) return FPC_OK;
    if (!dst || !src.ptr || offset + bytes > src.bytes) return FPC_EINVAL;
    hipStream_t st = ctx->stream;
    const char *h = static_cast<const char *>(src.ptr) + offset;
    void *mapped = nullptr;
    if (bytes % 4 || (uintptr_t)dst % 4 || (uintptr_t)h % 4 ||
        hipHostGetDevicePointer(&mapped, src.ptr, 0) != hipSuccess || !mapped) {
        (void)hipGetLastError();
        FPC_HIP(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, st));
        return FPC_OK;
    }
    const int64_t n = (int64_t)(bytes / 4);
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    upload_kernel<<<grid, 256, 0, st>>>(static_cast<uint32_t *>(dst),
                                        reinterpret_cast<const uint32_t *>(static_cast<const char *>(mapped) + offset),
                                        n);
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

int level_compact_enqueue(fpc_ctx *ctx, const uint64_t *minhit, int64_t n_edges, int64_t *d_pairs,
                          unsigned long long *d_count)
{
    if (n_edges > 0)
        compact_kernel<<<(unsigned)((n_edges + 255) / 256), 256, 0, ctx->stream>>>(minhit, n_edges, d_pairs, d_count);
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

int ci_batch(fpc_ctx *ctx, const void *C, int c_dtype, int p, int n, int l, const int32_t *B, int64_t b, double q,
             double *z_out, uint8_t *indep_out)
{
    if (!C || p < 2 || l < 0 || b < 0 || n - l - 3 <= 0 || l > p - 2) return FPC_EINVAL;
    if (c_dtype != FPC_F64 && c_dtype != FPC_F32) return FPC_EINVAL;
    if (b == 0) return FPC_OK;
    if (!B) return FPC_EINVAL;
    hipStream_t st = ctx->stream;
    const Thresholds th = make_thresholds(q, n, l, 0.0, 0.0);
    int rc = ctx->flag.ensure(64);
    if (rc) return rc;
    int *bad = ctx->flag.as<int>() + 6;
    FPC_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    if (l <= kMaxTemplL) {
        if ((b + 255) / 256 > 0x7fffffffLL) return FPC_EINVAL;
        dim3 g((unsigned)((b + 255) / 256));
        if (c_dtype == FPC_F64) launch_batch<double>(l, g, st, (const double *)C, p, B, b, th, z_out, indep_out, bad);
        else launch_batch<float>(l, g, st, (const float *)C, p, B, b, th, z_out, indep_out, bad);
    } else {
        const size_t shm = (c_dtype == FPC_F64 ? 8 : 4) * ((size_t)(l + 2) * (l + 3) / 2 + 1) + 16;
        if (shm > (size_t)ctx->lds_per_block) return FPC_EINVAL;
        if (b > 0x7fffffffLL) return FPC_EINVAL;
        dim3 g((unsigned)b);
        if (c_dtype == FPC_F64)
            batch_kernel_wide<double><<<g, 64, shm, st>>>((const double *)C, p, B, b, l, th, z_out, indep_out, bad);
        else
            batch_kernel_wide<float><<<g, 64, shm, st>>>((const float *)C, p, B, b, l, th, z_out, indep_out, bad);
    }
    FPC_HIP(hipGetLastError());
    int hbad = 0;
    FPC_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    FPC_HIP(hipStreamSynchronize(st));
    return hbad ? FPC_EINVAL : FPC_OK;
}

int level_series(fpc_ctx *ctx, const void *C, int c_dtype, int p, int n, int l, int i, int j, const int32_t *cand,
                 int m, int64_t rank_lo, int64_t rank_hi, int kernel, int ranks_per_wave, int pair_table, double q,
                 double band_z, double c_err, double ill_cond_tau, double *r_out, uint8_t *dec_out)
{
    if (std::isnan(ill_cond_tau)) return FPC_EINVAL;
    if (!C || !r_out || !dec_out || (m > 0 && !cand)) return FPC_EINVAL;
    if (c_dtype != FPC_F64 && c_dtype != FPC_F32) return FPC_EINVAL;
    if (p < 2 || i < 0 || j < 0 || i >= p || j >= p || i == j) return FPC_EINVAL;
    if (l < 0 || m < l || m >= kBinomRows || m > p - 2 || n - l - 3 <= 0) return FPC_EINVAL;
    if (kernel < FPC_KERNEL_AUTO || kernel > FPC_KERNEL_GLOBAL) return FPC_EINVAL;
    if (ranks_per_wave != 0 && (ranks_per_wave < 64 || ranks_per_wave > (1 << 20))) return FPC_EINVAL;
    if (pair_table < -1 || !(q >= 0.0) || !(c_err >= 0.0) || !(band_z >= 0.0)) return FPC_EINVAL;
    if (l > kMaxTemplL && c_dtype != FPC_F64) return FPC_EINVAL;  // levels above run in FP64 only
    const int64_t N = binom_sat(m, l);
    if (N == INT64_MAX || rank_lo < 0 || rank_hi > N || rank_lo >= rank_hi) return FPC_EINVAL;
    std::vector<uint8_t> seen((size_t)p, 0);
    for (int t = 0; t < m; ++t) {
        const int v = cand[t];
        if (v < 0 || v >= p || v == i || v == j || seen[(size_t)v]) return FPC_EINVAL;
        seen[(size_t)v] = 1;
    }
    hipStream_t st = ctx->stream;
    int rc;
    if ((rc = ctx->cand.ensure(sizeof(int32_t) * (size_t)(m + 1)))) return rc;
    if ((rc = ctx->edges.ensure(sizeof(EdgeRec)))) return rc;
    if ((rc = ctx->minhit.ensure(sizeof(uint64_t)))) return rc;
    if ((rc = ctx->counters.ensure(sizeof(unsigned long long) * 10))) return rc;
    const EdgeRec rec{i, j, m, 0, N, 0, 0};
    FPC_HIP(hipMemcpyAsync(ctx->edges.ptr, &rec, sizeof(rec), hipMemcpyHostToDevice, st));
    if (m > 0) FPC_HIP(hipMemcpyAsync(ctx->cand.ptr, cand, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, st));
    if ((rc = level_init(ctx, ctx->minhit.as<uint64_t>(), 1, ctx->counters.as<unsigned long long>(), 10))) return rc;
    const bool fp32 = c_dtype == FPC_F32;
    const LevelInst inst{fp32 ? static_cast<const float *>(C) : nullptr,
                         fp32 ? nullptr : static_cast<const double *>(C), p, n, q, c_err};
    LevelLaunch Lv{};
    Lv.l = l;
    Lv.max_m = m;
    Lv.n_edges = 1;
    Lv.edges = ctx->edges.as<EdgeRec>();
    Lv.cand = ctx->cand.as<int32_t>();
    Lv.insts = &inst;
    Lv.n_insts = 1;
    Lv.fp32 = fp32;
    Lv.band_z = band_z;
    Lv.ill_cond_tau = ill_cond_tau;
    Lv.minhit = ctx->minhit.as<uint64_t>();
    Lv.counters = ctx->counters.as<unsigned long long>();
    Lv.inst_cnt = Lv.counters + 8;
    Lv.diag_r = r_out;
    Lv.diag_dec = dec_out;
    Lv.diag_lo = rank_lo;
    Lv.diag_hi = rank_hi;
    Lv.force_kernel = kernel;
    Lv.force_pdec = pair_table;
    Lv.force_rpw = ranks_per_wave;
    // the kernel choice of a level run with the default flags
    const bool pair_was = ctx->use_pair_kernel;
    ctx->use_pair_kernel = true;
    LevelTiming tm;
    rc = level_tests(ctx, Lv, std::vector<int64_t>{N}, &tm);
    ctx->use_pair_kernel = pair_was;
    if (rc) return rc;
    FPC_HIP(hipStreamSynchronize(st));
    return FPC_OK;
}

}  // namespace fpc

extern "C" int fpc_level_series(fpc_ctx *ctx, const void *C, int c_dtype, int p, int n, int l, int i, int j,
                                const int32_t *cand, int m, int64_t rank_lo, int64_t rank_hi, int kernel,
                                int ranks_per_wave, int pair_table, double q, double band_z, double c_err,
                                double ill_cond_tau, double *r_out, uint8_t *dec_out)
{
    if (!ctx) return FPC_EINVAL;
    FPC_HIP(hipSetDevice(ctx->device));
    return fpc::level_series(ctx, C, c_dtype, p, n, l, i, j, cand, m, rank_lo, rank_hi, kernel, ranks_per_wave,
                             pair_table, q, band_z, c_err, ill_cond_tau, r_out, dec_out);
}

extern "C" int fpc_ci_batch(fpc_ctx *ctx, const void *C, int c_dtype, int p, int n, int l, const int32_t *B,
                            int64_t b, double q, double *z_out, uint8_t *indep_out)
{
    if (!ctx) return FPC_EINVAL;
    return fpc::ci_batch(ctx, C, c_dtype, p, n, l, B, b, q, z_out, indep_out);
}

namespace fpc {

void tuning_defaults(fpc_tuning *t)
{
    std::memset(t, 0, sizeof(*t));
    for (int l = 0; l < FPC_TUNE_LEVELS; ++l) {
        t->test_ranks_per_wave[l] = kRanksPerWave;
        t->shared_ranks_per_wave[l] = kPairRanksPerWave;
        t->window_growth[l] = 8;
        t->first_window_items[l] = 1;
        t->max_blocks_per_cu[l] = 0;
        t->shared_prefix_depth[l] = l >= 3 ? 3 : 2;
    }
}

}  // namespace fpc

extern "C" int fpc_get_tuning(const fpc_ctx *ctx, fpc_tuning *out)
{
    if (!ctx || !out) return FPC_EINVAL;
    *out = ctx->tuning;
    return FPC_OK;
}

extern "C" int fpc_set_tuning(fpc_ctx *ctx, const fpc_tuning *t)
{
    if (!ctx) return FPC_EINVAL;
    if (!t) {
        fpc::tuning_defaults(&ctx->tuning);
        return FPC_OK;
    }
    for (int l = 0; l < FPC_TUNE_LEVELS; ++l) {
        if (t->test_ranks_per_wave[l] < 64 || t->test_ranks_per_wave[l] > (1 << 20)) return FPC_EINVAL;
        if (t->shared_ranks_per_wave[l] < 64 || t->shared_ranks_per_wave[l] > (1 << 20)) return FPC_EINVAL;
        if (t->window_growth[l] < 2 || t->window_growth[l] > 64) return FPC_EINVAL;
        if (t->first_window_items[l] < 1 || t->first_window_items[l] > 64) return FPC_EINVAL;
        if (t->max_blocks_per_cu[l] < 0 || t->max_blocks_per_cu[l] > 32) return FPC_EINVAL;
        if (t->shared_prefix_depth[l] != 2 && t->shared_prefix_depth[l] != 3) return FPC_EINVAL;
        if (l < 3 && t->shared_prefix_depth[l] != 2) return FPC_EINVAL;
    }
    ctx->tuning = *t;
    return FPC_OK;
}
