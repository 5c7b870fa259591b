// Context management and the level loop of Phase I: Algorithm 2 (reverse
// order, Sec. 3.2) or Algorithm 1 (forward, Sec. 2.2.1), stable variant
// (deletions of a level collected in D and applied at its end), sampling
// version (Fisher-z test of Sec. 2.2.2).
//
// Per level (host): candidate sets of the frozen graph, the table of edges
// with |cand| >= l and their C(|cand|, l) counts, one upload; (device) the
// test kernels over growing windows of ranks, the FP64 recheck of queued
// FP32 tests, and the compaction of deleted edges; (host) one download of
// (edge, lowest separating rank) pairs, decoding of the separating sets and
// the level-end deletion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "fpc_internal.h"

namespace fpc {

namespace {
thread_local std::string g_last_hip;
}

int hip_fail(hipError_t e, const char *what)
{
    g_last_hip = std::string(hipGetErrorName(e)) + " (" + hipGetErrorString(e) + ") in " + what;
    return FPC_EDEVICE;
}

// FPC_FAIL_ALLOC=1: every device allocation fails with FPC_ENOMEM before
// the runtime is called (a test hook for the error path; read per call).
static bool alloc_hook_fails()
{
    const char *v = std::getenv("FPC_FAIL_ALLOC");
    return v && v[0] == '1' && v[1] == 0;
}

int DevBuf::ensure(size_t need)
{
    if (need <= bytes && ptr) return FPC_OK;
    if (alloc_hook_fails()) return FPC_ENOMEM;
    release();
    size_t want = std::max(need, (size_t)256);
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? FPC_ENOMEM : hip_fail(e, "hipMalloc");
    }
    bytes = want;
    return FPC_OK;
}

void DevBuf::release()
{
    if (ptr) {
        (void)hipDeviceSynchronize();  // no kernel may still use the old allocation
        (void)hipFree(ptr);
    }
    ptr = nullptr;
    bytes = 0;
}

int HostBuf::ensure(size_t need)
{
    if (need <= bytes && ptr) return FPC_OK;
    release();
    size_t want = std::max(need, (size_t)4096);
    hipError_t e = hipHostMalloc(&ptr, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return FPC_ENOMEM;
    }
    bytes = want;
    return FPC_OK;
}

void HostBuf::release()
{
    if (ptr) {
        (void)hipDeviceSynchronize();  // no copy may still read the old allocation
        (void)hipHostFree(ptr);
    }
    ptr = nullptr;
    bytes = 0;
}

int64_t binom_sat(int a, int b)
{
    if (b < 0 || a < 0 || b > a) return 0;
    b = std::min(b, a - b);
    unsigned __int128 v = 1;
    for (int t = 1; t <= b; ++t) {
        v = v * (unsigned)(a - b + t) / (unsigned)t;  // exact at every step
        if (v > (unsigned __int128)INT64_MAX) return INT64_MAX;
    }
    return (int64_t)v;
}

// FPC_TRACE=1 in the environment: phase timings of each level on stderr.
bool trace_on()
{
    static const bool on = [] {
        const char *v = std::getenv("FPC_TRACE");
        return v && *v && *v != '0';
    }();
    return on;
}

namespace {

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}


inline int64_t pair_index(int i, int j, int p)
{
    return (int64_t)i * p - (int64_t)i * (i + 1) / 2 + (j - i - 1);
}

// Lexicographic unranking of rank R among the l-subsets of m positions
// (tabT: the saturating binomial table column-major, C(a, b) at
// b * kBinomRows + a for b < kBinomCols; R < C(m, l)).
void unrank_host(int64_t R, int m, int l, const std::vector<int64_t> &tabT, std::vector<int> &out)
{
    out.resize(l);
    int x = 0;
    for (int t = 0; t < l; ++t) {
        // skip the subsets whose element t comes before x: C(m-1-x, l-1-t)
        // of them per position, read down one column of the table
        const int k = l - 1 - t;
        if (k < kBinomCols) {
            const int64_t *col = tabT.data() + (size_t)k * kBinomRows;
            for (;;) {
                const int64_t cnt = col[m - 1 - x];
                if (R < cnt) break;
                R -= cnt;
                ++x;
            }
        } else {
            for (;;) {
                const int64_t cnt = binom_sat(m - 1 - x, k);
                if (R < cnt) break;
                R -= cnt;
                ++x;
            }
        }
        out[t] = x++;
    }
}

// Separating sets found by the subset levels: one entry per deleted pair
// with its level (= set size) and the set's nodes in a flat array.  Pairs
// deleted by the first level are not listed: in the result they are the
// pairs absent from the graph and from this list (kind ALL_BUT).
struct SepList {
    int64_t pair;   // pair index (i < j, row-major upper triangle)
    int64_t off;    // offset into nodes
    int32_t level;  // set size
};
struct SepStore {
    std::vector<SepList> lists;
    std::vector<int32_t> nodes;
    bool first_level = false;  // the l = p-2 level ran (its deletions are implicit)
    void reset()
    {
        lists.clear();
        nodes.clear();
        first_level = false;
    }
};

}  // namespace

}  // namespace fpc

using namespace fpc;

extern "C" const char *fpc_strerror(int code)
{
    switch (code) {
    case FPC_OK: return "ok";
    case FPC_EINVAL: return "invalid argument";
    case FPC_ENONFINITE: return "non-finite value in the data";
    case FPC_ESINGULAR: return "correlation matrix is not positive definite";
    case FPC_EBUDGET: return "test budget exceeded";
    case FPC_ENOMEM: return "out of memory";
    case FPC_EDEVICE: return "HIP runtime error";
    case FPC_ESCRATCH: return "problem larger than the static workspace of the no-allocation entry point";
    case FPC_ETOOLARGE: return "a candidate set of 1024 or more variables at a subset level";
    default: return "unknown error";
    }
}

extern "C" const char *fpc_last_hip_error(void) { return g_last_hip.c_str(); }

extern "C" int fpc_create(fpc_ctx **out, int hip_device, void *hip_stream)
{
    if (!out) return FPC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (hip_device < 0 || hip_device >= ndev) return FPC_EINVAL;
    FPC_HIP(hipSetDevice(hip_device));
    fpc_ctx *c = new (std::nothrow) fpc_ctx();
    if (!c) return FPC_ENOMEM;
    c->device = hip_device;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device) == hipSuccess && v > 0)
        c->lds_per_block = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && v > 0)
        c->num_cus = v;
    fpc::tuning_defaults(&c->tuning);
    c->lds_per_cu = c->lds_per_block;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, hip_device) == hipSuccess &&
        v > c->lds_per_cu)
        c->lds_per_cu = v;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "hipStreamCreate");
        }
        c->own_stream = true;
    }
    if ((e = hipEventCreate(&c->ev0)) != hipSuccess || (e = hipEventCreate(&c->ev1)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_first, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_c32, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking)) != hipSuccess) {
        fpc_destroy(c);
        return hip_fail(e, "hipEventCreate");
    }
    for (hipEvent_t &ev : c->lev) {
        if ((e = hipEventCreate(&ev)) != hipSuccess) {
            fpc_destroy(c);
            return hip_fail(e, "hipEventCreate");
        }
    }
    c->binom_host.resize((size_t)kBinomRows * kBinomCols);
    for (int a = 0; a < kBinomRows; ++a)
        for (int b = 0; b < kBinomCols; ++b) c->binom_host[(size_t)a * kBinomCols + b] = binom_sat(a, b);
    int rc = c->binom.ensure(sizeof(int64_t) * c->binom_host.size());
    if (rc) {
        fpc_destroy(c);
        return rc;
    }
    e = hipMemcpy(c->binom.ptr, c->binom_host.data(), sizeof(int64_t) * c->binom_host.size(),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        fpc_destroy(c);
        return hip_fail(e, "hipMemcpy");
    }
    {
        std::vector<int64_t> &t = c->binomT_host;
        t.resize((size_t)kBinomRows * kBinomCols);
        for (int a = 0; a < kBinomRows; ++a)
            for (int b = 0; b < kBinomCols; ++b)
                t[(size_t)b * kBinomRows + a] = c->binom_host[(size_t)a * kBinomCols + b];
        if ((rc = c->binomT.ensure(sizeof(int64_t) * t.size()))) {
            fpc_destroy(c);
            return rc;
        }
        e = hipMemcpy(c->binomT.ptr, t.data(), sizeof(int64_t) * t.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            fpc_destroy(c);
            return hip_fail(e, "hipMemcpy");
        }
    }
    if ((rc = fpc::noalloc_init(c))) {
        fpc_destroy(c);
        return rc;
    }
    *out = c;
    return FPC_OK;
}

extern "C" int fpc_destroy(fpc_ctx *c)
{
    if (!c) return FPC_EINVAL;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->aux) (void)hipStreamSynchronize(c->aux);
    DevBuf *bufs[] = {&c->binom, &c->binomT, &c->x_copy, &c->colstat, &c->c64, &c->c32, &c->zsplit, &c->inv_work,
                      &c->flag, &c->cand, &c->edges, &c->blockoff, &c->minhit, &c->counters,
                      &c->queue, &c->dellist, &c->batch_tmp, &c->mlp_grad, &c->rfirst, &c->feat,
                      &c->cand2, &c->degs, &c->insts, &c->batch_c};
    for (DevBuf *b : bufs) b->release();
    c->h_stage.release();
    c->h_back.release();
    c->h_inst.release();
    c->h_flag.release();
    for (hipEvent_t ev : c->lev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto &slot : c->chain_ev)
        for (hipEvent_t ev : slot)
            if (ev) (void)hipEventDestroy(ev);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->ev_first) (void)hipEventDestroy(c->ev_first);
    if (c->ev_c32) (void)hipEventDestroy(c->ev_c32);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return FPC_OK;
}

extern "C" int fpc_set_recheck_queue(fpc_ctx *ctx, int64_t initial, int64_t max)
{
    if (!ctx || initial < 1 || max < initial || max > (int64_t(1) << 31)) return FPC_EINVAL;
    ctx->queue_init = initial;
    ctx->queue_max = max;
    ctx->queue.release();
    return FPC_OK;
}

extern "C" void fpc_checkpoint_of(const fpc_result *r, fpc_checkpoint *ck)
{
    if (!r || !ck) return;
    ck->p = r->p;
    ck->next_level = r->next_level;
    ck->adj = r->adj;
    ck->sep_level = r->sep_level;
    ck->sep_kind = r->sep_kind;
    ck->sep_off = r->sep_off;
    ck->sep_nodes = r->sep_nodes;
    ck->n_levels = r->n_levels;
    ck->levels = r->levels;
}

extern "C" void fpc_result_free(fpc_result *r)
{
    if (!r) return;
    std::free(r->adj);
    std::free(r->sep_level);
    std::free(r->sep_kind);
    std::free(r->sep_off);
    std::free(r->sep_nodes);
    std::free(r->levels);
    std::free(r->log_x);
    std::free(r->log_y);
    std::free(r->log_group);
    std::free(r->log_level);
    std::free(r->list_pairs);
    std::free(r);
}

namespace {

// Recheck queue entries: the queue starts at ctx->queue_init entries and,
// when a launch overflows it, grows 4x (up to ctx->queue_max) and the level
// is run again in the mixed form; past that the level runs in FP64.  The
// grown size stays with the context.

class ResultPrefetch;

// The per-pair arrays of a result (adjacency, set level, set kind, node
// offset), the set nodes and the pairs of the lists; freed unless handed
// over.
struct PairArrays {
    uint8_t *adj = nullptr;
    int32_t *sep_level = nullptr;
    int8_t *sep_kind = nullptr;
    int64_t *sep_off = nullptr;
    int32_t *sep_nodes = nullptr;
    int64_t *list_pairs = nullptr;
    int64_t n_lists = 0;
    PairArrays() = default;
    PairArrays(const PairArrays &) = delete;
    PairArrays &operator=(const PairArrays &) = delete;
    PairArrays(PairArrays &&o) noexcept { *this = std::move(o); }
    PairArrays &operator=(PairArrays &&o) noexcept
    {
        if (this != &o) {
            release();
            adj = o.adj;
            sep_level = o.sep_level;
            sep_kind = o.sep_kind;
            sep_off = o.sep_off;
            sep_nodes = o.sep_nodes;
            list_pairs = o.list_pairs;
            n_lists = o.n_lists;
            o.adj = nullptr;
            o.sep_level = nullptr;
            o.sep_kind = nullptr;
            o.sep_off = nullptr;
            o.sep_nodes = nullptr;
            o.list_pairs = nullptr;
        }
        return *this;
    }
    ~PairArrays() { release(); }
    void release()
    {
        std::free(adj);
        std::free(sep_level);
        std::free(sep_kind);
        std::free(sep_off);
        std::free(sep_nodes);
        std::free(list_pairs);
        adj = nullptr;
        sep_level = nullptr;
        sep_kind = nullptr;
        sep_off = nullptr;
        sep_nodes = nullptr;
        list_pairs = nullptr;
    }
};

struct Run {
    fpc_ctx *ctx;
    const fpc_params *P;
    int p, n;
    double q;
    bool mixed;
    const double *C64 = nullptr;
    const float *C32 = nullptr;
    double c_err = 0.0;
    std::vector<uint8_t> adj;
    SepStore sep;
    std::vector<fpc_level_stats> levels;
    int64_t spent_possible = 0;
    int64_t total_exec = 0;
    bool learned = false, logging = false;
    const double *Rfirst = nullptr;  // first-level partial correlations (device)
    std::vector<float> log_x;
    std::vector<uint8_t> log_y;
    std::vector<int32_t> log_group, log_level;
    int32_t log_serial = 0;
    int32_t next_level = -1;  // stopped at a level boundary: the level to continue with
    // the mixed form's FP32 matrix queued behind the first level, not yet
    // waited for (its error measure c_err is read before the first subset level)
    bool c32_pending = false;
    const void *X = nullptr;
    int x_dtype = 0;
    // the correlation's flag words not yet read (they come back with the
    // first level's results), and its device time
    bool corr_flags_pending = false;
    double corr_dev_ms = 0.0;
    // the result's per-pair arrays, filled ahead while the device runs the
    // last levels (valid while ahead_ok: the graph and sets have not changed
    // since), and the arrays allocated ahead by a helper thread
    PairArrays ahead;
    bool ahead_ok = false;
    ResultPrefetch *prefetch = nullptr;
};

int fill_pairs(Run &R, ResultPrefetch *pre, PairArrays &A);

// Runs fn(k) for k in [0, n) on the library's host threads.
template <class F>
void parallel_for(int n, F &&fn)
{
    host_parallel(n, std::function<void(int)>(fn));
}

// The learned order can only save tests of edges deleted at a level, and
// its passes (features, scores, reorder) cost about as much as a few dozen
// tests per candidate; a level with fewer possible tests per candidate than
// this (l <= 2 on the benchmark graphs) keeps the lexicographic order.  The
// skeleton does not depend on the order.
constexpr int64_t kLearnedMinTestsPerCand = 32;

// One level of one or more instances, each on its frozen graph with
// precomputed candidate sets, from its planning to its results: planned
// (eligible edges and test counts), built (records and lists in pinned
// memory), uploaded, launched, then, after the stream has passed its work,
// counted and decoded (every instance's deletions applied at once).  The
// learned order and feature logging are available for a single instance
// only.
struct LevelJob {
    struct Chunk {
        int k;
        int64_t e0, e1;         // edges [e0, e1) of instance k's candidate sets
        int64_t n_el = 0, n_cd = 0, possible = 0;
        int max_m = 0, sel_m = 0;
        bool bad = false;       // the level's test count overflows
        bool too_long = false;  // a list of kBinomRows candidates or more
        int64_t c = 0;          // first list slot (pass 2)
    };
    int l = 0;
    std::vector<Chunk> chunks;
    bool few = false;  // few enough chunks for the calling thread alone
    std::vector<fpc_level_stats> sts;
    int64_t E = 0, T = 0;  // eligible edges and their list entries
    int sel_max_m = 0;
    // records and lists (pinned, ctx->h_stage, uploaded in one piece),
    // counters and deletions (pinned, ctx->h_back, copied back in one piece):
    // byte offsets of this level's regions
    size_t stage_off = 0, back_off = 0;
    EdgeRec *hrec = nullptr;
    int32_t *cand = nullptr;  // the lists, in instance order
    const EdgeRec *recs = nullptr;  // the records as launched (hrec, read back by the host)
    std::vector<int64_t> ntests, cs_edge;  // cs_edge: edge index of each record in its candidate sets
    std::vector<LevelClass> classes;
    std::vector<LevelInst> insts;
    std::vector<float> hfeat;
    const int32_t *d_cand = nullptr;
    bool reorder = false, logging = false, fp32 = false;
    int64_t qcap = 0;
    size_t n_cnt = 0;
    // pinned copy of the device counters: n_cnt counters ([2]: deletions),
    // then the deletions as (edge, rank) pairs
    unsigned long long *cnt = nullptr;
    LevelLaunch Lv{};
    LevelTiming tm;
    const LevelEvents *events = nullptr;  // NULL: the context's
    size_t inst_off = 0;
    double t0 = 0, t_build = 0, t_copy = 0, t_order = 0, t_bufs = 0, t_tests0 = 0, t_tests1 = 0;
    double t_level0 = 0;  // start of the interval reported as level_ms
    double prev_all_ms = 0, prev_test_ms = 0;  // device time of discarded attempts
    int prev_launches = 0;

    size_t stage_bytes() const { return sizeof(EdgeRec) * (size_t)E + sizeof(int32_t) * (size_t)(T + 1); }
    size_t back_bytes() const { return sizeof(unsigned long long) * (n_cnt + 2 * (size_t)E); }
    template <class F>
    void for_chunks(F &&fn)
    {
        if (few)
            for (int u = 0; u < (int)chunks.size(); ++u) fn(u);
        else
            parallel_for((int)chunks.size(), fn);
    }
};

// Pass 1: eligible edges, list lengths and test counts per chunk of each
// instance's edges (chunks keep one instance on many host threads).  Checks
// the test budget without spending it.
int job_plan(const std::vector<Run *> &runs, int l, const std::vector<const CandSets *> &css, LevelJob &J)
{
    const int ni = (int)runs.size();
    J.l = l;
    J.sts.assign(ni, fpc_level_stats{});
    J.n_cnt = 8 + 2 * (size_t)ni;
    constexpr int64_t kEdgeChunk = 1024;
    for (int k = 0; k < ni; ++k) {
        J.sts[k].level = l;
        const int64_t Eall = (int64_t)css[k]->ei.size();
        for (int64_t e0 = 0; e0 < Eall; e0 += kEdgeChunk)
            J.chunks.push_back(LevelJob::Chunk{k, e0, std::min(Eall, e0 + kEdgeChunk)});
    }
    // a level of a few thousand edges runs on the calling thread: waking the
    // pool costs more than the work
    J.few = J.chunks.size() <= 4;
    J.for_chunks([&](int u) {
        LevelJob::Chunk &ch = J.chunks[u];
        const CandSets &cs = *css[ch.k];
        for (int64_t e = ch.e0; e < ch.e1; ++e) {
            const int m = (int)(cs.off[e + 1] - cs.off[e]);
            ch.max_m = std::max(ch.max_m, m);
            if (m < l) continue;
            if (m >= kBinomRows) {
                ch.too_long = true;
                return;
            }
            const int64_t N = binom_sat(m, l);
            if (N == INT64_MAX || ch.possible > INT64_MAX - N) {
                ch.bad = true;
                return;
            }
            ch.possible += N;
            ++ch.n_el;
            ch.n_cd += m;
            ch.sel_m = std::max(ch.sel_m, m);
        }
    });
    for (LevelJob::Chunk &ch : J.chunks) {  // in instance order, so each instance's records stay together
        if (ch.too_long) return FPC_ETOOLARGE;
        if (ch.bad) return FPC_EBUDGET;
        fpc_level_stats &st = J.sts[ch.k];
        st.max_cand = std::max(st.max_cand, ch.max_m);
        st.edges_eligible += ch.n_el;
        if (ch.possible > INT64_MAX - st.tests_possible) return FPC_EBUDGET;
        st.tests_possible += ch.possible;
        ch.c = J.T;
        J.E += ch.n_el;
        J.T += ch.n_cd;
        J.sel_max_m = std::max(J.sel_max_m, ch.sel_m);
    }
    for (int k = 0; k < ni; ++k) {
        const Run &R = *runs[k];
        if (R.P->max_tests > 0 && R.spent_possible + J.sts[k].tests_possible > R.P->max_tests) return FPC_EBUDGET;
    }
    if (J.T > INT32_MAX) return FPC_EBUDGET;
    return FPC_OK;
}

void job_spend(const std::vector<Run *> &runs, const LevelJob &J)
{
    for (size_t k = 0; k < runs.size(); ++k) runs[k]->spent_possible += J.sts[k].tests_possible;
}

// Pass 2: records and lists straight into the job's pinned region (J.hrec,
// J.cand), the records grouped by the size classes of their candidate
// lists: each class is launched with the LDS its own largest list needs, so
// a few long lists do not lower the occupancy (or the kernel choice) of all
// the others.  The records' places come from per-chunk class counts (a
// stable counting sort: within a class, the records keep their instance
// order, so each instance's edges stay together); the lists stay in
// instance order.
void job_build(const std::vector<Run *> &runs, const std::vector<const CandSets *> &css, LevelJob &J)
{
    fpc_ctx *ctx = runs[0]->ctx;
    const int l = J.l;
    const int64_t E = J.E;
    EdgeRec *hrec = J.hrec;
    int32_t *cand = J.cand;
    const bool fp32_cls = runs[0]->mixed && l <= kMaxTemplL;
    std::vector<int> key_of(J.sel_max_m + 1);
    int kmax = 0;
    for (int m = 0; m <= J.sel_max_m; ++m) kmax = std::max(kmax, key_of[m] = level_class_key(ctx, l, fp32_cls, m));
    const int ncls = kmax + 1, nck = (int)J.chunks.size();
    // first record of each (chunk, class): class-major, chunk-minor prefix
    std::vector<int64_t> at((size_t)nck * ncls, 0);
    std::vector<int> cls_max(ncls, 0);
    for (int u = 0; u < nck; ++u) {
        const LevelJob::Chunk &ch = J.chunks[u];
        const CandSets &cs = *css[ch.k];
        int64_t *a = at.data() + (size_t)u * ncls;
        for (int64_t e = ch.e0; e < ch.e1; ++e) {
            const int m = (int)(cs.off[e + 1] - cs.off[e]);
            if (m < l) continue;
            ++a[key_of[m]];
            cls_max[key_of[m]] = std::max(cls_max[key_of[m]], m);
        }
    }
    int64_t run = 0;
    for (int c = 0; c < ncls; ++c) {
        const int64_t begin = run;
        for (int u = 0; u < nck; ++u) {
            const int64_t n = at[(size_t)u * ncls + c];
            at[(size_t)u * ncls + c] = run;
            run += n;
        }
        if (run > begin) J.classes.push_back({begin, run, cls_max[c]});
    }
    J.ntests.resize(E);
    J.cs_edge.resize(E);
    J.for_chunks([&](int u) {
        const LevelJob::Chunk &ch = J.chunks[u];
        const CandSets &cs = *css[ch.k];
        std::vector<int64_t> pos(at.begin() + (size_t)u * ncls, at.begin() + (size_t)(u + 1) * ncls);
        int64_t c = ch.c;
        for (int64_t e = ch.e0; e < ch.e1; ++e) {
            const int m = (int)(cs.off[e + 1] - cs.off[e]);
            if (m < l) continue;
            const int64_t d = pos[key_of[m]]++;
            const int64_t N = binom_sat(m, l);
            hrec[d] = EdgeRec{cs.ei[e], cs.ej[e], m, (int32_t)c, N, ch.k, 0};
            J.ntests[d] = N;
            J.cs_edge[d] = e;
            std::memcpy(cand + c, cs.nodes.data() + cs.off[e], sizeof(int32_t) * m);
            c += m;
        }
    });
    J.recs = hrec;
    J.t_build = now_ms();
}

// Device buffers, the uploads of the job's region of h_stage, the learned
// order's passes and the instance table.
int job_upload(const std::vector<Run *> &runs, const std::vector<const CandSets *> &css, LevelJob &J)
{
    const int ni = (int)runs.size();
    fpc_ctx *ctx = runs[0]->ctx;
    hipStream_t s = ctx->stream;
    const int l = J.l;
    const int64_t E = J.E, T = J.T;
    int rc;
    // the records and the lists after them, as in the staging region
    if ((rc = ctx->edges.ensure(J.stage_bytes()))) return rc;
    if ((rc = ctx->minhit.ensure(sizeof(uint64_t) * E))) return rc;
    if ((rc = ctx->counters.ensure(J.back_bytes()))) return rc;
    if ((rc = upload_enqueue(ctx, ctx->edges.ptr, ctx->h_stage, J.stage_off, sizeof(EdgeRec) * E + sizeof(int32_t) * T)))
        return rc;
    J.t_copy = now_ms();

    // learned order: features, MLP scores, per-edge reorder of the lists
    // (at l = 0 each edge has one subset, so the order cannot matter)
    Run &R0 = *runs[0];
    J.d_cand = reinterpret_cast<const int32_t *>(ctx->edges.as<EdgeRec>() + E);
    J.reorder = ni == 1 && R0.learned && l >= 1 && J.sts[0].tests_possible >= kLearnedMinTestsPerCand * T;
    J.logging = ni == 1 && R0.logging;
    if (J.reorder || J.logging) {
        const CandSets &cs = *css[0];
        std::vector<int32_t> deg(R0.p, 0);  // degrees in the current graph, from its edge list
        for (size_t e = 0; e < cs.ei.size(); ++e) {
            ++deg[cs.ei[e]];
            ++deg[cs.ej[e]];
        }
        if ((rc = ctx->degs.ensure(sizeof(int32_t) * R0.p))) return rc;
        if ((rc = ctx->feat.ensure(sizeof(float) * 4 * (size_t)(T + 1)))) return rc;
        if ((rc = ctx->cand2.ensure(sizeof(int32_t) * (size_t)(T + 1)))) return rc;
        FPC_HIP(hipMemcpyAsync(ctx->degs.ptr, deg.data(), sizeof(int32_t) * R0.p, hipMemcpyHostToDevice, s));
        float *X = ctx->feat.as<float>(), *score = X + 3 * T;
        if ((rc = level_features(ctx, ctx->edges.as<EdgeRec>(), E, J.d_cand, T, R0.C64, R0.Rfirst,
                                 ctx->degs.as<int32_t>(), R0.p, X)))
            return rc;
        if (J.reorder) {
            if ((rc = mlp_forward(ctx, X, T, R0.P->order_model, score))) return rc;
            if ((rc = level_reorder(ctx, ctx->edges.as<EdgeRec>(), E, J.d_cand, score, ctx->cand2.as<int32_t>())))
                return rc;
            J.d_cand = ctx->cand2.as<int32_t>();
        }
        if (J.logging) {
            J.hfeat.resize(3 * (size_t)T);
            // features follow the original order; the reorder maps them
            FPC_HIP(hipMemcpyAsync(J.hfeat.data(), X, sizeof(float) * 3 * T, hipMemcpyDeviceToHost, s));
            FPC_HIP(hipStreamSynchronize(s));
        }
    }
    J.t_order = now_ms();
    J.insts.resize(ni);
    for (int k = 0; k < ni; ++k) {
        const Run &R = *runs[k];
        J.insts[k] = LevelInst{R.C32, R.C64, R.p, R.n, R.q, R.c_err};
    }
    J.fp32 = R0.mixed && l <= kMaxTemplL;
    J.qcap = std::max(ctx->queue_init, (int64_t)(ctx->queue.bytes / (2 * sizeof(int64_t))));
    if (J.fp32 && (rc = ctx->queue.ensure(sizeof(int64_t) * 2 * J.qcap))) return rc;
    J.t_bufs = now_ms();
    return FPC_OK;
}

// Queues the level's tests, the compaction of its hits and the copies of
// its deletions and counters into the job's region of h_back.
int job_launch(const std::vector<Run *> &runs, LevelJob &J)
{
    fpc_ctx *ctx = runs[0]->ctx;
    hipStream_t s = ctx->stream;
    const Run &R0 = *runs[0];
    int rc;
    if ((rc = level_init(ctx, ctx->minhit.as<uint64_t>(), J.E, ctx->counters.as<unsigned long long>(), (int)J.n_cnt)))
        return rc;
    LevelLaunch &Lv = J.Lv;
    Lv = LevelLaunch{};
    Lv.l = J.l;
    Lv.max_m = J.sel_max_m;
    Lv.n_edges = J.E;
    Lv.classes = J.classes.data();
    Lv.n_classes = (int)J.classes.size();
    Lv.edges = ctx->edges.as<EdgeRec>();
    Lv.cand = J.d_cand;
    Lv.insts = J.insts.data();
    Lv.n_insts = (int)runs.size();
    Lv.fp32 = J.fp32;
    Lv.graph = (R0.P->flags & FPC_FLAG_GRAPH) != 0;
    Lv.band_z = R0.P->recheck_margin > 0 ? R0.P->recheck_margin : 1e-3;
    Lv.ill_cond_tau = R0.P->ill_cond_tau;
    Lv.minhit = ctx->minhit.as<uint64_t>();
    Lv.counters = ctx->counters.as<unsigned long long>();
    Lv.inst_cnt = Lv.counters + 8;
    Lv.queue = J.fp32 ? ctx->queue.as<int64_t>() : nullptr;
    Lv.queue_cap = J.fp32 ? J.qcap : 0;
    Lv.events = J.events;
    Lv.inst_off = J.inst_off;
    J.t_tests0 = now_ms();
    if ((rc = level_tests(ctx, Lv, J.ntests, &J.tm))) return rc;
    // the host decodes separating sets against the lists the level used
    // (the uploads that read the staging buffer precede this copy on the stream)
    if (J.reorder && J.T)
        FPC_HIP(hipMemcpyAsync(J.cand, J.d_cand, sizeof(int32_t) * J.T, hipMemcpyDeviceToHost, s));
    if ((rc = level_compact_enqueue(ctx, Lv.minhit, J.E, reinterpret_cast<int64_t *>(Lv.counters + J.n_cnt),
                                    Lv.counters + 2)))
        return rc;
    FPC_HIP(hipMemcpyAsync(J.cnt, Lv.counters, J.back_bytes(), hipMemcpyDeviceToHost, s));
    return FPC_OK;
}

// Test counts of a completed launch (a discarded attempt's tests stay in
// the counts, so its device time stays in the timings).
void job_counts(const std::vector<Run *> &runs, LevelJob &J)
{
    for (size_t k = 0; k < runs.size(); ++k) {
        J.sts[k].tests_executed += (int64_t)J.cnt[8 + 2 * k];
        J.sts[k].tests_rechecked += (int64_t)J.cnt[8 + 2 * k + 1];
        runs[k]->total_exec += (int64_t)J.cnt[8 + 2 * k];
    }
}

// Sepsets and level-end deletion (stable: all of D at once) of a completed
// level, and its statistics.
void job_finish(const std::vector<Run *> &runs, const std::vector<const CandSets *> &css, LevelJob &J)
{
    const int ni = (int)runs.size();
    fpc_ctx *ctx = runs[0]->ctx;
    const int l = J.l;
    const EdgeRec *recs = J.recs;
    const int32_t *cand = J.cand;
    const int64_t ndel = (int64_t)J.cnt[2];
    const int64_t *pairs = reinterpret_cast<const int64_t *>(J.cnt + J.n_cnt);
    std::vector<fpc_level_stats> &sts = J.sts;
    for (int k = 0; k < ni; ++k) sts[k].tests_required = sts[k].tests_possible;
    for (int64_t t = 0; t < ndel; ++t) {
        const EdgeRec &er = recs[pairs[2 * t]];
        sts[er.inst].tests_required -= er.ntests - (pairs[2 * t + 1] + 1);
    }

    const double t_decode = now_ms();
    // each instance's deletions in pair order (the records are in class
    // order; the result lists every set in pair order, so the decoding order
    // is free: deletions are only grouped by instance, and put in pair order
    // for the feature log, whose rows follow it)
    std::vector<std::pair<int64_t, int64_t>> dl(ndel);
    std::vector<int64_t> d_lo(ni + 1, 0);  // deletions of instance k: dl[d_lo[k], d_lo[k+1])
    for (int64_t t = 0; t < ndel; ++t) ++d_lo[recs[pairs[2 * t]].inst + 1];
    for (int k = 0; k < ni; ++k) d_lo[k + 1] += d_lo[k];
    {
        std::vector<int64_t> at(d_lo.begin(), d_lo.end() - 1);
        for (int64_t t = 0; t < ndel; ++t) dl[at[recs[pairs[2 * t]].inst]++] = {pairs[2 * t], pairs[2 * t + 1]};
    }
    if (J.logging)
        std::sort(dl.begin(), dl.end(), [&](const std::pair<int64_t, int64_t> &a, const std::pair<int64_t, int64_t> &b) {
            const EdgeRec &x = recs[a.first], &y = recs[b.first];
            if (x.inst != y.inst) return x.inst < y.inst;
            if (x.i != y.i) return x.i < y.i;
            return x.j < y.j;
        });
    // every deletion owns l slots of its instance's node store and one list
    // entry, so the sets are decoded in parallel chunks
    std::vector<size_t> o0(ni), li0(ni);
    for (int k = 0; k < ni; ++k) {
        Run &R = *runs[k];
        const int64_t nd = d_lo[k + 1] - d_lo[k];
        o0[k] = R.sep.nodes.size();
        li0[k] = R.sep.lists.size();
        R.sep.nodes.resize(o0[k] + (size_t)nd * l);
        R.sep.lists.resize(li0[k] + (size_t)nd);
        sts[k].deleted += nd;
    }
    constexpr int64_t kChunk = 512;
    std::vector<std::pair<int, int64_t>> dchunks;  // (instance, first deletion)
    for (int k = 0; k < ni; ++k)
        for (int64_t t = d_lo[k]; t < d_lo[k + 1]; t += kChunk) dchunks.emplace_back(k, t);
    parallel_for((int)dchunks.size(), [&](int c) {
        const int k = dchunks[c].first;
        Run &R = *runs[k];
        std::vector<int> pos;
        const int64_t t1 = std::min(d_lo[k + 1], dchunks[c].second + kChunk);
        for (int64_t t = dchunks[c].second; t < t1; ++t) {
            const auto &d = dl[t];
            const EdgeRec &er = recs[d.first];
            unrank_host(d.second, er.m, l, ctx->binomT_host, pos);
            const int64_t pr = pair_index(er.i, er.j, R.p);
            const size_t o = o0[k] + (size_t)(t - d_lo[k]) * l;
            R.sep.lists[li0[k] + (size_t)(t - d_lo[k])] = {pr, (int64_t)o, l};
            int32_t *S = R.sep.nodes.data() + o;
            for (int q = 0; q < l; ++q) S[q] = cand[er.cand_off + pos[q]];
            std::sort(S, S + l);
            R.adj[(size_t)er.i * R.p + er.j] = R.adj[(size_t)er.j * R.p + er.i] = 0;
        }
    });
    if (J.logging) {
        // features were computed over the list sorted by id (the cs order)
        Run &R = *runs[0];
        const CandSets &cs = *css[0];
        for (int64_t t = 0; t < ndel; ++t) {
            const EdgeRec &er = recs[dl[t].first];
            const int32_t *orig = cs.nodes.data() + cs.off[J.cs_edge[dl[t].first]];
            const int32_t *S = R.sep.nodes.data() + o0[0] + (size_t)t * l;
            for (int a2 = 0; a2 < er.m; ++a2) {
                const int v = orig[a2];
                const bool in = std::binary_search(S, S + l, v);
                for (int f = 0; f < 3; ++f) R.log_x.push_back(J.hfeat[3 * ((size_t)er.cand_off + a2) + f]);
                R.log_y.push_back(in ? 1 : 0);
                R.log_group.push_back(R.log_serial);
                R.log_level.push_back(l);
            }
            ++R.log_serial;
        }
    }
    const double t_end = now_ms();
    if (trace_on())
        std::fprintf(stderr,
                     "[fpc] level %d: %d instance(s) %lld edges %lld candidates %d classes | setup %.2f upload+order "
                     "%.2f (copies %.2f, order %.2f, buffers %.2f) tests and compaction %.2f (device %.2f) counts %.2f "
                     "decode %.2f ms | deleted %lld, queued for FP64 in the last launch %llu\n",
                     l, ni, (long long)J.E, (long long)J.T, (int)J.classes.size(), J.t_build - J.t0,
                     J.t_tests0 - J.t_build, J.t_copy - J.t_build, J.t_order - J.t_copy, J.t_bufs - J.t_order,
                     J.t_tests1 - J.t_tests0, J.tm.all_ms, t_decode - J.t_tests1, t_end - t_decode, (long long)ndel,
                     J.fp32 ? J.cnt[1] : 0ull);
    for (auto &st : sts) {
        st.kernel_ms = J.prev_all_ms + J.tm.all_ms;
        st.test_kernel_ms = J.prev_test_ms + J.tm.test_ms;
        st.test_launches = J.prev_launches + J.tm.test_launches;
        st.level_ms = t_end - J.t_level0;
    }
}

// Runs one level (l >= 0) of one or more instances, each on its frozen
// graph with precomputed candidate sets, in shared launches; applies every
// instance's deletions at the end.
int run_level(const std::vector<Run *> &runs, int l, const std::vector<const CandSets *> &css,
              std::vector<fpc_level_stats> &sts)
{
    fpc_ctx *ctx = runs[0]->ctx;
    hipStream_t s = ctx->stream;
    LevelJob J;
    J.t0 = J.t_level0 = now_ms();
    int rc;
    if ((rc = job_plan(runs, l, css, J))) return rc;
    job_spend(runs, J);
    if (J.E == 0) {
        for (auto &st : J.sts) st.level_ms = now_ms() - J.t0;
        sts = std::move(J.sts);
        return FPC_OK;
    }
    FPC_HIP(hipStreamSynchronize(s));  // the staging buffers are free
    if ((rc = ctx->h_stage.ensure(J.stage_bytes()))) return rc;
    if ((rc = ctx->h_back.ensure(J.back_bytes()))) return rc;
    J.hrec = ctx->h_stage.as<EdgeRec>();
    J.cand = reinterpret_cast<int32_t *>(J.hrec + J.E);
    J.cnt = ctx->h_back.as<unsigned long long>();
    job_build(runs, css, J);
    if ((rc = job_upload(runs, css, J))) return rc;
    for (;;) {
        if ((rc = job_launch(runs, J))) return rc;
        // the deletions are decoded on the host threads: wake them when the
        // level's last launch starts (the start event of the last timed
        // launch), so that they are spinning when the level ends
        if (J.tm.n_events >= 2) FPC_HIP(hipEventSynchronize(J.tm.lev[2 * (J.tm.n_events - 1)]));
        host_wake();
        FPC_HIP(hipStreamSynchronize(s));  // the one wait of the level
        J.t_tests1 = now_ms();
        if ((rc = level_timing(ctx, &J.tm))) return rc;
        job_counts(runs, J);
        if (!J.cnt[3]) break;
        // the recheck queue overflowed: run the whole level again
        J.prev_all_ms += J.tm.all_ms;
        J.prev_test_ms += J.tm.test_ms;
        J.prev_launches += J.tm.test_launches;
        const int64_t grown = std::min(J.qcap * 4, ctx->queue_max);
        if (grown > J.qcap && ctx->queue.ensure(sizeof(int64_t) * 2 * grown) == FPC_OK) {
            J.qcap = grown;
        } else {
            J.fp32 = false;
        }
        if (trace_on())
            std::fprintf(stderr, "[fpc] level %d: recheck queue overflow, level re-run %s\n", l,
                         J.fp32 ? "with a 4x queue" : "in FP64");
    }
    job_finish(runs, css, J);
    sts = std::move(J.sts);
    return FPC_OK;
}

// Up to max_len small levels l_top, l_top - 1, ... of one instance on one
// unchanged graph, queued back to back with one wait for all of them.
// Level l - 1 runs on the graph that level l leaves, so its results hold
// only if level l deleted nothing: the levels are taken in order up to and
// including the first one that deletes an edge, and the rest are dropped
// (their tests counted nowhere).  A level whose recheck queue overflowed is
// dropped with those after it, for the caller to run on its own.
//
// *n_queued = 0: level l_top is not a small level (or the call takes one
// level at a time), nothing was queued; *n_taken = 0: nothing taken.  Else
// the levels taken are appended to out, *next_l is the level to run next and
// *changed whether the graph changed.
int run_chain(Run &R, int l_top, const CandSets &cs, int max_len, std::vector<fpc_level_stats> &out,
              int *n_queued, int *n_taken, int *next_l, bool *changed)
{
    // a level with at most this many possible tests takes at most a few
    // dozen microseconds on the device, less than a host round trip
    constexpr int64_t kChainMaxTests = int64_t(1) << 24;
    fpc_ctx *ctx = R.ctx;
    hipStream_t s = ctx->stream;
    const std::vector<Run *> runs{&R};
    const std::vector<const CandSets *> css{&cs};
    *n_taken = *n_queued = 0;
    const double t_start = now_ms();
    std::vector<LevelJob> jobs;
    jobs.reserve(fpc_ctx::kChainSlots);
    // the budget, the stop after a number of levels, feature logging and
    // captured levels take one level at a time, and so does a level that the
    // learned order reorders (the same test as in job_upload)
    const fpc_params *P = R.P;
    if (P->max_tests > 0 || P->stop_after_levels > 0 || R.logging || (P->flags & FPC_FLAG_GRAPH)) return FPC_OK;
    int64_t total = 0;
    for (int l = l_top; l >= 0 && (int)jobs.size() < std::min(max_len, fpc_ctx::kChainSlots); --l) {
        LevelJob J;
        J.t0 = now_ms();
        if (job_plan(runs, l, css, J) != FPC_OK || J.E == 0) break;  // such a level runs on its own
        if (R.learned && l >= 1 && J.sts[0].tests_possible >= kLearnedMinTestsPerCand * J.T) break;
        total += J.sts[0].tests_possible;
        if (total > kChainMaxTests) break;
        jobs.push_back(std::move(J));
    }
    if (jobs.empty()) return FPC_OK;
    *n_queued = (int)jobs.size();
    // a run down to level 0 that deletes nothing ends the call: the result's
    // per-pair arrays are filled on a helper thread (with the host threads)
    // while this thread queues the levels and the device runs them, and kept
    // if none of the levels deletes an edge (the levels' results are read
    // only after the helper has finished)
    const bool ahead = R.prefetch && jobs.back().l == 0;
    std::thread filler;
    if (ahead) {
        try {
            filler = std::thread([&R] { R.ahead_ok = fill_pairs(R, R.prefetch, R.ahead) == FPC_OK; });
        } catch (...) {  // no thread: filled before the wait
        }
    }
    struct Joiner {  // every return below waits for the helper
        std::thread &t;
        ~Joiner()
        {
            if (t.joinable()) t.join();
        }
    } joiner{filler};
    int rc;
    if (!ctx->chain_ev_ready) {
        for (auto &slot : ctx->chain_ev)
            for (hipEvent_t &ev : slot)
                if (!ev) FPC_HIP(hipEventCreate(&ev));
        ctx->chain_ev_ready = true;
    }
    // every buffer sized before anything is queued: none may be reallocated
    // while a queued level reads it (the last level has the most edges)
    size_t so = 0, bo = 0, inst_stride = 0;
    int64_t maxE = 0;
    size_t maxStage = 0, maxBack = 0;
    for (LevelJob &J : jobs) {
        J.stage_off = so;
        so += (J.stage_bytes() + 255) / 256 * 256;
        J.back_off = bo;
        bo += (J.back_bytes() + 255) / 256 * 256;
        maxE = std::max(maxE, J.E);
        maxStage = std::max(maxStage, J.stage_bytes());
        maxBack = std::max(maxBack, J.back_bytes());
    }
    FPC_HIP(hipStreamSynchronize(s));  // the staging buffers are free
    if ((rc = level_reserve(ctx, maxE, 1, (int)jobs.size(), &inst_stride))) return rc;
    if ((rc = ctx->h_stage.ensure(so))) return rc;
    if ((rc = ctx->h_back.ensure(bo))) return rc;
    if ((rc = ctx->edges.ensure(maxStage))) return rc;
    if ((rc = ctx->minhit.ensure(sizeof(uint64_t) * maxE))) return rc;
    if ((rc = ctx->counters.ensure(maxBack))) return rc;
    std::vector<LevelEvents> evs(jobs.size());
    for (size_t k = 0; k < jobs.size(); ++k) {
        LevelJob &J = jobs[k];
        evs[k] = LevelEvents{ctx->chain_ev[k][0], ctx->chain_ev[k][1], &ctx->chain_ev[k][2],
                             fpc_ctx::kChainLaunchEvents};
        J.events = &evs[k];
        J.inst_off = inst_stride * k;
        J.hrec = reinterpret_cast<EdgeRec *>(ctx->h_stage.as<char>() + J.stage_off);
        J.cand = reinterpret_cast<int32_t *>(J.hrec + J.E);
        J.cnt = reinterpret_cast<unsigned long long *>(ctx->h_back.as<char>() + J.back_off);
        job_build(runs, css, J);
        if ((rc = job_upload(runs, css, J))) return rc;
        if ((rc = job_launch(runs, J))) return rc;
    }
    host_wake();  // for the decoding and the result that follow
    if (ahead && !filler.joinable()) R.ahead_ok = fill_pairs(R, R.prefetch, R.ahead) == FPC_OK;
    FPC_HIP(hipStreamSynchronize(s));  // the one wait of the chained levels
    if (filler.joinable()) filler.join();
    const double t_done = now_ms();
    if (trace_on())
        std::fprintf(stderr, "[fpc] levels %d..%d queued back to back: %.2f ms to the end of the last\n", jobs[0].l,
                     jobs.back().l, t_done - t_start);
    double t_prev = t_start;
    *next_l = l_top;
    *changed = false;
    for (LevelJob &J : jobs) {
        J.t_tests1 = t_done;
        if ((rc = level_timing(ctx, &J.tm))) return rc;
        if (J.cnt[3]) break;  // recheck queue overflow: the caller runs this level on its own
        job_counts(runs, J);
        job_spend(runs, J);
        J.t_level0 = t_prev;  // the levels' intervals add up to the chain's time
        job_finish(runs, css, J);
        t_prev = now_ms();
        out.push_back(J.sts[0]);
        ++*n_taken;
        *next_l = J.l - 1;
        if (J.sts[0].deleted > 0) {
            *changed = true;
            break;
        }
    }
    // the arrays filled ahead hold only if every level was taken unchanged
    if (*changed || *n_taken < *n_queued) R.ahead_ok = false;
    return FPC_OK;
}

int validate(const fpc_params *P)
{
    if (!P || !P->X) return FPC_EINVAL;
    if (P->p < 2 || P->n <= P->p + 1) return FPC_EINVAL;
    if (P->x_dtype != FPC_F64 && P->x_dtype != FPC_F32) return FPC_EINVAL;
    if (P->precision != FPC_PREC_FP64 && P->precision != FPC_PREC_MIXED) return FPC_EINVAL;
    if (P->schedule != FPC_REVERSE && P->schedule != FPC_FORWARD) return FPC_EINVAL;
    if (P->order != FPC_ORDER_LEX && P->order != FPC_ORDER_LEARNED) return FPC_EINVAL;
    if (P->order == FPC_ORDER_LEARNED && (!P->order_model || P->schedule != FPC_REVERSE)) return FPC_EINVAL;
    if (std::isnan(P->q_override) && !(P->alpha > 0.0 && P->alpha < 1.0)) return FPC_EINVAL;
    if (!std::isnan(P->q_override) && !(P->q_override >= 0.0)) return FPC_EINVAL;
    if (P->max_tests < 0) return FPC_EINVAL;
    if (std::isnan(P->ill_cond_tau)) return FPC_EINVAL;
    if (P->c32_method != 0 && P->c32_method != FPC_CORR_BF16X3 && P->c32_method != FPC_CORR_BF16X6 &&
        P->c32_method != FPC_CORR_FP32)
        return FPC_EINVAL;
    if (P->stop_after_levels < 0) return FPC_EINVAL;
    if (const fpc_checkpoint *ck = P->resume) {
        if (ck->p != P->p || ck->next_level < -1 || ck->next_level > P->p - 3 || ck->n_levels < 0) return FPC_EINVAL;
        if (!ck->adj || !ck->sep_level || !ck->sep_kind || !ck->sep_off || (ck->n_levels && !ck->levels))
            return FPC_EINVAL;
        if (P->flags & FPC_FLAG_LOG_FEATURES) return FPC_EINVAL;
        const int64_t PP = (int64_t)P->p * (P->p - 1) / 2;
        if (ck->sep_off[0] != 0 || (ck->sep_off[PP] > 0 && !ck->sep_nodes)) return FPC_EINVAL;
        for (int64_t k = 0; k < PP; ++k) {
            const int8_t kind = ck->sep_kind[k];
            if (kind != FPC_SEP_NONE && kind != FPC_SEP_LIST && kind != FPC_SEP_ALL_BUT) return FPC_EINVAL;
            if (kind == FPC_SEP_LIST && (ck->sep_level[k] < 0 || ck->sep_off[k + 1] - ck->sep_off[k] != ck->sep_level[k]))
                return FPC_EINVAL;
        }
    }
    return FPC_OK;
}

// The run's state from a level-boundary checkpoint (validated).
void restore_run(Run &R, const fpc_checkpoint *ck)
{
    const int p = R.p;
    std::memcpy(R.adj.data(), ck->adj, (size_t)p * p);
    for (int i = 0; i < p; ++i) R.adj[(size_t)i * p + i] = 0;
    R.sep.reset();
    const int64_t PP = (int64_t)p * (p - 1) / 2;
    for (int64_t k = 0; k < PP; ++k) {
        if (ck->sep_kind[k] != FPC_SEP_LIST) continue;
        const int l = ck->sep_level[k];
        R.sep.lists.push_back(SepList{k, (int64_t)R.sep.nodes.size(), l});
        R.sep.nodes.insert(R.sep.nodes.end(), ck->sep_nodes + ck->sep_off[k], ck->sep_nodes + ck->sep_off[k] + l);
    }
    R.sep.first_level = R.P->schedule == FPC_REVERSE && ck->n_levels > 0 && ck->levels[0].level == p - 2;
    R.levels.assign(ck->levels, ck->levels + ck->n_levels);
    for (const fpc_level_stats &st : R.levels) {
        R.total_exec += st.tests_executed;
        R.spent_possible += st.tests_possible;
    }
}

// Instance state before the levels: the complete graph, no separating sets
// (full_graph false: the adjacency sized only, for a first level that
// writes all of it).
void init_run(Run &R, fpc_ctx *ctx, const fpc_params *P, int p, int n, bool full_graph = true)
{
    R.ctx = ctx;
    R.P = P;
    R.p = p;
    R.n = n;
    R.q = std::isnan(P->q_override) ? normal_quantile_upper(P->alpha) : P->q_override;
    R.mixed = P->precision == FPC_PREC_MIXED;
    R.learned = P->order == FPC_ORDER_LEARNED;
    R.logging = (P->flags & FPC_FLAG_LOG_FEATURES) != 0 && P->schedule == FPC_REVERSE;
    const size_t pp = (size_t)p * p;
    if (full_graph) {
        R.adj.assign(pp, 1);
        for (int i = 0; i < p; ++i) R.adj[(size_t)i * p + i] = 0;
    } else {
        R.adj.resize(pp);
    }
    R.sep.reset();
}

// Correlation matrices of the instance's data (device, n x p row-major):
// FP64 into C64, and in the mixed form the bf16x3 FP32 copy into C32 with
// its largest entry error against C64.
// The mixed form's FP32 matrix and its largest entry error against C64,
// queued on the context's stream.
int c32_enqueue(Run &R, float *C32)
{
    int rc;
    const int m32 = R.P->c32_method ? R.P->c32_method : FPC_CORR_BF16X6;
    if (m32 == FPC_CORR_FP32) {
        if ((rc = corr_round_enqueue(R.ctx, R.C64, C32, R.p, false))) return rc;
    } else if ((rc = corr_compute(R.ctx, R.X, R.x_dtype, R.n, R.p, m32, C32, true, false))) {
        return rc;
    }
    R.C32 = C32;
    return corr_max_abs_diff_enqueue(R.ctx, R.C64, R.C32, R.p);
}

// With defer_c32 (the first level runs next) only C64 is computed and
// checked here; the FP32 matrix is queued behind the first level
// (first_stage) and waited for by c32_finish, so it runs while the host
// builds the first candidate sets.
int corr_stage(Run &R, const void *X, int x_dtype, double *C64, float *C32, double *ms, bool defer_c32,
               bool first_follows = false)
{
    const double t0 = now_ms();
    int rc;
    fpc_ctx *ctx = R.ctx;
    R.X = X;
    R.x_dtype = x_dtype;
    const bool now = R.mixed && !defer_c32;
    // a first level queued next waits for the correlation with its own
    // results: the flag words are copied back then, with no wait here (an
    // event pair times the correlation on the device)
    const bool unchecked = first_follows && !now;
    if (unchecked) FPC_HIP(hipEventRecord(ctx->lev[0], ctx->stream));
    // a deferred product must find its work buffers allocated: growing one
    // behind the first level would free memory that level still uses
    if (R.mixed && defer_c32) {
        const int m32 = R.P->c32_method ? R.P->c32_method : FPC_CORR_BF16X6;
        if ((rc = corr_reserve(R.ctx, R.n, R.p, m32 == FPC_CORR_FP32 ? FPC_CORR_FP64 : m32))) return rc;
    }
    // the products and the error measure queued, then one wait
    if ((rc = corr_compute(R.ctx, X, x_dtype, R.n, R.p, FPC_CORR_FP64, C64, false, false))) return rc;
    R.C64 = C64;
    if (now && (rc = c32_enqueue(R, C32))) return rc;
    if (unchecked) {
        if ((rc = ctx->h_flag.ensure(64))) return rc;
        FPC_HIP(hipEventRecord(ctx->lev[1], ctx->stream));
        FPC_HIP(hipMemcpyAsync(ctx->h_flag.as<char>() + 48, ctx->flag.ptr, 2 * sizeof(int), hipMemcpyDeviceToHost,
                               ctx->stream));
        R.corr_flags_pending = true;
    } else if ((rc = corr_check(R.ctx, now ? &R.c_err : nullptr))) {
        return rc;
    }
    R.c32_pending = R.mixed && defer_c32;
    if (R.c32_pending) R.C32 = C32;
    *ms = unchecked ? 0.0 : now_ms() - t0;  // unchecked: the device time is added after the first level
    return FPC_OK;
}

// Waits for the FP32 matrix queued behind the first level and reads its
// error measure (the wait is added to the correlation time).
int c32_finish(Run &R, double *corr_ms)
{
    if (!R.c32_pending) return FPC_OK;
    const double t0 = now_ms();
    R.c32_pending = false;
    FPC_HIP(hipEventSynchronize(R.ctx->ev_c32));
    const char *h = R.ctx->h_flag.as<char>();
    std::memcpy(&R.c_err, h + 32, sizeof(double));
    int flags[2];
    std::memcpy(flags, h, sizeof(flags));
    if (flags[0]) return FPC_ENONFINITE;
    if (flags[1]) return FPC_ESINGULAR;
    *corr_ms += now_ms() - t0;
    return FPC_OK;
}

// The l = p - 2 level on the complete graph, through Omega = C^{-1}.
// The graph after the first level from its decisions (ind, p x p bytes, 1 =
// independent): adj = not independent, off the diagonal; the decision
// matrix is symmetric, so the deleted pairs are half its ones.
void first_marks(Run &R, const uint8_t *ind, fpc_level_stats &st)
{
    const int p = R.p;
    const size_t pp = (size_t)p * p;
    const int nblk = std::min(p, 16);
    std::vector<int64_t> dels(nblk, 0);
    parallel_for(nblk, [&](int b) {
        const size_t k0 = pp * (size_t)b / nblk, k1 = pp * (size_t)(b + 1) / nblk;
        const uint8_t *__restrict__ src = ind;
        uint8_t *__restrict__ dst = R.adj.data();
        int64_t ones = 0;
        for (size_t k = k0; k < k1; ++k) {
            dst[k] = (uint8_t)(src[k] ^ 1u);
            ones += src[k];
        }
        dels[b] = ones;
    });
    for (int i = 0; i < p; ++i) R.adj[(size_t)i * p + i] = 0;
    R.sep.first_level = true;
    st.deleted = 0;
    for (int64_t d : dels) st.deleted += d;
    st.deleted /= 2;
    R.total_exec += st.tests_executed;
    R.spent_possible += st.tests_possible;
}

// Statistics of a first level (l = p - 2) before its decisions are read.
fpc_level_stats first_level_stats(int p)
{
    fpc_level_stats st{};
    st.level = p - 2;
    st.max_cand = p - 2;
    st.edges_eligible = st.tests_possible = st.tests_executed = st.tests_required = (int64_t)p * (p - 1) / 2;
    return st;
}

int first_stage(Run &R, double *ms)
{
    fpc_ctx *ctx = R.ctx;
    hipStream_t s = ctx->stream;
    const int p = R.p;
    const size_t pp = (size_t)p * p;
    const double t0 = now_ms();
    fpc_level_stats st = first_level_stats(p);
    int rc;
    if ((rc = ctx->flag.ensure(64))) return rc;
    if ((rc = ctx->dellist.ensure(pp))) return rc;
    uint8_t *d_ind = ctx->dellist.as<uint8_t>();
    FPC_HIP(hipEventRecord(ctx->ev0, s));
    double *d_r = nullptr;
    if (R.learned || R.logging) {
        if ((rc = ctx->rfirst.ensure(sizeof(double) * pp))) return rc;
        d_r = ctx->rfirst.as<double>();
        R.Rfirst = d_r;
    }
    const int *d_bad = nullptr;
    if ((rc = first_level_enqueue(ctx, R.C64, p, R.n, R.q, d_r, d_ind, &d_bad))) return rc;
    FPC_HIP(hipEventRecord(ctx->ev1, s));
    // one round trip: the decisions and the positive-definiteness flag
    if ((rc = ctx->h_back.ensure(pp + 64))) return rc;
    const uint8_t *ind = ctx->h_back.as<uint8_t>();
    int *h_bad = reinterpret_cast<int *>(ctx->h_back.as<uint8_t>() + (pp + 15) / 16 * 16);
    FPC_HIP(hipMemcpyAsync(ctx->h_back.ptr, d_ind, pp, hipMemcpyDeviceToHost, s));
    FPC_HIP(hipMemcpyAsync(h_bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    FPC_HIP(hipEventRecord(ctx->ev_first, s));
    if (R.c32_pending) {
        // the FP32 matrix after the first level: it reuses the column
        // statistics and the work buffer the sweep has finished with
        if ((rc = ctx->h_flag.ensure(64))) return rc;
        if ((rc = c32_enqueue(R, const_cast<float *>(R.C32)))) return rc;
        FPC_HIP(hipMemcpyAsync(ctx->h_flag.ptr, ctx->flag.ptr, 40, hipMemcpyDeviceToHost, s));
        FPC_HIP(hipEventRecord(ctx->ev_c32, s));
    }
    const double tq = now_ms();
    host_wake();  // the candidate sets follow on the host threads
    FPC_HIP(hipEventSynchronize(ctx->ev_first));
    const double tw = now_ms();
    if (R.corr_flags_pending) {  // the correlation's flag words (bytes 48..55 of the pinned flag buffer)
        R.corr_flags_pending = false;
        int f[2];
        std::memcpy(f, ctx->h_flag.as<char>() + 48, sizeof(f));
        if (f[0]) return FPC_ENONFINITE;
        if (f[1]) return FPC_ESINGULAR;
        float cms = 0.f;
        FPC_HIP(hipEventElapsedTime(&cms, ctx->lev[0], ctx->lev[1]));
        R.corr_dev_ms = cms;
    }
    if (*h_bad) return FPC_ESINGULAR;
    float kms = 0.f;
    FPC_HIP(hipEventElapsedTime(&kms, ctx->ev0, ctx->ev1));
    st.kernel_ms = kms;
    first_marks(R, ind, st);
    *ms = now_ms() - t0;
    if (trace_on())
        std::fprintf(stderr, "[fpc] first level: queue %.2f wait %.2f (device %.2f) marks %.2f ms\n", tq - t0, tw - tq,
                     kms, now_ms() - tw);
    st.level_ms = *ms;
    R.levels.push_back(st);
    return FPC_OK;
}

// The first level's partial correlations (K = all but i, j) into ctx->rfirst
// without its decisions: the learned order's features on a resumed run.
int first_level_r(Run &R)
{
    fpc_ctx *ctx = R.ctx;
    int rc;
    if ((rc = ctx->rfirst.ensure(sizeof(double) * (size_t)R.p * R.p))) return rc;
    const int *d_bad = nullptr;
    if ((rc = first_level_enqueue(ctx, R.C64, R.p, R.n, R.q, ctx->rfirst.as<double>(), nullptr, &d_bad))) return rc;
    FPC_HIP(hipStreamSynchronize(ctx->stream));
    int h_bad = 0;
    FPC_HIP(hipMemcpy(&h_bad, d_bad, sizeof(int), hipMemcpyDeviceToHost));
    if (h_bad) return FPC_ESINGULAR;
    R.Rfirst = ctx->rfirst.as<double>();
    return FPC_OK;
}

int largest_cand(const CandSets &cs)
{
    int mmax = -1;
    for (size_t e = 0; e + 1 < cs.off.size(); ++e) mmax = std::max<int>(mmax, (int)(cs.off[e + 1] - cs.off[e]));
    return mmax;
}

// The per-pair arrays of a result (adjacency, separating-set level, kind and
// offset: 7.5 MB at p = 1000), allocated and first-touched on a helper
// thread while the device runs the call, so that assembling the result does
// not pay the page faults of fresh memory on the call's path.
class ResultPrefetch {
  public:
    explicit ResultPrefetch(int p) : p_(p)
    {
        try {
            th_ = std::thread([this] { fill(); });
        } catch (...) {  // no thread: the result allocates its arrays itself
        }
    }
    ~ResultPrefetch()
    {
        join();
        std::free(adj_);
        std::free(sep_level_);
        std::free(sep_kind_);
        std::free(sep_off_);
    }
    // Hands the arrays over (all four or none) to the caller, who frees them.
    bool take(uint8_t *&adj, int32_t *&sep_level, int8_t *&sep_kind, int64_t *&sep_off)
    {
        join();
        if (!adj_) return false;
        adj = adj_;
        sep_level = sep_level_;
        sep_kind = sep_kind_;
        sep_off = sep_off_;
        adj_ = nullptr;
        sep_level_ = nullptr;
        sep_kind_ = nullptr;
        sep_off_ = nullptr;
        return true;
    }

  private:
    void join()
    {
        if (th_.joinable()) th_.join();
    }
    void fill()
    {
        const size_t pp = (size_t)p_ * p_;
        const size_t PP = (size_t)p_ * (p_ - 1) / 2;
        uint8_t *a = (uint8_t *)std::malloc(pp);
        int32_t *l = (int32_t *)std::malloc(sizeof(int32_t) * PP);
        int8_t *k = (int8_t *)std::malloc(PP);
        int64_t *o = (int64_t *)std::malloc(sizeof(int64_t) * (PP + 1));
        if (!a || !l || !k || !o) {
            std::free(a);
            std::free(l);
            std::free(k);
            std::free(o);
            return;
        }
        std::memset(a, 0, pp);
        std::memset(l, 0, sizeof(int32_t) * PP);
        std::memset(k, 0, PP);
        std::memset(o, 0, sizeof(int64_t) * (PP + 1));
        adj_ = a;
        sep_level_ = l;
        sep_kind_ = k;
        sep_off_ = o;
    }
    int p_;
    std::thread th_;
    uint8_t *adj_ = nullptr;
    int32_t *sep_level_ = nullptr;
    int8_t *sep_kind_ = nullptr;
    int64_t *sep_off_ = nullptr;
};

// Fills A (its arrays reused if allocated, else those of the prefetch,
// else new ones) from the run's graph and separating sets: per pair the
// subset level's set, else the first level's deletion (absent from the
// graph), else kept; row blocks on the host threads, each writing its
// pairs' entries and its share of the set nodes.
int fill_pairs(Run &R, ResultPrefetch *pre, PairArrays &A)
{
    const int p = R.p;
    const size_t pp = (size_t)p * p;
    const int64_t PP = (int64_t)p * (p - 1) / 2;
    if (!A.adj) {
        if (!pre || !pre->take(A.adj, A.sep_level, A.sep_kind, A.sep_off)) {
            A.adj = (uint8_t *)std::malloc(pp);
            A.sep_level = (int32_t *)std::malloc(sizeof(int32_t) * PP);
            A.sep_kind = (int8_t *)std::malloc(PP);
            A.sep_off = (int64_t *)std::malloc(sizeof(int64_t) * (PP + 1));
        }
    }
    std::free(A.sep_nodes);
    std::free(A.list_pairs);
    const int64_t tot = (int64_t)R.sep.nodes.size();
    A.sep_nodes = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(tot, 1));
    A.n_lists = (int64_t)R.sep.lists.size();
    A.list_pairs = (int64_t *)std::malloc(sizeof(int64_t) * (size_t)std::max<int64_t>(A.n_lists, 1));
    if (!A.adj || !A.sep_level || !A.sep_kind || !A.sep_off || !A.sep_nodes || !A.list_pairs) {
        A.release();
        return FPC_ENOMEM;
    }
    std::sort(R.sep.lists.begin(), R.sep.lists.end(),
              [](const SepList &a, const SepList &b) { return a.pair < b.pair; });
    const int nblk = std::max(1, std::min(p, 16));
    std::vector<int> row0(nblk + 1, p);  // rows of block b: [row0[b], row0[b+1]), about PP / nblk pairs each
    {
        int64_t acc = 0;
        int b = 0;
        row0[0] = 0;
        for (int i = 0; i < p && b + 1 < nblk; ++i) {
            acc += p - 1 - i;
            if (acc * nblk >= PP * (b + 1)) row0[++b] = i + 1;
        }
        for (++b; b < nblk; ++b) row0[b] = p;
    }
    auto first_pair = [&](int i) { return i < p - 1 ? pair_index(i, i + 1, p) : PP; };  // first pair of row i on
    std::vector<size_t> li_lo(nblk + 1);
    std::vector<int64_t> node_lo(nblk + 1, 0);
    for (int b = 0; b <= nblk; ++b) {
        const int64_t pr0 = b < nblk ? first_pair(row0[b]) : PP;
        li_lo[b] = (size_t)(std::lower_bound(R.sep.lists.begin(), R.sep.lists.end(), pr0,
                                             [](const SepList &a, int64_t v) { return a.pair < v; }) -
                            R.sep.lists.begin());
    }
    for (int b = 0; b < nblk; ++b) {
        int64_t nn = 0;
        for (size_t t = li_lo[b]; t < li_lo[b + 1]; ++t) nn += R.sep.lists[t].level;
        node_lo[b + 1] = node_lo[b] + nn;
    }
    const bool implicit_first = R.sep.first_level;
    const int first_l = p - 2;
    parallel_for(nblk, [&](int b) {
        std::memcpy(A.adj + (size_t)row0[b] * p, R.adj.data() + (size_t)row0[b] * p,
                    (size_t)(row0[b + 1] - row0[b]) * p);
        size_t li = li_lo[b];
        int64_t o = node_lo[b];
        for (int i = row0[b]; i < row0[b + 1]; ++i) {
            const uint8_t *arow = R.adj.data() + (size_t)i * p;
            const int64_t base = first_pair(i) - (i + 1);  // pair (i, j) at base + j
            for (int j = i + 1; j < p; ++j) {
                const int64_t k = base + j;
                A.sep_off[k] = o;
                if (li < li_lo[b + 1] && R.sep.lists[li].pair == k) {
                    const SepList &e = R.sep.lists[li++];
                    A.sep_level[k] = e.level;
                    A.sep_kind[k] = FPC_SEP_LIST;
                    std::memcpy(A.sep_nodes + o, R.sep.nodes.data() + e.off, sizeof(int32_t) * e.level);
                    o += e.level;
                } else if (!arow[j] && implicit_first) {
                    A.sep_level[k] = first_l;
                    A.sep_kind[k] = FPC_SEP_ALL_BUT;
                } else {
                    A.sep_level[k] = -1;
                    A.sep_kind[k] = FPC_SEP_NONE;
                }
            }
        }
    });
    A.sep_off[PP] = node_lo[nblk];
    for (size_t t = 0; t < R.sep.lists.size(); ++t) A.list_pairs[t] = R.sep.lists[t].pair;
    return FPC_OK;
}

int assemble(Run &R, double corr_ms, double first_ms, double t_start, fpc_result **out,
             ResultPrefetch *pre = nullptr)
{
    const int p = R.p;
    fpc_result *res = (fpc_result *)std::calloc(1, sizeof(fpc_result));
    if (!res) return FPC_ENOMEM;
    res->p = p;
    res->n_levels = (int32_t)R.levels.size();
    if (!R.ahead_ok) {
        const int rc = fill_pairs(R, pre, R.ahead);
        if (rc) {
            std::free(res);
            return rc;
        }
    }
    PairArrays A = std::move(R.ahead);
    R.ahead_ok = false;
    res->adj = A.adj;
    res->sep_level = A.sep_level;
    res->sep_kind = A.sep_kind;
    res->sep_off = A.sep_off;
    res->sep_nodes = A.sep_nodes;
    res->list_pairs = A.list_pairs;
    res->n_lists = A.n_lists;
    A.adj = nullptr;
    A.sep_level = nullptr;
    A.sep_kind = nullptr;
    A.sep_off = nullptr;
    A.sep_nodes = nullptr;
    A.list_pairs = nullptr;
    res->levels = (fpc_level_stats *)std::malloc(sizeof(fpc_level_stats) * std::max<size_t>(R.levels.size(), 1));
    if (!res->levels) {
        fpc_result_free(res);
        return FPC_ENOMEM;
    }
    std::memcpy(res->levels, R.levels.data(), sizeof(fpc_level_stats) * R.levels.size());
    res->total_tests = R.total_exec;
    res->q = R.q;
    res->corr_ms = corr_ms;
    res->first_level_ms = first_ms;
    res->corr_max_abs_err = R.c_err;
    res->log_rows = (int64_t)R.log_y.size();
    if (res->log_rows) {
        res->log_x = (float *)std::malloc(sizeof(float) * R.log_x.size());
        res->log_y = (uint8_t *)std::malloc(R.log_y.size());
        res->log_group = (int32_t *)std::malloc(sizeof(int32_t) * R.log_group.size());
        res->log_level = (int32_t *)std::malloc(sizeof(int32_t) * R.log_level.size());
        if (!res->log_x || !res->log_y || !res->log_group || !res->log_level) {
            fpc_result_free(res);
            return FPC_ENOMEM;
        }
        std::memcpy(res->log_x, R.log_x.data(), sizeof(float) * R.log_x.size());
        std::memcpy(res->log_y, R.log_y.data(), R.log_y.size());
        std::memcpy(res->log_group, R.log_group.data(), sizeof(int32_t) * R.log_group.size());
        std::memcpy(res->log_level, R.log_level.data(), sizeof(int32_t) * R.log_level.size());
    }
    res->next_level = R.next_level;
    res->total_ms = now_ms() - t_start;
    *out = res;
    return FPC_OK;
}

int skeleton_impl(fpc_ctx *ctx, const fpc_params *P, fpc_result **out)
{
    const double t_start = now_ms();
    int rc = validate(P);
    if (rc) return rc;
    FPC_HIP(hipSetDevice(ctx->device));
    ctx->use_pair_kernel = !(P->flags & FPC_FLAG_PER_TEST_KERNEL);
    const int p = P->p, n = P->n;
    ResultPrefetch pre(p);
    const size_t pp = (size_t)p * p;
    hipStream_t s = ctx->stream;
    Run R;
    // the adjacency buffer is kept by the calling thread across calls; a
    // call that runs the first level writes all of it there, so it is
    // neither allocated nor filled before the correlation is queued
    thread_local std::vector<uint8_t> adj_kept;
    R.adj.swap(adj_kept);
    struct AdjBack {
        std::vector<uint8_t> &kept;
        Run &R;
        ~AdjBack() { kept.swap(R.adj); }
    } adj_back{adj_kept, R};
    init_run(R, ctx, P, p, n, !(P->schedule == FPC_REVERSE && !P->resume));
    R.prefetch = &pre;

    // data on the device
    const void *X = P->X;
    if (!P->x_on_device) {
        const size_t bytes = (size_t)n * p * (P->x_dtype == FPC_F64 ? 8 : 4);
        if ((rc = ctx->x_copy.ensure(bytes))) return rc;
        FPC_HIP(hipMemcpyAsync(ctx->x_copy.ptr, P->X, bytes, hipMemcpyHostToDevice, s));
        X = ctx->x_copy.ptr;
    }
    double corr_ms = 0.0, first_ms = 0.0;
    if ((rc = ctx->c64.ensure(sizeof(double) * pp))) return rc;
    if (R.mixed && (rc = ctx->c32.ensure(sizeof(float) * pp))) return rc;
    // the FP32 matrix is deferred behind the first level when that level runs
    const bool first_follows = P->schedule == FPC_REVERSE && !P->resume;
    const bool defer_c32 = R.mixed && first_follows;
    if ((rc = corr_stage(R, X, P->x_dtype, ctx->c64.as<double>(), ctx->c32.as<float>(), &corr_ms, defer_c32,
                         first_follows)))
        return rc;

    const int cap = P->max_level;
    // kept by the calling thread across calls: the lists of a p = 1000 graph
    // take 1.5 MB, whose allocation and zero fill cost 0.1-0.2 ms per call
    thread_local CandSets cs_kept;
    CandSets &cs = cs_kept;
    const std::vector<Run *> one_run{&R};
    const std::vector<const CandSets *> one_cs{&cs};
    // a call stopped by stop_after_levels ends at a level boundary and
    // reports the level it would run next (see fpc_checkpoint)
    int levels_run = 0;
    const int stop = P->stop_after_levels;
    const fpc_checkpoint *ck = P->resume;
    if (ck) restore_run(R, ck);
    if (P->schedule == FPC_REVERSE) {
        int l;
        if (ck) {
            if (R.learned && (rc = first_level_r(R))) return rc;
            l = ck->next_level;
        } else {
            if ((rc = first_stage(R, &first_ms))) return rc;
            // the first level's wait covered the correlation's device time
            corr_ms += R.corr_dev_ms;
            first_ms = std::max(0.0, first_ms - R.corr_dev_ms);
            ++levels_run;
            // following levels: l = min(p-3, cap, largest candidate set), down to 0
            l = p - 3;
            if (cap >= 0) l = std::min(l, cap);
        }
        bool cs_valid = false;  // the graph is unchanged since cs was computed
        int chain_len = fpc_ctx::kChainSlots;  // small levels queued at once
        while (l >= 0) {
            const double tc = now_ms();
            if (!cs_valid) candidate_sets(R.adj.data(), p, cs);
            if (trace_on())
                std::fprintf(stderr, "[fpc] candidate sets: %zu edges, %.2f ms%s\n", cs.ei.size(), now_ms() - tc,
                             cs_valid ? " (unchanged graph)" : "");
            const int mmax = largest_cand(cs);
            if (mmax < 0) break;  // no edges left
            l = std::min(l, mmax);
            if (stop > 0 && levels_run >= stop) {
                R.next_level = l;
                break;
            }
            if ((rc = c32_finish(R, &corr_ms))) return rc;
            std::vector<fpc_level_stats> lv;
            int queued = 0, taken = 0, next_l = l;
            bool changed = false;
            if ((rc = run_chain(R, l, cs, chain_len, lv, &queued, &taken, &next_l, &changed))) return rc;
            if (taken > 0) {  // small levels queued back to back
                R.levels.insert(R.levels.end(), lv.begin(), lv.end());
                levels_run += taken;
                cs_valid = !changed;
                l = next_l;
                // the run length follows the small levels' deletions: a run
                // cut by a deletion at its k-th level is k long next time
                // (1: one level at a time), one taken whole is twice as long
                if (changed) chain_len = taken;
                else if (taken == queued) chain_len = std::min(2 * chain_len, (int)fpc_ctx::kChainSlots);
                continue;
            }
            if ((rc = run_level(one_run, l, one_cs, lv))) return rc;
            R.levels.push_back(lv[0]);
            ++levels_run;
            cs_valid = lv[0].deleted == 0;
            --l;
        }
    } else {
        // Algorithm 1: l = 0, 1, ... while some edge has |cand| >= l
        for (int l = ck ? ck->next_level : 0; l >= 0; ++l) {
            if (cap >= 0 && l > cap) break;
            candidate_sets(R.adj.data(), p, cs);
            if (largest_cand(cs) < l) break;
            if (stop > 0 && levels_run >= stop) {
                R.next_level = l;
                break;
            }
            std::vector<fpc_level_stats> lv;
            if ((rc = run_level(one_run, l, one_cs, lv))) return rc;
            R.levels.push_back(lv[0]);
            ++levels_run;
        }
    }
    if ((rc = c32_finish(R, &corr_ms))) return rc;
    const double ta = now_ms();
    rc = assemble(R, corr_ms, first_ms, t_start, out, &pre);
    if (trace_on())
        std::fprintf(stderr, "[fpc] correlation %.2f ms, first level %.2f ms, result %.2f ms, total %.2f ms\n", corr_ms,
                     first_ms, now_ms() - ta, now_ms() - t_start);
    return rc;
}

int validate_batch(const fpc_params *P, int ni, const fpc_instance *inst)
{
    if (!P || ni < 1 || !inst) return FPC_EINVAL;
    if (P->x_dtype != FPC_F64 && P->x_dtype != FPC_F32) return FPC_EINVAL;
    if (P->precision != FPC_PREC_FP64 && P->precision != FPC_PREC_MIXED) return FPC_EINVAL;
    if (P->schedule != FPC_REVERSE || P->order != FPC_ORDER_LEX) return FPC_EINVAL;
    if (P->flags & FPC_FLAG_LOG_FEATURES) return FPC_EINVAL;
    if (P->stop_after_levels != 0 || P->resume) return FPC_EINVAL;
    if (std::isnan(P->q_override) && !(P->alpha > 0.0 && P->alpha < 1.0)) return FPC_EINVAL;
    if (!std::isnan(P->q_override) && !(P->q_override >= 0.0)) return FPC_EINVAL;
    if (P->max_tests < 0) return FPC_EINVAL;
    if (std::isnan(P->ill_cond_tau)) return FPC_EINVAL;
    if (P->c32_method != 0 && P->c32_method != FPC_CORR_BF16X3 && P->c32_method != FPC_CORR_BF16X6 &&
        P->c32_method != FPC_CORR_FP32)
        return FPC_EINVAL;
    for (int k = 0; k < ni; ++k) {
        const fpc_instance &I = inst[k];
        if (!I.X || I.p < 2 || I.n <= I.p + 1 || I.x_rows < 1) return FPC_EINVAL;
        if (!I.rows && I.x_rows < I.n) return FPC_EINVAL;
    }
    return FPC_OK;
}

// FPC_FLAG_GRAPH: the whole batch on the device in one captured graph
// (batch_graph.hip), then the results assembled as the host-driven batch
// would.  kGraphFallback: the call takes the host-driven path.
int skeleton_batch_device(fpc_ctx *ctx, const fpc_params *P, int ni, const fpc_instance *inst, fpc_result **outs,
                          double t_start)
{
    GraphBatchOut g;
    int rc = skeleton_batch_graph(ctx, P, ni, inst, g);
    if (rc) return rc;
    if (trace_on())
        std::fprintf(stderr,
                     "[fpc] batch of %d as one graph: device %.2f ms, call %.2f ms (prepare %.2f, capture %.2f, "
                     "instantiate %.2f, launch to results %.2f)\n",
                     ni, g.graph_ms, g.total_ms, g.prep_ms, g.capture_ms, g.instantiate_ms, g.run_ms);
    for (int k = 0; k < ni; ++k) {
        GraphBatchOut::Inst &o = g.inst[k];
        Run R;
        init_run(R, ctx, P, inst[k].p, inst[k].n);
        R.adj.swap(o.adj);
        R.c_err = o.c_err;
        R.sep.first_level = true;
        R.sep.nodes.swap(o.sep_nodes);
        R.sep.lists.resize(o.sep_pair.size());
        for (size_t t = 0; t < o.sep_pair.size(); ++t)
            R.sep.lists[t] = SepList{o.sep_pair[t], o.sep_off[t], o.sep_level[t]};
        R.levels.swap(o.levels);
        for (const fpc_level_stats &st : R.levels) R.total_exec += st.tests_executed;
        if ((rc = assemble(R, 0.0, 0.0, t_start, &outs[k]))) {
            for (int t = 0; t < k; ++t) {
                fpc_result_free(outs[t]);
                outs[t] = nullptr;
            }
            return rc;
        }
    }
    return FPC_OK;
}

// Several instances: correlation and first level one instance after the
// other, then every following level of all instances in shared launches.
// Each instance takes exactly the levels, in the same order, that a run of
// it alone would take: at every step each unfinished instance has a next
// level min(its current level, its largest candidate set), and the
// instances whose next level is the highest of all run it together.
// Correlation and first level of every instance of a batch, queued back to
// back with one wait for all of them.  Every device buffer they share is
// first sized for the largest instance (none may be reallocated while
// queued work reads it); each instance's decisions, flag words and
// positive-definiteness flag land in its own region of the pinned buffer.
// The errors are those of the instances one at a time: the first instance
// (in order) with non-finite data, a constant column or a singular matrix
// gives its error; a resample row out of range gives FPC_EINVAL.
int batch_prelude(fpc_ctx *ctx, const fpc_params *P, int ni, const fpc_instance *inst, char *base,
                  const std::vector<size_t> &off64, const std::vector<size_t> &off32, std::vector<Run> &runs,
                  std::vector<double> &corr_ms, std::vector<double> &first_ms)
{
    hipStream_t s = ctx->stream;
    const bool mixed = P->precision == FPC_PREC_MIXED;
    const int m32 = P->c32_method ? P->c32_method : FPC_CORR_BF16X6;
    const size_t esz = P->x_dtype == FPC_F64 ? 8 : 4;
    constexpr size_t kTail = 64;  // after the decisions: the flag words (40 B), then the first level's flag
    std::vector<size_t> hoff(ni);
    size_t host_bytes = 256, max_pp = 0, max_x = 0;  // [0, 4): the resample error word
    int max_p = 2;
    int rc;
    for (int k = 0; k < ni; ++k) {
        const fpc_instance &I = inst[k];
        const size_t pp = (size_t)I.p * I.p;
        hoff[k] = host_bytes;
        host_bytes += (pp + 255) / 256 * 256 + 256;
        max_pp = std::max(max_pp, pp);
        max_p = std::max(max_p, I.p);
        if (I.rows) max_x = std::max(max_x, esz * (size_t)I.n * I.p);
        if ((rc = corr_reserve(ctx, I.n, I.p, FPC_CORR_FP64))) return rc;
        if (mixed && m32 != FPC_CORR_FP32 && (rc = corr_reserve(ctx, I.n, I.p, m32))) return rc;
    }
    if ((rc = first_level_reserve(ctx, max_p))) return rc;
    if ((rc = ctx->dellist.ensure(max_pp))) return rc;
    if (max_x && (rc = ctx->x_copy.ensure(max_x))) return rc;
    FPC_HIP(hipStreamSynchronize(s));  // the pinned buffer is free
    if ((rc = ctx->h_back.ensure(host_bytes))) return rc;
    char *hb = ctx->h_back.as<char>();
    int *d_rows_bad = ctx->flag.as<int>() + 12;  // bytes 48..51 of the flag words: no other user
    FPC_HIP(hipMemsetAsync(d_rows_bad, 0, sizeof(int), s));
    // device time of each instance's correlation and first level (event
    // pairs of the context, for the first 128 instances)
    const int n_timed = std::min(ni, fpc_ctx::kLaunchEvents / 2);
    uint8_t *d_ind = ctx->dellist.as<uint8_t>();
    for (int k = 0; k < ni; ++k) {
        const fpc_instance &I = inst[k];
        Run &R = runs[k];
        init_run(R, ctx, P, I.p, I.n, false);
        const size_t pp = (size_t)I.p * I.p;
        if (k < n_timed) FPC_HIP(hipEventRecord(ctx->lev[4 * k], s));
        const void *X = I.X;
        if (I.rows) {  // resample: the listed rows of X, in order
            if ((rc = gather_rows_enqueue(ctx, I.X, P->x_dtype, I.x_rows, I.p, I.rows, I.n, ctx->x_copy.ptr,
                                          d_rows_bad)))
                return rc;
            X = ctx->x_copy.ptr;
        }
        R.X = X;
        R.x_dtype = P->x_dtype;
        R.C64 = reinterpret_cast<double *>(base + off64[k]);
        if ((rc = corr_compute(ctx, X, P->x_dtype, I.n, I.p, FPC_CORR_FP64, const_cast<double *>(R.C64), false,
                               false)))
            return rc;
        if (mixed && (rc = c32_enqueue(R, reinterpret_cast<float *>(base + off32[k])))) return rc;
        char *h = hb + hoff[k];
        FPC_HIP(hipMemcpyAsync(h + (pp + 255) / 256 * 256, ctx->flag.ptr, 40, hipMemcpyDeviceToHost, s));
        if (k < n_timed) {
            FPC_HIP(hipEventRecord(ctx->lev[4 * k + 1], s));
            FPC_HIP(hipEventRecord(ctx->lev[4 * k + 2], s));
        }
        const int *d_bad = nullptr;
        if ((rc = first_level_enqueue(ctx, R.C64, I.p, I.n, R.q, nullptr, d_ind, &d_bad))) return rc;
        if (k < n_timed) FPC_HIP(hipEventRecord(ctx->lev[4 * k + 3], s));
        FPC_HIP(hipMemcpyAsync(h, d_ind, pp, hipMemcpyDeviceToHost, s));
        FPC_HIP(hipMemcpyAsync(h + (pp + 255) / 256 * 256 + kTail - 8, d_bad, sizeof(int), hipMemcpyDeviceToHost,
                               s));
    }
    FPC_HIP(hipMemcpyAsync(hb, d_rows_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    host_wake();  // the decisions are read on the host threads
    FPC_HIP(hipStreamSynchronize(s));  // the one wait
    int rows_bad;
    std::memcpy(&rows_bad, hb, sizeof(int));
    if (rows_bad) return FPC_EINVAL;
    for (int k = 0; k < ni; ++k) {
        Run &R = runs[k];
        const size_t pp = (size_t)R.p * R.p;
        const char *h = hb + hoff[k];
        const char *tail = h + (pp + 255) / 256 * 256;
        int fl[2], bad;
        std::memcpy(fl, tail, sizeof(fl));
        std::memcpy(&bad, tail + kTail - 8, sizeof(int));
        if (fl[0]) return FPC_ENONFINITE;
        if (fl[1]) return FPC_ESINGULAR;
        if (mixed) std::memcpy(&R.c_err, tail + 32, sizeof(double));
        if (bad) return FPC_ESINGULAR;
        fpc_level_stats st = first_level_stats(R.p);
        if (k < n_timed) {
            float c = 0.f, f = 0.f;
            FPC_HIP(hipEventElapsedTime(&c, ctx->lev[4 * k], ctx->lev[4 * k + 1]));
            FPC_HIP(hipEventElapsedTime(&f, ctx->lev[4 * k + 2], ctx->lev[4 * k + 3]));
            corr_ms[k] = c;
            first_ms[k] = f;
            st.kernel_ms = f;
        }
        first_marks(R, reinterpret_cast<const uint8_t *>(h), st);
        st.level_ms = first_ms[k];
        R.levels.push_back(st);
    }
    return FPC_OK;
}

int skeleton_batch_impl(fpc_ctx *ctx, const fpc_params *P, int ni, const fpc_instance *inst, fpc_result **outs)
{
    const double t_start = now_ms();
    int rc = validate_batch(P, ni, inst);
    if (rc) return rc;
    FPC_HIP(hipSetDevice(ctx->device));
    ctx->use_pair_kernel = !(P->flags & FPC_FLAG_PER_TEST_KERNEL);
    if ((P->flags & FPC_FLAG_GRAPH) && ctx->use_pair_kernel) {
        rc = skeleton_batch_device(ctx, P, ni, inst, outs, t_start);
        if (rc != kGraphFallback) return rc;
        if (trace_on()) std::fprintf(stderr, "[fpc] batch of %d: host-driven levels\n", ni);
    }
    const bool mixed = P->precision == FPC_PREC_MIXED;
    // every instance's matrices stay resident through all levels
    std::vector<size_t> off64(ni), off32(ni);
    size_t total = 0;
    auto a256 = [](size_t x) { return (x + 255) / 256 * 256; };
    for (int k = 0; k < ni; ++k) {
        const size_t pp = (size_t)inst[k].p * inst[k].p;
        off64[k] = total;
        total += a256(sizeof(double) * pp);
        off32[k] = total;
        if (mixed) total += a256(sizeof(float) * pp);
    }
    if ((rc = ctx->batch_c.ensure(total))) return rc;
    char *base = ctx->batch_c.as<char>();
    std::vector<Run> runs(ni);
    std::vector<double> corr_ms(ni, 0.0), first_ms(ni, 0.0);
    const double t_prep = now_ms();
    if ((rc = batch_prelude(ctx, P, ni, inst, base, off64, off32, runs, corr_ms, first_ms))) return rc;
    if (trace_on())
        std::fprintf(stderr, "[fpc] batch of %d: correlation and first level %.2f ms\n", ni, now_ms() - t_prep);
    // following levels, level-synchronous over the instances
    const int cap = P->max_level;
    std::vector<CandSets> cs(ni);
    std::vector<int> next(ni);    // current level of each instance (as in a single run)
    std::vector<char> done(ni, 0), fresh(ni, 0);
    for (int k = 0; k < ni; ++k) next[k] = cap >= 0 ? std::min(inst[k].p - 3, cap) : inst[k].p - 3;
    for (;;) {
        int top = -1;
        std::vector<int> eff(ni, -1);
        // candidate sets of the instances whose graph changed, on host threads
        {
            std::vector<int> todo;
            for (int k = 0; k < ni; ++k)
                if (!done[k] && next[k] >= 0 && !fresh[k]) todo.push_back(k);
            if (todo.size() == 1)
                candidate_sets(runs[todo[0]].adj.data(), runs[todo[0]].p, cs[todo[0]]);
            else
                parallel_for((int)todo.size(), [&](int x) {
                    candidate_sets(runs[todo[x]].adj.data(), runs[todo[x]].p, cs[todo[x]], 1);
                });
            for (int k : todo) fresh[k] = 1;
            if (trace_on()) std::fprintf(stderr, "[fpc] candidate sets of %zu instance(s)\n", todo.size());
        }
        for (int k = 0; k < ni; ++k) {
            if (done[k]) continue;
            if (next[k] < 0) {
                done[k] = 1;
                continue;
            }
            const int mmax = largest_cand(cs[k]);
            if (mmax < 0) {  // no edges left
                done[k] = 1;
                continue;
            }
            eff[k] = std::min(next[k], mmax);
            top = std::max(top, eff[k]);
        }
        if (top < 0) break;
        std::vector<Run *> part;
        std::vector<const CandSets *> pcs;
        std::vector<int> ids;
        for (int k = 0; k < ni; ++k)
            if (!done[k] && eff[k] == top) {
                part.push_back(&runs[k]);
                pcs.push_back(&cs[k]);
                ids.push_back(k);
            }
        std::vector<fpc_level_stats> lv;
        if ((rc = run_level(part, top, pcs, lv))) return rc;
        for (size_t t = 0; t < ids.size(); ++t) {
            const int k = ids[t];
            runs[k].levels.push_back(lv[t]);
            next[k] = top - 1;
            fresh[k] = lv[t].deleted == 0;  // candidate sets stay valid while the graph is unchanged
        }
    }
    for (int k = 0; k < ni; ++k) {
        if ((rc = assemble(runs[k], corr_ms[k], first_ms[k], t_start, &outs[k]))) {
            for (int t = 0; t < k; ++t) {
                fpc_result_free(outs[t]);
                outs[t] = nullptr;
            }
            return rc;
        }
    }
    return FPC_OK;
}

}  // namespace

extern "C" int fpc_skeleton(fpc_ctx *ctx, const fpc_params *params, fpc_result **out)
{
    if (!out) return FPC_EINVAL;
    *out = nullptr;
    if (!ctx) return FPC_EINVAL;
    return skeleton_impl(ctx, params, out);
}

extern "C" int fpc_skeleton_batch(fpc_ctx *ctx, const fpc_params *params, int n_inst, const fpc_instance *inst,
                                  fpc_result **out)
{
    if (!out || n_inst < 1) return FPC_EINVAL;
    for (int k = 0; k < n_inst; ++k) out[k] = nullptr;
    if (!ctx) return FPC_EINVAL;
    return skeleton_batch_impl(ctx, params, n_inst, inst, out);
}
