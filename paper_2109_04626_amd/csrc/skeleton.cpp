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
#include <chrono>
#include <cmath>
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

int DevBuf::ensure(size_t need)
{
    if (need <= bytes && ptr) return FPC_OK;
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
// (tab: kBinomRows x kBinomCols saturating table; C(a,b) = C(a,a-b)).
void unrank_host(int64_t R, int m, int l, const std::vector<int64_t> &tab, std::vector<int> &out)
{
    out.resize(l);
    int x = 0;
    auto C = [&](int a, int b) -> int64_t {
        if (b < 0 || b > a) return 0;
        const int bb = std::min(b, a - b);
        return bb < kBinomCols ? tab[(size_t)a * kBinomCols + bb] : binom_sat(a, b);
    };
    for (int t = 0; t < l; ++t) {
        for (;;) {
            const int64_t cnt = C(m - 1 - x, l - 1 - t);
            if (R < cnt) break;
            R -= cnt;
            ++x;
        }
        out[t] = x++;
    }
}

// Separating sets: level and kind per pair, LIST nodes in a flat array.
struct SepStore {
    std::vector<int32_t> level;                        // per pair, -1 kept
    std::vector<int8_t> kind;                          // per pair
    std::vector<std::pair<int64_t, int64_t>> lists;    // (pair, offset into nodes)
    std::vector<int32_t> nodes;
    void reset(int64_t P)
    {
        level.assign(P, -1);
        kind.assign(P, FPC_SEP_NONE);
        lists.clear();
        nodes.clear();
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
    if ((e = hipEventCreate(&c->ev0)) != hipSuccess || (e = hipEventCreate(&c->ev1)) != hipSuccess) {
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
    *out = c;
    return FPC_OK;
}

extern "C" int fpc_destroy(fpc_ctx *c)
{
    if (!c) return FPC_EINVAL;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    DevBuf *bufs[] = {&c->binom, &c->x_copy, &c->colstat, &c->c64, &c->c32, &c->zsplit, &c->inv_work,
                      &c->flag, &c->cand, &c->edges, &c->blockoff, &c->minhit, &c->counters,
                      &c->queue, &c->dellist, &c->batch_tmp, &c->mlp_grad, &c->rfirst, &c->feat,
                      &c->cand2, &c->degs, &c->insts};
    for (DevBuf *b : bufs) b->release();
    c->h_stage.release();
    c->h_back.release();
    c->h_inst.release();
    for (hipEvent_t ev : c->lev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return FPC_OK;
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
    std::free(r);
}

namespace {

constexpr int64_t kQueueCap = 1 << 23;  // recheck queue entries

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
};

// Runs one level (l >= 0) on the frozen graph with precomputed candidate
// sets; applies its deletions at the end.
int run_level(Run &R, int l, const CandSets &cs, fpc_level_stats &st)
{
    fpc_ctx *ctx = R.ctx;
    hipStream_t s = ctx->stream;
    const double t0 = now_ms();
    std::memset(&st, 0, sizeof(st));
    st.level = l;
    const int64_t Eall = (int64_t)cs.ei.size();
    std::vector<int64_t> sel;
    int max_m = 0;
    for (int64_t e = 0; e < Eall; ++e) {
        const int m = (int)(cs.off[e + 1] - cs.off[e]);
        max_m = std::max(max_m, m);
        if (m >= l) sel.push_back(e);
    }
    st.max_cand = max_m;
    const int64_t E = (int64_t)sel.size();
    st.edges_eligible = E;
    if (E == 0) {
        st.level_ms = now_ms() - t0;
        return FPC_OK;
    }
    std::vector<EdgeRec> recs(E);
    std::vector<int64_t> ntests(E);
    std::vector<int32_t> cand;
    int sel_max_m = 0;
    int64_t possible = 0;
    for (int64_t k = 0; k < E; ++k) {
        const int64_t e = sel[k];
        const int m = (int)(cs.off[e + 1] - cs.off[e]);
        if (m >= kBinomRows) return FPC_EBUDGET;
        const int64_t N = binom_sat(m, l);
        if (N == INT64_MAX || possible > INT64_MAX - N) return FPC_EBUDGET;
        possible += N;
        sel_max_m = std::max(sel_max_m, m);
        recs[k] = EdgeRec{cs.ei[e], cs.ej[e], m, (int32_t)cand.size(), N, 0, 0};
        ntests[k] = N;
        cand.insert(cand.end(), cs.nodes.begin() + cs.off[e], cs.nodes.begin() + cs.off[e + 1]);
    }
    st.tests_possible = possible;
    if (R.P->max_tests > 0 && R.spent_possible + possible > R.P->max_tests) return FPC_EBUDGET;
    R.spent_possible += possible;

    int rc;
    if ((rc = ctx->edges.ensure(sizeof(EdgeRec) * E))) return rc;
    if ((rc = ctx->cand.ensure(sizeof(int32_t) * (cand.size() + 1)))) return rc;
    if ((rc = ctx->minhit.ensure(sizeof(uint64_t) * E))) return rc;
    if ((rc = ctx->counters.ensure(sizeof(unsigned long long) * 8))) return rc;
    const size_t up = sizeof(EdgeRec) * E + sizeof(int32_t) * (cand.size() + 1);
    FPC_HIP(hipStreamSynchronize(s));  // the staging buffer is free
    if ((rc = ctx->h_stage.ensure(up))) return rc;
    std::memcpy(ctx->h_stage.ptr, recs.data(), sizeof(EdgeRec) * E);
    std::memcpy(ctx->h_stage.as<char>() + sizeof(EdgeRec) * E, cand.data(), sizeof(int32_t) * cand.size());
    FPC_HIP(hipMemcpyAsync(ctx->edges.ptr, ctx->h_stage.ptr, sizeof(EdgeRec) * E, hipMemcpyHostToDevice, s));
    if (!cand.empty())
        FPC_HIP(hipMemcpyAsync(ctx->cand.ptr, ctx->h_stage.as<char>() + sizeof(EdgeRec) * E,
                               sizeof(int32_t) * cand.size(), hipMemcpyHostToDevice, s));
    // learned order: features, MLP scores, per-edge reorder of the lists
    // (at l = 0 each edge has one subset, so the order cannot matter)
    std::vector<float> hfeat;
    const int32_t *d_cand = ctx->cand.as<int32_t>();
    const bool reorder = R.learned && l >= 1;
    if (reorder || R.logging) {
        const int64_t T = (int64_t)cand.size();
        std::vector<int32_t> deg(R.p, 0);  // degrees in the current graph, from its edge list
        for (size_t e = 0; e < cs.ei.size(); ++e) {
            ++deg[cs.ei[e]];
            ++deg[cs.ej[e]];
        }
        if ((rc = ctx->degs.ensure(sizeof(int32_t) * R.p))) return rc;
        if ((rc = ctx->feat.ensure(sizeof(float) * 4 * (size_t)(T + 1)))) return rc;
        if ((rc = ctx->cand2.ensure(sizeof(int32_t) * (size_t)(T + 1)))) return rc;
        FPC_HIP(hipMemcpyAsync(ctx->degs.ptr, deg.data(), sizeof(int32_t) * R.p, hipMemcpyHostToDevice, s));
        float *X = ctx->feat.as<float>(), *score = X + 3 * T;
        if ((rc = level_features(ctx, ctx->edges.as<EdgeRec>(), E, d_cand, T, R.C64, R.Rfirst,
                                 ctx->degs.as<int32_t>(), R.p, X)))
            return rc;
        if (reorder) {
            if ((rc = mlp_forward(ctx, X, T, R.P->order_model, score))) return rc;
            if ((rc = level_reorder(ctx, ctx->edges.as<EdgeRec>(), E, d_cand, score, ctx->cand2.as<int32_t>())))
                return rc;
            d_cand = ctx->cand2.as<int32_t>();
        }
        if (R.logging) {
            hfeat.resize(3 * (size_t)T);
            // features follow the original order; the reorder maps them
            FPC_HIP(hipMemcpyAsync(hfeat.data(), X, sizeof(float) * 3 * T, hipMemcpyDeviceToHost, s));
            FPC_HIP(hipStreamSynchronize(s));
        }
    }
    bool fp32 = R.mixed && l <= kMaxTemplL;
    if (fp32 && (rc = ctx->queue.ensure(sizeof(int64_t) * 2 * kQueueCap))) return rc;
retry:
    FPC_HIP(hipMemsetAsync(ctx->minhit.ptr, 0xff, sizeof(uint64_t) * E, s));
    FPC_HIP(hipMemsetAsync(ctx->counters.ptr, 0, sizeof(unsigned long long) * 8, s));

    LevelLaunch Lv{};
    Lv.l = l;
    Lv.max_m = sel_max_m;
    Lv.n_edges = E;
    Lv.edges = ctx->edges.as<EdgeRec>();
    Lv.cand = d_cand;
    const LevelInst inst{R.C32, R.C64, R.p, R.n, R.q, R.c_err};
    Lv.insts = &inst;
    Lv.n_insts = 1;
    Lv.fp32 = fp32;
    Lv.graph = (R.P->flags & FPC_FLAG_GRAPH) != 0;
    Lv.band_z = R.P->recheck_margin > 0 ? R.P->recheck_margin : 1e-3;
    Lv.minhit = ctx->minhit.as<uint64_t>();
    Lv.counters = ctx->counters.as<unsigned long long>();
    Lv.queue = fp32 ? ctx->queue.as<int64_t>() : nullptr;
    Lv.queue_cap = fp32 ? kQueueCap : 0;
    LevelTiming tm;
    if ((rc = level_tests(ctx, Lv, ntests, &tm))) return rc;
    // the host decodes separating sets against the lists the level used
    // (through the pinned stage: the upload that read it precedes this
    // copy on the stream)
    if (reorder && !cand.empty())
        FPC_HIP(hipMemcpyAsync(ctx->h_stage.ptr, d_cand, sizeof(int32_t) * cand.size(), hipMemcpyDeviceToHost, s));
    st.kernel_ms = tm.all_ms;
    st.test_kernel_ms = tm.test_ms;
    st.test_launches = tm.test_launches;

    std::vector<int64_t> pairs(2 * E);
    int64_t ndel = 0;
    if ((rc = level_compact(ctx, Lv.minhit, E, pairs.data(), &ndel))) return rc;
    unsigned long long cnt[8];
    FPC_HIP(hipMemcpyAsync(cnt, Lv.counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
    FPC_HIP(hipStreamSynchronize(s));
    st.tests_executed = (int64_t)cnt[0];
    st.tests_rechecked = (int64_t)cnt[2];
    R.total_exec += st.tests_executed;
    if (cnt[3]) {  // the recheck queue overflowed: run the whole level again in FP64
        fp32 = false;
        goto retry;
    }
    if (reorder && !cand.empty()) std::memcpy(cand.data(), ctx->h_stage.ptr, sizeof(int32_t) * cand.size());

    // sepsets and level-end deletion (stable: all of D at once)
    std::vector<std::pair<int64_t, int64_t>> dl(ndel);
    for (int64_t k = 0; k < ndel; ++k) dl[k] = {pairs[2 * k], pairs[2 * k + 1]};
    std::sort(dl.begin(), dl.end());
    std::vector<int> pos;
    for (const auto &d : dl) {
        const EdgeRec &er = recs[d.first];
        unrank_host(d.second, er.m, l, ctx->binom_host, pos);
        const int64_t pr = pair_index(er.i, er.j, R.p);
        R.sep.level[pr] = l;
        R.sep.kind[pr] = FPC_SEP_LIST;
        const size_t o = R.sep.nodes.size();
        R.sep.lists.emplace_back(pr, (int64_t)o);
        for (int t = 0; t < l; ++t) R.sep.nodes.push_back(cand[er.cand_off + pos[t]]);
        std::sort(R.sep.nodes.begin() + o, R.sep.nodes.end());
        if (R.logging) {
            // features were computed over the list sorted by id (the cs order)
            const int32_t *orig = cs.nodes.data() + cs.off[sel[d.first]];
            const int32_t *S = R.sep.nodes.data() + o;
            for (int a = 0; a < er.m; ++a) {
                const int k = orig[a];
                const bool in = std::binary_search(S, S + l, k);
                for (int f = 0; f < 3; ++f) R.log_x.push_back(hfeat[3 * ((size_t)er.cand_off + a) + f]);
                R.log_y.push_back(in ? 1 : 0);
                R.log_group.push_back(R.log_serial);
                R.log_level.push_back(l);
            }
            ++R.log_serial;
        }
    }
    for (const auto &d : dl) {
        const EdgeRec &er = recs[d.first];
        R.adj[(size_t)er.i * R.p + er.j] = R.adj[(size_t)er.j * R.p + er.i] = 0;
    }
    st.deleted = ndel;
    st.level_ms = now_ms() - t0;
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
    return FPC_OK;
}

int skeleton_impl(fpc_ctx *ctx, const fpc_params *P, fpc_result **out)
{
    const double t_start = now_ms();
    int rc = validate(P);
    if (rc) return rc;
    FPC_HIP(hipSetDevice(ctx->device));
    ctx->use_pair_kernel = !(P->flags & FPC_FLAG_PER_TEST_KERNEL);
    Run R;
    R.ctx = ctx;
    R.P = P;
    R.p = P->p;
    R.n = P->n;
    R.q = std::isnan(P->q_override) ? normal_quantile_upper(P->alpha) : P->q_override;
    R.mixed = P->precision == FPC_PREC_MIXED;
    R.learned = P->order == FPC_ORDER_LEARNED;
    R.logging = (P->flags & FPC_FLAG_LOG_FEATURES) != 0 && P->schedule == FPC_REVERSE;
    const int p = P->p, n = P->n;
    const size_t pp = (size_t)p * p;
    hipStream_t s = ctx->stream;

    // data on the device
    const void *X = P->X;
    if (!P->x_on_device) {
        const size_t bytes = (size_t)n * p * (P->x_dtype == FPC_F64 ? 8 : 4);
        if ((rc = ctx->x_copy.ensure(bytes))) return rc;
        FPC_HIP(hipMemcpyAsync(ctx->x_copy.ptr, P->X, bytes, hipMemcpyHostToDevice, s));
        X = ctx->x_copy.ptr;
    }
    // correlation matrices
    double t0 = now_ms();
    if ((rc = ctx->c64.ensure(sizeof(double) * pp))) return rc;
    if ((rc = corr_compute(ctx, X, P->x_dtype, n, p, FPC_CORR_FP64, ctx->c64.ptr))) return rc;
    R.C64 = ctx->c64.as<double>();
    if (R.mixed) {
        if ((rc = ctx->c32.ensure(sizeof(float) * pp))) return rc;
        if ((rc = corr_compute(ctx, X, P->x_dtype, n, p, FPC_CORR_BF16X3, ctx->c32.ptr))) return rc;
        R.C32 = ctx->c32.as<float>();
        if ((rc = corr_max_abs_diff(ctx, R.C64, R.C32, p, &R.c_err))) return rc;
    }
    const double corr_ms = now_ms() - t0;

    R.adj.assign(pp, 1);
    for (int i = 0; i < p; ++i) R.adj[(size_t)i * p + i] = 0;
    R.sep.reset((int64_t)p * (p - 1) / 2);
    double first_ms = 0.0;
    const int cap = P->max_level;
    CandSets cs;
    if (P->schedule == FPC_REVERSE) {
        // l = p - 2 on the complete graph, through Omega = C^{-1}
        t0 = now_ms();
        fpc_level_stats st{};
        st.level = p - 2;
        st.max_cand = p - 2;
        st.edges_eligible = st.tests_possible = st.tests_executed = (int64_t)p * (p - 1) / 2;
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
        if ((rc = first_level(ctx, R.C64, p, n, R.q, d_r, d_ind, nullptr))) return rc;
        FPC_HIP(hipEventRecord(ctx->ev1, s));
        std::vector<uint8_t> ind(pp);
        FPC_HIP(hipMemcpyAsync(ind.data(), d_ind, pp, hipMemcpyDeviceToHost, s));
        FPC_HIP(hipStreamSynchronize(s));
        float kms = 0.f;
        FPC_HIP(hipEventElapsedTime(&kms, ctx->ev0, ctx->ev1));
        st.kernel_ms = kms;
        int64_t dels = 0;
        for (int i = 0; i < p; ++i)
            for (int j = i + 1; j < p; ++j)
                if (ind[(size_t)i * p + j]) {
                    const int64_t pr = pair_index(i, j, p);
                    R.sep.level[pr] = p - 2;
                    R.sep.kind[pr] = FPC_SEP_ALL_BUT;
                    R.adj[(size_t)i * p + j] = R.adj[(size_t)j * p + i] = 0;
                    ++dels;
                }
        st.deleted = dels;
        R.total_exec += st.tests_executed;
        R.spent_possible += st.tests_possible;
        first_ms = now_ms() - t0;
        st.level_ms = first_ms;
        R.levels.push_back(st);
        // following levels: l = min(p-3, cap, largest candidate set), down to 0
        int l = p - 3;
        if (cap >= 0) l = std::min(l, cap);
        while (l >= 0) {
            candidate_sets(R.adj.data(), p, cs);
            int mmax = -1;
            for (size_t e = 0; e + 1 < cs.off.size(); ++e) mmax = std::max<int>(mmax, (int)(cs.off[e + 1] - cs.off[e]));
            if (mmax < 0) break;  // no edges left
            l = std::min(l, mmax);
            fpc_level_stats lv{};
            if ((rc = run_level(R, l, cs, lv))) return rc;
            R.levels.push_back(lv);
            --l;
        }
    } else {
        // Algorithm 1: l = 0, 1, ... while some edge has |cand| >= l
        for (int l = 0;; ++l) {
            if (cap >= 0 && l > cap) break;
            candidate_sets(R.adj.data(), p, cs);
            int mmax = -1;
            for (size_t e = 0; e + 1 < cs.off.size(); ++e) mmax = std::max<int>(mmax, (int)(cs.off[e + 1] - cs.off[e]));
            if (mmax < l) break;
            fpc_level_stats lv{};
            if ((rc = run_level(R, l, cs, lv))) return rc;
            R.levels.push_back(lv);
        }
    }

    // result
    fpc_result *res = (fpc_result *)std::calloc(1, sizeof(fpc_result));
    if (!res) return FPC_ENOMEM;
    const int64_t PP = (int64_t)p * (p - 1) / 2;
    res->p = p;
    res->n_levels = (int32_t)R.levels.size();
    res->adj = (uint8_t *)std::malloc(pp);
    res->sep_level = (int32_t *)std::malloc(sizeof(int32_t) * PP);
    res->sep_kind = (int8_t *)std::malloc(PP);
    res->sep_off = (int64_t *)std::malloc(sizeof(int64_t) * (PP + 1));
    const int64_t tot = (int64_t)R.sep.nodes.size();
    res->sep_nodes = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(tot, 1));
    res->levels = (fpc_level_stats *)std::malloc(sizeof(fpc_level_stats) * std::max<size_t>(R.levels.size(), 1));
    if (!res->adj || !res->sep_level || !res->sep_kind || !res->sep_off || !res->sep_nodes || !res->levels) {
        fpc_result_free(res);
        return FPC_ENOMEM;
    }
    std::memcpy(res->adj, R.adj.data(), pp);
    // LIST sets in pair order; each pair is deleted at most once
    std::sort(R.sep.lists.begin(), R.sep.lists.end());
    std::memcpy(res->sep_level, R.sep.level.data(), sizeof(int32_t) * PP);
    std::memcpy(res->sep_kind, R.sep.kind.data(), PP);
    int64_t o = 0;
    size_t li = 0;
    for (int64_t k = 0; k < PP; ++k) {
        res->sep_off[k] = o;
        if (li < R.sep.lists.size() && R.sep.lists[li].first == k) {
            const int L = R.sep.level[k];
            std::memcpy(res->sep_nodes + o, R.sep.nodes.data() + R.sep.lists[li].second, sizeof(int32_t) * L);
            o += L;
            ++li;
        }
    }
    res->sep_off[PP] = o;
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
    res->total_ms = now_ms() - t_start;
    *out = res;
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
