// Internal declarations shared by the library's translation units.
// Not part of the ABI (see include/fastpc.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/fastpc.h"

namespace fpc {

// Records the HIP error text for fpc_last_hip_error() and maps it to FPC_EDEVICE.
int hip_fail(hipError_t e, const char *what);

#define FPC_HIP(call)                                                   \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) return ::fpc::hip_fail(_e, #call);        \
    } while (0)

// A device buffer that grows on demand and is freed with the context.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t need);  // FPC_OK / FPC_ENOMEM / FPC_EDEVICE
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Pinned host staging buffer.
struct HostBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t need);
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

constexpr int kMaxTemplL = 16;   // largest level with a register-resident test kernel
constexpr int kBinomRows = 1024; // binomial table: C(a, b), a < kBinomRows, b <= kBinomCols-1
constexpr int kBinomCols = 64;

}  // namespace fpc

struct fpc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int lds_per_block = 65536;  // max dynamic LDS bytes per workgroup
    int lds_per_cu = 65536;     // LDS bytes per compute unit
    bool use_pair_kernel = true; // shared-prefix kernel for levels l >= 2 (off with FPC_FLAG_PER_TEST_KERNEL)
    int num_cus = 256;
    fpc_tuning tuning{};          // launch shapes of the level kernels (fpc_set_tuning)
    int64_t queue_init = int64_t(1) << 23;  // recheck queue entries: first size and cap
    int64_t queue_max = int64_t(1) << 28;   // (fpc_set_recheck_queue)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // the first level's results copied back; the mixed form's FP32 matrix
    // and its error measure done (queued after the first level)
    hipEvent_t ev_first = nullptr, ev_c32 = nullptr;
    // second stream of a level's window: the size classes after the first
    // run on it, beside the first class (fork after the first plan, join
    // before the window's FP64 re-run)
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    static constexpr int kLaunchEvents = 256;
    hipEvent_t lev[2 * kLaunchEvents] = {};  // per-launch timing of the test kernels
    // timing events of the small levels queued back to back on one graph
    // (created on first use): per level ev0, ev1 and kChainLaunchEvents pairs
    static constexpr int kChainSlots = 8, kChainLaunchEvents = 8;
    hipEvent_t chain_ev[kChainSlots][2 + 2 * kChainLaunchEvents] = {};
    bool chain_ev_ready = false;

    // binomial table on the device (saturating int64), kBinomRows x kBinomCols
    fpc::DevBuf binom;
    // the same table column-major (C(a, b) at b * kBinomRows + a): a wave
    // reads C(a, b) for 64 consecutive a in one coalesced load
    fpc::DevBuf binomT;
    std::vector<int64_t> binom_host;
    std::vector<int64_t> binomT_host;  // the column-major copy on the host (separating sets' unranking)

    // correlation / first level
    fpc::DevBuf x_copy;           // X uploaded from host
    fpc::DevBuf colstat;          // mu, sd (FP64) + partials
    fpc::DevBuf c64, c32;         // correlation matrices
    fpc::DevBuf zsplit;           // bf16 hi/lo copies of the standardized data
    fpc::DevBuf inv_work;         // first level: matrix being inverted + panel buffers
    fpc::DevBuf flag;             // small device scalars (error flags, counters)

    // level workspace
    fpc::DevBuf cand;             // int32 candidate list of fpc_level_series
    fpc::DevBuf edges;            // EdgeRec per eligible edge, then the int32 candidate lists
    fpc::DevBuf blockoff;         // window plan: item counters, workgroup sums, per-edge item prefix
    fpc::DevBuf insts;            // per-instance matrices and thresholds of a level
    fpc::DevBuf batch_c;          // fpc_skeleton_batch: every instance's correlation matrices
    fpc::DevBuf minhit;           // uint64 per edge: lowest independent rank
    fpc::DevBuf counters;         // uint64 counters (tests executed, queue length, ...), then the deletions
    fpc::DevBuf queue;            // recheck queue (edge, rank)
    fpc::DevBuf dellist;          // first-level decisions
    fpc::DevBuf batch_tmp;        // fpc_ci_batch / MLP gradient partials
    fpc::DevBuf mlp_grad;         // MLP gradient + loss of one training step
    fpc::DevBuf rfirst;           // first-level partial correlations (learned order)
    fpc::DevBuf feat;             // per-position features and scores
    fpc::DevBuf cand2;            // reordered candidate lists
    fpc::DevBuf degs;             // node degrees of the current graph

    fpc::HostBuf h_stage;         // pinned staging for uploads
    fpc::HostBuf h_back;          // pinned staging for downloads
    fpc::HostBuf h_inst;          // pinned staging for the instance table
    fpc::HostBuf h_flag;          // pinned landing of the correlation flags
    void *scratch = nullptr;      // this device's address of the no-allocation workspace (first_level.hip)

};

namespace fpc {

// One eligible edge of a level, as the test kernels see it.
struct EdgeRec {
    int32_t i, j;      // variables, i < j (within the instance)
    int32_t m;         // |cand|
    int32_t cand_off;  // offset of its candidate list in the level's cand array
    int64_t ntests;    // C(m, l)
    int32_t inst;      // instance the edge belongs to (index into the level's instance table)
    int32_t reserved;
};

// ---- correlation (corr.hip)
// reuse_stats: the column statistics of the previous call on the same X
// (same n, p) are still in the context and are used as they are.
// keep_flags: the error flags (non-finite, constant column) are not cleared
// first, so several instances accumulate into them.
int corr_compute(fpc_ctx *ctx, const void *X, int x_dtype, int n, int p, int method, void *C_out,
                 bool reuse_stats = false, bool wait = true, bool keep_flags = false);
int corr_reserve(fpc_ctx *ctx, int n, int p, int method);
// With wait = false the products are only queued: corr_check waits once for
// every queued correlation (and max_abs_diff) and reports their flags.
// slot (device, 8 bytes; NULL: the context's flag word): the largest |c64 - c32| as FP64 bits
int corr_max_abs_diff_enqueue(fpc_ctx *ctx, const double *c64, const float *c32, int p,
                              unsigned long long *slot = nullptr);
// c32 := FP32 rounding of c64 (device, p x p), queued.
int corr_round_enqueue(fpc_ctx *ctx, const double *c64, float *c32, int p, bool wait);
int corr_check(fpc_ctx *ctx, double *max_abs_diff);
// The same queued, with an index out of range setting *bad (device).
int gather_rows_enqueue(fpc_ctx *ctx, const void *X, int x_dtype, int64_t x_rows, int p, const int32_t *rows, int n,
                        void *out, int *bad);
// out (device, n x p) := rows[r] of X (device, x_rows x p); FPC_EINVAL for an index out of range.
int gather_rows(fpc_ctx *ctx, const void *X, int x_dtype, int64_t x_rows, int p, const int32_t *rows, int n,
                void *out);

// FPC_TRACE=1 in the environment: phase timings and launch shapes on stderr.
bool trace_on();

// ---- first level (first_level.hip)
int first_level(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out,
                uint8_t *indep_out, int *n_singular);
// The same work queued on the context's stream without waiting for it;
// *d_bad (device int) becomes nonzero if C is not positive definite.
int first_level_enqueue(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out,
                        uint8_t *indep_out, const int **d_bad);
// Sizes first_level_enqueue's workspace for p (no buffer then grows for a
// p' <= p while queued work reads it).
int first_level_reserve(fpc_ctx *ctx, int p);
// Many instances at once: each instance's matrix C (FP64, p x p), two p x p
// sweep buffers, a panel workspace of seven 32 x 32 blocks (contiguous), its
// flag and counter, and its adjacency bytes (written: 1 = kept).
struct FirstLevelInst {
    const double *C;
    double *buf0, *buf1, *pinv;
    int *bad;
    unsigned long long *deleted;
    uint8_t *adj;
    int p, n;
    double q;
};
// Panel t of one instance (the prologue job: Ain = C, the other fields but
// pinv, bad and p unused): workgroups [tile0, tile0 + 2 + nbt (nbt + 1) / 2)
// of the launch.
struct SweepJob {
    const double *Ain;
    double *Aout;
    double *pinv;  // the instance's panel workspace (seven 32 x 32 blocks)
    int *bad;
    int p, t, nbt;
    int64_t tile0;
};
struct DecideJob {
    const double *Om;  // the swept matrix, -Omega
    uint8_t *adj;
    int *bad;
    unsigned long long *deleted;
    int p, n;
    double q;
    int64_t elem0;
};
struct FirstLevelBatchBufs {
    const SweepJob *first_jobs;        // device, one per instance
    const SweepJob *panel_jobs;        // device, every step's jobs
    const DecideJob *decide_jobs;      // device, one per instance
    std::vector<int> panel_job0, panel_njobs;
    std::vector<int64_t> panel_tiles;
    int64_t decide_elems;
};
int first_level_batch_plan(const std::vector<FirstLevelInst> &in, std::vector<SweepJob> &first,
                           std::vector<SweepJob> &panels, std::vector<int> &panel_job0, std::vector<int> &panel_njobs,
                           std::vector<int64_t> &panel_tiles, std::vector<DecideJob> &decide, int64_t &decide_elems);
int first_level_batch_enqueue(fpc_ctx *ctx, const std::vector<FirstLevelInst> &in, const FirstLevelBatchBufs &b);

// Sets ctx->scratch to the device address of the static no-allocation
// workspace (the context's device current).
int noalloc_init(fpc_ctx *ctx);

// ---- level tests (citest.hip)
// One problem instance of a level: its matrices and threshold.
struct LevelInst {
    const float *C32;              // device FP32 matrix (mixed form; may be NULL otherwise)
    const double *C64;             // device FP64 matrix
    int p, n;
    double q;                      // threshold
    double c_err;                  // bound on the entry error of the FP32 matrix
};
// A run of consecutive edge records launched together (one size class).
struct LevelClass {
    int64_t begin, end;            // edge records [begin, end)
    int max_m;                     // largest |cand| in the class
};
// Timing events of one level: ev0 and ev1 around its launches, lev[2k] and
// lev[2k + 1] around its k-th test launch (k < n_lev; later ones untimed).
struct LevelEvents {
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const hipEvent_t *lev = nullptr;
    int n_lev = 0;
};
struct LevelLaunch {
    int l;
    int max_m;                     // largest |cand| among the eligible edges
    int64_t n_edges;               // eligible edges (of every instance)
    const LevelClass *classes;     // host; NULL: one class of every edge
    int n_classes;
    const EdgeRec *edges;          // device
    const int32_t *cand;           // device
    const LevelInst *insts;        // host, n_insts entries; EdgeRec::inst indexes them
    int n_insts;
    bool fp32;                     // tests in FP32 with FP64 recheck
    bool graph;                    // capture the level's launches in one HIP graph
    double band_z;                 // recheck margin in z units
    double ill_cond_tau = -1.0;    // FP32 tests with rho below this go to FP64 (< 0: the default)
    uint64_t *minhit;              // device, per edge
    unsigned long long *counters;  // device: [1] recheck queue length, [2] deletions, [3] queue overflow
    unsigned long long *inst_cnt;  // device, per instance: [2k] tests executed, [2k+1] re-run in FP64
    int64_t *queue;                // device, 2 * queue_cap entries (edge, rank)
    int64_t queue_cap;
    const LevelEvents *events = nullptr;  // NULL: the context's ev0, ev1 and lev
    size_t inst_off = 0;           // byte offset of the level's instance records in ctx->h_inst
    // diagnostic run (fpc_level_series): one window [diag_lo, diag_hi) of
    // ranks, r and the decision of every rank written at [rank - diag_lo],
    // no early exit and no FP64 re-run
    double *diag_r = nullptr;
    uint8_t *diag_dec = nullptr;
    int64_t diag_lo = 0, diag_hi = 0;
    int force_kernel = 0;          // FPC_KERNEL_*; 0: the kernel the level would choose
    int force_pdec = -1;           // triple kernel: pair-table entries (-1: as the level would size it)
    int force_rpw = 0;             // ranks per wave of a work item (0: the tuning table)
};
struct LevelTiming {
    float all_ms = 0.f;       // first test launch to last recheck, one event pair
    float test_ms = 0.f;      // test-kernel launches alone: the union of their intervals
    int test_launches = 0;
    int n_events = 0;         // timed launches (event pairs)
    bool graph = false;       // the level ran as one captured graph
    hipEvent_t e0 = nullptr, e1 = nullptr;  // the events level_tests recorded
    const hipEvent_t *lev = nullptr;
};
// Size class of an edge with m candidates at level l: edges of one class
// share a kernel and the number of workgroups that fit on a CU.
int level_class_key(const fpc_ctx *ctx, int l, bool fp32, int m);
void tuning_defaults(fpc_tuning *t);
// Queues a level's tests on the context's stream (no wait); callers
// synchronise the stream before the next level and before level_timing.
int level_tests(fpc_ctx *ctx, const LevelLaunch &L, const std::vector<int64_t> &host_ntests,
                LevelTiming *timing);
// ---- level loop on the device (batch_graph.hip)
// Per-instance sources of the level's instance table (device array).
struct DevInstSrc {
    const float *C32;      // FP32 matrix (mixed form) or NULL
    const double *C64;     // FP64 matrix
    int p, n;
    double q;              // threshold
    const double *c_err;   // device: largest entry error of the FP32 matrix (NULL: 0)
};
struct DeviceLevelClass {
    int max_m;             // bound of the class's list lengths (fixes kernel and LDS)
    const int64_t *range;  // device [begin, end) of the class in the level's edge table
};
struct DeviceLevel {
    int l;
    bool fp32;
    const EdgeRec *edges;  // device, the level's table (classes contiguous)
    const int32_t *cand;
    const void *insts;     // device InstRec table (level_inst_table_enqueue)
    uint64_t *minhit;      // device, per record, all ones at the start
    unsigned long long *counters, *inst_cnt;
    int64_t *queue;
    int64_t queue_cap;
    int64_t *plan;         // plan buffer: 3 * n_classes + the level's table size entries
    int max_m_all;         // largest bound of the classes (FP64 re-run)
    const DeviceLevelClass *classes;  // host
    int n_classes;         // at most kMaxDeviceClasses
};

// List-length bounds of a device-built level's size classes (ascending,
// the last kBinomRows - 1): maximal runs of m that launch the same kernel
// with the same workgroups per CU (registers, the LDS of the run's bound,
// the tuning cap), so a class sized for its bound runs at the occupancy of
// any of its lists; at most kMaxDeviceClasses.
constexpr int kMaxDeviceClasses = 16;
std::vector<int> device_class_bounds(const fpc_ctx *ctx, int l, bool fp32);
size_t inst_rec_bytes();
// The whole batch call on the device in one captured graph
// (fpc_skeleton_batch with FPC_FLAG_GRAPH).  kGraphFallback: the call is
// outside what the graph path takes, or a capacity was outgrown; the
// host-driven batch runs instead.
constexpr int kGraphFallback = -1000;
constexpr int kMaxGraphLevel = 7;   // C(1023, 7) < 2^63: the widest list class stays countable
constexpr int kMaxGraphP = 4096;    // LDS of the per-node component search
struct GraphBatchOut {
    struct Inst {
        std::vector<uint8_t> adj;                 // p x p, 1 = edge kept
        std::vector<int64_t> sep_pair, sep_off;   // separating sets of the subset levels
        std::vector<int32_t> sep_level, sep_nodes;
        std::vector<fpc_level_stats> levels;      // first level, then the subset levels run
        double c_err = 0.0, q = 0.0;
    };
    std::vector<Inst> inst;
    double graph_ms = 0.0, total_ms = 0.0;  // device time of the graph (events), whole call
    double prep_ms = 0.0, capture_ms = 0.0, instantiate_ms = 0.0, run_ms = 0.0;  // host phases
};
int skeleton_batch_graph(fpc_ctx *ctx, const fpc_params *P, int ni, const fpc_instance *inst, GraphBatchOut &out);
int level_inst_table_enqueue(fpc_ctx *ctx, const DevInstSrc *src, int ni, int l, double band_z, double tau, bool fp32,
                             void *out);
int level_tests_device(fpc_ctx *ctx, const DeviceLevel &D);

// Reads the timings of a level_tests call once its work has completed.
int level_timing(fpc_ctx *ctx, LevelTiming *timing);
// Sizes the context's level buffers for n_levels levels of at most n_edges
// edges and n_insts instances queued back to back (no buffer may grow while
// queued work reads it); *inst_stride is the byte distance between the
// levels' instance records in ctx->h_inst.
int level_reserve(fpc_ctx *ctx, int64_t n_edges, int n_insts, int n_levels, size_t *inst_stride);
// Queues minhit[e] = all ones (no hit) for the level's edges and zeroes
// the n_cnt counters.
int level_init(fpc_ctx *ctx, uint64_t *minhit, int64_t n_edges, unsigned long long *counters, int n_cnt);
// Queues the compaction of the level's hits: the t-th deletion (in no set
// order) is d_pairs[2t] = edge, d_pairs[2t + 1] = its first independent
// rank; *d_count (zero beforehand) counts them.
int level_compact_enqueue(fpc_ctx *ctx, const uint64_t *minhit, int64_t n_edges, int64_t *d_pairs,
                          unsigned long long *d_count);
// Queues the copy of bytes [offset, offset + bytes) of the pinned buffer src
// into device memory dst by a kernel that reads src through its device
// mapping (the runtime's small host-to-device copies have held the calling
// thread for milliseconds); a buffer with no mapping, or a size or address
// that is not a multiple of 4, takes hipMemcpyAsync.  The host must not
// change those bytes before the stream has passed the copy.
int upload_enqueue(fpc_ctx *ctx, void *dst, const HostBuf &src, size_t offset, size_t bytes);
int ci_batch(fpc_ctx *ctx, const void *C, int c_dtype, int p, int n, int l, const int32_t *B,
             int64_t b, double q, double *z_out, uint8_t *indep_out);

// ---- learned order (order.hip, mlp.hip)
int level_features(fpc_ctx *ctx, const EdgeRec *edges, int64_t n_edges, const int32_t *cand, int64_t n_pos,
                   const double *C, const double *R, const int32_t *deg, int p, float *X);
int level_reorder(fpc_ctx *ctx, const EdgeRec *edges, int64_t n_edges, const int32_t *cand_in, const float *score,
                  int32_t *cand_out);
int mlp_forward(fpc_ctx *ctx, const float *X, int64_t N, const void *model, float *out);
int mlp_grad(fpc_ctx *ctx, const float *X, const float *Y, int64_t N, const void *model, float *grad_out);
size_t mlp_model_bytes();
int mlp_params();

// ---- host graph logic (graph.cpp)
// Candidate sets of every edge of the graph (row-major i<j order).
struct CandSets {
    std::vector<int32_t> ei, ej;
    std::vector<int64_t> off;   // E+1
    std::vector<int32_t> nodes;
};
// threads: host threads for the merge (0: up to 16).
void candidate_sets(const uint8_t *adj, int p, CandSets &out, int threads = 0);

// ---- host thread pool (hostpool.cpp)
// fn(k) for k in [0, n) on the library's persistent host threads (inline
// when the pool is busy or when called from inside a job).
void host_parallel(int n, const std::function<void(int)> &fn);
int host_threads();
// Wakes the sleeping host threads for another spin: called before a device
// wait whose end is followed by host-parallel work.
void host_wake();

// ---- quantile (quantile.cpp)
double normal_quantile_upper(double alpha);  // Phi^{-1}(1 - alpha/2)

// ---- binomials (skeleton.cpp)
int64_t binom_sat(int a, int b);  // C(a,b), saturating at INT64_MAX

}  // namespace fpc
