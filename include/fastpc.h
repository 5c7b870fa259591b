/*
 * fastpc.h -- C ABI of the MI355X (gfx950) skeleton library for the
 * reverse-order pruning PC algorithm (Zhang, Tian, Johnson, Zhang, Jiang,
 * "A Fast PC Algorithm with Reversed-order Pruning and A Parallelization
 * Strategy", arXiv 2109.04626).
 *
 * Notation: the paper writes n for the number of variables and N for the
 * number of samples; this interface writes p for variables and n for
 * samples, and l = |K| for the size of a conditioning set.
 *
 * Conventions for every call:
 *   - plain C types only; pointers are borrowed (the caller keeps
 *     ownership) unless a call says it allocates;
 *   - "device pointer" = memory on the context's HIP device, "host
 *     pointer" = ordinary process memory;
 *   - every int-returning call returns FPC_OK (0) or one of the FPC_E*
 *     codes below and leaves its outputs untouched or undefined on error
 *     (all-or-nothing for results that the library allocates);
 *   - calls on one context are not thread-safe; different contexts are
 *     independent.  Work is enqueued on the context's stream and every
 *     call returns only after that work is complete, unless stated.
 */
#ifndef FASTPC_H
#define FASTPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define FPC_OK 0
#define FPC_EINVAL 1     /* bad argument: p < 2, n <= p + 1, alpha not in (0,1), NULL pointer, ... */
#define FPC_ENONFINITE 2 /* NaN or Inf in the data                                                */
#define FPC_ESINGULAR 3  /* correlation matrix not positive definite at the first level            */
#define FPC_EBUDGET 4    /* test budget (max_tests) exceeded, or a level whose test count overflows */
#define FPC_ENOMEM 5     /* host or device allocation failed                                       */
#define FPC_EDEVICE 6    /* a HIP runtime call failed; fpc_last_hip_error() names it               */
#define FPC_ESCRATCH 7   /* problem larger than the static workspace of a no-allocation call       */
#define FPC_ETOOLARGE 8  /* a subset level (l <= p-3) met a candidate set of 1024 or more variables:
                            the level kernels enumerate lists of at most 1023 (e.g. the forward
                            schedule on p >= 1026 variables, whose level 0 sees lists of p - 2)   */

/* ---------------------------------------------------------------- enums */
#define FPC_F64 0 /* IEEE binary64 elements */
#define FPC_F32 1 /* IEEE binary32 elements */

/* Correlation-matrix methods (fpc_corr; fpc_params.c32_method picks the
 * FP32 matrix of the mixed form). */
#define FPC_CORR_FP64 0   /* FP64 centring and FP64 products                                  */
#define FPC_CORR_BF16X3 1 /* bf16 two-way split, three MFMA products, FP32 sums (the lo.lo
                             term is dropped: entry errors up to a few 1e-6)                  */
#define FPC_CORR_BF16X6 2 /* bf16 three-way split, the six MFMA products of weight above
                             2^-24, FP32 sums (entry errors of FP32-rounding order)           */
#define FPC_CORR_FP32 3   /* the FP64 matrix rounded to FP32                                  */

/* Arithmetic of the level tests (fpc_params.precision). */
#define FPC_PREC_FP64 0  /* FP64 correlation, FP64 tests                                   */
#define FPC_PREC_MIXED 1 /* bf16x3 correlation, FP32 tests, FP64 re-run near the threshold */

/* Level schedules (fpc_params.schedule). */
#define FPC_REVERSE 0 /* Algorithm 2: l = p-2 down to 0, no early termination (Sec. 3.2)  */
#define FPC_FORWARD 1 /* Algorithm 1 (PC-stable): l = 0 upward, early termination (2.2.1) */

/* Order of the conditioning sets inside one level (fpc_params.order). */
#define FPC_ORDER_LEX 0     /* lexicographic over the candidate list sorted by variable id      */
#define FPC_ORDER_LEARNED 1 /* lexicographic over the candidate list sorted by decreasing MLP
                               score (fpc_params.order_model); reverse schedule only.  A level
                               with fewer than 32 possible tests per candidate keeps the
                               lexicographic order (the passes would cost more than they
                               can save)                                                    */

/* fpc_params.flags bits. */
#define FPC_FLAG_PER_TEST_KERNEL 1u /* run levels l >= 2 with the per-test Cholesky kernel instead of
                                       the shared-prefix (Schur pair) kernel; same results            */
#define FPC_FLAG_LOG_FEATURES 2u    /* record the ranking features of every candidate of every edge
                                       deleted after the first level (fpc_result.log_*)              */
#define FPC_FLAG_GRAPH 4u           /* fpc_skeleton: capture each level's launches (window plans,
                                       persistent test kernels, FP64 rechecks) in one HIP graph and
                                       launch it once; fpc_skeleton_batch: the whole call on the
                                       device in one HIP graph (see there); same results, per-launch
                                       timings not reported separately                               */

/* Kinds of recorded separating sets (fpc_result.sep_kind). */
#define FPC_SEP_NONE 0    /* edge kept                                                  */
#define FPC_SEP_LIST 1    /* K listed in sep_nodes                                      */
#define FPC_SEP_ALL_BUT 2 /* K = every variable except i and j (the l = p-2 level)      */

typedef struct fpc_ctx fpc_ctx;

/* ------------------------------------------------------------- context */
/* Create a context on HIP device `hip_device`.  `hip_stream` is a
 * hipStream_t to enqueue on, or NULL for a library-owned stream.  The
 * context owns its device workspace (grown on demand, freed by
 * fpc_destroy).  Errors: FPC_EINVAL (NULL out), FPC_EDEVICE. */
int fpc_create(fpc_ctx **out, int hip_device, void *hip_stream);
int fpc_destroy(fpc_ctx *ctx);

/* Text of an error code (static storage). */
const char *fpc_strerror(int code);
/* Name of the last HIP error seen by any call on this thread ("" if none). */
const char *fpc_last_hip_error(void);

/* Phi^{-1}(1 - alpha/2): threshold of the two-sided Fisher-z test
 * (Sec. 2.2.2).  Host-only; NaN for alpha outside (0,1). */
double fpc_quantile(double alpha);

/* ------------------------------------------------- correlation matrix (Sec. 5, "corr")
 * X: device pointer, row-major n x p (sample t, variable j at X[t*p + j]),
 * dtype x_dtype (FPC_F64 / FPC_F32).  C_out: device pointer, p x p
 * row-major, FPC_F64 for FPC_CORR_FP64 and FPC_F32 for the other methods.
 * C_ij = S_ij / sqrt(S_ii S_jj) with S the covariance of the centred
 * columns; C_ii = 1 exactly.  Errors: FPC_EINVAL (n < 2, p < 1, NULL),
 * FPC_ENONFINITE (a non-finite sample), FPC_ESINGULAR (a constant column). */
int fpc_corr(fpc_ctx *ctx, const void *X, int x_dtype, int n, int p, int method, void *C_out);

/* --------------------------------------------- the first reverse level (Algorithm 2, l = p-2)
 * On the complete graph every pair is conditioned on all other p-2
 * variables, so r_ij = -Omega_ij / sqrt(Omega_ii Omega_jj) with
 * Omega = C^{-1} (Sec. 5 formula with K = V \ {i,j}).  C: device, FP64,
 * p x p.  r_out: device, FP64 p x p (diagonal set to 1).  indep_out:
 * device, uint8 p x p, 1 where sqrt(n - (p-2) - 3) |atanh r| <= q.
 * Either output may be NULL.  Errors: FPC_EINVAL (n <= p + 1),
 * FPC_ESINGULAR (C not positive definite). */
int fpc_first_level(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out,
                    uint8_t *indep_out);

/* The same without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the sweep's workspace (two p x p FP64 buffers, seven 32 x 32
 * panel blocks, a flag word; 4.2 MB) is a static device array that each
 * device the library runs on holds until the process ends.  Same arguments,
 * outputs and results as fpc_first_level; p > FPC_NOALLOC_MAX_P returns
 * FPC_ESCRATCH.  Every call on a device shares that device's workspace, so
 * calls that overlap on one device (other contexts, other threads) race;
 * each call clears the flag it reads and waits for its work before
 * returning.  The context itself is created beforehand (fpc_create
 * allocates). */
#define FPC_NOALLOC_MAX_P 512
int fpc_first_level_noalloc(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out,
                            uint8_t *indep_out);

/* ------------------------------------------ one batch of CI tests (Sec. 5, index matrix B)
 * B: device, int32, b rows of (2 + l) entries [i, j, k_1 .. k_l] (the
 * paper's B^{b x (2+l)}); all indices in [0, p), distinct within a row.
 * C: device, p x p, c_dtype FPC_F64 or FPC_F32; the tests run in that
 * precision.  For each row: H = H0 - H1 H2^{-1} H1^T, r = h12/sqrt(h11 h22),
 * z_out[row] = sqrt(n - l - 3) |atanh r| (FP64, device), indep_out[row] =
 * (z <= q) (uint8, device).  A row whose H2 is not positive definite, whose
 * h11 or h22 is not positive or whose |r| >= 1 is degenerate: z = NaN,
 * indep = 0.  Either output may be NULL.  Errors: FPC_EINVAL (l < 0,
 * n - l - 3 <= 0, b < 0, bad dtype). */
int fpc_ci_batch(fpc_ctx *ctx, const void *C, int c_dtype, int p, int n, int l, const int32_t *B,
                 int64_t b, double q, double *z_out, uint8_t *indep_out);

/* ------------------------------------------ the level tests of one edge, rank by rank
 * Diagnostic: runs the tests that level l of fpc_skeleton runs for one edge
 * (i, j) with candidate list cand, ranks rank_lo .. rank_hi-1, through the
 * same kernels and launch shapes, and writes what each test computed.  Rank
 * t conditions on the t-th l-subset of the list, lexicographic over list
 * positions (the subset loop of Algorithm 2, Sec. 3.2); each test is
 * H = H0 - H1 H2^{-1} H1^T, r = h12 / sqrt(h11 h22) (Sec. 5 formula).  Every
 * rank of the range runs (no stop at an independent test, no FP64 re-run).
 *   C, c_dtype  device p x p matrix: FPC_F64 runs the FP64 kernels, FPC_F32
 *               the FP32 kernels of the mixed form;
 *   cand        host, m distinct variables other than i and j (any order);
 *   kernel      FPC_KERNEL_AUTO (the one the level would take), or one forced;
 *   ranks_per_wave  work-item length (0: the context's tuning table);
 *   pair_table  triple kernel's pair-decode table entries (-1: as the level
 *               sizes it; 0: every pair decoded arithmetically);
 *   q, band_z, c_err, ill_cond_tau  threshold, recheck margin in z units,
 *               entry error bound of an FP32 matrix and ill-conditioning
 *               threshold (fpc_params), as the level would use them.
 * Outputs (device, rank_hi - rank_lo entries): r_out = r (FP64; NaN for a
 * degenerate test), dec_out = decision (0 dependent, 1 independent, 2 left
 * to the FP64 re-run; the FP64 kernels give 0 or 1).  Errors: FPC_EINVAL
 * (range outside [0, C(m, l)), bad index, an unavailable kernel for l or a
 * pair table beyond the LDS), FPC_EDEVICE. */
#define FPC_KERNEL_AUTO 0
#define FPC_KERNEL_PER_TEST 1 /* per-test Cholesky in registers, tile staged in LDS      */
#define FPC_KERNEL_PAIR 2     /* shared (l-2)-prefix factor, 2x2 elimination (l >= 2)    */
#define FPC_KERNEL_TRIPLE 3   /* shared (l-3)-prefix table, rank-1 update per element a
                                 and 2x2 elimination per pair (l >= 3)                   */
#define FPC_KERNEL_GLOBAL 4   /* per-test Cholesky reading C from global memory          */
int fpc_level_series(fpc_ctx *ctx, const void *C, int c_dtype, int p, int n, int l, int i, int j,
                     const int32_t *cand, int m, int64_t rank_lo, int64_t rank_hi, int kernel,
                     int ranks_per_wave, int pair_table, double q, double band_z, double c_err,
                     double ill_cond_tau, double *r_out, uint8_t *dec_out);

/* ------------------------------------------------------- candidate sets (Sec. 2.1)
 * Host-only.  For every edge (i<j, row-major order) of the undirected
 * graph adj (host, uint8 p x p, symmetric, zero diagonal), the sorted set
 * adj(G,i,j) n path(G,i,j): neighbours of i or j lying on a simple path
 * between them.  Outputs (host): edge_i/edge_j[E], off[E+1] and
 * nodes[off[E]].  Call once with nodes == NULL to get E (return value
 * via *n_edges) and off[E] (via *n_nodes); buffers may be NULL when only
 * counting.  Returns FPC_OK or FPC_EINVAL. */
int fpc_candidates(const uint8_t *adj, int p, int64_t *n_edges, int64_t *n_nodes, int32_t *edge_i,
                   int32_t *edge_j, int64_t *off, int32_t *nodes);

/* ------------------------------------------------------------- skeleton (Phase I)
 * Learns the skeleton and separating sets (Algorithm 2, stable variant,
 * sampling version: Sec. 3.2 and 2.2.2; Algorithm 1 with FPC_FORWARD).
 */
typedef struct fpc_params {
    int32_t n;            /* samples                                                         */
    int32_t p;            /* variables                                                       */
    const void *X;        /* data, row-major n x p                                           */
    int32_t x_dtype;      /* FPC_F64 or FPC_F32                                              */
    int32_t x_on_device;  /* 1: X is a device pointer, 0: host pointer (copied in)           */
    double alpha;         /* significance level in (0,1)                                     */
    int32_t max_level;    /* < 0 uncapped; else reverse levels after the first start at
                             min(max_level, p-3) (the first level always runs), forward
                             levels stop after max_level                                    */
    int32_t precision;    /* FPC_PREC_FP64 or FPC_PREC_MIXED                                 */
    double recheck_margin;/* mixed: FP32 tests with |z - q| below this (plus the per-test
                             error bound) are re-run in FP64; <= 0 selects 1e-3             */
    int32_t schedule;     /* FPC_REVERSE or FPC_FORWARD                                      */
    int32_t order;        /* FPC_ORDER_LEX or FPC_ORDER_LEARNED                              */
    const void *order_model; /* FPC_ORDER_LEARNED: device buffer of fpc_mlp_bytes() bytes
                                (fpc_mlp_init); NULL otherwise                                */
    int64_t max_tests;    /* 0 = unlimited, else FPC_EBUDGET past this many tests            */
    double q_override;    /* NaN: q = Phi^{-1}(1 - alpha/2); else this threshold            */
    uint32_t flags;       /* FPC_FLAG_* bits, 0 for the defaults                             */
    double ill_cond_tau;  /* mixed: FP32 tests whose conditioning rho = (smallest Cholesky
                             pivot of C_KK) * min(h11, h22) lies below this are re-run in
                             FP64 whatever their z (the Cholesky of ill-conditioned
                             submatrices in FP64).  Decisions never depend on it: the
                             FP32 error band already scales as 1/rho.  1e-4 (the Python
                             default) guards the first-order error bound; 0 disables;
                             < 0 selects the strict threshold sqrt(n-l-3) (l+2)
                             (2^-24 + e) / 2.5e-3, e the largest entry error of the FP32
                             matrix, under which the FP32 z of every test decided in FP32
                             lies within 1e-4 of the FP64 z (more tests re-run)          */
    int32_t c32_method;   /* mixed: FP32 matrix of the tests, FPC_CORR_BF16X6 (default, 0
                             selects it), FPC_CORR_BF16X3 or FPC_CORR_FP32                */
    int32_t stop_after_levels; /* > 0: return at the level boundary after this many levels
                             of this call (the first level, l = p-2, counts as one), with
                             fpc_result.next_level set; 0: run to the end                */
    const struct fpc_checkpoint *resume; /* NULL: start on the complete graph; else continue
                             the run whose level-boundary state this is (the same data
                             and parameters; see fpc_checkpoint)                        */
} fpc_params;

typedef struct fpc_level_stats {
    int32_t level;            /* l                                                      */
    int32_t max_cand;         /* largest |cand| among the level's edges                */
    int64_t edges_eligible;   /* edges with |cand| >= l                                 */
    int64_t tests_possible;   /* sum over eligible edges of C(|cand|, l)                */
    int64_t tests_executed;   /* tests the GPU ran (early exit per edge and tile)       */
    int64_t tests_rechecked;  /* mixed: FP32 tests re-run in FP64                       */
    int64_t deleted;          /* edges removed at the end of the level                  */
    double kernel_ms;         /* device time of the level: test kernels, rechecks and
                                 gaps between them (HIP events on the context stream)   */
    double test_kernel_ms;    /* device time of the test-kernel launches alone: the
                                 union of their intervals (an event pair around each of
                                 the first 256 launches, 8 for small levels queued back
                                 to back; the size classes of a window run on two
                                 streams and overlap)                                   */
    int32_t test_launches;    /* test-kernel launches of the level                      */
    int32_t reserved;
    double level_ms;          /* whole level, host clock (small levels queued back to
                                 back: intervals that add up to the run's time)         */
    int64_t tests_required;   /* tests the method needs: per eligible edge, C(|cand|, l)
                                 if kept, else the rank of its first separating set + 1
                                 (independent of launch shapes and scheduling)          */
} fpc_level_stats;

typedef struct fpc_result {
    int32_t p;
    int32_t n_levels;
    uint8_t *adj;             /* p*p, symmetric skeleton, zero diagonal                 */
    int32_t *sep_level;       /* per pair i<j (row-major upper triangle index), -1 kept */
    int8_t *sep_kind;         /* FPC_SEP_*                                              */
    int64_t *sep_off;         /* P+1 offsets into sep_nodes (LIST kind only)            */
    int32_t *sep_nodes;       /* sorted node ids                                        */
    fpc_level_stats *levels;  /* n_levels rows, in execution order                      */
    int64_t total_tests;      /* tests executed over all levels                          */
    double q;                 /* threshold used                                          */
    double corr_ms;           /* correlation matrix                                      */
    double first_level_ms;    /* l = p-2 level (reverse schedule)                        */
    double total_ms;          /* whole call, data resident on the device                 */
    double corr_max_abs_err;  /* mixed: max |C_bf16x3 - C_fp64|, else 0                  */
    /* FPC_FLAG_LOG_FEATURES: one row per candidate of each edge deleted
     * after the first level (features at that level, in the order the
     * level used) */
    int64_t log_rows;
    float *log_x;             /* log_rows x 3: the ranking features                      */
    uint8_t *log_y;           /* 1 if the candidate is in the recorded separating set    */
    int32_t *log_group;       /* serial number of the edge the row belongs to: deleted   */
                              /* edges in level order, pair order within a level (one    */
                              /* deleted with no candidates has a serial and no rows)    */
    int32_t *log_level;       /* level of the deletion                                   */
    int64_t n_lists;          /* pairs whose separating set is of LIST kind              */
    int64_t *list_pairs;      /* their pair indices, increasing (n_lists entries)        */
    int32_t next_level;       /* the level the run continues with (a call stopped by
                                 stop_after_levels), -1 when the run is complete          */
} fpc_result;

/* ------------------------------------------------------------- checkpoint / resume
 * The state of a run at a level boundary.  Under the stable schedule (Sec.
 * 4.1: deletions applied at the end of each level) the graph and the
 * separating sets found so far determine every later level, given C (which
 * is recomputed from the same data): resuming a run from any boundary
 * gives the result of the uninterrupted run (skeleton, separating sets,
 * level statistics in execution order).
 *   p           variables
 *   next_level  the next level to run: min(the level after the last one
 *               run, the largest candidate set) in reverse order, the level
 *               after it in forward order; -1: complete
 *   adj         p x p, 1 = edge (host)
 *   sep_*       per pair, as in fpc_result (host)
 *   levels      the statistics of the levels run so far (host)
 * All arrays are borrowed for the call.  A reverse run's checkpoint holds
 * the first level (levels[0].level = p-2), whose deleted pairs are those
 * absent from adj of kind FPC_SEP_ALL_BUT. */
typedef struct fpc_checkpoint {
    int32_t p;
    int32_t next_level;
    const uint8_t *adj;
    const int32_t *sep_level;
    const int8_t *sep_kind;
    const int64_t *sep_off;
    const int32_t *sep_nodes;
    int32_t n_levels;
    const fpc_level_stats *levels;
} fpc_checkpoint;

/* ck := views of r's arrays (valid while r lives). */
void fpc_checkpoint_of(const fpc_result *r, fpc_checkpoint *ck);

/* Errors: FPC_EINVAL (also: a checkpoint of another p, a next_level
 * outside [-1, p-3], NULL arrays, or feature logging with resume),
 * FPC_ENONFINITE, FPC_ESINGULAR, FPC_EBUDGET, FPC_ETOOLARGE, FPC_ENOMEM,
 * FPC_EDEVICE.  On success *out is a library allocation freed with
 * fpc_result_free; on error *out is NULL.  FPC_FAIL_ALLOC=1 in the
 * environment makes every device allocation the library attempts fail with
 * FPC_ENOMEM before the runtime is called (a test hook). */
int fpc_skeleton(fpc_ctx *ctx, const fpc_params *params, fpc_result **out);
void fpc_result_free(fpc_result *r);

/* ------------------------------------------------------------- launch tuning
 * Shapes of the level-test launches, per level l < FPC_TUNE_LEVELS (levels
 * above use the last entry).  They change only speed, never results:
 *   test_ranks_per_wave    ranks one wave of the per-test kernel (l <= 1,
 *                          or lists too long for the shared-prefix kernels)
 *                          takes per work item (64 .. 2^20)
 *   shared_ranks_per_wave  the same for the shared-prefix kernels (l >= 2)
 *   window_growth          ratio of consecutive rank windows (2 .. 64);
 *                          a window only runs edges with no separating set
 *   first_window_items     work items per edge in the first window (1 .. 64)
 *   max_blocks_per_cu      cap on resident workgroups per CU (0: none)
 *   shared_prefix_depth    2: tests share their first l-2 conditioning
 *                          variables (pair kernel); 3 (l >= 3 only): their
 *                          first l-3 and the next one per wave (triple kernel)
 * fpc_set_tuning(ctx, NULL) restores the defaults.  The autotuner
 * (paper_2109_04626_amd.autotune) measures settings on synthetic workloads
 * and writes a table the Python binding loads into each context. */
#define FPC_TUNE_LEVELS 17
typedef struct {
    int32_t test_ranks_per_wave[FPC_TUNE_LEVELS];
    int32_t shared_ranks_per_wave[FPC_TUNE_LEVELS];
    int32_t window_growth[FPC_TUNE_LEVELS];
    int32_t first_window_items[FPC_TUNE_LEVELS];
    int32_t max_blocks_per_cu[FPC_TUNE_LEVELS];
    int32_t shared_prefix_depth[FPC_TUNE_LEVELS];
} fpc_tuning;

int fpc_get_tuning(const fpc_ctx *ctx, fpc_tuning *out);
/* FPC_EINVAL for a value out of range (the context keeps its table). */
int fpc_set_tuning(fpc_ctx *ctx, const fpc_tuning *t);

/* ------------------------------------------------------------- recheck queue
 * Mixed form (FPC_PREC_MIXED): FP32 tests whose decision lies within the
 * error band of the threshold are queued and re-run in FP64 after each
 * launch (Sec. 2.2.2 decides the test; the band is a precision design).
 * The queue starts at `initial` entries (16 bytes each; default 2^23) and,
 * when a launch overflows it, grows 4x up to `max` entries (default 2^28)
 * and the level runs again in the mixed form; an overflow at `max` runs the
 * level in FP64.  Results never depend on these sizes.  Takes effect at the
 * next level run (the current queue is released).  FPC_EINVAL unless
 * 1 <= initial <= max <= 2^31. */
int fpc_set_recheck_queue(fpc_ctx *ctx, int64_t initial, int64_t max);

/* ------------------------------------------------------------- many instances
 * Runs the skeleton of several independent problems (bootstrap resamples of
 * one data set, separate data sets of uneven p) together: correlation and
 * first level per instance, then every following level of all instances in
 * shared launches (one edge table over the instances, persistent kernels).
 * Each result equals that of fpc_skeleton on the instance alone (same
 * skeleton, separating sets and level sequence); level timings in the
 * per-level stats are those of the shared launches, total_ms that of the
 * whole call.  Not in the paper: its batching concerns the tests of one
 * problem (Sec. 5).
 *
 * params: alpha or q_override, max_level, precision, recheck_margin, flags
 * (FPC_FLAG_GRAPH, FPC_FLAG_PER_TEST_KERNEL) and x_dtype apply to every
 * instance; schedule must be FPC_REVERSE and order FPC_ORDER_LEX (else
 * FPC_EINVAL); X, n, p and x_on_device are not read; max_tests is a
 * per-instance budget; stop_after_levels must be 0 and resume NULL.
 *
 * FPC_FLAG_GRAPH, with 0 <= max_level <= 7, max_tests = 0, no
 * FPC_FLAG_PER_TEST_KERNEL and every p <= 4096: the whole call runs on the
 * device as one HIP graph, captured and launched once -- correlations, the
 * first level of all instances in one launch per panel step, then for each
 * level its candidate sets (neighbours of v grouped by the components of
 * G - v), edge table, tests, FP64 re-runs and deletions -- and the host
 * reads the results once at the end.  The levels and results are those of
 * the host-driven batch; a capacity the work outgrows (separating-set
 * store, candidate pool, recheck queue, a list of 1024 candidates or more)
 * makes the call run host-driven instead.  Per-level kernel_ms, level_ms
 * and test_launches are 0 in that mode, corr_ms and first_level_ms 0 and
 * total_ms the whole call. */
typedef struct {
    int32_t n;            /* samples of the instance (> p + 1)                                  */
    int32_t p;            /* variables (>= 2)                                                   */
    const void *X;        /* device, row-major x_rows x p, params->x_dtype; borrowed            */
    int64_t x_rows;       /* rows of X                                                          */
    const int32_t *rows;  /* device, n row indices into X (a resample: the instance's data are
                             those rows in this order); NULL: the first n rows (x_rows >= n)    */
} fpc_instance;

/* out: caller array of n_inst pointers; on success each holds a result freed
 * with fpc_result_free; on error all are NULL.  Errors as fpc_skeleton, and
 * FPC_EINVAL for an instance field or row index out of range. */
int fpc_skeleton_batch(fpc_ctx *ctx, const fpc_params *params, int n_inst, const fpc_instance *inst,
                       fpc_result **out);

/* ------------------------------------------------------------- candidate-ranking MLP
 * Orders each edge's candidate list for FPC_ORDER_LEARNED.  Features of a
 * candidate k of the pair (i, j): max(|C_ik|, |C_jk|), max(|R_ik|, |R_jk|)
 * with R the first-level partial correlations, and deg(k)/(p-1) in the
 * current graph.  Network 3 -> 64 -> 64 -> 1 with ReLU; bf16 weights in the
 * passes, FP32 accumulation, FP32 master weights and Adam moments.
 * The model is an opaque device buffer of fpc_mlp_bytes() bytes; its
 * parameters are fpc_mlp_params() floats ordered W1[3][64], b1[64],
 * W2[64][64], b2[64], W3[64], b3 (row-major, input index first).  X is a
 * device n x 3 FP32 array, y a device n FP32 array of 0/1 labels.  Not part
 * of the paper: the stable schedule makes the skeleton independent of this
 * order, which only changes how soon a separating set is found. */
size_t fpc_mlp_bytes(void);
int fpc_mlp_params(void);
/* model := params (host, FP32) with zero Adam state.  FPC_EINVAL (model
 * untouched) if any parameter is NaN or infinite. */
int fpc_mlp_init(fpc_ctx *ctx, void *model, const float *params);
/* params_out (host) := the FP32 master parameters. */
int fpc_mlp_get(fpc_ctx *ctx, const void *model, float *params_out);
/* logits_out (device, n FP32) := network output; n = 0 is a no-op (X and
 * logits_out may then be NULL). */
int fpc_mlp_forward(fpc_ctx *ctx, const float *X, int64_t n, const void *model, float *logits_out);
/* grad_out (device, fpc_mlp_params() + 1 FP32) := gradient of the mean
 * binary cross-entropy with logits over the n rows (n > 0, else
 * FPC_EINVAL), then the loss. */
int fpc_mlp_grad(fpc_ctx *ctx, const float *X, const float *y, int64_t n, const void *model, float *grad_out);
/* One Adam step (beta 0.9 / 0.999) on the mean loss of the n rows;
 * *loss_out (host, may be NULL) receives the loss before the step. */
int fpc_mlp_train_step(fpc_ctx *ctx, const float *X, const float *y, int64_t n, void *model, float lr,
                       float *loss_out);

/* ------------------------------------------------------------- Phase II (orientation)
 * Host-only.  Orients the skeleton adj (host, uint8 p x p) into a CPDAG
 * from the separating sets, given as in fpc_result (sep_level, sep_kind,
 * sep_off, sep_nodes per pair i<j; sep_level is accepted for symmetry and
 * not read): unshielded triples i - k - j with k outside S(i, j) become
 * i -> k <- j (lexicographic (i, j, k) order; a triple that would reverse
 * an arrow already placed is skipped), then rules R1-R4 are applied in
 * row-major sweeps over the undirected edges until a sweep changes nothing
 * (Phase II listing of Algorithm 1, Sec. 2.2.1; reused by Algorithm 2,
 * Sec. 3.2.2).  cpdag_out (host, uint8 p x p): [a*p+b] = 1 when the edge
 * a-b may point a -> b (undirected: both 1; a -> b: [a][b] = 1, [b][a] = 0).
 * Returns FPC_OK or FPC_EINVAL. */
int fpc_orient(int p, const uint8_t *adj, const int32_t *sep_level, const int8_t *sep_kind,
               const int64_t *sep_off, const int32_t *sep_nodes, uint8_t *cpdag_out);

#ifdef __cplusplus
}
#endif

#endif /* FASTPC_H */
