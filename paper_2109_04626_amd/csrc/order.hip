// Learned order of the candidate lists (one level of the reverse schedule).
//
// For each eligible edge (i, j) and each candidate k the features are
//     x0 = max(|C_ik|, |C_jk|)          marginal correlation with the pair
//     x1 = max(|R_ik|, |R_jk|)          partial correlation given all other
//                                       variables (the first level, l = p-2)
//     x2 = deg(k) / (p - 1)             degree of k in the current graph
// The MLP scores them, and every edge's list is reordered by decreasing
// score (ties: original position).  The lexicographic enumeration of the
// level then runs over the reordered list, so the l-subsets made of the
// highest-scored candidates come first.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fpc_internal.h"

namespace fpc {

namespace {

// One wave per edge, lanes over its candidate positions (the edge records
// need not be in list order).
__global__ __launch_bounds__(64) void features_kernel(const EdgeRec *__restrict__ edges,
                                                      const int32_t *__restrict__ cand,
                                                      const double *__restrict__ C, const double *__restrict__ R,
                                                      const int32_t *__restrict__ deg, int p, float *__restrict__ X)
{
    const EdgeRec E = edges[blockIdx.x];
    for (int a = threadIdx.x; a < E.m; a += 64) {
        const int64_t t = (int64_t)E.cand_off + a;
        const int k = cand[t];
        X[3 * t + 0] = (float)fmax(fabs(C[(size_t)E.i * p + k]), fabs(C[(size_t)E.j * p + k]));
        X[3 * t + 1] = (float)fmax(fabs(R[(size_t)E.i * p + k]), fabs(R[(size_t)E.j * p + k]));
        X[3 * t + 2] = (float)deg[k] / (float)(p - 1);
    }
}

// One block per edge: position a goes to rank(a) = #{b : s_b > s_a or
// (s_b == s_a and b < a)}, NaN scores taken as -inf.  The edge's scores are staged in LDS (lists hold
// fewer than kBinomRows candidates), so the m^2 comparisons read LDS.
__global__ __launch_bounds__(256) void reorder_kernel(const EdgeRec *__restrict__ edges,
                                                      const int32_t *__restrict__ cand_in,
                                                      const float *__restrict__ score,
                                                      int32_t *__restrict__ cand_out)
{
    __shared__ float sc[kBinomRows];
    const EdgeRec E = edges[blockIdx.x];
    const int m = E.m, off = E.cand_off;
    // a NaN score ranks as -inf, so the ranks below are a total order and
    // the output a permutation of the list whatever the model computes
    for (int a = threadIdx.x; a < m; a += 256) {
        const float x = score[off + a];
        sc[a] = isnan(x) ? -INFINITY : x;
    }
    __syncthreads();
    for (int a = threadIdx.x; a < m; a += 256) {
        const float sa = sc[a];
        int rank = 0;
        for (int b = 0; b < m; ++b) {
            const float sb = sc[b];
            rank += (sb > sa) || (sb == sa && b < a);
        }
        cand_out[off + rank] = cand_in[off + a];
    }
}

}  // namespace

int level_features(fpc_ctx *ctx, const EdgeRec *edges, int64_t n_edges, const int32_t *cand, int64_t n_pos,
                   const double *C, const double *R, const int32_t *deg, int p, float *X)
{
    if (n_pos == 0 || n_edges == 0) return FPC_OK;
    if (n_edges > 0x7fffffffLL) return FPC_EINVAL;
    features_kernel<<<(unsigned)n_edges, 64, 0, ctx->stream>>>(edges, cand, C, R, deg, p, X);
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

int level_reorder(fpc_ctx *ctx, const EdgeRec *edges, int64_t n_edges, const int32_t *cand_in, const float *score,
                  int32_t *cand_out)
{
    if (n_edges == 0) return FPC_OK;
    reorder_kernel<<<(unsigned)n_edges, 256, 0, ctx->stream>>>(edges, cand_in, score, cand_out);
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

}  // namespace fpc
