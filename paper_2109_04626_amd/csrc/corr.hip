// Correlation matrix of the data ("corr", Sec. 5): C_ij = S_ij / sqrt(S_ii S_jj)
// with S the cross-product matrix of the centred columns.
//
// Two methods:
//   FP64     column means in FP64, centred FP64 products on the FP64
//            matrix cores (LDS-staged, upper-triangle tiles only, split over
//            the samples so that the launch fills the chip);
//   BF16X3   columns standardised in FP64, each value split as
//            z = hi + lo with hi, lo in bf16, and S ~ hi.hi + hi.lo + lo.hi
//            on the MFMA units (v_mfma_f32_16x16x32_bf16) with FP32
//            accumulation over chunks of 512 samples, the chunk sums folded
//            into FP64 registers.  The dropped lo.lo term is biased for
//            strongly correlated columns (entry errors up to ~3e-6).
//   BF16X6   the same with a three-way split z = hi + mid + lo and the six
//            products of weight above 2^-24: hi.hi, hi.mid, mid.hi,
//            mid.mid, hi.lo, lo.hi, folded into FP64 after every 32
//            samples (entry errors of FP32 rounding order).
//   FP32     the FP64 matrix rounded to FP32.
// The MFMA forms renormalise by the computed diagonal, so C_ii = 1 exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "fpc_internal.h"

namespace fpc {

namespace {

constexpr int kStatRows = 64;  // rows per partial in the column statistics (enough workgroups to hide load latency)

// One pass of column statistics: per chunk of rows, the sums of x - K and
// (x - K)^2 with K = X[0][j], a value of the column itself (the shifted-data
// form of the two-pass variance: its cancellation error scales with
// (mean - K)^2 / var, of order one for a sample of the column).
template <typename TX>
__global__ __launch_bounds__(256) void colstat_partial(const TX *__restrict__ X, int n, int p,
                                                       double *__restrict__ part, int *__restrict__ nonfinite)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= p) return;
    const int r0 = blockIdx.y * kStatRows, r1 = min(n, r0 + kStatRows);
    const double K = (double)X[j];
    double s1 = 0.0, s2 = 0.0;
    bool bad = false;
    for (int t = r0; t < r1; ++t) {
        const double x = (double)X[(size_t)t * p + j];
        bad |= !isfinite(x);
        const double d = x - K;
        s1 += d;
        s2 = fma(d, d, s2);
    }
    part[(size_t)blockIdx.y * 2 * p + j] = s1;
    part[(size_t)blockIdx.y * 2 * p + p + j] = s2;
    if (bad) atomicOr(nonfinite, 1);
}

// mean and standard deviation of each column from the partial sums: 64
// columns per workgroup, four lanes per column each summing every fourth
// chunk (coalesced over the columns), then the four sums in a fixed order
template <typename TX>
__global__ __launch_bounds__(256) void colstat_reduce(const TX *__restrict__ X, const double *__restrict__ part,
                                                      int nchunks, int n, int p, double *__restrict__ mu,
                                                      double *__restrict__ sd, int *__restrict__ constant)
{
    __shared__ double r1[4][64], r2[4][64];
    const int c64 = threadIdx.x % 64, g = threadIdx.x / 64;
    const int j = blockIdx.x * 64 + c64;
    double s1 = 0.0, s2 = 0.0;
    if (j < p)
        for (int c = g; c < nchunks; c += 4) {
            s1 += part[(size_t)c * 2 * p + j];
            s2 += part[(size_t)c * 2 * p + p + j];
        }
    r1[g][c64] = s1;
    r2[g][c64] = s2;
    __syncthreads();
    if (g != 0 || j >= p) return;
    s1 = ((r1[0][c64] + r1[1][c64]) + r1[2][c64]) + r1[3][c64];
    s2 = ((r2[0][c64] + r2[1][c64]) + r2[2][c64]) + r2[3][c64];
    const double m1 = s1 / n;
    mu[j] = (double)X[j] + m1;
    const double var = fmax(s2 / n - m1 * m1, 0.0);
    sd[j] = sqrt(var);
    if (!(var > 0.0)) atomicOr(constant, 1);
}

// ---------------------------------------------------------------- FP64 products
constexpr int kT = 64;   // output tile edge
constexpr int kK = 32;   // samples per LDS stage

__device__ inline void tile_of(int t, int nbt, int &bi, int &bj)
{
    int b = 0;
    while (t >= nbt - b) {
        t -= nbt - b;
        ++b;
    }
    bi = b;
    bj = b + t;
}

// S_part[split][i][j] for the upper-triangle tiles; split = blockIdx.y covers
// samples [split*chunk, (split+1)*chunk).  FP64 matrix cores: each wave owns
// a 32 x 32 quarter of the 64 x 64 tile as 2 x 2 blocks of
// v_mfma_f64_16x16x4_f64 (A = the tile rows' centred samples, B = the tile
// columns'); lane l feeds A[l % 16][l / 16] and B[l / 16][l % 16], and
// accumulator v of lane l is D[4 v + l / 16][l % 16].
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename TX>
__global__ __launch_bounds__(256) void syrk_f64(const TX *__restrict__ X, const double *__restrict__ mu,
                                                int n, int p, int nbt, int chunk,
                                                double *__restrict__ Spart)
{
    int bi, bj;
    tile_of(blockIdx.x, nbt, bi, bj);
    const int t0 = blockIdx.y * chunk, t1 = min(n, t0 + chunk);
    __shared__ double As[kK][kT + 1];
    __shared__ double Bs[kK][kT + 1];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wr = wave / 2, wc = wave % 2;  // the wave's 32 x 32 quarter
    // staging: thread t loads column t % 64 of the tile rows and columns,
    // samples t / 64 + 4 m (m < kK / 4) of each stage; the next stage's
    // samples are fetched into registers while the current one is multiplied
    constexpr int kM = kK * kT / 256;
    const int c = threadIdx.x % kT, r0 = threadIdx.x / kT;
    const int ca = bi * kT + c, cb = bj * kT + c;
    const bool va = ca < p, vb = cb < p;
    const double mua = va ? mu[ca] : 0.0, mub = vb ? mu[cb] : 0.0;
    TX ra[kM], rb[kM];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int m = 0; m < kM; ++m) {
            const int row = k0 + r0 + 4 * m;
            ra[m] = (row < t1 && va) ? X[(size_t)row * p + ca] : TX(0);
            rb[m] = (row < t1 && vb) ? X[(size_t)row * p + cb] : TX(0);
        }
    };
    v4d acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    if (t0 < t1) fetch(t0);
    for (int k0 = t0; k0 < t1; k0 += kK) {
#pragma unroll
        for (int m = 0; m < kM; ++m) {
            const int r = r0 + 4 * m;
            const bool in = k0 + r < t1;
            As[r][c] = (in && va) ? (double)ra[m] - mua : 0.0;
            Bs[r][c] = (in && vb) ? (double)rb[m] - mub : 0.0;
        }
        __syncthreads();
        if (k0 + kK < t1) fetch(k0 + kK);
#pragma unroll
        for (int kk = 0; kk < kK; kk += 4) {
            const int kr = kk + lane / 16;
            double av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                av[t] = As[kr][wr * 32 + t * 16 + lane % 16];
                bv[t] = Bs[kr][wc * 32 + t * 16 + lane % 16];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    double *out = Spart + (size_t)blockIdx.y * p * p;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = bi * kT + wr * 32 + a * 16 + 4 * v + lane / 16;
                const int j = bj * kT + wc * 32 + b * 16 + lane % 16;
                if (i < p && j < p) out[(size_t)i * p + j] = acc[a][b][v];
            }
}

// C[i][j] = S_ij / sqrt(S_ii S_jj), S summed over the splits in order and
// taken from the upper triangle (i <= j), so C is exactly symmetric; C_ii =
// 1.  One 32 x 32 tile (I <= J; the products write whole 64 x 64 tiles
// I <= J, which contain these) per workgroup: its split sums are read
// row-wise, written to C[I][J] and, through an LDS transpose, to C[J][I],
// so every access of the p x p arrays is coalesced.
constexpr int kNT = 32;
template <typename TC>
__global__ __launch_bounds__(256) void normalize(const double *__restrict__ Spart, int nsplit, int p, int nbt,
                                                 TC *__restrict__ C)
{
    int bi, bj;
    tile_of(blockIdx.x, nbt, bi, bj);
    __shared__ double t[kNT][kNT + 1];
    __shared__ double di[kNT], dj[kNT];
    const size_t pp = (size_t)p * p;
    if (threadIdx.x < 2 * kNT) {  // S_aa of the tile's rows, then of its columns
        const int r = threadIdx.x % kNT, a = (threadIdx.x < kNT ? bi : bj) * kNT + r;
        double sa = 0.0;
        if (a < p)
            for (int k = 0; k < nsplit; ++k) sa += Spart[(size_t)k * pp + (size_t)a * p + a];
        (threadIdx.x < kNT ? di : dj)[r] = sa;
    }
    const int tx = threadIdx.x % kNT, ty = threadIdx.x / kNT;  // 8 rows of 32 per pass
    for (int r = ty; r < kNT; r += 8) {
        const int a = bi * kNT + r, b = bj * kNT + tx;
        double sab = 0.0;
        if (a < p && b < p)
            for (int k = 0; k < nsplit; ++k) sab += Spart[(size_t)k * pp + (size_t)a * p + b];
        t[r][tx] = sab;
    }
    __syncthreads();
    for (int r = ty; r < kNT; r += 8) {
        const int a = bi * kNT + r, b = bj * kNT + tx;
        // a diagonal tile reads its upper half for both halves
        const double sab = bi == bj && r > tx ? t[tx][r] : t[r][tx];
        if (a < p && b < p) C[(size_t)a * p + b] = a == b ? (TC)1.0 : (TC)(sab / sqrt(di[r] * dj[tx]));
    }
    if (bi != bj) {
        for (int r = ty; r < kNT; r += 8) {  // C[b][a] for the row b = bj*kNT + r
            const int b = bj * kNT + r, a = bi * kNT + tx;
            if (a < p && b < p) C[(size_t)b * p + a] = (TC)(t[tx][r] / sqrt(di[tx] * dj[r]));
        }
    }
}

// ---------------------------------------------------------------- bf16x3 on MFMA
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Standardise and split, writing the transposed copies Zh[j][t], Zl[j][t]
// (and Zm[j][t] for the three-way split; t < npad, zero beyond n) through a
// 32x32 LDS tile.  Two parts: z = hi + lo; three: z = hi + mid + lo, each
// part the bf16 rounding of what the parts before it leave.
template <typename TX, int NPART>
__global__ __launch_bounds__(256) void split_bf16(const TX *__restrict__ X, const double *__restrict__ mu,
                                                  const double *__restrict__ sd, int n, int p, int npad,
                                                  __bf16 *__restrict__ Zh, __bf16 *__restrict__ Zm,
                                                  __bf16 *__restrict__ Zl)
{
    __shared__ float tile[32][33];
    const int t0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int lx = threadIdx.x % 32, ly = threadIdx.x / 32;  // 32 x 8
    for (int r = ly; r < 32; r += 8) {
        const int t = t0 + r, j = j0 + lx;
        float z = 0.0f;
        if (t < n && j < p) z = (float)(((double)X[(size_t)t * p + j] - mu[j]) / sd[j]);
        tile[r][lx] = z;
    }
    __syncthreads();
    for (int r = ly; r < 32; r += 8) {
        const int j = j0 + r, t = t0 + lx;
        if (j < p && t < npad) {
            const float z = tile[lx][r];
            const __bf16 hi = (__bf16)z;
            const float r1 = z - (float)hi;  // exact: hi holds the leading 8 bits of z
            Zh[(size_t)j * npad + t] = hi;
            if constexpr (NPART == 2) {
                Zl[(size_t)j * npad + t] = (__bf16)r1;
            } else {
                const __bf16 mid = (__bf16)r1;
                Zm[(size_t)j * npad + t] = mid;
                Zl[(size_t)j * npad + t] = (__bf16)(r1 - (float)mid);
            }
        }
    }
}

// Samples per FP32 accumulation chunk before the fold into FP64: the
// rounding of the FP32 sums grows with the chunk, so the three-way split
// (whose products reach 2^-24) folds after every 32-sample step.
template <int NPROD>
constexpr int fold_samples() { return NPROD == 6 ? 32 : 512; }

// One 64x64 upper-triangle tile per block (4 waves, each 32x32 = 2x2 MFMA
// 16x16 tiles); blockIdx.y is the sample split.  Operand layout of
// v_mfma_f32_16x16x32_bf16: lane l supplies row (l % 16) and the 8
// consecutive k values 8*(l/16) .. 8*(l/16)+7; the result element r of
// lane l is row 4*(l/16) + r, column l % 16.
// NPROD = 3: hi.hi + hi.lo + lo.hi over the two-way split (Zm unused);
// NPROD = 6: hi.hi + hi.mid + mid.hi + mid.mid + hi.lo + lo.hi over the
// three-way split.
template <int NPROD>
__global__ __launch_bounds__(256) void syrk_bf16(const __bf16 *__restrict__ Zh, const __bf16 *__restrict__ Zm,
                                                 const __bf16 *__restrict__ Zl, int p, int npad,
                                                 int nbt, int chunk, double *__restrict__ Spart)
{
    constexpr bool three = NPROD == 6;
    int bi, bj;
    tile_of(blockIdx.x, nbt, bi, bj);
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wr = wave / 2, wc = wave % 2;
    const int k_lo = blockIdx.y * chunk, k_hi = min(npad, k_lo + chunk);
    const int rowA[2] = {bi * kT + wr * 32 + lane % 16, bi * kT + wr * 32 + 16 + lane % 16};
    const int rowB[2] = {bj * kT + wc * 32 + lane % 16, bj * kT + wc * 32 + 16 + lane % 16};
    const int koff = 8 * (lane / 16);
    double sum[2][2][4];
    floatx4 acc[2][2];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            acc[g][h] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 4; ++r) sum[g][h][r] = 0.0;
        }
    const bf16x8 zero = {};
    // operand fragments of the next 32-sample step are loaded while the
    // current step's products run
    bf16x8 nah[2], nam[2], nal[2], nbh[2], nbm[2], nbl[2];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const bool okA = rowA[g] < p && k0 < k_hi, okB = rowB[g] < p && k0 < k_hi;
            const size_t oA = (size_t)rowA[g] * npad + k0 + koff;
            const size_t oB = (size_t)rowB[g] * npad + k0 + koff;
            nah[g] = okA ? *reinterpret_cast<const bf16x8 *>(Zh + oA) : zero;
            nal[g] = okA ? *reinterpret_cast<const bf16x8 *>(Zl + oA) : zero;
            nbh[g] = okB ? *reinterpret_cast<const bf16x8 *>(Zh + oB) : zero;
            nbl[g] = okB ? *reinterpret_cast<const bf16x8 *>(Zl + oB) : zero;
            if constexpr (three) {
                nam[g] = okA ? *reinterpret_cast<const bf16x8 *>(Zm + oA) : zero;
                nbm[g] = okB ? *reinterpret_cast<const bf16x8 *>(Zm + oB) : zero;
            }
        }
    };
    fetch(k_lo);
    constexpr int kFold = fold_samples<NPROD>();
    for (int kc = k_lo; kc < k_hi; kc += kFold) {
        const int kend = min(k_hi, kc + kFold);
        for (int k0 = kc; k0 < kend; k0 += 32) {
            bf16x8 ah[2], am[2], al[2], bh[2], bm[2], bl[2];
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                ah[g] = nah[g];
                al[g] = nal[g];
                bh[g] = nbh[g];
                bl[g] = nbl[g];
                if constexpr (three) {
                    am[g] = nam[g];
                    bm[g] = nbm[g];
                }
            }
            fetch(k0 + 32);
            // smallest products first, so each lands on a smaller partial sum
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if constexpr (three) {
                        acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[g], bl[h], acc[g][h], 0, 0, 0);
                        acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[g], bh[h], acc[g][h], 0, 0, 0);
                        acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[g], bm[h], acc[g][h], 0, 0, 0);
                        acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[g], bm[h], acc[g][h], 0, 0, 0);
                        acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[g], bh[h], acc[g][h], 0, 0, 0);
                        acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[g], bh[h], acc[g][h], 0, 0, 0);
                    } else {
                        acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[g], bh[h], acc[g][h], 0, 0, 0);
                        acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[g], bl[h], acc[g][h], 0, 0, 0);
                        acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[g], bh[h], acc[g][h], 0, 0, 0);
                    }
                }
        }
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int r = 0; r < 4; ++r) sum[g][h][r] += (double)acc[g][h][r];
                acc[g][h] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
    }
    double *out = Spart + (size_t)blockIdx.y * p * p;
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = bi * kT + wr * 32 + g * 16 + 4 * (lane / 16) + r;
                const int j = bj * kT + wc * 32 + h * 16 + lane % 16;
                if (i < p && j < p) out[(size_t)i * p + j] = sum[g][h][r];
            }
}

__global__ __launch_bounds__(256) void max_abs_diff(const double *__restrict__ a, const float *__restrict__ b,
                                                    size_t cnt, unsigned long long *__restrict__ out)
{
    double m = 0.0;
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < cnt; k += (size_t)gridDim.x * 256)
        m = fmax(m, fabs(a[k] - (double)b[k]));
    __shared__ double red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ __launch_bounds__(256) void round_f32(const double *__restrict__ a, float *__restrict__ b, size_t cnt)
{
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < cnt; k += (size_t)gridDim.x * 256) b[k] = (float)a[k];
}

__global__ void fill_u32(uint32_t *__restrict__ p, int n, uint32_t v)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// Sample splits of a product: per_cu workgroups per CU in all, at most one
// split per 512 samples.  About 8 per CU let the global-load latency of the
// operand streams hide behind other waves: at p = 1000, n = 1e4 (136 tiles,
// 16 splits) the bf16x6 product takes 188 us and the FP64 one 247 us,
// against 245 and 331 us with 4 splits; the split sums cost 31 us to reduce.
int splits_for(int tiles, int n, int num_cus, int per_cu)
{
    int s = (per_cu * num_cus + tiles - 1) / tiles;
    s = s < 1 ? 1 : (s > 32 ? 32 : s);
    const int maxs = (n + 511) / 512;
    return s > maxs ? (maxs < 1 ? 1 : maxs) : s;
}

}  // namespace

// Device buffers corr_compute needs for one (n, p, method), grown now (a
// captured graph cannot allocate).
int corr_reserve(fpc_ctx *ctx, int n, int p, int method)
{
    const int nchunks = (n + kStatRows - 1) / kStatRows;
    const int nbt = (p + kT - 1) / kT, tiles = nbt * (nbt + 1) / 2;
    const int npad = (n + 31) / 32 * 32;
    const int nsplit = splits_for(tiles, method == FPC_CORR_FP64 ? n : npad, ctx->num_cus, 8);
    int rc = ctx->colstat.ensure(sizeof(double) * ((size_t)2 * p + (size_t)nchunks * 2 * p));
    if (!rc) rc = ctx->flag.ensure(64);
    if (!rc) rc = ctx->inv_work.ensure(sizeof(double) * (size_t)p * p * nsplit);
    if (!rc && (method == FPC_CORR_BF16X3 || method == FPC_CORR_BF16X6))
        rc = ctx->zsplit.ensure(sizeof(__bf16) * (method == FPC_CORR_BF16X6 ? 3 : 2) * (size_t)p * npad);
    return rc;
}

int corr_compute(fpc_ctx *ctx, const void *X, int x_dtype, int n, int p, int method, void *C_out, bool reuse_stats,
                 bool wait, bool keep_flags)
{
    if (!X || !C_out || n < 2 || p < 1) return FPC_EINVAL;
    if (x_dtype != FPC_F64 && x_dtype != FPC_F32) return FPC_EINVAL;
    if (method != FPC_CORR_FP64 && method != FPC_CORR_BF16X3 && method != FPC_CORR_BF16X6 && method != FPC_CORR_FP32)
        return FPC_EINVAL;
    if (method == FPC_CORR_FP32) {
        // the FP64 matrix, rounded: computed into the context's FP64 buffer
        // unless the caller's statistics and matrix are already there
        int rc = ctx->c64.ensure(sizeof(double) * (size_t)p * p);
        if (rc) return rc;
        if ((rc = corr_compute(ctx, X, x_dtype, n, p, FPC_CORR_FP64, ctx->c64.ptr, reuse_stats, false, keep_flags)))
            return rc;
        return corr_round_enqueue(ctx, ctx->c64.as<double>(), static_cast<float *>(C_out), p, wait);
    }
    hipStream_t st = ctx->stream;
    const int nchunks = (n + kStatRows - 1) / kStatRows;
    const int nbt = (p + kT - 1) / kT, tiles = nbt * (nbt + 1) / 2;
    const int npad = (n + 31) / 32 * 32;
    const int nsplit = splits_for(tiles, method == FPC_CORR_FP64 ? n : npad, ctx->num_cus, 8);
    const size_t pp = (size_t)p * p;
    // colstat layout: mu[p], sd[p], partials[nchunks * 2p]
    int rc = ctx->colstat.ensure(sizeof(double) * ((size_t)2 * p + (size_t)nchunks * 2 * p));
    if (rc) return rc;
    if ((rc = ctx->flag.ensure(64))) return rc;
    if ((rc = ctx->inv_work.ensure(sizeof(double) * pp * nsplit))) return rc;
    double *mu = ctx->colstat.as<double>(), *sd = mu + p, *part = sd + p;
    int *flags = ctx->flag.as<int>();
    double *Spart = ctx->inv_work.as<double>();
    dim3 g0((p + 255) / 256, nchunks);
    // column means and deviations (kept from the previous call on the same
    // data when reuse_stats is set)
    if (!reuse_stats) {
        if (!keep_flags) fill_u32<<<1, 32, 0, st>>>(reinterpret_cast<uint32_t *>(flags), 2, 0u);
        if (x_dtype == FPC_F64) {
            colstat_partial<double><<<g0, 256, 0, st>>>((const double *)X, n, p, part, flags);
            colstat_reduce<double><<<(p + 63) / 64, 256, 0, st>>>((const double *)X, part, nchunks, n, p, mu, sd,
                                                                    flags + 1);
        } else {
            colstat_partial<float><<<g0, 256, 0, st>>>((const float *)X, n, p, part, flags);
            colstat_reduce<float><<<(p + 63) / 64, 256, 0, st>>>((const float *)X, part, nchunks, n, p, mu, sd,
                                                                   flags + 1);
        }
    }
    FPC_HIP(hipGetLastError());
    if (method == FPC_CORR_FP64) {
        const int chunk = ((n + nsplit - 1) / nsplit + kK - 1) / kK * kK;
        dim3 g(tiles, nsplit);
        if (x_dtype == FPC_F64)
            syrk_f64<double><<<g, 256, 0, st>>>((const double *)X, mu, n, p, nbt, chunk, Spart);
        else
            syrk_f64<float><<<g, 256, 0, st>>>((const float *)X, mu, n, p, nbt, chunk, Spart);
        const int nbn = (p + kNT - 1) / kNT;
        normalize<double><<<nbn * (nbn + 1) / 2, 256, 0, st>>>(Spart, nsplit, p, nbn, (double *)C_out);
    } else {
        const bool three = method == FPC_CORR_BF16X6;
        const int nparts = three ? 3 : 2;
        if ((rc = ctx->zsplit.ensure(sizeof(__bf16) * nparts * (size_t)p * npad))) return rc;
        __bf16 *Zh = ctx->zsplit.as<__bf16>(), *Zl = Zh + (size_t)p * npad;
        __bf16 *Zm = three ? Zl + (size_t)p * npad : nullptr;
        dim3 gs(npad / 32, (p + 31) / 32);
        if (three) {
            if (x_dtype == FPC_F64)
                split_bf16<double, 3><<<gs, 256, 0, st>>>((const double *)X, mu, sd, n, p, npad, Zh, Zm, Zl);
            else
                split_bf16<float, 3><<<gs, 256, 0, st>>>((const float *)X, mu, sd, n, p, npad, Zh, Zm, Zl);
        } else {
            if (x_dtype == FPC_F64)
                split_bf16<double, 2><<<gs, 256, 0, st>>>((const double *)X, mu, sd, n, p, npad, Zh, Zm, Zl);
            else
                split_bf16<float, 2><<<gs, 256, 0, st>>>((const float *)X, mu, sd, n, p, npad, Zh, Zm, Zl);
        }
        const int chunk = ((npad + nsplit - 1) / nsplit + 31) / 32 * 32;
        dim3 g(tiles, nsplit);
        if (three) syrk_bf16<6><<<g, 256, 0, st>>>(Zh, Zm, Zl, p, npad, nbt, chunk, Spart);
        else syrk_bf16<3><<<g, 256, 0, st>>>(Zh, Zm, Zl, p, npad, nbt, chunk, Spart);
        const int nbn = (p + kNT - 1) / kNT;
        normalize<float><<<nbn * (nbn + 1) / 2, 256, 0, st>>>(Spart, nsplit, p, nbn, (float *)C_out);
    }
    FPC_HIP(hipGetLastError());
    return wait ? corr_check(ctx, nullptr) : FPC_OK;
}

int corr_check(fpc_ctx *ctx, double *max_abs_diff)
{
    // flag words: [0] non-finite input, [1] constant column; bytes 32..39 the
    // largest |C64 - C32| as FP64 bits
    int rc = ctx->h_flag.ensure(64);
    if (rc) return rc;
    char *h = ctx->h_flag.as<char>();
    FPC_HIP(hipMemcpyAsync(h, ctx->flag.ptr, 40, hipMemcpyDeviceToHost, ctx->stream));
    FPC_HIP(hipStreamSynchronize(ctx->stream));
    int hflags[2];
    memcpy(hflags, h, sizeof(hflags));
    if (max_abs_diff) memcpy(max_abs_diff, h + 32, sizeof(double));
    if (hflags[0]) return FPC_ENONFINITE;
    if (hflags[1]) return FPC_ESINGULAR;
    return FPC_OK;
}

namespace {

// out[r][:] = X[rows[r]][:] (a resample of the rows); an index outside
// [0, x_rows) sets *bad and leaves the row unwritten.  One workgroup per
// row at a time, lanes along the row.
template <typename TX>
__global__ __launch_bounds__(256) void gather_rows_kernel(const TX *__restrict__ X, int64_t x_rows, int p,
                                                          const int32_t *__restrict__ rows, int n,
                                                          TX *__restrict__ out, int *__restrict__ bad)
{
    for (int r = blockIdx.x; r < n; r += gridDim.x) {
        const int32_t src = rows[r];
        if (src < 0 || (int64_t)src >= x_rows) {
            if (threadIdx.x == 0) atomicOr(bad, 1);
            continue;
        }
        for (int j = threadIdx.x; j < p; j += 256) out[(size_t)r * p + j] = X[(size_t)src * p + j];
    }
}

}  // namespace

int gather_rows_enqueue(fpc_ctx *ctx, const void *X, int x_dtype, int64_t x_rows, int p, const int32_t *rows, int n,
                        void *out, int *bad)
{
    if (!X || !rows || !out || p < 1 || n < 1 || !bad) return FPC_EINVAL;
    hipStream_t st = ctx->stream;
    const unsigned g = (unsigned)std::min(n, 8 * ctx->num_cus);
    if (x_dtype == FPC_F64)
        gather_rows_kernel<double><<<g, 256, 0, st>>>((const double *)X, x_rows, p, rows, n, (double *)out, bad);
    else
        gather_rows_kernel<float><<<g, 256, 0, st>>>((const float *)X, x_rows, p, rows, n, (float *)out, bad);
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

int gather_rows(fpc_ctx *ctx, const void *X, int x_dtype, int64_t x_rows, int p, const int32_t *rows, int n,
                void *out)
{
    if (!X || !rows || !out || p < 1 || n < 1) return FPC_EINVAL;
    hipStream_t st = ctx->stream;
    int rc = ctx->flag.ensure(64);
    if (rc) return rc;
    int *bad = ctx->flag.as<int>() + 8;
    FPC_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    const unsigned g = (unsigned)std::min(n, 8 * ctx->num_cus);
    if (x_dtype == FPC_F64)
        gather_rows_kernel<double><<<g, 256, 0, st>>>((const double *)X, x_rows, p, rows, n, (double *)out, bad);
    else
        gather_rows_kernel<float><<<g, 256, 0, st>>>((const float *)X, x_rows, p, rows, n, (float *)out, bad);
    FPC_HIP(hipGetLastError());
    int h = 0;
    FPC_HIP(hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    FPC_HIP(hipStreamSynchronize(st));
    return h ? FPC_EINVAL : FPC_OK;
}

int corr_round_enqueue(fpc_ctx *ctx, const double *c64, float *c32, int p, bool wait)
{
    const size_t cnt = (size_t)p * p;
    round_f32<<<(unsigned)std::min<size_t>((cnt + 255) / 256, 2048), 256, 0, ctx->stream>>>(c64, c32, cnt);
    FPC_HIP(hipGetLastError());
    return wait ? corr_check(ctx, nullptr) : FPC_OK;
}

int corr_max_abs_diff_enqueue(fpc_ctx *ctx, const double *c64, const float *c32, int p, unsigned long long *slot)
{
    int rc = ctx->flag.ensure(64);
    if (rc) return rc;
    unsigned long long *d = slot ? slot : reinterpret_cast<unsigned long long *>(ctx->flag.as<char>() + 32);
    fill_u32<<<1, 32, 0, ctx->stream>>>(reinterpret_cast<uint32_t *>(d), 2, 0u);
    max_abs_diff<<<512, 256, 0, ctx->stream>>>(c64, c32, (size_t)p * p, d);
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

}  // namespace fpc

extern "C" int fpc_corr(fpc_ctx *ctx, const void *X, int x_dtype, int n, int p, int method, void *C_out)
{
    if (!ctx) return FPC_EINVAL;
    return fpc::corr_compute(ctx, X, x_dtype, n, p, method, C_out);
}
