// First reverse level of Algorithm 2 (l = p-2, Sec. 3.2): on the complete
// graph every pair (i,j) is conditioned on all other variables.  By the
// Sec. 5 formula with K = V \ {i,j}, the 2x2 matrix H is the inverse of the
// {i,j} block of Omega = C^{-1}, so r_ij = -Omega_ij / sqrt(Omega_ii Omega_jj):
// one p x p FP64 inversion replaces p(p-1)/2 factorisations of size p-2.
//
// Omega is formed by a blocked sweep (Gauss-Jordan without pivoting, valid
// for a positive definite C).  For each panel K of kNB columns, with
// V = A[:,K] and U = A[K,K]^{-1} A[K,:] taken before the update:
//     A[I,J] -= V[I,:] U[:,J]          (I, J outside K)
//     A[I,K]  = -V[I,:] A[K,K]^{-1}     (I outside K)
//     A[K,J]  = U[:,J]                 (J outside K)
//     A[K,K]  = A[K,K]^{-1}
// After the last panel A = C^{-1}.  A non-positive pivot inside a panel
// inverse reports the matrix as not positive definite.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fpc_internal.h"

namespace fpc {

namespace {

constexpr int kNB = 32;
constexpr int kUT = 32;  // update tile

// Invert the nb x nb diagonal block at k0 in LDS (Gauss-Jordan, no pivoting).
__global__ __launch_bounds__(1024) void panel_inverse(const double *__restrict__ A, int p, int k0, int nb,
                                                      double *__restrict__ Pinv, int *__restrict__ bad)
{
    __shared__ double P[kNB][kNB + 1];
    __shared__ double rowk[kNB], colk[kNB];
    const int r = threadIdx.x / kNB, c = threadIdx.x % kNB;
    if (r < nb && c < nb) P[r][c] = A[(size_t)(k0 + r) * p + k0 + c];
    __syncthreads();
    for (int t = 0; t < nb; ++t) {
        const double piv = P[t][t];
        if (!(piv > 0.0)) {
            if (threadIdx.x == 0) atomicOr(bad, 1);
            return;  // uniform: every thread read the same pivot
        }
        if (r == 0 && c < nb) {
            rowk[c] = P[t][c];
            colk[c] = P[c][t];
        }
        __syncthreads();
        const double ip = 1.0 / piv;
        if (r < nb && c < nb) {
            double v;
            if (r == t && c == t) v = ip;
            else if (r == t) v = rowk[c] * ip;
            else if (c == t) v = -colk[r] * ip;
            else v = P[r][c] - colk[r] * rowk[c] * ip;
            P[r][c] = v;
        }
        __syncthreads();
    }
    // the whole kNB x kNB block, zero outside nb, so later passes may run
    // over kNB terms
    Pinv[r * kNB + c] = (r < nb && c < nb) ? P[r][c] : 0.0;
}

// U = Pinv A[K,:] (nb x p): a block takes 64 columns (lanes, coalesced
// rows of A) and kNB/4 panel rows (blockIdx.y); the panel column of A sits
// in registers.
__global__ __launch_bounds__(256) void panel_u(const double *__restrict__ A, int p, int k0, int nb,
                                               const double *__restrict__ Pinv, double *__restrict__ U)
{
    const int j = blockIdx.x * 64 + threadIdx.x % 64;
    if (j >= p) return;
    double a[kNB];
#pragma unroll
    for (int c = 0; c < kNB; ++c) a[c] = c < nb ? A[(size_t)(k0 + c) * p + j] : 0.0;
    const int r0 = blockIdx.y * (kNB / 4);
    for (int r = r0 + threadIdx.x / 64; r < r0 + kNB / 4 && r < nb; r += 4) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < kNB; ++c) s = fma(Pinv[r * kNB + c], a[c], s);
        U[(size_t)r * p + j] = s;
    }
}

// V = A[:,K] (p x kNB, row stride kNB): 8 rows per block, the panel
// columns along the low 5 bits of the thread index (coalesced).
__global__ __launch_bounds__(256) void panel_v(const double *__restrict__ A, int p, int k0, int nb,
                                               double *__restrict__ V)
{
    const int j = blockIdx.x * 8 + threadIdx.x / 32, r = threadIdx.x % 32;
    if (j < p && r < nb) V[(size_t)j * kNB + r] = A[(size_t)j * p + k0 + r];
}

// The sweep update over kUT x kUT tiles of A; lanes along the columns j
// (coalesced), each thread four rows.
__global__ __launch_bounds__(256) void sweep_update(double *__restrict__ A, int p, int k0, int nb,
                                                    const double *__restrict__ V, const double *__restrict__ U,
                                                    const double *__restrict__ Pinv)
{
    __shared__ double Vs[kUT][kNB + 1];
    __shared__ double Us[kNB][kUT + 1];
    const int i0 = blockIdx.y * kUT, j0 = blockIdx.x * kUT;
    for (int e = threadIdx.x; e < kUT * kNB; e += 256) {
        const int r = e / kNB, c = e % kNB, i = i0 + r;
        Vs[r][c] = (i < p && c < nb) ? V[(size_t)i * kNB + c] : 0.0;
    }
    for (int e = threadIdx.x; e < kNB * kUT; e += 256) {
        const int r = e / kUT, c = e % kUT, j = j0 + c;
        Us[r][c] = (j < p && r < nb) ? U[(size_t)r * p + j] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x % kUT, ty = threadIdx.x / kUT;  // 32 x 8
    const int j = j0 + tx;
    if (j >= p) return;  // no barrier follows
    const bool inK_j = j >= k0 && j < k0 + nb;
#pragma unroll
    for (int q = 0; q < kUT / 8; ++q) {
        const int ri = ty + 8 * q, i = i0 + ri;
        if (i >= p) break;
        const bool inK_i = i >= k0 && i < k0 + nb;
        double v;
        if (inK_i && inK_j) {
            v = Pinv[(i - k0) * kNB + (j - k0)];
        } else if (inK_i) {
            v = Us[i - k0][tx];
        } else if (inK_j) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < kNB; ++c) acc = fma(Vs[ri][c], Pinv[c * kNB + (j - k0)], acc);
            v = -acc;
        } else {
            double acc = A[(size_t)i * p + j];
#pragma unroll
            for (int c = 0; c < kNB; ++c) acc = fma(-Vs[ri][c], Us[c][tx], acc);
            v = acc;
        }
        A[(size_t)i * p + j] = v;
    }
}

// r_ij = -Omega_ij / sqrt(Omega_ii Omega_jj) (symmetrised), z, decision.
__global__ __launch_bounds__(256) void first_level_decide(const double *__restrict__ Om, int p, int n, double q,
                                                          double *__restrict__ r_out,
                                                          uint8_t *__restrict__ indep_out, int *__restrict__ bad)
{
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)p * p) return;
    const int i = (int)(idx / p), j = (int)(idx % p);
    if (i == j) {
        // Omega_ii = 1 / (1 - R^2_i): a variable determined by the others
        // (1 - R^2 < 1e-12) makes C singular for the tests.
        if (!(Om[idx] > 0.0) || !(Om[idx] <= 1e12)) atomicOr(bad, 1);
        if (r_out) r_out[idx] = 1.0;
        if (indep_out) indep_out[idx] = 0;
        return;
    }
    const double oij = 0.5 * (Om[(size_t)i * p + j] + Om[(size_t)j * p + i]);
    const double r = -oij / sqrt(Om[(size_t)i * p + i] * Om[(size_t)j * p + j]);
    if (r_out) r_out[idx] = r;
    if (indep_out) {
        const int l = p - 2;
        uint8_t ind = 0;
        if (fabs(r) < 1.0) {
            const double z = sqrt((double)(n - l - 3)) * fabs(atanh(r));
            ind = z <= q;
        }
        indep_out[idx] = ind;
    }
}

}  // namespace

int first_level_enqueue(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out,
                        uint8_t *indep_out, const int **d_bad)
{
    if (!C || p < 2 || n <= p + 1) return FPC_EINVAL;
    hipStream_t st = ctx->stream;
    const size_t pp = (size_t)p * p;
    // work: A (p*p), V (p*kNB), U (kNB*p), Pinv (kNB*kNB)
    int rc = ctx->inv_work.ensure(sizeof(double) * (pp + 2 * (size_t)p * kNB + kNB * kNB));
    if (rc) return rc;
    if ((rc = ctx->flag.ensure(64))) return rc;
    double *A = ctx->inv_work.as<double>(), *V = A + pp, *U = V + (size_t)p * kNB, *Pinv = U + (size_t)kNB * p;
    int *bad = ctx->flag.as<int>() + 4;
    FPC_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    FPC_HIP(hipMemcpyAsync(A, C, sizeof(double) * pp, hipMemcpyDeviceToDevice, st));
    const int nbt = (p + kUT - 1) / kUT;
    for (int k0 = 0; k0 < p; k0 += kNB) {
        const int nb = p - k0 < kNB ? p - k0 : kNB;
        panel_inverse<<<1, 1024, 0, st>>>(A, p, k0, nb, Pinv, bad);
        panel_u<<<dim3((p + 63) / 64, 4), 256, 0, st>>>(A, p, k0, nb, Pinv, U);
        panel_v<<<(p + 7) / 8, 256, 0, st>>>(A, p, k0, nb, V);
        sweep_update<<<dim3(nbt, nbt), 256, 0, st>>>(A, p, k0, nb, V, U, Pinv);
    }
    first_level_decide<<<(unsigned)((pp + 255) / 256), 256, 0, st>>>(A, p, n, q, r_out, indep_out, bad);
    FPC_HIP(hipGetLastError());
    *d_bad = bad;
    return FPC_OK;
}

int first_level(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out, uint8_t *indep_out,
                int *n_singular)
{
    const int *bad = nullptr;
    int rc = first_level_enqueue(ctx, C, p, n, q, r_out, indep_out, &bad);
    if (rc) return rc;
    int hbad = 0;
    FPC_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    FPC_HIP(hipStreamSynchronize(ctx->stream));
    if (n_singular) *n_singular = hbad;
    return hbad ? FPC_ESINGULAR : FPC_OK;
}

}  // namespace fpc

extern "C" int fpc_first_level(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out,
                               uint8_t *indep_out)
{
    if (!ctx) return FPC_EINVAL;
    return fpc::first_level(ctx, C, p, n, q, r_out, indep_out, nullptr);
}
