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
//
// One launch per panel: the sweep reads the matrix before the panel and
// writes a second buffer (the two alternate), so each kNB x kNB tile can
// form its own slice of U and read its slice of V; the tile that becomes
// the next panel's diagonal block inverts it in the same launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fpc_internal.h"

namespace fpc {

namespace {

constexpr int kNB = 32;  // panel width and tile size

// Gauss-Jordan inverse of the nb x nb block P (LDS, kNB x kNB tile) by a
// 256-thread block, thread (ty, tx) owning rows ty + 8q of column tx.  Two
// pivots per step: the 2 x 2 pivot block K2 = {t, t+1} is inverted in
// closed form and eliminated as one block (the sweep formulas above with a
// panel of two), with a single pivot for an odd last one.  The next step's
// pivot rows and columns are published into a second buffer by the threads
// that compute them, so each step needs one barrier.  Writes the whole
// kNB x kNB result (zero outside nb) to Pinv.
__device__ void tile_inverse(double (*P)[kNB + 1], double (*rowk)[2][kNB], double (*colk)[2][kNB], int nb,
                             double *__restrict__ Pinv, int *__restrict__ bad)
{
    const int tx = threadIdx.x % kNB, ty = threadIdx.x / kNB;
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = P[ty + 8 * q][tx];
    // the first step's pivot rows and columns
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        if (r < 2) rowk[0][r][tx] = v[q];
        if (tx < 2) colk[0][tx][r] = v[q];
    }
    __syncthreads();
    bool ok = true;
    int b = 0;
    for (int t = 0; t < nb;) {
        const bool two = t + 1 < nb;  // uniform
        const int c = tx;
        const double r1 = rowk[b][0][c], r2 = rowk[b][1][c];
        double c1[4], c2[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c1[q] = colk[b][0][ty + 8 * q];
            c2[q] = colk[b][1][ty + 8 * q];
        }
        if (two) {
            const double a = rowk[b][0][t], bt = rowk[b][0][t + 1], ct = rowk[b][1][t], d = rowk[b][1][t + 1];
            const double det = a * d - bt * ct;
            ok = ok && a > 0.0 && det > 0.0;
            const double idet = 1.0 / det;
            const double i00 = d * idet, i01 = -bt * idet, i10 = -ct * idet, i11 = a * idet;
            const double u1 = fma(i00, r1, i01 * r2), u2 = fma(i10, r1, i11 * r2);  // inv(K2) A[K2, c]
            const bool inC = c == t || c == t + 1;
            const double ic0 = c == t ? i00 : i01, ic1 = c == t ? i10 : i11;   // column c - t of inv(K2)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = ty + 8 * q;
                const bool inR = r == t || r == t + 1;
                double nv = fma(-c1[q], u1, fma(-c2[q], u2, v[q]));
                nv = inC ? -fma(c1[q], ic0, c2[q] * ic1) : nv;
                nv = inR ? (r == t ? u1 : u2) : nv;
                nv = (inR && inC) ? (r == t ? ic0 : ic1) : nv;
                v[q] = (r < nb && c < nb) ? nv : v[q];
            }
            t += 2;
        } else {
            const double piv = rowk[b][0][t];
            ok = ok && piv > 0.0;
            const double ip = 1.0 / piv, rti = r1 * ip;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = ty + 8 * q;
                double nv = fma(-c1[q], rti, v[q]);
                nv = c == t ? -c1[q] * ip : nv;
                nv = r == t ? rti : nv;
                nv = (r == t && c == t) ? ip : nv;
                v[q] = (r < nb && c < nb) ? nv : v[q];
            }
            t += 1;
        }
        b ^= 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ty + 8 * q;
            if (r == t) rowk[b][0][c] = v[q];
            if (r == t + 1) rowk[b][1][c] = v[q];
            if (c == t) colk[b][0][r] = v[q];
            if (c == t + 1) colk[b][1][r] = v[q];
        }
        __syncthreads();
    }
    if (!ok && threadIdx.x == 0) atomicOr(bad, 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        Pinv[r * kNB + tx] = (r < nb && tx < nb) ? v[q] : 0.0;
    }
}

typedef double v4d __attribute__((ext_vector_type(4)));

// One panel of the sweep over kNB x kNB tiles, from Ain to Aout.  The block
// of tile (I, J) stages Pinv = A[K,K]^{-1}, A[K,J] and V = A[I,K] in LDS,
// forms U[:,J] = Pinv A[K,J] and writes its tile of the updated matrix.
// The products run on the FP64 matrix cores: each wave owns a 16 x 16
// quarter, v_mfma_f64_16x16x4f64 with lane l feeding A[l%16][l/16] and
// B[l/16][l%16] and holding D[4v + l/16][l%16] in accumulator v.  The tile
// at (next_k0, next_k0), if any, then inverts its new values into
// Pinv_next.
__device__ __forceinline__ void sweep_tile(const double *__restrict__ Ain, double *__restrict__ Aout, int p, int k0,
                                           int nb, const double *__restrict__ Pinv, int next_k0, int next_nb,
                                           double *__restrict__ Pinv_next, int *__restrict__ bad, int i0, int j0)
{
    __shared__ double Ps[kNB][kNB + 1];
    __shared__ double Us[kNB][kNB + 1];
    __shared__ double Vs[kNB][kNB + 1];
    __shared__ double rowk[2][2][kNB], colk[2][2][kNB];
    const int tx = threadIdx.x % kNB, ty = threadIdx.x / kNB;  // 32 x 8
    const int j = j0 + tx;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q, i = i0 + r;
        Ps[r][tx] = Pinv[r * kNB + tx];  // zero outside nb
        Us[r][tx] = (r < nb && j < p) ? Ain[(size_t)(k0 + r) * p + j] : 0.0;
        Vs[r][tx] = (i < p && tx < nb) ? Ain[(size_t)i * p + k0 + tx] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int qr = (wave / 2) * 16, qc = (wave % 2) * 16;  // the wave's quarter
    const int ar = qr + lane % 16, bc = qc + lane % 16, kq = lane / 16;
    const bool rowK = i0 == k0, colK = j0 == k0;  // tile row / column of the panel (uniform)
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    if (rowK && colK) {  // A[K,K] <- Pinv
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = Ps[qr + 4 * v + kq][bc];
    } else if (colK) {  // A[I,K] <- -V Pinv
#pragma unroll
        for (int s4 = 0; s4 < kNB; s4 += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-Vs[ar][s4 + kq], Ps[s4 + kq][bc], acc, 0, 0, 0);
    } else {
        // U quarter = Pinv[qr.., :] A[K, qc..]
        v4d u = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < kNB; s4 += 4)
            u = __builtin_amdgcn_mfma_f64_16x16x4f64(Ps[ar][s4 + kq], Us[s4 + kq][bc], u, 0, 0, 0);
        if (rowK) {  // A[K,J] <- U
            acc = u;
        } else {  // A[I,J] <- A[I,J] - V U
            __syncthreads();  // every read of A[K,J] is done (uniform branch)
#pragma unroll
            for (int v = 0; v < 4; ++v) Us[qr + 4 * v + kq][bc] = u[v];
            __syncthreads();
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + qr + 4 * v + kq, jj = j0 + bc;
                acc[v] = (i < p && jj < p) ? Ain[(size_t)i * p + jj] : 0.0;
            }
#pragma unroll
            for (int s4 = 0; s4 < kNB; s4 += 4)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-Vs[ar][s4 + kq], Us[s4 + kq][bc], acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = i0 + qr + 4 * v + kq, jj = j0 + bc;
        if (i < p && jj < p) Aout[(size_t)i * p + jj] = acc[v];
    }
    if (next_nb > 0 && i0 == next_k0 && j0 == next_k0) {  // uniform over the block
        __syncthreads();  // Ps is free again
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Ps[qr + 4 * v + kq][bc] = (i0 + qr + 4 * v + kq < p && j0 + bc < p) ? acc[v] : 0.0;
        __syncthreads();
        tile_inverse(Ps, rowk, colk, next_nb, Pinv_next, bad);
    }
}

__global__ __launch_bounds__(256) void sweep_panel(const double *__restrict__ Ain, double *__restrict__ Aout, int p,
                                                   int k0, int nb, const double *__restrict__ Pinv,
                                                   int next_k0, int next_nb, double *__restrict__ Pinv_next,
                                                   int *__restrict__ bad)
{
    sweep_tile(Ain, Aout, p, k0, nb, Pinv, next_k0, next_nb, Pinv_next, bad, blockIdx.y * kNB, blockIdx.x * kNB);
}

// ---------------------------------------------------------------- many instances
// Panel t of every instance with p > 32 t in one launch: job q covers
// tiles [tile0[q], tile0[q] + nbt^2) of the flattened grid.
__global__ __launch_bounds__(256) void sweep_panel_batch(const SweepJob *__restrict__ jobs, int njobs)
{
    int lo = 0, hi = njobs;  // jobs[lo].tile0 <= blockIdx.x < jobs[hi].tile0
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jobs[mid].tile0 <= (int64_t)blockIdx.x) lo = mid;
        else hi = mid;
    }
    const SweepJob J = jobs[lo];
    const int t = (int)((int64_t)blockIdx.x - J.tile0);
    sweep_tile(J.Ain, J.Aout, J.p, J.k0, J.nb, J.Pinv, J.next_k0, J.next_nb, J.Pinv_next, J.bad, (t / J.nbt) * kNB,
               (t % J.nbt) * kNB);
}

// First panel's diagonal block of every instance (one block each).
__global__ __launch_bounds__(256) void first_tile_inverse_batch(const SweepJob *__restrict__ jobs)
{
    const SweepJob J = jobs[blockIdx.x];
    __shared__ double Ps[kNB][kNB + 1];
    __shared__ double rowk[2][2][kNB], colk[2][2][kNB];
    const int tx = threadIdx.x % kNB, ty = threadIdx.x / kNB;
    const int nb = J.p < kNB ? J.p : kNB;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        Ps[r][tx] = (r < nb && tx < nb) ? J.Ain[(size_t)r * J.p + tx] : 0.0;
    }
    __syncthreads();
    tile_inverse(Ps, rowk, colk, nb, const_cast<double *>(J.Pinv), J.bad);  // this job writes the inverse
}

// Decisions of every instance: adjacency byte = edge kept (not independent),
// zero diagonal; deletions counted per instance; the Omega_ii rule of the
// single-instance decision sets the instance's flag.
__global__ __launch_bounds__(256) void first_level_decide_batch(const DecideJob *__restrict__ jobs, int njobs)
{
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jobs[mid].elem0 <= (int64_t)blockIdx.x * 256) lo = mid;
        else hi = mid;
    }
    const DecideJob J = jobs[lo];
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x - J.elem0;
    const int64_t pp = (int64_t)J.p * J.p;
    bool del = false;
    if (idx >= 0 && idx < pp) {
        const int i = (int)(idx / J.p), j = (int)(idx % J.p);
        const double *Om = J.Om;
        if (i == j) {
            if (!(Om[idx] > 0.0) || !(Om[idx] <= 1e12)) atomicOr(J.bad, 1);
            J.adj[idx] = 0;
        } else {
            const double oij = 0.5 * (Om[(size_t)i * J.p + j] + Om[(size_t)j * J.p + i]);
            const double r = -oij / sqrt(Om[(size_t)i * J.p + i] * Om[(size_t)j * J.p + j]);
            uint8_t ind = 0;
            if (fabs(r) < 1.0) ind = sqrt((double)(J.n - (J.p - 2) - 3)) * fabs(atanh(r)) <= J.q;
            J.adj[idx] = ind ? 0 : 1;
            del = ind && i < j;
        }
    }
    const unsigned long long b = __ballot(del);
    if (b && threadIdx.x % 64 == __ffsll((long long)b) - 1) atomicAdd(J.deleted, (unsigned long long)__popcll(b));
}

// Inverse of the first panel's diagonal block.
__global__ __launch_bounds__(256) void first_tile_inverse(const double *__restrict__ A, int p, int nb,
                                                          double *__restrict__ Pinv, int *__restrict__ bad)
{
    __shared__ double Ps[kNB][kNB + 1];
    __shared__ double rowk[2][2][kNB], colk[2][2][kNB];
    const int tx = threadIdx.x % kNB, ty = threadIdx.x / kNB;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        Ps[r][tx] = (r < nb && tx < nb) ? A[(size_t)r * p + tx] : 0.0;
    }
    __syncthreads();
    tile_inverse(Ps, rowk, colk, nb, Pinv, bad);
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

__global__ void clear_flag(int *__restrict__ f) { *f = 0; }

// The sweep, the decisions and the positive-definiteness flag, queued on
// the context's stream, with the workspace given: two p x p buffers (the
// sweep reads one and writes the other), two kNB x kNB panel inverses and
// the flag word (cleared by a kernel here when clear_bad is set).
int first_level_enqueue_ws(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out, uint8_t *indep_out,
                           double *buf0, double *buf1, double *pinv0, double *pinv1, int *bad, bool clear_bad)
{
    hipStream_t st = ctx->stream;
    const size_t pp = (size_t)p * p;
    double *buf[2] = {buf0, buf1};
    double *pinv[2] = {pinv0, pinv1};
    if (clear_bad) clear_flag<<<1, 1, 0, st>>>(bad);
    const int nbt = (p + kNB - 1) / kNB;
    first_tile_inverse<<<1, 256, 0, st>>>(C, p, p < kNB ? p : kNB, pinv[0], bad);
    const double *Ain = C;
    int t = 0;
    for (int k0 = 0; k0 < p; k0 += kNB, ++t) {
        const int nb = p - k0 < kNB ? p - k0 : kNB;
        const int nk = k0 + kNB, nnb = nk < p ? (p - nk < kNB ? p - nk : kNB) : 0;
        sweep_panel<<<dim3(nbt, nbt), 256, 0, st>>>(Ain, buf[t & 1], p, k0, nb, pinv[t & 1], nk, nnb,
                                                     pinv[(t + 1) & 1], bad);
        Ain = buf[t & 1];
    }
    first_level_decide<<<(unsigned)((pp + 255) / 256), 256, 0, st>>>(Ain, p, n, q, r_out, indep_out, bad);
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

}  // namespace

int first_level_batch_enqueue(fpc_ctx *ctx, const std::vector<FirstLevelInst> &in, const FirstLevelBatchBufs &b)
{
    hipStream_t st = ctx->stream;
    const int ni = (int)in.size();
    int maxp = 0;
    for (const auto &I : in) maxp = std::max(maxp, I.p);
    const int npanels = (maxp + kNB - 1) / kNB;
    // job tables for every panel step (uploaded by the caller beforehand)
    for (int k = 0; k < ni; ++k) {
        if (in[k].p < 2) return FPC_EINVAL;
    }
    first_tile_inverse_batch<<<ni, 256, 0, st>>>(b.first_jobs);
    for (int t = 0; t < npanels; ++t) {
        const int nj = b.panel_njobs[t];
        if (nj == 0) continue;
        sweep_panel_batch<<<(unsigned)b.panel_tiles[t], 256, 0, st>>>(b.panel_jobs + b.panel_job0[t], nj);
    }
    first_level_decide_batch<<<(unsigned)((b.decide_elems + 255) / 256), 256, 0, st>>>(b.decide_jobs, ni);
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

// Host side of the job tables: fills `jobs_host` (first-tile jobs, then the
// panel jobs of every step, then the decision jobs) for instances whose
// matrices, buffers and outputs are given, and the launch shapes.
int first_level_batch_plan(const std::vector<FirstLevelInst> &in, std::vector<SweepJob> &first,
                           std::vector<SweepJob> &panels, std::vector<int> &panel_job0, std::vector<int> &panel_njobs,
                           std::vector<int64_t> &panel_tiles, std::vector<DecideJob> &decide, int64_t &decide_elems)
{
    int maxp = 0;
    for (const auto &I : in) maxp = std::max(maxp, I.p);
    const int npanels = (maxp + kNB - 1) / kNB;
    first.clear();
    panels.clear();
    decide.clear();
    panel_job0.assign(npanels, 0);
    panel_njobs.assign(npanels, 0);
    panel_tiles.assign(npanels, 0);
    for (const auto &I : in) {
        SweepJob J{};
        J.Ain = I.C;
        J.p = I.p;
        J.Pinv = I.pinv0;
        J.bad = I.bad;
        first.push_back(J);
    }
    for (int t = 0; t < npanels; ++t) {
        panel_job0[t] = (int)panels.size();
        int64_t tiles = 0;
        for (const auto &I : in) {
            const int k0 = t * kNB;
            if (k0 >= I.p) continue;
            SweepJob J{};
            J.Ain = t == 0 ? I.C : (t & 1 ? I.buf0 : I.buf1);
            J.Aout = t & 1 ? I.buf1 : I.buf0;
            J.p = I.p;
            J.k0 = k0;
            J.nb = std::min(kNB, I.p - k0);
            J.Pinv = t & 1 ? I.pinv1 : I.pinv0;
            J.next_k0 = k0 + kNB;
            J.next_nb = J.next_k0 < I.p ? std::min(kNB, I.p - J.next_k0) : 0;
            J.Pinv_next = t & 1 ? I.pinv0 : I.pinv1;
            J.bad = I.bad;
            J.nbt = (I.p + kNB - 1) / kNB;
            J.tile0 = tiles;
            tiles += (int64_t)J.nbt * J.nbt;
            panels.push_back(J);
        }
        panel_njobs[t] = (int)panels.size() - panel_job0[t];
        panel_tiles[t] = tiles;
    }
    int64_t elems = 0;
    for (const auto &I : in) {
        DecideJob D{};
        const int last = (I.p + kNB - 1) / kNB - 1;  // the last panel wrote buffer last & 1
        D.Om = last & 1 ? I.buf1 : I.buf0;
        D.p = I.p;
        D.n = I.n;
        D.q = I.q;
        D.adj = I.adj;
        D.bad = I.bad;
        D.deleted = I.deleted;
        D.elem0 = elems;
        elems += ((int64_t)I.p * I.p + 255) / 256 * 256;  // each instance starts a block
        decide.push_back(D);
    }
    decide_elems = elems;
    return FPC_OK;
}

namespace {

// Workspace of fpc_first_level_noalloc, held by every device the library
// runs on until the process ends: the two sweep buffers and the panel
// inverses for p <= FPC_NOALLOC_MAX_P, then the flag word.
constexpr size_t kNoAllocMats = 2 * (size_t)FPC_NOALLOC_MAX_P * FPC_NOALLOC_MAX_P + 2 * kNB * kNB;
constexpr size_t kNoAllocBytes = sizeof(double) * kNoAllocMats + 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

}  // namespace

int first_level_enqueue(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out,
                        uint8_t *indep_out, const int **d_bad)
{
    if (!C || p < 2 || n <= p + 1) return FPC_EINVAL;
    const size_t pp = (size_t)p * p;
    int rc = ctx->inv_work.ensure(sizeof(double) * (2 * pp + 2 * kNB * kNB));
    if (rc) return rc;
    if ((rc = ctx->flag.ensure(64))) return rc;
    double *w = ctx->inv_work.as<double>();
    int *bad = ctx->flag.as<int>() + 4;
    FPC_HIP(hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
    if ((rc = first_level_enqueue_ws(ctx, C, p, n, q, r_out, indep_out, w, w + pp, w + 2 * pp,
                                     w + 2 * pp + kNB * kNB, bad, false)))
        return rc;
    *d_bad = bad;
    return FPC_OK;
}

// Device address of this device's copy of `scratch`: host code must use it,
// never the array's name, in kernel arguments and copies.  Called with the
// context's device current when the context is created.
int noalloc_init(fpc_ctx *ctx)
{
    void *ptr = nullptr;
    FPC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return FPC_EDEVICE;
    ctx->scratch = ptr;
    return FPC_OK;
}

int first_level_noalloc(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out, uint8_t *indep_out)
{
    if (!C || p < 2 || n <= p + 1) return FPC_EINVAL;
    if (p > FPC_NOALLOC_MAX_P) return FPC_ESCRATCH;
    if (!ctx->scratch) return FPC_EDEVICE;
    const size_t pp = (size_t)p * p;
    double *w = static_cast<double *>(ctx->scratch);
    int *bad = reinterpret_cast<int *>(w + kNoAllocMats);
    int rc = first_level_enqueue_ws(ctx, C, p, n, q, r_out, indep_out, w, w + pp, w + 2 * pp,
                                    w + 2 * pp + kNB * kNB, bad, true);
    if (rc) return rc;
    int hbad = 0;
    FPC_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    FPC_HIP(hipStreamSynchronize(ctx->stream));
    return hbad ? FPC_ESINGULAR : FPC_OK;
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

extern "C" int fpc_first_level_noalloc(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out,
                                       uint8_t *indep_out)
{
    if (!ctx) return FPC_EINVAL;
    FPC_HIP(hipSetDevice(ctx->device));
    return fpc::first_level_noalloc(ctx, C, p, n, q, r_out, indep_out);
}
