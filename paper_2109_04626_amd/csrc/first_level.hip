// First reverse level of Algorithm 2 (l = p-2, Sec. 3.2): on the complete
// graph every pair (i,j) is conditioned on all other variables.  By the
// Sec. 5 formula with K = V \ {i,j}, the 2x2 matrix H is the inverse of the
// {i,j} block of Omega = C^{-1}, so r_ij = -Omega_ij / sqrt(Omega_ii Omega_jj):
// one p x p FP64 inversion replaces p(p-1)/2 factorisations of size p-2.
//
// Omega is formed by the symmetric sweep operator over panels of kNB
// columns (Gauss-Jordan without pivoting, valid for a positive definite C).
// Sweeping panel K with P = A[K,K]^{-1}, all blocks taken before the update:
//     A[I,J] -= A[I,K] P A[K,J]        (I, J outside K)
//     A[I,K]  = A[I,K] P               (I outside K)
//     A[K,J]  = P A[K,J]               (J outside K)
//     A[K,K]  = -P
// The swept matrix stays symmetric, and once every panel is swept it is
// -C^{-1}.  A non-positive pivot inside a panel inverse reports the matrix
// as not positive definite.
//
// One launch per panel t.  Each workgroup updates one tile (I, J) with
// I <= J from the matrix as it stood before the panel, forming its own slice
// of P_t A[K,J] on the FP64 matrix cores, and writes the tile and its
// transpose into the other of two buffers.  The panel inverses form the
// serial chain of the method, so they are taken two panels ahead:
// workgroup 0 of launch t brings the diagonal block of panel t+2 up to date
// through panels t and t+1 (from the matrix before panel t, P_t and
// P_{t+1}) and inverts it while the tile workgroups update the matrix.  A
// one-workgroup prologue inverts the first two diagonal blocks.  Three panel
// inverses rotate: panel t's sits in slot t mod 3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fpc_internal.h"

namespace fpc {

namespace {

constexpr int kNB = 32;  // panel width and tile size
constexpr int kPinv = kNB * kNB;
constexpr int kPanelWork = 7 * kPinv;  // panel inverses and look-ahead blocks
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double Tile[kNB][kNB + 1];  // an LDS tile (rows padded by one)
typedef double PivBuf[2][2][kNB];  // pivot rows or columns of two steps

// Two layouts of a 256-thread workgroup over a kNB x kNB tile.  Rows: thread
// (tx, ty) = (tid % 32, tid / 32) holds rows ty + 8q (q < 4) of column tx.
// Accumulator: wave w = tid / 64 holds the 16 x 16 quarter at row qr =
// 16 (w / 2), column qc = 16 (w % 2); lane l holds rows qr + 4v + l / 16
// (v < 4) of column qc + l % 16, the result layout of
// v_mfma_f64_16x16x4f64, which takes A[l % 16][l / 16] and B[l / 16][l % 16]
// from lane l.
struct Lay {
    int tx, ty, qr, ar, bc, kq;
    __device__ Lay()
    {
        tx = threadIdx.x % kNB;
        ty = threadIdx.x / kNB;
        const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
        qr = (wave / 2) * 16;
        ar = qr + lane % 16;
        bc = (wave % 2) * 16 + lane % 16;
        kq = lane / 16;
    }
};

// The nr x nc block of A (row length ld) at (r0, c0), zero outside it.
__device__ __forceinline__ void load_rows(const double *__restrict__ A, int ld, int r0, int c0, int nr, int nc,
                                          const Lay &L, double g[4])
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = L.ty + 8 * q;
        g[q] = (r < nr && L.tx < nc) ? A[(size_t)(r0 + r) * ld + c0 + L.tx] : 0.0;
    }
}

__device__ __forceinline__ void load_acc(const double *__restrict__ A, int ld, int r0, int c0, int nr, int nc,
                                         const Lay &L, v4d &a)
{
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = L.qr + 4 * v + L.kq;
        a[v] = (r < nr && L.bc < nc) ? A[(size_t)(r0 + r) * ld + c0 + L.bc] : 0.0;
    }
}

__device__ __forceinline__ void put_rows(Tile &T, const Lay &L, const double g[4])
{
#pragma unroll
    for (int q = 0; q < 4; ++q) T[L.ty + 8 * q][L.tx] = g[q];
}

__device__ __forceinline__ void put_acc(Tile &T, const Lay &L, const v4d &a)
{
#pragma unroll
    for (int v = 0; v < 4; ++v) T[L.qr + 4 * v + L.kq][L.bc] = a[v];
}

// a += X Y (NEG: a -= X Y) over the wave's quarter, X and Y in LDS.
template <bool NEG>
__device__ __forceinline__ void mma(v4d &a, const Tile &X, const Tile &Y, const Lay &L)
{
#pragma unroll
    for (int s4 = 0; s4 < kNB; s4 += 4) {
        const double x = X[L.ar][s4 + L.kq];
        a = __builtin_amdgcn_mfma_f64_16x16x4f64(NEG ? -x : x, Y[s4 + L.kq][L.bc], a, 0, 0, 0);
    }
}

// a -= X^T Y over the wave's quarter, X and Y in LDS.
__device__ __forceinline__ void mma_tn_sub(v4d &a, const Tile &X, const Tile &Y, const Lay &L)
{
#pragma unroll
    for (int s4 = 0; s4 < kNB; s4 += 4)
        a = __builtin_amdgcn_mfma_f64_16x16x4f64(-X[s4 + L.kq][L.ar], Y[s4 + L.kq][L.bc], a, 0, 0, 0);
}

// In-place Gauss-Jordan inverse of the leading nb x nb block of the LDS tile
// T (its other entries ignored) by the workgroup, two pivots per step.  With
// the pivot pair K = {t, t+1} and K2 = A[K,K], every entry takes the same
// update a_ij <- b_ij - w_i . u_j, where
//     u_j = K2^{-1} A[K,j], b_ij = a_ij    for j outside K,
//     u_j = K2^{-1} e_j,    b_ij = delta_ij for j in K,
//     w_i = A[i,K] for i outside K, w_i = (K2 - I)[i,:] for i in K;
// this is the sweep of the header for a panel of two.  The tile is padded
// with the identity beyond nb, so every call takes the same 16 steps.  The
// threads that own the next pivot rows and columns (the latter less the
// identity) publish them into the other half of rowk / colk: one barrier per
// step.  The inverse goes to Pinv (global, kNB x kNB, zero outside nb) and
// back into T; a barrier must precede reads of T.
__device__ __forceinline__ void tile_inverse(Tile &T, PivBuf &rowk, PivBuf &colk, int nb, double *__restrict__ Pinv,
                                             int *__restrict__ bad)
{
    const int c = threadIdx.x % kNB, ty = threadIdx.x / kNB;
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        v[q] = (r < nb && c < nb) ? T[r][c] : (r == c ? 1.0 : 0.0);
        if (r < 2) rowk[0][r][c] = v[q];
        if (c < 2) colk[0][c][r] = v[q] - (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    bool ok = true;
#pragma unroll
    for (int s = 0; s < kNB / 2; ++s) {
        const int t = 2 * s, b = s & 1;
        const double a = rowk[b][0][t], bt = rowk[b][0][t + 1], ct = rowk[b][1][t], d = rowk[b][1][t + 1];
        double x0 = rowk[b][0][c], x1 = rowk[b][1][c];
        double w0[4], w1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            w0[q] = colk[b][0][ty + 8 * q];
            w1[q] = colk[b][1][ty + 8 * q];
        }
        const double det = fma(a, d, -bt * ct);
        ok = ok && a > 0.0 && det > 0.0;
        const double idet = 1.0 / det;
        const bool inK = c == t || c == t + 1;
        if (inK) {
            x0 = c == t ? 1.0 : 0.0;
            x1 = c == t ? 0.0 : 1.0;
        }
        const double u0 = idet * fma(d, x0, -bt * x1), u1 = idet * fma(a, x1, -ct * x0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ty + 8 * q;
            double base = v[q];
            if (inK) base = r == c ? 1.0 : 0.0;
            v[q] = fma(-w1[q], u1, fma(-w0[q], u0, base));
        }
        if (s + 1 < kNB / 2) {
            // rows tn and tn + 1 are register tn / 8 of the threads with
            // ty = tn % 8 and tn % 8 + 1
            const int tn = t + 2, bn = b ^ 1, qn = tn / 8;
            if (ty == tn % 8) rowk[bn][0][c] = v[qn];
            if (ty == tn % 8 + 1) rowk[bn][1][c] = v[qn];
            if (c == tn || c == tn + 1) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = ty + 8 * q;
                    colk[bn][c - tn][r] = v[q] - (r == c ? 1.0 : 0.0);
                }
            }
            __syncthreads();
        }
    }
    if (!ok && threadIdx.x == 0) atomicOr(bad, 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        const double x = (r < nb && c < nb) ? v[q] : 0.0;
        Pinv[r * kNB + c] = x;
        T[r][c] = x;
    }
}

// Tile (i0, j0), i0 <= j0, of panel k0 (nb wide) from Ain to Aout, with the
// panel inverse Pinv: the workgroup stages Pinv, A[K,J] and A[I,K], forms
// its slice of P A[K,J] on the FP64 matrix cores and writes the updated tile
// and, off the diagonal, its transpose.  The target tile is loaded first,
// so its latency overlaps the staging.
__device__ __forceinline__ void sweep_tile(const double *__restrict__ Ain, double *__restrict__ Aout, int p, int k0,
                                           int nb, const double *__restrict__ Pinv, int i0, int j0, Tile *S)
{
    Tile &Ps = S[0], &Us = S[1], &Vs = S[2];
    const Lay L;
    const bool rowK = i0 == k0, colK = j0 == k0;  // uniform over the workgroup
    const int ni = std::min(kNB, p - i0), nj = std::min(kNB, p - j0);
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    if (!rowK && !colK) load_acc(Ain, p, i0, j0, ni, nj, L, acc);
    double gp[4], gu[4], gv[4];
    load_rows(Pinv, kNB, 0, 0, kNB, kNB, L, gp);
    load_rows(Ain, p, k0, j0, nb, nj, L, gu);
    load_rows(Ain, p, i0, k0, ni, nb, L, gv);
    put_rows(Ps, L, gp);
    put_rows(Us, L, gu);
    put_rows(Vs, L, gv);
    __syncthreads();
    if (rowK && colK) {  // A[K,K] <- -P
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = -Ps[L.qr + 4 * v + L.kq][L.bc];
    } else if (colK) {  // A[I,K] <- A[I,K] P
        mma<false>(acc, Vs, Ps, L);
    } else {
        v4d u = {0.0, 0.0, 0.0, 0.0};
        mma<false>(u, Ps, Us, L);  // P A[K,J]
        if (rowK) {                // A[K,J] <- P A[K,J]
            acc = u;
        } else {  // A[I,J] <- A[I,J] - A[I,K] P A[K,J]
            __syncthreads();  // every read of A[K,J] is done
            put_acc(Us, L, u);
            __syncthreads();
            mma<true>(acc, Vs, Us, L);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = L.qr + 4 * v + L.kq;
        if (r < ni && L.bc < nj) {
            Aout[(size_t)(i0 + r) * p + j0 + L.bc] = acc[v];
            if (i0 != j0) Aout[(size_t)(j0 + L.bc) * p + i0 + r] = acc[v];
        }
    }
}

// The look-ahead workspace beside the three panel inverses (slots 0-2):
// the diagonal block of panel t+2 as it stands after panel t, B_t =
// A_t[K2,K2], and the block above it, W_t = A_t[K1,K2], in slots 3 + t % 2
// and 5 + t % 2.
__device__ __forceinline__ double *slot_P(double *pw, int t) { return pw + (t % 3) * kPinv; }
__device__ __forceinline__ double *slot_B(double *pw, int t) { return pw + (3 + t % 2) * kPinv; }
__device__ __forceinline__ double *slot_W(double *pw, int t) { return pw + (5 + t % 2) * kPinv; }

// Workgroup 0 of panel t's launch (panel t+2 exists): the last step of the
// diagonal block of panel t+2 and its inverse,
//     P_{t+2} = (B_t - W_t^T P_{t+1} W_t)^{-1}.
__device__ __forceinline__ void la_inverse(double *__restrict__ pw, int p, int t, int *__restrict__ bad, Tile *S,
                                           PivBuf &rowk, PivBuf &colk)
{
    const Lay L;
    const int n2 = std::min(kNB, p - (t + 2) * kNB);
    double g_p1[4], g_w[4];
    v4d b;
    load_rows(slot_P(pw, t + 1), kNB, 0, 0, kNB, kNB, L, g_p1);
    load_rows(slot_W(pw, t), kNB, 0, 0, kNB, kNB, L, g_w);
    load_acc(slot_B(pw, t), kNB, 0, 0, kNB, kNB, L, b);
    put_rows(S[0], L, g_p1);
    put_rows(S[1], L, g_w);
    __syncthreads();
    v4d v = {0.0, 0.0, 0.0, 0.0};
    mma<false>(v, S[0], S[1], L);  // P_{t+1} W_t
    put_acc(S[2], L, v);
    __syncthreads();
    mma_tn_sub(b, S[1], S[2], L);
    put_acc(S[0], L, b);  // S[0] was last read before the previous barrier
    __syncthreads();
    tile_inverse(S[0], rowk, colk, n2, slot_P(pw, t + 2), bad);
}

// Workgroup 1 of panel t's launch (panel t+3 exists; panels K0..K3 = t ..
// t+3, the first three full): B_{t+1} = A_{t+1}[K3,K3] and W_{t+1} =
// A_{t+1}[K2,K3] from the matrix A before panel t, P_t and P_{t+1}:
//     U2 = P_t A[K0,K2],  U3 = P_t A[K0,K3]
//     A'[Ka,Kb] = A[Ka,Kb] - A[K0,Ka]^T Ub     (panel t; ab = 12, 13, 23, 33)
//     V = P_{t+1} A'[K1,K3]
//     B_{t+1} = A'[K3,K3] - A'[K1,K3]^T V,  W_{t+1} = A'[K2,K3] - A'[K1,K2]^T V
//                                                               (panel t+1)
// Every load is issued up front.
__device__ __forceinline__ void la_update(const double *__restrict__ A, double *__restrict__ pw, int p, int t,
                                          Tile *S)
{
    const Lay L;
    const int k0 = t * kNB, k1 = k0 + kNB, k2 = k1 + kNB, k3 = k2 + kNB, n3 = std::min(kNB, p - k3);
    double g_p0[4], g_01[4], g_02[4], g_03[4], g_p1[4];
    v4d t12, t13, t23, t33;
    load_rows(slot_P(pw, t), kNB, 0, 0, kNB, kNB, L, g_p0);
    load_rows(A, p, k0, k2, kNB, kNB, L, g_02);
    load_rows(A, p, k0, k3, kNB, n3, L, g_03);
    load_rows(A, p, k0, k1, kNB, kNB, L, g_01);
    load_rows(slot_P(pw, t + 1), kNB, 0, 0, kNB, kNB, L, g_p1);
    load_acc(A, p, k2, k3, kNB, n3, L, t23);
    load_acc(A, p, k3, k3, n3, n3, L, t33);
    load_acc(A, p, k1, k3, kNB, n3, L, t13);
    load_acc(A, p, k1, k2, kNB, kNB, L, t12);
    put_rows(S[0], L, g_p0);
    put_rows(S[1], L, g_02);
    put_rows(S[2], L, g_03);
    __syncthreads();
    v4d u2 = {0.0, 0.0, 0.0, 0.0}, u3 = {0.0, 0.0, 0.0, 0.0};
    mma<false>(u2, S[0], S[1], L);
    mma<false>(u3, S[0], S[2], L);
    __syncthreads();
    put_acc(S[0], L, u3);
    __syncthreads();
    mma_tn_sub(t23, S[1], S[0], L);
    mma_tn_sub(t33, S[2], S[0], L);
    __syncthreads();
    put_acc(S[1], L, u2);
    put_rows(S[2], L, g_01);
    __syncthreads();
    mma_tn_sub(t12, S[2], S[1], L);
    mma_tn_sub(t13, S[2], S[0], L);
    __syncthreads();
    put_acc(S[1], L, t13);
    put_rows(S[0], L, g_p1);
    put_acc(S[2], L, t12);
    __syncthreads();
    v4d v = {0.0, 0.0, 0.0, 0.0};
    mma<false>(v, S[0], S[1], L);  // P_{t+1} A'[K1,K3]
    __syncthreads();
    put_acc(S[0], L, v);
    __syncthreads();
    mma_tn_sub(t33, S[1], S[0], L);
    mma_tn_sub(t23, S[2], S[0], L);
    double *B = slot_B(pw, t + 1), *W = slot_W(pw, t + 1);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = L.qr + 4 * e + L.kq;
        B[r * kNB + L.bc] = t33[e];
        W[r * kNB + L.bc] = t23[e];
    }
}

// P_0 = A[K0,K0]^{-1}, P_1 = (A[K1,K1] - A[K0,K1]^T P_0 A[K0,K1])^{-1} and the
// look-ahead blocks of launch 0, B_0 = A[K2,K2] - A[K0,K2]^T P_0 A[K0,K2] and
// W_0 = A[K1,K2] - A[K0,K1]^T P_0 A[K0,K2], as far as the panels exist.
__device__ __forceinline__ void prologue(const double *__restrict__ C, int p, double *__restrict__ pw,
                                         int *__restrict__ bad, Tile *S, PivBuf &rowk, PivBuf &colk)
{
    const Lay L;
    // n1 <= 0: a single panel; n2 <= 0: two
    const int n0 = std::min(kNB, p), n1 = std::min(kNB, p - kNB), n2 = std::min(kNB, p - 2 * kNB);
    double g00[4], g01[4], g02[4];
    v4d t11 = {0.0, 0.0, 0.0, 0.0}, t12 = {0.0, 0.0, 0.0, 0.0}, t22 = {0.0, 0.0, 0.0, 0.0};
    load_rows(C, p, 0, 0, n0, n0, L, g00);
    if (n1 > 0) {
        load_rows(C, p, 0, kNB, n0, n1, L, g01);
        load_acc(C, p, kNB, kNB, n1, n1, L, t11);
    }
    if (n2 > 0) {
        load_rows(C, p, 0, 2 * kNB, kNB, n2, L, g02);
        load_acc(C, p, kNB, 2 * kNB, kNB, n2, L, t12);
        load_acc(C, p, 2 * kNB, 2 * kNB, n2, n2, L, t22);
    }
    put_rows(S[0], L, g00);
    __syncthreads();
    tile_inverse(S[0], rowk, colk, n0, slot_P(pw, 0), bad);
    if (n1 <= 0) return;  // uniform
    put_rows(S[1], L, g01);
    if (n2 > 0) put_rows(S[2], L, g02);
    __syncthreads();
    v4d u1 = {0.0, 0.0, 0.0, 0.0}, u2 = {0.0, 0.0, 0.0, 0.0};
    mma<false>(u1, S[0], S[1], L);  // P_0 A[K0,K1]
    if (n2 > 0) mma<false>(u2, S[0], S[2], L);
    __syncthreads();
    put_acc(S[0], L, u1);
    __syncthreads();
    mma_tn_sub(t11, S[1], S[0], L);
    if (n2 > 0) {
        __syncthreads();
        put_acc(S[0], L, u2);
        __syncthreads();
        mma_tn_sub(t12, S[1], S[0], L);
        mma_tn_sub(t22, S[2], S[0], L);
        double *B = slot_B(pw, 0), *W = slot_W(pw, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = L.qr + 4 * e + L.kq;
            B[r * kNB + L.bc] = t22[e];
            W[r * kNB + L.bc] = t12[e];
        }
    }
    __syncthreads();
    put_acc(S[0], L, t11);
    __syncthreads();
    tile_inverse(S[0], rowk, colk, n1, slot_P(pw, 1), bad);
}

// Tile (I, J), I <= J, number idx of the upper triangle of an nbt x nbt
// tile grid taken row by row: counted from the end, row nbt - 1 - m holds
// m + 1 tiles and starts m (m + 1) / 2 tiles before the end.
__device__ __forceinline__ void upper_tile(int idx, int nbt, int &I, int &J)
{
    const int r = nbt * (nbt + 1) / 2 - 1 - idx;
    int m = (int)((sqrtf(8.0f * (float)r + 1.0f) - 1.0f) * 0.5f);
    while ((m + 1) * (m + 2) / 2 <= r) ++m;
    while (m * (m + 1) / 2 > r) --m;
    I = nbt - 1 - m;
    J = nbt - 1 - (r - m * (m + 1) / 2);
}

// Workgroups of panel t's launch: 0 and 1 look ahead (while panels t+2 and
// t+3 exist), 2 + idx updates upper tile idx.
constexpr int kLookahead = 2;
__device__ __forceinline__ void panel_block(const double *__restrict__ Ain, double *__restrict__ Aout, int p, int t,
                                            int nbt, double *__restrict__ pw, int *__restrict__ bad, int64_t blk,
                                            Tile *S, PivBuf &rowk, PivBuf &colk)
{
    const int k0 = t * kNB;
    if (blk == 0) {
        if (k0 + 2 * kNB < p) la_inverse(pw, p, t, bad, S, rowk, colk);
        return;
    }
    if (blk == 1) {
        if (k0 + 3 * kNB < p) la_update(Ain, pw, p, t, S);
        return;
    }
    int I, J;
    upper_tile((int)(blk - kLookahead), nbt, I, J);
    sweep_tile(Ain, Aout, p, k0, std::min(kNB, p - k0), slot_P(pw, t), I * kNB, J * kNB, S);
}

__global__ __launch_bounds__(256) void first_prologue(const double *__restrict__ C, int p, double *__restrict__ pw,
                                                      int *__restrict__ bad)
{
    __shared__ Tile S[3];
    __shared__ PivBuf rowk, colk;
    prologue(C, p, pw, bad, S, rowk, colk);
}

__global__ __launch_bounds__(256) void sweep_panel(const double *__restrict__ Ain, double *__restrict__ Aout, int p,
                                                   int t, int nbt, double *__restrict__ pw, int *__restrict__ bad)
{
    __shared__ Tile S[3];
    __shared__ PivBuf rowk, colk;
    panel_block(Ain, Aout, p, t, nbt, pw, bad, blockIdx.x, S, rowk, colk);
}

// ---------------------------------------------------------------- many instances
// Panel t of every instance with p > 32 t in one launch: job q covers
// workgroups [tile0[q], tile0[q] + 2 + nbt (nbt + 1) / 2) of the flattened
// grid.
__global__ __launch_bounds__(256) void sweep_panel_batch(const SweepJob *__restrict__ jobs, int njobs)
{
    __shared__ Tile S[3];
    __shared__ PivBuf rowk, colk;
    int lo = 0, hi = njobs;  // jobs[lo].tile0 <= blockIdx.x < jobs[hi].tile0
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jobs[mid].tile0 <= (int64_t)blockIdx.x) lo = mid;
        else hi = mid;
    }
    const SweepJob J = jobs[lo];
    panel_block(J.Ain, J.Aout, J.p, J.t, J.nbt, J.pinv, J.bad, (int64_t)blockIdx.x - J.tile0, S, rowk, colk);
}

// The prologue of every instance (one workgroup each).
__global__ __launch_bounds__(256) void first_prologue_batch(const SweepJob *__restrict__ jobs)
{
    __shared__ Tile S[3];
    __shared__ PivBuf rowk, colk;
    const SweepJob J = jobs[blockIdx.x];
    prologue(J.Ain, J.p, J.pinv, J.bad, S, rowk, colk);
}

// Decisions of every instance from its swept matrix S = -Omega: adjacency
// byte = edge kept (not independent), zero diagonal; deletions counted per
// instance; the Omega_ii rule of the single-instance decision sets the
// instance's flag.
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
        // p * p fits 32 bits on this path (checked when it is queued)
        const int i = (int)idx / J.p, j = (int)idx - i * J.p;
        const double *Sw = J.Om;
        if (i == j) {
            if (!(-Sw[idx] > 0.0) || !(-Sw[idx] <= 1e12)) atomicOr(J.bad, 1);
            J.adj[idx] = 0;
        } else {
            // r = -Omega_ij / sqrt(Omega_ii Omega_jj) = S_ij / sqrt(S_ii S_jj)
            const double r = Sw[idx] / sqrt(Sw[(size_t)i * J.p + i] * Sw[(size_t)j * J.p + j]);
            uint8_t ind = 0;
            if (fabs(r) < 1.0) ind = sqrt((double)(J.n - (J.p - 2) - 3)) * fabs(atanh(r)) <= J.q;
            J.adj[idx] = ind ? 0 : 1;
            del = ind && i < j;
        }
    }
    // one atomic per workgroup: the four waves' counts are summed in LDS (a
    // workgroup's elements belong to one instance)
    __shared__ unsigned int wcount[4];
    const unsigned long long b = __ballot(del);
    if (threadIdx.x % 64 == 0) wcount[threadIdx.x / 64] = (unsigned int)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int c = wcount[0] + wcount[1] + wcount[2] + wcount[3];
        if (c) atomicAdd(J.deleted, (unsigned long long)c);
    }
}

// r_ij = -Omega_ij / sqrt(Omega_ii Omega_jj), z, decision, from the swept
// matrix S = -Omega (exactly symmetric).
__global__ __launch_bounds__(256) void first_level_decide(const double *__restrict__ Sw, int p, int n, double q,
                                                          double *__restrict__ r_out,
                                                          uint8_t *__restrict__ indep_out, int *__restrict__ bad)
{
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)p * p) return;
    const int i = (int)(idx / p), j = (int)(idx % p);
    if (i == j) {
        // Omega_ii = 1 / (1 - R^2_i): a variable determined by the others
        // (1 - R^2 < 1e-12) makes C singular for the tests.
        if (!(-Sw[idx] > 0.0) || !(-Sw[idx] <= 1e12)) atomicOr(bad, 1);
        if (r_out) r_out[idx] = 1.0;
        if (indep_out) indep_out[idx] = 0;
        return;
    }
    const double r = Sw[idx] / sqrt(Sw[(size_t)i * p + i] * Sw[(size_t)j * p + j]);
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
// sweep reads one and writes the other), the seven kNB x kNB blocks of the
// panel workspace (three panel inverses, two look-ahead blocks and two
// look-ahead rows) and the flag word (cleared by a kernel here when
// clear_bad is set).
int first_level_enqueue_ws(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out, uint8_t *indep_out,
                           double *buf0, double *buf1, double *pw, int *bad, bool clear_bad)
{
    hipStream_t st = ctx->stream;
    const size_t pp = (size_t)p * p;
    double *buf[2] = {buf0, buf1};
    if (clear_bad) clear_flag<<<1, 1, 0, st>>>(bad);
    const int nbt = (p + kNB - 1) / kNB;
    first_prologue<<<1, 256, 0, st>>>(C, p, pw, bad);
    const double *Ain = C;
    for (int t = 0; t < nbt; ++t) {
        sweep_panel<<<(unsigned)(nbt * (nbt + 1) / 2 + kLookahead), 256, 0, st>>>(Ain, buf[t & 1], p, t, nbt, pw,
                                                                                   bad);
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
        // the decisions index an instance's p x p elements in 32 bits
        if (in[k].p < 2 || (int64_t)in[k].p * in[k].p > INT32_MAX) return FPC_EINVAL;
    }
    first_prologue_batch<<<ni, 256, 0, st>>>(b.first_jobs);
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
        J.pinv = I.pinv;
        J.bad = I.bad;
        first.push_back(J);
    }
    for (int t = 0; t < npanels; ++t) {
        panel_job0[t] = (int)panels.size();
        int64_t tiles = 0;
        for (const auto &I : in) {
            if (t * kNB >= I.p) continue;
            SweepJob J{};
            J.Ain = t == 0 ? I.C : (t & 1 ? I.buf0 : I.buf1);
            J.Aout = t & 1 ? I.buf1 : I.buf0;
            J.pinv = I.pinv;
            J.bad = I.bad;
            J.p = I.p;
            J.t = t;
            J.nbt = (I.p + kNB - 1) / kNB;
            J.tile0 = tiles;
            tiles += (int64_t)J.nbt * (J.nbt + 1) / 2 + kLookahead;  // the upper tiles and the look-ahead
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
// workspace for p <= FPC_NOALLOC_MAX_P, then the flag word.
constexpr size_t kNoAllocMats = 2 * (size_t)FPC_NOALLOC_MAX_P * FPC_NOALLOC_MAX_P + kPanelWork;
constexpr size_t kNoAllocBytes = sizeof(double) * kNoAllocMats + 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

}  // namespace

int first_level_reserve(fpc_ctx *ctx, int p)
{
    const size_t pp = (size_t)p * p;
    int rc = ctx->inv_work.ensure(sizeof(double) * (2 * pp + kPanelWork));
    if (!rc) rc = ctx->flag.ensure(64);
    return rc;
}

int first_level_enqueue(fpc_ctx *ctx, const double *C, int p, int n, double q, double *r_out,
                        uint8_t *indep_out, const int **d_bad)
{
    if (!C || p < 2 || n <= p + 1) return FPC_EINVAL;
    const size_t pp = (size_t)p * p;
    int rc = ctx->inv_work.ensure(sizeof(double) * (2 * pp + kPanelWork));
    if (rc) return rc;
    if ((rc = ctx->flag.ensure(64))) return rc;
    double *w = ctx->inv_work.as<double>();
    int *bad = ctx->flag.as<int>() + 4;
    FPC_HIP(hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
    if ((rc = first_level_enqueue_ws(ctx, C, p, n, q, r_out, indep_out, w, w + pp, w + 2 * pp, bad, false)))
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
    int rc = first_level_enqueue_ws(ctx, C, p, n, q, r_out, indep_out, w, w + pp, w + 2 * pp, bad, true);
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
