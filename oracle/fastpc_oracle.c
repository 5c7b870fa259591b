/*
 * fastpc_oracle.c -- plain, slow FP64 CPU oracle for the skeleton phase of
 * the reverse-order pruning PC algorithm (Zhang, Tian, Johnson, Zhang,
 * Jiang, "A Fast PC Algorithm with Reversed-order Pruning and A
 * Parallelization Strategy", arXiv 2109.04626).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library under
 * paper_2109_04626_amd/ links, loads or calls this file; only the tests,
 * the smoke check and the benchmark's CPU-baseline leg do.  It shares no
 * code, header, table or helper with the GPU path.
 *
 * What it computes, in the paper's order and notation (paper n = our p
 * variables, paper N = our n samples, l = |K|):
 *
 *   orc_corr            Pearson correlation matrix of the data (Sec. 5,
 *                       the "corr" matrix the tensor formula gathers from).
 *   orc_ppnd16          Phi^{-1}, Wichura's algorithm AS 241 (PPND16),
 *                       for the threshold Phi^{-1}(1 - alpha/2) (Sec. 2.2.2).
 *   orc_pcor            one partial correlation by the Sec. 5 formula
 *                       H = H0 - H1 H2^{-1} H1^T, rho = h12 / sqrt(h11 h22),
 *                       with H2^{-1} H1^T obtained by a Cholesky solve.
 *   orc_pcor_inverse    the same quantity from the explicit inverse P of the
 *                       (l+2)x(l+2) matrix: r = -P12 / sqrt(P11 P22).
 *   orc_zstat           Fisher z: sqrt(N - |K| - 3) * |arctanh(r)|
 *                       (Sec. 2.2.2, Eq. for F_z and the test line).
 *   orc_candidates      adj(G,i,j) intersected with path(G,i,j) (Sec. 2.1
 *                       definitions), by breadth-first search.
 *   orc_skeleton        Phase I: Algorithm 2 (reverse order, l = n-2 .. 0,
 *                       no early termination) or Algorithm 1 (forward,
 *                       l = 0 .. with early termination), each with the
 *                       `stable` switch (level-end deletion through D).
 *
 * Readings of points the paper leaves open (each listed with its reason in
 * the design notes):
 *   - |adj(G,i,j) n path(G,i,j)| >= l   (the bars are missing in the
 *     algorithms' IF lines);
 *   - testing of an edge stops at its first independent K, and S(i,j)
 *     keeps that K (the lexicographically first one at that level);
 *   - the sampling test uses |F_z(r)| (the bars are missing in the
 *     sampling line of Algorithm 2), written as
 *     sqrt(N-|K|-3)*|arctanh r| <= Phi^{-1}(1-alpha/2), ties independent;
 *   - the first reverse level l = n-2 conditions each pair on all other
 *     variables, so r_ij = -Omega_ij / sqrt(Omega_ii Omega_jj) with
 *     Omega = corr^{-1} (Gauss-Jordan, partial pivoting);
 *   - a test whose H2 is not positive definite, whose h11 or h22 is not
 *     positive, or whose |r| >= 1 is "dependent" (edge kept), and counted;
 *   - max_level >= 0 caps the reverse levels after the first one at
 *     min(max_level, n-3); the first level always runs;
 *   - corr is rejected as singular when some Omega_aa = 1/(1 - R^2_a) is
 *     not positive or exceeds 1e12 (a variable determined by the others).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -o liboracle.so fastpc_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ESINGULAR 2
#define ORC_EBUDGET 3
#define ORC_ENOMEM 4

#define ORC_DEGENERATE 1

/* ------------------------------------------------------------------ */
/* Phi^{-1}: Wichura (1988), Algorithm AS 241, PPND16.                 */
/* Rational approximations in three regions of |p - 1/2|.              */
/* ------------------------------------------------------------------ */
double orc_ppnd16(double p)
{
    const double a[8] = {3.3871328727963666080e0, 1.3314166789178437745e+2,
                         1.9715909503065514427e+3, 1.3731693765509461125e+4,
                         4.5921953931549871457e+4, 6.7265770927008700853e+4,
                         3.3430575583588128105e+4, 2.5090809287301226727e+3};
    const double b[8] = {1.0, 4.2313330701600911252e+1,
                         6.8718700749205790830e+2, 5.3941960214247511077e+3,
                         2.1213794301586595867e+4, 3.9307895800092710610e+4,
                         2.8729085735721942674e+4, 5.2264952788528545610e+3};
    const double c[8] = {1.42343711074968357734e0, 4.63033784615654529590e0,
                         5.76949722146069140550e0, 3.64784832476320460504e0,
                         1.27045825245236838258e0, 2.41780725177450611770e-1,
                         2.27238449892691845833e-2, 7.74545014278341407640e-4};
    const double d[8] = {1.0, 2.05319162663775882187e0,
                         1.67638483018380384940e0, 6.89767334985100004550e-1,
                         1.48103976427480074590e-1, 1.51986665636164571966e-2,
                         5.47593808499534494600e-4, 1.05075007164441684324e-9};
    const double e[8] = {6.65790464350110377720e0, 5.46378491116411436990e0,
                         1.78482653991729133580e0, 2.96560571828504891230e-1,
                         2.65321895265761230930e-2, 1.24266094738807843860e-3,
                         2.71155556874348757815e-5, 2.01033439929228813265e-7};
    const double f[8] = {1.0, 5.99832206555887937690e-1,
                         1.36929880922735805310e-1, 1.48753612908506148525e-2,
                         7.86869131145613259100e-4, 1.84631831751005468180e-5,
                         1.42151175831644588870e-7, 2.04426310338993978564e-15};
    if (!(p > 0.0 && p < 1.0)) {
        if (p == 0.0) return -INFINITY;
        if (p == 1.0) return INFINITY;
        return NAN;
    }
    double q = p - 0.5;
    if (fabs(q) <= 0.425) {
        double r = 0.180625 - q * q, num = 0.0, den = 0.0;
        for (int k = 7; k >= 0; --k) {
            num = num * r + a[k];
            den = den * r + b[k];
        }
        return q * num / den;
    }
    double r = q < 0.0 ? p : 1.0 - p;
    r = sqrt(-log(r));
    double num = 0.0, den = 0.0;
    if (r <= 5.0) {
        r -= 1.6;
        for (int k = 7; k >= 0; --k) {
            num = num * r + c[k];
            den = den * r + d[k];
        }
    } else {
        r -= 5.0;
        for (int k = 7; k >= 0; --k) {
            num = num * r + e[k];
            den = den * r + f[k];
        }
    }
    double val = num / den;
    return q < 0.0 ? -val : val;
}

/* Threshold of the sampling test, Phi^{-1}(1 - alpha/2), taken as
 * -Phi^{-1}(alpha/2) (symmetry of the normal law) so that the upper tail
 * alpha/2 is never formed as 1 - alpha/2 in floating point. */
double orc_quantile(double alpha) { return -orc_ppnd16(alpha / 2.0); }

/* ------------------------------------------------------------------ */
/* Correlation matrix of the data (row-major n x p), FP64 loops.       */
/* mu_j = mean of column j; S_ij = (1/n) sum_t (x_ti-mu_i)(x_tj-mu_j); */
/* C_ij = S_ij / sqrt(S_ii S_jj), C_ii = 1.                            */
/* ------------------------------------------------------------------ */
int orc_corr(const double *X, int n, int p, double *C)
{
    if (!X || !C || n < 2 || p < 1) return ORC_EINVAL;
    double *mu = (double *)calloc((size_t)p, sizeof(double));
    double *Xc = (double *)malloc(sizeof(double) * (size_t)n * p); /* column-major copy */
    if (!mu || !Xc) { free(mu); free(Xc); return ORC_ENOMEM; }
    for (int t = 0; t < n; ++t)
        for (int j = 0; j < p; ++j) mu[j] += X[(size_t)t * p + j];
    for (int j = 0; j < p; ++j) mu[j] /= n;
    for (int t = 0; t < n; ++t)
        for (int j = 0; j < p; ++j) Xc[(size_t)j * n + t] = X[(size_t)t * p + j];
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < p; ++i) {
        const double *xi = Xc + (size_t)i * n;
        for (int j = i; j < p; ++j) {
            const double *xj = Xc + (size_t)j * n;
            double s = 0.0;
            for (int t = 0; t < n; ++t) s += (xi[t] - mu[i]) * (xj[t] - mu[j]);
            C[(size_t)i * p + j] = s / n;
        }
    }
    free(Xc);
    for (int i = 0; i < p; ++i)
        for (int j = i + 1; j < p; ++j) {
            double v = C[(size_t)i * p + j] /
                       sqrt(C[(size_t)i * p + i] * C[(size_t)j * p + j]);
            C[(size_t)i * p + j] = v;
            C[(size_t)j * p + i] = v;
        }
    for (int i = 0; i < p; ++i) C[(size_t)i * p + i] = 1.0;
    free(mu);
    return ORC_OK;
}

/* Covariance -> correlation (population mode input). */
int orc_cov_to_corr(const double *S, int p, double *C)
{
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
            C[(size_t)i * p + j] = (i == j)
                                       ? 1.0
                                       : S[(size_t)i * p + j] /
                                             sqrt(S[(size_t)i * p + i] * S[(size_t)j * p + j]);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* One partial correlation, Sec. 5 formula.                           */
/*   H0 = corr({i,j},{i,j}), H1 = corr({i,j},K), H2 = corr(K,K)        */
/*   H  = H0 - H1 H2^{-1} H1^T  ;  r = h12 / sqrt(h11 h22)             */
/* H2^{-1} H1^T is formed by a Cholesky factorisation H2 = L L^T and   */
/* two triangular solves per column of H1^T.                           */
/* Returns 0, or ORC_DEGENERATE when H2 is not positive definite,      */
/* h11 or h22 is not positive, or |r| >= 1 (then *r_out is NaN).       */
/* work must hold l*l + 2*l doubles.                                   */
/* ------------------------------------------------------------------ */
static int pcor_cholesky(const double *C, int p, int i, int j, const int *K,
                         int l, double *work, double *r_out)
{
    double h11 = C[(size_t)i * p + i], h22 = C[(size_t)j * p + j];
    double h12 = C[(size_t)i * p + j];
    if (l > 0) {
        double *L = work;          /* l x l, lower triangle */
        double *Y = work + l * l;  /* l x 2: H2^{-1} H1^T  */
        for (int a = 0; a < l; ++a)
            for (int b = 0; b <= a; ++b) L[a * l + b] = C[(size_t)K[a] * p + K[b]];
        for (int a = 0; a < l; ++a) {
            for (int b = 0; b <= a; ++b) {
                double s = L[a * l + b];
                for (int c = 0; c < b; ++c) s -= L[a * l + c] * L[b * l + c];
                if (a == b) {
                    if (!(s > 0.0)) { *r_out = NAN; return ORC_DEGENERATE; }
                    L[a * l + a] = sqrt(s);
                } else {
                    L[a * l + b] = s / L[b * l + b];
                }
            }
        }
        for (int col = 0; col < 2; ++col) {
            int e = col == 0 ? i : j;
            /* forward: L y = H1^T[:,col] */
            for (int a = 0; a < l; ++a) {
                double s = C[(size_t)e * p + K[a]];
                for (int c = 0; c < a; ++c) s -= L[a * l + c] * Y[c * 2 + col];
                Y[a * 2 + col] = s / L[a * l + a];
            }
            /* backward: L^T x = y */
            for (int a = l - 1; a >= 0; --a) {
                double s = Y[a * 2 + col];
                for (int c = a + 1; c < l; ++c) s -= L[c * l + a] * Y[c * 2 + col];
                Y[a * 2 + col] = s / L[a * l + a];
            }
        }
        /* H = H0 - H1 Y */
        for (int a = 0; a < l; ++a) {
            double ci = C[(size_t)i * p + K[a]], cj = C[(size_t)j * p + K[a]];
            h11 -= ci * Y[a * 2 + 0];
            h22 -= cj * Y[a * 2 + 1];
            h12 -= ci * Y[a * 2 + 1];
        }
    }
    if (!(h11 > 0.0) || !(h22 > 0.0)) { *r_out = NAN; return ORC_DEGENERATE; }
    double r = h12 / sqrt(h11 * h22);
    if (!(fabs(r) < 1.0)) { *r_out = NAN; return ORC_DEGENERATE; }
    *r_out = r;
    return 0;
}

int orc_pcor(const double *C, int p, int i, int j, const int *K, int l,
             double *r_out)
{
    if (!C || !r_out || l < 0 || (l > 0 && !K)) return -1;
    double *work = (double *)malloc(sizeof(double) * (size_t)(l * l + 2 * l + 1));
    if (!work) return -1;
    int st = pcor_cholesky(C, p, i, j, K, l, work, r_out);
    free(work);
    return st;
}

/* Gauss-Jordan inverse with partial pivoting, A is m x m (row-major),
 * destroyed; Ainv receives the inverse.  Returns ORC_ESINGULAR if a pivot
 * is exactly zero or not finite. */
static int gauss_jordan(double *A, double *Ainv, int m)
{
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) Ainv[(size_t)a * m + b] = (a == b) ? 1.0 : 0.0;
    for (int col = 0; col < m; ++col) {
        int piv = col;
        double best = fabs(A[(size_t)col * m + col]);
        for (int r = col + 1; r < m; ++r) {
            double v = fabs(A[(size_t)r * m + col]);
            if (v > best) { best = v; piv = r; }
        }
        if (!(best > 0.0) || !isfinite(best)) return ORC_ESINGULAR;
        if (piv != col) {
            for (int b = 0; b < m; ++b) {
                double t = A[(size_t)col * m + b];
                A[(size_t)col * m + b] = A[(size_t)piv * m + b];
                A[(size_t)piv * m + b] = t;
                t = Ainv[(size_t)col * m + b];
                Ainv[(size_t)col * m + b] = Ainv[(size_t)piv * m + b];
                Ainv[(size_t)piv * m + b] = t;
            }
        }
        double inv = 1.0 / A[(size_t)col * m + col];
        for (int b = 0; b < m; ++b) {
            A[(size_t)col * m + b] *= inv;
            Ainv[(size_t)col * m + b] *= inv;
        }
        for (int r = 0; r < m; ++r) {
            if (r == col) continue;
            double fac = A[(size_t)r * m + col];
            if (fac == 0.0) continue;
            for (int b = 0; b < m; ++b) {
                A[(size_t)r * m + b] -= fac * A[(size_t)col * m + b];
                Ainv[(size_t)r * m + b] -= fac * Ainv[(size_t)col * m + b];
            }
        }
    }
    return ORC_OK;
}

int orc_inverse(const double *A, int m, double *Ainv)
{
    double *tmp = (double *)malloc(sizeof(double) * (size_t)m * m);
    if (!tmp) return ORC_ENOMEM;
    memcpy(tmp, A, sizeof(double) * (size_t)m * m);
    int st = gauss_jordan(tmp, Ainv, m);
    free(tmp);
    return st;
}

/* Partial correlation from the explicit inverse of the (l+2)x(l+2)
 * matrix over (i, j, K): P = inverse, r = -P12 / sqrt(P11 P22). */
int orc_pcor_inverse(const double *C, int p, int i, int j, const int *K, int l,
                     double *r_out)
{
    int m = l + 2;
    double *A = (double *)malloc(sizeof(double) * (size_t)m * m);
    double *P = (double *)malloc(sizeof(double) * (size_t)m * m);
    int *idx = (int *)malloc(sizeof(int) * (size_t)m);
    if (!A || !P || !idx) { free(A); free(P); free(idx); return -1; }
    idx[0] = i;
    idx[1] = j;
    for (int a = 0; a < l; ++a) idx[2 + a] = K[a];
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) A[a * m + b] = C[(size_t)idx[a] * p + idx[b]];
    int st = gauss_jordan(A, P, m);
    int ret = 0;
    if (st != ORC_OK || !(P[0] > 0.0) || !(P[m + 1] > 0.0)) {
        *r_out = NAN;
        ret = ORC_DEGENERATE;
    } else {
        double r = -P[1] / sqrt(P[0] * P[m + 1]);
        if (!(fabs(r) < 1.0)) { *r_out = NAN; ret = ORC_DEGENERATE; }
        else *r_out = r;
    }
    free(A);
    free(P);
    free(idx);
    return ret;
}

/* ------------------------------------------------------------------ */
/* The tests one edge runs at level l, as a series over ranks: the      */
/* rank-t test conditions on the t-th l-subset of the list cand (subsets */
/* of positions 0..m-1 in lexicographic order, the subset loop of the    */
/* algorithms), and r_out[t - r0] receives its partial correlation by    */
/* the Sec. 5 formula (NaN when degenerate) for t in [r0, r1).  The walk */
/* starts at rank 0 and steps through the subsets one by one.  z_out    */
/* (may be NULL) receives the Fisher z of each test, NaN when           */
/* degenerate.  Returns 0, or -1 for bad arguments (r1 beyond the last   */
/* subset included).                                                    */
/* ------------------------------------------------------------------ */
double orc_zstat(double r, int n, int l);

int orc_edge_series(const double *C, int p, int n, int i, int j, const int *cand, int m, int l,
                    int64_t r0, int64_t r1, double *r_out, double *z_out)
{
    if (!C || !r_out || l < 0 || m < l || r0 < 0 || r1 < r0 || (m > 0 && !cand)) return -1;
    int *ix = (int *)malloc(sizeof(int) * (size_t)(l + 1));
    int *K = (int *)malloc(sizeof(int) * (size_t)(l + 1));
    double *work = (double *)malloc(sizeof(double) * (size_t)(l * l + 2 * l + 1));
    if (!ix || !K || !work) { free(ix); free(K); free(work); return -1; }
    for (int a = 0; a < l; ++a) ix[a] = a;
    int ret = 0;
    for (int64_t t = 0; t < r1; ++t) {
        if (t >= r0) {
            for (int a = 0; a < l; ++a) K[a] = cand[ix[a]];
            double r;
            const int deg = pcor_cholesky(C, p, i, j, K, l, work, &r) == ORC_DEGENERATE;
            r_out[t - r0] = deg ? NAN : r;
            if (z_out) z_out[t - r0] = deg ? NAN : orc_zstat(r, n, l);
        }
        /* next subset in lexicographic order */
        int a = l - 1;
        while (a >= 0 && ix[a] == m - l + a) --a;
        if (a < 0) {
            if (t + 1 < r1) ret = -1; /* r1 lies beyond the last subset */
            break;
        }
        ++ix[a];
        for (int b = a + 1; b < l; ++b) ix[b] = ix[b - 1] + 1;
    }
    free(ix);
    free(K);
    free(work);
    return ret;
}

/* Fisher z statistic of the sampling test: sqrt(N - |K| - 3) |atanh r|. */
double orc_zstat(double r, int n, int l)
{
    return sqrt((double)(n - l - 3)) * fabs(atanh(r));
}

/* ------------------------------------------------------------------ */
/* Candidate set adj(G,i,j) n path(G,i,j) for the pair (i,j).          */
/* k in adj(G,i) \ {j} lies on a simple i..j path iff k reaches j in   */
/* G without i; symmetrically for k in adj(G,j) \ {i}.  Plain BFS.     */
/* out receives the sorted candidates; returns their number.          */
/* ------------------------------------------------------------------ */
/* Neighbour lists of the frozen graph: nb[off[u] .. off[u+1]) */
typedef struct {
    int *off, *nb;
} nblist_t;

static int nblist_build(const uint8_t *adj, int p, nblist_t *g)
{
    int64_t cnt = 0;
    for (int64_t k = 0; k < (int64_t)p * p; ++k) cnt += adj[k] != 0;
    g->off = (int *)malloc(sizeof(int) * (size_t)(p + 1));
    g->nb = (int *)malloc(sizeof(int) * (size_t)(cnt + 1));
    if (!g->off || !g->nb) return -1;
    int64_t t = 0;
    for (int u = 0; u < p; ++u) {
        g->off[u] = (int)t;
        for (int v = 0; v < p; ++v)
            if (adj[(size_t)u * p + v]) g->nb[t++] = v;
    }
    g->off[p] = (int)t;
    return 0;
}

static void nblist_free(nblist_t *g) { free(g->off); free(g->nb); }

/* seen[v] = 1 for every v reachable from src in G - {avoid}. */
static void bfs_avoid(const nblist_t *g, int p, int src, int avoid,
                      uint8_t *seen, int *queue)
{
    memset(seen, 0, (size_t)p);
    int head = 0, tail = 0;
    seen[src] = 1;
    seen[avoid] = 1; /* never enter the avoided node */
    queue[tail++] = src;
    while (head < tail) {
        int u = queue[head++];
        for (int t = g->off[u]; t < g->off[u + 1]; ++t) {
            int v = g->nb[t];
            if (!seen[v]) {
                seen[v] = 1;
                queue[tail++] = v;
            }
        }
    }
    seen[avoid] = 0;
}

static int candidates_ws(const uint8_t *adj, const nblist_t *g, int p, int i, int j,
                         int *out, uint8_t *reach_j, uint8_t *reach_i, int *queue)
{
    bfs_avoid(g, p, j, i, reach_j, queue); /* reachable from j in G - i */
    bfs_avoid(g, p, i, j, reach_i, queue); /* reachable from i in G - j */
    int m = 0;
    for (int k = 0; k < p; ++k) {
        if (k == i || k == j) continue;
        int on_path = (adj[(size_t)i * p + k] && reach_j[k]) ||
                      (adj[(size_t)j * p + k] && reach_i[k]);
        if (on_path) out[m++] = k;
    }
    return m;
}

int orc_candidates(const uint8_t *adj, int p, int i, int j, int *out)
{
    uint8_t *a = (uint8_t *)malloc((size_t)p), *b = (uint8_t *)malloc((size_t)p);
    int *q = (int *)malloc(sizeof(int) * (size_t)p);
    nblist_t g;
    if (!a || !b || !q || nblist_build(adj, p, &g)) { free(a); free(b); free(q); return -1; }
    int m = candidates_ws(adj, &g, p, i, j, out, a, b, q);
    nblist_free(&g);
    free(a);
    free(b);
    free(q);
    return m;
}

/* ------------------------------------------------------------------ */
/* Phase I.                                                            */
/* ------------------------------------------------------------------ */
typedef struct {
    int level;
    int64_t edges_eligible; /* edges with |cand| >= l */
    int64_t tests;          /* tests executed (break at first hit) */
    int64_t deleted;
    int64_t degenerate;
    double seconds;
} orc_level;

typedef struct {
    int p;
    int status;
    uint8_t *adj;       /* p*p */
    int32_t *sep_level; /* per pair (i<j), -1 = edge kept */
    int8_t *sep_kind;   /* 0 none, 1 list, 2 all-but-{i,j} */
    int32_t **sep_nodes;/* per pair, LIST kind only */
    int nlev, caplev;
    orc_level *lev;
    int64_t total_tests;
    double min_margin;  /* min |z - q| over all tests that ran */
    double q;
    int next_level;     /* stopped at a level boundary: the level to run next; -1: complete */
} orc_result;

#define PAIR(i, j, p) ((int64_t)(i) * (p) - (int64_t)(i) * ((i) + 1) / 2 + ((j) - (i) - 1))

static orc_level *push_level(orc_result *R)
{
    if (R->nlev == R->caplev) {
        int nc = R->caplev ? 2 * R->caplev : 64;
        orc_level *nl = (orc_level *)realloc(R->lev, sizeof(orc_level) * nc);
        if (!nl) return NULL;
        R->lev = nl;
        R->caplev = nc;
    }
    orc_level *L = &R->lev[R->nlev++];
    memset(L, 0, sizeof(*L));
    return L;
}

void orc_result_free(orc_result *R)
{
    if (!R) return;
    if (R->sep_nodes) {
        int64_t P = (int64_t)R->p * (R->p - 1) / 2;
        for (int64_t k = 0; k < P; ++k) free(R->sep_nodes[k]);
        free(R->sep_nodes);
    }
    free(R->adj);
    free(R->sep_level);
    free(R->sep_kind);
    free(R->lev);
    free(R);
}

/* Per-thread workspace for one level. */
typedef struct {
    int *cand, *K, *queue;
    uint8_t *ra, *rb;
    double *work;
} ws_t;

static int ws_alloc(ws_t *w, int p)
{
    w->cand = (int *)malloc(sizeof(int) * (size_t)p);
    w->K = (int *)malloc(sizeof(int) * (size_t)p);
    w->queue = (int *)malloc(sizeof(int) * (size_t)p);
    w->ra = (uint8_t *)malloc((size_t)p);
    w->rb = (uint8_t *)malloc((size_t)p);
    w->work = (double *)malloc(sizeof(double) * ((size_t)p * p + 2 * (size_t)p + 1));
    return (w->cand && w->K && w->queue && w->ra && w->rb && w->work) ? 0 : -1;
}

static void ws_free(ws_t *w)
{
    free(w->cand); free(w->K); free(w->queue); free(w->ra); free(w->rb); free(w->work);
}

/* Test every l-subset of cand (lexicographic order) for the pair (i,j)
 * until the first independent one.  Returns 1 and writes the separating K
 * when found. */
static int test_edge(const double *C, int p, int n, double q, int i, int j,
                     const int *cand, int m, int l, ws_t *w, int64_t *ntests,
                     int64_t *ndegen, double *min_margin, int64_t budget_left,
                     int *over_budget)
{
    int idx[1024];
    int *ix = l <= 1024 ? idx : (int *)malloc(sizeof(int) * (size_t)l);
    for (int a = 0; a < l; ++a) ix[a] = a;
    int found = 0;
    for (;;) {
        if (budget_left >= 0 && *ntests >= budget_left) { *over_budget = 1; break; }
        for (int a = 0; a < l; ++a) w->K[a] = cand[ix[a]];
        double r;
        int st = pcor_cholesky(C, p, i, j, w->K, l, w->work, &r);
        ++*ntests;
        if (st == ORC_DEGENERATE) {
            ++*ndegen;
        } else {
            double z = orc_zstat(r, n, l);
            double mg = fabs(z - q);
            if (mg < *min_margin) *min_margin = mg;
            if (z <= q) { found = 1; break; }
        }
        /* next combination in lexicographic order */
        int a = l - 1;
        while (a >= 0 && ix[a] == m - l + a) --a;
        if (a < 0) break;
        ++ix[a];
        for (int b = a + 1; b < l; ++b) ix[b] = ix[b - 1] + 1;
    }
    if (ix != idx) free(ix);
    return found;
}

/*
 * orc_skeleton -- Phase I of Algorithm 2 (reverse = 1) or Algorithm 1
 * (reverse = 0), sampling version.
 *   C       correlation matrix, p x p row-major (FP64)
 *   n       sample size N in the test statistic
 *   q       threshold Phi^{-1}(1 - alpha/2) (pass orc_quantile(alpha))
 *   max_level  < 0: uncapped.  Reverse: levels after the first start at
 *           min(max_level, p-3).  Forward: levels stop after max_level.
 *   stable  1: deletions collected in D and applied at level end;
 *           0: immediate deletion, edges processed serially in (i<j)
 *           row-major order with candidates taken from the current G.
 *   max_tests  0 = unlimited, else ORC_EBUDGET once exceeded.
 *   nthreads   0 = OpenMP default.  verbose: per-level line on stderr.
 */
orc_result *orc_skeleton_ex(const double *C, int p, int n, double q, int max_level,
                            int reverse, int stable, int64_t max_tests, int nthreads,
                            int verbose, int stop_after_levels, const uint8_t *adj0,
                            const int32_t *sep_level0, const int8_t *sep_kind0,
                            const int64_t *sep_off0, const int32_t *sep_nodes0,
                            int next_level0);

orc_result *orc_skeleton(const double *C, int p, int n, double q, int max_level,
                         int reverse, int stable, int64_t max_tests,
                         int nthreads, int verbose)
{
    return orc_skeleton_ex(C, p, n, q, max_level, reverse, stable, max_tests, nthreads,
                           verbose, 0, NULL, NULL, NULL, NULL, NULL, 0);
}

/*
 * orc_skeleton_ex -- orc_skeleton that can stop at a level boundary and
 * continue from one.  Under the stable schedule the graph and the
 * separating sets at the end of a level determine every later level (C
 * given), so a run stopped and continued ends as the uninterrupted one.
 *   stop_after_levels  > 0: return after this many levels of this call
 *           (the first level of a reverse run counts as one), with
 *           next_level set (-1 if the run is complete); 0: run to the end
 *   adj0    NULL: start on the complete graph.  Else the state of a
 *           stopped run (stable schedule only): its graph (p x p), per
 *           pair its separating-set level and kind, offsets and nodes (the
 *           layout of orc_result_sepsets), and the level to run next,
 *           next_level0 (-1: the run is complete).  The statistics returned
 *           are those of the levels this call runs.
 */
orc_result *orc_skeleton_ex(const double *C, int p, int n, double q, int max_level,
                            int reverse, int stable, int64_t max_tests, int nthreads,
                            int verbose, int stop_after_levels, const uint8_t *adj0,
                            const int32_t *sep_level0, const int8_t *sep_kind0,
                            const int64_t *sep_off0, const int32_t *sep_nodes0,
                            int next_level0)
{
    orc_result *R = (orc_result *)calloc(1, sizeof(orc_result));
    if (!R) return NULL;
    R->p = p;
    R->q = q;
    R->min_margin = INFINITY;
    R->next_level = -1;
    if (adj0 && (!stable || !sep_level0 || !sep_kind0 || !sep_off0 || next_level0 < -1 || next_level0 > p - 3)) {
        R->status = ORC_EINVAL;
        return R;
    }
    if (!C || p < 2 || n <= p + 1 || !(q >= 0.0)) { R->status = ORC_EINVAL; return R; }
    for (int64_t k = 0; k < (int64_t)p * p; ++k)
        if (!isfinite(C[k])) { R->status = ORC_EINVAL; return R; }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int nth = omp_get_max_threads();
#else
    int nth = 1;
    (void)nthreads;
#endif
    int64_t P = (int64_t)p * (p - 1) / 2;
    R->adj = (uint8_t *)malloc((size_t)p * p);
    R->sep_level = (int32_t *)malloc(sizeof(int32_t) * (size_t)P);
    R->sep_kind = (int8_t *)calloc((size_t)P, 1);
    R->sep_nodes = (int32_t **)calloc((size_t)P, sizeof(int32_t *));
    uint8_t *D = (uint8_t *)calloc((size_t)P, 1);
    int *ei = (int *)malloc(sizeof(int) * (size_t)P);
    int *ej = (int *)malloc(sizeof(int) * (size_t)P);
    int *em = (int *)malloc(sizeof(int) * (size_t)P);
    ws_t *ws = (ws_t *)calloc((size_t)nth, sizeof(ws_t));
    if (!R->adj || !R->sep_level || !R->sep_kind || !R->sep_nodes || !D || !ei ||
        !ej || !em || !ws) {
        R->status = ORC_ENOMEM;
        goto done;
    }
    for (int t = 0; t < nth; ++t)
        if (ws_alloc(&ws[t], p)) { R->status = ORC_ENOMEM; goto done; }
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b) R->adj[(size_t)a * p + b] = (a != b);
    for (int64_t k = 0; k < P; ++k) R->sep_level[k] = -1;

    int l = reverse ? p - 2 : 0;
    int first = 1;
    if (adj0) {
        /* continue a stopped run: its graph, separating sets and next level */
        for (int a = 0; a < p; ++a)
            for (int b = 0; b < p; ++b) R->adj[(size_t)a * p + b] = a != b && adj0[(size_t)a * p + b];
        for (int64_t k = 0; k < P; ++k) {
            R->sep_level[k] = sep_level0[k];
            R->sep_kind[k] = sep_kind0[k];
            if (sep_kind0[k] == 1 && sep_level0[k] > 0) {
                R->sep_nodes[k] = (int32_t *)malloc(sizeof(int32_t) * (size_t)sep_level0[k]);
                if (!R->sep_nodes[k]) { R->status = ORC_ENOMEM; goto done; }
                memcpy(R->sep_nodes[k], sep_nodes0 + sep_off0[k], sizeof(int32_t) * (size_t)sep_level0[k]);
            }
        }
        if (next_level0 < 0) { R->status = ORC_OK; goto done; }
        l = next_level0;
        first = 0;
    }
    int levels_run = 0;
    for (;;) {
        orc_level *LV = push_level(R);
        if (!LV) { R->status = ORC_ENOMEM; goto done; }
        LV->level = l;
        double t0 = 0.0;
#ifdef _OPENMP
        t0 = omp_get_wtime();
#endif
        if (reverse && first && stable) {
            /* l = p-2 on the complete graph: K = V \ {i,j} for every pair,
             * r_ij = -Omega_ij / sqrt(Omega_ii Omega_jj), Omega = C^{-1}. */
            double *A = (double *)malloc(sizeof(double) * (size_t)p * p);
            double *Om = (double *)malloc(sizeof(double) * (size_t)p * p);
            if (!A || !Om) { free(A); free(Om); R->status = ORC_ENOMEM; goto done; }
            memcpy(A, C, sizeof(double) * (size_t)p * p);
            int st = gauss_jordan(A, Om, p);
            free(A);
            if (st != ORC_OK) { free(Om); R->status = ORC_ESINGULAR; goto done; }
            /* Omega_aa = 1 / (1 - R^2_a), R^2_a the squared multiple correlation of
             * variable a on all others: a variable (numerically) determined by the
             * others, 1 - R^2 < 1e-12, makes C singular for the test. */
            for (int a = 0; a < p; ++a) {
                const double oaa = Om[(size_t)a * p + a];
                if (!(oaa > 0.0) || !(oaa <= 1e12)) { free(Om); R->status = ORC_ESINGULAR; goto done; }
            }
            for (int i = 0; i < p; ++i)
                for (int j = i + 1; j < p; ++j) {
                    int64_t pr = PAIR(i, j, p);
                    double r = -Om[(size_t)i * p + j] /
                               sqrt(Om[(size_t)i * p + i] * Om[(size_t)j * p + j]);
                    LV->edges_eligible++;
                    LV->tests++;
                    if (!(fabs(r) < 1.0)) { LV->degenerate++; continue; }
                    double z = orc_zstat(r, n, p - 2);
                    double mg = fabs(z - q);
                    if (mg < R->min_margin) R->min_margin = mg;
                    if (z <= q) {
                        D[pr] = 1;
                        R->sep_level[pr] = p - 2;
                        R->sep_kind[pr] = 2;
                        LV->deleted++;
                    }
                }
            free(Om);
        } else if (stable) {
            /* freeze G: list edges and candidate sets first */
            nblist_t g;
            if (nblist_build(R->adj, p, &g)) { R->status = ORC_ENOMEM; goto done; }
            int64_t E = 0;
            for (int i = 0; i < p; ++i)
                for (int j = i + 1; j < p; ++j)
                    if (R->adj[(size_t)i * p + j]) { ei[E] = i; ej[E] = j; ++E; }
            int64_t tests = 0, degen = 0, dels = 0, elig = 0;
            double mmin = R->min_margin;
            int over = 0;
            int64_t budget = max_tests > 0 ? max_tests - R->total_tests : -1;
            int64_t spent = 0; /* tests so far in this level, all threads */
#pragma omp parallel reduction(+ : tests, degen, dels, elig) reduction(min : mmin) reduction(| : over)
            {
#ifdef _OPENMP
                ws_t *w = &ws[omp_get_thread_num()];
#else
                ws_t *w = &ws[0];
#endif
#pragma omp for schedule(dynamic, 1)
                for (int64_t e = 0; e < E; ++e) {
                    int i = ei[e], j = ej[e];
                    int m = candidates_ws(R->adj, &g, p, i, j, w->cand, w->ra, w->rb, w->queue);
                    em[e] = m;
                    if (m < l) continue;
                    ++elig;
                    int64_t t_e = 0, sp;
                    int ob = 0;
#pragma omp atomic read
                    sp = spent;
                    if (budget >= 0 && sp >= budget) { over = 1; continue; }
                    int hit = test_edge(C, p, n, q, i, j, w->cand, m, l, w, &t_e,
                                        &degen, &mmin, budget < 0 ? -1 : budget - sp, &ob);
#pragma omp atomic update
                    spent += t_e;
                    tests += t_e;
                    over |= ob;
                    if (hit) {
                        int64_t pr = PAIR(i, j, p);
                        D[pr] = 1;
                        R->sep_level[pr] = l;
                        R->sep_kind[pr] = 1;
                        if (l > 0) {
                            R->sep_nodes[pr] = (int32_t *)malloc(sizeof(int32_t) * (size_t)l);
                            for (int a = 0; a < l; ++a) R->sep_nodes[pr][a] = w->K[a];
                        }
                        ++dels;
                    }
                }
            }
            nblist_free(&g);
            LV->tests = tests; LV->degenerate = degen; LV->deleted = dels;
            LV->edges_eligible = elig;
            R->min_margin = mmin;
            if (over) { R->total_tests += tests; R->status = ORC_EBUDGET; goto done; }
        } else {
            /* immediate deletion, serial, candidates from the current G */
            ws_t *w = &ws[0];
            int64_t budget = max_tests > 0 ? max_tests - R->total_tests : -1;
            for (int i = 0; i < p; ++i)
                for (int j = i + 1; j < p; ++j) {
                    if (!R->adj[(size_t)i * p + j]) continue;
                    nblist_t g;
                    if (nblist_build(R->adj, p, &g)) { R->status = ORC_ENOMEM; goto done; }
                    int m = candidates_ws(R->adj, &g, p, i, j, w->cand, w->ra, w->rb, w->queue);
                    nblist_free(&g);
                    if (m < l) continue;
                    LV->edges_eligible++;
                    int64_t t_e = 0;
                    int ob = 0;
                    int hit = test_edge(C, p, n, q, i, j, w->cand, m, l, w, &t_e,
                                        &LV->degenerate, &R->min_margin,
                                        budget < 0 ? -1 : budget - LV->tests, &ob);
                    LV->tests += t_e;
                    if (ob) { R->total_tests += LV->tests; R->status = ORC_EBUDGET; goto done; }
                    if (hit) {
                        int64_t pr = PAIR(i, j, p);
                        R->adj[(size_t)i * p + j] = R->adj[(size_t)j * p + i] = 0;
                        R->sep_level[pr] = l;
                        R->sep_kind[pr] = 1;
                        if (l > 0) {
                            R->sep_nodes[pr] = (int32_t *)malloc(sizeof(int32_t) * (size_t)l);
                            for (int a = 0; a < l; ++a) R->sep_nodes[pr][a] = w->K[a];
                        }
                        LV->deleted++;
                    }
                }
        }
        /* level end: delete D (stable) */
        for (int i = 0; i < p; ++i)
            for (int j = i + 1; j < p; ++j) {
                int64_t pr = PAIR(i, j, p);
                if (D[pr]) {
                    R->adj[(size_t)i * p + j] = R->adj[(size_t)j * p + i] = 0;
                    D[pr] = 0;
                }
            }
        R->total_tests += LV->tests;
#ifdef _OPENMP
        LV->seconds = omp_get_wtime() - t0;
#endif
        if (verbose)
            fprintf(stderr, "[oracle] l=%d eligible=%lld tests=%lld deleted=%lld degenerate=%lld %.2fs\n",
                    l, (long long)LV->edges_eligible, (long long)LV->tests,
                    (long long)LV->deleted, (long long)LV->degenerate, LV->seconds);
        if (max_tests > 0 && R->total_tests > max_tests) { R->status = ORC_EBUDGET; goto done; }

        /* largest candidate set in the updated graph */
        int mmax = -1;
        {
            nblist_t g;
            if (nblist_build(R->adj, p, &g)) { R->status = ORC_ENOMEM; goto done; }
            int64_t E = 0;
            for (int i = 0; i < p; ++i)
                for (int j = i + 1; j < p; ++j)
                    if (R->adj[(size_t)i * p + j]) { ei[E] = i; ej[E] = j; ++E; }
#pragma omp parallel reduction(max : mmax)
            {
#ifdef _OPENMP
                ws_t *w = &ws[omp_get_thread_num()];
#else
                ws_t *w = &ws[0];
#endif
#pragma omp for schedule(dynamic, 16)
                for (int64_t e = 0; e < E; ++e) {
                    int m = candidates_ws(R->adj, &g, p, ei[e], ej[e], w->cand, w->ra, w->rb, w->queue);
                    if (m > mmax) mmax = m;
                }
            }
            nblist_free(&g);
        }
        int next;
        if (reverse) {
            next = l - 1;
            if (first && max_level >= 0 && max_level < next) next = max_level;
            if (mmax < next) next = mmax; /* levels with no eligible edge change nothing */
            if (l == 0 || next < 0) next = -1;
        } else {
            /* continue only while some edge has |cand| > l (Algorithm 1's flag
             * is set at this level by |cand| >= l, the next level needs > l) */
            next = l + 1;
            if (LV->edges_eligible == 0 || mmax < l + 1) next = -1;
            if (max_level >= 0 && l + 1 > max_level) next = -1;
        }
        if (stop_after_levels > 0 && ++levels_run >= stop_after_levels) {
            R->next_level = next;
            break;
        }
        if (next < 0) break;
        l = next;
        first = 0;
    }
    R->status = ORC_OK;
done:
    if (ws) for (int t = 0; t < nth; ++t) ws_free(&ws[t]);
    free(ws);
    free(D);
    free(ei);
    free(ej);
    free(em);
    return R;
}

/* ---- result accessors (plain copies, for ctypes) ---- */
int orc_result_status(const orc_result *R) { return R ? R->status : ORC_ENOMEM; }
int orc_result_next_level(const orc_result *R) { return R->next_level; }
int orc_result_nlevels(const orc_result *R) { return R->nlev; }
int64_t orc_result_total_tests(const orc_result *R) { return R->total_tests; }
double orc_result_min_margin(const orc_result *R) { return R->min_margin; }

void orc_result_adj(const orc_result *R, uint8_t *out)
{
    memcpy(out, R->adj, (size_t)R->p * R->p);
}

/* sep_level[P], sep_kind[P], sep_off[P+1]; nodes written only if
 * nodes != NULL and cap suffices.  Returns the total LIST node count. */
int64_t orc_result_sepsets(const orc_result *R, int32_t *level, int8_t *kind,
                           int64_t *off, int32_t *nodes, int64_t cap)
{
    int64_t P = (int64_t)R->p * (R->p - 1) / 2, tot = 0;
    for (int64_t k = 0; k < P; ++k) {
        if (level) level[k] = R->sep_level[k];
        if (kind) kind[k] = R->sep_kind[k];
        if (off) off[k] = tot;
        if (R->sep_kind[k] == 1) {
            int L = R->sep_level[k];
            if (nodes && tot + L <= cap)
                for (int a = 0; a < L; ++a) nodes[tot + a] = R->sep_nodes[k][a];
            tot += L;
        }
    }
    if (off) off[P] = tot;
    return tot;
}

/* per-level rows: level, eligible, tests, deleted, degenerate (int64 x5),
 * seconds (double). */
void orc_result_levels(const orc_result *R, int64_t *rows, double *secs)
{
    for (int k = 0; k < R->nlev; ++k) {
        rows[5 * k + 0] = R->lev[k].level;
        rows[5 * k + 1] = R->lev[k].edges_eligible;
        rows[5 * k + 2] = R->lev[k].tests;
        rows[5 * k + 3] = R->lev[k].deleted;
        rows[5 * k + 4] = R->lev[k].degenerate;
        if (secs) secs[k] = R->lev[k].seconds;
    }
}
