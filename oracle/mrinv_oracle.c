/*
 * CPU FP64 oracle for finite-horizon inversion of matrix-valued sequences and
 * the Markov renewal quantities built on it.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library, and never calls it.
 *
 * Every routine is the plain definition from the paper, written out in double
 * precision with no blocking, fusion or reordering beyond what the definition
 * states.  Sequences are time-major: X[k][i][j] at X[(k*rows + i)*cols + j].
 *
 * Paper references (Kordalis & Trevezas, "Algebraic and FFT-Based Methods for
 * Discrete-Time Matrix Convolutions with Applications to Semi-Markov Models"):
 *   convolution ............ Section 2, eq. (convolution)
 *   inverse recursion ...... Section 2.2, eq. (inverse-recursion) and the
 *                            two-sided inverse of Theorem 2.1
 *   finite-horizon inverse . Proposition 2.3
 *   survival sequence Hbar . Section 4.1
 *   transition matrix ...... Section 4.1, eq. (transition-discrete): P = psi*Hbar
 *   first entrance ......... Section 4.1, eqs. (first-entrance-mass, -cdf)
 *   occupation/availability  Section 4.1, A_B(k) = alpha P(k) 1_{E,B}
 *   resolvent identity ..... Proposition 2.5 (basis of the adjoint)
 *
 * OpenMP parallelises only over independent output entries.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void);

#define IDX3(k, i, j, r, c) ((((size_t)(k)) * (size_t)(r) + (size_t)(i)) * (size_t)(c) + (size_t)(j))

/* ------------------------------------------------------------------------- */
/* Gauss-Jordan inverse of a constant d x d matrix with partial pivoting.     */
/* Returns 0 on success, 1 if a pivot is exactly zero or below               */
/* d * 2^-53 * max|A| (singular to working precision).                       */
/* ------------------------------------------------------------------------- */
int orc_gj_inverse(const double *A, int d, double *Ainv)
{
    double *W = (double *)malloc(sizeof(double) * (size_t)d * 2 * d);
    if (!W) return 2;
    double amax = 0.0;
    for (int i = 0; i < d; ++i) {
        for (int j = 0; j < d; ++j) {
            W[i * 2 * d + j] = A[i * d + j];
            W[i * 2 * d + d + j] = (i == j) ? 1.0 : 0.0;
            if (fabs(A[i * d + j]) > amax) amax = fabs(A[i * d + j]);
        }
    }
    const double tol = d * ldexp(1.0, -53) * amax;
    for (int c = 0; c < d; ++c) {
        int piv = c;
        for (int r = c + 1; r < d; ++r)
            if (fabs(W[r * 2 * d + c]) > fabs(W[piv * 2 * d + c])) piv = r;
        if (!(fabs(W[piv * 2 * d + c]) > tol)) { free(W); return 1; }
        if (piv != c)
            for (int j = 0; j < 2 * d; ++j) {
                double t = W[c * 2 * d + j]; W[c * 2 * d + j] = W[piv * 2 * d + j]; W[piv * 2 * d + j] = t;
            }
        double inv = 1.0 / W[c * 2 * d + c];
        for (int j = 0; j < 2 * d; ++j) W[c * 2 * d + j] *= inv;
        for (int r = 0; r < d; ++r) {
            if (r == c) continue;
            double f = W[r * 2 * d + c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * d; ++j) W[r * 2 * d + j] -= f * W[c * 2 * d + j];
        }
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) Ainv[i * d + j] = W[i * 2 * d + d + j];
    free(W);
    return 0;
}

/* Summation chunks of the recursions' inner sums: one chunk (a plain sum in
   increasing index) while the order-k sum is small, else ORC_CHUNKS (or k, if
   fewer) contiguous chunks.  The count never depends on the thread count. */
#define ORC_CHUNKS 64
static int chunks_for(double work, long k)
{
    if (work <= 2e5) return 1;
    return k < ORC_CHUNKS ? (int)k : ORC_CHUNKS;
}

/* ------------------------------------------------------------------------- */
/* Left (column-decoupled) coefficient recursion.  From the order-k          */
/* coefficient of A*X = e0:  X(0) = A(0)^-1 and, for k >= 1,                 */
/*     X(k) = -A(0)^-1 sum_{l=1..k} A(l) X(k-l).                             */
/* Column c of X depends only on column c of earlier X, so only the columns   */
/* listed in cols[0..nc) are produced: X is [n][d][nc].                      */
/* Returns 0 on success, 1 if A(0) is singular.                              */
/* ------------------------------------------------------------------------- */
int orc_inverse_left_cols(const double *A, int d, long n, const int *cols, int nc, double *X)
{
    double *A0inv = (double *)malloc(sizeof(double) * (size_t)d * d);
    if (orc_gj_inverse(A, d, A0inv)) { free(A0inv); return 1; }
    for (int i = 0; i < d; ++i)
        for (int c = 0; c < nc; ++c) X[IDX3(0, i, c, d, nc)] = A0inv[i * d + cols[c]];
    /* AT[l][t][r] = A(l)[r][t]: a plain transposed copy so the sums below
       run over contiguous memory. */
    double *AT = (double *)malloc(sizeof(double) * (size_t)n * d * d);
    for (long l = 0; l < n; ++l)
        for (int r = 0; r < d; ++r)
            for (int t = 0; t < d; ++t) AT[IDX3(l, t, r, d, d)] = A[IDX3(l, r, t, d, d)];
    size_t blk = (size_t)nc * d;
    double *part = (double *)malloc(sizeof(double) * blk * (size_t)ORC_CHUNKS);
    double *S = (double *)malloc(sizeof(double) * blk);   /* S[c][r] */
    for (long k = 1; k < n; ++k) {
        /* S[c][r] = sum_{l=1..k} sum_t A(l)[r][t] X(k-l)[t][c].  The l-range is
           cut into a number of contiguous chunks that depends on k, d and nc
           only (never on the thread count); each chunk sums in increasing l
           and the chunk sums are added in chunk order, so the rounding is the
           same on every host. */
        const int nch = chunks_for((double)k * d * d * nc, k);
#pragma omp parallel for schedule(static)
        for (int ch = 0; ch < nch; ++ch) {
            double *P = part + (size_t)ch * blk;
            memset(P, 0, sizeof(double) * blk);
            long lo = 1 + (k * ch) / nch, hi = 1 + (k * (ch + 1)) / nch;
            for (long l = lo; l < hi; ++l)
                for (int t = 0; t < d; ++t) {
                    const double *at = AT + IDX3(l, t, 0, d, d);
                    for (int c = 0; c < nc; ++c) {
                        double x = X[IDX3(k - l, t, c, d, nc)];
                        double *pc = P + (size_t)c * d;
                        for (int r = 0; r < d; ++r) pc[r] += at[r] * x;
                    }
                }
        }
        for (size_t e = 0; e < blk; ++e) {
            double s = 0.0;
            for (int ch = 0; ch < nch; ++ch) s += part[(size_t)ch * blk + e];
            S[e] = s;
        }
        for (int i = 0; i < d; ++i)
            for (int c = 0; c < nc; ++c) {
                double s = 0.0;
                for (int r = 0; r < d; ++r) s += A0inv[i * d + r] * S[(size_t)c * d + r];
                X[IDX3(k, i, c, d, nc)] = -s;
            }
    }
    free(S); free(part); free(AT); free(A0inv);
    return 0;
}

int orc_inverse_left(const double *A, int d, long n, double *X)
{
    int *cols = (int *)malloc(sizeof(int) * (size_t)d);
    for (int c = 0; c < d; ++c) cols[c] = c;
    int rc = orc_inverse_left_cols(A, d, n, cols, d, X);
    free(cols);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Right (row-decoupled) recursion, the paper's own form:                    */
/*     X(0) = A(0)^-1,   X(k) = -sum_{l=0..k-1} X(l) A(k-l) A(0)^-1.          */
/* Row i of X depends only on row i of earlier X.  orc_inverse_row returns   */
/* the row vector r(k) = alpha X(k) for a given alpha (length d): r is [n][d].*/
/* ------------------------------------------------------------------------- */
int orc_inverse_row(const double *A, int d, long n, const double *alpha, double *r)
{
    double *A0inv = (double *)malloc(sizeof(double) * (size_t)d * d);
    if (orc_gj_inverse(A, d, A0inv)) { free(A0inv); return 1; }
    for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int i = 0; i < d; ++i) s += alpha[i] * A0inv[i * d + j];
        r[j] = s;
    }
    double *part = (double *)malloc(sizeof(double) * (size_t)d * ORC_CHUNKS);
    double *S = (double *)malloc(sizeof(double) * (size_t)d);
    for (long k = 1; k < n; ++k) {
        /* S = sum_{l=0..k-1} r(l) A(k-l); fixed chunks of the l-range as in
           orc_inverse_left_cols, added in chunk order. */
        const int nch = chunks_for((double)k * d * d, k);
#pragma omp parallel for schedule(static)
        for (int ch = 0; ch < nch; ++ch) {
            double *P = part + (size_t)ch * d;
            memset(P, 0, sizeof(double) * (size_t)d);
            long lo = (k * ch) / nch, hi = (k * (ch + 1)) / nch;
            for (long l = lo; l < hi; ++l)
                for (int u = 0; u < d; ++u) {
                    const double a = r[(size_t)l * d + u];
                    const double *row = A + IDX3(k - l, u, 0, d, d);
                    for (int t = 0; t < d; ++t) P[t] += a * row[t];
                }
        }
        for (int t = 0; t < d; ++t) {
            double s = 0.0;
            for (int ch = 0; ch < nch; ++ch) s += part[(size_t)ch * d + t];
            S[t] = s;
        }
        for (int j = 0; j < d; ++j) {
            double s = 0.0;
            for (int t = 0; t < d; ++t) s += S[t] * A0inv[t * d + j];
            r[(size_t)k * d + j] = -s;
        }
    }
    free(S); free(part); free(A0inv);
    return 0;
}

int orc_inverse_right(const double *A, int d, long n, double *X)
{
    /* Row i of X is alpha = e_i pushed through the right recursion. */
    double *alpha = (double *)calloc((size_t)d, sizeof(double));
    double *r = (double *)malloc(sizeof(double) * (size_t)n * d);
    int rc = 0;
    for (int i = 0; i < d && rc == 0; ++i) {
        memset(alpha, 0, sizeof(double) * (size_t)d);
        alpha[i] = 1.0;
        rc = orc_inverse_row(A, d, n, alpha, r);
        for (long k = 0; k < n && rc == 0; ++k)
            for (int j = 0; j < d; ++j) X[IDX3(k, i, j, d, d)] = r[(size_t)k * d + j];
    }
    free(r);
    free(alpha);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Truncated convolution (A*B)(k) = sum_{l=0..k} A(l) B(k-l), k < n.         */
/* A is [n][ra][m], B is [n][m][cb], C is [n][ra][cb].                       */
/* ------------------------------------------------------------------------- */
void orc_conv(const double *A, const double *B, int ra, int m, int cb, long n, double *C)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < n; ++k) {
        double *ck = C + IDX3(k, 0, 0, ra, cb);
        memset(ck, 0, sizeof(double) * (size_t)ra * cb);
        for (long l = 0; l <= k; ++l)
            for (int i = 0; i < ra; ++i)
                for (int t = 0; t < m; ++t) {
                    const double a = A[IDX3(l, i, t, ra, m)];
                    const double *brow = B + IDX3(k - l, t, 0, m, cb);
                    double *crow = ck + (size_t)i * cb;
                    for (int j = 0; j < cb; ++j) crow[j] += a * brow[j];
                }
    }
}

/* ------------------------------------------------------------------------- */
/* Left residual of a candidate inverse X of A at selected coefficients:     */
/*     rho(k) = e0(k) - sum_{l=0..k} A(l) X(k-l)   for k in ks[0..nk),        */
/* e0(0) = I, e0(k) = 0 otherwise (Section 2, eq. (convolution); Proposition  */
/* 2.6 bounds the inverse's error by this residual).  With e0_minus != 0 the  */
/* array holds q and A = e0 - q is formed entry by entry (A(0) = I - q(0),    */
/* A(l) = -q(l)).  A, X are [n][d][d] with n > max ks; out is [nk][d][d].     */
/* Each rho(k) is its own plain sum in increasing l; OpenMP runs the sampled  */
/* coefficients in parallel.                                                 */
/* ------------------------------------------------------------------------- */
void orc_residual_at(const double *A, int e0_minus, const double *X, int d, const long *ks, int nk, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < nk; ++s) {
        const long k = ks[s];
        double *rk = out + IDX3(s, 0, 0, d, d);
        memset(rk, 0, sizeof(double) * (size_t)d * d);
        for (long l = 0; l <= k; ++l)
            for (int i = 0; i < d; ++i)
                for (int t = 0; t < d; ++t) {
                    double a = A[IDX3(l, i, t, d, d)];
                    if (e0_minus) a = (l == 0 && i == t ? 1.0 : 0.0) - a;
                    const double *xrow = X + IDX3(k - l, t, 0, d, d);
                    double *rrow = rk + (size_t)i * d;
                    for (int j = 0; j < d; ++j) rrow[j] += a * xrow[j];
                }
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                const double e = (k == 0 && i == j) ? 1.0 : 0.0;
                rk[i * d + j] = e - rk[i * d + j];
            }
    }
}

/* ------------------------------------------------------------------------- */
/* Survival sequence: hb[k][i] = 1 - sum_j sum_{l=1..k} q_ij(l).             */
/* ------------------------------------------------------------------------- */
void orc_hbar(const double *q, int d, long n, double *hb)
{
    for (int i = 0; i < d; ++i) {
        double acc = 0.0;
        hb[i] = 1.0;
        for (long k = 1; k < n; ++k) {
            for (int j = 0; j < d; ++j) acc += q[IDX3(k, i, j, d, d)];
            hb[(size_t)k * d + i] = 1.0 - acc;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Transition matrix P = psi * Hbar with Hbar diagonal:                      */
/*     P(k)[i][j] = sum_{l=0..k} psi(l)[i][j] hb[k-l][j].                    */
/* ------------------------------------------------------------------------- */
void orc_transition(const double *psi, const double *q, int d, long n, double *P)
{
    double *hb = (double *)malloc(sizeof(double) * (size_t)n * d);
    orc_hbar(q, d, n, hb);
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < n; ++k) {
        double *pk = P + IDX3(k, 0, 0, d, d);
        memset(pk, 0, sizeof(double) * (size_t)d * d);
        for (long l = 0; l <= k; ++l) {
            const double *h = hb + (size_t)(k - l) * d;
            for (int i = 0; i < d; ++i) {
                const double *ps = psi + IDX3(l, i, 0, d, d);
                for (int j = 0; j < d; ++j) pk[i * d + j] += ps[j] * h[j];
            }
        }
    }
    free(hb);
}

/* ------------------------------------------------------------------------- */
/* Occupation probability A_B(k) = alpha P(k) 1_B computed from the row      */
/* vector r = alpha psi (right recursion on e0 - q):                          */
/*     A_B(k) = sum_{j in B} sum_{l=0..k} r(l)_j hb[k-l][j].                  */
/* inB is a 0/1 mask of length d.  Out is [n].                                */
/* ------------------------------------------------------------------------- */
int orc_availability(const double *q, int d, long n, const double *alpha, const int *inB, double *out)
{
    size_t nd2 = (size_t)n * d * d;
    double *A = (double *)malloc(sizeof(double) * nd2);
    for (size_t t = 0; t < nd2; ++t) A[t] = -q[t];
    for (int i = 0; i < d; ++i) A[IDX3(0, i, i, d, d)] += 1.0;
    double *r = (double *)malloc(sizeof(double) * (size_t)n * d);
    int rc = orc_inverse_row(A, d, n, alpha, r);
    free(A);
    if (rc) { free(r); return rc; }
    double *hb = (double *)malloc(sizeof(double) * (size_t)n * d);
    orc_hbar(q, d, n, hb);
#pragma omp parallel for schedule(dynamic, 64)
    for (long k = 0; k < n; ++k) {
        double s = 0.0;
        for (int j = 0; j < d; ++j) {
            if (!inB[j]) continue;
            for (long l = 0; l <= k; ++l) s += r[(size_t)l * d + j] * hb[(size_t)(k - l) * d + j];
        }
        out[k] = s;
    }
    free(hb);
    free(r);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* First entrance into D (mask inD, C = complement), initial law alpha on E   */
/* (entries outside C ignored).  g_D = (e0^C - q_CC)^-1 * q_CD; the scalar     */
/* mass ga(k) = alpha_C g_D(k) 1_D and F(k) = sum_{l<=k} ga(l).              */
/* alpha_C psi_C is taken from the right recursion on e0^C - q_CC.            */
/* ------------------------------------------------------------------------- */
int orc_first_entrance(const double *q, int d, long n, const int *inD, const double *alpha,
                       double *ga, double *F)
{
    int nc = 0, nd = 0;
    int *ci = (int *)malloc(sizeof(int) * (size_t)d), *di = (int *)malloc(sizeof(int) * (size_t)d);
    for (int i = 0; i < d; ++i) { if (inD[i]) di[nd++] = i; else ci[nc++] = i; }
    if (nc == 0) {
        /* Already in D at time 0: the entrance time is 0. */
        for (long k = 0; k < n; ++k) { ga[k] = (k == 0) ? 1.0 : 0.0; F[k] = 1.0; }
        free(ci); free(di);
        return 0;
    }
    size_t ncc = (size_t)nc * nc;
    double *A = (double *)malloc(sizeof(double) * (size_t)n * ncc);
    for (long k = 0; k < n; ++k)
        for (int a = 0; a < nc; ++a)
            for (int b = 0; b < nc; ++b)
                A[IDX3(k, a, b, nc, nc)] = (k == 0 && a == b ? 1.0 : 0.0) - q[IDX3(k, ci[a], ci[b], d, d)];
    double *al = (double *)malloc(sizeof(double) * (size_t)nc);
    for (int a = 0; a < nc; ++a) al[a] = alpha[ci[a]];
    double *r = (double *)malloc(sizeof(double) * (size_t)n * nc);
    int rc = orc_inverse_row(A, nc, n, al, r);
    free(A);
    if (rc == 0) {
        /* v(l)_a = sum_{j in D} q(l)[C_a][j] */
        double *v = (double *)malloc(sizeof(double) * (size_t)n * nc);
        for (long l = 0; l < n; ++l)
            for (int a = 0; a < nc; ++a) {
                double s = 0.0;
                for (int b = 0; b < nd; ++b) s += q[IDX3(l, ci[a], di[b], d, d)];
                v[(size_t)l * nc + a] = s;
            }
#pragma omp parallel for schedule(dynamic, 64)
        for (long k = 0; k < n; ++k) {
            double s = 0.0;
            for (long l = 0; l <= k; ++l)
                for (int a = 0; a < nc; ++a) s += r[(size_t)l * nc + a] * v[(size_t)(k - l) * nc + a];
            ga[k] = s;
        }
        double acc = 0.0;
        for (long k = 0; k < n; ++k) { acc += ga[k]; F[k] = acc; }
        free(v);
    }
    free(r); free(al); free(ci); free(di);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Adjoint of psi = (e0 - q)^-1 on the horizon.  Linearising the resolvent    */
/* identity gives dpsi = psi * dq * psi, so for a cotangent psibar            */
/*     qbar(b) = sum_{a + b + c < n} psi(a)^T psibar(a+b+c) psi(c)^T,         */
/* evaluated in two correlation stages:                                      */
/*     V(j)    = sum_{c=0..n-1-j} psibar(j+c) psi(c)^T                        */
/*     qbar(b) = sum_{a=0..n-1-b} psi(a)^T V(a+b).                            */
/* ------------------------------------------------------------------------- */
void orc_adjoint(const double *psi, const double *psibar, int d, long n, double *qbar)
{
    size_t d2 = (size_t)d * d;
    double *V = (double *)calloc((size_t)n * d2, sizeof(double));
    double *PT = (double *)malloc(sizeof(double) * (size_t)n * d2);   /* PT[c][u][t] = psi(c)[t][u] */
    for (long c = 0; c < n; ++c)
        for (int t = 0; t < d; ++t)
            for (int u = 0; u < d; ++u) PT[IDX3(c, u, t, d, d)] = psi[IDX3(c, t, u, d, d)];
    /* V(j)[i][t] = sum_c sum_u psibar(j+c)[i][u] psi(c)[t][u] */
#pragma omp parallel for schedule(dynamic, 16)
    for (long j = 0; j < n; ++j)
        for (long c = 0; c + j < n; ++c)
            for (int i = 0; i < d; ++i)
                for (int u = 0; u < d; ++u) {
                    const double a = psibar[IDX3(j + c, i, u, d, d)];
                    const double *pt = PT + IDX3(c, u, 0, d, d);
                    double *v = V + IDX3(j, i, 0, d, d);
                    for (int t = 0; t < d; ++t) v[t] += a * pt[t];
                }
    /* qbar(b)[i][t] = sum_a sum_u psi(a)[u][i] V(a+b)[u][t] */
#pragma omp parallel for schedule(dynamic, 16)
    for (long b = 0; b < n; ++b) {
        double *qb = qbar + IDX3(b, 0, 0, d, d);
        memset(qb, 0, sizeof(double) * d2);
        for (long a = 0; a + b < n; ++a)
            for (int u = 0; u < d; ++u)
                for (int i = 0; i < d; ++i) {
                    const double x = psi[IDX3(a, u, i, d, d)];
                    const double *v = V + IDX3(a + b, u, 0, d, d);
                    double *q = qb + (size_t)i * d;
                    for (int t = 0; t < d; ++t) q[t] += x * v[t];
                }
    }
    free(PT);
    free(V);
}

/* ------------------------------------------------------------------------- */
/* Forward-mode derivative of the renewal equation psi = e0 + q*psi:         */
/*     dpsi(0) = 0,  dpsi(k) = sum_{l=1..k} [dq(l) psi(k-l) + q(l) dpsi(k-l)] */
/* (q(0) = dq(0) = 0).                                                       */
/* ------------------------------------------------------------------------- */
void orc_forward_mode(const double *q, const double *psi, const double *dq, int d, long n, double *dpsi)
{
    size_t d2 = (size_t)d * d;
    memset(dpsi, 0, sizeof(double) * d2);
    for (long k = 1; k < n; ++k) {
#pragma omp parallel for schedule(static) if ((double)k * d2 * d > 2e5)
        for (int i = 0; i < d; ++i) {
            double *out = dpsi + IDX3(k, i, 0, d, d);
            memset(out, 0, sizeof(double) * (size_t)d);
            for (long l = 1; l <= k; ++l)
                for (int t = 0; t < d; ++t) {
                    const double a = dq[IDX3(l, i, t, d, d)], b = q[IDX3(l, i, t, d, d)];
                    const double *ps = psi + IDX3(k - l, t, 0, d, d);
                    const double *dp = dpsi + IDX3(k - l, t, 0, d, d);
                    for (int j = 0; j < d; ++j) out[j] += a * ps[j] + b * dp[j];
                }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Pathwise Monte Carlo of a finite semi-Markov process (Section 5.2, the     */
/* validation of the lognormal model by simulated trajectories).             */
/* Random numbers: Philox4x32-10 as published by Salmon, Moraes, Dror and     */
/* Shaw (SC 2011): per round, with the multipliers M0 = 0xD2511F53 and        */
/* M1 = 0xCD9E8D57, (hi0, lo0) = M0 * c0 and (hi1, lo1) = M1 * c2 as 64-bit    */
/* products, and c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); ten rounds,   */
/* the key raised by (0x9E3779B9, 0xBB67AE85) between rounds.                 */
/* Stream layout and sampling as stated in the library's interface: jump k of */
/* trajectory t uses counters (k, 0, t_lo, t_hi) and (k, 1, t_lo, t_hi) under */
/* the key (seed_lo, seed_hi); a uniform is (x + 1/2) 2^-53 with x the top 27 */
/* and 26 bits of two words; the next state is the first j whose cumulative */
/* row sum exceeds the uniform; the sojourn of i -> j is lognormal            */
/* exp(mu + sigma z) with the Box-Muller z = sqrt(-2 ln u1) cos(2 pi u2)      */
/* (family 0), Weibull scale (-ln u1)^(1/shape) (1), exponential             */
/* -ln(u1)/rate (2).  The state at grid time m h is the one whose sojourn    */
/* [a, b) has ceil(a/h) <= m < ceil(b/h).                                   */
/* Outputs: counts A_cnt[m] of trajectories up at t_m, R_cnt[m] of those not */
/* yet in a down state on [0, t_m]; per trajectory (optional) the first     */
/* entrance time into the down set (-1 if none by t_{n-1}) and the number of  */
/* jumps at times <= t_{n-1}.                                                 */
/* ------------------------------------------------------------------------- */
static void orc_philox(unsigned int c[4], unsigned int k0, unsigned int k1)
{
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        unsigned long long p0 = 0xD2511F53ull * (unsigned long long)c[0];
        unsigned long long p1 = 0xCD9E8D57ull * (unsigned long long)c[2];
        unsigned int hi0 = (unsigned int)(p0 >> 32), lo0 = (unsigned int)p0;
        unsigned int hi1 = (unsigned int)(p1 >> 32), lo1 = (unsigned int)p1;
        unsigned int n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

void orc_philox4x32_10(const unsigned int *ctr, const unsigned int *key, unsigned int *out)
{
    unsigned int c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    orc_philox(c, key[0], key[1]);
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

static double orc_u01(unsigned int a, unsigned int b)
{
    unsigned long long x = ((unsigned long long)(a >> 5) << 26) | (unsigned long long)(b >> 6);
    return ((double)x + 0.5) / 9007199254740992.0;
}

static long orc_grid_ceil(double t, double h, long n)
{
    double q = ceil(t / h);
    return q >= (double)n ? n : (long)q;
}

void orc_semi_markov_mc(int d, int family, int initial, const double *P, const double *p1, const double *p2,
                        const int *up, double h, long n, long trajectories, unsigned long long seed,
                        long long *A_cnt, long long *R_cnt, double *tau_out, int *jumps_out)
{
    const double tmax = (double)(n - 1) * h;
    const unsigned int key0 = (unsigned int)seed, key1 = (unsigned int)(seed >> 32);
    long long *dA = (long long *)calloc((size_t)n + 1, sizeof(long long));
    long long *dR = (long long *)calloc((size_t)n + 1, sizeof(long long));
#pragma omp parallel
    {
        long long *lA = (long long *)calloc((size_t)n + 1, sizeof(long long));
        long long *lR = (long long *)calloc((size_t)n + 1, sizeof(long long));
#pragma omp for schedule(dynamic, 256)
        for (long t = 0; t < trajectories; ++t) {
            int s = initial;
            double now = 0.0;
            double tau = up[s] ? -1.0 : 0.0;
            int jumps = 0;
            if (up[s]) lR[0] += 1;
            for (unsigned int k = 0; now <= tmax; ++k) {
                unsigned int b0[4] = {k, 0u, (unsigned int)t, (unsigned int)((unsigned long long)t >> 32)};
                unsigned int b1[4] = {k, 1u, (unsigned int)t, (unsigned int)((unsigned long long)t >> 32)};
                orc_philox(b0, key0, key1);
                orc_philox(b1, key0, key1);
                double un = orc_u01(b0[0], b0[1]), ua = orc_u01(b0[2], b0[3]), ub = orc_u01(b1[0], b1[1]);
                /* next state: first j with un < cumulative row sum; the last state with
                   positive probability if rounding leaves the row sum below un */
                int j = -1, last = -1;
                double cum = 0.0;
                for (int c = 0; c < d; ++c) {
                    cum += P[s * d + c];
                    if (P[s * d + c] > 0.0) last = c;
                    if (j < 0 && un < cum) j = c;
                }
                if (j < 0) j = last;
                double a = p1[s * d + j], b = p2[s * d + j], T;
                if (family == 0) T = exp(a + b * (sqrt(-2.0 * log(ua)) * cos(6.283185307179586476925 * ub)));
                else if (family == 1) T = b * pow(-log(ua), 1.0 / a);
                else T = -log(ua) / a;
                double next = now + T;
                if (up[s]) {
                    long ia = orc_grid_ceil(now, h, n), ib = orc_grid_ceil(next, h, n);
                    if (ia < ib) { lA[ia] += 1; lA[ib] -= 1; }
                }
                now = next;
                s = j;
                if (now <= tmax) {
                    ++jumps;
                    if (tau < 0.0 && !up[s]) { tau = now; lR[orc_grid_ceil(now, h, n)] -= 1; }
                }
            }
            if (tau_out) tau_out[t] = tau;
            if (jumps_out) jumps_out[t] = jumps;
        }
#pragma omp critical
        for (long i = 0; i <= n; ++i) { dA[i] += lA[i]; dR[i] += lR[i]; }
        free(lA);
        free(lR);
    }
    long long ra = 0, rr = 0;
    for (long i = 0; i < n; ++i) {
        ra += dA[i];
        rr += dR[i];
        A_cnt[i] = ra;
        R_cnt[i] = rr;
    }
    free(dA);
    free(dR);
}

/* Number of OpenMP threads the oracle will use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
