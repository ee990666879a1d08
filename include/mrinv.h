/*
 * mrinv — finite-horizon inversion of matrix-valued sequences on MI355X (gfx950).
 *
 * The library inverts a d x d matrix-valued sequence in the truncated
 * noncommutative series ring M_d[x]/<x^n>: psi = (e0 - q)^(-1) coefficients
 * 0..n-1 (Kordalis & Trevezas, Section 2.2, Proposition 2.3 and eq. (newton);
 * Section 4.1 eq. (renewal-sequence)), by Newton iteration with doubling
 * truncation where every product is a zero-padded FFT along time, a
 * per-frequency complex matrix product, and an inverse FFT (Section 2.1,
 * eq. (fft-convolution); Appendix "Algorithmic details").  On top of psi it
 * forms the Markov renewal quantities of Section 4.1 / Table 2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Sequences are DEVICE pointers to caller-owned, contiguous, time-major
 *   arrays: X[k][i][j] at X[(k*rows + i)*cols + j], k = 0..n-1, IEEE float64.
 *   Small vectors/masks documented as "host" are host pointers.
 * - Horizon: n coefficients, k = 0..n-1 (I_N of Section 2).
 * - The library allocates device memory only in mrinv_create (twiddle
 *   tables, the status word and a 16 MiB per-handle scratch area for small
 *   vectors and time scans).  Every other buffer is the caller's: scratch
 *   memory is a device workspace `ws` of at least mrinv_workspace_size(...)
 *   bytes (256-byte aligned).
 * - Calls only enqueue work on the handle's HIP stream and return, with these
 *   exceptions, each stated at its declaration: mrinv_sync_status,
 *   mrinv_residual_norms, mrinv_autotune, mrinv_kernel_stats, mrinv_hbm_probe
 *   and mrinv_psi_inverse_batched_prepare (hence mrinv_psi_inverse_batched) wait
 *   for the stream.  Calls that only enqueue can be recorded into a HIP graph
 *   (stream capture) and replayed; the mrinv_create of the handle must come
 *   before the capture.
 *   Argument errors are reported synchronously and enqueue nothing.
 *   Conditions found on the device (singular A(0), non-finite values) set a
 *   sticky device status word that mrinv_sync_status() reads and clears;
 *   affected outputs are NaN.
 * - Outputs must not alias inputs.  A handle is not thread-safe and its
 *   scratch area is used in stream order: use one handle per stream.
 * - No C++ exception crosses this interface.
 */
#ifndef MRINV_H
#define MRINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MRINV_FP64 = 0,          /* every FFT and product in float64; Newton step m -> m' at cyclic length m' */
    MRINV_MIXED_FP32 = 1,    /* float32 Newton, then float64 residual sweeps (see mrinv_psi_inverse) */
    MRINV_MIXED_BF16X3 = 2,  /* as MIXED_FP32, but the float32 frequency-domain products for d > 8 run as
                                split-BF16 triple products (hi*hi + hi*lo + lo*hi) on the BF16 matrix cores
                                with FP32 accumulation */
    MRINV_FP64_PADDED = 3    /* float64 with every Newton step at the zero-padded length 2m' of the
                                Appendix (no wrap-around), twice the transform work of MRINV_FP64.  On
                                recurrent kernels the cyclic first product's rounding grows with the
                                coefficient index; padding removes that term (d = 3, n = 300000: 8.7e-13
                                instead of 3.6e-12) but doubles the transform length, whose own rounding
                                dominates at the largest horizons (n = 2^21: 5.3e-12 instead of 2.0e-12) */
} mrinv_precision_t;

typedef enum {
    MRINV_OK = 0,
    MRINV_E_ARG = 1,            /* invalid argument (null pointer, size out of range) */
    MRINV_E_SINGULAR_A0 = 2,    /* A(0) singular to working precision (Theorem 2.1) */
    MRINV_E_NONFINITE = 3,      /* NaN or Inf met on the device */
    MRINV_E_WORKSPACE = 4,      /* workspace too small or misaligned */
    MRINV_E_UNSUPPORTED = 5,    /* valid but unsupported size (d > MRINV_MAX_D) */
    MRINV_E_HIP = 6             /* HIP runtime error; see mrinv_last_error() */
} mrinv_status_t;

/* Largest supported matrix dimension (rows, cols and inner dimension). */
#define MRINV_MAX_D 64
/* Largest supported horizon. */
#define MRINV_MAX_N (1LL << 21)

/* Operation codes for mrinv_workspace_size. */
typedef enum {
    MRINV_OP_PSI_INVERSE = 0,       /* mrinv_psi_inverse / mrinv_series_inverse */
    MRINV_OP_APPLY = 1,             /* mrinv_markov_renewal_apply (r = columns of L) */
    MRINV_OP_TRANSITION = 2,        /* mrinv_transition */
    MRINV_OP_PSI_BACKWARD = 3,      /* mrinv_psi_inverse_backward */
    MRINV_OP_APPLY_BACKWARD = 4,    /* mrinv_markov_renewal_apply_backward */
    MRINV_OP_TRANSITION_BACKWARD = 5,
    MRINV_OP_FIRST_ENTRANCE = 6,    /* mrinv_first_entrance / mrinv_reliability (r = |D|) */
    MRINV_OP_AVAILABILITY = 7,
    MRINV_OP_RESIDUAL = 8,          /* mrinv_residual_norms */
    MRINV_OP_MRE = 9,               /* mrinv_mre_solve (r = columns of L) */
    MRINV_OP_GJ = 10                /* mrinv_series_inverse_gj / mrinv_psi_inverse_gj */
} mrinv_op_t;

typedef struct mrinv_handle_s *mrinv_handle_t;

/* Create a handle bound to `stream` (a hipStream_t; NULL = default stream)
 * on the current device.  Allocates the twiddle tables, the device status
 * word and the 16 MiB scratch area (the only device allocations the library
 * makes) and waits for the device.  mrinv_destroy waits for the stream and
 * frees them. */
mrinv_status_t mrinv_create(mrinv_handle_t *handle, void *stream);
mrinv_status_t mrinv_destroy(mrinv_handle_t handle);
mrinv_status_t mrinv_set_stream(mrinv_handle_t handle, void *stream);

/* Synchronise the handle's stream, then return and clear the device status
 * word (MRINV_OK, MRINV_E_SINGULAR_A0 or MRINV_E_NONFINITE). */
mrinv_status_t mrinv_sync_status(mrinv_handle_t handle);

const char *mrinv_status_string(mrinv_status_t status);
/* Detail of the last error on the calling thread (empty if none). */
const char *mrinv_last_error(void);

/* Bytes of device workspace needed by `op` for matrix dimension d, horizon n,
 * extra dimension r (columns of L for APPLY, |D| for FIRST_ENTRANCE, else
 * ignored) and precision.  Returns 0 for invalid arguments. */
size_t mrinv_workspace_size(mrinv_op_t op, int d, int64_t n, int r, mrinv_precision_t precision);

/*
 * psi = (e0 - q)^(-1) on the horizon (Section 4.1, eq. (renewal-sequence);
 * exact in M_d[x]/<x^n> by Proposition 2.3).
 *   q    : device [n][d][d] float64, the semi-Markov kernel (q(0) may be
 *          nonzero; only A(0) = I - q(0) nonsingular is required).
 *   psi  : device [n][d][d] float64 output.
 * Method: B0 = A(0)^-1 by Gauss-Jordan with partial pivoting, then Newton
 * B <- B*(2 e0 - A*B) (eq. (newton)) doubling the number of exact
 * coefficients each step, the final step truncated to n.
 * MRINV_MIXED_FP32 runs the Newton steps with float32 transforms and products,
 * then two residual sweeps: each forms R = e0 - A*X in float64 over the whole
 * horizon (transforms of length 2^ceil(log2(2n-1)), no wrap-around) and sets
 * X <- X + X*R with the correction product in float32.  Each sweep squares
 * the residual (Appendix, algorithmic details: e0 - A*B_{r+1} =
 * (e0 - A*B_r)^2); Proposition 2.6 bounds the remaining error by it.
 * 1 <= d <= 64, 1 <= n <= MRINV_MAX_N.
 */
mrinv_status_t mrinv_psi_inverse(mrinv_handle_t h, const double *q, int d, int64_t n,
                                 mrinv_precision_t precision, double *psi,
                                 void *ws, size_t ws_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * inversion as mrinv_psi_inverse, computed by the same kernels with the same
 * result, but its workspace is a library-owned device array of
 * MRINV_NOALLOC_SCRATCH_BYTES per GPU (set up by mrinv_create, held until the
 * process ends), so the call allocates nothing; the caller passes q and psi.
 * Sizes whose workspace (mrinv_workspace_size(MRINV_OP_PSI_INVERSE, ...))
 * exceeds the array return MRINV_E_WORKSPACE and enqueue nothing.  Every
 * call on one GPU uses that GPU's single array: calls that overlap in time on
 * one GPU (other streams, other threads) race and return wrong results; calls
 * on one stream are ordered and safe.  The array keeps the last call's
 * contents; nothing in it needs to start at zero.  The use_graph tuning is
 * ignored. */
#define MRINV_NOALLOC_SCRATCH_BYTES (64u << 20)
mrinv_status_t mrinv_psi_inverse_noalloc(mrinv_handle_t h, const double *q, int d, int64_t n,
                                         mrinv_precision_t precision, double *psi);

/* Same as mrinv_psi_inverse for a general sequence A (A^(-1) of Theorem 2.1):
 * A is device [n][d][d] float64 with A(0) nonsingular. */
mrinv_status_t mrinv_series_inverse(mrinv_handle_t h, const double *A, int d, int64_t n,
                                    mrinv_precision_t precision, double *Ainv,
                                    void *ws, size_t ws_bytes);

/* The same inverse by Gauss-Jordan elimination over the truncated series
 * ring C[[x]]/<x^n> (Appendix, Gauss-Jordan paragraph; cost
 * O(d^3 n log n), Proposition 2.4): on the augmented sequence [A | I], pivot i
 * takes the row whose column-i series has the largest |constant coefficient|
 * (row pivoting; A(0) nonsingular guarantees a nonzero one), inverts that
 * series by scalar Newton iteration, normalises its row and eliminates column
 * i from the other rows with truncated series products (transform length
 * 2^ceil(log2(2n-1))).  FP64.  The result agrees with mrinv_series_inverse to
 * rounding (the inverse is unique).  A, Ainv : device [n][d][d];
 * mrinv_psi_inverse_gj takes q and inverts e0 - q.  A singular A(0) (pivot
 * below d 2^-53 max|A(0)|) sets MRINV_E_SINGULAR_A0 on the device. */
mrinv_status_t mrinv_series_inverse_gj(mrinv_handle_t h, const double *A, int d, int64_t n, double *Ainv,
                                       void *ws, size_t ws_bytes);
mrinv_status_t mrinv_psi_inverse_gj(mrinv_handle_t h, const double *q, int d, int64_t n, double *psi,
                                    void *ws, size_t ws_bytes);

/* M = psi * L truncated at n (eq. (convolution) with rectangular
 * coefficients; reward-type equation V = psi*r, eq. (reward), and the
 * first-entrance kernel g_D = psi_CC * q_CD, eq. (first-entrance-mass)).
 *   psi : device [n][d][d];  L : device [n][d][r];  M : device [n][d][r].
 * 1 <= d, r <= 64. */
mrinv_status_t mrinv_markov_renewal_apply(mrinv_handle_t h, const double *psi, int d, int64_t n,
                                          const double *L, int r, double *M,
                                          void *ws, size_t ws_bytes);

/* P = psi * Hbar(q) (eq. (transition-discrete)), Hbar(k) = diag(1 - sum_j
 * sum_{l=1..k} q_ij(l)).  psi, q, P : device [n][d][d]. */
mrinv_status_t mrinv_transition(mrinv_handle_t h, const double *psi, const double *q, int d,
                                int64_t n, double *P, void *ws, size_t ws_bytes);

/* Hbar(q) diagonal: hb : device [n][d], hb[k][i] = 1 - sum_j sum_{l=1..k} q_ij(l)
 * (Section 4.1).  No workspace. */
mrinv_status_t mrinv_survival(mrinv_handle_t h, const double *q, int d, int64_t n, double *hb);

/* out(k) = offset + scale * u^T X(k) v, or with cumulative != 0
 * out(k) = offset + scale * sum_{l<=k} u^T X(l) v, for k < n.
 * X : device [n][rows][cols]; u : device [rows]; v : device [cols];
 * out : device [n].  Occupation probability alpha P(k) 1_B, first-entrance
 * cdf alpha_C G_D(k) 1_D and survival 1 - F_D (Table 2).  No workspace. */
mrinv_status_t mrinv_contract(mrinv_handle_t h, const double *X, int64_t n, int rows, int cols,
                              const double *u, const double *v, int cumulative,
                              double offset, double scale, double *out);

/* Y(k) = X(k)[row_idx, col_idx]: block extraction (q_CC, q_CD of Section 4.1).
 * X : device [n][rows][cols]; row_idx/col_idx : device int32 [nr]/[nc];
 * Y : device [n][nr][nc]. */
mrinv_status_t mrinv_gather_block(mrinv_handle_t h, const double *X, int64_t n, int rows, int cols,
                                  const int *row_idx, int nr, const int *col_idx, int nc, double *Y);

/* Composite functionals (Section 4.1 / Table 2), all float64 outputs [n].
 * in_D / up : host int masks of length d; alpha : host float64 [d] initial
 * law (entries outside C, resp. U, are ignored).  The host arrays are read
 * during the call and travel to the device as kernel arguments: they may be
 * reused as soon as the call returns, and a recorded graph keeps their values.
 *   first entrance: g(k) = alpha_C g_D(k) 1_D and F(k) = sum_{l<=k} g(l) with
 *     g_D = (e0^C - q_CC)^-1 * q_CD  (eqs. (first-entrance-mass), (first-entrance-cdf)).
 *   reliability:    R(k) = 1 - F_D(k) with D = complement of `up`.
 *   availability:   A(k) = alpha P(k) 1_U from a given P (device [n][d][d]).
 * `g` may be NULL. */
mrinv_status_t mrinv_first_entrance(mrinv_handle_t h, const double *q, int d, int64_t n,
                                    const int *in_D, const double *alpha,
                                    mrinv_precision_t precision, double *g, double *F,
                                    void *ws, size_t ws_bytes);
mrinv_status_t mrinv_reliability(mrinv_handle_t h, const double *q, int d, int64_t n,
                                 const int *up, const double *alpha,
                                 mrinv_precision_t precision, double *R,
                                 void *ws, size_t ws_bytes);
mrinv_status_t mrinv_availability(mrinv_handle_t h, const double *P, int d, int64_t n,
                                  const int *up, const double *alpha, double *A);

/* Expected renewal visits to B up to time k, counting the renewal at time
 * zero (Section 4.1, eq. (renewal-visits); Table 2):
 *   N_B(k) = alpha sum_{l<=k} psi(l) I_B 1,  k < n.
 * psi : device [n][d][d]; in_B : host int mask [d]; alpha : host float64 [d]
 * (both read during the call and passed as kernel arguments); N : device [n]. */
mrinv_status_t mrinv_renewal_visits(mrinv_handle_t h, const double *psi, int d, int64_t n, const int *in_B,
                                    const double *alpha, double *N);

/*
 * Mean-value (endpoint) discretisation of the continuous-time Markov renewal
 * equation K = L + Q (Stieltjes) K on the grid t_m = m h (Section 4.2,
 * eqs. (mre-discrete) and (mre-solution)):
 *   K_h = (e0 - Qbar_h)^(-1) * [L_h - (1/2) Delta+Q_h * (L_h(0) e0)],
 *   Delta Q_h(0) = 0,  Delta Q_h(m) = Q_h(m) - Q_h(m-1),
 *   Delta+Q_h(m) = Delta Q_h(m+1),  Qbar_h = (Delta Q_h + Delta+Q_h) / 2.
 *   Qs : device [n+1][d][d], Qs[m] = Q(m h) for m = 0..n (the value at n
 *        enters Delta+Q_h(n-1));
 *   L  : device [n][d][r], L[m] = L(m h);
 *   K  : device [n][d][r] output, K_h(m) for m = 0..n-1.
 * L = Hbar_h gives the transition function P_h; L = Q_UD on the up block gives
 * the first-entrance distribution of reliability.  Qbar_h(0) = Delta Q_h(1)/2
 * is not zero: the inverse runs its Gauss-Jordan path on I - Qbar_h(0).
 * `precision` selects the inverse's form; the product with the right-hand
 * side is float64.  1 <= d, r <= 64. */
mrinv_status_t mrinv_mre_solve(mrinv_handle_t h, const double *Qs, int d, int64_t n, const double *L, int r,
                               mrinv_precision_t precision, double *K, void *ws, size_t ws_bytes);

/*
 * Pathwise Monte Carlo of a finite semi-Markov process on the grid
 * t_m = m * step, m < n: the independent validation of the continuous-time
 * approximations in Section 5.2 (lognormal model, 10^6 trajectories,
 * pointwise 95% normal confidence intervals).  Each trajectory starts in
 * `initial`; at a jump from i it draws j from row i of P and a sojourn from
 * F_ij (kernel Q_ij(t) = P_ij F_ij(t)).  The state at t_m is the one whose
 * sojourn [a, b) has ceil(a/step) <= m < ceil(b/step).
 *   A[m] : fraction of trajectories in an up state at t_m (availability);
 *   R[m] : fraction that has not entered a down state on [0, t_m] (reliability);
 *   tau_D (optional, device double [trajectories]): first entrance time into
 *          the down set, -1 if none by t_{n-1} (0 if `initial` is down);
 *   jumps (optional, device int [trajectories]): jumps at times <= t_{n-1}.
 * Random numbers: Philox4x32-10 (Salmon et al., SC 2011); jump k of
 * trajectory t uses counters (k, 0, t_lo, t_hi) and (k, 1, t_lo, t_hi) under
 * the key (seed_lo, seed_hi): the first block's words 0-1 pick the next state,
 * words 2-3 give the sojourn's first uniform, the second block's words 0-1 its
 * second; a uniform is (x + 1/2) 2^-53 with x the top 27 and 26 bits of two
 * words.  Sojourns: lognormal exp(mu + sigma z), z = sqrt(-2 ln u1)
 * cos(2 pi u2); Weibull scale (-ln u1)^(1/shape); exponential -ln(u1)/rate.
 * Results are deterministic (integer atomics).  Model arrays are host
 * memory read during the call; A, R are device [n]; ws holds
 * mrinv_mc_workspace_size(n) bytes.  1 <= d <= MRINV_MC_MAX_D.
 */
#define MRINV_MC_MAX_D 8
typedef enum {
    MRINV_SOJOURN_LOGNORMAL = 0,    /* p1 = mu, p2 = sigma: F(t) = Phi((ln t - mu) / sigma) */
    MRINV_SOJOURN_WEIBULL = 1,      /* p1 = shape, p2 = scale: F(t) = 1 - exp(-(t/scale)^shape) */
    MRINV_SOJOURN_EXPONENTIAL = 2   /* p1 = rate: F(t) = 1 - exp(-rate t) */
} mrinv_sojourn_t;
typedef struct {
    int d;                  /* states */
    int family;             /* mrinv_sojourn_t, one family for every transition */
    int initial;            /* initial state */
    const double *P;        /* host [d][d] embedded jump matrix (rows sum to 1) */
    const double *p1;       /* host [d][d] sojourn parameters of i -> j (used where P_ij > 0) */
    const double *p2;       /* host [d][d] */
    const int *up;          /* host [d] up-state mask */
} mrinv_mc_model_t;
size_t mrinv_mc_workspace_size(int64_t n);
mrinv_status_t mrinv_semi_markov_mc(mrinv_handle_t h, const mrinv_mc_model_t *model, double step, int64_t n,
                                    int64_t trajectories, uint64_t seed, double *A, double *R, double *tau_D,
                                    int *jumps, void *ws, size_t ws_bytes);

/*
 * Adjoint of psi = (e0 - q)^-1: given psi and a cotangent psi_bar (device
 * [n][d][d]), q_bar(b) = sum_{a+b+c<n} psi(a)^T psi_bar(a+b+c) psi(c)^T, i.e.
 * q_bar = Rev(psi^T * Rev(psi_bar) * psi^T) with Rev(x)(k) = x(n-1-k).  This is
 * the linearisation of the resolvent identity of Proposition 2.5
 * (d psi = psi * dq * psi).  q_bar is written (not accumulated).
 */
mrinv_status_t mrinv_psi_inverse_backward(mrinv_handle_t h, const double *psi, const double *psi_bar,
                                          int d, int64_t n, double *q_bar, void *ws, size_t ws_bytes);

/* Adjoint of M = psi * L: psi_bar_accum += Rev(Rev(M_bar) * L^T) and
 * L_bar = Rev(psi^T * Rev(M_bar)).  Either output may be NULL to skip it. */
mrinv_status_t mrinv_markov_renewal_apply_backward(mrinv_handle_t h, const double *psi, const double *L,
                                                   const double *M_bar, int d, int64_t n, int r,
                                                   double *psi_bar_accum, double *L_bar,
                                                   void *ws, size_t ws_bytes);

/* Adjoint of P = psi * Hbar(q): psi_bar_accum += Rev(Rev(P_bar) * Hbar) and
 * q_bar_accum(l) += -sum_{k>=l} hb_bar(k) for l >= 1 (row-broadcast), where
 * hb_bar = diag(Rev(psi^T * Rev(P_bar))).  Either output may be NULL. */
mrinv_status_t mrinv_transition_backward(mrinv_handle_t h, const double *psi, const double *q,
                                         const double *P_bar, int d, int64_t n,
                                         double *psi_bar_accum, double *q_bar_accum,
                                         void *ws, size_t ws_bytes);

/* Adjoint of mrinv_contract: X_bar(l) += scale * w(l) u v^T with w = out_bar,
 * or its reverse cumulative sum when cumulative != 0. */
mrinv_status_t mrinv_contract_backward(mrinv_handle_t h, const double *out_bar, int64_t n, int rows,
                                       int cols, const double *u, const double *v, int cumulative,
                                       double scale, double *X_bar_accum);

/* Adjoint of mrinv_gather_block: X_bar[k][row_idx[a]][col_idx[b]] += Y_bar[k][a][b]
 * (indices within each list must be distinct). */
mrinv_status_t mrinv_scatter_block_add(mrinv_handle_t h, const double *Y_bar, int64_t n, int rows,
                                       int cols, const int *row_idx, int nr, const int *col_idx,
                                       int nc, double *X_bar_accum);

/*
 * Batched inversion of many independent problems of uneven d and n: every
 * phase of a Newton step (transform pass, product class, direct product) is
 * one launch over all problems that take part in it, driven by a device table
 * of per-problem descriptors.
 *   q_ptrs, psi_ptrs : host arrays of `count` device pointers;
 *   d, n             : host arrays of sizes (1 <= d <= 64, 1 <= n <= MRINV_MAX_N).
 * Each problem's result equals the single-problem call with the same precision
 * and tuning.  mrinv_batched_workspace_size gives the workspace bytes for the
 * tuning of handle h (NULL: the tuning of a new handle), or 0 for invalid
 * sizes; it needs no GPU.
 */
mrinv_status_t mrinv_psi_inverse_batched(mrinv_handle_t h, int count, const double *const *q_ptrs,
                                         const int *d, const int64_t *n, mrinv_precision_t precision,
                                         double *const *psi_ptrs, void *ws, size_t ws_bytes);
/* mrinv_psi_inverse_batched in two parts.  _prepare plans every launch, writes
 * the descriptor table into the head of ws (from host memory the plan owns)
 * and waits for the stream until it is there; the plan is kept in the handle,
 * replacing an earlier one.  _launch enqueues the prepared launches on the
 * handle's current stream and only enqueues, so it can be recorded into a HIP
 * graph and replayed; ws must still hold the table (the launches do not
 * write it), q must hold the inputs and psi receives the results each time.
 * mrinv_psi_inverse_batched = _prepare, then _launch.  _launch without a
 * prepared plan returns MRINV_E_ARG. */
mrinv_status_t mrinv_psi_inverse_batched_prepare(mrinv_handle_t h, int count, const double *const *q_ptrs,
                                                 const int *d, const int64_t *n, mrinv_precision_t precision,
                                                 double *const *psi_ptrs, void *ws, size_t ws_bytes);
mrinv_status_t mrinv_psi_inverse_batched_launch(mrinv_handle_t h);
size_t mrinv_batched_workspace_size(mrinv_handle_t h, int count, const int *d, const int64_t *n,
                                    mrinv_precision_t precision);

/* Residual norms of a computed inverse X of A = e0 - q (Proposition 2.6,
 * Section 5 accuracy measures): out[0] = sum_k ||(e0 - A*X)(k)||_F,
 * out[1] = sum_k ||(e0 - X*A)(k)||_F, out[2] = max |(e0 - A*X)(k)_ij|.
 * q, X : device [n][d][d]; out : host double[3].  Synchronises the stream. */
mrinv_status_t mrinv_residual_norms(mrinv_handle_t h, const double *q, const double *X, int d,
                                    int64_t n, double *out, void *ws, size_t ws_bytes);

/* Launch-shape and schedule choices of a handle.  Defaults come from
 * mrinv_create; mrinv_autotune measures alternatives on a given problem and
 * keeps the fastest.  None of them changes what is computed. */
typedef struct {
    int lgp_max;        /* largest FFT pass radix exponent, 5..9 (default 9: passes of <= 512 rows) */
    int lanes_fp64;     /* complex lanes per FFT workgroup in float64: 8, 16 or 32 (32 only for passes
                           of <= 256 rows; fewer for transforms too small to fill the GPU), or 0
                           (default): automatic, 32 for passes of <= 128 rows when d >= 32, else 16.
                           Batched calls use at most 16 (16 for 0). */
    int lanes_fp32;     /* the same in float32; automatic: 32 for passes of <= 256 rows when d >= 32 */
    int seed_m0;        /* coefficients formed by the coefficient recursion (Section 2.2) before
                           Newton starts; rounded down to a power of two, 1..256 (default 1: none).
                           A call whose seed needs more than 64 KiB of LDS ((m0 d + d^2 + 256 + d) * 8
                           bytes; at d = 64 that is m0 > 32) returns MRINV_E_UNSUPPORTED. */
    int pair_forward;   /* nonzero: forward transforms of both Newton operands in one launch (default 1) */
    int twiddle_tables; /* 0: every twiddle is a product of two table entries formed on the fly;
                           1: in-workgroup twiddles from a 512-root table; 2: also per-pass outer
                           twiddle tables built in the workspace (default 1).  Values are identical. */
    int block_order;    /* FFT workgroup order: 0 = the lane chunks of one column together,
                           1 = columns first (default 0) */
    int use_graph;      /* nonzero: mrinv_psi_inverse records its launches once into a HIP graph per
                           (pointers, sizes, tuning) and replays it on later identical calls (default 0) */
    int mfma;           /* square frequency-domain products for d > 8 on the matrix cores (16x16x4 MFMA in
                           the working precision, d padded to a multiple of 16): 0 never (vector kernels),
                           1 or 2 always (default 1).  Results agree to rounding. */
    int direct_m;       /* Newton steps m -> m2 with m2 <= direct_m (rounded down to a power of two) form
                           their two truncated products directly in the time domain on the matrix cores
                           instead of through transforms: -1 automatic from d (default), 0 never. */
} mrinv_tuning_t;

/* A table of tunings by problem class, typically written by the library's
 * autotuning script (paper_2605_30379_amd/tune_table.py, which runs
 * mrinv_autotune on one representative problem per class).  A call takes the
 * first entry whose inclusive ranges hold its (d, n) and whose precision
 * matches (-1: any); without a match the handle's tuning applies.  Single
 * inversions (also those inside first_entrance, reliability, mre_solve) use
 * the whole entry; batched inversions take each problem's recursion seed
 * (seed_m0) and direct-step limit (direct_m) from its entry and every
 * launch-shape field from the handle, so with a table installed a batched
 * result equals the single call's to rounding, and bit for bit when the
 * entries' launch-shape fields equal the handle's.  count = 0 clears the
 * table; the entries are copied. */
typedef struct {
    int d_lo, d_hi;         /* inclusive range of the matrix dimension */
    int64_t n_lo, n_hi;     /* inclusive range of the horizon */
    int precision;          /* mrinv_precision_t, or -1 for every precision */
    mrinv_tuning_t tune;
} mrinv_tuning_entry_t;
mrinv_status_t mrinv_set_tuning_table(mrinv_handle_t h, const mrinv_tuning_entry_t *entries, int count);

mrinv_status_t mrinv_get_tuning(mrinv_handle_t h, mrinv_tuning_t *out);
mrinv_status_t mrinv_set_tuning(mrinv_handle_t h, const mrinv_tuning_t *t);

/* Time mrinv_psi_inverse on q (device [n][d][d]) under candidate tunings,
 * one field of mrinv_tuning_t at a time starting from the handle's current
 * tuning (a coordinate search), keep the fastest in the handle and report it
 * in *chosen (may be NULL).  psi receives the result; ws as for
 * mrinv_psi_inverse.  Synchronises. */
mrinv_status_t mrinv_autotune(mrinv_handle_t h, const double *q, int d, int64_t n,
                              mrinv_precision_t precision, double *psi, void *ws, size_t ws_bytes,
                              mrinv_tuning_t *chosen);

/* Per-kernel timing, a profiling aid that is off by default.  While enabled,
 * every kernel launch of the library carries a start and a stop HIP event
 * that the runtime stamps at the kernel's own start and end
 * (hipExtLaunchKernelGGL), and is tagged with the algorithmic bytes (one read
 * of each input element the launch needs, one write of each output element)
 * and flops of that launch.  mrinv_set_timing also clears earlier records. */
typedef struct {
    char name[96];      /* kernel name with its template arguments */
    int64_t launches;
    double total_ms;    /* sum of the launches' execution times */
    double bytes;       /* sum of algorithmic bytes */
    double flops;       /* sum of algorithmic flops (0 for pure data movement) */
} mrinv_kernel_stat_t;

mrinv_status_t mrinv_set_timing(mrinv_handle_t h, int enabled);
/* Synchronises the stream; fills up to max_out entries, returns the number of
 * distinct kernels recorded (or -1 on error). */
int mrinv_kernel_stats(mrinv_handle_t h, mrinv_kernel_stat_t *out, int max_out);

/* Measurement utility, not an operation of the paper: the rate at which this
 * GPU reads and writes HBM for one access pattern, the practical ceiling for
 * the transform and product kernels above (whose published peak, 8 TB/s, no
 * kernel reaches).  buf: caller-owned device memory of `bytes` bytes; its
 * contents are overwritten.  pattern:
 *   MRINV_HBM_COPY: the first half of buf is copied to the second half, one
 *     16-byte element per thread (bytes >= 2 MiB);
 *   MRINV_HBM_PASS_FIRST, MRINV_HBM_PASS_LAST: every element of an array of
 *     L rows x 2048 complex doubles (L the largest power of two that fits,
 *     bytes >= 32 MiB) is read and written in place with the addressing of the
 *     first (rows m + (L/512) i) or the last (rows 512 m + i) 512-row FFT
 *     pass, `lanes` (8, 16 or 32) consecutive lanes per workgroup, and its
 *     real part increased by 1 (so each launch visits every element once).
 * Runs `reps` (1..100) launches on the handle's stream, waits for each, and
 * writes the best rate in GB/s (bytes read + bytes written, over the
 * launch's event-timed duration) to *gbps.  Allocates nothing. */
typedef enum { MRINV_HBM_COPY = 0, MRINV_HBM_PASS_FIRST = 1, MRINV_HBM_PASS_LAST = 2 } mrinv_hbm_pattern_t;
mrinv_status_t mrinv_hbm_probe(mrinv_handle_t h, void *buf, size_t bytes, int pattern, int lanes, int reps,
                               double *gbps);

#ifdef __cplusplus
}
#endif
#endif /* MRINV_H */
