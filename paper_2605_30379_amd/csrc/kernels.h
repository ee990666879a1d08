// Kernel launch interface of the mrinv library (internal).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"



namespace mrinv {

// Optional launch timing (see mrinv_set_timing).  While a timer is active,
// timed_events() records one launch (name, algorithmic bytes and flops) and
// hands out the start/stop events that the launch carries; otherwise it
// returns false and the kernel is launched without events.
void timer_activate(void *timer, hipStream_t st);
bool timed_events(const char *name, double bytes, double flops, hipEvent_t *start, hipEvent_t *stop);
void *timer_create();
void timer_destroy(void *t);
void timer_reset(void *t);

// Launches kernel(args...) on st.  A timed launch goes through
// hipExtLaunchKernelGGL, whose events the runtime stamps from the kernel's own
// dispatch packet, so their difference is the kernel's execution time (an
// event pair recorded around the launch would add the packet gaps).
template <typename F, typename... Args>
inline void launch_kernel(const char *name, double bytes, double flops, F kernel, dim3 grid, dim3 block, size_t lds,
                          hipStream_t st, Args... args) {
    hipEvent_t a = nullptr, b = nullptr;
    if (timed_events(name, bytes, flops, &a, &b))
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, st, a, b, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
}

constexpr unsigned int STATUS_SINGULAR = 1u;
constexpr unsigned int STATUS_NONFINITE = 2u;

constexpr int MAX_PASSES = 4;
constexpr int LGP_MAX = 9;   // largest radix of one FFT pass (512 rows in LDS)

// Pass plan of one transform length.
struct FftPlan {
    int lgL;
    int npass;
    int lgP[MAX_PASSES];          // pass radices, first pass = outermost (largest stride)
    const void *outer[MAX_PASSES];  // optional precomputed outer twiddles of each pass
};

// Outer-twiddle tables to generate in one launch: table t holds
// W_B^(m kr) at [m * P + kr] for B = 2^lgB, P = 2^lgP (B entries), stored as
// float64 or float32 pairs.
constexpr int MAX_TW_TABLES = 32;
struct TwGen {
    int count;
    int64_t total;                 // entries over all tables
    int64_t begin[MAX_TW_TABLES];  // first entry index of each table
    void *dst[MAX_TW_TABLES];
    int lgB[MAX_TW_TABLES], lgP[MAX_TW_TABLES], dbl[MAX_TW_TABLES];
};
hipError_t gen_outer_twiddles(const TwGen &g, const double2 *hi, const double2 *lo, hipStream_t st);

// Geometry of one pass (device side).
struct PassGeom {
    int64_t L;
    int64_t S;        // row stride inside a column
    int lgB;          // block size 2^lgB
    int nl;           // complex lanes per row
    int nchunks;      // lane chunks per column
    int col_fastest;  // workgroup order: 0 = all lane chunks of a column together, 1 = columns first
};

enum SrcKind { SRC_Z = 0, SRC_REAL64 = 1, SRC_REAL32 = 2 };
enum DstKind { DST_Z = 0, DST_REAL64 = 1, DST_REAL32 = 2 };
enum DstOp { OP_STORE = 0, OP_NEG = 1, OP_E0MINUS = 2, OP_ADD = 3, OP_XPLUS = 4 };

// Real source of the first forward pass: rows t in [lo, hi) hold
// p[row * ld + e] for e < nreal with row = t (or rev - t when rev >= 0);
// every other row is zero (implicit zero padding).  e0_d > 0 turns the value
// into e0 - x for a d x d matrix sequence.
struct SrcDesc {
    int kind;
    const void *p;
    int64_t ld;
    int nreal;
    int64_t lo, hi;
    int64_t rev;
    int e0_d;
};

// Real destination of the last inverse pass (rows t in [lo, hi) written,
// row = t or rev - t), value = op(scale * v).  In the fused inverse/forward
// mode only lo, hi, scale and op (OP_STORE / OP_NEG) are used, as a mask.
struct DstDesc {
    int kind;
    void *p;
    int64_t ld;
    int nreal;
    int64_t lo, hi;
    int64_t rev;
    int op;
    int e0_d;
    const void *aux;       // OP_XPLUS: float32 array with the same layout, added to the result;
                           // a float64 forward pass to DST_Z: float32 copy of its output
    double scale;
    unsigned int *status;  // optional: set STATUS_NONFINITE on non-finite output
};

// One problem of a batched pass launch: its spectrum buffer, lane count and
// (for the first / last pass) real source and destination.  Workgroups
// [wg_begin, wg_begin + nchunks * L / P) of the launch belong to it.
template <typename T> struct PassProblem {
    cplx<T> *z;
    int nl;
    int nchunks;
    int64_t wg_begin;
    SrcDesc src;
    DstDesc dst;
};

// One problem of a batched square product launch.
template <typename T> struct GemmProblem {
    const cplx<T> *A;
    const cplx<T> *B;
    cplx<T> *C;
    int d;
    int64_t wg_begin;
};

// One truncated product in the time domain (the first Newton steps):
//     out(k) = sign * sum_{j = jlo}^{min(jhi, k)} L(k - j) R(j),  k in [k0, k1),
// d x d matrices, L(l) at L + l d^2 (float64 or the working precision),
// R(j) at R + (j - r_off) d^2, out(k) at out + (k - out_off) d^2.  The
// workgroups of a batched launch from wg_begin on belong to it.
struct ConvDesc {
    const void *L;
    const void *R;
    void *out;
    int l_f64;
    int d;
    double sign;
    int64_t k0, k1, jlo, jhi, r_off, out_off;
    unsigned int *status;   // optional: STATUS_NONFINITE on a non-finite output
    int64_t wg_begin;
};

// One problem of a batched Gauss-Jordan launch (one workgroup each).
struct GjProblem {
    const double *A0;
    double *out64;
    float *out32;
    int d;
    int e0_minus;
};

inline SrcDesc src_z() { SrcDesc s{}; s.kind = SRC_Z; s.rev = -1; return s; }
inline DstDesc dst_z() { DstDesc d{}; d.kind = DST_Z; d.rev = -1; d.scale = 1.0; return d; }

int fft_lanes_per_block(bool dbl, int nl, int lgP, int mode);

// mode 0 forward, 1 inverse, 2 inverse + mask + forward (same pass).
// lanes: complex lanes per workgroup (8 or 16), 0 for the default;
// order: workgroup order (see PassGeom::col_fastest).
template <typename T>
hipError_t fft_pass(int mode, const FftPlan &plan, int pass, int nl, cplx<T> *z, const SrcDesc &src,
                    const DstDesc &dst, const Twiddles<T> &tw, hipStream_t st, int lanes = 0, int order = 0);
// Forward pass of two problems of the same plan in one launch (z, nl, src set).
template <typename T>
hipError_t fft_pass_pair(const FftPlan &plan, int pass, PassProblem<T> a, PassProblem<T> b, const Twiddles<T> &tw,
                         hipStream_t st, int lanes = 0, int order = 0);
// The same pass over many problems in one launch.  probs is a device array of
// nprob descriptors with wg_begin filled by fft_batch_layout; every problem
// uses C lanes per workgroup.  Returns the total workgroup count via *total.
template <typename T>
int64_t fft_batch_layout(const FftPlan &plan, int pass, PassProblem<T> *host_probs, int nprob, int C);
template <typename T>
hipError_t fft_pass_batched(int mode, const FftPlan &plan, int pass, int C, const PassProblem<T> *dev_probs,
                            int nprob, int64_t total_wg, double bytes, const Twiddles<T> &tw, hipStream_t st);

// Frequency-domain products.  Spectra are packed (two real lanes per complex
// lane) in the digit-reversed order of `plan`.
struct GemmDesc {
    int ra, m, cb;          // C[ra x cb] = A[ra x m] * B[m x cb]
    int transA, transB;     // operand stored transposed (A stored m x ra, B stored cb x m)
    int nlA, nlB, nlC;      // complex lanes of the stored sequences
    int mfma;               // square products: 0 vector kernel; 1 matrix cores, three real products per complex
                            // product for padded d >= 48; 2 matrix cores, four real products
    int bf3;                // float square products on the matrix cores as split-BF16 triple products
};
template <typename T>
hipError_t freq_gemm(const FftPlan &plan, const GemmDesc &g, const cplx<T> *ZA, const cplx<T> *ZB, cplx<T> *ZC,
                     hipStream_t st);
// Square products of many problems with the same product class (vector
// kernel with d rounded up to a multiple of 8, or matrix-core kernel with d
// rounded up to a multiple of 16) in one launch.
int gemm_sq_class(int d, int mfma);
template <typename T>
int64_t gemm_batch_layout(const FftPlan &plan, GemmProblem<T> *host_probs, int nprob, int mfma);
template <typename T>
hipError_t freq_gemm_batched(const FftPlan &plan, int dclass, int mfma, int bf3, const GemmProblem<T> *dev_probs,
                             int nprob, int64_t total_wg, double bytes, double flops, hipStream_t st);
// C = A * diag(h): A ra x cb, h has cb lanes.
template <typename T>
hipError_t freq_diag(const FftPlan &plan, int ra, int cb, const cplx<T> *ZA, const cplx<T> *ZH, cplx<T> *ZC,
                     hipStream_t st);
// h_j = sum_i A_ij B_ij (diagonal of A^T B), A and B ra x cb.
template <typename T>
hipError_t freq_coldot(const FftPlan &plan, int ra, int cb, const cplx<T> *ZA, const cplx<T> *ZB, cplx<T> *ZH,
                       hipStream_t st);

// Gauss-Jordan inverse of A(0) (or of I - q(0) when e0_minus) written as row 0
// of out (float64 and/or float32 copies, either may be null).
hipError_t gj_inverse(const double *A0, int d, int e0_minus, double *out64, float *out32, unsigned int *status,
                      hipStream_t st);

// One problem of a batched recursion seed launch (d workgroups each).
struct SeedProblem {
    const double *A;
    void *out;          // float64 or float32 per the launch
    int d, m0, e0;
    int col_begin;
};
template <typename T>
hipError_t seed_recursion_batched(const SeedProblem *probs, int nprob, int total_cols, int dmax, int m0max,
                                  hipStream_t st);

// X(1..m0-1) by the coefficient recursion, X(0) already in out row 0;
// e0 != 0 means the source is q and A = e0 - q.
template <typename T>
hipError_t seed_recursion(const double *A, int e0, int d, int m0, T *out, hipStream_t st);
// Direct products (ConvDesc) on the matrix cores: one launch, or one launch
// over many descriptors of the same padded dimension 16 * cls (device table,
// wg_begin from conv_batch_layout).
int conv_class(int d);
template <typename T>
hipError_t conv_direct(const ConvDesc &c, hipStream_t st);
int64_t conv_batch_layout(ConvDesc *host_descs, int n);
template <typename T>
hipError_t conv_direct_batched(int cls, int l_f64, const ConvDesc *dev_descs, int n, int64_t total, double flops,
                               hipStream_t st);

hipError_t gj_inverse_batched(const GjProblem *dev_probs, int nprob, int dmax, unsigned int *status,
                              hipStream_t st);

// tmp: scan workspace of scan_tmp_bytes(n, lanes) bytes.
size_t scan_tmp_bytes(int64_t n, int w);
hipError_t survival(const double *q, int d, int64_t n, double *hb, double *tmp, hipStream_t st);
hipError_t contract(const double *X, int64_t n, int rows, int cols, const double *u, const double *v,
                    int cumulative, double offset, double scale, double *out, double *tmp, hipStream_t st);
hipError_t contract_backward(const double *ob, int64_t n, int rows, int cols, const double *u, const double *v,
                             int cumulative, double scale, double *Xb, double *tmp, hipStream_t st);
hipError_t gather_block(const double *X, int64_t n, int rows, int cols, const int *ri, int nr, const int *ci,
                        int nc, double *Y, hipStream_t st);
hipError_t scatter_block_add(const double *Yb, int64_t n, int rows, int cols, const int *ri, int nr,
                             const int *ci, int nc, double *Xb, hipStream_t st);
// q_bar(l)[i][j] += -sum_{k>=l} hb_bar(k)[i] for l >= 1.
hipError_t survival_backward(const double *hbb, int d, int64_t n, double *qb, double *tmp, hipStream_t st);
// Small host vectors of a functional (index lists, initial law, indicator),
// passed by value as kernel arguments and written to device memory by one
// small kernel, so the entry points neither wait for the stream nor keep
// host buffers alive (and can be recorded into a HIP graph).
constexpr int SMALL_MAX = 64;
struct SmallVecArgs {
    int nci, ndi, nalpha, nones;
    int ci[SMALL_MAX];
    int di[SMALL_MAX];
    double alpha[SMALL_MAX];
    double ones[SMALL_MAX];
};
hipError_t put_small_vectors(const SmallVecArgs &v, int *ci, int *di, double *alpha, double *ones, hipStream_t st);
// LDS bytes of the recursion seed launch (m0 coefficients of a d x d problem).
size_t seed_lds_bytes(int m0, int d);
// Qbar_h and the right-hand side of the mean-value scheme (Section 4.2).
hipError_t mre_prepare(const double *Qs, const double *L, int64_t n, int d, int r, double *Qbar, double *R,
                       hipStream_t st);
// Series Gauss-Jordan (Appendix): W = [A | I] ([n][d][2d]); one pivot step's
// pivot choice, row swap and gathers (pivot series u, multipliers col); the
// right block as the result.
hipError_t gjs_init(const double *A, int e0_minus, int64_t n, int d, double *W, hipStream_t st);
hipError_t gjs_pivot_step(double *W, int64_t n, int d, int i, int *piv, double *aux, double *u, double *col,
                          unsigned int *status, hipStream_t st);
hipError_t gjs_result(const double *W, int64_t n, int d, double *out, unsigned int *status, hipStream_t st);
// Monte Carlo of a semi-Markov process (mc.hip); the model travels by value.
constexpr int MC_MAX_D = 8;
constexpr uint32_t MC_MAX_JUMPS = 1u << 22;   // every trajectory stops after this many jumps
struct McModel {
    int d, family, initial;
    int up[MC_MAX_D];
    int last[MC_MAX_D];                        // last state with positive jump probability, per row
    double cum[MC_MAX_D * MC_MAX_D];           // cumulative row sums of the embedded matrix
    double p1[MC_MAX_D * MC_MAX_D], p2[MC_MAX_D * MC_MAX_D];
};
hipError_t semi_markov_mc(const McModel &m, double step, int64_t n, int64_t trajectories, uint64_t seed, double *A,
                          double *R, double *tau, int *jumps, int *diffA, int *diffR, hipStream_t st);
hipError_t fill_f64(double *p, int64_t count, double v, hipStream_t st);
hipError_t fill_u32(unsigned int *p, int64_t count, unsigned int v, hipStream_t st);
hipError_t residual_norms(const double *R_L, const double *R_R, int d, int64_t n, double *acc, hipStream_t st);

}  // namespace mrinv
