// Host runtime and C-ABI of mrinv: handles, FFT plans, workspace layout, the
// Newton driver for (e0 - q)^-1 and the Markov renewal functionals.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mrinv.h"
#include "common.h"
#include "kernels.h"

using namespace mrinv;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static mrinv_status_t fail(mrinv_status_t s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static mrinv_status_t fail(mrinv_status_t s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t _e = (expr);                                                                     \
        if (_e != hipSuccess) return fail(MRINV_E_HIP, "%s: %s", #expr, hipGetErrorString(_e));     \
    } while (0)

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------
// Handle scratch: MRINV_MAX_N doubles (1-lane scan input copies), 4096
// doubles of small vectors, then the time-scan workspace for up to 256 lanes.
constexpr size_t SCRATCH_SCAN_OFF = (size_t)MRINV_MAX_N + 4096;   // in doubles
constexpr size_t SCRATCH_BYTES =
    SCRATCH_SCAN_OFF * sizeof(double) + ((MRINV_MAX_N + 1023) / 1024) * 256 * sizeof(double);

// ---------------------------------------------------------------------------
// Library-owned workspace of mrinv_psi_inverse_noalloc: one device array of
// MRINV_NOALLOC_SCRATCH_BYTES on every GPU the library runs on, held until
// the process ends.  In host code `scratch` only names the array: its device
// address is looked up once per device (hipGetSymbolAddress with that device
// current, in mrinv_create) and that address is what the kernels receive.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[MRINV_NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_addr[NOALLOC_MAX_DEVICES];

// Device address of `scratch` on device dev (the current device).
static mrinv_status_t noalloc_scratch_lookup(int dev, void **out) {
    *out = nullptr;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(MRINV_E_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MRINV_E_HIP, "no device address for the library workspace");
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return MRINV_OK;
}

// Tuning of a new handle, also used where no handle is given (workspace
// queries), so that both plan the same launches.
static const mrinv_tuning_t kDefaultTune = {9, 0, 0, 1, 1, 1, 0, 0, 1, -1};

struct mrinv_handle_s {
    hipStream_t stream = nullptr;
    int device = 0;
    cplx<double> *tw64 = nullptr;   // hi[TW_HI_SIZE] then lo[TW_LO_SIZE] (used by both precisions)
    unsigned int *status = nullptr;
    double *scratch = nullptr;      // small per-handle scratch (index lists, vectors, 1-lane scans)
    void *timer = nullptr;          // launch timing records (mrinv_set_timing)
    bool timing = false;
    mrinv_tuning_t tune = kDefaultTune;
    // Graph of the last captured psi inversion and the call it belongs to.
    struct {
        bool valid = false;
        const void *src = nullptr, *out = nullptr, *ws = nullptr;
        size_t wsb = 0;
        int d = 0, e0 = 0, prec = 0;
        int64_t n = 0;
        mrinv_tuning_t tune{};
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    } gc;
    hipStream_t cap_stream = nullptr;
    void *batch = nullptr;          // plan of the last mrinv_psi_inverse_batched_prepare (BatchPlan)
    void *noalloc = nullptr;        // device address of `scratch` on this handle's device
    std::vector<mrinv_tuning_entry_t> table;   // per-(d, n, precision) tunings (mrinv_set_tuning_table)
    Twiddles<double> t64() const { return {tw64, tw64 + TW_HI_SIZE, tw64 + TW_HI_SIZE + TW_LO_SIZE, nullptr}; }
    Twiddles<float> t32() const { return {tw64, tw64 + TW_HI_SIZE, tw64 + TW_HI_SIZE + TW_LO_SIZE, nullptr}; }
};

static void host_twiddles(std::vector<double2> &hi, std::vector<double2> &lo) {
    hi.resize(TW_HI_SIZE);
    lo.resize(TW_LO_SIZE);
    auto w = [](int64_t a) {
        long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)a / (long double)TW_LMAX;
        double2 z;
        z.x = (double)cosl(ang);
        z.y = -(double)sinl(ang);
        return z;
    };
    for (int j = 0; j < TW_HI_SIZE; ++j) hi[j] = w((int64_t)j << TW_LO_BITS);
    for (int j = 0; j < TW_LO_SIZE; ++j) lo[j] = w(j);
}

static void batch_plan_free(void *plan);

extern "C" mrinv_status_t mrinv_create(mrinv_handle_t *handle, void *stream) {
    if (!handle) return fail(MRINV_E_ARG, "handle is NULL");
    *handle = nullptr;
    auto *h = new (std::nothrow) mrinv_handle_s();
    if (!h) return fail(MRINV_E_ARG, "out of host memory");
    h->stream = (hipStream_t)stream;
    // Any failure below releases what was made so far.
    auto init = [&]() -> mrinv_status_t {
        HIP_TRY(hipGetDevice(&h->device));
        const mrinv_status_t sst = noalloc_scratch_lookup(h->device, &h->noalloc);
        if (sst != MRINV_OK) return sst;
        std::vector<double2> hi, lo;
        host_twiddles(hi, lo);
        const size_t n64 = (TW_HI_SIZE + TW_LO_SIZE + 512) * sizeof(double2);
        // 512th roots W_512^j = W_{2^22}^{j 2^13} = hi[4j] (the lo factor is 1).
        std::vector<double2> root(512);
        for (int j = 0; j < 512; ++j) root[j] = hi[4 * j];
        HIP_TRY(hipMalloc((void **)&h->tw64, n64));
        HIP_TRY(hipMalloc((void **)&h->status, 256));
        HIP_TRY(hipMalloc((void **)&h->scratch, SCRATCH_BYTES));
        HIP_TRY(hipMemcpy(h->tw64, hi.data(), TW_HI_SIZE * sizeof(double2), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(h->tw64 + TW_HI_SIZE, lo.data(), TW_LO_SIZE * sizeof(double2), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(h->tw64 + TW_HI_SIZE + TW_LO_SIZE, root.data(), 512 * sizeof(double2),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemset(h->status, 0, 256));
        HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipDeviceSynchronize());
        return MRINV_OK;
    };
    const mrinv_status_t st = init();
    if (st != MRINV_OK) {
        const std::string msg = g_last_error;
        mrinv_destroy(h);
        g_last_error = msg;
        return st;
    }
    *handle = h;
    g_last_error.clear();
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_destroy(mrinv_handle_t h) {
    if (!h) return MRINV_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    if (h->tw64) (void)hipFree(h->tw64);
    if (h->status) (void)hipFree(h->status);
    if (h->scratch) (void)hipFree(h->scratch);
    if (h->timer) timer_destroy(h->timer);
    if (h->gc.exec) (void)hipGraphExecDestroy(h->gc.exec);
    if (h->gc.graph) (void)hipGraphDestroy(h->gc.graph);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    batch_plan_free(h->batch);
    delete h;
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_set_stream(mrinv_handle_t h, void *stream) {
    if (!h) return fail(MRINV_E_ARG, "handle is NULL");
    h->stream = (hipStream_t)stream;
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_sync_status(mrinv_handle_t h) {
    if (!h) return fail(MRINV_E_ARG, "handle is NULL");
    HIP_TRY(hipStreamSynchronize(h->stream));
    unsigned int s = 0;
    HIP_TRY(hipMemcpy(&s, h->status, sizeof s, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(h->status, 0, sizeof s));
    HIP_TRY(hipDeviceSynchronize());
    if (s & STATUS_SINGULAR) return fail(MRINV_E_SINGULAR_A0, "A(0) is singular to working precision");
    if (s & STATUS_NONFINITE) return fail(MRINV_E_NONFINITE, "non-finite value met on the device");
    return MRINV_OK;
}

extern "C" const char *mrinv_status_string(mrinv_status_t s) {
    switch (s) {
        case MRINV_OK: return "ok";
        case MRINV_E_ARG: return "invalid argument";
        case MRINV_E_SINGULAR_A0: return "A(0) singular";
        case MRINV_E_NONFINITE: return "non-finite value";
        case MRINV_E_WORKSPACE: return "workspace too small";
        case MRINV_E_UNSUPPORTED: return "unsupported size";
        case MRINV_E_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

extern "C" const char *mrinv_last_error(void) { return g_last_error.c_str(); }

// Activates launch timing for the duration of one entry point; entry points
// that call others keep the outermost scope's setting.
static thread_local int g_timer_depth = 0;
struct TimerScope {
    explicit TimerScope(mrinv_handle_t h) {
        if (g_timer_depth++ == 0) timer_activate(h && h->timing ? h->timer : nullptr, h ? h->stream : nullptr);
    }
    ~TimerScope() {
        if (--g_timer_depth == 0) timer_activate(nullptr, nullptr);
    }
};

extern "C" mrinv_status_t mrinv_set_timing(mrinv_handle_t h, int enabled) {
    if (!h) return fail(MRINV_E_ARG, "handle is NULL");
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (!h->timer) h->timer = timer_create();
    timer_reset(h->timer);
    h->timing = enabled != 0;
    return MRINV_OK;
}

namespace mrinv {
int timer_stats(void *t, hipStream_t st, mrinv_kernel_stat_t *out, int max_out);
}

extern "C" int mrinv_kernel_stats(mrinv_handle_t h, mrinv_kernel_stat_t *out, int max_out) {
    if (!h || !h->timer) return -1;
    return timer_stats(h->timer, h->stream, out, max_out);
}

namespace mrinv {
size_t hbm_probe_min_bytes();
hipError_t hbm_probe(hipStream_t st, void *buf, size_t bytes, int pattern, int lanes, int reps, double *gbps);
}

extern "C" mrinv_status_t mrinv_hbm_probe(mrinv_handle_t h, void *buf, size_t bytes, int pattern, int lanes,
                                          int reps, double *gbps) {
    if (!h || !buf || !gbps) return fail(MRINV_E_ARG, "NULL handle or pointer");
    if (pattern < MRINV_HBM_COPY || pattern > MRINV_HBM_PASS_LAST) return fail(MRINV_E_ARG, "unknown pattern %d", pattern);
    if (reps < 1 || reps > 100) return fail(MRINV_E_ARG, "reps %d not in 1..100", reps);
    if (((uintptr_t)buf & 15) != 0) return fail(MRINV_E_ARG, "buffer not 16-byte aligned");
    if (pattern == MRINV_HBM_COPY) {
        if (bytes < ((size_t)2 << 20)) return fail(MRINV_E_ARG, "copy probe needs at least 2 MiB");
    } else {
        if (lanes != 8 && lanes != 16 && lanes != 32) return fail(MRINV_E_ARG, "lanes %d not 8, 16 or 32", lanes);
        if (bytes < hbm_probe_min_bytes())
            return fail(MRINV_E_ARG, "pass probe needs at least %zu bytes", hbm_probe_min_bytes());
    }
    *gbps = 0.0;
    HIP_TRY(hbm_probe(h->stream, buf, bytes, pattern, lanes, reps, gbps));
    return MRINV_OK;
}

// ---------------------------------------------------------------------------
// Plans and workspace
// ---------------------------------------------------------------------------
static int ceil_log2(int64_t x) {
    int l = 0;
    while (((int64_t)1 << l) < x) ++l;
    return l;
}

// Transform length of a product truncated at n whose operands have n terms.
static int lg_full(int64_t n) { return std::max(1, ceil_log2(2 * n - 1)); }

// Radices of a transform of length 2^lgL, each at most 2^lgp_max.  One or two
// passes split the length evenly (the larger radix first).  Three or more
// passes give the last, contiguous pass the largest radix and split the rest
// evenly: the first pass then visits few rows of a zero-padded window.  At
// L = 2^19 (the mixed form's sweeps at d = 64) 5/5/9 beats the even 7/6/6
// by 4.5% per inversion (alternating runs on one GPU); the same rule for two
// passes (8/9 at 2^17, 7/9 at 2^16) was 1-2% slower.
static FftPlan make_plan(int lgL, int lgp_max = LGP_MAX) {
    FftPlan p{};
    p.lgL = lgL;
    p.npass = (lgL + lgp_max - 1) / lgp_max;
    if (p.npass < 1) p.npass = 1;
    int rem = lgL;
    int even = p.npass;                   // passes split evenly
    if (p.npass >= 3) {
        p.lgP[p.npass - 1] = lgp_max;
        rem -= lgp_max;
        even = p.npass - 1;
    }
    for (int j = 0; j < even; ++j) {
        const int left = even - j;
        p.lgP[j] = (rem + left - 1) / left;
        rem -= p.lgP[j];
    }
    return p;
}

static inline int nl_of(int64_t lanes) { return (int)((lanes + 1) / 2); }
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
// Bytes of one packed spectrum of length 2^lgL with `lanes` real lanes.
static size_t spec_bytes(int lgL, int64_t lanes, bool dbl) {
    return align256(((size_t)1 << lgL) * nl_of(lanes) * (dbl ? 16 : 8));
}

struct Carve {
    char *p;
    size_t used = 0;
    explicit Carve(void *base) : p((char *)base) {}
    template <typename X> X *take(size_t bytes) {
        X *r = (X *)(p + used);
        used += align256(bytes);
        return r;
    }
};

// Precisions: FP64 (cyclic length m' per Newton step), FP64_PADDED (the
// zero-padded length 2m' of every step), and the two mixed forms (float32
// Newton with float32 or split-BF16 products, then float64 residual sweeps).
static bool prec_valid(mrinv_precision_t p) { return p >= MRINV_FP64 && p <= MRINV_FP64_PADDED; }
static bool prec_mixed(mrinv_precision_t p) { return p == MRINV_MIXED_FP32 || p == MRINV_MIXED_BF16X3; }
static int prec_pad(mrinv_precision_t p) { return p == MRINV_FP64_PADDED ? 1 : 0; }
static int prec_bf3(mrinv_precision_t p) { return p == MRINV_MIXED_BF16X3 ? 1 : 0; }

// Outer-twiddle tables of all Newton steps up to 2^lgN plus, for the mixed
// form, the sweep length 2^lg2 in both precisions (bounds valid for every
// pass split: tables of one plan hold at most 1.1 L entries).
static size_t ws_twiddles(int lgN, int lg2, mrinv_precision_t prec) {
    const size_t L = (size_t)1 << lgN;
    if (!prec_mixed(prec)) return align256(3 * L * 16) + 4096;
    return align256(3 * L * 8) + align256(2 * ((size_t)1 << lg2) * 16) + align256(2 * ((size_t)1 << lg2) * 8) + 4096;
}

// Spectra of one problem's residual sweeps at length 2^lg: A, X and the
// products in float64 (slots 0-2), then X's spectrum in float32 (slot 3).
// The float32 spectra of R and of the correction reuse slots 1-2 once the
// float64 residual is formed.
static size_t sweep_bytes(int lg, int64_t d2) { return 3 * spec_bytes(lg, d2, true) + spec_bytes(lg, d2, false); }

static size_t ws_psi(int d, int64_t n, mrinv_precision_t prec) {
    const int64_t d2 = (int64_t)d * d;
    const int lgN = std::max(1, ceil_log2(n));
    const int lg2 = lg_full(n);
    if (!prec_mixed(prec)) {
        const int lgS = lgN + prec_pad(prec);
        return 3 * spec_bytes(lgS, d2, true) + ws_twiddles(lgS, lg2, prec);
    }
    // Sweeps: three float64 spectra at 2^lg2 plus the float32 copy of X's spectrum.
    size_t spec = std::max(3 * spec_bytes(lgN, d2, false), sweep_bytes(lg2, d2));
    return spec + 2 * align256((size_t)n * d2 * sizeof(float)) + ws_twiddles(lgN, lg2, prec);
}

static size_t ws_apply(int d, int64_t n, int r) {
    const int lg = lg_full(n);
    return spec_bytes(lg, (int64_t)d * d, true) + 2 * spec_bytes(lg, (int64_t)d * r, true);
}

static size_t ws_transition(int d, int64_t n) {
    const int lg = lg_full(n);
    return align256((size_t)n * d * sizeof(double)) + spec_bytes(lg, (int64_t)d * d, true) + spec_bytes(lg, d, true);
}

static size_t ws_residual(int d, int64_t n) {
    const int64_t d2 = (int64_t)d * d;
    return 3 * spec_bytes(lg_full(n), d2, true) + 2 * align256((size_t)n * d2 * 8);
}

static size_t ws_psi_backward(int d, int64_t n) { return 3 * spec_bytes(lg_full(n), (int64_t)d * d, true); }

static size_t ws_apply_backward(int d, int64_t n, int r) {
    const int lg = lg_full(n);
    return spec_bytes(lg, (int64_t)d * d, true) + 2 * spec_bytes(lg, (int64_t)d * r, true);
}

static size_t ws_transition_backward(int d, int64_t n) {
    const int lg = lg_full(n);
    return align256((size_t)n * d * sizeof(double)) * 2 + 2 * spec_bytes(lg, (int64_t)d * d, true) +
           spec_bytes(lg, d, true);
}

static size_t ws_first_entrance(int d, int64_t n, int nD, mrinv_precision_t prec) {
    const int nC = d - nD;
    if (nC <= 0) return 256;
    // q_CC, psi_C, q_CD and g_D, then the larger of the inverse and apply workspaces.
    const size_t blocks = 2 * align256((size_t)n * nC * nC * 8) + 2 * align256((size_t)n * nC * nD * 8);
    return blocks + std::max(ws_psi(nC, n, prec), ws_apply(nC, n, nD));
}

// Series Gauss-Jordan: W [n][d][2d], the pivot series and its inverse, the
// multipliers, the pivot bookkeeping, five spectra at the product length
// (pivot inverse, pivot row, normalised row, multipliers, update) and the
// scalar inverse's own workspace.
static size_t ws_gj(int d, int64_t n) {
    const int lg = lg_full(n);
    return align256((size_t)n * d * 2 * d * 8) + 2 * align256((size_t)n * 8) + align256((size_t)n * d * 8) + 256 +
           spec_bytes(lg, 1, true) + 2 * spec_bytes(lg, 2 * d, true) + spec_bytes(lg, d, true) +
           spec_bytes(lg, (int64_t)2 * d * d, true) + ws_psi(1, n, MRINV_FP64_PADDED);
}

static size_t ws_mre(int d, int64_t n, int r, mrinv_precision_t prec) {
    // Qbar, (e0 - Qbar)^-1 and the right-hand side, then the inverse's or the product's workspace.
    return 2 * align256((size_t)n * d * d * 8) + align256((size_t)n * d * r * 8) +
           std::max(ws_psi(d, n, prec), ws_apply(d, n, r));
}

extern "C" size_t mrinv_workspace_size(mrinv_op_t op, int d, int64_t n, int r, mrinv_precision_t prec) {
    if (d < 1 || d > MRINV_MAX_D || n < 1 || n > MRINV_MAX_N) return 0;
    switch (op) {
        case MRINV_OP_PSI_INVERSE: return ws_psi(d, n, prec);
        case MRINV_OP_APPLY: return (r < 1 || r > MRINV_MAX_D) ? 0 : ws_apply(d, n, r);
        case MRINV_OP_TRANSITION: return ws_transition(d, n);
        case MRINV_OP_PSI_BACKWARD: return ws_psi_backward(d, n);
        case MRINV_OP_APPLY_BACKWARD: return (r < 1 || r > MRINV_MAX_D) ? 0 : ws_apply_backward(d, n, r);
        case MRINV_OP_TRANSITION_BACKWARD: return ws_transition_backward(d, n);
        case MRINV_OP_FIRST_ENTRANCE: return (r < 1 || r > d) ? 0 : ws_first_entrance(d, n, r, prec);
        case MRINV_OP_AVAILABILITY: return 256;
        case MRINV_OP_RESIDUAL: return ws_residual(d, n);
        case MRINV_OP_MRE: return (r < 1 || r > MRINV_MAX_D) ? 0 : ws_mre(d, n, r, prec);
        case MRINV_OP_GJ: return ws_gj(d, n);
    }
    return 0;
}

// ---------------------------------------------------------------------------
// Transform helpers
// ---------------------------------------------------------------------------
template <typename T> static Twiddles<T> tw_of(mrinv_handle_t h);
template <> Twiddles<double> tw_of<double>(mrinv_handle_t h) {
    if (!h) return Twiddles<double>{};
    Twiddles<double> t = h->t64();
    if (h->tune.twiddle_tables == 0) t.root = nullptr;
    return t;
}
template <> Twiddles<float> tw_of<float>(mrinv_handle_t h) {
    if (!h) return Twiddles<float>{};
    Twiddles<float> t = h->t32();
    if (h->tune.twiddle_tables == 0) t.root = nullptr;
    return t;
}

static SrcDesc src_real(const void *p, bool dbl, int64_t ld, int nreal, int64_t lo, int64_t hi, int64_t rev = -1,
                        int e0_d = 0) {
    SrcDesc s{};
    s.kind = dbl ? SRC_REAL64 : SRC_REAL32;
    s.p = p;
    s.ld = ld;
    s.nreal = nreal;
    s.lo = lo;
    s.hi = hi;
    s.rev = rev;
    s.e0_d = e0_d;
    return s;
}

static DstDesc dst_real(void *p, bool dbl, int64_t ld, int nreal, int64_t lo, int64_t hi, double scale, int op,
                        int64_t rev = -1, unsigned int *status = nullptr) {
    DstDesc d{};
    d.kind = dbl ? DST_REAL64 : DST_REAL32;
    d.p = p;
    d.ld = ld;
    d.nreal = nreal;
    d.lo = lo;
    d.hi = hi;
    d.scale = scale;
    d.op = op;
    d.rev = rev;
    d.status = status;
    return d;
}

static const mrinv_tuning_t &tune_of(mrinv_handle_t h) { return h ? h->tune : kDefaultTune; }

// Tuning of a problem: the first table entry whose ranges hold (d, n) and
// whose precision matches (-1 matches any), else the handle's.
static const mrinv_tuning_t &tune_for(mrinv_handle_t h, int d, int64_t n, int prec) {
    if (h)
        for (const auto &e : h->table)
            if (d >= e.d_lo && d <= e.d_hi && n >= e.n_lo && n <= e.n_hi && (e.precision < 0 || e.precision == prec))
                return e.tune;
    return tune_of(h);
}

// The table's tuning for one call: installed in the handle for the call's
// duration and restored after it (calls made inside keep their own scope).
struct TuneScope {
    mrinv_handle_t h = nullptr;
    mrinv_tuning_t saved{};
    TuneScope(mrinv_handle_t hh, int d, int64_t n, int prec) {
        if (!hh || hh->table.empty()) return;
        h = hh;
        saved = hh->tune;
        const mrinv_tuning_t t = tune_for(hh, d, n, prec);
        hh->tune = t;
    }
    ~TuneScope() {
        if (h) h->tune = saved;
    }
};
static int order_of(mrinv_handle_t h) { return tune_of(h).block_order; }
template <typename T> static int lanes_of(mrinv_handle_t h) {
    return sizeof(T) == 8 ? tune_of(h).lanes_fp64 : tune_of(h).lanes_fp32;
}
static FftPlan hplan(mrinv_handle_t h, int lgL) { return make_plan(lgL, tune_of(h).lgp_max); }

// Destination of forward pass j: in place, and for the last pass of a float64
// transform optionally also a float32 copy of the spectrum at aux32.
static DstDesc fwd_dst(const FftPlan &p, int j, const void *aux32) {
    DstDesc d = dst_z();
    if (j == p.npass - 1) d.aux = aux32;
    return d;
}

// Forward transform of a real source into Z (all passes).
template <typename T>
static hipError_t fwd(mrinv_handle_t h, const FftPlan &p, int nl, cplx<T> *Z, const SrcDesc &src,
                      const void *aux32 = nullptr) {
    const Twiddles<T> tw = tw_of<T>(h);
    const int ln = lanes_of<T>(h);
    hipError_t e = fft_pass<T>(0, p, 0, nl, Z, src, fwd_dst(p, 0, aux32), tw, h->stream, ln, order_of(h));
    for (int j = 1; j < p.npass && e == hipSuccess; ++j)
        e = fft_pass<T>(0, p, j, nl, Z, src_z(), fwd_dst(p, j, aux32), tw, h->stream, ln, order_of(h));
    return e;
}

// Forward transforms of two real sources (same plan) into ZA and ZB; with
// pair_forward each pass of both is one launch.
template <typename T>
static hipError_t fwd2(mrinv_handle_t h, const FftPlan &p, int nl, cplx<T> *ZA, const SrcDesc &sa, cplx<T> *ZB,
                       const SrcDesc &sb, const void *aux32_b = nullptr) {
    if (!h->tune.pair_forward) {
        hipError_t e = fwd<T>(h, p, nl, ZA, sa);
        return e == hipSuccess ? fwd<T>(h, p, nl, ZB, sb, aux32_b) : e;
    }
    const Twiddles<T> tw = tw_of<T>(h);
    PassProblem<T> a{}, b{};
    a.z = ZA; a.nl = nl; a.src = sa; a.dst = dst_z();
    b.z = ZB; b.nl = nl; b.src = sb; b.dst = fwd_dst(p, 0, aux32_b);
    hipError_t e = fft_pass_pair<T>(p, 0, a, b, tw, h->stream, lanes_of<T>(h), order_of(h));
    a.src = src_z();
    b.src = src_z();
    for (int j = 1; j < p.npass && e == hipSuccess; ++j) {
        b.dst = fwd_dst(p, j, aux32_b);
        e = fft_pass_pair<T>(p, j, a, b, tw, h->stream, lanes_of<T>(h), order_of(h));
    }
    return e;
}

// Inverse transform of Z into a real destination (all passes).
template <typename T>
static hipError_t inv(mrinv_handle_t h, const FftPlan &p, int nl, cplx<T> *Z, const DstDesc &dst) {
    const Twiddles<T> tw = tw_of<T>(h);
    const int ln = lanes_of<T>(h);
    hipError_t e = hipSuccess;
    for (int j = p.npass - 1; j >= 1 && e == hipSuccess; --j)
        e = fft_pass<T>(1, p, j, nl, Z, src_z(), dst_z(), tw, h->stream, ln, order_of(h));
    if (e == hipSuccess) e = fft_pass<T>(1, p, 0, nl, Z, src_z(), dst, tw, h->stream, ln, order_of(h));
    return e;
}

// Z <- DFT(mask(IDFT(Z))): time rows outside [lo, hi) are zeroed, the rest
// scaled by 1/L (and negated when neg).
template <typename T>
static hipError_t remask(mrinv_handle_t h, const FftPlan &p, int nl, cplx<T> *Z, int64_t lo, int64_t hi, bool neg) {
    const Twiddles<T> tw = tw_of<T>(h);
    const int ln = lanes_of<T>(h);
    hipError_t e = hipSuccess;
    for (int j = p.npass - 1; j >= 1 && e == hipSuccess; --j)
        e = fft_pass<T>(1, p, j, nl, Z, src_z(), dst_z(), tw, h->stream, ln, order_of(h));
    DstDesc m = dst_z();
    m.lo = lo;
    m.hi = hi;
    m.op = neg ? OP_NEG : OP_STORE;
    m.scale = 1.0 / (double)((int64_t)1 << p.lgL);
    if (e == hipSuccess) e = fft_pass<T>(2, p, 0, nl, Z, src_z(), m, tw, h->stream, ln, order_of(h));
    for (int j = 1; j < p.npass && e == hipSuccess; ++j)
        e = fft_pass<T>(0, p, j, nl, Z, src_z(), dst_z(), tw, h->stream, ln, order_of(h));
    return e;
}

static GemmDesc gdesc(mrinv_handle_t h, int ra, int m, int cb, int ta = 0, int tb = 0) {
    GemmDesc g{};
    g.mfma = tune_of(h).mfma;
    g.ra = ra;
    g.m = m;
    g.cb = cb;
    g.transA = ta;
    g.transB = tb;
    g.nlA = nl_of((int64_t)ra * m);
    g.nlB = nl_of((int64_t)m * cb);
    g.nlC = nl_of((int64_t)ra * cb);
    return g;
}

// Length of the recursion seed: the largest power of two <= min(seed_m0, n).
static int64_t seed_len(const mrinv_tuning_t &t, int64_t n) {
    const int64_t cap = std::min<int64_t>(t.seed_m0, n);
    int64_t m0 = 1;
    while (2 * m0 <= cap) m0 *= 2;
    return m0;
}
static int64_t seed_len(mrinv_handle_t h, int64_t n) { return seed_len(tune_of(h), n); }

// Newton steps m -> m2 with m2 <= direct_limit run as direct products in the
// time domain.  Automatic choice: the largest power of two M for which the
// step M/2 -> M costs at most 1.2e8 multiply-adds (1.5 (M/2)^2 D^3 with D = d
// rounded up to the 16-wide matrix tiles); below that the transform launches'
// fixed latency costs more (measured crossover: M = 256 at d = 16).  0 turns
// the direct steps off.
static int64_t direct_limit(const mrinv_tuning_t &t, int d) {
    const int v = t.direct_m;
    if (v == 0) return 0;
    int64_t M = 1;
    if (v > 0) {
        while (2 * M <= v) M *= 2;
        return M;
    }
    const double D = 16.0 * ((d + 15) / 16);
    while (1.5 * (double)M * (double)M * D * D * D <= 1.2e8) M *= 2;   // M is twice the step's m
    return M;
}
static int64_t direct_limit(mrinv_handle_t h, int d) { return direct_limit(tune_of(h), d); }

// Register the outer-twiddle tables of plan p (every pass but the last,
// whose column offset is always 0) in g, carving them from region.
static void add_tables(TwGen &g, FftPlan &p, bool dbl, char *&region, char *end) {
    int lgB = p.lgL;
    for (int j = 0; j < p.npass; ++j) {
        const size_t bytes = align256(((size_t)1 << lgB) * (dbl ? 16 : 8));
        if (j < p.npass - 1 && g.count < MAX_TW_TABLES && region + bytes <= end) {
            g.begin[g.count] = g.total;
            g.dst[g.count] = region;
            g.lgB[g.count] = lgB;
            g.lgP[g.count] = p.lgP[j];
            g.dbl[g.count] = dbl ? 1 : 0;
            g.total += (int64_t)1 << lgB;
            g.count++;
            p.outer[j] = region;
            region += bytes;
        }
        lgB -= p.lgP[j];
    }
}

// ---------------------------------------------------------------------------
// Newton inversion (eq. (newton)) in precision T.  src is A (e0 == 0) or q
// (e0 == 1, A = e0 - q); the result's coefficients are written to out
// (float64 when T is double, float32 otherwise), rows 0..n-1.
// Step m -> m' = min(2m, n) at length L = 2^ceil(log2 m'):
//   T  = A mod x^m' * B  (cyclic of length L; wrap-around lands in [0, m))
//   E  = -T on [m, m')   (A*B = e0 mod x^m, so e0 - A*B vanishes below m)
//   B[m, m') = (B * E)[m, m')
// ---------------------------------------------------------------------------
template <typename T>
static mrinv_status_t newton(mrinv_handle_t h, const double *src, int e0, int d, int64_t n, void *out,
                             cplx<T> *SA, cplx<T> *SB, cplx<T> *ST, char *twr, char *twr_end, int pad, int bf3) {
    const bool dbl = sizeof(T) == 8;
    const int d2 = d * d;
    const int nl = nl_of(d2);
    HIP_TRY(gj_inverse(src, d, e0, dbl ? (double *)out : nullptr, dbl ? nullptr : (float *)out, h->status, h->stream));
    // The first m0 coefficients by the coefficient recursion (one launch),
    // then Newton doubling from m0.
    int64_t m0 = seed_len(h, n);
    if (m0 > 1) HIP_TRY(seed_recursion<T>(src, e0, d, (int)m0, (T *)out, h->stream));
    // Direct steps: E = -A*X on [m, m2) into scratch (SA), then X[m, m2) = X*E.
    const int64_t dlim = direct_limit(h, d);
    for (; m0 < n && std::min(2 * m0, n) <= dlim; m0 = std::min(2 * m0, n)) {
        const int64_t m2 = std::min(2 * m0, n);
        ConvDesc c{};
        c.L = src;
        c.l_f64 = 1;
        c.R = out;
        c.out = SA;
        c.d = d;
        c.sign = e0 ? 1.0 : -1.0;   // -A(l) = q(l) for l >= 1 in the renewal form
        c.k0 = m0;
        c.k1 = m2;
        c.jlo = 0;
        c.jhi = m0 - 1;
        c.r_off = 0;
        c.out_off = m0;
        HIP_TRY(conv_direct<T>(c, h->stream));
        ConvDesc u{};
        u.L = out;
        u.l_f64 = dbl;
        u.R = SA;
        u.out = out;
        u.d = d;
        u.sign = 1.0;
        u.k0 = m0;
        u.k1 = m2;
        u.jlo = m0;
        u.jhi = m2;
        u.r_off = m0;
        u.out_off = 0;
        u.status = dbl ? h->status : nullptr;
        HIP_TRY(conv_direct<T>(u, h->stream));
    }
    GemmDesc g = gdesc(h, d, d, d);
    g.bf3 = bf3;
    // Plans of every step and their outer-twiddle tables (one launch).
    // At most log2(MRINV_MAX_N) + 1 steps; a fixed array keeps the driver free
    // of host allocations.
    FftPlan plans[32];
    int nplans = 0;
    TwGen tg{};
    for (int64_t m = m0; m < n && nplans < 32; m = std::min(2 * m, n)) {
        plans[nplans] = hplan(h, ceil_log2(std::min(2 * m, n)) + pad);
        if (twr && h->tune.twiddle_tables >= 2) add_tables(tg, plans[nplans], dbl, twr, twr_end);
        ++nplans;
    }
    HIP_TRY(gen_outer_twiddles(tg, h->tw64, h->tw64 + TW_HI_SIZE, h->stream));
    size_t step = 0;
    for (int64_t m = m0; m < n;) {
        const int64_t m2 = std::min(2 * m, n);
        const FftPlan p = plans[step++];
        const double invL = 1.0 / (double)((int64_t)1 << p.lgL);
        HIP_TRY(fwd2<T>(h, p, nl, SA, src_real(src, true, d2, d2, 0, m2, -1, e0 ? d : 0), SB,
                        src_real(out, dbl, d2, d2, 0, m)));
        HIP_TRY(freq_gemm<T>(p, g, SA, SB, ST, h->stream));
        HIP_TRY(remask<T>(h, p, nl, ST, m, m2, true));
        HIP_TRY(freq_gemm<T>(p, g, SB, ST, SA, h->stream));
        HIP_TRY(inv<T>(h, p, nl, SA, dst_real(out, dbl, d2, d2, m, m2, invL, OP_STORE, -1, h->status)));
        m = m2;
    }
    return MRINV_OK;
}

static mrinv_status_t check_dn(int d, int64_t n) {
    if (d < 1 || n < 1) return fail(MRINV_E_ARG, "need d >= 1 and n >= 1 (d=%d, n=%lld)", d, (long long)n);
    if (d > MRINV_MAX_D) return fail(MRINV_E_UNSUPPORTED, "d=%d exceeds %d", d, MRINV_MAX_D);
    if (n > MRINV_MAX_N) return fail(MRINV_E_UNSUPPORTED, "n=%lld exceeds %lld", (long long)n, (long long)MRINV_MAX_N);
    return MRINV_OK;
}

// The recursion seed keeps a column's history, A(0)^-1 and its partial sums in
// LDS; launches stay within the 64 KiB of dynamic LDS a kernel gets without
// a raised limit (at d = 64 that allows seeds of up to 32 coefficients).
constexpr size_t SEED_LDS_MAX = 64 * 1024;

static mrinv_status_t check_seed(int64_t m0, int d) {
    if (m0 > 1 && seed_lds_bytes((int)m0, d) > SEED_LDS_MAX)
        return fail(MRINV_E_UNSUPPORTED, "seed_m0=%lld at d=%d needs %zu bytes of LDS (limit %zu)", (long long)m0, d,
                    seed_lds_bytes((int)m0, d), SEED_LDS_MAX);
    return MRINV_OK;
}

static mrinv_status_t check_ws(void *ws, size_t have, size_t need) {
    if (need > have) return fail(MRINV_E_WORKSPACE, "workspace %zu bytes < %zu needed", have, need);
    if (need && !ws) return fail(MRINV_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws) & 255) return fail(MRINV_E_WORKSPACE, "workspace not 256-byte aligned");
    return MRINV_OK;
}

#define CHECK(expr)                          \
    do {                                     \
        mrinv_status_t _s = (expr);          \
        if (_s != MRINV_OK) return _s;       \
    } while (0)

// Residual sweeps of the mixed form.  Each one forms R = e0 - A*X in float64
// over the whole horizon and applies X <- X + X*R, which squares the residual
// (Appendix "Algorithmic details": e0 - A*B_{r+1} = (e0 - A*B_r)^2).  With the
// float32 Newton error of long renewal horizons (about 1e-6), one sweep leaves
// about 1e-10 and a second one reaches float64 rounding.
constexpr int MIXED_SWEEPS = 2;

static mrinv_status_t inverse_impl(mrinv_handle_t h, const double *src, int e0, int d, int64_t n,
                                   mrinv_precision_t prec, double *out, void *ws, size_t wsb) {
    if (!h || !src || !out) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    if (!prec_valid(prec)) return fail(MRINV_E_ARG, "unknown precision %d", (int)prec);
    CHECK(check_ws(ws, wsb, ws_psi(d, n, prec)));
    CHECK(check_seed(seed_len(h, n), d));
    const int64_t d2 = (int64_t)d * d;
    const int nl = nl_of(d2);
    const int lgN = std::max(1, ceil_log2(n));
    Carve cv(ws);
    const int pad = prec_pad(prec), bf3 = prec_bf3(prec);
    const size_t twb = ws_twiddles(lgN + pad, lg_full(n), prec);
    char *twr = cv.take<char>(twb);
    char *twr_end = twr + twb;
    if (!prec_mixed(prec)) {
        const size_t sb = spec_bytes(lgN + pad, d2, true);
        auto *SA = cv.take<cplx<double>>(sb);
        auto *SB = cv.take<cplx<double>>(sb);
        auto *ST = cv.take<cplx<double>>(sb);
        return newton<double>(h, src, e0, d, n, out, SA, SB, ST, twr, twr_end, pad, 0);
    }
    // Mixed: float32 Newton into X, then one sweep with a float64 residual.
    float *X = cv.take<float>((size_t)n * d2 * sizeof(float));
    float *R = cv.take<float>((size_t)n * d2 * sizeof(float));
    char *spec = cv.p + cv.used;
    {
        const size_t sb = spec_bytes(lgN, d2, false);
        auto *SA = (cplx<float> *)spec;
        auto *SB = (cplx<float> *)(spec + sb);
        auto *ST = (cplx<float> *)(spec + 2 * sb);
        CHECK(newton<float>(h, src, e0, d, n, X, SA, SB, ST, twr, twr_end, 0, bf3));
    }
    // The sweep plan in both precisions, each with its own outer tables
    // (carved after the Newton tables, which newton() left in the region).
    FftPlan p2 = hplan(h, lg_full(n));
    FftPlan p2f = p2;
    {
        char *r2 = twr + align256(3 * ((size_t)1 << lgN) * 8);
        TwGen tg{};
        if (h->tune.twiddle_tables >= 2) {
            add_tables(tg, p2, true, r2, twr_end);
            add_tables(tg, p2f, false, r2, twr_end);
        }
        HIP_TRY(gen_outer_twiddles(tg, h->tw64, h->tw64 + TW_HI_SIZE, h->stream));
    }
    const double invL = 1.0 / (double)((int64_t)1 << p2.lgL);
    const GemmDesc g = gdesc(h, d, d, d);
    GemmDesc g32 = g;
    g32.bf3 = bf3;
    // Slots (sweep_bytes): A's float64 spectrum, formed once and kept for
    // every sweep; X's float64 spectrum, whose last forward pass also writes
    // the float32 copy into slot 3 for the correction product; the float64
    // product.  The float32 spectra of R and of the correction take slots 1-2
    // once R is formed.
    const size_t s64 = spec_bytes(p2.lgL, d2, true), s32 = spec_bytes(p2.lgL, d2, false);
    auto *SA = (cplx<double> *)spec;
    auto *SB = (cplx<double> *)(spec + s64);
    auto *ST = (cplx<double> *)(spec + 2 * s64);
    auto *X32 = (cplx<float> *)(spec + 3 * s64);
    auto *R32 = (cplx<float> *)(spec + s64);
    auto *T32 = (cplx<float> *)(spec + s64 + s32);
    for (int sweep = 0; sweep < MIXED_SWEEPS; ++sweep) {
        const bool last = sweep == MIXED_SWEEPS - 1;
        // R = e0 - A*X on [0, n) in float64 (full product, no wrap-around at L >= 2n-1).
        const SrcDesc sa = src_real(src, true, d2, d2, 0, n, -1, e0 ? d : 0), sx = src_real(X, false, d2, d2, 0, n);
        if (sweep == 0) HIP_TRY(fwd2<double>(h, p2, nl, SA, sa, SB, sx, X32));
        else HIP_TRY(fwd<double>(h, p2, nl, SB, sx, X32));
        HIP_TRY(freq_gemm<double>(p2, g, SA, SB, ST, h->stream));
        DstDesc dr = dst_real(R, false, d2, d2, 0, n, invL, OP_E0MINUS);
        dr.e0_d = d;
        HIP_TRY(inv<double>(h, p2, nl, ST, dr));
        // X <- X + X*R, the correction product in float32; the last sweep
        // writes the float64 result, earlier ones update X in place.
        HIP_TRY(fwd<float>(h, p2f, nl, R32, src_real(R, false, d2, d2, 0, n)));
        HIP_TRY(freq_gemm<float>(p2f, g32, X32, R32, T32, h->stream));
        DstDesc dx = last ? dst_real(out, true, d2, d2, 0, n, invL, OP_XPLUS, -1, h->status)
                          : dst_real(X, false, d2, d2, 0, n, invL, OP_XPLUS);
        dx.aux = X;
        HIP_TRY(inv<float>(h, p2f, nl, T32, dx));
    }
    return MRINV_OK;
}

// inverse_impl, recorded into a HIP graph on the handle's capture stream the
// first time a (pointers, sizes, tuning) key is seen and replayed on the
// caller's stream afterwards.  Argument errors are reported before recording.
static mrinv_status_t inverse_graphed(mrinv_handle_t h, const double *src, int e0, int d, int64_t n,
                                      mrinv_precision_t prec, double *out, void *ws, size_t wsb) {
    auto &gc = h->gc;
    const bool hit = gc.valid && gc.src == src && gc.out == out && gc.ws == ws && gc.wsb == wsb && gc.d == d &&
                     gc.n == n && gc.e0 == e0 && gc.prec == (int)prec &&
                     memcmp(&gc.tune, &h->tune, sizeof(mrinv_tuning_t)) == 0;
    if (!hit) {
        if (!src || !out) return fail(MRINV_E_ARG, "NULL handle or pointer");
        CHECK(check_dn(d, n));
        CHECK(check_ws(ws, wsb, ws_psi(d, n, prec)));
        if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
        if (gc.graph) (void)hipGraphDestroy(gc.graph);
        gc.exec = nullptr;
        gc.graph = nullptr;
        gc.valid = false;
        hipStream_t caller = h->stream;
        h->stream = h->cap_stream;
        HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        mrinv_status_t st = inverse_impl(h, src, e0, d, n, prec, out, ws, wsb);
        hipGraph_t g = nullptr;
        hipError_t ec = hipStreamEndCapture(h->cap_stream, &g);
        h->stream = caller;
        if (st != MRINV_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        HIP_TRY(ec);
        hipGraphExec_t ex = nullptr;
        HIP_TRY(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        gc.graph = g;
        gc.exec = ex;
        gc.src = src;
        gc.out = out;
        gc.ws = ws;
        gc.wsb = wsb;
        gc.d = d;
        gc.n = n;
        gc.e0 = e0;
        gc.prec = (int)prec;
        gc.tune = h->tune;
        gc.valid = true;
    }
    HIP_TRY(hipGraphLaunch(gc.exec, h->stream));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_psi_inverse(mrinv_handle_t h, const double *q, int d, int64_t n,
                                            mrinv_precision_t precision, double *psi, void *ws, size_t ws_bytes) {
    TimerScope _ts(h);
    TuneScope _tn(h, d, n, (int)precision);
    if (h && h->tune.use_graph && !h->timing) return inverse_graphed(h, q, 1, d, n, precision, psi, ws, ws_bytes);
    return inverse_impl(h, q, 1, d, n, precision, psi, ws, ws_bytes);
}

extern "C" mrinv_status_t mrinv_series_inverse(mrinv_handle_t h, const double *A, int d, int64_t n,
                                               mrinv_precision_t precision, double *Ainv, void *ws,
                                               size_t ws_bytes) {
    TimerScope _ts(h);
    TuneScope _tn(h, d, n, (int)precision);
    if (h && h->tune.use_graph && !h->timing) return inverse_graphed(h, A, 0, d, n, precision, Ainv, ws, ws_bytes);
    return inverse_impl(h, A, 0, d, n, precision, Ainv, ws, ws_bytes);
}

extern "C" mrinv_status_t mrinv_psi_inverse_noalloc(mrinv_handle_t h, const double *q, int d, int64_t n,
                                                    mrinv_precision_t precision, double *psi) {
    if (!h || !q || !psi) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    if (!prec_valid(precision)) return fail(MRINV_E_ARG, "unknown precision %d", (int)precision);
    const size_t need = ws_psi(d, n, precision);
    if (need > (size_t)MRINV_NOALLOC_SCRATCH_BYTES)
        return fail(MRINV_E_WORKSPACE,
                    "d=%d n=%lld needs %zu bytes of workspace; the library-owned array holds %zu "
                    "(use mrinv_psi_inverse with a caller workspace)",
                    d, (long long)n, need, (size_t)MRINV_NOALLOC_SCRATCH_BYTES);
    if (!h->noalloc) return fail(MRINV_E_HIP, "library workspace not set up on this handle's device");
    TuneScope _tn(h, d, n, (int)precision);
    return inverse_impl(h, q, 1, d, n, precision, psi, h->noalloc, MRINV_NOALLOC_SCRATCH_BYTES);
}

// ---------------------------------------------------------------------------
// FFT-Gauss-Jordan inversion over C[[x]]/<x^n> (Appendix, Gauss-Jordan
// paragraph).  On W = [A | I], pivot i: choose the row with the largest
// |constant coefficient| in column i and swap it into row i; invert the pivot
// series by Newton's iteration (the d = 1 inverse); normalise row i by that
// inverse; subtract from every other row r its multiplier W_ri times the
// normalised row.  Every series product is a transform product at length
// 2^ceil(log2(2n-1)) truncated to n.  After d pivots the right block is
// A^(-1) mod x^n.
// ---------------------------------------------------------------------------
static mrinv_status_t gj_series_impl(mrinv_handle_t h, const double *src, int e0, int d, int64_t n, double *out,
                                     void *ws, size_t wsb) {
    if (!h || !src || !out) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    CHECK(check_ws(ws, wsb, ws_gj(d, n)));
    CHECK(check_seed(seed_len(h, n), 1));
    const FftPlan p = hplan(h, lg_full(n));
    const int lg = p.lgL;
    const int64_t w = 2 * d, ww = (int64_t)d * w;
    const double invL = 1.0 / (double)((int64_t)1 << lg);
    Carve cv(ws);
    double *W = cv.take<double>((size_t)n * ww * 8);
    double *u = cv.take<double>((size_t)n * 8);
    double *v = cv.take<double>((size_t)n * 8);
    double *col = cv.take<double>((size_t)n * d * 8);
    char *book = cv.take<char>(256);
    int *piv = (int *)book;
    double *aux = (double *)(book + 128);
    auto *SV = cv.take<cplx<double>>(spec_bytes(lg, 1, true));
    auto *SR = cv.take<cplx<double>>(spec_bytes(lg, w, true));
    auto *SP = cv.take<cplx<double>>(spec_bytes(lg, w, true));
    auto *SC = cv.take<cplx<double>>(spec_bytes(lg, d, true));
    auto *SU = cv.take<cplx<double>>(spec_bytes(lg, ww, true));
    void *wsi = cv.p + cv.used;
    const size_t wsib = ws_psi(1, n, MRINV_FP64_PADDED);
    HIP_TRY(gjs_init(src, e0, n, d, W, h->stream));
    for (int i = 0; i < d; ++i) {
        double *row = W + (int64_t)i * w;   // row i of every coefficient: stride ww between time rows
        HIP_TRY(gjs_pivot_step(W, n, d, i, piv, aux, u, col, h->status, h->stream));
        // the pivot series' inverse with zero-padded Newton products (no wrap-around)
        CHECK(inverse_impl(h, u, 0, 1, n, MRINV_FP64_PADDED, v, wsi, wsib));
        // row_i <- v * row_i  (1x1 times 1x2d series products, truncated to n)
        HIP_TRY(fwd<double>(h, p, 1, SV, src_real(v, true, 1, 1, 0, n)));
        HIP_TRY(fwd<double>(h, p, nl_of(w), SR, src_real(row, true, ww, (int)w, 0, n)));
        HIP_TRY(freq_gemm<double>(p, gdesc(h, 1, 1, (int)w), SV, SR, SP, h->stream));
        HIP_TRY(inv<double>(h, p, nl_of(w), SP, dst_real(row, true, ww, (int)w, 0, n, invL, OP_STORE)));
        // W <- W - col * row_i  (d x 1 times 1 x 2d; col_i = 0 leaves row i alone)
        HIP_TRY(fwd<double>(h, p, nl_of(d), SC, src_real(col, true, d, d, 0, n)));
        HIP_TRY(fwd<double>(h, p, nl_of(w), SR, src_real(row, true, ww, (int)w, 0, n)));
        HIP_TRY(freq_gemm<double>(p, gdesc(h, d, 1, (int)w), SC, SR, SU, h->stream));
        HIP_TRY(inv<double>(h, p, nl_of(ww), SU, dst_real(W, true, ww, (int)ww, 0, n, -invL, OP_ADD)));
    }
    HIP_TRY(gjs_result(W, n, d, out, h->status, h->stream));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_series_inverse_gj(mrinv_handle_t h, const double *A, int d, int64_t n, double *Ainv,
                                                  void *ws, size_t ws_bytes) {
    TimerScope _ts(h);
    return gj_series_impl(h, A, 0, d, n, Ainv, ws, ws_bytes);
}

extern "C" mrinv_status_t mrinv_psi_inverse_gj(mrinv_handle_t h, const double *q, int d, int64_t n, double *psi,
                                               void *ws, size_t ws_bytes) {
    TimerScope _ts(h);
    return gj_series_impl(h, q, 1, d, n, psi, ws, ws_bytes);
}

// ---------------------------------------------------------------------------
// Tuning and autotuning
// ---------------------------------------------------------------------------
static mrinv_status_t check_tuning(const mrinv_tuning_t &t) {
    if (t.lgp_max < 5 || t.lgp_max > LGP_MAX) return fail(MRINV_E_ARG, "lgp_max %d not in 5..%d", t.lgp_max, LGP_MAX);
    if (t.lanes_fp64 != 0 && t.lanes_fp64 != 8 && t.lanes_fp64 != 16 && t.lanes_fp64 != 32)
        return fail(MRINV_E_ARG, "lanes_fp64 must be 0 (automatic), 8, 16 or 32");
    if (t.lanes_fp32 != 0 && t.lanes_fp32 != 8 && t.lanes_fp32 != 16 && t.lanes_fp32 != 32)
        return fail(MRINV_E_ARG, "lanes_fp32 must be 0 (automatic), 8, 16 or 32");
    if (t.seed_m0 < 1 || t.seed_m0 > 256) return fail(MRINV_E_ARG, "seed_m0 %d not in 1..256", t.seed_m0);
    if (t.twiddle_tables < 0 || t.twiddle_tables > 2) return fail(MRINV_E_ARG, "twiddle_tables must be 0, 1 or 2");
    if (t.block_order < 0 || t.block_order > 1) return fail(MRINV_E_ARG, "block_order must be 0 or 1");
    if (t.use_graph < 0 || t.use_graph > 1) return fail(MRINV_E_ARG, "use_graph must be 0 or 1");
    if (t.mfma < 0 || t.mfma > 2) return fail(MRINV_E_ARG, "mfma must be 0, 1 or 2");
    if (t.direct_m < -1 || t.direct_m > 65536) return fail(MRINV_E_ARG, "direct_m %d not in -1..65536", t.direct_m);
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_get_tuning(mrinv_handle_t h, mrinv_tuning_t *out) {
    if (!h || !out) return fail(MRINV_E_ARG, "NULL handle or pointer");
    *out = h->tune;
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_set_tuning(mrinv_handle_t h, const mrinv_tuning_t *t) {
    if (!h || !t) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_tuning(*t));
    h->tune = *t;
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_set_tuning_table(mrinv_handle_t h, const mrinv_tuning_entry_t *entries, int count) {
    if (!h || count < 0 || (count > 0 && !entries)) return fail(MRINV_E_ARG, "NULL handle or entries");
    for (int i = 0; i < count; ++i) {
        const auto &e = entries[i];
        if (e.d_lo < 1 || e.d_hi < e.d_lo || e.n_lo < 1 || e.n_hi < e.n_lo || e.precision < -1 ||
            e.precision > (int)MRINV_FP64_PADDED)
            return fail(MRINV_E_ARG, "table entry %d has bad ranges", i);
        CHECK(check_tuning(e.tune));
    }
    h->table.assign(entries, entries + count);
    return MRINV_OK;
}

// Milliseconds per inversion under the handle's current tuning.
static mrinv_status_t time_inverse(mrinv_handle_t h, const double *q, int d, int64_t n, mrinv_precision_t prec,
                                   double *psi, void *ws, size_t wsb, int reps, float *ms) {
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    mrinv_status_t st = mrinv_psi_inverse(h, q, d, n, prec, psi, ws, wsb);
    if (st == MRINV_OK) (void)hipEventRecord(a, h->stream);
    for (int r = 0; r < reps && st == MRINV_OK; ++r) st = mrinv_psi_inverse(h, q, d, n, prec, psi, ws, wsb);
    if (st == MRINV_OK) {
        (void)hipEventRecord(b, h->stream);
        (void)hipEventSynchronize(b);
        float t = 0.f;
        (void)hipEventElapsedTime(&t, a, b);
        *ms = t / reps;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

extern "C" mrinv_status_t mrinv_autotune(mrinv_handle_t h, const double *q, int d, int64_t n,
                                         mrinv_precision_t precision, double *psi, void *ws, size_t wsb,
                                         mrinv_tuning_t *chosen) {
    if (!h || !q || !psi) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    CHECK(check_ws(ws, wsb, ws_psi(d, n, precision)));
    // The table (if any) steps aside while candidates are timed.
    struct TableAside {
        mrinv_handle_t h;
        std::vector<mrinv_tuning_entry_t> saved;
        explicit TableAside(mrinv_handle_t hh) : h(hh) { saved.swap(hh->table); }
        ~TableAside() { h->table.swap(saved); }
    } aside(h);
    // Coordinate search from the current tuning: one knob at a time.
    mrinv_tuning_t best = h->tune;
    float best_ms = 0.f;
    h->tune = best;
    CHECK(time_inverse(h, q, d, n, precision, psi, ws, wsb, 3, &best_ms));
    auto trial = [&](mrinv_tuning_t t) -> mrinv_status_t {
        if (check_tuning(t) != MRINV_OK) return MRINV_OK;
        h->tune = t;
        float ms = 0.f;
        mrinv_status_t st = time_inverse(h, q, d, n, precision, psi, ws, wsb, 3, &ms);
        if (st != MRINV_OK) {
            h->tune = best;   // a failed trial leaves the best tuning so far in the handle
            // a candidate this problem cannot run (e.g. a seed too long for LDS) is skipped
            return st == MRINV_E_UNSUPPORTED ? MRINV_OK : st;
        }
        if (ms < best_ms) { best_ms = ms; best = t; }
        return MRINV_OK;
    };
    for (int v : {7, 8, 9}) { mrinv_tuning_t t = best; t.lgp_max = v; CHECK(trial(t)); }
    for (int v : {0, 8, 16, 32}) { mrinv_tuning_t t = best; t.lanes_fp64 = v; CHECK(trial(t)); }
    if (prec_mixed(precision))
        for (int v : {0, 8, 16, 32}) { mrinv_tuning_t t = best; t.lanes_fp32 = v; CHECK(trial(t)); }
    for (int v : {1, 16, 32, 64}) { mrinv_tuning_t t = best; t.seed_m0 = v; CHECK(trial(t)); }
    for (int v : {0, 1}) { mrinv_tuning_t t = best; t.pair_forward = v; CHECK(trial(t)); }
    for (int v : {0, 1, 2}) { mrinv_tuning_t t = best; t.twiddle_tables = v; CHECK(trial(t)); }
    for (int v : {0, 1}) { mrinv_tuning_t t = best; t.block_order = v; CHECK(trial(t)); }
    for (int v : {0, 1}) { mrinv_tuning_t t = best; t.use_graph = v; CHECK(trial(t)); }
    for (int v : {0, 1, 2}) { mrinv_tuning_t t = best; t.mfma = v; CHECK(trial(t)); }
    for (int v : {0, -1, 64, 128, 256, 512, 1024}) { mrinv_tuning_t t = best; t.direct_m = v; CHECK(trial(t)); }
    h->tune = best;
    CHECK(mrinv_psi_inverse(h, q, d, n, precision, psi, ws, wsb));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (chosen) *chosen = best;
    return MRINV_OK;
}

// ---------------------------------------------------------------------------
// Products with psi
// ---------------------------------------------------------------------------
extern "C" mrinv_status_t mrinv_markov_renewal_apply(mrinv_handle_t h, const double *psi, int d, int64_t n,
                                                     const double *L, int r, double *M, void *ws, size_t wsb) {
    TimerScope _ts(h);
    if (!h || !psi || !L || !M) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    if (r < 1 || r > MRINV_MAX_D) return fail(r < 1 ? MRINV_E_ARG : MRINV_E_UNSUPPORTED, "bad r=%d", r);
    CHECK(check_ws(ws, wsb, ws_apply(d, n, r)));
    const FftPlan p = hplan(h, lg_full(n));
    const int64_t d2 = (int64_t)d * d, dr = (int64_t)d * r;
    Carve cv(ws);
    auto *SP = cv.take<cplx<double>>(spec_bytes(p.lgL, d2, true));
    auto *SL = cv.take<cplx<double>>(spec_bytes(p.lgL, dr, true));
    auto *SM = cv.take<cplx<double>>(spec_bytes(p.lgL, dr, true));
    HIP_TRY(fwd<double>(h, p, nl_of(d2), SP, src_real(psi, true, d2, (int)d2, 0, n)));
    HIP_TRY(fwd<double>(h, p, nl_of(dr), SL, src_real(L, true, dr, (int)dr, 0, n)));
    HIP_TRY(freq_gemm<double>(p, gdesc(h, d, d, r), SP, SL, SM, h->stream));
    const double invL = 1.0 / (double)((int64_t)1 << p.lgL);
    HIP_TRY(inv<double>(h, p, nl_of(dr), SM, dst_real(M, true, dr, (int)dr, 0, n, invL, OP_STORE, -1, h->status)));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_survival(mrinv_handle_t h, const double *q, int d, int64_t n, double *hb) {
    TimerScope _ts(h);
    if (!h || !q || !hb) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    HIP_TRY(survival(q, d, n, hb, h->scratch + SCRATCH_SCAN_OFF, h->stream));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_transition(mrinv_handle_t h, const double *psi, const double *q, int d, int64_t n,
                                           double *P, void *ws, size_t wsb) {
    TimerScope _ts(h);
    if (!h || !psi || !q || !P) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    CHECK(check_ws(ws, wsb, ws_transition(d, n)));
    const FftPlan p = hplan(h, lg_full(n));
    const int64_t d2 = (int64_t)d * d;
    Carve cv(ws);
    double *hb = cv.take<double>((size_t)n * d * sizeof(double));
    auto *SP = cv.take<cplx<double>>(spec_bytes(p.lgL, d2, true));
    auto *SH = cv.take<cplx<double>>(spec_bytes(p.lgL, d, true));
    HIP_TRY(survival(q, d, n, hb, h->scratch + SCRATCH_SCAN_OFF, h->stream));
    HIP_TRY(fwd<double>(h, p, nl_of(d2), SP, src_real(psi, true, d2, (int)d2, 0, n)));
    HIP_TRY(fwd<double>(h, p, nl_of(d), SH, src_real(hb, true, d, d, 0, n)));
    HIP_TRY(freq_diag<double>(p, d, d, SP, SH, SP, h->stream));
    const double invL = 1.0 / (double)((int64_t)1 << p.lgL);
    HIP_TRY(inv<double>(h, p, nl_of(d2), SP, dst_real(P, true, d2, (int)d2, 0, n, invL, OP_STORE, -1, h->status)));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_contract(mrinv_handle_t h, const double *X, int64_t n, int rows, int cols,
                                         const double *u, const double *v, int cumulative, double offset,
                                         double scale, double *out) {
    TimerScope _ts(h);
    if (!h || !X || !u || !v || !out) return fail(MRINV_E_ARG, "NULL handle or pointer");
    if (n < 1 || rows < 1 || cols < 1 || n > MRINV_MAX_N) return fail(MRINV_E_ARG, "bad sizes");
    HIP_TRY(contract(X, n, rows, cols, u, v, cumulative, offset, scale, out, h->scratch + SCRATCH_SCAN_OFF,
                     h->stream));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_contract_backward(mrinv_handle_t h, const double *out_bar, int64_t n, int rows,
                                                  int cols, const double *u, const double *v, int cumulative,
                                                  double scale, double *X_bar_accum) {
    TimerScope _ts(h);
    if (!h || !out_bar || !u || !v || !X_bar_accum) return fail(MRINV_E_ARG, "NULL handle or pointer");
    if (n < 1 || rows < 1 || cols < 1 || n > MRINV_MAX_N) return fail(MRINV_E_ARG, "bad sizes");
    const double *w = out_bar;
    if (cumulative) {
        HIP_TRY(hipMemcpyAsync(h->scratch, out_bar, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
        w = h->scratch;
    }
    HIP_TRY(contract_backward(w, n, rows, cols, u, v, cumulative, scale, X_bar_accum, h->scratch + SCRATCH_SCAN_OFF,
                              h->stream));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_gather_block(mrinv_handle_t h, const double *X, int64_t n, int rows, int cols,
                                             const int *row_idx, int nr, const int *col_idx, int nc, double *Y) {
    TimerScope _ts(h);
    if (!h || !X || !row_idx || !col_idx || !Y) return fail(MRINV_E_ARG, "NULL handle or pointer");
    if (n < 1 || nr < 1 || nc < 1 || rows < 1 || cols < 1) return fail(MRINV_E_ARG, "bad sizes");
    HIP_TRY(gather_block(X, n, rows, cols, row_idx, nr, col_idx, nc, Y, h->stream));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_scatter_block_add(mrinv_handle_t h, const double *Y_bar, int64_t n, int rows,
                                                  int cols, const int *row_idx, int nr, const int *col_idx, int nc,
                                                  double *X_bar_accum) {
    TimerScope _ts(h);
    if (!h || !Y_bar || !row_idx || !col_idx || !X_bar_accum) return fail(MRINV_E_ARG, "NULL handle or pointer");
    if (n < 1 || nr < 1 || nc < 1 || rows < 1 || cols < 1) return fail(MRINV_E_ARG, "bad sizes");
    HIP_TRY(scatter_block_add(Y_bar, n, rows, cols, row_idx, nr, col_idx, nc, X_bar_accum, h->stream));
    return MRINV_OK;
}

// Device copies of small host vectors, placed in the handle scratch after the
// first MRINV_MAX_N doubles (which the 1-lane scans use).  They travel as
// kernel arguments (put_small_vectors), so no host buffer has to outlive the
// call and nothing waits for the stream.
struct SmallVecs {
    int *ci, *di;
    double *alpha, *ones;
};

static mrinv_status_t put_small(mrinv_handle_t h, const int *ci, int nci, const int *di, int ndi, const double *alpha,
                                int nalpha, const double *ones, int nones, SmallVecs &sv) {
    char *base = (char *)(h->scratch + MRINV_MAX_N);
    sv.ci = (int *)base;
    sv.di = (int *)(base + 1024);
    sv.alpha = (double *)(base + 2048);
    sv.ones = (double *)(base + 2048 + 1024);
    if (nci > SMALL_MAX || ndi > SMALL_MAX || nalpha > SMALL_MAX || nones > SMALL_MAX)
        return fail(MRINV_E_UNSUPPORTED, "small vector longer than %d", SMALL_MAX);
    SmallVecArgs v{};
    v.nci = nci;
    v.ndi = ndi;
    v.nalpha = nalpha;
    v.nones = nones;
    for (int i = 0; i < nci; ++i) v.ci[i] = ci[i];
    for (int i = 0; i < ndi; ++i) v.di[i] = di[i];
    for (int i = 0; i < nalpha; ++i) v.alpha[i] = alpha[i];
    for (int i = 0; i < nones; ++i) v.ones[i] = ones ? ones[i] : 1.0;
    HIP_TRY(put_small_vectors(v, sv.ci, sv.di, sv.alpha, sv.ones, h->stream));
    return MRINV_OK;
}

static mrinv_status_t first_entrance_impl(mrinv_handle_t h, const double *q, int d, int64_t n, const int *in_D,
                                          const double *alpha, mrinv_precision_t prec, double *g, double *F,
                                          double offset, double scale, void *ws, size_t wsb) {
    if (!h || !q || !in_D || !alpha || !F) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    int ci[SMALL_MAX], di[SMALL_MAX];
    int nC = 0, nD = 0;
    for (int i = 0; i < d; ++i) {
        if (in_D[i]) di[nD++] = i;
        else ci[nC++] = i;
    }
    if (nD == 0) return fail(MRINV_E_ARG, "target set D is empty");
    CHECK(check_ws(ws, wsb, ws_first_entrance(d, n, nD, prec)));
    if (nC == 0) {
        // Already in D at time 0.
        HIP_TRY(fill_f64(F, n, offset + scale, h->stream));
        if (g) {
            HIP_TRY(fill_f64(g, n, 0.0, h->stream));
            HIP_TRY(fill_f64(g, 1, 1.0, h->stream));
        }
        return MRINV_OK;
    }
    double aC[SMALL_MAX];
    for (int a = 0; a < nC; ++a) aC[a] = alpha[ci[a]];
    SmallVecs sv;
    CHECK(put_small(h, ci, nC, di, nD, aC, nC, nullptr, std::max(nD, nC), sv));
    Carve cv(ws);
    double *qCC = cv.take<double>((size_t)n * nC * nC * 8);
    double *qCD = cv.take<double>((size_t)n * nC * nD * 8);
    double *gD = cv.take<double>((size_t)n * nC * nD * 8);
    void *rest = cv.p + cv.used;
    const size_t rest_b = wsb - cv.used;
    HIP_TRY(gather_block(q, n, d, d, sv.ci, nC, sv.ci, nC, qCC, h->stream));
    HIP_TRY(gather_block(q, n, d, d, sv.ci, nC, sv.di, nD, qCD, h->stream));
    // psi_C is written into the gD slot's neighbour: reuse qCC's storage after
    // inversion is not possible (input), so place psi_C in the workspace tail.
    double *psiC = (double *)rest;
    const size_t psib = align256((size_t)n * nC * nC * 8);
    void *ws2 = (char *)rest + psib;
    const size_t need_inv = ws_psi(nC, n, prec), need_app = ws_apply(nC, n, nD);
    if (rest_b < psib + std::max(need_inv, need_app)) return fail(MRINV_E_WORKSPACE, "workspace too small");
    CHECK(mrinv_psi_inverse(h, qCC, nC, n, prec, psiC, ws2, rest_b - psib));
    CHECK(mrinv_markov_renewal_apply(h, psiC, nC, n, qCD, nD, gD, ws2, rest_b - psib));
    if (g)
        HIP_TRY(contract(gD, n, nC, nD, sv.alpha, sv.ones, 0, 0.0, 1.0, g, h->scratch + SCRATCH_SCAN_OFF, h->stream));
    HIP_TRY(contract(gD, n, nC, nD, sv.alpha, sv.ones, 1, offset, scale, F, h->scratch + SCRATCH_SCAN_OFF, h->stream));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_first_entrance(mrinv_handle_t h, const double *q, int d, int64_t n,
                                               const int *in_D, const double *alpha, mrinv_precision_t precision,
                                               double *g, double *F, void *ws, size_t wsb) {
    TimerScope _ts(h);
    return first_entrance_impl(h, q, d, n, in_D, alpha, precision, g, F, 0.0, 1.0, ws, wsb);
}

extern "C" mrinv_status_t mrinv_reliability(mrinv_handle_t h, const double *q, int d, int64_t n, const int *up,
                                            const double *alpha, mrinv_precision_t precision, double *R, void *ws,
                                            size_t wsb) {
    TimerScope _ts(h);
    if (!up) return fail(MRINV_E_ARG, "NULL up mask");
    if (d < 1 || d > MRINV_MAX_D) return check_dn(d, n);
    int down[MRINV_MAX_D];
    for (int i = 0; i < d; ++i) down[i] = up[i] ? 0 : 1;
    return first_entrance_impl(h, q, d, n, down, alpha, precision, nullptr, R, 1.0, -1.0, ws, wsb);
}

extern "C" mrinv_status_t mrinv_availability(mrinv_handle_t h, const double *P, int d, int64_t n, const int *up,
                                             const double *alpha, double *A) {
    TimerScope _ts(h);
    if (!h || !P || !up || !alpha || !A) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    double ind[MRINV_MAX_D];
    for (int i = 0; i < d; ++i) ind[i] = up[i] ? 1.0 : 0.0;
    SmallVecs sv;
    CHECK(put_small(h, nullptr, 0, nullptr, 0, alpha, d, ind, d, sv));
    HIP_TRY(contract(P, n, d, d, sv.alpha, sv.ones, 0, 0.0, 1.0, A, h->scratch + SCRATCH_SCAN_OFF, h->stream));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_renewal_visits(mrinv_handle_t h, const double *psi, int d, int64_t n,
                                               const int *in_B, const double *alpha, double *N) {
    TimerScope _ts(h);
    if (!h || !psi || !in_B || !alpha || !N) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    double ind[MRINV_MAX_D];
    for (int i = 0; i < d; ++i) ind[i] = in_B[i] ? 1.0 : 0.0;
    SmallVecs sv;
    CHECK(put_small(h, nullptr, 0, nullptr, 0, alpha, d, ind, d, sv));
    HIP_TRY(contract(psi, n, d, d, sv.alpha, sv.ones, 1, 0.0, 1.0, N, h->scratch + SCRATCH_SCAN_OFF, h->stream));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_mre_solve(mrinv_handle_t h, const double *Qs, int d, int64_t n, const double *L,
                                          int r, mrinv_precision_t precision, double *K, void *ws, size_t wsb) {
    TimerScope _ts(h);
    if (!h || !Qs || !L || !K) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    if (r < 1 || r > MRINV_MAX_D) return fail(r < 1 ? MRINV_E_ARG : MRINV_E_UNSUPPORTED, "bad r=%d", r);
    if (!prec_valid(precision)) return fail(MRINV_E_ARG, "unknown precision %d", (int)precision);
    CHECK(check_ws(ws, wsb, ws_mre(d, n, r, precision)));
    CHECK(check_seed(seed_len(h, n), d));
    Carve cv(ws);
    double *Qbar = cv.take<double>((size_t)n * d * d * 8);
    double *X = cv.take<double>((size_t)n * d * d * 8);
    double *R = cv.take<double>((size_t)n * d * r * 8);
    void *rest = cv.p + cv.used;
    const size_t rest_b = wsb - cv.used;
    HIP_TRY(mre_prepare(Qs, L, n, d, r, Qbar, R, h->stream));
    // (e0 - Qbar_h)^-1: Qbar_h(0) = Delta Q_h(1)/2, so A(0) = I - Qbar_h(0) takes the Gauss-Jordan path.
    {
        TuneScope _tn(h, d, n, (int)precision);
        CHECK(inverse_impl(h, Qbar, 1, d, n, precision, X, rest, rest_b));
    }
    return mrinv_markov_renewal_apply(h, X, d, n, R, r, K, rest, rest_b);
}

extern "C" size_t mrinv_mc_workspace_size(int64_t n) {
    if (n < 1 || n > MRINV_MAX_N) return 0;
    return 2 * align256((size_t)(n + 1) * sizeof(int));
}

extern "C" mrinv_status_t mrinv_semi_markov_mc(mrinv_handle_t h, const mrinv_mc_model_t *model, double step,
                                               int64_t n, int64_t trajectories, uint64_t seed, double *A, double *R,
                                               double *tau_D, int *jumps, void *ws, size_t wsb) {
    TimerScope _ts(h);
    if (!h || !model || !A || !R) return fail(MRINV_E_ARG, "NULL handle or pointer");
    if (!model->P || !model->p1 || !model->p2 || !model->up) return fail(MRINV_E_ARG, "NULL model array");
    const int d = model->d;
    if (d < 1 || d > MRINV_MC_MAX_D) return fail(MRINV_E_UNSUPPORTED, "Monte Carlo needs 1 <= d <= %d", MRINV_MC_MAX_D);
    if (n < 1 || n > MRINV_MAX_N) return fail(MRINV_E_ARG, "bad n=%lld", (long long)n);
    if (trajectories < 1 || trajectories > ((int64_t)1 << 31) - 1)
        return fail(MRINV_E_ARG, "trajectories must be in 1..2^31-1 (counts are int32)");
    if (!(step > 0.0) || !isfinite(step)) return fail(MRINV_E_ARG, "step must be positive");
    if (model->family < MRINV_SOJOURN_LOGNORMAL || model->family > MRINV_SOJOURN_EXPONENTIAL)
        return fail(MRINV_E_ARG, "unknown sojourn family %d", model->family);
    if (model->initial < 0 || model->initial >= d) return fail(MRINV_E_ARG, "initial state out of range");
    McModel m{};
    m.d = d;
    m.family = model->family;
    m.initial = model->initial;
    for (int i = 0; i < d; ++i) {
        double acc = 0.0;
        m.up[i] = model->up[i] ? 1 : 0;
        m.last[i] = -1;
        for (int j = 0; j < d; ++j) {
            const double pij = model->P[i * d + j];
            if (!(pij >= 0.0) || !isfinite(pij)) return fail(MRINV_E_ARG, "P[%d][%d] is not a probability", i, j);
            acc += pij;
            m.cum[i * MC_MAX_D + j] = acc;
            m.p1[i * MC_MAX_D + j] = model->p1[i * d + j];
            m.p2[i * MC_MAX_D + j] = model->p2[i * d + j];
            if (pij > 0.0) {
                m.last[i] = j;
                const double a = model->p1[i * d + j], b = model->p2[i * d + j];
                const bool ok = model->family == MRINV_SOJOURN_LOGNORMAL ? (isfinite(a) && b > 0.0 && isfinite(b))
                                : model->family == MRINV_SOJOURN_WEIBULL ? (a > 0.0 && b > 0.0 && isfinite(a) && isfinite(b))
                                                                         : (a > 0.0 && isfinite(a));
                if (!ok) return fail(MRINV_E_ARG, "bad sojourn parameters for %d -> %d", i, j);
            }
        }
        if (fabs(acc - 1.0) > 1e-12) return fail(MRINV_E_ARG, "row %d of P sums to %.17g, not 1", i, acc);
    }
    CHECK(check_ws(ws, wsb, mrinv_mc_workspace_size(n)));
    int *diffA = (int *)ws;
    int *diffR = (int *)((char *)ws + align256((size_t)(n + 1) * sizeof(int)));
    HIP_TRY(semi_markov_mc(m, step, n, trajectories, seed, A, R, tau_D, jumps, diffA, diffR, h->stream));
    return MRINV_OK;
}

// ---------------------------------------------------------------------------
// Adjoints
// ---------------------------------------------------------------------------
extern "C" mrinv_status_t mrinv_psi_inverse_backward(mrinv_handle_t h, const double *psi, const double *psi_bar,
                                                     int d, int64_t n, double *q_bar, void *ws, size_t wsb) {
    TimerScope _ts(h);
    if (!h || !psi || !psi_bar || !q_bar) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    CHECK(check_ws(ws, wsb, ws_psi_backward(d, n)));
    const FftPlan p = hplan(h, lg_full(n));
    const int64_t d2 = (int64_t)d * d;
    const int nl = nl_of(d2);
    Carve cv(ws);
    const size_t sb = spec_bytes(p.lgL, d2, true);
    auto *S1 = cv.take<cplx<double>>(sb);
    auto *S2 = cv.take<cplx<double>>(sb);
    auto *S3 = cv.take<cplx<double>>(sb);
    const double invL = 1.0 / (double)((int64_t)1 << p.lgL);
    HIP_TRY(fwd<double>(h, p, nl, S1, src_real(psi, true, d2, (int)d2, 0, n)));
    HIP_TRY(fwd<double>(h, p, nl, S2, src_real(psi_bar, true, d2, (int)d2, 0, n, n - 1)));
    // V^r = Rev(psi_bar) * psi^T, kept on [0, n)
    HIP_TRY(freq_gemm<double>(p, gdesc(h, d, d, d, 0, 1), S2, S1, S3, h->stream));
    HIP_TRY(remask<double>(h, p, nl, S3, 0, n, false));
    // q_bar^r = psi^T * V^r
    HIP_TRY(freq_gemm<double>(p, gdesc(h, d, d, d, 1, 0), S1, S3, S2, h->stream));
    HIP_TRY(inv<double>(h, p, nl, S2, dst_real(q_bar, true, d2, (int)d2, 0, n, invL, OP_STORE, n - 1, h->status)));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_markov_renewal_apply_backward(mrinv_handle_t h, const double *psi, const double *L,
                                                              const double *M_bar, int d, int64_t n, int r,
                                                              double *psi_bar_accum, double *L_bar, void *ws,
                                                              size_t wsb) {
    TimerScope _ts(h);
    if (!h || !psi || !L || !M_bar) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    if (r < 1 || r > MRINV_MAX_D) return fail(r < 1 ? MRINV_E_ARG : MRINV_E_UNSUPPORTED, "bad r=%d", r);
    CHECK(check_ws(ws, wsb, ws_apply_backward(d, n, r)));
    const FftPlan p = hplan(h, lg_full(n));
    const int64_t d2 = (int64_t)d * d, dr = (int64_t)d * r;
    Carve cv(ws);
    auto *SP = cv.take<cplx<double>>(spec_bytes(p.lgL, d2, true));
    auto *SM = cv.take<cplx<double>>(spec_bytes(p.lgL, dr, true));
    auto *SL = cv.take<cplx<double>>(spec_bytes(p.lgL, dr, true));
    const double invL = 1.0 / (double)((int64_t)1 << p.lgL);
    HIP_TRY(fwd<double>(h, p, nl_of(dr), SM, src_real(M_bar, true, dr, (int)dr, 0, n, n - 1)));
    if (psi_bar_accum) {
        // psi_bar^r += Rev(M_bar) * L^T   (d x r times r x d)
        HIP_TRY(fwd<double>(h, p, nl_of(dr), SL, src_real(L, true, dr, (int)dr, 0, n)));
        HIP_TRY(freq_gemm<double>(p, gdesc(h, d, r, d, 0, 1), SM, SL, SP, h->stream));
        HIP_TRY(inv<double>(h, p, nl_of(d2), SP,
                            dst_real(psi_bar_accum, true, d2, (int)d2, 0, n, invL, OP_ADD, n - 1, h->status)));
    }
    if (L_bar) {
        // L_bar^r = psi^T * Rev(M_bar)
        HIP_TRY(fwd<double>(h, p, nl_of(d2), SP, src_real(psi, true, d2, (int)d2, 0, n)));
        HIP_TRY(freq_gemm<double>(p, gdesc(h, d, d, r, 1, 0), SP, SM, SL, h->stream));
        HIP_TRY(inv<double>(h, p, nl_of(dr), SL, dst_real(L_bar, true, dr, (int)dr, 0, n, invL, OP_STORE, n - 1, h->status)));
    }
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_transition_backward(mrinv_handle_t h, const double *psi, const double *q,
                                                    const double *P_bar, int d, int64_t n, double *psi_bar_accum,
                                                    double *q_bar_accum, void *ws, size_t wsb) {
    TimerScope _ts(h);
    if (!h || !psi || !q || !P_bar) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    CHECK(check_ws(ws, wsb, ws_transition_backward(d, n)));
    const FftPlan p = hplan(h, lg_full(n));
    const int64_t d2 = (int64_t)d * d;
    Carve cv(ws);
    double *hb = cv.take<double>((size_t)n * d * 8);
    double *hbb = cv.take<double>((size_t)n * d * 8);
    auto *S1 = cv.take<cplx<double>>(spec_bytes(p.lgL, d2, true));
    auto *S2 = cv.take<cplx<double>>(spec_bytes(p.lgL, d2, true));
    auto *SH = cv.take<cplx<double>>(spec_bytes(p.lgL, d, true));
    const double invL = 1.0 / (double)((int64_t)1 << p.lgL);
    HIP_TRY(fwd<double>(h, p, nl_of(d2), S1, src_real(P_bar, true, d2, (int)d2, 0, n, n - 1)));
    if (psi_bar_accum) {
        HIP_TRY(survival(q, d, n, hb, h->scratch + SCRATCH_SCAN_OFF, h->stream));
        HIP_TRY(fwd<double>(h, p, nl_of(d), SH, src_real(hb, true, d, d, 0, n)));
        HIP_TRY(freq_diag<double>(p, d, d, S1, SH, S2, h->stream));
        HIP_TRY(inv<double>(h, p, nl_of(d2), S2,
                            dst_real(psi_bar_accum, true, d2, (int)d2, 0, n, invL, OP_ADD, n - 1, h->status)));
    }
    if (q_bar_accum) {
        HIP_TRY(fwd<double>(h, p, nl_of(d2), S2, src_real(psi, true, d2, (int)d2, 0, n)));
        HIP_TRY(freq_coldot<double>(p, d, d, S2, S1, SH, h->stream));
        HIP_TRY(inv<double>(h, p, nl_of(d), SH, dst_real(hbb, true, d, d, 0, n, invL, OP_STORE, n - 1)));
        HIP_TRY(survival_backward(hbb, d, n, q_bar_accum, h->scratch + SCRATCH_SCAN_OFF, h->stream));
    }
    return MRINV_OK;
}

// ---------------------------------------------------------------------------
// Residual diagnostics
// ---------------------------------------------------------------------------
extern "C" mrinv_status_t mrinv_residual_norms(mrinv_handle_t h, const double *q, const double *X, int d, int64_t n,
                                               double *out, void *ws, size_t wsb) {
    TimerScope _ts(h);
    if (!h || !q || !X || !out) return fail(MRINV_E_ARG, "NULL handle or pointer");
    CHECK(check_dn(d, n));
    const FftPlan p = hplan(h, lg_full(n));
    const int64_t d2 = (int64_t)d * d;
    const int nl = nl_of(d2);
    CHECK(check_ws(ws, wsb, ws_residual(d, n)));
    Carve cv(ws);
    const size_t sb = spec_bytes(p.lgL, d2, true);
    auto *SA = cv.take<cplx<double>>(sb);
    auto *SX = cv.take<cplx<double>>(sb);
    auto *ST = cv.take<cplx<double>>(sb);
    double *RL = cv.take<double>((size_t)n * d2 * 8);
    double *RR = cv.take<double>((size_t)n * d2 * 8);
    const double invL = 1.0 / (double)((int64_t)1 << p.lgL);
    const GemmDesc g = gdesc(h, d, d, d);
    HIP_TRY(fwd<double>(h, p, nl, SA, src_real(q, true, d2, (int)d2, 0, n, -1, d)));
    HIP_TRY(fwd<double>(h, p, nl, SX, src_real(X, true, d2, (int)d2, 0, n)));
    DstDesc dl = dst_real(RL, true, d2, (int)d2, 0, n, invL, OP_E0MINUS);
    dl.e0_d = d;
    HIP_TRY(freq_gemm<double>(p, g, SA, SX, ST, h->stream));
    HIP_TRY(inv<double>(h, p, nl, ST, dl));
    DstDesc dr = dl;
    dr.p = RR;
    HIP_TRY(freq_gemm<double>(p, g, SX, SA, ST, h->stream));
    HIP_TRY(inv<double>(h, p, nl, ST, dr));
    double *acc = h->scratch;
    HIP_TRY(fill_f64(acc, 3, 0.0, h->stream));
    HIP_TRY(residual_norms(RL, RR, d, n, acc, h->stream));
    HIP_TRY(hipMemcpyAsync(out, acc, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return MRINV_OK;
}

// ---------------------------------------------------------------------------
// Batched inversion.  All problems active at Newton step r share the length
// L = 2^(r+1) (the truncated last step of a problem has the same L), so each
// phase of a step is one launch over every active problem, grouped only by
// lanes per workgroup (FFT passes) or by padded dimension class (products).
// Descriptors of every launch are planned on the host, copied to the device
// in one transfer, then the launches are enqueued.  Problems are split into
// sub-batches so that the spectra of one phase fit under BATCH_SPEC_CAP.
// ---------------------------------------------------------------------------
// Handle fields for the planner, which also runs without a handle to size
// the workspace.
static unsigned int *status_of(mrinv_handle_t h) { return h ? h->status : nullptr; }

constexpr size_t BATCH_SPEC_CAP = (size_t)24 << 30;

struct BatchPlan {
    std::vector<unsigned char> table;        // host image of the device descriptor table
    std::vector<std::function<hipError_t(char *, hipStream_t)>> launches;   // device table base, stream
    size_t table_bytes = 0, x_off = 0, r_off = 0, spec_off = 0, spec_bytes = 0, total = 0;
    char *ws = nullptr;                                       // workspace the table was uploaded to
    template <typename D> size_t put(const std::vector<D> &v) {
        const size_t off = align256(table.size());
        table.resize(off + v.size() * sizeof(D));
        memcpy(table.data() + off, v.data(), v.size() * sizeof(D));
        return off;
    }
};

template <typename T>
static void plan_fft(BatchPlan &bp, mrinv_handle_t h, int mode, const FftPlan &p, int pass,
                     const std::vector<PassProblem<T>> &probs) {
    if (probs.empty()) return;
    const bool dbl = sizeof(T) == 8;
    // Group by lanes per workgroup, chosen per problem as for a single
    // transform: the handle's choice, else the automatic rule (32 lanes for
    // small-tile passes of wide rows, 8 for the fused 512-row float64 pass,
    // 16 otherwise); 2 for problems of at most 2 lanes.
    const int lgP = p.lgP[pass];
    auto lanes_for = [&](const PassProblem<T> &q) {
        if (q.nl <= 2) return 2;
        int C = lanes_of<T>(h) ? lanes_of<T>(h) : fft_lanes_per_block(dbl, q.nl, lgP, mode);
        if (C == 32 && (lgP > 8 || q.nl <= 16)) C = 16;
        return C;
    };
    for (int C : {2, 8, 16, 32}) {
        std::vector<PassProblem<T>> g;
        for (auto &q : probs)
            if (lanes_for(q) == C) g.push_back(q);
        if (g.empty()) continue;
        const int64_t total = fft_batch_layout<T>(p, pass, g.data(), (int)g.size(), C);
        double bytes = 0;
        for (auto &q : g) bytes += 2.0 * ((double)((int64_t)1 << p.lgL)) * q.nl * sizeof(cplx<T>);
        const size_t off = bp.put(g);
        const int cnt = (int)g.size();
        const Twiddles<T> tw = tw_of<T>(h);
        bp.launches.push_back([=](char *base, hipStream_t st) {
            return fft_pass_batched<T>(mode, p, pass, C, (const PassProblem<T> *)(base + off), cnt, total, bytes, tw, st);
        });
    }
}

template <typename T>
static void plan_gemm(BatchPlan &bp, mrinv_handle_t h, const FftPlan &p, const std::vector<GemmProblem<T>> &probs,
                      int bf3 = 0) {
    for (int cls = 1; cls <= 16; ++cls) {
        std::vector<GemmProblem<T>> g;
        for (auto &q : probs)
            if (gemm_sq_class(q.d, tune_of(h).mfma) == cls) g.push_back(q);
        if (g.empty()) continue;
        const int64_t total = gemm_batch_layout<T>(p, g.data(), (int)g.size(), tune_of(h).mfma);
        double bytes = 0, flops = 0;
        const double Lr = (double)((int64_t)1 << p.lgL);
        for (auto &q : g) {
            bytes += Lr * 3.0 * nl_of((int64_t)q.d * q.d) * sizeof(cplx<T>);
            flops += (Lr / 2 + 1) * 8.0 * q.d * q.d * q.d;
        }
        const size_t off = bp.put(g);
        const int cnt = (int)g.size();
        const int mf = tune_of(h).mfma;
        bp.launches.push_back([=](char *base, hipStream_t st) {
            return freq_gemm_batched<T>(p, cls, mf, bf3, (const GemmProblem<T> *)(base + off), cnt, total, bytes, flops,
                                        st);
        });
    }
}

// Forward transform of a real source per problem into its spectrum.  aux32
// (optional, float64 only): per problem, where the last pass also writes a
// float32 copy of the spectrum.
template <typename T>
static void plan_fwd(BatchPlan &bp, mrinv_handle_t h, const FftPlan &p, const std::vector<cplx<T> *> &Z,
                     const std::vector<int> &nl, const std::vector<SrcDesc> &src,
                     const std::vector<const void *> *aux32 = nullptr) {
    std::vector<PassProblem<T>> v(Z.size());
    auto dsts = [&](int j) {
        for (size_t i = 0; i < Z.size(); ++i) v[i].dst = fwd_dst(p, j, aux32 ? (*aux32)[i] : nullptr);
    };
    for (size_t i = 0; i < Z.size(); ++i) {
        v[i] = PassProblem<T>{};
        v[i].z = Z[i];
        v[i].nl = nl[i];
        v[i].src = src[i];
    }
    dsts(0);
    plan_fft<T>(bp, h, 0, p, 0, v);
    for (auto &x : v) x.src = src_z();
    for (int j = 1; j < p.npass; ++j) {
        dsts(j);
        plan_fft<T>(bp, h, 0, p, j, v);
    }
}

template <typename T>
static void plan_inv(BatchPlan &bp, mrinv_handle_t h, const FftPlan &p, const std::vector<cplx<T> *> &Z,
                     const std::vector<int> &nl, const std::vector<DstDesc> &dst) {
    std::vector<PassProblem<T>> v(Z.size());
    for (size_t i = 0; i < Z.size(); ++i) {
        v[i] = PassProblem<T>{};
        v[i].z = Z[i];
        v[i].nl = nl[i];
        v[i].src = src_z();
        v[i].dst = dst_z();
    }
    for (int j = p.npass - 1; j >= 1; --j) plan_fft<T>(bp, h, 1, p, j, v);
    for (size_t i = 0; i < Z.size(); ++i) v[i].dst = dst[i];
    plan_fft<T>(bp, h, 1, p, 0, v);
}

template <typename T>
static void plan_remask(BatchPlan &bp, mrinv_handle_t h, const FftPlan &p, const std::vector<cplx<T> *> &Z,
                        const std::vector<int> &nl, const std::vector<int64_t> &lo, const std::vector<int64_t> &hi,
                        bool neg) {
    std::vector<PassProblem<T>> v(Z.size());
    for (size_t i = 0; i < Z.size(); ++i) {
        v[i] = PassProblem<T>{};
        v[i].z = Z[i];
        v[i].nl = nl[i];
        v[i].src = src_z();
        v[i].dst = dst_z();
    }
    for (int j = p.npass - 1; j >= 1; --j) plan_fft<T>(bp, h, 1, p, j, v);
    for (size_t i = 0; i < Z.size(); ++i) {
        v[i].dst.lo = lo[i];
        v[i].dst.hi = hi[i];
        v[i].dst.op = neg ? OP_NEG : OP_STORE;
        v[i].dst.scale = 1.0 / (double)((int64_t)1 << p.lgL);
    }
    plan_fft<T>(bp, h, 2, p, 0, v);
    for (auto &x : v) x.dst = dst_z();
    for (int j = 1; j < p.npass; ++j) plan_fft<T>(bp, h, 0, p, j, v);
}

struct BatchProblem {
    const double *q;
    double *psi;
    int d;
    int64_t n;
    float *X, *R;   // mixed form
    int64_t seed;   // recursion seed length and direct-step limit of this problem's tuning
    int64_t dlim;
};

// Sub-batches of `idx` whose summed need stays under the cap (at least one each).
static std::vector<std::vector<int>> split_by_cap(const std::vector<int> &idx, const std::vector<size_t> &need) {
    std::vector<std::vector<int>> out;
    std::vector<int> cur;
    size_t acc = 0;
    for (size_t k = 0; k < idx.size(); ++k) {
        if (!cur.empty() && acc + need[k] > BATCH_SPEC_CAP) {
            out.push_back(cur);
            cur.clear();
            acc = 0;
        }
        cur.push_back(idx[k]);
        acc += need[k];
    }
    if (!cur.empty()) out.push_back(cur);
    return out;
}

template <typename T>
static void plan_newton(BatchPlan &bp, mrinv_handle_t h, std::vector<BatchProblem> &P, char *spec, size_t &spec_max,
                        int pad, int bf3) {
    const bool dbl = sizeof(T) == 8;
    const int64_t nmax = [&] { int64_t m = 0; for (auto &b : P) m = std::max(m, b.n); return m; }();
    // Seeds: the first m0 coefficients of each problem by the recursion.
    {
        std::vector<SeedProblem> sp;
        int cols = 0, dmax = 0, m0max = 0;
        for (auto &b : P) {
            const int64_t m0 = b.seed;
            if (m0 <= 1) continue;
            SeedProblem x{};
            x.A = b.q;
            x.out = dbl ? (void *)b.psi : (void *)b.X;
            x.d = b.d;
            x.m0 = (int)m0;
            x.e0 = 1;
            x.col_begin = cols;
            cols += b.d;
            dmax = std::max(dmax, b.d);
            m0max = std::max(m0max, (int)m0);
            sp.push_back(x);
        }
        if (!sp.empty()) {
            const size_t off = bp.put(sp);
            const int cnt = (int)sp.size();
            bp.launches.push_back([=](char *base, hipStream_t st) {
                return seed_recursion_batched<T>((const SeedProblem *)(base + off), cnt, cols, dmax, m0max, st);
            });
        }
    }
    for (int64_t m = 1; m < nmax; m *= 2) {
        const FftPlan p = hplan(h, ceil_log2(2 * m) + pad);
        const int64_t L = (int64_t)1 << p.lgL;
        // Direct steps of this m (as in the single-problem call), E scratch at
        // the start of the spectrum region; the transform steps below reuse it
        // after them in stream order.
        {
            std::vector<ConvDesc> ce[5], cu[5];
            size_t used = 0;
            for (int i = 0; i < (int)P.size(); ++i) {
                const BatchProblem &b = P[i];
                const int64_t m2 = std::min(2 * m, b.n);
                if (!(b.n > m && m >= b.seed && m2 <= b.dlim)) continue;
                const int64_t d2 = (int64_t)b.d * b.d;
                void *out = dbl ? (void *)b.psi : (void *)b.X;
                void *E = spec + used;
                used += align256((size_t)(m2 - m) * d2 * sizeof(T));
                ConvDesc c{};
                c.L = b.q; c.l_f64 = 1; c.R = out; c.out = E; c.d = b.d; c.sign = 1.0;
                c.k0 = m; c.k1 = m2; c.jlo = 0; c.jhi = m - 1; c.r_off = 0; c.out_off = m;
                ConvDesc u{};
                u.L = out; u.l_f64 = dbl; u.R = E; u.out = out; u.d = b.d; u.sign = 1.0;
                u.k0 = m; u.k1 = m2; u.jlo = m; u.jhi = m2; u.r_off = m; u.out_off = 0;
                u.status = dbl ? status_of(h) : nullptr;
                ce[conv_class(b.d)].push_back(c);
                cu[conv_class(b.d)].push_back(u);
            }
            spec_max = std::max(spec_max, used);
            for (int pass = 0; pass < 2; ++pass)
                for (int cls = 1; cls <= 4; ++cls) {
                    std::vector<ConvDesc> &v = pass == 0 ? ce[cls] : cu[cls];
                    if (v.empty()) continue;
                    const int64_t total = conv_batch_layout(v.data(), (int)v.size());
                    double flops = 0;
                    for (auto &x : v) flops += 1.5 * (double)(x.k1 - x.k0) * (double)(x.k1 - x.k0) * 2.0 * x.d * x.d * x.d;
                    const size_t off = bp.put(v);
                    const int cnt = (int)v.size();
                    const int lf = pass == 0 ? 1 : (dbl ? 1 : 0);
                    bp.launches.push_back([=](char *base, hipStream_t st) {
                        return conv_direct_batched<T>(cls, lf, (const ConvDesc *)(base + off), cnt, total, flops, st);
                    });
                }
        }
        std::vector<int> act;
        std::vector<size_t> need;
        for (int i = 0; i < (int)P.size(); ++i)
            if (P[i].n > m && m >= P[i].seed && std::min(2 * m, P[i].n) > P[i].dlim) {
                act.push_back(i);
                need.push_back(3 * spec_bytes(p.lgL, (int64_t)P[i].d * P[i].d, dbl));
            }
        for (auto &sub : split_by_cap(act, need)) {
            std::vector<cplx<T> *> SA, SB, ST;
            std::vector<int> nl;
            std::vector<SrcDesc> sa, sb;
            std::vector<DstDesc> du;
            std::vector<int64_t> lo, hi;
            std::vector<GemmProblem<T>> g1, g2;
            size_t used = 0;
            for (int i : sub) {
                const BatchProblem &b = P[i];
                const int64_t d2 = (int64_t)b.d * b.d;
                const size_t sbz = spec_bytes(p.lgL, d2, dbl);
                SA.push_back((cplx<T> *)(spec + used));
                SB.push_back((cplx<T> *)(spec + used + sbz));
                ST.push_back((cplx<T> *)(spec + used + 2 * sbz));
                used += 3 * sbz;
                nl.push_back(nl_of(d2));
                const int64_t m2 = std::min(2 * m, b.n);
                void *out = dbl ? (void *)b.psi : (void *)b.X;
                sa.push_back(src_real(b.q, true, d2, (int)d2, 0, m2, -1, b.d));
                sb.push_back(src_real(out, dbl, d2, (int)d2, 0, m));
                du.push_back(dst_real(out, dbl, d2, (int)d2, m, m2, 1.0 / (double)L, OP_STORE, -1,
                                      dbl ? status_of(h) : nullptr));
                lo.push_back(m);
                hi.push_back(m2);
                GemmProblem<T> x{};
                x.A = SA.back(); x.B = SB.back(); x.C = ST.back(); x.d = b.d;
                g1.push_back(x);
                GemmProblem<T> y{};
                y.A = SB.back(); y.B = ST.back(); y.C = SA.back(); y.d = b.d;
                g2.push_back(y);
            }
            spec_max = std::max(spec_max, used);
            plan_fwd<T>(bp, h, p, SA, nl, sa);
            plan_fwd<T>(bp, h, p, SB, nl, sb);
            plan_gemm<T>(bp, h, p, g1, bf3);
            plan_remask<T>(bp, h, p, ST, nl, lo, hi, true);
            plan_gemm<T>(bp, h, p, g2, bf3);
            plan_inv<T>(bp, h, p, SA, nl, du);
        }
    }
}

static void plan_sweeps(BatchPlan &bp, mrinv_handle_t h, std::vector<BatchProblem> &P, char *spec, size_t &spec_max,
                        int bf3) {
    // Group by the residual length 2^ceil(log2(2n-1)).
    std::vector<int> lgs;
    for (auto &b : P) lgs.push_back(lg_full(b.n));
    std::vector<int> uniq = lgs;
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    for (int lg : uniq) {
        const FftPlan p = hplan(h, lg);
        const double invL = 1.0 / (double)((int64_t)1 << lg);
        std::vector<int> grp;
        std::vector<size_t> need;
        for (int i = 0; i < (int)P.size(); ++i)
            if (lgs[i] == lg) {
                grp.push_back(i);
                need.push_back(sweep_bytes(lg, (int64_t)P[i].d * P[i].d));
            }
        for (auto &sub : split_by_cap(grp, need)) {
            for (int sweep = 0; sweep < MIXED_SWEEPS; ++sweep) {
                const bool last = sweep == MIXED_SWEEPS - 1;
                std::vector<cplx<double> *> A64, B64, T64;
                std::vector<cplx<float> *> X32, R32, T32;
                std::vector<const void *> X32c;
                std::vector<int> nl;
                std::vector<SrcDesc> sq, sx, sr;
                std::vector<DstDesc> dr, dx;
                std::vector<GemmProblem<double>> g64;
                std::vector<GemmProblem<float>> g32;
                size_t used = 0;
                for (int i : sub) {
                    const BatchProblem &b = P[i];
                    const int64_t d2 = (int64_t)b.d * b.d;
                    const size_t s64 = spec_bytes(lg, d2, true), s32 = spec_bytes(lg, d2, false);
                    // The slots of the single-problem call (sweep_bytes).
                    A64.push_back((cplx<double> *)(spec + used));
                    B64.push_back((cplx<double> *)(spec + used + s64));
                    T64.push_back((cplx<double> *)(spec + used + 2 * s64));
                    X32.push_back((cplx<float> *)(spec + used + 3 * s64));
                    X32c.push_back(X32.back());
                    R32.push_back((cplx<float> *)(spec + used + s64));
                    T32.push_back((cplx<float> *)(spec + used + s64 + s32));
                    used += sweep_bytes(lg, d2);
                    nl.push_back(nl_of(d2));
                    sq.push_back(src_real(b.q, true, d2, (int)d2, 0, b.n, -1, b.d));
                    sx.push_back(src_real(b.X, false, d2, (int)d2, 0, b.n));
                    sr.push_back(src_real(b.R, false, d2, (int)d2, 0, b.n));
                    DstDesc r = dst_real(b.R, false, d2, (int)d2, 0, b.n, invL, OP_E0MINUS);
                    r.e0_d = b.d;
                    dr.push_back(r);
                    DstDesc x = last ? dst_real(b.psi, true, d2, (int)d2, 0, b.n, invL, OP_XPLUS, -1, status_of(h))
                                     : dst_real(b.X, false, d2, (int)d2, 0, b.n, invL, OP_XPLUS);
                    x.aux = b.X;
                    dx.push_back(x);
                    GemmProblem<double> u{};
                    u.A = A64.back(); u.B = B64.back(); u.C = T64.back(); u.d = b.d;
                    g64.push_back(u);
                    GemmProblem<float> w{};
                    w.A = X32.back(); w.B = R32.back(); w.C = T32.back(); w.d = b.d;
                    g32.push_back(w);
                }
                spec_max = std::max(spec_max, used);
                if (sweep == 0) plan_fwd<double>(bp, h, p, A64, nl, sq);
                plan_fwd<double>(bp, h, p, B64, nl, sx, &X32c);
                plan_gemm<double>(bp, h, p, g64);
                plan_inv<double>(bp, h, p, T64, nl, dr);
                plan_fwd<float>(bp, h, p, R32, nl, sr);
                plan_gemm<float>(bp, h, p, g32, bf3);
                plan_inv<float>(bp, h, p, T32, nl, dx);
            }
        }
    }
}

// Builds the whole schedule for a workspace at `ws` (nullptr: sizing only).
static mrinv_status_t plan_batched(mrinv_handle_t h, int count, const double *const *q_ptrs, const int *d,
                                   const int64_t *n, mrinv_precision_t prec, double *const *psi_ptrs, char *ws,
                                   BatchPlan &bp) {
    if (count < 1 || !d || !n) return fail(MRINV_E_ARG, "bad batch");
    if (!prec_valid(prec)) return fail(MRINV_E_ARG, "unknown precision");
    std::vector<BatchProblem> P(count);
    int64_t m0max = 1;
    int dmax_all = 1;
    for (int b = 0; b < count; ++b) {
        CHECK(check_dn(d[b], n[b]));
        m0max = std::max(m0max, seed_len(tune_for(h, d[b], n[b], (int)prec), n[b]));
        dmax_all = std::max(dmax_all, d[b]);
    }
    CHECK(check_seed(m0max, dmax_all));
    for (int b = 0; b < count; ++b) {
        const mrinv_tuning_t &tb = tune_for(h, d[b], n[b], (int)prec);
        P[b].seed = seed_len(tb, n[b]);
        P[b].dlim = direct_limit(tb, d[b]);
        P[b].q = q_ptrs ? q_ptrs[b] : nullptr;
        P[b].psi = psi_ptrs ? psi_ptrs[b] : nullptr;
        P[b].d = d[b];
        P[b].n = n[b];
    }
    // Pass 1 sizes the table; pass 2 fills it with final addresses.
    const bool mixed = prec_mixed(prec);
    size_t xr = 0;
    if (mixed)
        for (auto &b : P) xr += align256((size_t)b.n * b.d * b.d * sizeof(float));
    for (int round = 0; round < 2; ++round) {
        const size_t table_guess = round == 0 ? 0 : bp.table_bytes;
        BatchPlan cur;
        char *base = ws ? ws : nullptr;
        const size_t x_off = align256(table_guess), r_off = x_off + xr, spec_off = r_off + xr;
        size_t xo = 0;
        for (auto &b : P) {
            if (mixed) {
                b.X = (float *)((base ? base : (char *)0) + x_off + xo);
                b.R = (float *)((base ? base : (char *)0) + r_off + xo);
                xo += align256((size_t)b.n * b.d * b.d * sizeof(float));
            }
        }
        char *spec = (base ? base : (char *)0) + spec_off;
        size_t spec_max = 0;
        // Seeds for every problem in one launch.
        std::vector<GjProblem> gj(count);
        int dmax = 0;
        for (int b = 0; b < count; ++b) {
            gj[b].A0 = P[b].q;
            gj[b].d = P[b].d;
            gj[b].e0_minus = 1;
            gj[b].out64 = mixed ? nullptr : P[b].psi;
            gj[b].out32 = mixed ? P[b].X : nullptr;
            dmax = std::max(dmax, P[b].d);
        }
        const size_t goff = cur.put(gj);
        {
            unsigned int *status = status_of(h);
            const int cnt = count;
            cur.launches.push_back([=](char *tb, hipStream_t st) {
                return gj_inverse_batched((const GjProblem *)(tb + goff), cnt, dmax, status, st);
            });
        }
        if (mixed) {
            plan_newton<float>(cur, h, P, spec, spec_max, 0, prec_bf3(prec));
            plan_sweeps(cur, h, P, spec, spec_max, prec_bf3(prec));
        } else {
            plan_newton<double>(cur, h, P, spec, spec_max, prec_pad(prec), 0);
        }
        cur.table_bytes = align256(cur.table.size());
        if (round == 0) {
            bp.table_bytes = cur.table_bytes;
            continue;
        }
        cur.x_off = x_off;
        cur.r_off = r_off;
        cur.spec_off = spec_off;
        cur.spec_bytes = spec_max;
        cur.total = spec_off + spec_max;
        bp = std::move(cur);
    }
    return MRINV_OK;
}

extern "C" size_t mrinv_batched_workspace_size(mrinv_handle_t h, int count, const int *d, const int64_t *n,
                                               mrinv_precision_t prec) {
    if (count < 1 || !d || !n) return 0;
    BatchPlan bp;
    if (plan_batched(h, count, nullptr, d, n, prec, nullptr, nullptr, bp) != MRINV_OK) return 0;
    return bp.total;
}

static void batch_plan_free(void *plan) { delete (BatchPlan *)plan; }

extern "C" mrinv_status_t mrinv_psi_inverse_batched_prepare(mrinv_handle_t h, int count, const double *const *q_ptrs,
                                                            const int *d, const int64_t *n,
                                                            mrinv_precision_t precision, double *const *psi_ptrs,
                                                            void *ws, size_t wsb) {
    if (!h || count < 1 || !q_ptrs || !d || !n || !psi_ptrs) return fail(MRINV_E_ARG, "NULL handle or pointer");
    for (int b = 0; b < count; ++b)
        if (!q_ptrs[b] || !psi_ptrs[b]) return fail(MRINV_E_ARG, "NULL problem pointer %d", b);
    auto *bp = new (std::nothrow) BatchPlan();
    if (!bp) return fail(MRINV_E_ARG, "out of host memory");
    mrinv_status_t st = plan_batched(h, count, q_ptrs, d, n, precision, psi_ptrs, (char *)ws, *bp);
    if (st == MRINV_OK) st = check_ws(ws, wsb, bp->total);
    if (st != MRINV_OK) {
        delete bp;
        return st;
    }
    // The descriptor table goes into the head of the workspace from pageable
    // host memory owned by the plan; the call waits for it, so the table is in
    // place before any launch of the plan is enqueued.
    bp->ws = (char *)ws;
    hipError_t e = hipMemcpyAsync(ws, bp->table.data(), bp->table.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        delete bp;
        return fail(MRINV_E_HIP, "descriptor upload: %s", hipGetErrorString(e));
    }
    batch_plan_free(h->batch);
    h->batch = bp;
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_psi_inverse_batched_launch(mrinv_handle_t h) {
    TimerScope _ts(h);
    if (!h) return fail(MRINV_E_ARG, "NULL handle");
    auto *bp = (BatchPlan *)h->batch;
    if (!bp) return fail(MRINV_E_ARG, "no batched plan prepared on this handle");
    for (auto &launch : bp->launches) HIP_TRY(launch(bp->ws, h->stream));
    return MRINV_OK;
}

extern "C" mrinv_status_t mrinv_psi_inverse_batched(mrinv_handle_t h, int count, const double *const *q_ptrs,
                                                    const int *d, const int64_t *n, mrinv_precision_t precision,
                                                    double *const *psi_ptrs, void *ws, size_t wsb) {
    CHECK(mrinv_psi_inverse_batched_prepare(h, count, q_ptrs, d, n, precision, psi_ptrs, ws, wsb));
    return mrinv_psi_inverse_batched_launch(h);
}
