// Batched FFTs along the time axis of time-major matrix sequences.
//
// A real sequence X[t][e] (t = time, e = matrix entry "lane", e < nreal) is
// read as complex lanes z_c(t) = X[t][2c] + i X[t][2c+1] (the second entry is
// zero when nreal is odd), so one complex transform carries two real
// sequences; the frequency-domain product kernels separate them with the
// Hermitian symmetry of real spectra.  Spectra are stored in a complex buffer
// Z[row][c] with nl = ceil(nreal/2) lanes per row.
//
// Length L = 2^lgL is split into passes of radix P_1..P_p (each <= 512).  The
// forward transform is decimation in frequency, in place: pass j works on
// blocks of B_j = L/(P_1..P_{j-1}) rows, takes P_j rows at stride
// S_j = B_j/P_j, does a P_j-point DFT and multiplies output r by
// W_{B_j}^{m r} (m = offset of the column inside its block).  The result is
// in digit-reversed order: frequency k = k_1 + P_1 k_2 + P_1 P_2 k_3 + ... sits
// at row k_1 S_1 + k_2 S_2 + ...  The inverse runs the passes in reverse order
// with conjugate twiddles applied before each DFT (decimation in time) and
// returns natural time order.  The digit-reversed spectrum never leaves the
// library; the product kernels address frequencies through it.
//
// Inside a workgroup a P-point DFT over C lanes is a Stockham autosort FFT of
// up to three register-radix stages (radix <= 16); the first stage reads global
// memory directly, the last stage writes global memory directly, and LDS holds
// the data between stages.
#include <stdio.h>

#include "common.h"
#include "kernels.h"

namespace mrinv {

template <typename T>
struct PassCtx {
    cplx<T> *z;
    int64_t base;   // row of r = 0 in this column
    int64_t S;      // row stride inside the column
    uint32_t m;     // column offset inside its block (twiddle index)
    int lgB;
    int lane;       // complex lane
    bool lane_ok;
    int nl;
};

// One Stockham stage of radix 2^LGR inside a 2^LGP-point transform.
template <typename T, int LGR, bool INV, typename Load, typename Store>
__device__ __forceinline__ void fft_stage(int LGP, int lgNs, int grp, const Load &load, const Store &store,
                                          const Twiddles<T> &tw, bool sync_between) {
    constexpr int R = 1 << LGR;
    const int nbf = 1 << (LGP - LGR);
    const bool active = grp < nbf;
    cplx<T> v[R];
    const int j = grp;
    const int k0 = j & ((1 << lgNs) - 1);
    if (active) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = load(j + (r << (LGP - LGR)));
        if (lgNs > 0) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul<T>(v[r], root_twiddle<T, INV>(tw, (uint32_t)(k0 * r), lgNs + LGR));
        }
        Dft<T, R, INV>::run(v);
    }
    if (sync_between) __syncthreads();
    if (active) {
        const int base = ((j >> lgNs) << (lgNs + LGR)) + k0;
#pragma unroll
        for (int r = 0; r < R; ++r) store(base + (r << lgNs), v[r]);
    }
}

// Full 2^LGP-point DFT of one column of C lanes.  gload(idx) / gstore(idx, v)
// access natural-order element idx; src_lds / dst_lds say whether they are
// the LDS buffer itself (then stages that read and write it synchronise).
template <typename T, int LGP, bool INV, typename GL, typename GS>
__device__ __forceinline__ void wg_fft(cplx<T> *lds, int lds_stride, int c, int grp, const GL &gload,
                                       const GS &gstore, bool src_lds, bool dst_lds, const Twiddles<T> &tw) {
    constexpr int NS = num_stages(LGP);
    constexpr int R0 = stage_lg(LGP, 0), R1 = stage_lg(LGP, 1), R2 = stage_lg(LGP, 2);
    auto lload = [&](int idx) { return lds[idx * lds_stride + c]; };
    auto lstore = [&](int idx, cplx<T> v) { lds[idx * lds_stride + c] = v; };
    if constexpr (NS == 1) {
        fft_stage<T, R0, INV>(LGP, 0, grp, gload, gstore, tw, src_lds && dst_lds);
    } else if constexpr (NS == 2) {
        fft_stage<T, R0, INV>(LGP, 0, grp, gload, lstore, tw, src_lds);
        __syncthreads();
        fft_stage<T, R1, INV>(LGP, R0, grp, lload, gstore, tw, dst_lds);
    } else {
        fft_stage<T, R0, INV>(LGP, 0, grp, gload, lstore, tw, src_lds);
        __syncthreads();
        fft_stage<T, R1, INV>(LGP, R0, grp, lload, lstore, tw, true);
        __syncthreads();
        fft_stage<T, R2, INV>(LGP, R0 + R1, grp, lload, gstore, tw, dst_lds);
    }
}

template <typename T>
__device__ __forceinline__ bool is_diag_lane(int e, int e0_d) {
    return e < e0_d * e0_d && (e % (e0_d + 1)) == 0;
}

// Read complex lane `lane` of real row t of the source (zero outside [lo, hi)).
template <typename T>
__device__ __forceinline__ cplx<T> load_real(const SrcDesc &s, int64_t t, int lane) {
    if (t < s.lo || t >= s.hi) return mk<T>(0, 0);
    const int64_t row = s.rev >= 0 ? s.rev - t : t;
    const int e = 2 * lane;
    T a = 0, b = 0;
    if (s.kind == SRC_REAL64) {
        const double *p = (const double *)s.p + row * s.ld;
        a = (T)p[e];
        if (e + 1 < s.nreal) b = (T)p[e + 1];
    } else {
        const float *p = (const float *)s.p + row * s.ld;
        a = (T)p[e];
        if (e + 1 < s.nreal) b = (T)p[e + 1];
    }
    if (s.e0_d > 0) {
        a = (t == 0 && is_diag_lane<T>(e, s.e0_d) ? (T)1 : (T)0) - a;
        b = (e + 1 < s.nreal) ? ((t == 0 && is_diag_lane<T>(e + 1, s.e0_d) ? (T)1 : (T)0) - b) : (T)0;
    }
    return mk<T>(a, b);
}

__device__ __forceinline__ void flag_nonfinite(unsigned int *status, double a, double b) {
    if (status && (!isfinite(a) || !isfinite(b))) atomicOr(status, STATUS_NONFINITE);
}

// Write complex lane `lane` (two real entries) of real row t of the destination.
template <typename T>
__device__ __forceinline__ void store_real(const DstDesc &d, int64_t t, int lane, cplx<T> v) {
    if (t < d.lo || t >= d.hi) return;
    const int64_t row = d.rev >= 0 ? d.rev - t : t;
    const int e = 2 * lane;
    const bool two = e + 1 < d.nreal;
    double a = (double)v.x * d.scale, b = (double)v.y * d.scale;
    switch (d.op) {
        case OP_NEG: a = -a; b = -b; break;
        case OP_E0MINUS:
            a = (t == 0 && is_diag_lane<T>(e, d.e0_d) ? 1.0 : 0.0) - a;
            b = (t == 0 && is_diag_lane<T>(e + 1, d.e0_d) ? 1.0 : 0.0) - b;
            break;
        default: break;
    }
    if (d.op == OP_XPLUS) {
        const float *x = (const float *)d.aux + row * d.ld;
        a += (double)x[e];
        if (two) b += (double)x[e + 1];
    }
    if (d.kind == DST_REAL64) {
        double *p = (double *)d.p + row * d.ld;
        if (d.op == OP_ADD) { a += p[e]; if (two) b += p[e + 1]; }
        p[e] = a;
        if (two) p[e + 1] = b;
    } else {
        float *p = (float *)d.p + row * d.ld;
        if (d.op == OP_ADD) { a += p[e]; if (two) b += p[e + 1]; }
        p[e] = (float)a;
        if (two) p[e + 1] = (float)b;
    }
    flag_nonfinite(d.status, a, two ? b : 0.0);
}

// MODE 0: forward pass; MODE 1: inverse pass; MODE 2: inverse pass, then the
// mask/scale/negate of `dst` (rows outside [lo, hi) become zero), then the
// forward pass of the same geometry, in place.
// The body of one pass for one column of one problem.
template <typename T, int LGP, int C, int MODE>
__device__ __forceinline__ void fft_pass_body(cplx<T> *z, const PassGeom &g, int nl, int nchunks, int64_t blk,
                                              const SrcDesc &src, const DstDesc &dst, const Twiddles<T> &tw) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *lds = reinterpret_cast<cplx<T> *>(smem_raw);
    constexpr int LDS_STRIDE = C + 1;
    const int c = threadIdx.x % C;
    const int grp = threadIdx.x / C;
    int chunk;
    int64_t col;
    if (g.col_fastest) {
        const int64_t ncols = g.L >> LGP;
        col = blk % ncols;
        chunk = (int)(blk / ncols);
    } else {
        chunk = (int)(blk % nchunks);
        col = blk / nchunks;
    }
    const int64_t S = g.S;
    const int64_t b = col >> (g.lgB - LGP);          // S = 2^(lgB - LGP)
    const uint32_t m = (uint32_t)(col & (S - 1));
    const int64_t base = b * ((int64_t)1 << g.lgB) + m;
    const int lane = chunk * C + c;
    const bool lane_ok = lane < nl;

    // Forward twiddle on output r: W_B^{m r}; inverse on input r: W_B^{-m r},
    // from the pass's table when there is one.
    const cplx<T> *otw = reinterpret_cast<const cplx<T> *>(tw.outer) + ((size_t)m << LGP);
    auto outer = [&](int idx, bool inv) {
        if (tw.outer) {
            const cplx<T> w = otw[idx];
            return inv ? cconj<T>(w) : w;
        }
        return inv ? twiddle<T, true>(tw, m * (uint32_t)idx, g.lgB) : twiddle<T, false>(tw, m * (uint32_t)idx, g.lgB);
    };
    auto fwd_store = [&](int idx, cplx<T> v) {
        if (!lane_ok) return;
        if (m) v = cmul<T>(v, outer(idx, false));
        z[(base + idx * S) * nl + lane] = v;
    };
    auto inv_load = [&](int idx) {
        if (!lane_ok) return mk<T>(0, 0);
        cplx<T> v = z[(base + idx * S) * nl + lane];
        if (m) v = cmul<T>(v, outer(idx, true));
        return v;
    };

    if constexpr (MODE == 0) {
        auto gload = [&](int idx) {
            if (!lane_ok) return mk<T>(0, 0);
            const int64_t row = base + idx * S;
            if (src.kind == SRC_Z) return z[row * nl + lane];
            return load_real<T>(src, row, lane);
        };
        wg_fft<T, LGP, false>(lds, LDS_STRIDE, c, grp, gload, fwd_store, false, false, tw);
    } else if constexpr (MODE == 1) {
        auto gstore = [&](int idx, cplx<T> v) {
            if (!lane_ok) return;
            const int64_t row = base + idx * S;
            if (dst.kind == DST_Z) z[row * nl + lane] = v;
            else store_real<T>(dst, row, lane, v);
        };
        wg_fft<T, LGP, true>(lds, LDS_STRIDE, c, grp, inv_load, gstore, false, false, tw);
    } else {
        const T sc = (T)dst.scale;
        auto mask_store = [&](int idx, cplx<T> v) {
            const int64_t t = base + idx * S;
            const bool keep = t >= dst.lo && t < dst.hi;
            const T s = dst.op == OP_NEG ? -sc : sc;
            lds[idx * LDS_STRIDE + c] = keep ? cscale<T>(v, s) : mk<T>(0, 0);
        };
        wg_fft<T, LGP, true>(lds, LDS_STRIDE, c, grp, inv_load, mask_store, false, true, tw);
        __syncthreads();
        auto lds_load = [&](int idx) { return lds[idx * LDS_STRIDE + c]; };
        wg_fft<T, LGP, false>(lds, LDS_STRIDE, c, grp, lds_load, fwd_store, true, false, tw);
    }
}

template <typename T, int LGP, int C, int MODE>
__global__ void __launch_bounds__(C << (LGP - min_stage_lg(LGP)))
fft_pass_kernel(cplx<T> *z, PassGeom g, SrcDesc src, DstDesc dst, Twiddles<T> tw) {
    fft_pass_body<T, LGP, C, MODE>(z, g, g.nl, g.nchunks, blockIdx.x, src, dst, tw);
}

// Two problems of the same geometry by value (the forward transforms of both
// operands of a product in one launch).
template <typename T, int LGP, int C, int MODE>
__global__ void __launch_bounds__(C << (LGP - min_stage_lg(LGP)))
fft_pass_pair_kernel(PassProblem<T> a, PassProblem<T> b, PassGeom g, Twiddles<T> tw) {
    const int64_t bid = blockIdx.x;
    if (bid < b.wg_begin) fft_pass_body<T, LGP, C, MODE>(a.z, g, a.nl, a.nchunks, bid, a.src, a.dst, tw);
    else fft_pass_body<T, LGP, C, MODE>(b.z, g, b.nl, b.nchunks, bid - b.wg_begin, b.src, b.dst, tw);
}

// Batched: the workgroup's problem is found by binary search over wg_begin.
template <typename T, int LGP, int C, int MODE>
__global__ void __launch_bounds__(C << (LGP - min_stage_lg(LGP)))
fft_pass_batched_kernel(const PassProblem<T> *probs, int nprob, PassGeom g, Twiddles<T> tw) {
    int lo = 0, hi = nprob - 1;
    const int64_t bid = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].wg_begin <= bid) lo = mid;
        else hi = mid - 1;
    }
    const PassProblem<T> &pp = probs[lo];
    fft_pass_body<T, LGP, C, MODE>(pp.z, g, pp.nl, pp.nchunks, bid - pp.wg_begin, pp.src, pp.dst, tw);
}

// ---------------------------------------------------------------------------
// Host-side launch: dispatch on (T, lgP, C, mode).
// ---------------------------------------------------------------------------
static double window_rows(int64_t L, int64_t lo, int64_t hi) {
    const int64_t a = lo > 0 ? lo : 0, b = hi < L ? hi : L;
    return b > a ? (double)(b - a) : 0.0;
}

// Algorithmic bytes of one pass: each input element the pass needs read once,
// each output element written once.
template <typename T>
static double pass_bytes(int mode, const PassGeom &g, const SrcDesc &src, const DstDesc &dst) {
    const double zc = (double)g.L * g.nl * sizeof(cplx<T>);
    double rd = zc, wr = zc;
    if (mode == 0 && src.kind != SRC_Z)
        rd = window_rows(g.L, src.lo, src.hi) * src.nreal * (src.kind == SRC_REAL64 ? 8.0 : 4.0);
    if (mode == 1 && dst.kind != DST_Z) {
        const double rows = window_rows(g.L, dst.lo, dst.hi);
        const double w = dst.kind == DST_REAL64 ? 8.0 : 4.0;
        wr = rows * dst.nreal * w;
        if (dst.op == OP_ADD) rd += rows * dst.nreal * w;
        if (dst.op == OP_XPLUS) rd += rows * dst.nreal * 4.0;
    }
    return rd + wr;
}

template <typename T, int LGP, int C, int MODE>
static hipError_t launch_pass_t(cplx<T> *z, const PassGeom &g, const SrcDesc &src, const DstDesc &dst,
                                const Twiddles<T> &tw, hipStream_t st) {
    const int threads = C << (LGP - min_stage_lg(LGP));
    const size_t lds = (num_stages(LGP) > 1 || MODE == 2) ? ((size_t)1 << LGP) * (C + 1) * sizeof(cplx<T>) : 0;
    auto kern = fft_pass_kernel<T, LGP, C, MODE>;
    static bool attr_set = false;
    if (!attr_set && lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
        attr_set = true;
    }
    const int64_t cols = g.L >> LGP;
    const int64_t blocks = cols * g.nchunks;
    char name[96];
    snprintf(name, sizeof name, "fft_pass_kernel<%s, %d, %d, %d>", sizeof(T) == 8 ? "double" : "float", LGP, C, MODE);
    launch_begin(name, pass_bytes<T>(MODE, g, src, dst), 0.0);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(threads), lds, st, z, g, src, dst, tw);
    launch_end();
    return hipGetLastError();
}

template <typename T, int C, int MODE>
static hipError_t launch_pass_c(int lgP, cplx<T> *z, const PassGeom &g, const SrcDesc &src, const DstDesc &dst,
                                const Twiddles<T> &tw, hipStream_t st) {
    switch (lgP) {
        case 1: return launch_pass_t<T, 1, C, MODE>(z, g, src, dst, tw, st);
        case 2: return launch_pass_t<T, 2, C, MODE>(z, g, src, dst, tw, st);
        case 3: return launch_pass_t<T, 3, C, MODE>(z, g, src, dst, tw, st);
        case 4: return launch_pass_t<T, 4, C, MODE>(z, g, src, dst, tw, st);
        case 5: return launch_pass_t<T, 5, C, MODE>(z, g, src, dst, tw, st);
        case 6: return launch_pass_t<T, 6, C, MODE>(z, g, src, dst, tw, st);
        case 7: return launch_pass_t<T, 7, C, MODE>(z, g, src, dst, tw, st);
        case 8: return launch_pass_t<T, 8, C, MODE>(z, g, src, dst, tw, st);
        case 9: return launch_pass_t<T, 9, C, MODE>(z, g, src, dst, tw, st);
        default: return hipErrorInvalidValue;
    }
}

// 32 lanes per workgroup only up to 256-row passes (LDS).
template <typename T, int MODE>
static hipError_t launch_pass_c32(int lgP, cplx<T> *z, const PassGeom &g, const SrcDesc &src, const DstDesc &dst,
                                  const Twiddles<T> &tw, hipStream_t st) {
    switch (lgP) {
        case 1: return launch_pass_t<T, 1, 32, MODE>(z, g, src, dst, tw, st);
        case 2: return launch_pass_t<T, 2, 32, MODE>(z, g, src, dst, tw, st);
        case 3: return launch_pass_t<T, 3, 32, MODE>(z, g, src, dst, tw, st);
        case 4: return launch_pass_t<T, 4, 32, MODE>(z, g, src, dst, tw, st);
        case 5: return launch_pass_t<T, 5, 32, MODE>(z, g, src, dst, tw, st);
        case 6: return launch_pass_t<T, 6, 32, MODE>(z, g, src, dst, tw, st);
        case 7: return launch_pass_t<T, 7, 32, MODE>(z, g, src, dst, tw, st);
        case 8: return launch_pass_t<T, 8, 32, MODE>(z, g, src, dst, tw, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int MODE>
static hipError_t launch_pass_m(int lgP, int C, cplx<T> *z, const PassGeom &g, const SrcDesc &src,
                                const DstDesc &dst, const Twiddles<T> &tw, hipStream_t st) {
    switch (C) {
        case 2: return launch_pass_c<T, 2, MODE>(lgP, z, g, src, dst, tw, st);
        case 8: return launch_pass_c<T, 8, MODE>(lgP, z, g, src, dst, tw, st);
        case 16: return launch_pass_c<T, 16, MODE>(lgP, z, g, src, dst, tw, st);
        case 32: return launch_pass_c32<T, MODE>(lgP, z, g, src, dst, tw, st);
        default: return hipErrorInvalidValue;
    }
}

int fft_lanes_per_block(bool dbl, int nl) {
    if (nl <= 2) return 2;
    if (dbl) return 8;
    return nl <= 8 ? 8 : 16;
}

template <typename T>
hipError_t fft_pass(int mode, const FftPlan &plan, int pass, int nl, cplx<T> *z, const SrcDesc &src,
                    const DstDesc &dst, const Twiddles<T> &tw, hipStream_t st, int lanes, int order) {
    PassGeom g{};
    g.col_fastest = order;
    g.L = (int64_t)1 << plan.lgL;
    int lgB = plan.lgL;
    for (int j = 0; j < pass; ++j) lgB -= plan.lgP[j];
    g.lgB = lgB;
    g.S = (int64_t)1 << (lgB - plan.lgP[pass]);
    g.nl = nl;
    const int lgP = plan.lgP[pass];
    int C = nl <= 2 ? 2 : (lanes ? lanes : fft_lanes_per_block(sizeof(T) == 8, nl));
    if (C == 32 && (lgP > 8 || nl <= 16)) C = 16;
    g.nchunks = (nl + C - 1) / C;
    Twiddles<T> t = tw;
    t.outer = plan.outer[pass];
    switch (mode) {
        case 0: return launch_pass_m<T, 0>(lgP, C, z, g, src, dst, t, st);
        case 1: return launch_pass_m<T, 1>(lgP, C, z, g, src, dst, t, st);
        default: return launch_pass_m<T, 2>(lgP, C, z, g, src, dst, t, st);
    }
}

template <typename T, int LGP, int C, int MODE>
static hipError_t launch_batched_t(const PassProblem<T> *probs, int nprob, int64_t total, const PassGeom &g,
                                   double bytes, const Twiddles<T> &tw, hipStream_t st) {
    const int threads = C << (LGP - min_stage_lg(LGP));
    const size_t lds = (num_stages(LGP) > 1 || MODE == 2) ? ((size_t)1 << LGP) * (C + 1) * sizeof(cplx<T>) : 0;
    auto kern = fft_pass_batched_kernel<T, LGP, C, MODE>;
    static bool attr_set = false;
    if (!attr_set && lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
        attr_set = true;
    }
    char name[96];
    snprintf(name, sizeof name, "fft_pass_batched_kernel<%s, %d, %d, %d>", sizeof(T) == 8 ? "double" : "float", LGP,
             C, MODE);
    launch_begin(name, bytes, 0.0);
    hipLaunchKernelGGL(kern, dim3((unsigned)total), dim3(threads), lds, st, probs, nprob, g, tw);
    launch_end();
    return hipGetLastError();
}

template <typename T, int LGP, int C, int MODE>
static hipError_t launch_pair_t(const PassProblem<T> &a, const PassProblem<T> &b, int64_t total, const PassGeom &g,
                                double bytes, const Twiddles<T> &tw, hipStream_t st) {
    const int threads = C << (LGP - min_stage_lg(LGP));
    const size_t lds = (num_stages(LGP) > 1 || MODE == 2) ? ((size_t)1 << LGP) * (C + 1) * sizeof(cplx<T>) : 0;
    auto kern = fft_pass_pair_kernel<T, LGP, C, MODE>;
    static bool attr_set = false;
    if (!attr_set && lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
        attr_set = true;
    }
    char name[96];
    snprintf(name, sizeof name, "fft_pass_pair_kernel<%s, %d, %d, %d>", sizeof(T) == 8 ? "double" : "float", LGP, C,
             MODE);
    launch_begin(name, bytes, 0.0);
    hipLaunchKernelGGL(kern, dim3((unsigned)total), dim3(threads), lds, st, a, b, g, tw);
    launch_end();
    return hipGetLastError();
}

template <typename T, int C>
static hipError_t launch_pair_c(int lgP, const PassProblem<T> &a, const PassProblem<T> &b, int64_t total,
                                const PassGeom &g, double bytes, const Twiddles<T> &tw, hipStream_t st) {
    if (C == 32 && lgP > 8) return hipErrorInvalidValue;
    switch (lgP) {
        case 1: return launch_pair_t<T, 1, C, 0>(a, b, total, g, bytes, tw, st);
        case 2: return launch_pair_t<T, 2, C, 0>(a, b, total, g, bytes, tw, st);
        case 3: return launch_pair_t<T, 3, C, 0>(a, b, total, g, bytes, tw, st);
        case 4: return launch_pair_t<T, 4, C, 0>(a, b, total, g, bytes, tw, st);
        case 5: return launch_pair_t<T, 5, C, 0>(a, b, total, g, bytes, tw, st);
        case 6: return launch_pair_t<T, 6, C, 0>(a, b, total, g, bytes, tw, st);
        case 7: return launch_pair_t<T, 7, C, 0>(a, b, total, g, bytes, tw, st);
        case 8: return launch_pair_t<T, 8, C, 0>(a, b, total, g, bytes, tw, st);
        case 9: return launch_pair_t<T, 9, (C > 16 ? 16 : C), 0>(a, b, total, g, bytes, tw, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int C, int MODE>
static hipError_t launch_batched_c(int lgP, const PassProblem<T> *probs, int nprob, int64_t total,
                                   const PassGeom &g, double bytes, const Twiddles<T> &tw, hipStream_t st) {
    switch (lgP) {
        case 1: return launch_batched_t<T, 1, C, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 2: return launch_batched_t<T, 2, C, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 3: return launch_batched_t<T, 3, C, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 4: return launch_batched_t<T, 4, C, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 5: return launch_batched_t<T, 5, C, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 6: return launch_batched_t<T, 6, C, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 7: return launch_batched_t<T, 7, C, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 8: return launch_batched_t<T, 8, C, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 9: return launch_batched_t<T, 9, C, MODE>(probs, nprob, total, g, bytes, tw, st);
        default: return hipErrorInvalidValue;
    }
}

static PassGeom pass_geom(const FftPlan &plan, int pass) {
    PassGeom g{};
    g.L = (int64_t)1 << plan.lgL;
    int lgB = plan.lgL;
    for (int j = 0; j < pass; ++j) lgB -= plan.lgP[j];
    g.lgB = lgB;
    g.S = (int64_t)1 << (lgB - plan.lgP[pass]);
    return g;
}

template <typename T>
int64_t fft_batch_layout(const FftPlan &plan, int pass, PassProblem<T> *probs, int nprob, int C) {
    const int64_t cols = ((int64_t)1 << plan.lgL) >> plan.lgP[pass];
    int64_t acc = 0;
    for (int i = 0; i < nprob; ++i) {
        probs[i].nchunks = (probs[i].nl + C - 1) / C;
        probs[i].wg_begin = acc;
        acc += cols * probs[i].nchunks;
    }
    return acc;
}

template <typename T>
hipError_t fft_pass_batched(int mode, const FftPlan &plan, int pass, int C, const PassProblem<T> *probs, int nprob,
                            int64_t total, double bytes, const Twiddles<T> &tw_in, hipStream_t st) {
    const PassGeom g = pass_geom(plan, pass);
    const int lgP = plan.lgP[pass];
    Twiddles<T> tw = tw_in;
    tw.outer = plan.outer[pass];
    switch (mode * 100 + C) {
        case 2: return launch_batched_c<T, 2, 0>(lgP, probs, nprob, total, g, bytes, tw, st);
        case 8: return launch_batched_c<T, 8, 0>(lgP, probs, nprob, total, g, bytes, tw, st);
        case 16: return launch_batched_c<T, 16, 0>(lgP, probs, nprob, total, g, bytes, tw, st);
        case 102: return launch_batched_c<T, 2, 1>(lgP, probs, nprob, total, g, bytes, tw, st);
        case 108: return launch_batched_c<T, 8, 1>(lgP, probs, nprob, total, g, bytes, tw, st);
        case 116: return launch_batched_c<T, 16, 1>(lgP, probs, nprob, total, g, bytes, tw, st);
        case 202: return launch_batched_c<T, 2, 2>(lgP, probs, nprob, total, g, bytes, tw, st);
        case 208: return launch_batched_c<T, 8, 2>(lgP, probs, nprob, total, g, bytes, tw, st);
        case 216: return launch_batched_c<T, 16, 2>(lgP, probs, nprob, total, g, bytes, tw, st);
        default: return hipErrorInvalidValue;
    }
}

template int64_t fft_batch_layout<double>(const FftPlan &, int, PassProblem<double> *, int, int);
template int64_t fft_batch_layout<float>(const FftPlan &, int, PassProblem<float> *, int, int);
template hipError_t fft_pass_batched<double>(int, const FftPlan &, int, int, const PassProblem<double> *, int,
                                             int64_t, double, const Twiddles<double> &, hipStream_t);
template hipError_t fft_pass_batched<float>(int, const FftPlan &, int, int, const PassProblem<float> *, int,
                                            int64_t, double, const Twiddles<float> &, hipStream_t);

// Outer-twiddle tables (see TwGen); values are the same two-level products
// the passes would otherwise form on the fly.
__global__ void gen_outer_twiddles_kernel(TwGen g, const double2 *hi, const double2 *lo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.total) return;
    int t = 0;
    while (t + 1 < g.count && g.begin[t + 1] <= i) ++t;
    const int64_t e = i - g.begin[t];
    const uint32_t m = (uint32_t)(e >> g.lgP[t]), kr = (uint32_t)(e & ((1 << g.lgP[t]) - 1));
    Twiddles<double> tw{hi, lo, nullptr, nullptr};
    const double2 w = twiddle<double, false>(tw, m * kr, g.lgB[t]);
    if (g.dbl[t]) ((double2 *)g.dst[t])[e] = w;
    else ((float2 *)g.dst[t])[e] = make_float2((float)w.x, (float)w.y);
}

hipError_t gen_outer_twiddles(const TwGen &g, const double2 *hi, const double2 *lo, hipStream_t st) {
    if (g.count == 0 || g.total == 0) return hipSuccess;
    launch_begin("gen_outer_twiddles_kernel", 0.0, 0.0);
    hipLaunchKernelGGL(gen_outer_twiddles_kernel, dim3((unsigned)((g.total + 255) / 256)), dim3(256), 0, st, g, hi, lo);
    launch_end();
    return hipGetLastError();
}

template hipError_t fft_pass<double>(int, const FftPlan &, int, int, cplx<double> *, const SrcDesc &,
                                     const DstDesc &, const Twiddles<double> &, hipStream_t, int, int);
template hipError_t fft_pass<float>(int, const FftPlan &, int, int, cplx<float> *, const SrcDesc &,
                                    const DstDesc &, const Twiddles<float> &, hipStream_t, int, int);

template <typename T>
hipError_t fft_pass_pair(const FftPlan &plan, int pass, PassProblem<T> a, PassProblem<T> b, const Twiddles<T> &tw,
                         hipStream_t st, int lanes, int order) {
    PassGeom g = pass_geom(plan, pass);
    g.col_fastest = order;
    const int nlmin = a.nl < b.nl ? a.nl : b.nl;
    int C = nlmin <= 2 ? 2 : (lanes ? lanes : fft_lanes_per_block(sizeof(T) == 8, a.nl > b.nl ? a.nl : b.nl));
    if (C == 32 && (plan.lgP[pass] > 8 || nlmin <= 16)) C = 16;
    const int64_t cols = g.L >> plan.lgP[pass];
    a.nchunks = (a.nl + C - 1) / C;
    b.nchunks = (b.nl + C - 1) / C;
    a.wg_begin = 0;
    b.wg_begin = cols * a.nchunks;
    const int64_t total = b.wg_begin + cols * b.nchunks;
    PassGeom ga = g, gb = g;
    ga.nl = a.nl; ga.nchunks = a.nchunks;
    gb.nl = b.nl; gb.nchunks = b.nchunks;
    const double bytes = pass_bytes<T>(0, ga, a.src, a.dst) + pass_bytes<T>(0, gb, b.src, b.dst);
    const int lgP = plan.lgP[pass];
    Twiddles<T> t = tw;
    t.outer = plan.outer[pass];
    switch (C) {
        case 2: return launch_pair_c<T, 2>(lgP, a, b, total, g, bytes, t, st);
        case 8: return launch_pair_c<T, 8>(lgP, a, b, total, g, bytes, t, st);
        case 16: return launch_pair_c<T, 16>(lgP, a, b, total, g, bytes, t, st);
        case 32: return launch_pair_c<T, 32>(lgP, a, b, total, g, bytes, t, st);
        default: return hipErrorInvalidValue;
    }
}
template hipError_t fft_pass_pair<double>(const FftPlan &, int, PassProblem<double>, PassProblem<double>,
                                          const Twiddles<double> &, hipStream_t, int, int);
template hipError_t fft_pass_pair<float>(const FftPlan &, int, PassProblem<float>, PassProblem<float>,
                                         const Twiddles<float> &, hipStream_t, int, int);

}  // namespace mrinv
