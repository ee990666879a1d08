// Frequency-domain matrix products (Section 2.1, eq. (fft-convolution):
// the product of two sequences is the inverse DFT of the frequency-wise matrix
// products, in the original operand order).
//
// Inputs are packed spectra (complex lane c of a real sequence carries real
// entries 2c and 2c+1) in the digit-reversed row order of the FFT plan.  For
// a real sequence x with spectrum X, X(L-k) = conj(X(k)), so the two real
// entries of lane c are separated as
//     X_2c(k)   = (z(k) + conj(z(L-k))) / 2
//     X_2c+1(k) = (z(k) - conj(z(L-k))) / (2i).
// Each kernel therefore visits frequencies k = 0..L/2 once, reads rows k and
// L-k, forms the product at k, and writes the packed result at both rows
// (the value at L-k is the conjugate by the same symmetry).
#include <stdio.h>

#include <algorithm>
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace mrinv {

// Row holding frequency k in the digit-reversed order of the plan.
__device__ __forceinline__ int64_t freq_row(const FftPlan &p, int64_t k) {
    int64_t pos = 0;
    int rem = p.lgL;
#pragma unroll
    for (int j = 0; j < MAX_PASSES; ++j) {
        if (j < p.npass) {
            rem -= p.lgP[j];
            pos += (k & ((1LL << p.lgP[j]) - 1)) << rem;
            k >>= p.lgP[j];
        }
    }
    return pos;
}

template <typename T>
__device__ __forceinline__ cplx<T> unpack(const cplx<T> *Z, int nl, int64_t r1, int64_t r2, int e) {
    const cplx<T> z1 = Z[r1 * nl + (e >> 1)];
    const cplx<T> z2 = Z[r2 * nl + (e >> 1)];
    if ((e & 1) == 0) return mk<T>((z1.x + z2.x) * (T)0.5, (z1.y - z2.y) * (T)0.5);
    return mk<T>((z1.y + z2.y) * (T)0.5, (z2.x - z1.x) * (T)0.5);
}

// Packed value for row k and row L-k from the two real-sequence values.
template <typename T>
__device__ __forceinline__ void pack_store(cplx<T> *Z, int nl, int64_t r1, int64_t r2, int c, cplx<T> ce,
                                           cplx<T> co) {
    Z[r1 * nl + c] = mk<T>(ce.x - co.y, ce.y + co.x);
    if (r2 != r1) Z[r2 * nl + c] = mk<T>(ce.x + co.y, co.x - ce.y);
}

constexpr int GEMM_THREADS = 256;

template <typename T, int TM, int TN>
__global__ void __launch_bounds__(GEMM_THREADS)
freq_gemm_kernel(const cplx<T> *__restrict__ ZA, const cplx<T> *__restrict__ ZB, cplx<T> *__restrict__ ZC,
                 FftPlan plan, GemmDesc g, int NF, int KC, int tiles_j, int tiles) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *As = reinterpret_cast<cplx<T> *>(smem_raw);          // [NF][ra][KC+1]
    cplx<T> *Bs = As + (size_t)NF * g.ra * (KC + 1);               // [NF][KC][cb+1]
    __shared__ int64_t rows1[GEMM_THREADS], rows2[GEMM_THREADS];
    const int64_t L = (int64_t)1 << plan.lgL;
    const int64_t F = L / 2 + 1;
    const int64_t k0 = (int64_t)blockIdx.x * NF;
    const int tid = threadIdx.x;
    if (tid < NF) {
        const int64_t k = k0 + tid;
        rows1[tid] = k < F ? freq_row(plan, k) : 0;
        rows2[tid] = k < F ? freq_row(plan, (L - k) & (L - 1)) : 0;
    }
    __syncthreads();
    const int ra = g.ra, m = g.m, cb = g.cb;
    const int f = tid / tiles, tile = tid - f * tiles;
    const int i0 = (tile / tiles_j) * TM, j0 = (tile % tiles_j) * TN;
    const bool active = f < NF && k0 + f < F;
    cplx<T> acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = mk<T>(0, 0);

    for (int kc = 0; kc < m; kc += KC) {
        const int kw = min(KC, m - kc);
        for (int idx = tid; idx < NF * ra * kw; idx += GEMM_THREADS) {
            const int ff = idx / (ra * kw), rem = idx - ff * ra * kw;
            const int i = rem / kw, t = rem - i * kw;
            cplx<T> v = mk<T>(0, 0);
            if (k0 + ff < F) {
                const int e = g.transA ? (kc + t) * ra + i : i * m + kc + t;
                v = unpack<T>(ZA, g.nlA, rows1[ff], rows2[ff], e);
            }
            As[((size_t)ff * ra + i) * (KC + 1) + t] = v;
        }
        for (int idx = tid; idx < NF * kw * cb; idx += GEMM_THREADS) {
            const int ff = idx / (kw * cb), rem = idx - ff * kw * cb;
            const int t = rem / cb, j = rem - t * cb;
            cplx<T> v = mk<T>(0, 0);
            if (k0 + ff < F) {
                const int e = g.transB ? j * m + kc + t : (kc + t) * cb + j;
                v = unpack<T>(ZB, g.nlB, rows1[ff], rows2[ff], e);
            }
            Bs[((size_t)ff * KC + t) * (cb + 1) + j] = v;
        }
        __syncthreads();
        if (active) {
            const cplx<T> *Af = As + (size_t)f * ra * (KC + 1);
            const cplx<T> *Bf = Bs + (size_t)f * KC * (cb + 1);
            for (int t = 0; t < kw; ++t) {
                cplx<T> av[TM], bv[TN];
#pragma unroll
                for (int a = 0; a < TM; ++a) av[a] = (i0 + a < ra) ? Af[(i0 + a) * (KC + 1) + t] : mk<T>(0, 0);
#pragma unroll
                for (int b = 0; b < TN; ++b) bv[b] = (j0 + b < cb) ? Bf[t * (cb + 1) + j0 + b] : mk<T>(0, 0);
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b) {
                        acc[a][b].x += av[a].x * bv[b].x - av[a].y * bv[b].y;
                        acc[a][b].y += av[a].x * bv[b].y + av[a].y * bv[b].x;
                    }
            }
        }
        __syncthreads();
    }

    if ((cb & 1) == 0 && (TN & 1) == 0) {
        // Every thread owns whole lane pairs (j0 even, cb even).
        if (active) {
#pragma unroll
            for (int a = 0; a < TM; ++a) {
                const int i = i0 + a;
                if (i >= ra) continue;
#pragma unroll
                for (int b = 0; b < TN; b += 2) {
                    const int j = j0 + b;
                    if (j >= cb) continue;
                    pack_store<T>(ZC, g.nlC, rows1[f], rows2[f], (i * cb + j) >> 1, acc[a][b], acc[a][b + 1]);
                }
            }
        }
    } else {
        // Stage the result in LDS, then write lane pairs.
        cplx<T> *Cs = As;   // [NF][ra*cb + 1]
        const int ld = ra * cb + 1;
        if (active) {
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b)
                    if (i0 + a < ra && j0 + b < cb) Cs[(size_t)f * ld + (i0 + a) * cb + j0 + b] = acc[a][b];
        }
        __syncthreads();
        const int nlC = g.nlC;
        for (int idx = tid; idx < NF * nlC; idx += GEMM_THREADS) {
            const int ff = idx / nlC, c = idx - ff * nlC;
            if (k0 + ff >= F) continue;
            const int e = 2 * c;
            const cplx<T> ce = Cs[(size_t)ff * ld + e];
            const cplx<T> co = (e + 1 < ra * cb) ? Cs[(size_t)ff * ld + e + 1] : mk<T>(0, 0);
            pack_store<T>(ZC, nlC, rows1[ff], rows2[ff], c, ce, co);
        }
    }
}

template <typename T, int TM, int TN>
static hipError_t launch_gemm(const FftPlan &plan, const GemmDesc &g, const cplx<T> *ZA, const cplx<T> *ZB,
                              cplx<T> *ZC, hipStream_t st) {
    const int tiles_i = (g.ra + TM - 1) / TM, tiles_j = (g.cb + TN - 1) / TN;
    const int tiles = tiles_i * tiles_j;
    int NF = GEMM_THREADS / tiles;
    if (NF < 1) return hipErrorInvalidValue;
    const int KC = g.m < 16 ? g.m : 16;
    const bool staged = (g.cb & 1) || (TN & 1);   // output goes through LDS (see kernel epilogue)
    auto bytes = [&](int nf) {
        size_t ab = ((size_t)nf * g.ra * (KC + 1) + (size_t)nf * KC * (g.cb + 1)) * sizeof(cplx<T>);
        size_t cs = staged ? (size_t)nf * (g.ra * g.cb + 1) * sizeof(cplx<T>) : 0;
        return ab > cs ? ab : cs;
    };
    while (NF > 1 && bytes(NF) > 64 * 1024) --NF;
    const int64_t F = ((int64_t)1 << plan.lgL) / 2 + 1;
    const int64_t blocks = (F + NF - 1) / NF;
    char name[96];
    snprintf(name, sizeof name, "freq_gemm_kernel<%s, %d, %d>", sizeof(T) == 8 ? "double" : "float", TM, TN);
    const double Lr = (double)((int64_t)1 << plan.lgL);
    launch_kernel(name, Lr * (g.nlA + g.nlB + g.nlC) * sizeof(cplx<T>), (double)F * 8.0 * g.ra * g.m * g.cb,
                  (freq_gemm_kernel<T, TM, TN>), dim3((unsigned)blocks), dim3(GEMM_THREADS), bytes(NF), st, ZA, ZB,
                  ZC, plan, g, NF, KC, tiles_j, tiles);
    return hipGetLastError();
}

// Square products C = A B (d x d, no transposes) with the padded dimension DP
// a compile-time constant: TM x TN register tiles, NF frequencies per
// workgroup, the contraction staged through LDS in chunks of KC.
template <int DP> struct SqCfg {
    static constexpr int TM = DP <= 8 ? 1 : DP <= 16 ? 2 : DP <= 24 ? 3 : 4;
    static constexpr int TN = DP <= 8 ? 2 : DP <= 16 ? 2 : 4;
    static constexpr int TI = (DP + TM - 1) / TM, TJ = (DP + TN - 1) / TN;
    static constexpr int TILES = TI * TJ;
    static constexpr int NF = TILES >= 256 ? 1 : 256 / TILES;
    static constexpr int THREADS = NF * TILES;
    static constexpr int KC = DP <= 16 ? DP : 8;
    static constexpr int AS = NF * DP * (KC + 1);          // complex elements of the A chunk
    static constexpr int BS = NF * KC * (DP + 1);          // complex elements of the B chunk
};

template <typename T, int DP>
__device__ __forceinline__ void freq_gemm_sq_body(const cplx<T> *__restrict__ ZA, const cplx<T> *__restrict__ ZB,
                                                  cplx<T> *__restrict__ ZC, const FftPlan &plan, int d,
                                                  int64_t blk) {
    using Cfg = SqCfg<DP>;
    constexpr int TM = Cfg::TM, TN = Cfg::TN, NF = Cfg::NF, KC = Cfg::KC, NT = Cfg::THREADS;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *As = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *Bs = As + Cfg::AS;
    __shared__ int64_t rows1[NF], rows2[NF];
    const int64_t L = (int64_t)1 << plan.lgL;
    const int64_t F = L / 2 + 1;
    const int64_t k0 = blk * NF;
    const int tid = threadIdx.x;
    const int nl = (d * d + 1) >> 1;
    if (tid < NF) {
        const int64_t k = k0 + tid;
        rows1[tid] = k < F ? freq_row(plan, k) : 0;
        rows2[tid] = k < F ? freq_row(plan, (L - k) & (L - 1)) : 0;
    }
    __syncthreads();
    const int f = tid / Cfg::TILES, tile = tid - f * Cfg::TILES;
    const int i0 = (tile / Cfg::TJ) * TM, j0 = (tile % Cfg::TJ) * TN;
    const bool active = k0 + f < F;
    cplx<T> acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = mk<T>(0, 0);

    for (int kc = 0; kc < d; kc += KC) {
        for (int idx = tid; idx < NF * DP * KC; idx += NT) {
            const int ff = idx / (DP * KC), rem = idx - ff * (DP * KC);
            const int i = rem / KC, t = rem - i * KC;
            cplx<T> v = mk<T>(0, 0);
            if (i < d && kc + t < d && k0 + ff < F) v = unpack<T>(ZA, nl, rows1[ff], rows2[ff], i * d + kc + t);
            As[(ff * DP + i) * (KC + 1) + t] = v;
        }
        for (int idx = tid; idx < NF * KC * DP; idx += NT) {
            const int ff = idx / (KC * DP), rem = idx - ff * (KC * DP);
            const int t = rem / DP, j = rem - t * DP;
            cplx<T> v = mk<T>(0, 0);
            if (j < d && kc + t < d && k0 + ff < F) v = unpack<T>(ZB, nl, rows1[ff], rows2[ff], (kc + t) * d + j);
            Bs[(ff * KC + t) * (DP + 1) + j] = v;
        }
        __syncthreads();
        const cplx<T> *Af = As + f * DP * (KC + 1);
        const cplx<T> *Bf = Bs + f * KC * (DP + 1);
#pragma unroll
        for (int t = 0; t < KC; ++t) {
            cplx<T> av[TM], bv[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a) av[a] = (i0 + a < DP) ? Af[(i0 + a) * (KC + 1) + t] : mk<T>(0, 0);
#pragma unroll
            for (int b = 0; b < TN; ++b) bv[b] = (j0 + b < DP) ? Bf[t * (DP + 1) + j0 + b] : mk<T>(0, 0);
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    acc[a][b].x = fma(av[a].x, bv[b].x, fma(-av[a].y, bv[b].y, acc[a][b].x));
                    acc[a][b].y = fma(av[a].x, bv[b].y, fma(av[a].y, bv[b].x, acc[a][b].y));
                }
        }
        __syncthreads();
    }

    if ((d & 1) == 0) {
        // d even and TN even: each thread owns whole lane pairs of its rows.
        if (active) {
#pragma unroll
            for (int a = 0; a < TM; ++a) {
                const int i = i0 + a;
                if (i >= d) continue;
#pragma unroll
                for (int b = 0; b < TN; b += 2) {
                    const int j = j0 + b;
                    if (j >= d) continue;
                    pack_store<T>(ZC, nl, rows1[f], rows2[f], (i * d + j) >> 1, acc[a][b], acc[a][b + 1]);
                }
            }
        }
    } else {
        cplx<T> *Cs = As;   // [NF][d*d + 1], fits in the A and B chunk area
        const int ld = d * d + 1;
        if (active) {
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b)
                    if (i0 + a < d && j0 + b < d) Cs[f * ld + (i0 + a) * d + j0 + b] = acc[a][b];
        }
        __syncthreads();
        for (int idx = tid; idx < NF * nl; idx += NT) {
            const int ff = idx / nl, c = idx - ff * nl;
            if (k0 + ff >= F) continue;
            const int e = 2 * c;
            const cplx<T> ce = Cs[ff * ld + e];
            const cplx<T> co = (e + 1 < d * d) ? Cs[ff * ld + e + 1] : mk<T>(0, 0);
            pack_store<T>(ZC, nl, rows1[ff], rows2[ff], c, ce, co);
        }
    }
}

template <typename T, int DP>
__global__ void __launch_bounds__(SqCfg<DP>::THREADS)
freq_gemm_sq_kernel(const cplx<T> *__restrict__ ZA, const cplx<T> *__restrict__ ZB, cplx<T> *__restrict__ ZC,
                    FftPlan plan, int d) {
    freq_gemm_sq_body<T, DP>(ZA, ZB, ZC, plan, d, blockIdx.x);
}

template <typename T, int DP>
__global__ void __launch_bounds__(SqCfg<DP>::THREADS)
freq_gemm_sq_batched_kernel(const GemmProblem<T> *probs, int nprob, FftPlan plan) {
    const int64_t bid = blockIdx.x;
    const int lo = owner_of<SqCfg<DP>::THREADS>(probs, nprob, bid);
    const GemmProblem<T> &pp = probs[lo];
    freq_gemm_sq_body<T, DP>(pp.A, pp.B, pp.C, plan, pp.d, bid - pp.wg_begin);
}

// ---------------------------------------------------------------------------
// Matrix-core form of the square products (d > 8).  The complex product
// C = A B is four real products on the 16x16x4 MFMA tiles,
//     Re C = Re A Re B - Im A Im B,   Im C = Re A Im B + Im A Re B,
// accumulated in the working precision (FP64 MFMA for the FP64 path, FP32
// MFMA for the FP32 path).  The matrix is padded to DP = 16 * ceil(d / 16);
// wave w of a frequency owns the 16-row strip I = w of C (DP/16 output tiles),
// the contraction is staged through LDS in chunks of 16.
//
// Operand and accumulator layouts of the 16x16x4 instructions (lane l):
//     A[i][k] at lane i + 16 k,  B[k][j] at lane j + 16 k,
//     FP64: accumulator r holds C[l/16 + 4r][l % 16],
//     FP32: accumulator r holds C[4 (l/16) + r][l % 16].
// ---------------------------------------------------------------------------
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaOp;
template <> struct MfmaOp<double> {
    using V = mf_d4;
    __device__ static __forceinline__ V mac(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <> struct MfmaOp<float> {
    using V = mf_f4;
    __device__ static __forceinline__ V mac(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// JS (column split): two waves per 16-row strip, each owning half of the
// strip's column tiles, so a wave holds half the accumulators.  Used by the
// three-product FP64 form at d = 64, whose 3 x 4 accumulator tiles (96
// registers) would otherwise hold it at 148 registers and 3 waves per SIMD.
template <typename T, int DP, bool JS = false> struct MfCfg {
    static constexpr int WPF = DP / 16;                  // 16-row strips per frequency
    static constexpr int JSPLIT = JS ? 2 : 1;            // waves per strip
    static constexpr int WPFX = WPF * JSPLIT;            // waves per frequency
    static constexpr int JW = WPF / JSPLIT;              // 16-column tiles per wave
    static constexpr int NF = WPFX >= 3 ? 1 : 4 / WPFX;  // frequencies per workgroup
    static constexpr int THREADS = 64 * WPFX * NF;
    // Contraction chunk and register budget.  FP64 products with d > 16 take
    // 8-wide chunks (half the LDS of 16-wide ones) and a register budget of
    // 4 (d <= 32) or 3 (d <= 64) waves per SIMD, so more workgroups share a CU.
    // The column split takes 16-wide chunks (one A pair and one B pair per
    // thread) and 4 waves per SIMD: two 512-thread workgroups per CU.
    static constexpr int WAVES = JS ? 4 : (sizeof(T) == 8 && DP >= 32 ? (DP == 32 ? 4 : 3) : 1);
    static constexpr int KC = JS ? 16 : (WAVES > 1 ? 8 : 16);
    static constexpr int LDA = KC + 1;                   // As[f][i][t], i < DP, t < KC
    static constexpr int LDB = DP + 1;                   // Bs[f][t][j]
    static constexpr int AS = DP * LDA;
    static constexpr int BS = KC * LDB;
    static constexpr int NBUF = DP > KC ? 2 : 1;         // chunk buffers (double-buffered when d > 16)
};

// LDS bytes of one workgroup; odd d stages C (d*d complex per frequency).
template <typename T, int DP, bool JS = false>
static size_t mf_lds_bytes(int dmax_odd) {
    using Cfg = MfCfg<T, DP, JS>;
    const size_t ab = (size_t)Cfg::NBUF * Cfg::NF * (Cfg::AS + Cfg::BS) * sizeof(cplx<T>);
    const size_t cs = (size_t)Cfg::NF * ((size_t)dmax_odd * dmax_odd + 1) * sizeof(cplx<T>);
    return cs > ab ? cs : ab;
}

// Value of lane l ^ 1 (a DPP quad permutation, no LDS traffic).
__device__ __forceinline__ float lane_xor1(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_xor1(double x) {
    const long long u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// TA / TB: operand stored transposed (A(i, t) at entry t d + i, B(t, j) at
// entry j d + t), staged entry by entry.
template <typename T, int DP, bool G3>
__host__ __device__ constexpr bool mf_js() { return G3 && sizeof(T) == 8 && DP == 64; }

template <typename T, int DP, bool ODD, bool TA = false, bool TB = false, bool G3 = false>
__device__ __forceinline__ void freq_gemm_mfma_body(const cplx<T> *__restrict__ ZA, const cplx<T> *__restrict__ ZB,
                                                    cplx<T> *__restrict__ ZC, const FftPlan &plan, int d,
                                                    int64_t blk) {
    using Cfg = MfCfg<T, DP, mf_js<T, DP, G3>()>;
    using Op = MfmaOp<T>;
    using V = typename Op::V;
    constexpr int WPF = Cfg::WPF, WPFX = Cfg::WPFX, JW = Cfg::JW, NF = Cfg::NF, KC = Cfg::KC, NT = Cfg::THREADS;
    constexpr int LDA = Cfg::LDA, LDB = Cfg::LDB;
    // Staging work per thread and chunk: entry pairs (even d) or entries
    // (odd d) of A and of B; NT = 4 DP NF makes both counts exact.
    constexpr int PA = DP * (KC / 2), PB = KC * (DP / 2);
    constexpr int NPR = NF * PA / NT;                 // pairs of A (and of B) per thread
    constexpr int NEN = NF * DP * KC / NT;            // entries of A (and of B) per thread
    static_assert(NF * PA == NPR * NT && NF * PB == NPR * NT && NF * DP * KC == NEN * NT, "staging split");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // Chunk buffer b: A part at As + b * NF * (AS + BS), B part right after it.
    cplx<T> *As = reinterpret_cast<cplx<T> *>(smem_raw);
    constexpr int BUF = NF * (Cfg::AS + Cfg::BS);
    __shared__ int64_t rows1[NF], rows2[NF];
    const int64_t L = (int64_t)1 << plan.lgL;
    const int64_t F = L / 2 + 1;
    const int64_t k0 = blk * NF;
    const int tid = threadIdx.x;
    const int nl = (d * d + 1) >> 1;
    if (tid < NF) {
        const int64_t k = k0 + tid;
        rows1[tid] = k < F ? freq_row(plan, k) : 0;
        rows2[tid] = k < F ? freq_row(plan, (L - k) & (L - 1)) : 0;
    }
    __syncthreads();
    const int l = tid & 63, w = tid >> 6;
    const int f = w / WPFX, wr = w - f * WPFX;
    const int I = wr % WPF, J0 = (wr / WPF) * JW;   // row strip, first column tile
    constexpr bool even = !ODD;               // C entries (i, j), (i, j^1) share a packed lane
    constexpr bool pairs = !ODD && !TA && !TB; // operands staged by packed lanes
    // Four real products per complex product: accR = Re A Re B - Im A Im B,
    // accI = Re A Im B + Im A Re B.  With G3 (three real products, Gauss's
    // form of the complex product): accR = Re A Re B, accI = Im A Im B and
    // acc3 = (Re A + Im A)(Re B + Im B), combined after the contraction into
    // Re C = accR - accI and Im C = acc3 - accR - accI.
    V accR[JW], accI[JW], acc3[G3 ? JW : 1];
#pragma unroll
    for (int J = 0; J < JW; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) accR[J][r] = accI[J][r] = (T)0;
#pragma unroll
    for (int J = 0; J < (G3 ? JW : 1); ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc3[J][r] = (T)0;

    // Packed values of the current chunk in flight: rows k and L-k of the
    // lane holding each staged pair (even d) or entry (odd d).  Addresses of
    // unused slots are clamped to lane 0 of row 0, so every load is issued
    // unconditionally and the results are masked when staged.
    constexpr int NR = pairs ? NPR : NEN;
    cplx<T> xa1[NR], xa2[NR], xb1[NR], xb2[NR];
    auto fetch = [&](int kc) {
        if constexpr (pairs) {
#pragma unroll
            for (int u = 0; u < NPR; ++u) {
                const int idx = tid + u * NT;
                const int ff = idx / PA, p = idx - ff * PA;
                const int i = p / (KC / 2), t = 2 * (p - i * (KC / 2));
                const bool ok = i < d && kc + t < d;
                const int c = ok ? (i * d + kc + t) >> 1 : 0;
                xa1[u] = ZA[rows1[ff] * nl + c];
                xa2[u] = ZA[rows2[ff] * nl + c];
                const int t2 = p / (DP / 2), jb = 2 * (p - t2 * (DP / 2));
                const bool okb = jb < d && kc + t2 < d;
                const int cb = okb ? ((kc + t2) * d + jb) >> 1 : 0;
                xb1[u] = ZB[rows1[ff] * nl + cb];
                xb2[u] = ZB[rows2[ff] * nl + cb];
            }
        } else {
#pragma unroll
            for (int u = 0; u < NEN; ++u) {
                const int idx = tid + u * NT;
                const int ff = idx / (DP * KC), p = idx - ff * (DP * KC);
                const int i = p / KC, t = p - i * KC;
                const bool ok = i < d && kc + t < d;
                const int c = ok ? (TA ? (kc + t) * d + i : i * d + kc + t) >> 1 : 0;
                xa1[u] = ZA[rows1[ff] * nl + c];
                xa2[u] = ZA[rows2[ff] * nl + c];
                const int t2 = p / DP, j = p - t2 * DP;
                const bool okb = j < d && kc + t2 < d;
                const int cb = okb ? (TB ? j * d + kc + t2 : (kc + t2) * d + j) >> 1 : 0;
                xb1[u] = ZB[rows1[ff] * nl + cb];
                xb2[u] = ZB[rows2[ff] * nl + cb];
            }
        }
    };
    // Separate the two real sequences of each packed lane (Hermitian
    // symmetry) and write the chunk to LDS, zero outside the d x d block and
    // past the last frequency.
    auto stage = [&](int kc, int buf) {
        cplx<T> *Ab = As + buf * BUF;
        cplx<T> *Bb = Ab + NF * Cfg::AS;
        if constexpr (pairs) {
#pragma unroll
            for (int u = 0; u < NPR; ++u) {
                const int idx = tid + u * NT;
                const int ff = idx / PA, p = idx - ff * PA;
                const bool fok = k0 + ff < F;
                {
                    const int i = p / (KC / 2), t = 2 * (p - i * (KC / 2));
                    const bool ok = fok && i < d && kc + t < d;
                    const cplx<T> z1 = xa1[u], z2 = xa2[u];
                    const cplx<T> ev = ok ? mk<T>((z1.x + z2.x) * (T)0.5, (z1.y - z2.y) * (T)0.5) : mk<T>(0, 0);
                    const cplx<T> od = ok ? mk<T>((z1.y + z2.y) * (T)0.5, (z2.x - z1.x) * (T)0.5) : mk<T>(0, 0);
                    cplx<T> *dst = Ab + ff * Cfg::AS + i * LDA + t;
                    dst[0] = ev;
                    dst[1] = od;
                }
                {
                    const int t = p / (DP / 2), j = 2 * (p - t * (DP / 2));
                    const bool ok = fok && j < d && kc + t < d;
                    const cplx<T> z1 = xb1[u], z2 = xb2[u];
                    const cplx<T> ev = ok ? mk<T>((z1.x + z2.x) * (T)0.5, (z1.y - z2.y) * (T)0.5) : mk<T>(0, 0);
                    const cplx<T> od = ok ? mk<T>((z1.y + z2.y) * (T)0.5, (z2.x - z1.x) * (T)0.5) : mk<T>(0, 0);
                    cplx<T> *dst = Bb + ff * Cfg::BS + t * LDB + j;
                    dst[0] = ev;
                    dst[1] = od;
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < NEN; ++u) {
                const int idx = tid + u * NT;
                const int ff = idx / (DP * KC), p = idx - ff * (DP * KC);
                const bool fok = k0 + ff < F;
                {
                    const int i = p / KC, t = p - i * KC;
                    const int e = TA ? (kc + t) * d + i : i * d + kc + t;
                    const bool ok = fok && i < d && kc + t < d;
                    const cplx<T> z1 = xa1[u], z2 = xa2[u];
                    cplx<T> v = (e & 1) == 0 ? mk<T>((z1.x + z2.x) * (T)0.5, (z1.y - z2.y) * (T)0.5)
                                             : mk<T>((z1.y + z2.y) * (T)0.5, (z2.x - z1.x) * (T)0.5);
                    Ab[ff * Cfg::AS + i * LDA + t] = ok ? v : mk<T>(0, 0);
                }
                {
                    const int t = p / DP, j = p - t * DP;
                    const int e = TB ? j * d + kc + t : (kc + t) * d + j;
                    const bool ok = fok && j < d && kc + t < d;
                    const cplx<T> z1 = xb1[u], z2 = xb2[u];
                    cplx<T> v = (e & 1) == 0 ? mk<T>((z1.x + z2.x) * (T)0.5, (z1.y - z2.y) * (T)0.5)
                                             : mk<T>((z1.y + z2.y) * (T)0.5, (z2.x - z1.x) * (T)0.5);
                    Bb[ff * Cfg::BS + t * LDB + j] = ok ? v : mk<T>(0, 0);
                }
            }
        }
    };

    // Chunk kc is read from buffer b while chunk kc + KC is fetched and
    // staged into the other buffer; one barrier per chunk.
    fetch(0);
    stage(0, 0);
    __syncthreads();
    int cur = 0;
    for (int kc = 0; kc < d; kc += KC) {
        const bool more = kc + KC < d;   // only when d > KC, i.e. NBUF == 2
        if (more) fetch(kc + KC);
        const cplx<T> *Af = As + cur * BUF + f * Cfg::AS + (I * 16 + (l & 15)) * LDA;
        const cplx<T> *Bf = As + cur * BUF + NF * Cfg::AS + f * Cfg::BS + (l & 15);
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            const int t = 4 * ks + (l >> 4);
            const cplx<T> a = Af[t];
            if constexpr (G3) {
                const T as = a.x + a.y;
#pragma unroll
                for (int J = 0; J < JW; ++J) {
                    const cplx<T> b = Bf[t * LDB + (J0 + J) * 16];
                    accR[J] = Op::mac(a.x, b.x, accR[J]);
                    accI[J] = Op::mac(a.y, b.y, accI[J]);
                    acc3[J] = Op::mac(as, b.x + b.y, acc3[J]);
                }
            } else {
#pragma unroll
                for (int J = 0; J < JW; ++J) {
                    const cplx<T> b = Bf[t * LDB + (J0 + J) * 16];
                    accR[J] = Op::mac(a.x, b.x, accR[J]);
                    accR[J] = Op::mac(-a.y, b.y, accR[J]);
                    accI[J] = Op::mac(a.x, b.y, accI[J]);
                    accI[J] = Op::mac(a.y, b.x, accI[J]);
                }
            }
        }
        if (more) stage(kc + KC, cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
    if constexpr (G3) {
#pragma unroll
        for (int J = 0; J < JW; ++J)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const T p1 = accR[J][r], p2 = accI[J][r];
                accR[J][r] = p1 - p2;
                accI[J][r] = acc3[J][r] - p1 - p2;
            }
    }

    const bool fok = k0 + f < F;
    if constexpr (even) {
        // Entries (i, j) and (i, j^1) sit in lanes l and l^1 of the same
        // accumulator element: the even lane writes row k, the odd lane row L-k.
        const int64_t r1 = rows1[f], r2 = rows2[f];
        const bool odd_lane = (l & 1) != 0;
#pragma unroll
        for (int J = 0; J < JW; ++J) {
            const int j = (J0 + J) * 16 + (l & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = I * 16 + Op::row(l, r);
                const T vr = accR[J][r], vi = accI[J][r];
                const T pr = lane_xor1(vr), pi = lane_xor1(vi);
                if (fok && i < d && j < d) {
                    const int c = (i * d + (j & ~1)) >> 1;
                    if (!odd_lane) ZC[r1 * nl + c] = mk<T>(vr - pi, vi + pr);
                    else if (r2 != r1) ZC[r2 * nl + c] = mk<T>(pr + vi, vr - pi);
                }
            }
        }
    } else {
        cplx<T> *Cs = As;   // [NF][d*d + 1]
        const int ld = d * d + 1;
#pragma unroll
        for (int J = 0; J < JW; ++J) {
            const int j = (J0 + J) * 16 + (l & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = I * 16 + Op::row(l, r);
                if (i < d && j < d) Cs[f * ld + i * d + j] = mk<T>(accR[J][r], accI[J][r]);
            }
        }
        __syncthreads();
        for (int idx = tid; idx < NF * nl; idx += NT) {
            const int ff = idx / nl, c = idx - ff * nl;
            if (k0 + ff >= F) continue;
            const int e = 2 * c;
            const cplx<T> ce = Cs[ff * ld + e];
            const cplx<T> co = (e + 1 < d * d) ? Cs[ff * ld + e + 1] : mk<T>(0, 0);
            pack_store<T>(ZC, nl, rows1[ff], rows2[ff], c, ce, co);
        }
    }
}

// Streamed form of the even-d, untransposed product with one frequency per
// workgroup (padded d >= 48): a grid of resident workgroups walks the
// frequencies k = blockIdx.x, blockIdx.x + gridDim.x, ... < F.  While a
// workgroup multiplies the last contraction chunk of frequency k it loads and
// stages the first chunk of its next frequency, so neither its first loads
// nor its epilogue stores leave the matrix cores and the memory idle.  The
// arithmetic per frequency is that of freq_gemm_mfma_body (same chunks, same
// order, same bits).
template <typename T, int DP, bool G3>
__device__ __forceinline__ void freq_gemm_mfma_stream_body(const cplx<T> *__restrict__ ZA,
                                                           const cplx<T> *__restrict__ ZB, cplx<T> *__restrict__ ZC,
                                                           const FftPlan &plan, int d) {
    using Cfg = MfCfg<T, DP, mf_js<T, DP, G3>()>;
    using Op = MfmaOp<T>;
    using V = typename Op::V;
    static_assert(Cfg::NF == 1 && Cfg::NBUF == 2, "one frequency per workgroup, double-buffered chunks");
    constexpr int WPF = Cfg::WPF, JW = Cfg::JW, KC = Cfg::KC, NT = Cfg::THREADS;
    constexpr int LDA = Cfg::LDA, LDB = Cfg::LDB;
    constexpr int PA = DP * (KC / 2), PB = KC * (DP / 2);
    constexpr int NPR = PA / NT;                      // pairs of A (and of B) per thread
    static_assert(PA == NPR * NT && PB == NPR * NT, "staging split");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *As = reinterpret_cast<cplx<T> *>(smem_raw);
    constexpr int BUF = Cfg::AS + Cfg::BS;
    const int64_t L = (int64_t)1 << plan.lgL;
    const int64_t F = L / 2 + 1;
    const int tid = threadIdx.x;
    const int nl = (d * d + 1) >> 1;
    const int l = tid & 63, w = tid >> 6;
    const int I = w % WPF, J0 = (w / WPF) * JW;      // row strip, first column tile

    cplx<T> xa1[NPR], xa2[NPR], xb1[NPR], xb2[NPR];
    // Packed values of chunk kc of the frequency in rows r1 (k) and r2 (L-k);
    // addresses of entries outside the d x d block are clamped to lane 0.
    auto fetch = [&](int64_t r1, int64_t r2, int kc) {
#pragma unroll
        for (int u = 0; u < NPR; ++u) {
            const int p = tid + u * NT;
            const int i = p / (KC / 2), t = 2 * (p - i * (KC / 2));
            const int c = (i < d && kc + t < d) ? (i * d + kc + t) >> 1 : 0;
            xa1[u] = ZA[r1 * nl + c];
            xa2[u] = ZA[r2 * nl + c];
            const int t2 = p / (DP / 2), jb = 2 * (p - t2 * (DP / 2));
            const int cb = (jb < d && kc + t2 < d) ? ((kc + t2) * d + jb) >> 1 : 0;
            xb1[u] = ZB[r1 * nl + cb];
            xb2[u] = ZB[r2 * nl + cb];
        }
    };
    // Separate the two real sequences of each packed lane and write the
    // chunk to LDS buffer buf, zero outside the d x d block.
    auto stage = [&](int kc, int buf) {
        cplx<T> *Ab = As + buf * BUF;
        cplx<T> *Bb = Ab + Cfg::AS;
#pragma unroll
        for (int u = 0; u < NPR; ++u) {
            const int p = tid + u * NT;
            {
                const int i = p / (KC / 2), t = 2 * (p - i * (KC / 2));
                const bool ok = i < d && kc + t < d;
                const cplx<T> z1 = xa1[u], z2 = xa2[u];
                const cplx<T> ev = ok ? mk<T>((z1.x + z2.x) * (T)0.5, (z1.y - z2.y) * (T)0.5) : mk<T>(0, 0);
                const cplx<T> od = ok ? mk<T>((z1.y + z2.y) * (T)0.5, (z2.x - z1.x) * (T)0.5) : mk<T>(0, 0);
                cplx<T> *dst = Ab + i * LDA + t;
                dst[0] = ev;
                dst[1] = od;
            }
            {
                const int t = p / (DP / 2), j = 2 * (p - t * (DP / 2));
                const bool ok = j < d && kc + t < d;
                const cplx<T> z1 = xb1[u], z2 = xb2[u];
                const cplx<T> ev = ok ? mk<T>((z1.x + z2.x) * (T)0.5, (z1.y - z2.y) * (T)0.5) : mk<T>(0, 0);
                const cplx<T> od = ok ? mk<T>((z1.y + z2.y) * (T)0.5, (z2.x - z1.x) * (T)0.5) : mk<T>(0, 0);
                cplx<T> *dst = Bb + t * LDB + j;
                dst[0] = ev;
                dst[1] = od;
            }
        }
    };

    int64_t k = blockIdx.x;
    if (k >= F) return;                               // the whole workgroup leaves together
    int64_t r1 = freq_row(plan, k), r2 = freq_row(plan, (L - k) & (L - 1));
    fetch(r1, r2, 0);
    stage(0, 0);
    __syncthreads();
    int cur = 0;
    for (;;) {
        const int64_t kn = k + gridDim.x;
        const bool next = kn < F;
        const int64_t n1 = next ? freq_row(plan, kn) : 0, n2 = next ? freq_row(plan, (L - kn) & (L - 1)) : 0;
        V accR[JW], accI[JW], acc3[G3 ? JW : 1];
#pragma unroll
        for (int J = 0; J < JW; ++J)
#pragma unroll
            for (int r = 0; r < 4; ++r) accR[J][r] = accI[J][r] = (T)0;
#pragma unroll
        for (int J = 0; J < (G3 ? JW : 1); ++J)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc3[J][r] = (T)0;
        // Chunk kc is read from buffer cur while the following chunk (the
        // next frequency's first after the last) is fetched and staged into
        // the other buffer; one barrier per chunk.
        for (int kc = 0; kc < d; kc += KC) {
            const bool more = kc + KC < d;
            if (more) fetch(r1, r2, kc + KC);
            else if (next) fetch(n1, n2, 0);
            const cplx<T> *Af = As + cur * BUF + (I * 16 + (l & 15)) * LDA;
            const cplx<T> *Bf = As + cur * BUF + Cfg::AS + (l & 15);
#pragma unroll
            for (int ks = 0; ks < KC / 4; ++ks) {
                const int t = 4 * ks + (l >> 4);
                const cplx<T> a = Af[t];
                if constexpr (G3) {
                    const T as = a.x + a.y;
#pragma unroll
                    for (int J = 0; J < JW; ++J) {
                        const cplx<T> b = Bf[t * LDB + (J0 + J) * 16];
                        accR[J] = Op::mac(a.x, b.x, accR[J]);
                        accI[J] = Op::mac(a.y, b.y, accI[J]);
                        acc3[J] = Op::mac(as, b.x + b.y, acc3[J]);
                    }
                } else {
#pragma unroll
                    for (int J = 0; J < JW; ++J) {
                        const cplx<T> b = Bf[t * LDB + (J0 + J) * 16];
                        accR[J] = Op::mac(a.x, b.x, accR[J]);
                        accR[J] = Op::mac(-a.y, b.y, accR[J]);
                        accI[J] = Op::mac(a.x, b.y, accI[J]);
                        accI[J] = Op::mac(a.y, b.x, accI[J]);
                    }
                }
            }
            if (more) stage(kc + KC, cur ^ 1);
            else if (next) stage(0, cur ^ 1);
            __syncthreads();
            cur ^= 1;
        }
        if constexpr (G3) {
#pragma unroll
            for (int J = 0; J < JW; ++J)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const T p1 = accR[J][r], p2 = accI[J][r];
                    accR[J][r] = p1 - p2;
                    accI[J][r] = acc3[J][r] - p1 - p2;
                }
        }
        // Entries (i, j) and (i, j^1) sit in lanes l and l^1 of the same
        // accumulator element: the even lane writes row k, the odd lane row L-k.
        const bool odd_lane = (l & 1) != 0;
#pragma unroll
        for (int J = 0; J < JW; ++J) {
            const int j = (J0 + J) * 16 + (l & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = I * 16 + Op::row(l, r);
                const T vr = accR[J][r], vi = accI[J][r];
                const T pr = lane_xor1(vr), pi = lane_xor1(vi);
                if (i < d && j < d) {
                    const int c = (i * d + (j & ~1)) >> 1;
                    if (!odd_lane) ZC[r1 * nl + c] = mk<T>(vr - pi, vi + pr);
                    else if (r2 != r1) ZC[r2 * nl + c] = mk<T>(pr + vi, vr - pi);
                }
            }
        }
        if (!next) break;
        k = kn;
        r1 = n1;
        r2 = n2;
    }
}

template <typename T, int DP, bool G3>
__global__ void __launch_bounds__((MfCfg<T, DP, mf_js<T, DP, G3>()>::THREADS))
__attribute__((amdgpu_waves_per_eu(MfCfg<T, DP, mf_js<T, DP, G3>()>::WAVES)))
freq_gemm_mfma_stream_kernel(const cplx<T> *__restrict__ ZA, const cplx<T> *__restrict__ ZB,
                             cplx<T> *__restrict__ ZC, FftPlan plan, int d) {
    freq_gemm_mfma_stream_body<T, DP, G3>(ZA, ZB, ZC, plan, d);
}

// Streamed products (freq_gemm_mfma_stream_body) are used for the
// column-split FP64 d = 64 product only: there the streamed kernel keeps its
// two workgroups per CU (120 registers) and is 2-3% faster per C3 inversion
// (20.9-21.4 against 21.7-21.8 ms, alternating runs on one GPU).  The FP32
// d = 64 product grows from 60 to 132 registers when streamed, halves its
// resident workgroups and slows down by 9%, so it stays one frequency per
// workgroup.
constexpr bool MF_STREAM = true;

// Workgroups of `kern` resident on the current device at once (occupancy per
// CU times the CU count), queried once per kernel and device.
static int64_t resident_workgroups(const void *kern, int threads, size_t lds) {
    struct Entry { const void *k; int dev; int64_t n; };
    static Entry cache[64];
    static int used = 0;
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < used; ++i)
        if (cache[i].k == kern && cache[i].dev == dev) return cache[i].n;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int64_t n = (int64_t)per_cu * cus;
    if (used < 64) cache[used++] = Entry{kern, dev, n};
    return n;
}

template <typename T, int DP, bool ODD, bool TA, bool TB, bool G3>
__global__ void __launch_bounds__((MfCfg<T, DP, mf_js<T, DP, G3>()>::THREADS))
__attribute__((amdgpu_waves_per_eu(MfCfg<T, DP, mf_js<T, DP, G3>()>::WAVES)))
freq_gemm_mfma_kernel(const cplx<T> *__restrict__ ZA, const cplx<T> *__restrict__ ZB, cplx<T> *__restrict__ ZC,
                      FftPlan plan, int d) {
    freq_gemm_mfma_body<T, DP, ODD, TA, TB, G3>(ZA, ZB, ZC, plan, d, blockIdx.x);
}

template <typename T, int DP, bool ODD, bool G3>
__global__ void __launch_bounds__((MfCfg<T, DP, mf_js<T, DP, G3>()>::THREADS))
__attribute__((amdgpu_waves_per_eu(MfCfg<T, DP, mf_js<T, DP, G3>()>::WAVES)))
freq_gemm_mfma_batched_kernel(const GemmProblem<T> *probs, int nprob, FftPlan plan) {
    const int64_t bid = blockIdx.x;
    const int lo = owner_of<MfCfg<T, DP, mf_js<T, DP, G3>()>::THREADS>(probs, nprob, bid);
    const GemmProblem<T> &pp = probs[lo];
    freq_gemm_mfma_body<T, DP, ODD, false, false, G3>(pp.A, pp.B, pp.C, plan, pp.d, bid - pp.wg_begin);
}

template <typename T, int DP, bool ODD, bool TA = false, bool TB = false, bool G3 = false>
static hipError_t launch_gemm_mfma_t(const FftPlan &plan, int d, const cplx<T> *ZA, const cplx<T> *ZB, cplx<T> *ZC,
                                     hipStream_t st) {
    using Cfg = MfCfg<T, DP, mf_js<T, DP, G3>()>;
    const size_t lds = mf_lds_bytes<T, DP, mf_js<T, DP, G3>()>(ODD ? d : 0);
    const int64_t F = ((int64_t)1 << plan.lgL) / 2 + 1;
    const double Lr = (double)((int64_t)1 << plan.lgL);
    const int nl = (d * d + 1) / 2;
    if constexpr (MF_STREAM && !ODD && !TA && !TB && mf_js<T, DP, G3>()) {
        auto skern = freq_gemm_mfma_stream_kernel<T, DP, G3>;
        if (lds > 64 * 1024) {
            (void)hipFuncSetAttribute((const void *)skern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            (void)hipGetLastError();
        }
        const int64_t res = resident_workgroups((const void *)skern, Cfg::THREADS, lds);
        if (res > 0) {
            const int64_t blocks = std::min<int64_t>(F, res);
            char name[96];
            snprintf(name, sizeof name, "freq_gemm_mfma_stream_kernel<%s, %d, %s>",
                     sizeof(T) == 8 ? "double" : "float", DP, G3 ? "true" : "false");
            launch_kernel(name, Lr * 3.0 * nl * sizeof(cplx<T>), (double)F * 8.0 * d * d * d, skern,
                          dim3((unsigned)blocks), dim3(Cfg::THREADS), lds, st, ZA, ZB, ZC, plan, d);
            return hipGetLastError();
        }
    }
    auto kern = freq_gemm_mfma_kernel<T, DP, ODD, TA, TB, G3>;
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    }
    const int64_t blocks = (F + Cfg::NF - 1) / Cfg::NF;
    char name[96];
    snprintf(name, sizeof name, "freq_gemm_mfma_kernel<%s, %d, %s, %s, %s, %s>", sizeof(T) == 8 ? "double" : "float",
             DP, ODD ? "true" : "false", TA ? "true" : "false", TB ? "true" : "false", G3 ? "true" : "false");
    launch_kernel(name, Lr * 3.0 * nl * sizeof(cplx<T>), (double)F * 8.0 * d * d * d,
                  kern, dim3((unsigned)blocks), dim3(Cfg::THREADS), lds, st, ZA, ZB, ZC, plan, d);
    return hipGetLastError();
}

// Three real products per complex product (Gauss's form) where the matrix
// cores bound the product (padded d >= 48: intensity d/6 flop/B in FP64, near
// or above the ridge); mfma == 2 keeps the four-product form everywhere.
template <int DP> static bool use_g3(int mfma) { return mfma == 1 && DP >= 48; }

// ---------------------------------------------------------------------------
// Split-BF16 form of the float square products (precision MRINV_MIXED_BF16X3):
// every float operand entry x is held as hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (about 16 significant bits together), and a real product
// is hi*hi + hi*lo + lo*hi on the 16x16x32 BF16 matrix cores with FP32
// accumulation (the lo*lo term, about 2^-16 relative, is dropped).  The
// complex product takes four real products, so one 16x16 output tile and one
// 32-wide contraction chunk cost 12 BF16 MFMAs.
//
// Operand layout of the 16x16x32 instruction (lane l): A[i][k] for i = l % 16,
// k = 8 (l / 16) + 0..7, eight values of a row; B[k][j] for j = l % 16 and the
// same k; the FP32 accumulator holds C[4 (l / 16) + r][l % 16] like the
// 16x16x4 FP32 form, so the packing epilogue is shared.
// LDS: per frequency and operand, four planes (re hi, im hi, re lo, im lo) of
// DP rows x 32 contraction entries (B stored transposed, [j][k]), rows padded
// to 40 entries (80 bytes) so the 16-byte row reads of a wave spread over the
// banks.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

template <int DP> struct BfCfg {
    static constexpr int WPF = DP / 16;
    static constexpr int NF = WPF >= 3 ? 1 : 4 / WPF;
    static constexpr int THREADS = 64 * WPF * NF;
    static constexpr int KC = 32;
    static constexpr int LDK = 40;
    static constexpr int PLANE = DP * LDK;            // bf16 entries of one plane
};

template <int DP>
static size_t bf3_lds_bytes(int dmax_odd) {
    using Cfg = BfCfg<DP>;
    const size_t ab = (size_t)Cfg::NF * 2 * 4 * Cfg::PLANE * sizeof(__bf16);
    const size_t cs = (size_t)Cfg::NF * ((size_t)dmax_odd * dmax_odd + 1) * sizeof(float2);
    return cs > ab ? cs : ab;
}

__device__ __forceinline__ void bf3_put(__bf16 *pl, int plane, int off, float2 v) {
    const __bf16 rh = (__bf16)v.x, ih = (__bf16)v.y;
    pl[off] = rh;
    pl[plane + off] = ih;
    pl[2 * plane + off] = (__bf16)(v.x - (float)rh);
    pl[3 * plane + off] = (__bf16)(v.y - (float)ih);
}

template <int DP, bool ODD>
__device__ __forceinline__ void freq_gemm_bf3_body(const float2 *__restrict__ ZA, const float2 *__restrict__ ZB,
                                                   float2 *__restrict__ ZC, const FftPlan &plan, int d, int64_t blk) {
    using Cfg = BfCfg<DP>;
    using V = mf_f4;
    constexpr int WPF = Cfg::WPF, NF = Cfg::NF, KC = Cfg::KC, NT = Cfg::THREADS, LDK = Cfg::LDK;
    constexpr int PL = Cfg::PLANE;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __bf16 *S = reinterpret_cast<__bf16 *>(smem_raw);     // [NF][operand A, B][4 planes][DP][LDK]
    __shared__ int64_t rows1[NF], rows2[NF];
    const int64_t L = (int64_t)1 << plan.lgL;
    const int64_t F = L / 2 + 1;
    const int64_t k0 = blk * NF;
    const int tid = threadIdx.x;
    const int nl = (d * d + 1) >> 1;
    if (tid < NF) {
        const int64_t k = k0 + tid;
        rows1[tid] = k < F ? freq_row(plan, k) : 0;
        rows2[tid] = k < F ? freq_row(plan, (L - k) & (L - 1)) : 0;
    }
    __syncthreads();
    const int l = tid & 63, w = tid >> 6;
    const int f = w / WPF, I = w - f * WPF;
    V accR[WPF], accI[WPF];
#pragma unroll
    for (int J = 0; J < WPF; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) accR[J][r] = accI[J][r] = 0.f;
    auto base = [&](int ff, int op) { return S + (size_t)(ff * 2 + op) * 4 * PL; };

    for (int kc = 0; kc < d; kc += KC) {
        // Stage the chunk: A entries (i, t) at [i][t], B entries (t, j) at [j][t],
        // separated from the packed lanes by the Hermitian symmetry and split.
        if constexpr (!ODD) {
            // Even d: a packed lane holds an aligned entry pair of one row.
            for (int idx = tid; idx < NF * DP * (KC / 2); idx += NT) {
                const int ff = idx / (DP * (KC / 2)), p = idx - ff * (DP * (KC / 2));
                const bool fok = k0 + ff < F;
                {
                    const int i = p / (KC / 2), t = 2 * (p - i * (KC / 2));
                    const bool ok = fok && i < d && kc + t < d;
                    const int c = ok ? (i * d + kc + t) >> 1 : 0;
                    const float2 z1 = ZA[rows1[ff] * nl + c], z2 = ZA[rows2[ff] * nl + c];
                    const float2 ev = ok ? make_float2((z1.x + z2.x) * 0.5f, (z1.y - z2.y) * 0.5f) : make_float2(0.f, 0.f);
                    const float2 od = ok ? make_float2((z1.y + z2.y) * 0.5f, (z2.x - z1.x) * 0.5f) : make_float2(0.f, 0.f);
                    __bf16 *a = base(ff, 0);
                    bf3_put(a, PL, i * LDK + t, ev);
                    bf3_put(a, PL, i * LDK + t + 1, od);
                }
                {
                    const int t = p / (DP / 2), j = 2 * (p - t * (DP / 2));
                    const bool ok = fok && j < d && kc + t < d;
                    const int c = ok ? ((kc + t) * d + j) >> 1 : 0;
                    const float2 z1 = ZB[rows1[ff] * nl + c], z2 = ZB[rows2[ff] * nl + c];
                    const float2 ev = ok ? make_float2((z1.x + z2.x) * 0.5f, (z1.y - z2.y) * 0.5f) : make_float2(0.f, 0.f);
                    const float2 od = ok ? make_float2((z1.y + z2.y) * 0.5f, (z2.x - z1.x) * 0.5f) : make_float2(0.f, 0.f);
                    __bf16 *b = base(ff, 1);
                    bf3_put(b, PL, j * LDK + t, ev);
                    bf3_put(b, PL, (j + 1) * LDK + t, od);
                }
            }
        } else {
            for (int idx = tid; idx < NF * DP * KC; idx += NT) {
                const int ff = idx / (DP * KC), p = idx - ff * (DP * KC);
                const bool fok = k0 + ff < F;
                {
                    const int i = p / KC, t = p - i * KC;
                    const bool ok = fok && i < d && kc + t < d;
                    const float2 v = ok ? unpack<float>(ZA, nl, rows1[ff], rows2[ff], i * d + kc + t) : make_float2(0.f, 0.f);
                    bf3_put(base(ff, 0), PL, i * LDK + t, v);
                }
                {
                    const int j = p / KC, t = p - j * KC;
                    const bool ok = fok && j < d && kc + t < d;
                    const float2 v = ok ? unpack<float>(ZB, nl, rows1[ff], rows2[ff], (kc + t) * d + j) : make_float2(0.f, 0.f);
                    bf3_put(base(ff, 1), PL, j * LDK + t, v);
                }
            }
        }
        __syncthreads();
        {
            const __bf16 *Ab = base(f, 0) + (I * 16 + (l & 15)) * LDK + 8 * (l >> 4);
            const bf16x8_t arh = *(const bf16x8_t *)(Ab);
            const bf16x8_t aih = *(const bf16x8_t *)(Ab + PL);
            const bf16x8_t arl = *(const bf16x8_t *)(Ab + 2 * PL);
            const bf16x8_t ail = *(const bf16x8_t *)(Ab + 3 * PL);
            const bf16x8_t naih = -aih, nail = -ail;
#pragma unroll
            for (int J = 0; J < WPF; ++J) {
                const __bf16 *Bb = base(f, 1) + (J * 16 + (l & 15)) * LDK + 8 * (l >> 4);
                const bf16x8_t brh = *(const bf16x8_t *)(Bb);
                const bf16x8_t bih = *(const bf16x8_t *)(Bb + PL);
                const bf16x8_t brl = *(const bf16x8_t *)(Bb + 2 * PL);
                const bf16x8_t bil = *(const bf16x8_t *)(Bb + 3 * PL);
                // Re C += Re A Re B - Im A Im B,  Im C += Re A Im B + Im A Re B
                accR[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, brh, accR[J], 0, 0, 0);
                accR[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, brl, accR[J], 0, 0, 0);
                accR[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, brh, accR[J], 0, 0, 0);
                accR[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(naih, bih, accR[J], 0, 0, 0);
                accR[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(naih, bil, accR[J], 0, 0, 0);
                accR[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nail, bih, accR[J], 0, 0, 0);
                accI[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bih, accI[J], 0, 0, 0);
                accI[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bil, accI[J], 0, 0, 0);
                accI[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, bih, accI[J], 0, 0, 0);
                accI[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, brh, accI[J], 0, 0, 0);
                accI[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, brl, accI[J], 0, 0, 0);
                accI[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, brh, accI[J], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    const bool fok = k0 + f < F;
    if constexpr (!ODD) {
        const int64_t r1 = rows1[f], r2 = rows2[f];
        const bool odd_lane = (l & 1) != 0;
#pragma unroll
        for (int J = 0; J < WPF; ++J) {
            const int j = J * 16 + (l & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = I * 16 + 4 * (l >> 4) + r;
                const float vr = accR[J][r], vi = accI[J][r];
                const float pr = lane_xor1(vr), pi = lane_xor1(vi);
                if (fok && i < d && j < d) {
                    const int c = (i * d + (j & ~1)) >> 1;
                    if (!odd_lane) ZC[r1 * nl + c] = make_float2(vr - pi, vi + pr);
                    else if (r2 != r1) ZC[r2 * nl + c] = make_float2(pr + vi, vr - pi);
                }
            }
        }
    } else {
        float2 *Cs = reinterpret_cast<float2 *>(smem_raw);   // [NF][d*d + 1]
        const int ld = d * d + 1;
#pragma unroll
        for (int J = 0; J < WPF; ++J) {
            const int j = J * 16 + (l & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = I * 16 + 4 * (l >> 4) + r;
                if (i < d && j < d) Cs[f * ld + i * d + j] = make_float2(accR[J][r], accI[J][r]);
            }
        }
        __syncthreads();
        for (int idx = tid; idx < NF * nl; idx += NT) {
            const int ff = idx / nl, c = idx - ff * nl;
            if (k0 + ff >= F) continue;
            const int e = 2 * c;
            const float2 ce = Cs[ff * ld + e];
            const float2 co = (e + 1 < d * d) ? Cs[ff * ld + e + 1] : make_float2(0.f, 0.f);
            pack_store<float>(ZC, nl, rows1[ff], rows2[ff], c, ce, co);
        }
    }
}

template <int DP, bool ODD>
__global__ void __launch_bounds__(BfCfg<DP>::THREADS)
freq_gemm_bf3_kernel(const float2 *__restrict__ ZA, const float2 *__restrict__ ZB, float2 *__restrict__ ZC,
                     FftPlan plan, int d) {
    freq_gemm_bf3_body<DP, ODD>(ZA, ZB, ZC, plan, d, blockIdx.x);
}

template <int DP, bool ODD>
__global__ void __launch_bounds__(BfCfg<DP>::THREADS)
freq_gemm_bf3_batched_kernel(const GemmProblem<float> *probs, int nprob, FftPlan plan) {
    const int64_t bid = blockIdx.x;
    const int lo = owner_of<BfCfg<DP>::THREADS>(probs, nprob, bid);
    const GemmProblem<float> &pp = probs[lo];
    freq_gemm_bf3_body<DP, ODD>(pp.A, pp.B, pp.C, plan, pp.d, bid - pp.wg_begin);
}

template <int DP, bool ODD>
static hipError_t launch_gemm_bf3(const FftPlan &plan, int d, const float2 *ZA, const float2 *ZB, float2 *ZC,
                                  hipStream_t st) {
    using Cfg = BfCfg<DP>;
    const size_t lds = bf3_lds_bytes<DP>(ODD ? d : 0);
    auto kern = freq_gemm_bf3_kernel<DP, ODD>;
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    }
    const int64_t F = ((int64_t)1 << plan.lgL) / 2 + 1;
    const int64_t blocks = (F + Cfg::NF - 1) / Cfg::NF;
    char name[96];
    snprintf(name, sizeof name, "freq_gemm_bf3_kernel<%d, %s>", DP, ODD ? "true" : "false");
    const double Lr = (double)((int64_t)1 << plan.lgL);
    const int nl = (d * d + 1) / 2;
    launch_kernel(name, Lr * 3.0 * nl * sizeof(float2), (double)F * 8.0 * d * d * d, kern, dim3((unsigned)blocks),
                  dim3(Cfg::THREADS), lds, st, ZA, ZB, ZC, plan, d);
    return hipGetLastError();
}

template <int DP, bool ODD>
static hipError_t launch_gemm_bf3_batched(const FftPlan &plan, const GemmProblem<float> *probs, int nprob,
                                          int64_t total, double bytes, double flops, hipStream_t st) {
    using Cfg = BfCfg<DP>;
    const size_t lds = bf3_lds_bytes<DP>(ODD ? DP - 1 : 0);
    auto kern = freq_gemm_bf3_batched_kernel<DP, ODD>;
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    }
    char name[96];
    snprintf(name, sizeof name, "freq_gemm_bf3_batched_kernel<%d, %s>", DP, ODD ? "true" : "false");
    launch_kernel(name, bytes, flops, kern, dim3((unsigned)total), dim3(Cfg::THREADS), lds, st, probs, nprob, plan);
    return hipGetLastError();
}

// Square split-BF16 product of matrix-core class cls (9..16, see gemm_sq_class).
static hipError_t gemm_bf3(const FftPlan &plan, int cls, int d, const float2 *ZA, const float2 *ZB, float2 *ZC,
                           hipStream_t st) {
    switch (cls) {
        case 9: return launch_gemm_bf3<16, false>(plan, d, ZA, ZB, ZC, st);
        case 10: return launch_gemm_bf3<32, false>(plan, d, ZA, ZB, ZC, st);
        case 11: return launch_gemm_bf3<48, false>(plan, d, ZA, ZB, ZC, st);
        case 12: return launch_gemm_bf3<64, false>(plan, d, ZA, ZB, ZC, st);
        case 13: return launch_gemm_bf3<16, true>(plan, d, ZA, ZB, ZC, st);
        case 14: return launch_gemm_bf3<32, true>(plan, d, ZA, ZB, ZC, st);
        case 15: return launch_gemm_bf3<48, true>(plan, d, ZA, ZB, ZC, st);
        default: return launch_gemm_bf3<64, true>(plan, d, ZA, ZB, ZC, st);
    }
}

static hipError_t gemm_bf3_batched(const FftPlan &plan, int cls, const GemmProblem<float> *probs, int nprob,
                                   int64_t total, double bytes, double flops, hipStream_t st) {
    switch (cls) {
        case 9: return launch_gemm_bf3_batched<16, false>(plan, probs, nprob, total, bytes, flops, st);
        case 10: return launch_gemm_bf3_batched<32, false>(plan, probs, nprob, total, bytes, flops, st);
        case 11: return launch_gemm_bf3_batched<48, false>(plan, probs, nprob, total, bytes, flops, st);
        case 12: return launch_gemm_bf3_batched<64, false>(plan, probs, nprob, total, bytes, flops, st);
        case 13: return launch_gemm_bf3_batched<16, true>(plan, probs, nprob, total, bytes, flops, st);
        case 14: return launch_gemm_bf3_batched<32, true>(plan, probs, nprob, total, bytes, flops, st);
        case 15: return launch_gemm_bf3_batched<48, true>(plan, probs, nprob, total, bytes, flops, st);
        default: return launch_gemm_bf3_batched<64, true>(plan, probs, nprob, total, bytes, flops, st);
    }
}

template <typename T, int DP, bool ODD, bool TA = false, bool TB = false>
static hipError_t launch_gemm_mfma(const FftPlan &plan, int d, int mfma, const cplx<T> *ZA, const cplx<T> *ZB,
                                   cplx<T> *ZC, hipStream_t st) {
    if (use_g3<DP>(mfma)) return launch_gemm_mfma_t<T, DP, ODD, TA, TB, true>(plan, d, ZA, ZB, ZC, st);
    return launch_gemm_mfma_t<T, DP, ODD, TA, TB, false>(plan, d, ZA, ZB, ZC, st);
}

template <typename T, int DP, bool ODD, bool G3>
static hipError_t launch_gemm_mfma_batched_t(const FftPlan &plan, const GemmProblem<T> *probs, int nprob,
                                             int64_t total, double bytes, double flops, hipStream_t st) {
    using Cfg = MfCfg<T, DP, mf_js<T, DP, G3>()>;
    const size_t lds = mf_lds_bytes<T, DP, mf_js<T, DP, G3>()>(ODD ? DP - 1 : 0);
    auto kern = freq_gemm_mfma_batched_kernel<T, DP, ODD, G3>;
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    }
    char name[96];
    snprintf(name, sizeof name, "freq_gemm_mfma_batched_kernel<%s, %d, %s, %s>", sizeof(T) == 8 ? "double" : "float",
             DP, ODD ? "true" : "false", G3 ? "true" : "false");
    launch_kernel(name, bytes, flops,
                  kern, dim3((unsigned)total), dim3(Cfg::THREADS), lds, st, probs, nprob, plan);
    return hipGetLastError();
}

template <typename T, int DP, bool ODD>
static hipError_t launch_gemm_mfma_batched(const FftPlan &plan, int mfma, const GemmProblem<T> *probs, int nprob,
                                           int64_t total, double bytes, double flops, hipStream_t st) {
    if (use_g3<DP>(mfma)) return launch_gemm_mfma_batched_t<T, DP, ODD, true>(plan, probs, nprob, total, bytes, flops, st);
    return launch_gemm_mfma_batched_t<T, DP, ODD, false>(plan, probs, nprob, total, bytes, flops, st);
}

// ---------------------------------------------------------------------------
// Direct truncated products of the first Newton steps (the definition of the
// product in the truncated ring, Section 2.1, without transforms): for small m
// the 1.5 m^2 d^3 multiply-adds of a step cost less than the latency of the
// transform launches.  One workgroup per (k, 16x16 output tile); its CONV_WAVES
// waves take every CONV_WAVES-th j and their tiles are summed through LDS.
// ---------------------------------------------------------------------------
constexpr int CONV_WAVES = 16;
constexpr int CONV_THREADS = 64 * CONV_WAVES;

template <typename T, typename TL, int DP>
__device__ __forceinline__ void conv_direct_body(const ConvDesc &c, int64_t blk) {
    using Op = MfmaOp<T>;
    using V = typename Op::V;
    constexpr int NT = DP / 16;
    const int64_t k = c.k0 + blk / (NT * NT);
    const int tile = (int)(blk % (NT * NT));
    const int I = tile / NT, J = tile - I * NT;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int d = c.d;
    const int64_t dd = (int64_t)d * d;
    const int64_t jhi = c.jhi < k ? c.jhi : k;
    const int ia = I * 16 + (l & 15);         // row of the L operand
    const int cb = J * 16 + (l & 15);         // column of the R operand
    const int tq = l >> 4;
    // When the tiles cover the matrix exactly (d == DP: aligned rows, no
    // padding), lane quarter tq holds the contraction indices t = tq KQ + tb
    // (tb < KQ), a contiguous piece of row ia of L read with 16-byte loads;
    // otherwise t = 4 tb + tq with masked scalar loads.  Both operands use the
    // same assignment, so each MFMA contracts matching indices.
    constexpr int KQ = DP / 4;
    const bool vecA = d == DP;
    const TL *Lp = (const TL *)c.L;
    const T *Rp = (const T *)c.R;
    const T sg = (T)c.sign;
    V acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = (T)0;
    auto tix = [&](int tb) { return vecA ? tq * KQ + tb : 4 * tb + tq; };
    auto load_l = [&](const TL *Lmat, bool ok, T (&a)[KQ]) {
        if (vecA) {
            const TL *Lrow = Lmat + (int64_t)ia * d + tq * KQ;
            if constexpr (sizeof(TL) == 8) {
#pragma unroll
                for (int u = 0; u < KQ / 2; ++u) {
                    const double2 v = ok ? reinterpret_cast<const double2 *>(Lrow)[u] : make_double2(0.0, 0.0);
                    a[2 * u] = (T)v.x;
                    a[2 * u + 1] = (T)v.y;
                }
            } else {
#pragma unroll
                for (int u = 0; u < KQ / 4; ++u) {
                    const float4 v = ok ? reinterpret_cast<const float4 *>(Lrow)[u] : make_float4(0.f, 0.f, 0.f, 0.f);
                    a[4 * u] = (T)v.x;
                    a[4 * u + 1] = (T)v.y;
                    a[4 * u + 2] = (T)v.z;
                    a[4 * u + 3] = (T)v.w;
                }
            }
        } else {
#pragma unroll
            for (int tb = 0; tb < KQ; ++tb) {
                const int t = 4 * tb + tq;
                a[tb] = (ok && ia < d && t < d) ? (T)Lmat[ia * d + t] : (T)0;
            }
        }
    };
    // Two values of j per iteration keep twice the loads in flight.
    for (int64_t j = c.jlo + w; j <= jhi; j += 2 * CONV_WAVES) {
        const bool two = j + CONV_WAVES <= jhi;
        T a0[KQ], b0[KQ], a1[KQ], b1[KQ];
        const TL *L0 = Lp + (k - j) * dd, *L1 = Lp + (k - j - CONV_WAVES) * dd;
        const T *R0 = Rp + (j - c.r_off) * dd, *R1 = Rp + (j + CONV_WAVES - c.r_off) * dd;
        load_l(L0, true, a0);
        load_l(L1, two, a1);
#pragma unroll
        for (int tb = 0; tb < KQ; ++tb) {
            const int t = tix(tb);
            const bool okB = t < d && cb < d;
            b0[tb] = okB ? R0[t * d + cb] : (T)0;
            b1[tb] = (two && okB) ? R1[t * d + cb] : (T)0;
        }
#pragma unroll
        for (int tb = 0; tb < DP / 4; ++tb) acc = Op::mac(a0[tb] * sg, b0[tb], acc);
#pragma unroll
        for (int tb = 0; tb < DP / 4; ++tb) acc = Op::mac(a1[tb] * sg, b1[tb], acc);
    }
    __shared__ T red[CONV_WAVES][4][64];
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w][r][l] = acc[r];
    __syncthreads();
    if (w == 0) {
        T *out = (T *)c.out + (k - c.out_off) * dd;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = I * 16 + Op::row(l, r), col = J * 16 + (l & 15);
            T v = (T)0;
#pragma unroll
            for (int u = 0; u < CONV_WAVES; ++u) v += red[u][r][l];
            if (row < d && col < d) {
                out[row * d + col] = v;
                if (c.status && !isfinite((double)v)) atomicOr(c.status, 2u);
            }
        }
    }
}

template <typename T, typename TL, int DP>
__global__ void __launch_bounds__(CONV_THREADS) conv_direct_kernel(ConvDesc c) {
    conv_direct_body<T, TL, DP>(c, blockIdx.x);
}

template <typename T, typename TL, int DP>
__global__ void __launch_bounds__(CONV_THREADS) conv_direct_batched_kernel(const ConvDesc *cs, int n) {
    // Few, long workgroups: the serial search costs nothing here, and the
    // wave-level lookup would add registers to a kernel that already spills.
    int lo = 0, hi = n - 1;
    const int64_t bid = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cs[mid].wg_begin <= bid) lo = mid;
        else hi = mid - 1;
    }
    conv_direct_body<T, TL, DP>(cs[lo], bid - cs[lo].wg_begin);
}

int conv_class(int d) { return (d + 15) / 16; }

static int64_t conv_blocks(const ConvDesc &c) {
    const int nt = conv_class(c.d);
    return (c.k1 - c.k0) * nt * nt;
}

static double conv_flops(const ConvDesc &c) {
    double terms = 0;   // sum over k of the number of j
    for (int64_t k = c.k0; k < c.k1; ++k) {
        const int64_t hi = c.jhi < k ? c.jhi : k;
        if (hi >= c.jlo) terms += (double)(hi - c.jlo + 1);
    }
    return terms * 2.0 * c.d * c.d * c.d;
}

template <typename T, typename TL, int DP>
static hipError_t launch_conv(const ConvDesc &c, hipStream_t st) {
    char name[96];
    snprintf(name, sizeof name, "conv_direct_kernel<%s, %s, %d>", sizeof(T) == 8 ? "double" : "float",
             sizeof(TL) == 8 ? "double" : "float", DP);
    launch_kernel(name, 0.0, conv_flops(c),
                  (conv_direct_kernel<T, TL, DP>), dim3((unsigned)conv_blocks(c)), dim3(CONV_THREADS), 0, st, c);
    return hipGetLastError();
}

template <typename T, typename TL>
static hipError_t conv_dispatch(const ConvDesc &c, hipStream_t st) {
    switch (conv_class(c.d)) {
        case 1: return launch_conv<T, TL, 16>(c, st);
        case 2: return launch_conv<T, TL, 32>(c, st);
        case 3: return launch_conv<T, TL, 48>(c, st);
        default: return launch_conv<T, TL, 64>(c, st);
    }
}

template <typename T>
hipError_t conv_direct(const ConvDesc &c, hipStream_t st) {
    if (c.k1 <= c.k0) return hipSuccess;
    if constexpr (sizeof(T) == 8) return conv_dispatch<T, double>(c, st);
    else return c.l_f64 ? conv_dispatch<T, double>(c, st) : conv_dispatch<T, float>(c, st);
}

int64_t conv_batch_layout(ConvDesc *cs, int n) {
    int64_t acc = 0;
    for (int i = 0; i < n; ++i) {
        cs[i].wg_begin = acc;
        acc += conv_blocks(cs[i]);
    }
    return acc;
}

template <typename T, typename TL, int DP>
static hipError_t launch_conv_batched(const ConvDesc *cs, int n, int64_t total, double flops, hipStream_t st) {
    char name[96];
    snprintf(name, sizeof name, "conv_direct_batched_kernel<%s, %s, %d>", sizeof(T) == 8 ? "double" : "float",
             sizeof(TL) == 8 ? "double" : "float", DP);
    launch_kernel(name, 0.0, flops,
                  (conv_direct_batched_kernel<T, TL, DP>), dim3((unsigned)total), dim3(CONV_THREADS), 0, st, cs, n);
    return hipGetLastError();
}

template <typename T, typename TL>
static hipError_t conv_batched_dispatch(int cls, const ConvDesc *cs, int n, int64_t total, double flops,
                                        hipStream_t st) {
    switch (cls) {
        case 1: return launch_conv_batched<T, TL, 16>(cs, n, total, flops, st);
        case 2: return launch_conv_batched<T, TL, 32>(cs, n, total, flops, st);
        case 3: return launch_conv_batched<T, TL, 48>(cs, n, total, flops, st);
        default: return launch_conv_batched<T, TL, 64>(cs, n, total, flops, st);
    }
}

template <typename T>
hipError_t conv_direct_batched(int cls, int l_f64, const ConvDesc *cs, int n, int64_t total, double flops,
                               hipStream_t st) {
    if (total <= 0) return hipSuccess;
    if constexpr (sizeof(T) == 8) return conv_batched_dispatch<T, double>(cls, cs, n, total, flops, st);
    else return l_f64 ? conv_batched_dispatch<T, double>(cls, cs, n, total, flops, st)
                      : conv_batched_dispatch<T, float>(cls, cs, n, total, flops, st);
}

template hipError_t conv_direct<double>(const ConvDesc &, hipStream_t);
template hipError_t conv_direct<float>(const ConvDesc &, hipStream_t);
template hipError_t conv_direct_batched<double>(int, int, const ConvDesc *, int, int64_t, double, hipStream_t);
template hipError_t conv_direct_batched<float>(int, int, const ConvDesc *, int, int64_t, double, hipStream_t);

template <typename T, int DP>
static size_t sq_lds_bytes(int dmax_odd) {
    using Cfg = SqCfg<DP>;
    size_t lds = (size_t)(Cfg::AS + Cfg::BS) * sizeof(cplx<T>);
    const size_t cs = (size_t)Cfg::NF * (dmax_odd * dmax_odd + 1) * sizeof(cplx<T>);
    return cs > lds ? cs : lds;
}

template <typename T, int DP>
static hipError_t launch_gemm_sq_batched(const FftPlan &plan, const GemmProblem<T> *probs, int nprob, int64_t total,
                                         double bytes, double flops, hipStream_t st) {
    using Cfg = SqCfg<DP>;
    const size_t lds = sq_lds_bytes<T, DP>(DP - 1);
    char name[96];
    snprintf(name, sizeof name, "freq_gemm_sq_batched_kernel<%s, %d>", sizeof(T) == 8 ? "double" : "float", DP);
    launch_kernel(name, bytes, flops,
                  (freq_gemm_sq_batched_kernel<T, DP>), dim3((unsigned)total), dim3(Cfg::THREADS), lds, st, probs,
                  nprob, plan);
    return hipGetLastError();
}

// Product class of dimension d: 1..8 = vector kernel padded to 8*cls,
// 9..12 = matrix-core kernel padded to 16*(cls-8) for even d, 13..16 the same
// for odd d.  mfma: 0 never, otherwise for every d > 8 (measured: even at
// d = 33, padded to 48, the matrix cores give 1.3x the vector kernel's
// useful flop rate in FP64 and 2x in FP32).
int gemm_sq_class(int d, int mfma) {
    if (d > 8 && d <= 64 && mfma != 0) return ((d & 1) ? 12 : 8) + (d + 15) / 16;
    return (d + 7) / 8;
}

template <typename T>
int64_t gemm_batch_layout(const FftPlan &plan, GemmProblem<T> *probs, int nprob, int mfma) {
    const int64_t F = ((int64_t)1 << plan.lgL) / 2 + 1;
    int64_t acc = 0;
    for (int i = 0; i < nprob; ++i) {
        int nf = 1;
        switch (gemm_sq_class(probs[i].d, mfma)) {
            case 1: nf = SqCfg<8>::NF; break;
            case 2: nf = SqCfg<16>::NF; break;
            case 3: nf = SqCfg<24>::NF; break;
            case 4: nf = SqCfg<32>::NF; break;
            case 5: nf = SqCfg<40>::NF; break;
            case 6: nf = SqCfg<48>::NF; break;
            case 7: nf = SqCfg<56>::NF; break;
            case 8: nf = SqCfg<64>::NF; break;
            case 9: case 13: nf = MfCfg<double, 16>::NF; break;
            case 10: case 14: nf = MfCfg<double, 32>::NF; break;
            case 11: case 15: nf = MfCfg<double, 48>::NF; break;
            default: nf = MfCfg<double, 64>::NF; break;
        }
        probs[i].wg_begin = acc;
        acc += (F + nf - 1) / nf;
    }
    return acc;
}

template <typename T>
hipError_t freq_gemm_batched(const FftPlan &plan, int dclass, int mfma, int bf3, const GemmProblem<T> *probs,
                             int nprob, int64_t total, double bytes, double flops, hipStream_t st) {
    if constexpr (sizeof(T) == 4) {
        if (bf3 && dclass >= 9) return gemm_bf3_batched(plan, dclass, probs, nprob, total, bytes, flops, st);
    }
    switch (dclass) {
        case 1: return launch_gemm_sq_batched<T, 8>(plan, probs, nprob, total, bytes, flops, st);
        case 2: return launch_gemm_sq_batched<T, 16>(plan, probs, nprob, total, bytes, flops, st);
        case 3: return launch_gemm_sq_batched<T, 24>(plan, probs, nprob, total, bytes, flops, st);
        case 4: return launch_gemm_sq_batched<T, 32>(plan, probs, nprob, total, bytes, flops, st);
        case 5: return launch_gemm_sq_batched<T, 40>(plan, probs, nprob, total, bytes, flops, st);
        case 6: return launch_gemm_sq_batched<T, 48>(plan, probs, nprob, total, bytes, flops, st);
        case 7: return launch_gemm_sq_batched<T, 56>(plan, probs, nprob, total, bytes, flops, st);
        case 8: return launch_gemm_sq_batched<T, 64>(plan, probs, nprob, total, bytes, flops, st);
        case 9: return launch_gemm_mfma_batched<T, 16, false>(plan, mfma, probs, nprob, total, bytes, flops, st);
        case 10: return launch_gemm_mfma_batched<T, 32, false>(plan, mfma, probs, nprob, total, bytes, flops, st);
        case 11: return launch_gemm_mfma_batched<T, 48, false>(plan, mfma, probs, nprob, total, bytes, flops, st);
        case 12: return launch_gemm_mfma_batched<T, 64, false>(plan, mfma, probs, nprob, total, bytes, flops, st);
        case 13: return launch_gemm_mfma_batched<T, 16, true>(plan, mfma, probs, nprob, total, bytes, flops, st);
        case 14: return launch_gemm_mfma_batched<T, 32, true>(plan, mfma, probs, nprob, total, bytes, flops, st);
        case 15: return launch_gemm_mfma_batched<T, 48, true>(plan, mfma, probs, nprob, total, bytes, flops, st);
        default: return launch_gemm_mfma_batched<T, 64, true>(plan, mfma, probs, nprob, total, bytes, flops, st);
    }
}

template int64_t gemm_batch_layout<double>(const FftPlan &, GemmProblem<double> *, int, int);
template int64_t gemm_batch_layout<float>(const FftPlan &, GemmProblem<float> *, int, int);
template hipError_t freq_gemm_batched<double>(const FftPlan &, int, int, int, const GemmProblem<double> *, int,
                                              int64_t, double, double, hipStream_t);
template hipError_t freq_gemm_batched<float>(const FftPlan &, int, int, int, const GemmProblem<float> *, int, int64_t,
                                             double, double, hipStream_t);

template <typename T, int DP>
static hipError_t launch_gemm_sq(const FftPlan &plan, int d, const cplx<T> *ZA, const cplx<T> *ZB, cplx<T> *ZC,
                                 hipStream_t st) {
    using Cfg = SqCfg<DP>;
    const size_t lds = sq_lds_bytes<T, DP>((d & 1) ? d : 0);
    const int64_t F = ((int64_t)1 << plan.lgL) / 2 + 1;
    const int64_t blocks = (F + Cfg::NF - 1) / Cfg::NF;
    char name[96];
    snprintf(name, sizeof name, "freq_gemm_sq_kernel<%s, %d>", sizeof(T) == 8 ? "double" : "float", DP);
    const double Lr = (double)((int64_t)1 << plan.lgL);
    const int nl = (d * d + 1) / 2;
    launch_kernel(name, Lr * 3.0 * nl * sizeof(cplx<T>), (double)F * 8.0 * d * d * d,
                  (freq_gemm_sq_kernel<T, DP>), dim3((unsigned)blocks), dim3(Cfg::THREADS), lds, st, ZA, ZB, ZC, plan,
                  d);
    return hipGetLastError();
}

template <typename T>
static hipError_t gemm_sq(const FftPlan &plan, int d, int mfma, const cplx<T> *ZA, const cplx<T> *ZB, cplx<T> *ZC,
                          hipStream_t st) {
    switch (gemm_sq_class(d, mfma)) {
        case 1: return launch_gemm_sq<T, 8>(plan, d, ZA, ZB, ZC, st);
        case 2: return launch_gemm_sq<T, 16>(plan, d, ZA, ZB, ZC, st);
        case 3: return launch_gemm_sq<T, 24>(plan, d, ZA, ZB, ZC, st);
        case 4: return launch_gemm_sq<T, 32>(plan, d, ZA, ZB, ZC, st);
        case 5: return launch_gemm_sq<T, 40>(plan, d, ZA, ZB, ZC, st);
        case 6: return launch_gemm_sq<T, 48>(plan, d, ZA, ZB, ZC, st);
        case 7: return launch_gemm_sq<T, 56>(plan, d, ZA, ZB, ZC, st);
        case 8: return launch_gemm_sq<T, 64>(plan, d, ZA, ZB, ZC, st);
        case 9: return launch_gemm_mfma<T, 16, false>(plan, d, mfma, ZA, ZB, ZC, st);
        case 10: return launch_gemm_mfma<T, 32, false>(plan, d, mfma, ZA, ZB, ZC, st);
        case 11: return launch_gemm_mfma<T, 48, false>(plan, d, mfma, ZA, ZB, ZC, st);
        case 12: return launch_gemm_mfma<T, 64, false>(plan, d, mfma, ZA, ZB, ZC, st);
        case 13: return launch_gemm_mfma<T, 16, true>(plan, d, mfma, ZA, ZB, ZC, st);
        case 14: return launch_gemm_mfma<T, 32, true>(plan, d, mfma, ZA, ZB, ZC, st);
        case 15: return launch_gemm_mfma<T, 48, true>(plan, d, mfma, ZA, ZB, ZC, st);
        default: return launch_gemm_mfma<T, 64, true>(plan, d, mfma, ZA, ZB, ZC, st);
    }
}

// Square products with one operand stored transposed (the adjoints), on the
// matrix cores.
template <typename T, bool TA, bool TB>
static hipError_t gemm_sq_t(const FftPlan &plan, int d, int mfma, const cplx<T> *ZA, const cplx<T> *ZB, cplx<T> *ZC,
                            hipStream_t st) {
    const bool odd = d & 1;
    switch ((d + 15) / 16) {
        case 1: return odd ? launch_gemm_mfma<T, 16, true, TA, TB>(plan, d, mfma, ZA, ZB, ZC, st)
                           : launch_gemm_mfma<T, 16, false, TA, TB>(plan, d, mfma, ZA, ZB, ZC, st);
        case 2: return odd ? launch_gemm_mfma<T, 32, true, TA, TB>(plan, d, mfma, ZA, ZB, ZC, st)
                           : launch_gemm_mfma<T, 32, false, TA, TB>(plan, d, mfma, ZA, ZB, ZC, st);
        case 3: return odd ? launch_gemm_mfma<T, 48, true, TA, TB>(plan, d, mfma, ZA, ZB, ZC, st)
                           : launch_gemm_mfma<T, 48, false, TA, TB>(plan, d, mfma, ZA, ZB, ZC, st);
        default: return odd ? launch_gemm_mfma<T, 64, true, TA, TB>(plan, d, mfma, ZA, ZB, ZC, st)
                            : launch_gemm_mfma<T, 64, false, TA, TB>(plan, d, mfma, ZA, ZB, ZC, st);
    }
}

template <typename T>
hipError_t freq_gemm(const FftPlan &plan, const GemmDesc &g, const cplx<T> *ZA, const cplx<T> *ZB, cplx<T> *ZC,
                     hipStream_t st) {
    if constexpr (sizeof(T) == 4) {
        if (g.bf3 && g.ra == g.m && g.m == g.cb && !g.transA && !g.transB && g.ra <= 64 &&
            gemm_sq_class(g.ra, g.mfma) >= 9)
            return gemm_bf3(plan, gemm_sq_class(g.ra, g.mfma), g.ra, ZA, ZB, ZC, st);
    }
    if (g.ra == g.m && g.m == g.cb && !g.transA && !g.transB && g.ra <= 64)
        return gemm_sq<T>(plan, g.ra, g.mfma, ZA, ZB, ZC, st);
    const bool sq = g.ra == g.m && g.m == g.cb && g.ra <= 64 && !(g.transA && g.transB);
    if (sq && gemm_sq_class(g.ra, g.mfma) >= 9) {
        if (g.transA) return gemm_sq_t<T, true, false>(plan, g.ra, g.mfma, ZA, ZB, ZC, st);
        return gemm_sq_t<T, false, true>(plan, g.ra, g.mfma, ZA, ZB, ZC, st);
    }
    const int dmax = g.ra > g.cb ? g.ra : g.cb;
    // Thin products (a matrix times a vector, and its adjoints) take 1 x 1
    // register tiles: with wider tiles a frequency has too few of them, and
    // the A operand's LDS share caps the frequencies per workgroup, so most
    // threads would idle.
    if (dmax <= 8 || g.ra <= 2 || g.cb <= 2) return launch_gemm<T, 1, 1>(plan, g, ZA, ZB, ZC, st);
    if (dmax <= 24) return launch_gemm<T, 2, 2>(plan, g, ZA, ZB, ZC, st);
    return launch_gemm<T, 4, 4>(plan, g, ZA, ZB, ZC, st);
}

// C = A * diag(h)
template <typename T>
__global__ void freq_diag_kernel(const cplx<T> *ZA, const cplx<T> *__restrict__ ZH,
                                 cplx<T> *ZC, FftPlan plan, int ra, int cb, int nl, int nlh) {
    const int64_t L = (int64_t)1 << plan.lgL;
    const int64_t F = L / 2 + 1;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = gid / nl;
    const int c = (int)(gid - k * nl);
    if (k >= F) return;
    const int64_t r1 = freq_row(plan, k), r2 = freq_row(plan, (L - k) & (L - 1));
    const int e = 2 * c;
    cplx<T> ce = cmul<T>(unpack<T>(ZA, nl, r1, r2, e), unpack<T>(ZH, nlh, r1, r2, e % cb));
    cplx<T> co = mk<T>(0, 0);
    if (e + 1 < ra * cb) co = cmul<T>(unpack<T>(ZA, nl, r1, r2, e + 1), unpack<T>(ZH, nlh, r1, r2, (e + 1) % cb));
    pack_store<T>(ZC, nl, r1, r2, c, ce, co);
}

template <typename T>
hipError_t freq_diag(const FftPlan &plan, int ra, int cb, const cplx<T> *ZA, const cplx<T> *ZH, cplx<T> *ZC,
                     hipStream_t st) {
    const int nl = (ra * cb + 1) / 2, nlh = (cb + 1) / 2;
    const int64_t F = ((int64_t)1 << plan.lgL) / 2 + 1;
    const int64_t total = F * nl;
    const int threads = 256;
    launch_kernel(sizeof(T) == 8 ? "freq_diag_kernel<double>" : "freq_diag_kernel<float>",
                  (double)((int64_t)1 << plan.lgL) * (2 * nl + nlh) * sizeof(cplx<T>), (double)F * ra * cb * 6.0,
                  freq_diag_kernel<T>, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, st, ZA, ZH,
                  ZC, plan, ra, cb, nl, nlh);
    return hipGetLastError();
}

// h_j = sum_i A_ij B_ij
template <typename T>
__global__ void freq_coldot_kernel(const cplx<T> *__restrict__ ZA, const cplx<T> *__restrict__ ZB,
                                   cplx<T> *__restrict__ ZH, FftPlan plan, int ra, int cb, int nl, int nlh) {
    const int64_t L = (int64_t)1 << plan.lgL;
    const int64_t F = L / 2 + 1;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = gid / nlh;
    const int c = (int)(gid - k * nlh);
    if (k >= F) return;
    const int64_t r1 = freq_row(plan, k), r2 = freq_row(plan, (L - k) & (L - 1));
    cplx<T> h[2] = {mk<T>(0, 0), mk<T>(0, 0)};
    for (int u = 0; u < 2; ++u) {
        const int j = 2 * c + u;
        if (j >= cb) break;
        for (int i = 0; i < ra; ++i) {
            const int e = i * cb + j;
            h[u] = cadd<T>(h[u], cmul<T>(unpack<T>(ZA, nl, r1, r2, e), unpack<T>(ZB, nl, r1, r2, e)));
        }
    }
    pack_store<T>(ZH, nlh, r1, r2, c, h[0], h[1]);
}

template <typename T>
hipError_t freq_coldot(const FftPlan &plan, int ra, int cb, const cplx<T> *ZA, const cplx<T> *ZB, cplx<T> *ZH,
                       hipStream_t st) {
    const int nl = (ra * cb + 1) / 2, nlh = (cb + 1) / 2;
    const int64_t F = ((int64_t)1 << plan.lgL) / 2 + 1;
    const int64_t total = F * nlh;
    const int threads = 256;
    hipLaunchKernelGGL(freq_coldot_kernel<T>, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0,
                       st, ZA, ZB, ZH, plan, ra, cb, nl, nlh);
    return hipGetLastError();
}

template hipError_t freq_gemm<double>(const FftPlan &, const GemmDesc &, const cplx<double> *, const cplx<double> *,
                                      cplx<double> *, hipStream_t);
template hipError_t freq_gemm<float>(const FftPlan &, const GemmDesc &, const cplx<float> *, const cplx<float> *,
                                     cplx<float> *, hipStream_t);
template hipError_t freq_diag<double>(const FftPlan &, int, int, const cplx<double> *, const cplx<double> *,
                                      cplx<double> *, hipStream_t);
template hipError_t freq_diag<float>(const FftPlan &, int, int, const cplx<float> *, const cplx<float> *,
                                     cplx<float> *, hipStream_t);
template hipError_t freq_coldot<double>(const FftPlan &, int, int, const cplx<double> *, const cplx<double> *,
                                        cplx<double> *, hipStream_t);
template hipError_t freq_coldot<float>(const FftPlan &, int, int, const cplx<float> *, const cplx<float> *,
                                       cplx<float> *, hipStream_t);

}  // namespace mrinv
