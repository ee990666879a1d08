// Internal definitions shared by the mrinv HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrinv {

// ---------------------------------------------------------------------------
// Complex helpers on HIP vector types (float2 / double2).
// ---------------------------------------------------------------------------
template <typename T> struct C2;
template <> struct C2<double> { using type = double2; };
template <> struct C2<float> { using type = float2; };
template <typename T> using cplx = typename C2<T>::type;

template <typename T> __host__ __device__ __forceinline__ cplx<T> mk(T re, T im) {
    cplx<T> z; z.x = re; z.y = im; return z;
}
template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
// The products are written with explicit fused multiply-adds, so their
// rounding does not depend on how the compiler contracts the surrounding code.
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return mk<T>(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
    return mk<T>(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -(a.x * b.y)));
}
template <typename T> __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return mk<T>(a.x, -a.y); }
template <typename T> __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV> __device__ __forceinline__ cplx<T> mul_mi(cplx<T> a) {
    return INV ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Twiddles.  W(a) = exp(-2 pi i a / TW_LMAX), a in [0, TW_LMAX), is the product
// of two table entries: hi[a >> TW_LO_BITS] * lo[a & (TW_LO_SIZE-1)].  Both
// tables are filled on the host from the exact dyadic angle in extended
// precision, so each factor is correctly rounded and the product carries at
// most a few ulps.
// ---------------------------------------------------------------------------
constexpr int TW_LG = 22;
constexpr int64_t TW_LMAX = int64_t(1) << TW_LG;
constexpr int TW_LO_BITS = 11;
constexpr int TW_LO_SIZE = 1 << TW_LO_BITS;
constexpr int TW_HI_SIZE = 1 << (TW_LG - TW_LO_BITS);

// The tables are float64 for both precisions: a float32 twiddle is the
// float64 product rounded once, so it is within half an ulp of the exact value.
template <typename T> struct Twiddles {
    const double2 *hi;
    const double2 *lo;
    const double2 *root;   // W_512^j, j < 512 (the 512th roots, equal to hi[4j]); may be null
    const void *outer;     // outer twiddles of the current pass, [m][kr] in precision T; may be null
};

// exp(-2 pi i * num / den) with den a power of two dividing TW_LMAX, num in [0, den).
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> twiddle(const Twiddles<T> &tw, uint32_t num, int lg_den) {
    uint32_t a = num << (TW_LG - lg_den);
    const double2 w = cmul<double>(tw.hi[a >> TW_LO_BITS], tw.lo[a & (TW_LO_SIZE - 1)]);
    return mk<T>((T)w.x, INV ? -(T)w.y : (T)w.y);
}

// ---------------------------------------------------------------------------
// In-register DFT of size R in natural order (R = 1, 2, 4, 8, 16), forward
// (exp(-2 pi i/R)) or inverse (exp(+2 pi i/R)), unnormalised.  Radix-2
// decimation in time with the R-th roots as literal constants.
// ---------------------------------------------------------------------------
template <typename T, int R, bool INV> struct Dft;

template <typename T, bool INV> struct Dft<T, 1, INV> {
    __device__ __forceinline__ static void run(cplx<T> *) {}
};
template <typename T, bool INV> struct Dft<T, 2, INV> {
    __device__ __forceinline__ static void run(cplx<T> *v) {
        cplx<T> a = v[0], b = v[1];
        v[0] = cadd<T>(a, b);
        v[1] = csub<T>(a, b);
    }
};
template <typename T, bool INV> struct Dft<T, 4, INV> {
    __device__ __forceinline__ static void run(cplx<T> *v) {
        cplx<T> s0 = cadd<T>(v[0], v[2]), d0 = csub<T>(v[0], v[2]);
        cplx<T> s1 = cadd<T>(v[1], v[3]), d1 = mul_mi<T, INV>(csub<T>(v[1], v[3]));
        v[0] = cadd<T>(s0, s1);
        v[2] = csub<T>(s0, s1);
        v[1] = cadd<T>(d0, d1);
        v[3] = csub<T>(d0, d1);
    }
};

// Root table for R = 8 and R = 16: cos/sin of 2 pi k / 16, k = 0..7.
__device__ __forceinline__ double root16_cos(int k) {
    constexpr double c[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                             0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
    return c[k];
}
__device__ __forceinline__ double root16_sin(int k) {
    constexpr double s[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                             1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};
    return s[k];
}

template <typename T, int R, bool INV> struct Dft {
    static_assert(R == 8 || R == 16, "radix");
    __device__ __forceinline__ static void run(cplx<T> *v) {
        constexpr int H = R / 2;
        cplx<T> e[H], o[H];
#pragma unroll
        for (int i = 0; i < H; ++i) { e[i] = v[2 * i]; o[i] = v[2 * i + 1]; }
        Dft<T, H, INV>::run(e);
        Dft<T, H, INV>::run(o);
#pragma unroll
        for (int k = 0; k < H; ++k) {
            // w = exp(-+ 2 pi i k / R) = cos - i sin (forward)
            const int idx = k * (16 / R);
            const T c = (T)root16_cos(idx), s = (T)root16_sin(idx);
            cplx<T> w = mk<T>(c, INV ? s : -s);
            // k / R = 1/4: w = -i (forward) or +i (inverse), a swap and a sign
            cplx<T> t = (k == 0) ? o[k] : (4 * k == R) ? mul_mi<T, INV>(o[k]) : cmul<T>(w, o[k]);
            v[k] = cadd<T>(e[k], t);
            v[k + H] = csub<T>(e[k], t);
        }
    }
};

__host__ __device__ constexpr int ilog2c(int64_t x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

// Radix of stage s of a 2^lgP-point in-workgroup FFT (0 = no such stage).
__host__ __device__ constexpr int stage_lg(int lgP, int s) {
    // lgP: 0..12. Balanced split into stages of at most 4 bits, larger first.
    return lgP <= 4 ? (s == 0 ? lgP : 0)
         : lgP <= 8 ? (s == 0 ? (lgP + 1) / 2 : s == 1 ? lgP / 2 : 0)
                    : (s == 0 ? (lgP + 2) / 3 : s == 1 ? (lgP + 1) / 3 : s == 2 ? lgP / 3 : 0);
}
__host__ __device__ constexpr int num_stages(int lgP) {
    return lgP <= 4 ? 1 : lgP <= 8 ? 2 : 3;
}
__host__ __device__ constexpr int min_stage_lg(int lgP) {
    return lgP <= 4 ? lgP : lgP <= 8 ? lgP / 2 : lgP / 3;
}

// Index of the problem that owns workgroup bid in a batched launch of NT
// threads per workgroup: the last i with probs[i].wg_begin <= bid (the begins
// ascend from 0).  With whole waves (NT a multiple of 64) each wave finds it
// on its own: its 64 lanes test 64 evenly spaced begins at once, the ballot
// of the hits (a prefix, the begins being sorted) picks the span that holds
// the answer, and the next round tests that span; one round for up to 64
// problems, two for up to 4096, where a serial search waits for log2(nprob)
// dependent loads before the workgroup touches its data.  The ballots keep
// the result wave-uniform, so the descriptor loads stay scalar.  Workgroups
// with a partial wave search serially.
template <int NT, typename P>
__device__ __forceinline__ int owner_of(const P *probs, int nprob, int64_t bid) {
    int lo = 0;
    if constexpr (NT % 64 != 0) {
        int hi = nprob - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (probs[mid].wg_begin <= bid) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    } else {
        if (nprob <= 1) return 0;
        const int lane = (int)(threadIdx.x & 63);
        int span = nprob;                     // the answer lies in [lo, lo + span)
        for (;;) {
            const int stride = (span + 63) >> 6;
            const int j = lo + lane * stride;
            const bool hit = lane * stride < span && probs[j].wg_begin <= bid;
            const int k = __popcll(__ballot(hit)) - 1;   // >= 0 while probs[lo].wg_begin <= bid
            lo += (k > 0 ? k : 0) * stride;
            if (stride == 1) return lo;
            span = stride < nprob - lo ? stride : nprob - lo;
        }
    }
}

}  // namespace mrinv
