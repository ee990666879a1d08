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
// No multiply-add contraction in this file: a pass computes the same bits
// whatever its lanes per workgroup or LDS tiling, so batched and single
// transforms of one problem agree exactly.
#pragma clang fp contract(off)

#include <stdio.h>

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace mrinv {

// Number of elements of a register array (the stage radix) in the generic
// load/store callbacks.
#define MR_RADIX(v) ((int)std::extent<std::remove_reference_t<decltype(v)>>::value)

// One Stockham stage of radix R = 2^LGR inside a 2^LGP-point transform.
// Group j = grp reads its elements j + r 2^(LGP-LGR) (r < R) through
// load_all(j, LGP - LGR, v), multiplies element r by the stage twiddle
// W_{2^(lgNs+LGR)}^{k r} (k = j mod 2^lgNs, from the workgroup's table
// roots[i] = W_P^i), runs the R-point DFT and writes elements b + r 2^lgNs
// through store_all(b, lgNs, v).  The callbacks issue all R memory accesses
// before any result is used.
template <typename T, int LGR, bool INV, typename LoadAll, typename StoreAll>
__device__ __forceinline__ void fft_stage(int LGP, int lgNs, int grp, const LoadAll &load_all,
                                          const StoreAll &store_all, const cplx<T> *roots, bool sync_between) {
    constexpr int R = 1 << LGR;
    const int nbf = 1 << (LGP - LGR);
    const bool active = grp < nbf;
    cplx<T> v[R];
    const int j = grp;
    const int k0 = j & ((1 << lgNs) - 1);
    if (active) {
        load_all(j, LGP - LGR, v);
        if (lgNs > 0) {
            const int sh = LGP - lgNs - LGR;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cplx<T> w = roots[(k0 * r) << sh];
                v[r] = INV ? cmulc<T>(v[r], w) : cmul<T>(v[r], w);
            }
        }
        Dft<T, R, INV>::run(v);
    }
    if (sync_between) __syncthreads();
    if (active) store_all(((j >> lgNs) << (lgNs + LGR)) + k0, lgNs, v);
}

// Full 2^LGP-point DFT of one column of C lanes.  gload_all / gstore_all
// access natural-order elements (see fft_stage); src_lds / dst_lds say whether
// they are the LDS tile itself (then stages that read and write it
// synchronise).
template <typename T, int LGP, bool INV, typename GL, typename GS>
__device__ __forceinline__ void wg_fft(cplx<T> *lds, int lds_stride, int c, int grp, const GL &gload_all,
                                       const GS &gstore_all, bool src_lds, bool dst_lds, const cplx<T> *roots) {
    constexpr int NS = num_stages(LGP);
    constexpr int R0 = stage_lg(LGP, 0), R1 = stage_lg(LGP, 1), R2 = stage_lg(LGP, 2);
    auto lload_all = [&](int j, int lgs, auto &v) {
#pragma unroll
        for (int r = 0; r < MR_RADIX(v); ++r) v[r] = lds[(j + (r << lgs)) * lds_stride + c];
    };
    auto lstore_all = [&](int b, int lgs, auto &v) {
#pragma unroll
        for (int r = 0; r < MR_RADIX(v); ++r) lds[(b + (r << lgs)) * lds_stride + c] = v[r];
    };
    if constexpr (NS == 1) {
        fft_stage<T, R0, INV>(LGP, 0, grp, gload_all, gstore_all, roots, src_lds && dst_lds);
    } else if constexpr (NS == 2) {
        fft_stage<T, R0, INV>(LGP, 0, grp, gload_all, lstore_all, roots, src_lds);
        __syncthreads();
        fft_stage<T, R1, INV>(LGP, R0, grp, lload_all, gstore_all, roots, dst_lds);
    } else {
        fft_stage<T, R0, INV>(LGP, 0, grp, gload_all, lstore_all, roots, src_lds);
        __syncthreads();
        fft_stage<T, R1, INV>(LGP, R0, grp, lload_all, lstore_all, roots, true);
        __syncthreads();
        fft_stage<T, R2, INV>(LGP, R0 + R1, grp, lload_all, gstore_all, roots, dst_lds);
    }
}

// A wave-uniform 64-bit value passed through readfirstlane: the same number,
// which the compiler can no longer prove equal to its source.  The stores of
// a pass use it for their row stride, so their addresses are formed anew
// instead of keeping the first stage's load addresses (the same rows in the
// 512-row passes) alive across the transform: without it the 512-row inverse
// pass spills 44 bytes per lane at its 64-register budget.
__device__ __forceinline__ int64_t uniform_copy(int64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ bool is_diag_lane(int e, int e0_d) {
    return e < e0_d * e0_d && (e % (e0_d + 1)) == 0;
}

__device__ __forceinline__ void flag_nonfinite(unsigned int *status, double a, double b) {
    if (status && (!isfinite(a) || !isfinite(b))) atomicOr(status, STATUS_NONFINITE);
}

// LDS layout of a pass workgroup.  The data tile holds P rows of C lanes
// (stride C + 1), or, for the float64 passes of 256 rows (16 lanes) and 512
// rows (8 or 16 lanes), P rows of C/2 lanes that the two lane halves use in
// turn (stride C/2).  512 rows, 16 lanes: 80 KB instead of 155 KB, two
// 1024-thread workgroups per CU, compiled for 8 waves per SIMD (64 VGPRs);
// 512 rows, 8 lanes: 48 KB, three 512-thread workgroups, 6 waves (80 VGPRs);
// 256 rows, 16 lanes: 40 KB, four 256-thread workgroups, 4 waves (128 VGPRs).
// P outer twiddles and P stage roots follow the tile.
template <typename T, int LGP, int C, int MODE>
__host__ __device__ constexpr int pass_split() {
    return (sizeof(T) == 8 && (((LGP == 9 || LGP == 8) && C == 16) || (LGP == 9 && C == 8))) ? 2 : 1;
}
// Waves per SIMD the pass kernels are compiled for (VGPR budget 512 / waves).
template <typename T, int LGP, int C, int MODE>
__host__ __device__ constexpr int pass_waves() {
    if (sizeof(T) == 4 && LGP == 9 && C == 16) return 8;   // two 1024-thread workgroups per CU
    if (sizeof(T) == 4 && LGP == 7 && C >= 16) return 8;   // as many workgroups as the LDS allows
    return pass_split<T, LGP, C, MODE>() == 2 ? (LGP == 9 ? (C == 8 ? 6 : 8) : 4) : 1;
}
template <typename T, int LGP, int C, int MODE>
__host__ __device__ constexpr int pass_lds_stride() {
    return pass_split<T, LGP, C, MODE>() == 2 ? C / 2 : C + 1;
}
template <typename T, int LGP, int C, int MODE>
__host__ __device__ constexpr size_t pass_lds_bytes() {
    return ((size_t)1 << LGP) * (pass_lds_stride<T, LGP, C, MODE>() + 2) * sizeof(cplx<T>);
}

__device__ __forceinline__ int stage_store_base(int j, int lgNs, int LGR) {
    return ((j >> lgNs) << (lgNs + LGR)) + (j & ((1 << lgNs) - 1));
}

// Stage twiddles and DFT of one stage, in registers (see fft_stage).
template <typename T, int LGR, bool INV>
__device__ __forceinline__ void stage_math(int LGP, int lgNs, int j, cplx<T> (&v)[1 << LGR], const cplx<T> *roots) {
    constexpr int R = 1 << LGR;
    if (lgNs > 0) {
        const int k0 = j & ((1 << lgNs) - 1);
        const int sh = LGP - lgNs - LGR;
#pragma unroll
        for (int r = 1; r < R; ++r) {
            const cplx<T> w = roots[(k0 * r) << sh];
            v[r] = INV ? cmulc<T>(v[r], w) : cmul<T>(v[r], w);
        }
    }
    Dft<T, R, INV>::run(v);
}

// Moves v from one stage's store layout (elements b + r 2^lgs_out) to the
// next stage's load layout (elements j + r 2^lgs_in) through a tile holding
// HC lanes: lanes [h HC, (h + 1) HC) in round h.
template <typename T, int R, int HC>
__device__ __forceinline__ void split_exchange(cplx<T> *tile, int half, int ch, int b, int lgs_out, int j, int lgs_in,
                                               cplx<T> (&v)[R]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (half == h) {
#pragma unroll
            for (int r = 0; r < R; ++r) tile[(b + (r << lgs_out)) * HC + ch] = v[r];
        }
        __syncthreads();
        if (half == h) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = tile[(j + (r << lgs_in)) * HC + ch];
        }
        __syncthreads();
    }
}

// All stages of a 2^LGP-point DFT whose stages share one register radix, from
// v in stage 0's load layout of group j to v in the last stage's store layout.
template <typename T, int LGP, bool INV, int HC>
__device__ __forceinline__ void split_stages(cplx<T> *tile, int half, int ch, int j,
                                             cplx<T> (&v)[1 << stage_lg(LGP, 0)], const cplx<T> *roots) {
    constexpr int LGR = stage_lg(LGP, 0), NS = num_stages(LGP), R = 1 << LGR;
    static_assert(stage_lg(LGP, 1) == LGR && (NS < 3 || stage_lg(LGP, 2) == LGR), "uniform radix");
    stage_math<T, LGR, INV>(LGP, 0, j, v, roots);
#pragma unroll
    for (int st = 1; st < NS; ++st) {
        const int lo = (st - 1) * LGR;
        split_exchange<T, R, HC>(tile, half, ch, stage_store_base(j, lo, LGR), lo, j, LGP - LGR, v);
        stage_math<T, LGR, INV>(LGP, st * LGR, j, v, roots);
    }
}

// MODE 0: forward pass; MODE 1: inverse pass; MODE 2: inverse pass, then the
// mask/scale/negate of `dst` (rows outside [lo, hi) become zero), then the
// forward pass of the same geometry, in place.
// The body of one pass for one column of one problem.
template <typename T, int LGP, int C, int MODE>
__device__ __forceinline__ void fft_pass_body(cplx<T> *z, const PassGeom &g, int nl, int nchunks, int64_t blk,
                                              const SrcDesc &src, const DstDesc &dst, const Twiddles<T> &tw) {
    constexpr int P = 1 << LGP;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *lds = reinterpret_cast<cplx<T> *>(smem_raw);
    constexpr int SPLIT = pass_split<T, LGP, C, MODE>();
    constexpr int LDS_STRIDE = pass_lds_stride<T, LGP, C, MODE>();
    cplx<T> *tws = lds + P * LDS_STRIDE;   // outer twiddles of this column
    cplx<T> *roots = tws + P;              // roots[i] = W_P^i
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
    // Lanes past nl read a valid lane and never store.
    const int lane_c = lane_ok ? lane : nl - 1;
    const int64_t rs = S * nl;                        // elements from row idx to row idx + 1
    cplx<T> *zc = z + base * nl + lane_c;

    // Forward twiddle on output r: W_B^{m r}; inverse on input r: W_B^{-m r}.
    // They depend on the column only, so the workgroup forms its P outer
    // twiddles (from the pass's table when there is one) and the P roots of
    // its in-workgroup stages once; every lane reads them from LDS.  Each
    // thread issues its first stage's data loads before filling the tables,
    // so the two memory latencies overlap.
    auto fill_tables = [&]() {
        const cplx<T> *otw = reinterpret_cast<const cplx<T> *>(tw.outer) + ((size_t)m << LGP);
        for (int i = threadIdx.x; i < P; i += blockDim.x) {
            if (m) tws[i] = tw.outer ? otw[i] : twiddle<T, false>(tw, m * (uint32_t)i, g.lgB);
            if (tw.root) {
                const double2 w = tw.root[i << (9 - LGP)];
                roots[i] = mk<T>((T)w.x, (T)w.y);
            } else {
                roots[i] = twiddle<T, false>(tw, (uint32_t)i, LGP);
            }
        }
    };
    constexpr int LG0 = stage_lg(LGP, 0);              // first stage: radix 2^LG0
    const bool first_active = grp < (P >> LG0);
    cplx<T> pre[1 << LG0];                              // its elements, loaded early

    auto z_load_all = [&](int j, int lgs, auto &v) {
        const cplx<T> *q = zc + (int64_t)j * rs;
        const int64_t step = rs << lgs;
#pragma unroll
        for (int r = 0; r < MR_RADIX(v); ++r) {
            v[r] = *q;
            q += step;
        }
    };
    auto z_store_all = [&](int b0, int lgs, auto &v) {
        if (!lane_ok) return;
        const int64_t rsu = uniform_copy(rs);    // rs is the same in every lane
        // The lane's address is formed again from the thread index (hidden
        // from the optimiser), so the 64-bit load address zc need not stay
        // live through the stages.
        int tx = (int)threadIdx.x;
        asm volatile("" : "+v"(tx));
        cplx<T> *q = z + base * nl + (chunk * C + tx % C) + (int64_t)b0 * rsu;
        const int64_t step = rsu << lgs;
#pragma unroll
        for (int r = 0; r < MR_RADIX(v); ++r) {
            *q = v[r];
            q += step;
        }
    };
    auto fwd_store_all = [&](int b0, int lgs, auto &v) {
        if (m) {
#pragma unroll
            for (int r = 0; r < MR_RADIX(v); ++r) v[r] = cmul<T>(v[r], tws[b0 + (r << lgs)]);
        }
        z_store_all(b0, lgs, v);
        if constexpr (MODE == 0 && sizeof(T) == 8) {
            // Optional float32 copy of the float64 output, same layout.
            if (dst.aux && lane_ok) {
                float2 *qa = (float2 *)dst.aux + (zc - z) + (int64_t)b0 * rs;
                const int64_t step = rs << lgs;
#pragma unroll
                for (int r = 0; r < MR_RADIX(v); ++r) {
                    *qa = make_float2((float)v[r].x, (float)v[r].y);
                    qa += step;
                }
            }
        }
    };
    // First-stage loads from the early copy (the forward stage has no input
    // twiddle; the inverse one multiplies by the conjugate outer twiddles).
    auto pre_load = [&](int, int, auto &v) {
#pragma unroll
        for (int r = 0; r < MR_RADIX(v); ++r) v[r] = pre[r];
    };
    auto pre_inv_load = [&](int j, int lgs, auto &v) {
#pragma unroll
        for (int r = 0; r < MR_RADIX(v); ++r) v[r] = pre[r];
        if (m) {
#pragma unroll
            for (int r = 0; r < MR_RADIX(v); ++r) v[r] = cmulc<T>(v[r], tws[j + (r << lgs)]);
        }
    };
    // Inverse first stages: raw early loads, then the tables.
    auto start_inverse = [&]() {
        if (first_active) z_load_all(grp, LGP - LG0, pre);
        fill_tables();
        __syncthreads();
    };

    // Two lane halves sharing the tile: all stages in registers, exchanges
    // in two rounds.
    constexpr int LGR = stage_lg(LGP, 0);
    constexpr int LGL = (num_stages(LGP) - 1) * LGR;   // last stage's store stride exponent
    const int half = c / (C / 2 > 0 ? C / 2 : 1), ch = c % (C / 2 > 0 ? C / 2 : 1);
    const int jb = grp, bl = stage_store_base(grp, LGL, LGR);
    (void)half;
    (void)ch;
    (void)bl;
    (void)jb;

    if constexpr (MODE == 0) {
        // Real source: complex lane = entries (2 lane, 2 lane + 1) of row t
        // (or rev - t), zero outside [lo, hi); e0 - source when e0_d > 0.
        auto real_load_all = [&](int j, int lgs, auto &v) {
            constexpr int R = MR_RADIX(v);
            const int64_t t0 = base + (int64_t)j * S, dt = S << lgs;
            const int e = 2 * lane_c;
            const bool two = e + 1 < src.nreal;
            const int64_t rstep = (src.rev >= 0 ? -dt : dt) * src.ld;
            const int64_t row0 = src.rev >= 0 ? src.rev - t0 : t0;
            // With an even row length and entry count every lane is an aligned
            // pair: one vector load per element.
            const bool vec = ((src.ld | src.nreal) & 1) == 0;
            if (src.kind == SRC_REAL64) {
                const double *q = (const double *)src.p + row0 * src.ld + e;
                if (vec) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int64_t t = t0 + r * dt;
                        double2 w = make_double2(0.0, 0.0);
                        if (t >= src.lo && t < src.hi) w = *(const double2 *)q;
                        v[r] = mk<T>((T)w.x, (T)w.y);
                        q += rstep;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int64_t t = t0 + r * dt;
                        T a = 0, bb = 0;
                        if (t >= src.lo && t < src.hi) {
                            a = (T)q[0];
                            if (two) bb = (T)q[1];
                        }
                        v[r] = mk<T>(a, bb);
                        q += rstep;
                    }
                }
            } else {
                const float *q = (const float *)src.p + row0 * src.ld + e;
                if (vec) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int64_t t = t0 + r * dt;
                        float2 w = make_float2(0.f, 0.f);
                        if (t >= src.lo && t < src.hi) w = *(const float2 *)q;
                        v[r] = mk<T>((T)w.x, (T)w.y);
                        q += rstep;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int64_t t = t0 + r * dt;
                        T a = 0, bb = 0;
                        if (t >= src.lo && t < src.hi) {
                            a = (T)q[0];
                            if (two) bb = (T)q[1];
                        }
                        v[r] = mk<T>(a, bb);
                        q += rstep;
                    }
                }
            }
            if (src.e0_d > 0) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t t = t0 + r * dt;
                    if (t < src.lo || t >= src.hi) continue;
                    T a = -v[r].x, bb = two ? -v[r].y : (T)0;
                    if (t == 0) {
                        if (is_diag_lane(e, src.e0_d)) a += (T)1;
                        if (two && is_diag_lane(e + 1, src.e0_d)) bb += (T)1;
                    }
                    v[r] = mk<T>(a, bb);
                }
            }
        };
        auto gload_all = [&](int j, int lgs, auto &v) {
            if (src.kind == SRC_Z) z_load_all(j, lgs, v);
            else real_load_all(j, lgs, v);
        };
        if (first_active) gload_all(grp, LGP - LG0, pre);
        fill_tables();
        __syncthreads();
        if constexpr (SPLIT == 2) {
            cplx<T> v[1 << LGR];
            pre_load(jb, LGP - LGR, v);
            split_stages<T, LGP, false, C / 2>(lds, half, ch, jb, v, roots);
            fwd_store_all(bl, LGL, v);
        } else {
            wg_fft<T, LGP, false>(lds, LDS_STRIDE, c, grp, pre_load, fwd_store_all, false, false, roots);
        }
    } else if constexpr (MODE == 1) {
        // Real destination: value = op(scale * v) (+ the old value or the
        // float32 aux entry), rows t in [lo, hi) of row t (or rev - t).
        auto real_store_all = [&](int b0, int lgs, auto &v) {
            constexpr int R = MR_RADIX(v);
            if (!lane_ok) return;
            const int64_t t0 = base + (int64_t)b0 * S, dt = S << lgs;
            const int e = 2 * lane;
            const bool two = e + 1 < dst.nreal;
            const bool dbl = dst.kind == DST_REAL64;
            const bool vec = ((dst.ld | dst.nreal) & 1) == 0;   // aligned pairs (see the loads)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t t = t0 + r * dt;
                if (t < dst.lo || t >= dst.hi) continue;
                const int64_t row = dst.rev >= 0 ? dst.rev - t : t;
                double a = (double)v[r].x * dst.scale, bb = (double)v[r].y * dst.scale;
                if (dst.op == OP_NEG) {
                    a = -a;
                    bb = -bb;
                } else if (dst.op == OP_E0MINUS) {
                    a = (t == 0 && is_diag_lane(e, dst.e0_d) ? 1.0 : 0.0) - a;
                    bb = (t == 0 && is_diag_lane(e + 1, dst.e0_d) ? 1.0 : 0.0) - bb;
                }
                if (dst.op == OP_ADD || dst.op == OP_XPLUS) {
                    // the old value (OP_ADD) or the float32 aux entry (OP_XPLUS)
                    if (dst.op == OP_XPLUS || !dbl) {
                        const float *x = (const float *)(dst.op == OP_XPLUS ? dst.aux : dst.p) + row * dst.ld + e;
                        a += (double)x[0];
                        if (two) bb += (double)x[1];
                    } else {
                        const double *x = (const double *)dst.p + row * dst.ld + e;
                        a += x[0];
                        if (two) bb += x[1];
                    }
                }
                if (dbl) {
                    double *p = (double *)dst.p + row * dst.ld + e;
                    if (vec) {
                        *(double2 *)p = make_double2(a, bb);
                    } else {
                        p[0] = a;
                        if (two) p[1] = bb;
                    }
                } else {
                    float *p = (float *)dst.p + row * dst.ld + e;
                    if (vec) {
                        *(float2 *)p = make_float2((float)a, (float)bb);
                    } else {
                        p[0] = (float)a;
                        if (two) p[1] = (float)bb;
                    }
                }
                flag_nonfinite(dst.status, a, two ? bb : 0.0);
            }
        };
        auto gstore_all = [&](int b0, int lgs, auto &v) {
            if (dst.kind == DST_Z) z_store_all(b0, lgs, v);
            else real_store_all(b0, lgs, v);
        };
        start_inverse();
        if constexpr (SPLIT == 2) {
            cplx<T> v[1 << LGR];
            pre_inv_load(jb, LGP - LGR, v);
            split_stages<T, LGP, true, C / 2>(lds, half, ch, jb, v, roots);
            gstore_all(bl, LGL, v);
        } else {
            wg_fft<T, LGP, true>(lds, LDS_STRIDE, c, grp, pre_inv_load, gstore_all, false, false, roots);
        }
    } else {
        const T sc = dst.op == OP_NEG ? -(T)dst.scale : (T)dst.scale;
        // The column's rows base + idx * S rise with idx, so the window
        // [lo, hi) is the index range [ilo, ihi) (S = 2^(lgB - LGP)); both
        // bounds are the same for the whole workgroup.
        const int lgS = g.lgB - LGP;
        auto first_idx = [&](int64_t x) {
            if (x <= base) return 0;
            const int64_t q = (x - base + S - 1) >> lgS;
            return q >= P ? P : (int)q;
        };
        const int ilo = first_idx(dst.lo), ihi = first_idx(dst.hi);
        start_inverse();
        if constexpr (SPLIT == 2) {
            cplx<T> v[1 << LGR];
            pre_inv_load(jb, LGP - LGR, v);
            split_stages<T, LGP, true, C / 2>(lds, half, ch, jb, v, roots);
#pragma unroll
            for (int r = 0; r < (1 << LGR); ++r) {
                const int idx = bl + (r << LGL);
                v[r] = idx >= ilo && idx < ihi ? cscale<T>(v[r], sc) : mk<T>(0, 0);
            }
            split_exchange<T, 1 << LGR, C / 2>(lds, half, ch, bl, LGL, jb, LGP - LGR, v);
            split_stages<T, LGP, false, C / 2>(lds, half, ch, jb, v, roots);
            fwd_store_all(bl, LGL, v);
            return;
        }
        auto mask_store_all = [&](int b0, int lgs, auto &v) {
#pragma unroll
            for (int r = 0; r < MR_RADIX(v); ++r) {
                const int idx = b0 + (r << lgs);
                lds[idx * LDS_STRIDE + c] = idx >= ilo && idx < ihi ? cscale<T>(v[r], sc) : mk<T>(0, 0);
            }
        };
        wg_fft<T, LGP, true>(lds, LDS_STRIDE, c, grp, pre_inv_load, mask_store_all, false, true, roots);
        __syncthreads();
        auto lds_load_all = [&](int j, int lgs, auto &v) {
#pragma unroll
            for (int r = 0; r < MR_RADIX(v); ++r) v[r] = lds[(j + (r << lgs)) * LDS_STRIDE + c];
        };
        wg_fft<T, LGP, false>(lds, LDS_STRIDE, c, grp, lds_load_all, fwd_store_all, true, false, roots);
    }
}

template <typename T, int LGP, int C, int MODE>
__global__ void __launch_bounds__(C << (LGP - min_stage_lg(LGP)))
__attribute__((amdgpu_waves_per_eu(pass_waves<T, LGP, C, MODE>())))
fft_pass_kernel(cplx<T> *z, PassGeom g, SrcDesc src, DstDesc dst, Twiddles<T> tw) {
    fft_pass_body<T, LGP, C, MODE>(z, g, g.nl, g.nchunks, blockIdx.x, src, dst, tw);
}

// Two problems of the same geometry by value (the forward transforms of both
// operands of a product in one launch).
template <typename T, int LGP, int C, int MODE>
__global__ void __launch_bounds__(C << (LGP - min_stage_lg(LGP)))
__attribute__((amdgpu_waves_per_eu(pass_waves<T, LGP, C, MODE>())))
fft_pass_pair_kernel(PassProblem<T> a, PassProblem<T> b, PassGeom g, Twiddles<T> tw) {
    const int64_t bid = blockIdx.x;
    if (bid < b.wg_begin) fft_pass_body<T, LGP, C, MODE>(a.z, g, a.nl, a.nchunks, bid, a.src, a.dst, tw);
    else fft_pass_body<T, LGP, C, MODE>(b.z, g, b.nl, b.nchunks, bid - b.wg_begin, b.src, b.dst, tw);
}

// Batched: the workgroup's problem is found by binary search over wg_begin.
template <typename T, int LGP, int C, int MODE>
__global__ void __launch_bounds__(C << (LGP - min_stage_lg(LGP)))
__attribute__((amdgpu_waves_per_eu(pass_waves<T, LGP, C, MODE>())))
fft_pass_batched_kernel(const PassProblem<T> *probs, int nprob, PassGeom g, Twiddles<T> tw) {
    const int64_t bid = blockIdx.x;
    const PassProblem<T> &pp = probs[owner_of<(C << (LGP - min_stage_lg(LGP)))>(probs, nprob, bid)];
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
    if (mode == 0 && sizeof(T) == 8 && dst.kind == DST_Z && dst.aux) wr += (double)g.L * g.nl * 8.0;
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
    const size_t lds = pass_lds_bytes<T, LGP, C, MODE>();
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
    launch_kernel(name, pass_bytes<T>(MODE, g, src, dst), 0.0,
                  kern, dim3((unsigned)blocks), dim3(threads), lds, st, z, g, src, dst, tw);
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

// Small transforms (the first Newton steps) have too few workgroups to fill
// the GPU; fewer lanes per workgroup give more, shorter workgroups.  Halves
// C (32 -> 16 -> 8 -> 2) while fewer than 512 workgroups would run.
static int fewer_lanes_when_small(int C, int64_t cols, int nl_a, int nl_b) {
    auto blocks = [&](int c) { return cols * ((nl_a + c - 1) / c + (nl_b + c - 1) / c); };
    while (C > 2 && blocks(C) < 512) C = C == 32 ? 16 : C == 16 ? 8 : 2;
    return C;
}

// Automatic lanes per workgroup (tuning value 0): 32 lanes (256 contiguous
// bytes of a float64 row, 128 of a float32 one) where the 32-lane tile stays
// small enough for two workgroups per CU (float64 passes of at most 128 rows,
// float32 passes of at most 256) and there are at least 512 lanes (d >= 32);
// 16 otherwise.
int fft_lanes_per_block(bool dbl, int nl, int lgP, int mode) {
    if (nl <= 2) return 2;
    return nl >= 512 && lgP <= (dbl ? 7 : 8) ? 32 : 16;
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
    int C = nl <= 2 ? 2 : (lanes ? lanes : fft_lanes_per_block(sizeof(T) == 8, nl, lgP, mode));
    if (C == 32 && (lgP > 8 || nl <= 16)) C = 16;
    C = fewer_lanes_when_small(C, g.L >> lgP, nl, 0);
    g.nchunks = (nl + C - 1) / C;
    // The fused pass at 8 lanes (128-byte row segments, the first pass's
    // strided rows) runs about 7% faster with consecutive workgroups on
    // different columns, unless the tuning fixes the order.
    if (mode == 2 && C == 8 && order == 0) g.col_fastest = 1;
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
    const size_t lds = pass_lds_bytes<T, LGP, C, MODE>();
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
    launch_kernel(name, bytes, 0.0,
                  kern, dim3((unsigned)total), dim3(threads), lds, st, probs, nprob, g, tw);
    return hipGetLastError();
}

template <typename T, int LGP, int C, int MODE>
static hipError_t launch_pair_t(const PassProblem<T> &a, const PassProblem<T> &b, int64_t total, const PassGeom &g,
                                double bytes, const Twiddles<T> &tw, hipStream_t st) {
    const int threads = C << (LGP - min_stage_lg(LGP));
    const size_t lds = pass_lds_bytes<T, LGP, C, MODE>();
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
    launch_kernel(name, bytes, 0.0,
                  kern, dim3((unsigned)total), dim3(threads), lds, st, a, b, g, tw);
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

// 32 lanes per workgroup only up to 256-row passes (LDS).
template <typename T, int MODE>
static hipError_t launch_batched_c32(int lgP, const PassProblem<T> *probs, int nprob, int64_t total,
                                     const PassGeom &g, double bytes, const Twiddles<T> &tw, hipStream_t st) {
    switch (lgP) {
        case 1: return launch_batched_t<T, 1, 32, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 2: return launch_batched_t<T, 2, 32, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 3: return launch_batched_t<T, 3, 32, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 4: return launch_batched_t<T, 4, 32, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 5: return launch_batched_t<T, 5, 32, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 6: return launch_batched_t<T, 6, 32, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 7: return launch_batched_t<T, 7, 32, MODE>(probs, nprob, total, g, bytes, tw, st);
        case 8: return launch_batched_t<T, 8, 32, MODE>(probs, nprob, total, g, bytes, tw, st);
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
        case 32: return launch_batched_c32<T, 0>(lgP, probs, nprob, total, g, bytes, tw, st);
        case 132: return launch_batched_c32<T, 1>(lgP, probs, nprob, total, g, bytes, tw, st);
        case 232: return launch_batched_c32<T, 2>(lgP, probs, nprob, total, g, bytes, tw, st);
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
    launch_kernel("gen_outer_twiddles_kernel", 0.0, 0.0,
                  gen_outer_twiddles_kernel, dim3((unsigned)((g.total + 255) / 256)), dim3(256), 0, st, g, hi, lo);
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
    int C = nlmin <= 2 ? 2 : (lanes ? lanes : fft_lanes_per_block(sizeof(T) == 8, nlmin, plan.lgP[pass], 0));
    if (C == 32 && (plan.lgP[pass] > 8 || nlmin <= 16)) C = 16;
    const int64_t cols = g.L >> plan.lgP[pass];
    C = fewer_lanes_when_small(C, cols, a.nl, b.nl);
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
