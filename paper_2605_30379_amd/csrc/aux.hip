// Small kernels around the inversion: the Gauss-Jordan seed A(0)^-1, the
// survival sequence, contractions to scalar functionals, block extraction and
// their adjoints, residual reductions.
#include "common.h"
#include "kernels.h"

namespace mrinv {

// ---------------------------------------------------------------------------
// Gauss-Jordan inverse of the constant coefficient (Newton seed B0(0) =
// A(0)^-1, eq. (newton)).  One workgroup, partial pivoting on max |.|; a pivot
// at or below d * 2^-53 * max|A(0)| marks A(0) singular (Theorem 2.1: the
// sequence is invertible iff A(0) is) and the output becomes NaN.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gj_body(const double *A0, int d, int e0_minus, double *out64, float *out32,
                                        unsigned int *status) {
    // One wavefront; lane r owns row r of W = [A(0) | I] (kept in LDS).  Row r
    // is stored rotated by r (column j at slot (j + r) mod 2d), so the lanes'
    // simultaneous accesses to one column fall into different LDS banks.
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *W = reinterpret_cast<double *>(smem_raw);   // [d][2d]
    const int lane = threadIdx.x;
    const int w = 2 * d;
    auto at = [&](int r, int j) {
        const int s = j + r;
        return r * w + (s >= w ? s - w : s);
    };
    double amax = 0.0;
    bool finite = true;
    if (lane < d) {
        for (int j = 0; j < d; ++j) {
            const double a = A0[lane * d + j];
            const double v = e0_minus ? ((lane == j ? 1.0 : 0.0) - a) : a;
            W[at(lane, j)] = v;
            W[at(lane, d + j)] = lane == j ? 1.0 : 0.0;
            finite = finite && isfinite(v);
            amax = fmax(amax, fabs(v));
        }
    }
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    int sing = __any(!finite) ? 2 : 0;
    const double tol = d * 0x1p-53 * amax;
    // A diagonal A(0) (the identity when q(0) = 0) needs no elimination: the
    // pivots are the diagonal entries in order, and row r of the result is
    // row r of I scaled by 1 / a_rr, exactly what the general sweep computes.
    bool offdiag = false;
    if (lane < d)
        for (int j = 0; j < d; ++j) offdiag = offdiag || (j != lane && W[at(lane, j)] != 0.0);
    if (!sing && !__any(offdiag)) {
        const double arr = lane < d ? W[at(lane, lane)] : 1.0;
        const bool bad = __any(lane < d && !(fabs(arr) > tol));
        if (bad && lane == 0 && status) atomicOr(status, STATUS_SINGULAR);
        if (lane < d) {
            const double inv = 1.0 / arr;
            for (int j = 0; j < d; ++j) {
                const double v = bad ? __longlong_as_double(0x7ff8000000000000LL) : (j == lane ? 1.0 : 0.0) * inv;
                if (out64) out64[lane * d + j] = v;
                if (out32) out32[lane * d + j] = (float)v;
            }
        }
        return;
    }
    __syncthreads();
    for (int c = 0; c < d && !sing; ++c) {
        // Partial pivoting: argmax over rows c..d-1 of |W[r][c]| (lowest row on ties).
        double best = (lane >= c && lane < d) ? fabs(W[at(lane, c)]) : -1.0;
        int piv = lane;
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int op = __shfl_xor(piv, off, 64);
            if (ob > best || (ob == best && op < piv)) { best = ob; piv = op; }
        }
        if (!(best > tol)) { sing = 1; break; }
        if (piv != c) {
            for (int j = lane; j < w; j += 64) {
                const double t = W[at(c, j)];
                W[at(c, j)] = W[at(piv, j)];
                W[at(piv, j)] = t;
            }
        }
        __syncthreads();
        const double inv = 1.0 / W[at(c, c)];
        __syncthreads();
        for (int j = lane; j < w; j += 64) W[at(c, j)] *= inv;
        __syncthreads();
        if (lane < d && lane != c) {
            const double f = W[at(lane, c)];
            if (f != 0.0)
                for (int j = 0; j < w; ++j) W[at(lane, j)] = fma(-f, W[at(c, j)], W[at(lane, j)]);
        }
        __syncthreads();
    }
    const bool bad = sing != 0;
    if (bad && lane == 0 && status) atomicOr(status, sing == 1 ? STATUS_SINGULAR : STATUS_NONFINITE);
    for (int idx = lane; idx < d * d; idx += 64) {
        const int i = idx / d, j = idx - i * d;
        const double v = bad ? __longlong_as_double(0x7ff8000000000000LL) : W[at(i, d + j)];
        if (out64) out64[idx] = v;
        if (out32) out32[idx] = (float)v;
    }
}

__global__ void __launch_bounds__(64) gj_kernel(const double *A0, int d, int e0_minus, double *out64, float *out32,
                                                unsigned int *status) {
    gj_body(A0, d, e0_minus, out64, out32, status);
}

__global__ void __launch_bounds__(64) gj_batched_kernel(const GjProblem *probs, unsigned int *status) {
    const GjProblem &p = probs[blockIdx.x];
    gj_body(p.A0, p.d, p.e0_minus, p.out64, p.out32, status);
}

hipError_t gj_inverse_batched(const GjProblem *probs, int nprob, int dmax, unsigned int *status, hipStream_t st) {
    const size_t lds = (size_t)dmax * 2 * dmax * sizeof(double);
    launch_kernel("gj_batched_kernel", (double)nprob * dmax * dmax * 16.0, 2.0 * nprob * dmax * dmax * dmax,
                  gj_batched_kernel, dim3(nprob), dim3(64), lds, st, probs, status);
    return hipGetLastError();
}

hipError_t gj_inverse(const double *A0, int d, int e0_minus, double *out64, float *out32, unsigned int *status,
                      hipStream_t st) {
    const size_t lds = (size_t)d * 2 * d * sizeof(double);
    launch_kernel("gj_kernel", (double)d * d * 8.0 * 2, 2.0 * d * d * d,
                  gj_kernel, dim3(1), dim3(64), lds, st, A0, d, e0_minus, out64, out32, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// First coefficients by the coefficient recursion (Section 2.2): from the
// order-k coefficient of A*X = e0,
//     X(k) = -A(0)^-1 sum_{l=1..k} A(l) X(k-l),   k = 1..m0-1,
// with X(0) = A(0)^-1 already in out row 0.  Column c of X depends only on
// column c of earlier coefficients, so workgroup c computes column c; its
// threads split (row, range of l) and the partial sums are reduced in LDS.
// The sums are formed in float64 whatever the output type.
// ---------------------------------------------------------------------------
constexpr int SEED_THREADS = 256;

template <typename T>
__device__ __forceinline__ void seed_recursion_body(const double *A, int e0, int d, int m0, T *out, int c) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *xcol = reinterpret_cast<double *>(smem_raw);   // [m0][d] history of column c
    double *a0 = xcol + (size_t)m0 * d;                      // [d][d] A(0)^-1
    double *part = a0 + (size_t)d * d;                       // [chunks][d]
    double *Ssum = part + (size_t)SEED_THREADS;              // [d]
    const int tid = threadIdx.x;
    const int chunks = SEED_THREADS / d;                     // d <= 64 -> at least 4
    const int r = tid % d, ch = tid / d;
    const size_t dd = (size_t)d * d;
    for (int e = tid; e < d * d; e += SEED_THREADS) a0[e] = (double)out[e];
    for (int i = tid; i < d; i += SEED_THREADS) xcol[i] = (double)out[(size_t)i * d + c];
    __syncthreads();
    for (int k = 1; k < m0; ++k) {
        double s = 0.0;
        if (ch < chunks) {
            // l in [1, k], split into `chunks` interleaved ranges
            for (int l = 1 + ch; l <= k; l += chunks) {
                const double *Al = A + (size_t)l * dd + (size_t)r * d;
                const double *xk = xcol + (size_t)(k - l) * d;
                double acc = 0.0;
                for (int t = 0; t < d; ++t) acc = fma(e0 ? -Al[t] : Al[t], xk[t], acc);
                s += acc;
            }
            part[ch * d + r] = s;
        }
        __syncthreads();
        if (tid < d) {
            double tot = 0.0;
            for (int q = 0; q < chunks; ++q) tot += part[q * d + tid];
            Ssum[tid] = tot;
        }
        __syncthreads();
        if (tid < d) {
            double v = 0.0;
            for (int u = 0; u < d; ++u) v = fma(a0[tid * d + u], Ssum[u], v);
            v = -v;
            xcol[(size_t)k * d + tid] = v;
            out[(size_t)k * dd + (size_t)tid * d + c] = (T)v;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(SEED_THREADS)
seed_recursion_kernel(const double *A, int e0, int d, int m0, T *out) {
    seed_recursion_body<T>(A, e0, d, m0, out, blockIdx.x);
}

// Batched: one workgroup per (problem, column); the problem is found by
// binary search over col_begin.
template <typename T>
__global__ void __launch_bounds__(SEED_THREADS) seed_recursion_batched_kernel(const SeedProblem *probs, int nprob) {
    int lo = 0, hi = nprob - 1;
    const int bid = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].col_begin <= bid) lo = mid;
        else hi = mid - 1;
    }
    const SeedProblem &p = probs[lo];
    seed_recursion_body<T>(p.A, p.e0, p.d, p.m0, (T *)p.out, bid - p.col_begin);
}

template <typename T>
hipError_t seed_recursion_batched(const SeedProblem *probs, int nprob, int total_cols, int dmax, int m0max,
                                  hipStream_t st) {
    const size_t lds = seed_lds_bytes(m0max, dmax);
    launch_kernel(sizeof(T) == 8 ? "seed_recursion_batched_kernel<double>" : "seed_recursion_batched_kernel<float>",
                  0.0, 0.0, seed_recursion_batched_kernel<T>, dim3(total_cols), dim3(SEED_THREADS), lds, st, probs,
                  nprob);
    return hipGetLastError();
}
template hipError_t seed_recursion_batched<double>(const SeedProblem *, int, int, int, int, hipStream_t);
template hipError_t seed_recursion_batched<float>(const SeedProblem *, int, int, int, int, hipStream_t);

size_t seed_lds_bytes(int m0, int d) {
    return ((size_t)m0 * d + (size_t)d * d + SEED_THREADS + d) * sizeof(double);
}

template <typename T>
hipError_t seed_recursion(const double *A, int e0, int d, int m0, T *out, hipStream_t st) {
    const size_t lds = seed_lds_bytes(m0, d);
    launch_kernel(sizeof(T) == 8 ? "seed_recursion_kernel<double>" : "seed_recursion_kernel<float>",
                  (double)m0 * d * d * 8.0 * 2, (double)m0 * m0 * d * d * d, seed_recursion_kernel<T>, dim3(d),
                  dim3(SEED_THREADS), lds, st, A, e0, d, m0, out);
    return hipGetLastError();
}

template hipError_t seed_recursion<double>(const double *, int, int, int, double *, hipStream_t);
template hipError_t seed_recursion<float>(const double *, int, int, int, float *, hipStream_t);

// ---------------------------------------------------------------------------
// Inclusive scan over time of w lanes, Y[k][i] <- a + b * sum_{l<=k} Y[l][i]
// (reverse != 0: sum over l >= k), w <= 256.  Three launches: chunk totals,
// an exclusive scan of the totals, and the rescan of every chunk from its
// offset.  Inside a chunk of SCAN_ROWS time steps, thread (s, i) of a
// workgroup handles lane i over sub-segment s; reads of one time step are
// contiguous across lanes.
// ---------------------------------------------------------------------------
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ROWS = 1024;

__device__ __forceinline__ int64_t scan_row(int64_t k, int64_t n, int reverse) { return reverse ? n - 1 - k : k; }

// Thread layout of one chunk: lanes i < w, sub-segments s < nsub = 256 / w.
struct ScanGeom {
    int w, nsub, i, s;
    int64_t k0, k1;     // rows of this thread's sub-segment
    bool ok;
};

__device__ __forceinline__ ScanGeom scan_geom(int64_t n, int w, int64_t chunk) {
    ScanGeom g;
    g.w = w;
    g.nsub = SCAN_THREADS / w;
    g.i = threadIdx.x % w;
    g.s = threadIdx.x / w;
    g.ok = g.s < g.nsub;
    const int64_t c0 = chunk * SCAN_ROWS, c1 = min(n, c0 + SCAN_ROWS);
    const int64_t seg = (SCAN_ROWS + g.nsub - 1) / g.nsub;
    g.k0 = min(c1, c0 + g.s * seg);
    g.k1 = min(c1, g.k0 + seg);
    return g;
}

__global__ void __launch_bounds__(SCAN_THREADS) scan_totals_kernel(const double *Y, int64_t n, int w, int reverse,
                                                                   double *tot) {
    __shared__ double part[SCAN_THREADS];
    const ScanGeom g = scan_geom(n, w, blockIdx.x);
    double s = 0.0;
    if (g.ok)
        for (int64_t k = g.k0; k < g.k1; ++k) s += Y[scan_row(k, n, reverse) * w + g.i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < w) {
        double t = 0.0;
        for (int u = 0; u < g.nsub; ++u) t += part[u * w + threadIdx.x];
        tot[(int64_t)blockIdx.x * w + threadIdx.x] = t;
    }
}

// Exclusive scan of the chunk totals per lane, in place (one thread per lane).
__global__ void __launch_bounds__(SCAN_THREADS) scan_offsets_kernel(double *tot, int64_t nchunks, int w) {
    const int i = threadIdx.x;
    if (i >= w) return;
    double run = 0.0;
    for (int64_t c = 0; c < nchunks; ++c) {
        const double v = tot[c * w + i];
        tot[c * w + i] = run;
        run += v;
    }
}

__global__ void __launch_bounds__(SCAN_THREADS) scan_apply_kernel(double *Y, int64_t n, int w, int reverse,
                                                                  const double *off, double a, double b) {
    __shared__ double part[SCAN_THREADS];
    const ScanGeom g = scan_geom(n, w, blockIdx.x);
    double s = 0.0;
    if (g.ok)
        for (int64_t k = g.k0; k < g.k1; ++k) s += Y[scan_row(k, n, reverse) * w + g.i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (!g.ok) return;
    double run = off[(int64_t)blockIdx.x * w + g.i];
    for (int u = 0; u < g.s; ++u) run += part[u * w + g.i];
    for (int64_t k = g.k0; k < g.k1; ++k) {
        double &y = Y[scan_row(k, n, reverse) * w + g.i];
        run += y;
        y = a + b * run;
    }
}

// tmp: ceil(n / SCAN_ROWS) * w doubles.
static hipError_t scan_lanes(double *Y, int64_t n, int w, int reverse, double a, double b, double *tmp,
                             hipStream_t st) {
    if (w < 1 || w > SCAN_THREADS) return hipErrorInvalidValue;
    const int64_t nch = (n + SCAN_ROWS - 1) / SCAN_ROWS;
    launch_kernel("scan_totals_kernel", (double)n * w * 8.0, 0.0, scan_totals_kernel, dim3((unsigned)nch),
                  dim3(SCAN_THREADS), 0, st, Y, n, w, reverse, tmp);
    launch_kernel("scan_offsets_kernel", 2.0 * nch * w * 8.0, 0.0, scan_offsets_kernel, dim3(1), dim3(SCAN_THREADS), 0,
                  st, tmp, nch, w);
    launch_kernel("scan_apply_kernel", 2.0 * n * w * 8.0, 0.0, scan_apply_kernel, dim3((unsigned)nch),
                  dim3(SCAN_THREADS), 0, st, Y, n, w, reverse, (const double *)tmp, a, b);
    return hipGetLastError();
}

size_t scan_tmp_bytes(int64_t n, int w) { return (size_t)((n + SCAN_ROWS - 1) / SCAN_ROWS) * w * sizeof(double); }

// rho[k][i] = sum_j q_ij(k) for k >= 1, rho[0][i] = 0.  Row (k, i) is summed
// by a group of G = 2^ceil(log2 d) lanes of one wavefront (coalesced reads,
// butterfly reduction).
__global__ void rowsum_kernel(const double *q, int d, int lgG, int64_t n, double *rho) {
    const int G = 1 << lgG;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = gid >> lgG;            // (k, i) flattened
    const int j = (int)(gid & (G - 1));
    const bool in = row < n * d;
    double v = 0.0;
    if (in && j < d && row >= d) v = q[row * d + j];
    for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    if (in && j == 0) rho[row] = v;
}

// Survival sequence Hbar(k)_ii = 1 - sum_j sum_{l=1..k} q_ij(l) (Section 4.1).
hipError_t survival(const double *q, int d, int64_t n, double *hb, double *tmp, hipStream_t st) {
    int lgG = 0;
    while ((1 << lgG) < d) ++lgG;
    const int64_t total = (n * d) << lgG;
    launch_kernel("rowsum_kernel", (double)n * d * (d + 1) * 8.0, 0.0,
                  rowsum_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, q, d, lgG, n, hb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scan_lanes(hb, n, d, 0, 1.0, -1.0, tmp, st);
}

// q_bar(l)[i][j] += -sum_{k>=l} hb_bar(k)[i] for l >= 1.  hbb is scanned in place.
__global__ void bcast_sub_kernel(const double *s, int d, int64_t n, double *qb) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n * d * d) return;
    const int64_t k = gid / ((int64_t)d * d);
    if (k == 0) return;
    const int i = (int)((gid / d) % d);
    qb[gid] -= s[k * d + i];
}

hipError_t survival_backward(const double *hbb, int d, int64_t n, double *qb, double *tmp, hipStream_t st) {
    hipError_t e = scan_lanes(const_cast<double *>(hbb), n, d, 1, 0.0, 1.0, tmp, st);
    if (e != hipSuccess) return e;
    const int64_t total = n * d * d;
    hipLaunchKernelGGL(bcast_sub_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, hbb, d, n, qb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Contractions out(k) = offset + scale * u^T X(k) v (optionally cumulative).
// One wavefront per time step.
// ---------------------------------------------------------------------------
__global__ void contract_kernel(const double *X, int64_t n, int rows, int cols, const double *u, const double *v,
                                double *out) {
    const int lane = threadIdx.x & 63;
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (k >= n) return;
    const int rc = rows * cols;
    const double *xk = X + k * rc;
    double s = 0.0;
    for (int e = lane; e < rc; e += 64) {
        const int i = e / cols, j = e - i * cols;
        s += u[i] * xk[e] * v[j];
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) out[k] = s;
}

__global__ void affine_kernel(double *y, int64_t n, double a, double b) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) y[k] = a + b * y[k];
}

hipError_t contract(const double *X, int64_t n, int rows, int cols, const double *u, const double *v,
                    int cumulative, double offset, double scale, double *out, double *tmp, hipStream_t st) {
    const int64_t threads = n * 64;
    hipLaunchKernelGGL(contract_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, X, n, rows, cols,
                       u, v, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (cumulative) return scan_lanes(out, n, 1, 0, offset, scale, tmp, st);
    hipLaunchKernelGGL(affine_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, n, offset, scale);
    return hipGetLastError();
}

// X_bar(l) += scale * w(l) u v^T
__global__ void outer_accum_kernel(const double *w, int64_t n, int rows, int cols, const double *u,
                                   const double *v, double scale, double *Xb) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t rc = (int64_t)rows * cols;
    if (gid >= n * rc) return;
    const int64_t k = gid / rc;
    const int e = (int)(gid - k * rc);
    const int i = e / cols, j = e - i * cols;
    Xb[gid] += scale * w[k] * u[i] * v[j];
}

hipError_t contract_backward(const double *ob, int64_t n, int rows, int cols, const double *u, const double *v,
                             int cumulative, double scale, double *Xb, double *tmp, hipStream_t st) {
    // The cumulative form needs the reverse cumulative sum of out_bar; it is
    // formed in place in the caller's out_bar buffer copy (see api).
    if (cumulative) {
        hipError_t e = scan_lanes(const_cast<double *>(ob), n, 1, 1, 0.0, 1.0, tmp, st);
        if (e != hipSuccess) return e;
    }
    const int64_t total = n * rows * cols;
    hipLaunchKernelGGL(outer_accum_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, ob, n, rows, cols,
                       u, v, scale, Xb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block extraction and its adjoint.
// ---------------------------------------------------------------------------
__global__ void gather_kernel(const double *X, int64_t n, int rows, int cols, const int *ri, int nr, const int *ci,
                              int nc, double *Y) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t rc = (int64_t)nr * nc;
    if (gid >= n * rc) return;
    const int64_t k = gid / rc;
    const int e = (int)(gid - k * rc);
    const int a = e / nc, b = e - a * nc;
    Y[gid] = X[(k * rows + ri[a]) * cols + ci[b]];
}

hipError_t gather_block(const double *X, int64_t n, int rows, int cols, const int *ri, int nr, const int *ci,
                        int nc, double *Y, hipStream_t st) {
    const int64_t total = n * nr * nc;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, X, n, rows, cols, ri,
                       nr, ci, nc, Y);
    return hipGetLastError();
}

__global__ void scatter_add_kernel(const double *Yb, int64_t n, int rows, int cols, const int *ri, int nr,
                                   const int *ci, int nc, double *Xb) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t rc = (int64_t)nr * nc;
    if (gid >= n * rc) return;
    const int64_t k = gid / rc;
    const int e = (int)(gid - k * rc);
    const int a = e / nc, b = e - a * nc;
    Xb[(k * rows + ri[a]) * cols + ci[b]] += Yb[gid];
}

hipError_t scatter_block_add(const double *Yb, int64_t n, int rows, int cols, const int *ri, int nr,
                             const int *ci, int nc, double *Xb, hipStream_t st) {
    const int64_t total = n * nr * nc;
    hipLaunchKernelGGL(scatter_add_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, Yb, n, rows, cols,
                       ri, nr, ci, nc, Xb);
    return hipGetLastError();
}

__global__ void put_small_kernel(SmallVecArgs v, int *ci, int *di, double *alpha, double *ones) {
    const int t = threadIdx.x;
    if (t < v.nci) ci[t] = v.ci[t];
    if (t < v.ndi) di[t] = v.di[t];
    if (t < v.nalpha) alpha[t] = v.alpha[t];
    if (t < v.nones) ones[t] = v.ones[t];
}

hipError_t put_small_vectors(const SmallVecArgs &v, int *ci, int *di, double *alpha, double *ones, hipStream_t st) {
    if (v.nci > SMALL_MAX || v.ndi > SMALL_MAX || v.nalpha > SMALL_MAX || v.nones > SMALL_MAX)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(put_small_kernel, dim3(1), dim3(SMALL_MAX), 0, st, v, ci, di, alpha, ones);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Mean-value discretisation of a continuous-time Markov renewal equation
// (Section 4.2): from the kernel on the grid, Qs[m] = Q(m h) for m = 0..n,
//   Qbar_h(m) = (Delta Q_h(m) + Delta Q_h(m+1)) / 2,  Delta Q_h(0) = 0,
// and the right-hand side of eq. (mre-solution),
//   R(m) = L_h(m) - (1/2) Delta Q_h(m+1) L_h(0)
// (the product Delta+Q_h * (L_h(0) e0) has this single term per m).
// ---------------------------------------------------------------------------
__global__ void mre_qbar_kernel(const double *Qs, int64_t n, int d, double *Qbar) {
    const int64_t dd = (int64_t)d * d;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n * dd) return;
    const int64_t m = gid / dd;
    const double q0 = Qs[gid], q1 = Qs[gid + dd];
    const double dm = m > 0 ? q0 - Qs[gid - dd] : 0.0;
    Qbar[gid] = 0.5 * (dm + (q1 - q0));
}

__global__ void mre_rhs_kernel(const double *Qs, const double *L, int64_t n, int d, int r, double *R) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t dr = (int64_t)d * r;
    if (gid >= n * dr) return;
    const int64_t m = gid / dr;
    const int e = (int)(gid - m * dr);
    const int i = e / r, c = e - i * r;
    const int64_t dd = (int64_t)d * d;
    const double *q1 = Qs + (m + 1) * dd + (int64_t)i * d, *q0 = Qs + m * dd + (int64_t)i * d;
    double s = 0.0;
    for (int t = 0; t < d; ++t) s += (q1[t] - q0[t]) * L[(int64_t)t * r + c];
    R[gid] = L[gid] - 0.5 * s;
}

hipError_t mre_prepare(const double *Qs, const double *L, int64_t n, int d, int r, double *Qbar, double *R,
                       hipStream_t st) {
    const int64_t t1 = n * d * d, t2 = n * d * r;
    launch_kernel("mre_qbar_kernel", (double)t1 * 8.0 * 3.0, 0.0, mre_qbar_kernel,
                  dim3((unsigned)((t1 + 255) / 256)), dim3(256), 0, st, Qs, n, d, Qbar);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    launch_kernel("mre_rhs_kernel", ((double)t1 * 2.0 + (double)t2 * 2.0) * 8.0, (double)t2 * 3.0 * d,
                  mre_rhs_kernel, dim3((unsigned)((t2 + 255) / 256)), dim3(256), 0, st, Qs, L, n, d, r, R);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gauss-Jordan elimination over the truncated series ring C[[x]]/<x^n>
// (Appendix, Gauss-Jordan paragraph).  The augmented sequence W = [A | I] is
// held time-major, W[k][r][c] with 2d columns.  These kernels do the
// bookkeeping of one pivot step; the series products run through the
// transform and product kernels.
// ---------------------------------------------------------------------------
__global__ void gjs_init_kernel(const double *A, int e0_minus, int64_t n, int d, double *W) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int w = 2 * d;
    if (gid >= n * d * w) return;
    const int64_t k = gid / ((int64_t)d * w);
    const int e = (int)(gid - k * d * w);
    const int r = e / w, c = e - r * w;
    double v;
    if (c < d) {
        v = A[(k * d + r) * d + c];
        if (e0_minus) v = (k == 0 && r == c ? 1.0 : 0.0) - v;
    } else {
        v = (k == 0 && c - d == r) ? 1.0 : 0.0;
    }
    W[gid] = v;
}

// Pivot of column i: the row r >= i whose series has the largest |constant
// coefficient| (the constant coefficients follow Gauss-Jordan on A(0)
// exactly).  A pivot with |W(0)_ri| <= d 2^-53 max|A(0)| marks A(0) singular.
// aux[0] holds max|A(0)|, set at i = 0.  One wavefront.
__global__ void gjs_pivot_kernel(const double *W, int d, int i, int *piv, double *aux, unsigned int *status) {
    const int lane = threadIdx.x;
    const int w = 2 * d;
    double amax;
    if (i == 0) {
        double m = 0.0;
        for (int e = lane; e < d * d; e += 64) m = fmax(m, fabs(W[(e / d) * w + e % d]));
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
        amax = m;                       // every lane holds the maximum after the butterfly
        if (lane == 0) aux[0] = m;
    } else {
        amax = aux[0];
    }
    double best = -1.0;
    int row = i;
    if (lane >= i && lane < d) {
        best = fabs(W[lane * w + i]);
        row = lane;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int orow = __shfl_xor(row, o, 64);
        if (ob > best || (ob == best && orow < row)) {
            best = ob;
            row = orow;
        }
    }
    if (lane == 0) {
        piv[i] = row;
        if (!(best > d * 1.1102230246251565e-16 * amax)) atomicOr(status, STATUS_SINGULAR);
    }
}

// Swap rows i and piv[i] of W over the whole horizon.
__global__ void gjs_swap_kernel(double *W, int64_t n, int d, int i, const int *piv) {
    const int p = piv[i];
    if (p == i) return;
    const int w = 2 * d;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n * w) return;
    const int64_t k = gid / w;
    const int c = (int)(gid - k * w);
    double *a = W + (k * d + i) * w + c, *b = W + (k * d + p) * w + c;
    const double t = *a;
    *a = *b;
    *b = t;
}

// u(k) = W(k)_ii (the pivot series) and col(k)_r = W(k)_ri for r != i,
// col(k)_i = 0 (the multipliers of the elimination).
__global__ void gjs_gather_kernel(const double *W, int64_t n, int d, int i, double *u, double *col) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n * d) return;
    const int64_t k = gid / d;
    const int r = (int)(gid - k * d);
    const double v = W[(k * d + r) * 2 * d + i];
    col[gid] = r == i ? 0.0 : v;
    if (r == i) u[k] = v;
}

// Ainv(k) = right block of W(k).
__global__ void gjs_result_kernel(const double *W, int64_t n, int d, double *out, unsigned int *status) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n * d * d) return;
    const int64_t k = gid / ((int64_t)d * d);
    const int e = (int)(gid - k * d * d);
    const int r = e / d, c = e - r * d;
    const double v = W[(k * d + r) * 2 * d + d + c];
    out[gid] = v;
    if (status && !isfinite(v)) atomicOr(status, STATUS_NONFINITE);
}

hipError_t gjs_init(const double *A, int e0_minus, int64_t n, int d, double *W, hipStream_t st) {
    const int64_t t = n * d * 2 * d;
    launch_kernel("gjs_init_kernel", (double)t * 8.0 * 1.5, 0.0, gjs_init_kernel, dim3((unsigned)((t + 255) / 256)),
                  dim3(256), 0, st, A, e0_minus, n, d, W);
    return hipGetLastError();
}

hipError_t gjs_pivot_step(double *W, int64_t n, int d, int i, int *piv, double *aux, double *u, double *col,
                          unsigned int *status, hipStream_t st) {
    launch_kernel("gjs_pivot_kernel", 0.0, 0.0, gjs_pivot_kernel, dim3(1), dim3(64), 0, st, (const double *)W, d, i,
                  piv, aux, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t t1 = n * 2 * d;
    launch_kernel("gjs_swap_kernel", (double)t1 * 32.0, 0.0, gjs_swap_kernel, dim3((unsigned)((t1 + 255) / 256)),
                  dim3(256), 0, st, W, n, d, i, (const int *)piv);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t t2 = n * d;
    launch_kernel("gjs_gather_kernel", (double)t2 * 16.0 + (double)n * 8.0, 0.0, gjs_gather_kernel,
                  dim3((unsigned)((t2 + 255) / 256)), dim3(256), 0, st, (const double *)W, n, d, i, u, col);
    return hipGetLastError();
}

hipError_t gjs_result(const double *W, int64_t n, int d, double *out, unsigned int *status, hipStream_t st) {
    const int64_t t = n * d * d;
    launch_kernel("gjs_result_kernel", (double)t * 16.0, 0.0, gjs_result_kernel, dim3((unsigned)((t + 255) / 256)),
                  dim3(256), 0, st, W, n, d, out, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fills and residual reductions.
// ---------------------------------------------------------------------------
__global__ void fill_f64_kernel(double *p, int64_t count, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}
__global__ void fill_u32_kernel(unsigned int *p, int64_t count, unsigned int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}
hipError_t fill_f64(double *p, int64_t count, double v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}
hipError_t fill_u32(unsigned int *p, int64_t count, unsigned int v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

// acc[0] += sum_k ||R_L(k)||_F, acc[1] += sum_k ||R_R(k)||_F, acc[2] = max |R_L|
// (max taken through the bit pattern of non-negative doubles).  One wavefront
// per time step.
__global__ void resid_kernel(const double *RL, const double *RR, int d, int64_t n, double *acc) {
    const int lane = threadIdx.x & 63;
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (k >= n) return;
    const int d2 = d * d;
    double sl = 0.0, sr = 0.0, mx = 0.0;
    for (int e = lane; e < d2; e += 64) {
        const double a = RL[k * d2 + e], b = RR[k * d2 + e];
        sl += a * a;
        sr += b * b;
        mx = fmax(mx, fabs(a));
    }
    for (int off = 32; off > 0; off >>= 1) {
        sl += __shfl_xor(sl, off, 64);
        sr += __shfl_xor(sr, off, 64);
        mx = fmax(mx, __shfl_xor(mx, off, 64));
    }
    if (lane == 0) {
        atomicAdd(&acc[0], sqrt(sl));
        atomicAdd(&acc[1], sqrt(sr));
        atomicMax((unsigned long long *)&acc[2], (unsigned long long)__double_as_longlong(mx));
    }
}

hipError_t residual_norms(const double *RL, const double *RR, int d, int64_t n, double *acc, hipStream_t st) {
    const int64_t threads = n * 64;
    hipLaunchKernelGGL(resid_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, RL, RR, d, n, acc);
    return hipGetLastError();
}

}  // namespace mrinv
