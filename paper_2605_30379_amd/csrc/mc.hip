// Pathwise Monte Carlo of a finite semi-Markov process observed on a time
// grid: the independent validation of the continuous-time approximations in
// Section 5.2 (the lognormal model, 10^6 trajectories, pointwise 95% normal
// confidence intervals).
//
// A trajectory starts in the initial state at time 0.  At each jump from
// state i it draws the next state j from row i of the embedded matrix and a
// sojourn from F_ij (the kernel Q_ij(t) = P_ij F_ij(t)), so its law is the
// process of the kernel.  On the grid t_m = m h (m < n) it counts, per m,
// the trajectories in an up state at t_m (availability) and those that have
// not entered a down state up to t_m (reliability).  The state at t_m is the
// one whose sojourn [a, b) holds m, i.e. ceil(a/h) <= m < ceil(b/h).  Counts
// go into difference arrays with integer atomics (exact, in any order) and
// a scan turns them into the estimates.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC 2011), a counter-based generator.
// Jump k of trajectory t uses the two blocks of counter (k, s, t_lo, t_hi),
// s = 0, 1, under the key (seed_lo, seed_hi): block 0 gives the uniform that
// picks the next state and the first uniform of the sojourn, block 1 the
// second.  A uniform is 53 bits of two words, (x + 1/2) 2^-53, in (0, 1).
#include <stdio.h>

#include "common.h"
#include "kernels.h"

namespace mrinv {

__device__ __forceinline__ void philox_round(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

// Ten rounds with the key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        philox_round(c, k0, k1);
    }
}

__device__ __forceinline__ double u01(uint32_t a, uint32_t b) {
    const uint64_t x = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)x + 0.5) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ int64_t grid_ceil(double t, double step, int64_t n) {
    const double q = ceil(t / step);
    return q >= (double)n ? n : (int64_t)q;
}

__global__ void mc_kernel(McModel m, double step, int64_t n, int64_t trajectories, uint32_t key0, uint32_t key1,
                          int *diffA, int *diffR, double *tau_out, int *jumps_out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= trajectories) return;
    const double tmax = (double)(n - 1) * step;
    int s = m.initial;
    double now = 0.0;
    double tau = m.up[s] ? -1.0 : 0.0;   // first entrance time into the down set (-1: none by tmax)
    if (m.up[s]) atomicAdd(&diffR[0], 1);
    int jumps = 0;
    const uint32_t tlo = (uint32_t)t, thi = (uint32_t)((uint64_t)t >> 32);
    for (uint32_t k = 0; k < MC_MAX_JUMPS && now <= tmax; ++k) {
        uint32_t b0[4] = {k, 0u, tlo, thi}, b1[4] = {k, 1u, tlo, thi};
        philox4x32_10(b0, key0, key1);
        philox4x32_10(b1, key0, key1);
        const double un = u01(b0[0], b0[1]), ua = u01(b0[2], b0[3]), ub = u01(b1[0], b1[1]);
        // next state: the first j with un < cumulative row sum (the last state with
        // positive probability when rounding leaves the row sum below un)
        int j = m.last[s];
        for (int c = 0; c < m.d; ++c)
            if (un < m.cum[s * MC_MAX_D + c]) {
                j = c;
                break;
            }
        const double p1 = m.p1[s * MC_MAX_D + j], p2 = m.p2[s * MC_MAX_D + j];
        double T;
        if (m.family == 0) {
            const double z = sqrt(-2.0 * log(ua)) * cos(6.283185307179586476925 * ub);
            T = exp(p1 + p2 * z);                        // lognormal(mu, sigma)
        } else if (m.family == 1) {
            T = p2 * pow(-log(ua), 1.0 / p1);            // Weibull(shape, scale)
        } else {
            T = -log(ua) / p1;                           // exponential(rate)
        }
        const double next = now + T;
        if (m.up[s]) {
            const int64_t ia = grid_ceil(now, step, n), ib = grid_ceil(next, step, n);
            if (ia < ib) {
                atomicAdd(&diffA[ia], 1);
                atomicAdd(&diffA[ib], -1);
            }
        }
        now = next;
        s = j;
        if (now <= tmax) {
            ++jumps;
            if (tau < 0.0 && !m.up[s]) {
                tau = now;
                atomicAdd(&diffR[grid_ceil(now, step, n)], -1);
            }
        }
    }
    if (tau_out) tau_out[t] = tau;
    if (jumps_out) jumps_out[t] = jumps;
}

// est[m] = (sum_{i <= m} diff[i]) / trajectories for both difference arrays;
// one workgroup, each thread a contiguous segment.
__global__ void __launch_bounds__(1024) mc_scan_kernel(const int *diffA, const int *diffR, int64_t n, double inv,
                                                       double *A, double *R) {
    __shared__ long long sa[1024], sr[1024];
    const int tid = threadIdx.x;
    const int64_t seg = (n + 1023) / 1024;
    const int64_t a = tid * seg, b = a + seg < n ? a + seg : n;
    long long ta = 0, tr = 0;
    for (int64_t i = a; i < b; ++i) {
        ta += diffA[i];
        tr += diffR[i];
    }
    sa[tid] = ta;
    sr[tid] = tr;
    __syncthreads();
    if (tid == 0) {
        long long ra = 0, rr = 0;
        for (int i = 0; i < 1024; ++i) {
            const long long xa = sa[i], xr = sr[i];
            sa[i] = ra;
            sr[i] = rr;
            ra += xa;
            rr += xr;
        }
    }
    __syncthreads();
    long long ra = sa[tid], rr = sr[tid];
    for (int64_t i = a; i < b; ++i) {
        ra += diffA[i];
        rr += diffR[i];
        A[i] = (double)ra * inv;
        R[i] = (double)rr * inv;
    }
}

hipError_t semi_markov_mc(const McModel &m, double step, int64_t n, int64_t trajectories, uint64_t seed, double *A,
                          double *R, double *tau, int *jumps, int *diffA, int *diffR, hipStream_t st) {
    hipError_t e = fill_u32((unsigned int *)diffA, n + 1, 0u, st);
    if (e == hipSuccess) e = fill_u32((unsigned int *)diffR, n + 1, 0u, st);
    if (e != hipSuccess) return e;
    const int64_t blocks = (trajectories + 255) / 256;
    launch_kernel("mc_kernel", 0.0, 0.0, mc_kernel, dim3((unsigned)blocks), dim3(256), 0, st, m, step, n, trajectories,
                  (uint32_t)seed, (uint32_t)(seed >> 32), diffA, diffR, tau, jumps);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    launch_kernel("mc_scan_kernel", (double)n * 24.0, 0.0, mc_scan_kernel, dim3(1), dim3(1024), 0, st,
                  (const int *)diffA, (const int *)diffR, n, 1.0 / (double)trajectories, A, R);
    return hipGetLastError();
}

}  // namespace mrinv
