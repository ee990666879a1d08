// Optional per-kernel timing.  When a handle enables it, every kernel launch
// of the library carries a start and a stop event stamped at the kernel's own
// start and end (hipExtLaunchKernelGGL) and is tagged with the kernel's name
// and the algorithmic bytes and flops of that launch; mrinv_kernel_stats()
// aggregates them per kernel name.
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "../../include/mrinv.h"
#include "kernels.h"

namespace mrinv {

struct TimedLaunch {
    std::string name;
    hipEvent_t start, stop;
    double bytes, flops;
};

struct Timer {
    std::vector<TimedLaunch> launches;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        (void)hipEventCreate(&e);
        return e;
    }
};

static thread_local Timer *g_timer = nullptr;

void timer_activate(void *timer, hipStream_t) { g_timer = (Timer *)timer; }

bool timed_events(const char *name, double bytes, double flops, hipEvent_t *start, hipEvent_t *stop) {
    if (!g_timer) return false;
    TimedLaunch t;
    t.name = name;
    t.start = g_timer->get();
    t.stop = g_timer->get();
    t.bytes = bytes;
    t.flops = flops;
    g_timer->launches.push_back(t);
    *start = t.start;
    *stop = t.stop;
    return true;
}

void *timer_create() { return new Timer(); }

void timer_destroy(void *t) {
    Timer *tm = (Timer *)t;
    if (!tm) return;
    for (auto &l : tm->launches) {
        (void)hipEventDestroy(l.start);
        (void)hipEventDestroy(l.stop);
    }
    for (auto e : tm->pool) (void)hipEventDestroy(e);
    delete tm;
}

void timer_reset(void *t) {
    Timer *tm = (Timer *)t;
    for (auto &l : tm->launches) {
        tm->pool.push_back(l.start);
        tm->pool.push_back(l.stop);
    }
    tm->launches.clear();
}

int timer_stats(void *t, hipStream_t st, mrinv_kernel_stat_t *out, int max_out) {
    Timer *tm = (Timer *)t;
    (void)hipStreamSynchronize(st);
    std::map<std::string, mrinv_kernel_stat_t> agg;
    std::vector<std::string> order;
    for (auto &l : tm->launches) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, l.start, l.stop) != hipSuccess) ms = 0.f;
        auto it = agg.find(l.name);
        if (it == agg.end()) {
            mrinv_kernel_stat_t s{};
            strncpy(s.name, l.name.c_str(), sizeof(s.name) - 1);
            it = agg.emplace(l.name, s).first;
            order.push_back(l.name);
        }
        it->second.launches += 1;
        it->second.total_ms += ms;
        it->second.bytes += l.bytes;
        it->second.flops += l.flops;
    }
    int k = 0;
    for (auto &nm : order) {
        if (k < max_out && out) out[k] = agg[nm];
        ++k;
    }
    return k;
}

// ---------------------------------------------------------------------------
// HBM probes: the practical read + write rate of two access patterns, the
// ceilings against which the kernels' bandwidth is judged.  The copy moves
// one 16-byte element per thread.  The pass patterns read and write, in
// place, every element of an L x PROBE_NL complex-double array with the
// addressing of one 512-row FFT pass of fft.hip: workgroup (chunk, column),
// lanes [chunk C, chunk C + C) of the column's 512 rows, each thread R rows
// at stride 512/R rows; the first pass takes rows m + (L/512) i, the last
// pass rows 512 m + i.  They add 1 to the real part of every element, so a
// test can check that each element is visited exactly once per launch.
// ---------------------------------------------------------------------------
constexpr int PROBE_NL = 2048;   // complex lanes per row (d = 64)
constexpr int PROBE_LGP = 9;     // rows per column

__global__ void __launch_bounds__(256) hbm_copy_kernel(const double2 *__restrict__ a, double2 *__restrict__ b,
                                                       int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

template <int R, int C>
__global__ void __launch_bounds__(C * ((1 << PROBE_LGP) / R)) hbm_pass_kernel(double2 *z, int lgL, int first) {
    constexpr int P = 1 << PROBE_LGP, NCH = PROBE_NL / C;
    const int64_t blk = blockIdx.x;
    const int64_t col = blk / NCH;
    const int chunk = (int)(blk % NCH);
    const int c = threadIdx.x % C, grp = threadIdx.x / C;
    const int64_t S = first ? (int64_t)1 << (lgL - PROBE_LGP) : 1;
    const int64_t base = first ? col : col << PROBE_LGP;
    const int64_t rs = S * PROBE_NL;
    double2 *q = z + base * PROBE_NL + chunk * C + c + grp * rs;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = q[r * (P / R) * rs];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        v[r].x += 1.0;
        q[r * (P / R) * rs] = v[r];
    }
}

// One launch of `pattern` over buf (bytes already checked by the caller).
static hipError_t hbm_launch(hipStream_t st, void *buf, size_t bytes, int pattern, int lanes, double *moved) {
    if (pattern == 0) {
        const int64_t n = (int64_t)(bytes / 2 / sizeof(double2));
        const double2 *a = (const double2 *)buf;
        double2 *b = (double2 *)buf + n;
        hbm_copy_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(a, b, n);
        *moved = 2.0 * (double)n * sizeof(double2);
        return hipGetLastError();
    }
    int lgL = 0;
    while (((size_t)2 << lgL) * PROBE_NL * sizeof(double2) <= bytes) ++lgL;
    const int64_t L = (int64_t)1 << lgL;
    const unsigned blocks = (unsigned)((L >> PROBE_LGP) * (PROBE_NL / lanes));
    double2 *z = (double2 *)buf;
    const int first = pattern == 1;
    if (lanes == 8) hbm_pass_kernel<8, 8><<<dim3(blocks), dim3(8 * 64), 0, st>>>(z, lgL, first);
    else if (lanes == 16) hbm_pass_kernel<8, 16><<<dim3(blocks), dim3(16 * 64), 0, st>>>(z, lgL, first);
    else hbm_pass_kernel<16, 32><<<dim3(blocks), dim3(32 * 32), 0, st>>>(z, lgL, first);
    *moved = 2.0 * (double)L * PROBE_NL * sizeof(double2);
    return hipGetLastError();
}

// Smallest buffer the pass patterns accept: two columns of 512 rows.
size_t hbm_probe_min_bytes() { return ((size_t)2 << PROBE_LGP) * PROBE_NL * sizeof(double2); }

hipError_t hbm_probe(hipStream_t st, void *buf, size_t bytes, int pattern, int lanes, int reps, double *gbps) {
    hipEvent_t e0, e1;
    hipError_t err = hipEventCreate(&e0);
    if (err != hipSuccess) return err;
    err = hipEventCreate(&e1);
    if (err != hipSuccess) {
        (void)hipEventDestroy(e0);
        return err;
    }
    double best = 0.0;
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
        double moved = 0.0;
        err = hipEventRecord(e0, st);
        if (err == hipSuccess) err = hbm_launch(st, buf, bytes, pattern, lanes, &moved);
        if (err == hipSuccess) err = hipEventRecord(e1, st);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess && ms > 0.f) best = std::max(best, moved / (ms * 1e-3) / 1e9);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *gbps = best;
    return err;
}

}  // namespace mrinv
