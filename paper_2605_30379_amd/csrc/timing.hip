// Optional per-kernel timing.  When a handle enables it, every kernel launch
// of the library carries a start and a stop event stamped at the kernel's own
// start and end (hipExtLaunchKernelGGL) and is tagged with the kernel's name
// and the algorithmic bytes and flops of that launch; mrinv_kernel_stats()
// aggregates them per kernel name.
#include <string.h>

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

}  // namespace mrinv
