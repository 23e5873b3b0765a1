// timer.hip -- measurement support: the GPU time of chosen kernel classes inside ordinary calls,
// from HIP events recorded on the launching stream right before and right after each launch of
// a chosen class (kernel_timer_start / kernel_timer_read).  The interval of a launch is its
// execution plus the dispatch of the kernel behind the first event.  Launches issued while the
// stream is being captured into a graph are not timed.
#include <mutex>
#include <vector>

#include "internal.h"

namespace ps {

constexpr int kTimerClasses = 10;          // kernel classes 1..9 (KernelClass)
constexpr size_t kTimerMaxPairs = 16384;   // launches timed per class at most

struct TimerState {
    std::mutex m;
    uint32_t mask = 0;
    std::vector<hipEvent_t> pool;            // created lazily, reused across sessions
    size_t used = 0;
    std::vector<std::pair<size_t, size_t>> pairs[kTimerClasses];
    size_t open[kTimerClasses] = {};         // event index of the last begin, + 1 (0 = none)
};

static TimerState &timer() {
    static TimerState t;
    return t;
}

static bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

static bool next_event(TimerState &t, size_t *idx) {
    if (t.used == t.pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return false;
        t.pool.push_back(e);
    }
    *idx = t.used++;
    return true;
}

void timer_mark(int kc, hipStream_t st, bool begin) {
    TimerState &t = timer();
    if (kc <= 0 || kc >= kTimerClasses) return;
    // the mask is read without the lock first: launches pay nothing while no timer runs
    if (!(__atomic_load_n(&t.mask, __ATOMIC_RELAXED) & (1u << kc))) return;
    if (capturing(st)) return;
    std::lock_guard<std::mutex> lock(t.m);
    if (!(t.mask & (1u << kc))) return;
    if (begin) {
        if (t.pairs[kc].size() >= kTimerMaxPairs) return;
        size_t i;
        if (!next_event(t, &i) || hipEventRecord(t.pool[i], st) != hipSuccess) return;
        t.open[kc] = i + 1;
    } else {
        if (t.open[kc] == 0) return;
        size_t i;
        if (!next_event(t, &i) || hipEventRecord(t.pool[i], st) != hipSuccess) {
            t.open[kc] = 0;
            return;
        }
        t.pairs[kc].emplace_back(t.open[kc] - 1, i);
        t.open[kc] = 0;
    }
}

}  // namespace ps

using namespace ps;

extern "C" ps_status kernel_timer_start(uint32_t class_mask) {
    clear_error();
    if (class_mask & ~((1u << kTimerClasses) - 2u)) return fail(PS_EINVAL, "kernel class mask 0x%x", class_mask);
    TimerState &t = timer();
    std::lock_guard<std::mutex> lock(t.m);
    t.used = 0;
    for (int c = 0; c < kTimerClasses; ++c) {
        t.pairs[c].clear();
        t.open[c] = 0;
    }
    __atomic_store_n(&t.mask, class_mask, __ATOMIC_RELAXED);
    return PS_OK;
}

extern "C" ps_status kernel_timer_read(int32_t kernel_class, double *total_ms, int32_t *launches) {
    clear_error();
    if (kernel_class <= 0 || kernel_class >= kTimerClasses) return fail(PS_EINVAL, "kernel class %d", kernel_class);
    if (!total_ms || !launches) return fail(PS_EINVAL, "null output");
    TimerState &t = timer();
    std::lock_guard<std::mutex> lock(t.m);
    double sum = 0.0;
    for (const auto &p : t.pairs[kernel_class]) {
        PS_HIP(hipEventSynchronize(t.pool[p.second]));
        float ms = 0.f;
        PS_HIP(hipEventElapsedTime(&ms, t.pool[p.first], t.pool[p.second]));
        sum += ms;
    }
    *total_ms = sum;
    *launches = static_cast<int32_t>(t.pairs[kernel_class].size());
    return PS_OK;
}

extern "C" ps_status kernel_timer_stop(void) {
    clear_error();
    TimerState &t = timer();
    std::lock_guard<std::mutex> lock(t.m);
    __atomic_store_n(&t.mask, 0u, __ATOMIC_RELAXED);
    return PS_OK;
}
