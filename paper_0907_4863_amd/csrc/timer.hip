// Opt-in per-class kernel timing with HIP events bound to the timed kernel dispatches.
#include <mutex>
#include <vector>

#include "common.h"

namespace saamg {
namespace {

constexpr int kMaxSlots = 65536;

struct Slot {
    hipEvent_t a = nullptr, b = nullptr;
    int kind = 0;
    long units = 0;
};

struct Timers {
    std::mutex mu;
    bool enabled[T_NKIND] = {};
    std::vector<Slot> slots;
    int used = 0;
};

Timers& timers() {
    static Timers t;
    return t;
}

}  // namespace

KTimer::KTimer(int k, hipStream_t st, long units) : kind(k), s(st) {
    Timers& T = timers();
    if (!T.enabled[k]) return;
    std::lock_guard<std::mutex> g(T.mu);
    if (T.used >= kMaxSlots) return;
    if ((int)T.slots.size() <= T.used) {
        Slot sl;
        if (hipEventCreate(&sl.a) != hipSuccess || hipEventCreate(&sl.b) != hipSuccess) return;
        T.slots.push_back(sl);
    }
    slot = T.used++;
    T.slots[slot].kind = k;
    T.slots[slot].units = units;
}

hipEvent_t KTimer::start() {
    if (slot < 0 || started) return nullptr;
    started = true;
    return timers().slots[slot].a;
}

hipEvent_t KTimer::stop() {
    if (slot < 0) return nullptr;
    stopped = true;
    return timers().slots[slot].b;
}

KTimer::~KTimer() {
    if (slot < 0) return;
    // a scope that launched nothing reads as zero time
    if (!started) (void)hipEventRecord(timers().slots[slot].a, s);
    if (!stopped) (void)hipEventRecord(timers().slots[slot].b, s);
}

}  // namespace saamg

extern "C" {

int saamg_timer_enable(int kind, int enable) {
    if (kind < 0 || kind >= saamg::T_NKIND) return SAAMG_INVALID_ARG;
    saamg::timers().enabled[kind] = enable != 0;
    return SAAMG_OK;
}

int saamg_timer_read(int kind, double* total_ms, int64_t* launches, int64_t* units) {
    if (kind < 0 || kind >= saamg::T_NKIND) return SAAMG_INVALID_ARG;
    auto& T = saamg::timers();
    std::lock_guard<std::mutex> g(T.mu);
    double ms = 0.0;
    int64_t n = 0, u = 0;
    for (int i = 0; i < T.used; ++i) {
        auto& sl = T.slots[i];
        if (sl.kind != kind) continue;
        if (hipEventSynchronize(sl.b) != hipSuccess) return SAAMG_HIP_ERROR;
        float e = 0.f;
        if (hipEventElapsedTime(&e, sl.a, sl.b) != hipSuccess) return SAAMG_HIP_ERROR;
        ms += e;
        ++n;
        u += sl.units;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    if (units) *units = u;
    return SAAMG_OK;
}

int saamg_timer_reset(void) {
    auto& T = saamg::timers();
    std::lock_guard<std::mutex> g(T.mu);
    for (int i = 0; i < T.used; ++i) (void)hipEventSynchronize(T.slots[i].b);
    T.used = 0;
    return SAAMG_OK;
}

}  // extern "C"
