// prof.hpp -- optional kernel timing with HIP events on the launch stream.
// Enabled by miid_prof_begin(); a sampled launch is bracketed by two events
// recorded on the stream it runs on, so the elapsed time is that kernel's.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/miid.h"

namespace miid {

struct ProfSlot {
    hipEvent_t a, b;
    miid_prof_record rec;
};

struct ProfState {
    int every = 0;
    std::vector<ProfSlot> used;
    std::vector<ProfSlot> pool;
};

inline ProfState& prof_state() {
    static ProfState s;
    return s;
}

// Returns a slot index when launch number `step` of `kernel` is sampled,
// else -1.  The start event is recorded on `stream` before the launch.
inline int prof_open(int32_t kernel, int32_t step, int64_t rows, int64_t cols, hipStream_t stream) {
    ProfState& s = prof_state();
    if (s.every <= 0 || (step % s.every) != 0 || s.used.size() >= 65536) return -1;
    ProfSlot slot;
    if (!s.pool.empty()) {
        slot = s.pool.back();
        s.pool.pop_back();
    } else {
        // no system-scope release on record: the events must not flush the
        // caches the timed kernel would otherwise find warm
        if (hipEventCreateWithFlags(&slot.a, hipEventDisableSystemFence) != hipSuccess) return -1;
        if (hipEventCreateWithFlags(&slot.b, hipEventDisableSystemFence) != hipSuccess) return -1;
    }
    slot.rec = miid_prof_record{kernel, step, rows, cols, 0.0f};
    hipEventRecord(slot.a, stream);
    s.used.push_back(slot);
    return (int)s.used.size() - 1;
}

// Records the end event of slot `idx` (after the launch).
inline void prof_close(int idx, hipStream_t stream) {
    if (idx >= 0) hipEventRecord(prof_state().used[idx].b, stream);
}

}  // namespace miid
