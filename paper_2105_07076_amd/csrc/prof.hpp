// prof.hpp -- optional kernel timing with HIP events.  A sampled launch is
// preceded by an empty marker kernel whose dispatch carries the start event
// (stamped when the marker ends, i.e. after everything before it on the
// stream has finished) and is itself launched through hipExtLaunchKernelGGL
// with the stop event; the elapsed time is the kernel's execution plus one
// inter-kernel gap.  (An event carried by the timed dispatch itself is stamped
// when the command processor takes the packet, which can be while the
// previous kernel still runs.)
#pragma once
#include <hip/hip_ext.h>
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
// else -1.
inline int prof_take(int32_t kernel, int32_t step, int64_t rows, int64_t cols) {
    ProfState& s = prof_state();
    if (s.every <= 0 || (step % s.every) != 0 || s.used.size() >= 65536) return -1;
    ProfSlot slot;
    if (!s.pool.empty()) {
        slot = s.pool.back();
        s.pool.pop_back();
    } else {
        if (hipEventCreate(&slot.a) != hipSuccess) return -1;
        if (hipEventCreate(&slot.b) != hipSuccess) return -1;
    }
    slot.rec = miid_prof_record{kernel, step, rows, cols, 0.0f};
    s.used.push_back(slot);
    return (int)s.used.size() - 1;
}

inline hipEvent_t prof_a(int slot) { return prof_state().used[slot].a; }

__global__ void k_prof_marker(int);
inline hipEvent_t prof_b(int slot) { return prof_state().used[slot].b; }

}  // namespace miid

// Launch `K` (parenthesise template kernels) plainly, or with the timing
// events of profiling slot `SLOT` when it is sampled.
#define MIID_LAUNCH(SLOT, K, GRID, BLOCK, SHMEM, STREAM, ...)                                                   \
    do {                                                                                                        \
        if ((SLOT) >= 0) {                                                                                      \
            hipExtLaunchKernelGGL(::miid::k_prof_marker, dim3(1), dim3(64), 0, STREAM, nullptr,                 \
                                  ::miid::prof_a(SLOT), 0, 0);                                                  \
            hipExtLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, nullptr, ::miid::prof_b(SLOT), 0, __VA_ARGS__); \
        } else                                                                                                  \
            hipLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                                     \
    } while (0)
