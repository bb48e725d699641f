// abi.hip -- library-wide C ABI entry points: version, last HIP error,
// kernel-timing instrumentation.
#include <algorithm>

#include "common.hpp"
#include "prof.hpp"

#include <cstdio>
#include <cstdlib>

namespace miid {
thread_local int g_last_hip_error = 0;

// empty kernel whose dispatch carries the start event of a timed launch
__global__ void k_prof_marker(int) {}

// Records the error code; with MIID_DEBUG set in the environment also prints
// the failing call.
void report_hip_error(int code, const char* what, const char* file, int line) {
    g_last_hip_error = code;
    if (std::getenv("MIID_DEBUG"))
        std::fprintf(stderr, "miid: %s failed with HIP error %d (%s) at %s:%d\n", what, code,
                     hipGetErrorString((hipError_t)code), file, line);
}
}

using namespace miid;

extern "C" {

const char* miid_version(void) { return "miid 0.1 (gfx950)"; }

int miid_last_hip_error(void) { return g_last_hip_error; }

int miid_prof_begin(int sample_every) {
    ProfState& s = prof_state();
    s.every = sample_every > 0 ? sample_every : 0;
    for (auto& slot : s.used) s.pool.push_back(slot);
    s.used.clear();
    return 0;
}

int miid_prof_end(miid_prof_record* out, int max_records) {
    ProfState& s = prof_state();
    int count = 0;
    for (auto& slot : s.used) {
        if (hipEventSynchronize(slot.b) != hipSuccess) {
            g_last_hip_error = (int)hipGetLastError();
            return MIID_E_HIP;
        }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, slot.a, slot.b);
        slot.rec.ms = ms;
        if (out && count < max_records) out[count] = slot.rec;
        ++count;
    }
    for (auto& slot : s.used) s.pool.push_back(slot);
    s.used.clear();
    s.every = 0;
    return std::min(count, max_records);
}

}  // extern "C"
