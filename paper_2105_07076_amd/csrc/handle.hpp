// handle.hpp -- per-device library state and the miid_handle of the C ABI.
//
// Every entry point takes a miid_handle first (NULL = no tuning table).  The
// handle names the device it was created on and holds a read-only table of
// tuned launch shapes; the per-device facts the plans need (compute-unit
// count, which kernels already had their LDS limit raised) live in one
// library-wide record per device, filled once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/miid.h"

namespace miid {

// routines of the tuning table (the first word of a table row)
enum TuneRoutine : int { kTuneId = 0, kTuneRid, kTuneRidSample, kTuneTwoSided, kTuneCur, kTuneBatched };

// one row: routine, dtype and shape (0 = any) -> panel width and hint fields
struct TuneRow {
    int routine;
    int dtype;
    int64_t m, n, k;
    int32_t nb;
    uint32_t hints;
};

// The current device's ordinal and compute-unit count, queried once per
// device.  Without a visible device: device -1 and 256 compute units (the
// MI355X figure), so that workspace queries also answer on a host.
struct DevInfo {
    int device;
    int cus;
};
DevInfo dev_info();

// Raises the dynamic-LDS limit of kernel `fn` to `bytes` on the current
// device, once per (device, kernel).
hipError_t lds_limit_once(const void* fn, int bytes);

// The options a call runs with: *in, with nb and the hint fields of flags
// taken from the handle's table when the caller left both at 0 and a row
// matches (the most specific row wins).  Returns 0, or -1 when the handle
// belongs to another device than the current one.
int resolve_opts(miid_handle h, int routine, miid_dtype dtype, int64_t m, int64_t n, int64_t k,
                 const miid_opts* in, miid_opts* out);

// Looks up the current device's copy of the allocation-free entry point's
// static scratch (once per device); 0 or a negative MIID code.
int batched_noalloc_setup();

// Checks only that the handle belongs to the current device (0 or -1).
int check_handle(miid_handle h);

// The bodies number their arguments from the first one after the handle;
// the ABI counts the handle as argument 1.
inline int shift_arg(int rc) { return (rc < 0 && rc > -100) ? rc - 1 : rc; }
// the four 4-bit MIID_HINT fields of miid_opts.flags
constexpr uint32_t kHintMask = 0xFFFF00u;

}  // namespace miid
