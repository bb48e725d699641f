// common.hpp -- device helpers shared by the miid HIP kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/miid.h"

namespace miid {

constexpr int kWave = 64;

// HIP error code behind the last MIID_E_HIP return (defined in abi.hip).
extern thread_local int g_last_hip_error;

void report_hip_error(int code, const char* what, const char* file, int line);

#define MIID_HIP(call)                                                 \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) {                                        \
            ::miid::report_hip_error((int)e_, #call, __FILE__, __LINE__); \
            return MIID_E_HIP;                                         \
        }                                                              \
    } while (0)

// Butterfly sum over the 64 lanes of a wave.  Every lane ends with the same
// value (each stage adds the same two operands on both partners), so the
// result is identical on all lanes and from run to run.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// (value, index) pair ordered by larger value, then smaller index.
struct ArgMax {
    double v;
    int32_t i;
};

__device__ __forceinline__ bool argmax_better(double va, int32_t ia, double vb, int32_t ib) {
    return va > vb || (va == vb && ia < ib);
}

__device__ __forceinline__ ArgMax wave_argmax(ArgMax a) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(a.v, off, kWave);
        int32_t oi = __shfl_xor(a.i, off, kWave);
        if (argmax_better(ov, oi, a.v, a.i)) {
            a.v = ov;
            a.i = oi;
        }
    }
    return a;
}

// Per-workgroup partial result of a pass over the alive columns: the best
// residual norm with its column, and the sum of squared residual norms.
struct ColPartial {
    double best;    // largest residual norm (-1 when the workgroup has no alive column)
    int32_t idx;    // its column (INT32_MAX when none)
    int32_t nonfinite;
    double sumsq;   // sum of squared residual norms of the alive columns
    double pad;
};

// Device-side control block of one factorisation.
struct DevState {
    int32_t stop;       // 1 once the factorisation stopped before the host's last step
    int32_t k_out;      // steps completed when stop was set
    uint32_t status;    // MIID_* bits
    int32_t pad0;
    double a_norm;      // ||A||_F
    double pad1;
};

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
};
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
};

__device__ __forceinline__ double get(const double2& v, int e) { return e == 0 ? v.x : v.y; }
__device__ __forceinline__ double get(const float4& v, int e) {
    return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}

__device__ __forceinline__ bool is_finite_d(double x) { return !(isnan(x) || isinf(x)); }

}  // namespace miid
