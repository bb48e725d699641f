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

// Workgroup barrier that orders LDS only: global loads and stores issued
// before it stay in flight (a plain __syncthreads also waits for them).  For
// kernels whose threads exchange data through LDS alone.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Cross-lane moves within rows of 16 lanes through DPP (a VALU operand
// modifier, no LDS crossbar round trip).  The four patterns used are
// butterflies over a row: lane i pairs with i^1 and i^2 (quad permutes),
// with 7-i within its half row and with 15-i within its row, so after the
// four steps every lane of a row holds the combination of all sixteen.
enum : int {
    kDppXor1 = 0xB1,          // quad_perm [1,0,3,2]
    kDppXor2 = 0x4E,          // quad_perm [2,3,0,1]
    kDppHalfMirror = 0x141,   // row_half_mirror
    kDppMirror = 0x140,       // row_mirror
};

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int64_t b = __builtin_bit_cast(int64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((int64_t)hi << 32) | (uint32_t)lo);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}

// Sum over each row of 16 lanes; every lane of the row ends with the same
// value (both partners of a step add the same two operands).
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    v += dpp_f64<kDppHalfMirror>(v);
    v += dpp_f64<kDppMirror>(v);
    return v;
}

// Sum over the wave: rows by DPP, then the four row sums read from lanes
// 0, 16, 32, 48 in a fixed order (the result is wave-uniform).
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v = row16_sum(v);
    double t = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t b = __builtin_bit_cast(int64_t, v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 16 * r);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * r);
        t += __builtin_bit_cast(double, ((int64_t)hi << 32) | (uint32_t)lo);
    }
    return t;
}

// Butterfly sum over the 64 lanes of a wave.  Every lane ends with the same
// value (each stage adds the same two operands on both partners), so the
// result is identical on all lanes and from run to run.  Doubles take the
// DPP form (wave_sum_dpp) instead.  Both need every lane of the wave active.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }

// (value, index) pair ordered by larger value, then smaller index.
struct ArgMax {
    double v;
    int32_t i;
};

__device__ __forceinline__ bool argmax_better(double va, int32_t ia, double vb, int32_t ib) {
    return va > vb || (va == vb && ia < ib);
}

template <int CTRL>
__device__ __forceinline__ ArgMax argmax_step(ArgMax a) {
    const double ov = dpp_f64<CTRL>(a.v);
    const int32_t oi = dpp_i32<CTRL>(a.i);
    if (argmax_better(ov, oi, a.v, a.i)) {
        a.v = ov;
        a.i = oi;
    }
    return a;
}

// Argmax over the wave: rows by DPP, then the four row winners in a fixed
// order (wave-uniform result).
__device__ __forceinline__ ArgMax wave_argmax_dpp(ArgMax a) {
    a = argmax_step<kDppXor1>(a);
    a = argmax_step<kDppXor2>(a);
    a = argmax_step<kDppHalfMirror>(a);
    a = argmax_step<kDppMirror>(a);
    ArgMax b{-1.0, INT32_MAX};
    bool first = true;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t bits = __builtin_bit_cast(int64_t, a.v);
        const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffff), 16 * r);
        const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), 16 * r);
        const double v = __builtin_bit_cast(double, ((int64_t)hi << 32) | (uint32_t)lo);
        const int32_t i = __builtin_amdgcn_readlane(a.i, 16 * r);
        if (first || argmax_better(v, i, b.v, b.i)) b = {v, i};
        first = false;
    }
    return b;
}

// Argmax over the wave (every lane active); wave-uniform result.
__device__ __forceinline__ ArgMax wave_argmax(ArgMax a) { return wave_argmax_dpp(a); }

// Fold W per-wave (value, index, sum, flag) entries from LDS: every load is
// issued before the first comparison, then the fixed-order fold (the same
// result in every thread).
template <int W>
__device__ __forceinline__ void fold_waves(const double* bv, const int32_t* bi, const double* bs, const int32_t* bf,
                                           ArgMax& best, double& sum, int& flag) {
    double v[W], s[W];
    int32_t id[W], f[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        v[w] = bv[w];
        id[w] = bi[w];
        s[w] = bs[w];
        f[w] = bf[w];
    }
    best = ArgMax{v[0], id[0]};
    sum = s[0];
    flag = f[0];
#pragma unroll
    for (int w = 1; w < W; ++w) {
        if (argmax_better(v[w], id[w], best.v, best.i)) best = ArgMax{v[w], id[w]};
        sum += s[w];
        flag |= f[w];
    }
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

// 16-byte load marked nontemporal (not kept in the caches on its way in)
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double2 load_nt(const double2* p) {
    const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    return double2(v.x, v.y);
}
__device__ __forceinline__ float4 load_nt(const float4* p) {
    const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
    return float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ double get(const double2& v, int e) { return e == 0 ? v.x : v.y; }
__device__ __forceinline__ double get(const float4& v, int e) {
    return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}

__device__ __forceinline__ bool is_finite_d(double x) { return !(isnan(x) || isinf(x)); }

// p[idx] where ok, else `other`, with no branch: the load always issues (from
// p[safe], a valid element, where !ok) and the choice is a bitwise merge
// under a mask the compiler cannot see through.  A load written under a
// condition becomes a branch whose other side writes the same register, and
// the compiler then waits for the load before that write, so a run of such
// loads goes out one memory round trip at a time; a plain select on the
// loaded value is turned back into such a branch.
template <typename X>
__device__ __forceinline__ X load_or(const X* p, int64_t idx, bool ok, int64_t safe, X other) {
    static_assert(sizeof(X) % 4 == 0, "whole 32-bit words");
    constexpr int W = (int)(sizeof(X) / 4);
    const X v = p[ok ? idx : safe];
    uint32_t m = ok ? 0xffffffffu : 0u;
    asm volatile("" : "+v"(m));
    uint32_t a[W], b[W];
    __builtin_memcpy(a, &v, sizeof(X));
    __builtin_memcpy(b, &other, sizeof(X));
#pragma unroll
    for (int w = 0; w < W; ++w) a[w] = (a[w] & m) | (b[w] & ~m);
    X r;
    __builtin_memcpy(&r, a, sizeof(X));
    return r;
}

}  // namespace miid
