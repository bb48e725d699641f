// rid.hip -- randomized ID with a Gaussian row sketch on gfx950.
//
// Paper: Advani & O'Hagan, Section 2.2 (the randomized method runs the same
// column-pivoted QR on a smaller matrix and maps the chosen columns back to
// A) and Section 2.2.1 (the key is a smaller matrix with which to compute the
// ID).  The smaller matrix here is the row sketch Y = Omega A (l x n) with a
// Gaussian Omega; the CPQR of Y (the driver shared with id_cpqr, FP32 with
// FP64 norms and an FP64 triangular solve) gives J and T, and C = A[:, J].
//
// The sketch runs on the matrix cores: v_mfma_f32_16x16x32_bf16, Omega exact
// in bfloat16, A rounded to bfloat16 once (mode 0) or split as hi + lo with
// hi = bf16(a), lo = bf16(a - hi) (mode 1, two passes, relative error of Y
// about 2^-16), FP32 accumulation.
#include <algorithm>

#include "common.hpp"
#include "handle.hpp"
#include "cpqr.hpp"
#include "prof.hpp"

namespace miid {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f4v_t __attribute__((ext_vector_type(4)));

constexpr int kSkThreads = 256;
constexpr int kSkCols = 64;   // columns of A (and Y) per workgroup, 16 per wave
constexpr int kSkK = 32;      // K per MFMA
constexpr int kSkLdsRow = kSkK + 8;  // bf16 per LDS row (padding against bank conflicts)

// Omega (l x m, column-major, bf16 bits) -> Wt (lpad x mpad, k contiguous),
// zero padded.
__global__ void k_omega_t(const uint16_t* __restrict__ Om, int l, int64_t m, int64_t ldo, uint16_t* __restrict__ Wt,
                          int lpad, int64_t mpad) {
    __shared__ uint16_t tile[64][65];
    const int64_t k0 = (int64_t)blockIdx.x * 64;  // columns of Omega
    const int i0 = blockIdx.y * 64;               // rows of Omega
    const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
    for (int e = ty; e < 64; e += 4) {
        const int i = i0 + tx;
        const int64_t k = k0 + e;
        tile[e][tx] = (i < l && k < m) ? Om[i + k * ldo] : (uint16_t)0;
    }
    __syncthreads();
    for (int e = ty; e < 64; e += 4) {
        const int i = i0 + e;
        const int64_t k = k0 + tx;
        if (i < lpad && k < mpad) Wt[(int64_t)i * mpad + k] = tile[tx][e];
    }
}

// Y tile (16 * mtb rows starting at tile mt0, 64 columns) = Omega A.
// D = A_tile^T Omega_tile^T so that one accumulator element of 16
// neighbouring lanes is 16 consecutive rows of one column of Y.
// Operand layout (measured on gfx950): lane l holds row l % 16 and
// k = 8 (l / 16) + e of the A operand, k = 8 (l / 16) + e and column l % 16
// of the B operand; output element r of lane l is row 4 (l / 16) + r,
// column l % 16.
// K advances in chunks of KC (KC / 32 MFMA steps): the Omega chunk
// (16 MTB rows x KC) is double-buffered in LDS and the next chunk's Omega
// and A loads are in flight while the current chunk is multiplied, so there
// is one barrier per chunk.
template <bool SPLIT, bool VEC, int MTB, int KC>
__global__ void __launch_bounds__(kSkThreads) k_sketch(const float* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                       const uint16_t* __restrict__ Wt, int64_t mpad, int mt_total,
                                                       float* __restrict__ S, int64_t ldw, float* __restrict__ Yout,
                                                       int64_t ldy, int l) {
    constexpr int LR = KC + 8;             // bf16 per LDS row (padding against bank conflicts)
    constexpr int KS = KC / kSkK;          // MFMA steps per chunk
    constexpr int ROWS = MTB * 16;
    constexpr int SEG = KC / 8;            // 16-byte segments of a row of the chunk
    constexpr int NSEG = ROWS * SEG;
    constexpr int SPT = (NSEG + kSkThreads - 1) / kSkThreads;  // segments staged per thread
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint16_t* sW = reinterpret_cast<uint16_t*>(smem_raw);  // [2][ROWS][LR]
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int mt0 = blockIdx.y * MTB;
    const int mtb = min(MTB, mt_total - mt0);
    const int64_t col = (int64_t)blockIdx.x * kSkCols + wave * 16 + lane % 16;  // this lane's A column
    const int kl = 8 * (lane / 16);                                            // this lane's k offset
    const bool colok = col < n;
    const float* ac = A + (colok ? col : 0) * lda;

    f4v_t acc[MTB];
#pragma unroll
    for (int t = 0; t < MTB; ++t) acc[t] = f4v_t{0.f, 0.f, 0.f, 0.f};

    uint4 stg[SPT];
    auto load_w = [&](int64_t k0) {
#pragma unroll
        for (int i = 0; i < SPT; ++i) {
            const int seg = tid + kSkThreads * i;
            const int row = seg / SEG, sg = seg % SEG;
            const int64_t kk = k0 + 8 * sg;
            stg[i] = (seg < NSEG && row < 16 * mtb && kk < mpad)
                         ? *reinterpret_cast<const uint4*>(Wt + (int64_t)(mt0 * 16 + row) * mpad + kk)
                         : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    auto store_w = [&](int buf) {
#pragma unroll
        for (int i = 0; i < SPT; ++i) {
            const int seg = tid + kSkThreads * i;
            const int row = seg / SEG, sg = seg % SEG;
            if (seg < NSEG) *reinterpret_cast<uint4*>(sW + (buf * ROWS + row) * LR + 8 * sg) = stg[i];
        }
    };
    auto load_a = [&](int64_t k0, float (&x)[KS][8]) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int64_t kb = k0 + kSkK * ks + kl;
            if (VEC && colok && kb + 8 <= m) {
                const float4 v0 = *reinterpret_cast<const float4*>(ac + kb);
                const float4 v1 = *reinterpret_cast<const float4*>(ac + kb + 4);
                x[ks][0] = v0.x; x[ks][1] = v0.y; x[ks][2] = v0.z; x[ks][3] = v0.w;
                x[ks][4] = v1.x; x[ks][5] = v1.y; x[ks][6] = v1.z; x[ks][7] = v1.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) x[ks][e] = (colok && kb + e < m) ? ac[kb + e] : 0.f;
            }
        }
    };

    float xa[KS][8], xn[KS][8];
    load_w(0);
    load_a(0, xa);
    store_w(0);
    __syncthreads();
    int cur = 0;
    for (int64_t k0 = 0; k0 < mpad; k0 += KC) {
        const bool more = k0 + KC < mpad;
        if (more) {
            load_w(k0 + KC);
            load_a(k0 + KC, xn);
        }
        const uint16_t* wb = sW + cur * ROWS * LR;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            bf16x8_t hi, lo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const __bf16 h = (__bf16)xa[ks][e];
                hi[e] = h;
                if (SPLIT) lo[e] = (__bf16)(xa[ks][e] - (float)h);
            }
#pragma unroll
            for (int t = 0; t < MTB; ++t) {
                if (t < mtb) {
                    const bf16x8_t w =
                        *reinterpret_cast<const bf16x8_t*>(wb + (t * 16 + lane % 16) * LR + kSkK * ks + kl);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi, w, acc[t], 0, 0, 0);
                    if (SPLIT) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo, w, acc[t], 0, 0, 0);
                }
            }
        }
        if (more) {
            store_w(cur ^ 1);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int e = 0; e < 8; ++e) xa[ks][e] = xn[ks][e];
        }
        __syncthreads();
        cur ^= 1;
    }
    // output element r of lane l: Y[row = tile row + l % 16][col = wave col + 4 (l / 16) + r]
    // (a predicate, not a break: a data-dependent exit from the unrolled loop
    // would put acc in scratch memory)
#pragma unroll
    for (int t = 0; t < MTB; ++t) {
        const int64_t row = (int64_t)(mt0 + t) * 16 + lane % 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t c = (int64_t)blockIdx.x * kSkCols + wave * 16 + 4 * (lane / 16) + r;
            if (t < mtb && c < n && row < ldw) S[row + c * ldw] = acc[t][r];
            if (t < mtb && Yout && c < n && row < l) Yout[row + c * ldy] = acc[t][r];
        }
    }
}

// LDS bytes of a k_sketch instantiation (two Omega chunks)
constexpr size_t sketch_lds(int mtb, int kc) { return (size_t)2 * mtb * 16 * (kc + 8) * 2; }

template <bool SPLIT, bool VEC, int MTB, int KC>
static hipError_t launch_sketch(int pr, hipStream_t s, int64_t n, int mt_total, const float* A, int64_t lda, int64_t m,
                                const uint16_t* Wt, int64_t mpad, float* S, int64_t ldw, float* Y, int64_t ldy,
                                int l) {
    constexpr size_t lds = sketch_lds(MTB, KC);
    {
        const hipError_t e = lds_limit_once((const void*)k_sketch<SPLIT, VEC, MTB, KC>, (int)lds);
        if (e != hipSuccess) return e;
    }
    dim3 grid((unsigned)((n + kSkCols - 1) / kSkCols), (unsigned)((mt_total + MTB - 1) / MTB));
    MIID_LAUNCH(pr, (k_sketch<SPLIT, VEC, MTB, KC>), grid, dim3(kSkThreads), lds, s, A, lda, m, n, Wt, mpad,
                mt_total, S, ldw, Y, ldy, l);
    return hipGetLastError();
}

// Tile rows per workgroup: every 16-row tile of Y in one workgroup when
// l <= 528 (A is then read once), 33 tiles per workgroup row beyond.
template <bool SPLIT, bool VEC>
static hipError_t launch_sketch_mt(int pr, hipStream_t s, int64_t n, int mt_total, const float* A, int64_t lda,
                                   int64_t m, const uint16_t* Wt, int64_t mpad, float* S, int64_t ldw, float* Y,
                                   int64_t ldy, int l) {
    if (mt_total <= 9)
        return launch_sketch<SPLIT, VEC, 9, 128>(pr, s, n, mt_total, A, lda, m, Wt, mpad, S, ldw, Y, ldy, l);
    if (mt_total <= 17)
        return launch_sketch<SPLIT, VEC, 17, 128>(pr, s, n, mt_total, A, lda, m, Wt, mpad, S, ldw, Y, ldy, l);
    return launch_sketch<SPLIT, VEC, 33, 64>(pr, s, n, mt_total, A, lda, m, Wt, mpad, S, ldw, Y, ldy, l);
}

template <typename T>
__global__ void k_fill_rid(T* __restrict__ p, int64_t count, T value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

struct RidPlan {
    IdPlan id;
    int lpad;        // rows of Wt (16-row tiles)
    int mt_total;    // 16-row tiles of Y
    int64_t mpad;    // K padded to 32
    size_t oWt, total;
    // least-squares Z over the full A for the sketch's skeleton
    bool lstsq;
    LsPlan ls;
    size_t oLs;
};

// a breakdown of the least-squares pass's Cholesky into the status
__global__ void k_ls_status(miid_info* __restrict__ info, const uint32_t* __restrict__ flag) {
    if (threadIdx.x == 0 && flag[0]) info->status |= MIID_LSTSQ_BREAKDOWN;
}

static int make_rid_plan(int64_t m, int64_t n, int32_t l, const miid_opts* opts, RidPlan* R) {
    if (m < 1) return -2;
    if (n < 1) return -3;
    if (l < 1 || l > 1024) return -6;
    if (m > n || l > n) return MIID_E_UNSUPPORTED;
    const int rc = make_plan(l, n, MIID_F32, opts, &R->id);
    if (rc != 0) return rc == -2 ? -6 : (rc == -6 ? -9 : rc);
    R->mt_total = (l + 15) / 16;
    R->lpad = R->mt_total * 16;
    if (R->lpad > R->id.ldw) return MIID_E_UNSUPPORTED;
    R->mpad = (int64_t)align_up((size_t)m, kSkK);
    R->oWt = align_up(R->id.total, 256);
    R->total = align_up(R->oWt + (size_t)R->lpad * R->mpad * 2, 256);
    R->lstsq = opts && (opts->flags & MIID_LSTSQ_Z);
    if (R->lstsq) {
        if (opts->k < 1 || opts->k > m) return MIID_E_UNSUPPORTED;
        const int rc2 = ls_plan(m, n, opts->k, 4, &R->ls);
        if (rc2 != 0) return rc2;
        R->oLs = R->total;
        R->total = align_up(R->oLs + R->ls.total, 256);
    }
    return 0;
}

}  // namespace miid

using namespace miid;

extern "C" {

static size_t rid_workspace_body(int64_t m, int64_t n, int32_t l, const miid_opts* opts) {
    RidPlan R;
    if (make_rid_plan(m, n, l, opts, &R) != 0) return 0;
    return R.total;
}

static int rid_body(const float* A, int64_t m, int64_t n, int64_t lda, const uint16_t* Omega, int32_t l, int64_t ldo,
                    int32_t mode, const miid_opts* opts, int32_t* J, float* Z, int64_t ldz, float* C, int64_t ldc,
                    float* Y, int64_t ldy, double* R11, int64_t ldr, miid_info* info, void* ws, size_t ws_bytes,
                    void* stream) {
    if (!A) return -1;
    if (!Omega) return -5;
    RidPlan R;
    const int rc = make_rid_plan(m, n, l, opts, &R);
    if (rc != 0) return rc;
    if (lda < m) return -4;
    if (ldo < l) return -7;
    if (mode != 0 && mode != 1) return -8;
    if (!J) return -10;
    if (!Z) return -11;
    if (ldz < R.id.kmax) return -12;
    if (C && ldc < m) return -14;
    if (Y && ldy < l) return -16;
    if (R11 && ldr < R.id.kmax) return -18;
    if (!info) return -19;
    if (!ws) return -20;
    if (ws_bytes < R.total) return MIID_E_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    float* S = reinterpret_cast<float*>(w + R.id.oS);
    uint16_t* Wt = reinterpret_cast<uint16_t*>(w + R.oWt);
    const int64_t ldw = R.id.ldw;

    // rows of S beyond the sketch tiles must be zero
    {
        const int64_t cnt = ldw * n;
        const int blocks = (int)std::min<int64_t>((cnt + 255) / 256, 8192);
        hipLaunchKernelGGL(k_fill_rid<float>, dim3(blocks), dim3(256), 0, s, S, cnt, 0.f);
    }
    {
        dim3 grid((unsigned)((R.mpad + 63) / 64), (unsigned)((R.lpad + 63) / 64));
        hipLaunchKernelGGL(k_omega_t, grid, dim3(256), 0, s, Omega, l, m, ldo, Wt, R.lpad, R.mpad);
    }
    {
        const bool vec = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
        const int pr = prof_take(MIID_K_SKETCH, 0, m, n);
        hipError_t e;
        if (mode == 1)
            e = vec ? launch_sketch_mt<true, true>(pr, s, n, R.mt_total, A, lda, m, Wt, R.mpad, S, ldw, Y, ldy, l)
                    : launch_sketch_mt<true, false>(pr, s, n, R.mt_total, A, lda, m, Wt, R.mpad, S, ldw, Y, ldy, l);
        else
            e = vec ? launch_sketch_mt<false, true>(pr, s, n, R.mt_total, A, lda, m, Wt, R.mpad, S, ldw, Y, ldy, l)
                    : launch_sketch_mt<false, false>(pr, s, n, R.mt_total, A, lda, m, Wt, R.mpad, S, ldw, Y, ldy, l);
        MIID_HIP(e);
    }
    MIID_HIP(hipGetLastError());
    const int rc2 = run_id<float>(R.id, A, lda, J, Z, ldz, R11, ldr, C, ldc, info, w, s, true, A, lda, m);
    if (rc2 != 0 || !R.lstsq) return rc2;
    // Z = C^+ A for the sketch's skeleton (a skeleton cut short by an exact
    // zero residual has k_out < k: the rest of J is -1 and Z's rows there
    // stay zero)
    unsigned char* wl = w + R.oLs;
    const int rc3 = run_lstsq<float>(R.ls, A, m, n, lda, J, R.id.kmax, info, Z, ldz, R11, ldr, wl, s);
    if (rc3 != 0) return rc3;
    hipLaunchKernelGGL(k_ls_status, dim3(1), dim3(64), 0, s, info, reinterpret_cast<const uint32_t*>(wl + R.ls.oFlag));
    MIID_HIP(hipGetLastError());
    return 0;
}

// ---- entry points: the handle resolved, then the bodies above -----------
size_t miid_rid_workspace(miid_handle h, int64_t m, int64_t n, int32_t l, const miid_opts* opts) {
    miid_opts o;
    if (resolve_opts(h, kTuneRid, MIID_F32, m, n, opts ? opts->k : 0, opts, &o) != 0) return 0;
    return rid_workspace_body(m, n, l, opts ? &o : nullptr);
}

int rid_sketch_cpqr(miid_handle h, const float* A, int64_t m, int64_t n, int64_t lda, const uint16_t* Omega,
                    int32_t l, int64_t ldo, int32_t mode, const miid_opts* opts, int32_t* J, float* Z, int64_t ldz,
                    float* C, int64_t ldc, float* Y, int64_t ldy, double* R11, int64_t ldr, miid_info* info,
                    void* ws, size_t ws_bytes, void* stream) {
    miid_opts o;
    if (resolve_opts(h, kTuneRid, MIID_F32, m, n, opts ? opts->k : 0, opts, &o) != 0) return -1;
    return shift_arg(rid_body(A, m, n, lda, Omega, l, ldo, mode, opts ? &o : nullptr, J, Z, ldz, C, ldc, Y, ldy, R11,
                              ldr, info, ws, ws_bytes, stream));
}

}  // extern "C"
