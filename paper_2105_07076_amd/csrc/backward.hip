// backward.hip -- adjoint of the ID with the pivots held fixed.
//
// The paper has no derivatives.  With J fixed, C = A[:, J] and the ID's
// Z = C^+ A (Z[:, J] = I and T = C^+ A_rest, the least-squares solution of
// Section 2.1).  Differentiating T = (C^T C)^{-1} C^T A_rest gives, for
// upstream gradients gC (of C) and gZ (of Z), with Gz = gZ with its J columns
// zeroed and M = (C^T C)^{-1} Gz = R11^{-1} R11^{-T} Gz:
//     gA          = C M
//     gA[:, J]    = gC + A M^T - C (Z M^T + M Z^T)    (C M is zero there)
// Kernels: the two FP64 triangular solves for M in one launch (the blocked
// solve of the forward pass, run transposed then forward, on the FP64 matrix
// cores with the right-hand-side tiles in LDS); the products C M and A M^T on
// the matrix cores (16x16x4 MFMA in the working
// precision; A M^T split over n with a fixed-order second pass, so the result
// is deterministic); the small k x k and m x k terms on the vector units.
#include <algorithm>

#include "common.hpp"
#include "handle.hpp"
#include "cpqr.hpp"
#include "prof.hpp"

namespace miid {

constexpr int kBwThreads = 256;
constexpr int kBwMaxK = 1024;
constexpr int kBwChunk = 512;  // columns of n per split-K partial

typedef double bd4_t __attribute__((ext_vector_type(4)));
typedef float bf4_t __attribute__((ext_vector_type(4)));
template <typename T> struct BwAcc;
template <> struct BwAcc<double> {
    using type = bd4_t;
    // output element e of lane l: row l / 16 + 4 e (f64, measured on gfx950)
    static __device__ __forceinline__ int row(int lg, int e) { return lg + 4 * e; }
    static __device__ __forceinline__ type mfma(double a, double b, type c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct BwAcc<float> {
    using type = bf4_t;
    // output element e of lane l: row 4 (l / 16) + e (f32)
    static __device__ __forceinline__ int row(int lg, int e) { return 4 * lg + e; }
    static __device__ __forceinline__ type mfma(float a, float b, type c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

__global__ void k_bw_sel(const int32_t* __restrict__ J, int k, int64_t n, int32_t* __restrict__ sel) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        sel[c] = -1;
}
__global__ void k_bw_sel2(const int32_t* __restrict__ J, int k, int32_t* __restrict__ sel) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) sel[J[i]] = i;
}

// C = A[:, J]  (m x k, leading dimension m)
template <typename T>
__global__ void k_bw_gather(const T* __restrict__ A, int64_t lda, int64_t m, const int32_t* __restrict__ J,
                            T* __restrict__ C) {
    const int q = blockIdx.y;
    const int64_t src = J[q];
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x)
        C[r + (int64_t)q * m] = A[r + src * lda];
}

template <typename T>
__global__ void k_bw_zero(T* __restrict__ p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

// OUT (rows x cols, ldo) = X (rows x K, ldx) * Y (K x cols, ldy), K small.
// Computed as OUT^T = Y^T X^T so that one output element of 16 neighbouring
// lanes is 16 consecutive rows of one column of OUT.  64 x 64 tile per
// workgroup, 32 x 32 per wave.
template <typename T>
__global__ void __launch_bounds__(kBwThreads) k_bw_gemm_nn(const T* __restrict__ X, int64_t ldx,
                                                           const T* __restrict__ Y, int64_t ldy, T* __restrict__ OUT,
                                                           int64_t ldo, int64_t rows, int64_t cols, int K) {
    using A4 = typename BwAcc<T>::type;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int64_t r0 = (int64_t)blockIdx.x * 64 + (wave & 1) * 32;
    const int64_t c0 = (int64_t)blockIdx.y * 64 + (wave >> 1) * 32;
    const int l16 = lane % 16, lg = lane / 16;
    A4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = A4{0, 0, 0, 0};
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int q = k0 + lg;
        T ya[2], xb[2];
#pragma unroll
        for (int bc = 0; bc < 2; ++bc) {
            const int64_t c = c0 + bc * 16 + l16;
            ya[bc] = (q < K && c < cols) ? Y[q + c * ldy] : T(0);
        }
#pragma unroll
        for (int br = 0; br < 2; ++br) {
            const int64_t r = r0 + br * 16 + l16;
            xb[br] = (q < K && r < rows) ? X[r + (int64_t)q * ldx] : T(0);
        }
#pragma unroll
        for (int bc = 0; bc < 2; ++bc)
#pragma unroll
            for (int br = 0; br < 2; ++br) acc[bc][br] = BwAcc<T>::mfma(ya[bc], xb[br], acc[bc][br]);
    }
#pragma unroll
    for (int bc = 0; bc < 2; ++bc)
#pragma unroll
        for (int br = 0; br < 2; ++br) {
            const int64_t r = r0 + br * 16 + l16;
            if (r >= rows) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t c = c0 + bc * 16 + BwAcc<T>::row(lg, e);
                if (c < cols) OUT[r + c * ldo] = acc[bc][br][e];
            }
        }
}

// Split-K partial of OUT (rows x cols) = X (rows x K) * Y^T (Y: cols x K):
// workgroup (x, y, z) covers a 64 x 64 output tile and K range
// [z * kBwChunk, (z + 1) * kBwChunk); the partial goes to PART[z].
template <typename T>
__global__ void __launch_bounds__(kBwThreads) k_bw_gemm_nt(const T* __restrict__ X, int64_t ldx,
                                                           const T* __restrict__ Y, int64_t ldy, T* __restrict__ PART,
                                                           int64_t rows, int64_t cols, int64_t K) {
    using A4 = typename BwAcc<T>::type;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int64_t r0 = (int64_t)blockIdx.x * 64 + (wave & 1) * 32;
    const int64_t c0 = (int64_t)blockIdx.y * 64 + (wave >> 1) * 32;
    const int64_t kbeg = (int64_t)blockIdx.z * kBwChunk;
    const int64_t kend = std::min<int64_t>(K, kbeg + kBwChunk);
    const int l16 = lane % 16, lg = lane / 16;
    A4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = A4{0, 0, 0, 0};
    for (int64_t k0 = kbeg; k0 < kend; k0 += 4) {
        const int64_t q = k0 + lg;
        T ya[2], xb[2];
#pragma unroll
        for (int bc = 0; bc < 2; ++bc) {
            const int64_t c = c0 + bc * 16 + l16;
            ya[bc] = (q < kend && c < cols) ? Y[c + q * ldy] : T(0);
        }
#pragma unroll
        for (int br = 0; br < 2; ++br) {
            const int64_t r = r0 + br * 16 + l16;
            xb[br] = (q < kend && r < rows) ? X[r + q * ldx] : T(0);
        }
#pragma unroll
        for (int bc = 0; bc < 2; ++bc)
#pragma unroll
            for (int br = 0; br < 2; ++br) acc[bc][br] = BwAcc<T>::mfma(ya[bc], xb[br], acc[bc][br]);
    }
    T* P = PART + (int64_t)blockIdx.z * rows * cols;
#pragma unroll
    for (int bc = 0; bc < 2; ++bc)
#pragma unroll
        for (int br = 0; br < 2; ++br) {
            const int64_t r = r0 + br * 16 + l16;
            if (r >= rows) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t c = c0 + bc * 16 + BwAcc<T>::row(lg, e);
                if (c < cols) P[r + c * rows] = acc[bc][br][e];
            }
        }
}

// OUT[e] = sum_z PART[z][e] in a fixed order
template <typename T>
__global__ void k_bw_reduce(const T* __restrict__ PART, int nz, int64_t count, T* __restrict__ OUT) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        T s = T(0);
        for (int z = 0; z < nz; ++z) s += PART[(int64_t)z * count + e];
        OUT[e] = s;
    }
}

// gA[:, J[q]] = gC[:, q] + P[:, q] - sum_t C[:, t] (Q[t, q] + Q[q, t])
template <typename T>
__global__ void k_bw_jcols(const T* __restrict__ C, const T* __restrict__ P, const T* __restrict__ Q,
                           const T* __restrict__ gC, int64_t ldgc, const int32_t* __restrict__ J, int64_t m, int k,
                           T* __restrict__ gA, int64_t ldga) {
    const int q = blockIdx.y;
    const int64_t dst = J[q];
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
        double s = (double)P[r + (int64_t)q * m];
        if (gC) s += (double)gC[r + (int64_t)q * ldgc];
        for (int t = 0; t < k; ++t)
            s -= (double)C[r + (int64_t)t * m] * ((double)Q[t + (int64_t)q * k] + (double)Q[q + (int64_t)t * k]);
        gA[r + dst * ldga] = (T)s;
    }
}

struct BwPlan {
    int nz;
    size_t oSel, oC, oM, oPart, oP, oQ, oSemi, total;
};

static BwPlan bw_plan(int64_t m, int64_t n, int32_t k, size_t esz) {
    BwPlan B;
    B.nz = (int)((n + kBwChunk - 1) / kBwChunk);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    B.oSel = take((size_t)n * 4);
    B.oC = take((size_t)m * k * esz);
    B.oM = take((size_t)k * n * esz);
    const size_t part_elems = std::max((size_t)m * k, (size_t)k * k) * (size_t)B.nz;
    B.oPart = take(part_elems * esz);
    B.oP = take((size_t)m * k * esz);
    B.oQ = take((size_t)k * k * esz);
    B.oSemi = take(semi_solve_workspace(k));
    B.total = off;
    return B;
}

template <typename T>
static int run_bw(const T* A, int64_t m, int64_t n, int64_t lda, const int32_t* J, int k, const double* R11,
                  int64_t ldr, const T* Z, int64_t ldz, const T* gC, int64_t ldgc, const T* gZ, int64_t ldgz, T* gA,
                  int64_t ldga, unsigned char* ws, const BwPlan& B, hipStream_t s) {
    int32_t* sel = reinterpret_cast<int32_t*>(ws + B.oSel);
    T* C = reinterpret_cast<T*>(ws + B.oC);
    T* M = reinterpret_cast<T*>(ws + B.oM);
    T* part = reinterpret_cast<T*>(ws + B.oPart);
    T* P = reinterpret_cast<T*>(ws + B.oP);
    T* Q = reinterpret_cast<T*>(ws + B.oQ);
    hipLaunchKernelGGL(k_bw_sel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, s, J, k, n,
                       sel);
    hipLaunchKernelGGL(k_bw_sel2, dim3((k + 255) / 256), dim3(256), 0, s, J, k, sel);
    hipLaunchKernelGGL(k_bw_gather<T>, dim3((unsigned)std::min<int64_t>((m + 255) / 256, 64), (unsigned)k), dim3(256), 0,
                       s, A, lda, m, J, C);
    // M = R11^{-1} R11^{-T} Gz (Gz = gZ with the J columns zeroed) on the
    // matrix cores: the block triangular solve, transposed then forward
    if (gZ) {
        const int rc = semi_solve<T>(R11, ldr, k, gZ, (int64_t)1, ldgz, n, sel, 1, M, (int64_t)k, ws + B.oSemi, s);
        if (rc != 0) return rc;
    } else {
        const int64_t cnt = (int64_t)k * n;
        hipLaunchKernelGGL(k_bw_zero<T>, dim3((unsigned)std::min<int64_t>((cnt + 255) / 256, 4096)), dim3(256), 0, s, M,
                           cnt);
    }
    int pr = prof_take(MIID_K_BWD_GEMM, 0, m, n);
    // gA = C M  (J columns come out zero: M[:, J] = 0)
    MIID_LAUNCH(pr, k_bw_gemm_nn<T>, dim3((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64)), dim3(kBwThreads),
                       0, s, C, m, M, (int64_t)k, gA, ldga, m, n, k);
    // P = A M^T (m x k), split over n
    pr = prof_take(MIID_K_BWD_GEMM, 0, m, n);
    MIID_LAUNCH(pr, k_bw_gemm_nt<T>, dim3((unsigned)((m + 63) / 64), (unsigned)((k + 63) / 64), (unsigned)B.nz),
                dim3(kBwThreads), 0, s, A, lda, M, (int64_t)k, part, m, (int64_t)k, n);
    hipLaunchKernelGGL(k_bw_reduce<T>, dim3((unsigned)std::min<int64_t>((m * k + 255) / 256, 4096)), dim3(256), 0, s,
                       part, B.nz, m * k, P);
    // Q = Z M^T (k x k), split over n
    hipLaunchKernelGGL(k_bw_gemm_nt<T>, dim3((unsigned)((k + 63) / 64), (unsigned)((k + 63) / 64), (unsigned)B.nz),
                       dim3(kBwThreads), 0, s, Z, ldz, M, (int64_t)k, part, (int64_t)k, (int64_t)k, n);
    hipLaunchKernelGGL(k_bw_reduce<T>, dim3((unsigned)std::min<int64_t>(((int64_t)k * k + 255) / 256, 4096)), dim3(256),
                       0, s, part, B.nz, (int64_t)k * k, Q);
    hipLaunchKernelGGL(k_bw_jcols<T>, dim3((unsigned)std::min<int64_t>((m + 255) / 256, 64), (unsigned)k), dim3(256), 0,
                       s, C, P, Q, gC, ldgc, J, m, k, gA, ldga);
    MIID_HIP(hipGetLastError());
    return 0;
}

}  // namespace miid

using namespace miid;

extern "C" {

static size_t backward_workspace_body(int64_t m, int64_t n, int32_t k, miid_dtype dtype) {
    if (m < 1 || n < 1 || k < 1 || k > kBwMaxK || k > m || k > n) return 0;
    if (dtype != MIID_F32 && dtype != MIID_F64) return 0;
    return bw_plan(m, n, k, dtype == MIID_F64 ? 8 : 4).total;
}

static int backward_body(const void* A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype, const int32_t* J, int32_t k,
                const double* R11, int64_t ldr, const void* Z, int64_t ldz, const void* gC, int64_t ldgc,
                const void* gZ, int64_t ldgz, void* gA, int64_t ldga, void* ws, size_t ws_bytes, void* stream) {
    if (!A) return -1;
    if (m < 1) return -2;
    if (n < 1 || m > n) return -3;
    if (lda < m) return -4;
    if (dtype != MIID_F32 && dtype != MIID_F64) return -5;
    if (!J) return -6;
    if (k < 1 || k > m || k > kBwMaxK) return -7;
    if (!R11) return -8;
    if (ldr < k) return -9;
    if (!Z) return -10;
    if (ldz < k) return -11;
    if (gC && ldgc < m) return -13;
    if (gZ && ldgz < k) return -15;
    if (!gA) return -16;
    if (ldga < m) return -17;
    if (!ws) return -18;
    const size_t esz = dtype == MIID_F64 ? 8 : 4;
    const BwPlan B = bw_plan(m, n, k, esz);
    if (ws_bytes < B.total) return MIID_E_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    if (dtype == MIID_F64)
        return run_bw<double>((const double*)A, m, n, lda, J, k, R11, ldr, (const double*)Z, ldz, (const double*)gC,
                              ldgc, (const double*)gZ, ldgz, (double*)gA, ldga, w, B, s);
    return run_bw<float>((const float*)A, m, n, lda, J, k, R11, ldr, (const float*)Z, ldz, (const float*)gC, ldgc,
                         (const float*)gZ, ldgz, (float*)gA, ldga, w, B, s);
}

// ---- entry points: the handle checked, then the bodies above ------------
size_t miid_backward_workspace(miid_handle h, int64_t m, int64_t n, int32_t k, miid_dtype dtype) {
    if (check_handle(h) != 0) return 0;
    return backward_workspace_body(m, n, k, dtype);
}

int id_backward(miid_handle h, const void* A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype, const int32_t* J,
                int32_t k, const double* R11, int64_t ldr, const void* Z, int64_t ldz, const void* gC, int64_t ldgc,
                const void* gZ, int64_t ldgz, void* gA, int64_t ldga, void* ws, size_t ws_bytes, void* stream) {
    if (check_handle(h) != 0) return -1;
    return shift_arg(backward_body(A, m, n, lda, dtype, J, k, R11, ldr, Z, ldz, gC, ldgc, gZ, ldgz, gA, ldga, ws,
                                   ws_bytes, stream));
}

}  // extern "C"
