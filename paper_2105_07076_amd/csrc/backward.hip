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

// FP32 products on the matrix cores with LDS tiles (v_mfma_f32_32x32x2f32):
// OUT (rows x cols, column-major, ldo) = X Y over the K range of this
// workgroup, X rows x K column-major (ldx), and Y either K x cols column-major
// (YKC: K contiguous, ldy) or stored as cols x K column-major (Y[kk][c] at
// c + kk ldy).  128 x 128 output tile per workgroup, 64 x 64 per wave (2 x 2
// tiles of 32 x 32); K in chunks of 32, both operands staged in LDS as
// [k][row] / [k][col] (every lane of an MFMA operand read hits consecutive
// words), the next chunk's loads in flight while the current one is
// multiplied.  Operand layout: lane l holds row (column) l % 32 and
// k = l / 32; accumulator element r of lane l is row 8 (r / 4) + 4 (l / 32) +
// r % 4, column l % 32.  Workgroup z takes K range [z kper, (z + 1) kper)
// and writes OUT + z zstride (a split-K partial when gridDim.z > 1).
constexpr int kGlT = 128;  // output tile side
constexpr int kGlK = 32;   // K per chunk
constexpr int kGlLd = 132;  // LDS row stride (floats) of the row-contiguous tiles
constexpr int kGlLdT = 129; // LDS row stride of a transposed (K-contiguous) tile

typedef float bwf16_t __attribute__((ext_vector_type(16)));

template <bool YKC, bool VEC>
__global__ void __launch_bounds__(kBwThreads) k_bw_gemm_lds(const float* __restrict__ X, int64_t ldx,
                                                            const float* __restrict__ Y, int64_t ldy,
                                                            float* __restrict__ OUT, int64_t ldo, int64_t zstride,
                                                            int64_t rows, int64_t cols, int64_t K, int64_t kper) {
    __shared__ __align__(16) float sX[2][kGlK * kGlLd];
    __shared__ __align__(16) float sY[2][kGlK * kGlLd];
    constexpr int LY = YKC ? kGlLdT : kGlLd;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int64_t r0 = (int64_t)blockIdx.x * kGlT, c0 = (int64_t)blockIdx.y * kGlT;
    const int wr = (wave & 1) * 64, wcol = (wave >> 1) * 64;
    const int64_t kbeg = (int64_t)blockIdx.z * kper;
    const int64_t kend = std::min<int64_t>(K, kbeg + kper);
    OUT += (int64_t)blockIdx.z * zstride;

    // a chunk of a row-contiguous operand (P: rows x K, ld): 32 k of 128
    // rows, four rows per 16-byte load, four loads per thread
    auto load_rc = [&](const float* P, int64_t ld, int64_t p0, int64_t plim, int64_t k0, float4 (&v)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = tid + kBwThreads * i;
            const int kk = f / 32, q = f % 32;
            const int64_t p = p0 + 4 * q, k = k0 + kk;
            if (VEC && k < kend && p + 4 <= plim) {
                v[i] = *reinterpret_cast<const float4*>(P + p + k * ld);
            } else {
                float e[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) e[t] = (k < kend && p + t < plim) ? P[p + t + k * ld] : 0.f;
                v[i] = float4(e[0], e[1], e[2], e[3]);
            }
        }
    };
    auto store_rc = [&](float* S, const float4 (&v)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = tid + kBwThreads * i;
            *reinterpret_cast<float4*>(S + (f / 32) * kGlLd + 4 * (f % 32)) = v[i];
        }
    };
    // a chunk of a K-contiguous operand (Y: K x cols, ldy): 32 k of 128
    // columns, four k per 16-byte load, stored transposed
    auto load_kc = [&](int64_t k0, float4 (&v)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = tid + kBwThreads * i;
            const int c = f / 8, q = f % 8;
            const int64_t col = c0 + c, k = k0 + 4 * q;
            if (VEC && col < cols && k + 4 <= kend) {
                v[i] = *reinterpret_cast<const float4*>(Y + k + col * ldy);
            } else {
                float e[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) e[t] = (col < cols && k + t < kend) ? Y[k + t + col * ldy] : 0.f;
                v[i] = float4(e[0], e[1], e[2], e[3]);
            }
        }
    };
    auto store_kc = [&](float* S, const float4 (&v)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = tid + kBwThreads * i;
            const int c = f / 8, q = f % 8;
            S[(4 * q + 0) * kGlLdT + c] = v[i].x;
            S[(4 * q + 1) * kGlLdT + c] = v[i].y;
            S[(4 * q + 2) * kGlLdT + c] = v[i].z;
            S[(4 * q + 3) * kGlLdT + c] = v[i].w;
        }
    };
    auto load = [&](int64_t k0, float4 (&vx)[4], float4 (&vy)[4]) {
        load_rc(X, ldx, r0, rows, k0, vx);
        if (YKC)
            load_kc(k0, vy);
        else
            load_rc(Y, ldy, c0, cols, k0, vy);
    };
    auto store = [&](int buf, const float4 (&vx)[4], const float4 (&vy)[4]) {
        store_rc(sX[buf], vx);
        if (YKC)
            store_kc(sY[buf], vy);
        else
            store_rc(sY[buf], vy);
    };

    bwf16_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    float4 vx[4], vy[4];
    load(kbeg, vx, vy);
    store(0, vx, vy);
    __syncthreads();
    int cur = 0;
    const int hl = lane / 32, l32 = lane % 32;
    for (int64_t k0 = kbeg; k0 < kend; k0 += kGlK) {
        const bool more = k0 + kGlK < kend;
        if (more) load(k0 + kGlK, vx, vy);
        const float* xs = sX[cur] + hl * kGlLd + wr + l32;
        const float* ys = sY[cur] + hl * LY + wcol + l32;
#pragma unroll
        for (int ks = 0; ks < kGlK / 2; ++ks) {
            const float a0 = xs[2 * ks * kGlLd], a1 = xs[2 * ks * kGlLd + 32];
            const float b0 = ys[2 * ks * LY], b1 = ys[2 * ks * LY + 32];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (more) store(cur ^ 1, vx, vy);
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t col = c0 + wcol + 32 * j + l32;
            if (col >= cols) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = r0 + wr + 32 * i + 8 * q + 4 * hl;
                float* o = OUT + row + col * ldo;
                if (VEC && row + 4 <= rows) {
                    *reinterpret_cast<float4*>(o) =
                        float4(acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]);
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (row + t < rows) o[t] = acc[i][j][4 * q + t];
                }
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
    if constexpr (sizeof(T) == 4) {
        // FP32: LDS-tiled products on the 32x32x2 matrix-core instruction
        const uintptr_t al = 15;
        const bool vec = ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(Z) |
                           reinterpret_cast<uintptr_t>(gA)) & al) == 0 &&
                         lda % 4 == 0 && ldz % 4 == 0 && ldga % 4 == 0 && m % 4 == 0 && k % 4 == 0;
        auto gemm = [&](int pr, bool ykc, const T* X, int64_t ldx, const T* Y, int64_t ldy, T* OUT, int64_t ldo,
                        int64_t zstride, int64_t rows, int64_t cols, int64_t K, int nz) -> hipError_t {
            const int64_t kper = (int64_t)align_up((size_t)((K + nz - 1) / nz), kGlK);
            const dim3 grid((unsigned)((rows + kGlT - 1) / kGlT), (unsigned)((cols + kGlT - 1) / kGlT),
                            (unsigned)((K + kper - 1) / kper));
            if (ykc) {
                if (vec)
                    MIID_LAUNCH(pr, (k_bw_gemm_lds<true, true>), grid, dim3(kBwThreads), 0, s, X, ldx, Y, ldy, OUT,
                                ldo, zstride, rows, cols, K, kper);
                else
                    MIID_LAUNCH(pr, (k_bw_gemm_lds<true, false>), grid, dim3(kBwThreads), 0, s, X, ldx, Y, ldy, OUT,
                                ldo, zstride, rows, cols, K, kper);
            } else {
                if (vec)
                    MIID_LAUNCH(pr, (k_bw_gemm_lds<false, true>), grid, dim3(kBwThreads), 0, s, X, ldx, Y, ldy, OUT,
                                ldo, zstride, rows, cols, K, kper);
                else
                    MIID_LAUNCH(pr, (k_bw_gemm_lds<false, false>), grid, dim3(kBwThreads), 0, s, X, ldx, Y, ldy,
                                OUT, ldo, zstride, rows, cols, K, kper);
            }
            return hipGetLastError();
        };
        // gA = C M  (J columns come out zero: M[:, J] = 0)
        MIID_HIP(gemm(prof_take(MIID_K_BWD_GEMM, 0, m, n), true, C, m, M, (int64_t)k, gA, ldga, 0, m, n, k, 1));
        // P = A M^T (m x k): Y[kk][c] = M[c, kk]; split over n, fixed-order sum
        MIID_HIP(gemm(prof_take(MIID_K_BWD_GEMM, 1, m, n), false, A, lda, M, (int64_t)k, part, m, m * k, m, k, n,
                      B.nz));
        hipLaunchKernelGGL(k_bw_reduce<T>, dim3((unsigned)std::min<int64_t>((m * k + 255) / 256, 4096)), dim3(256), 0,
                           s, part, B.nz, m * k, P);
        // Q = Z M^T (k x k), split over n
        MIID_HIP(gemm(-1, false, Z, ldz, M, (int64_t)k, part, (int64_t)k, (int64_t)k * k, (int64_t)k, (int64_t)k, n,
                      B.nz));
        hipLaunchKernelGGL(k_bw_reduce<T>, dim3((unsigned)std::min<int64_t>(((int64_t)k * k + 255) / 256, 4096)),
                           dim3(256), 0, s, part, B.nz, (int64_t)k * k, Q);
    } else {
        int pr = prof_take(MIID_K_BWD_GEMM, 0, m, n);
        // gA = C M  (J columns come out zero: M[:, J] = 0)
        MIID_LAUNCH(pr, k_bw_gemm_nn<T>, dim3((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64)),
                    dim3(kBwThreads), 0, s, C, m, M, (int64_t)k, gA, ldga, m, n, k);
        // P = A M^T (m x k), split over n
        pr = prof_take(MIID_K_BWD_GEMM, 0, m, n);
        MIID_LAUNCH(pr, k_bw_gemm_nt<T>, dim3((unsigned)((m + 63) / 64), (unsigned)((k + 63) / 64), (unsigned)B.nz),
                    dim3(kBwThreads), 0, s, A, lda, M, (int64_t)k, part, m, (int64_t)k, n);
        hipLaunchKernelGGL(k_bw_reduce<T>, dim3((unsigned)std::min<int64_t>((m * k + 255) / 256, 4096)), dim3(256), 0,
                           s, part, B.nz, m * k, P);
        // Q = Z M^T (k x k), split over n
        hipLaunchKernelGGL(k_bw_gemm_nt<T>, dim3((unsigned)((k + 63) / 64), (unsigned)((k + 63) / 64),
                                                 (unsigned)B.nz),
                           dim3(kBwThreads), 0, s, Z, ldz, M, (int64_t)k, part, (int64_t)k, (int64_t)k, n);
        hipLaunchKernelGGL(k_bw_reduce<T>, dim3((unsigned)std::min<int64_t>(((int64_t)k * k + 255) / 256, 4096)),
                           dim3(256), 0, s, part, B.nz, (int64_t)k * k, Q);
    }
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
