// batched.hip -- many independent small IDs in one persistent launch.
//
// Paper: Advani & O'Hagan, Section 2.1 (column-pivoted QR selects C, Z from
// the triangular solves), Section 4.1 (stop the QR once enough columns are
// chosen), Definition 1 (Z[:, J] = I).  Here each block stops at the smallest
// k whose residual ||R22||_F <= eps ||A_b||_F.
//
// Design: one workgroup works on one block at a time and takes the next block
// from an atomic queue over the blocks sorted by decreasing m * n (longest
// first), so uneven sizes balance across the chip.  The block is copied into
// the workgroup's slab of the workspace and factored with unblocked
// Householder steps: every step applies the reflector to each remaining column
// and recomputes that column's residual norm exactly (FP64 accumulation) in
// the same pass -- at eps = 1e-6 in FP32 the downdated norms would have lost
// all their digits anyway.  R stays in the slab's first k rows (no column
// swaps); the k x k triangle is staged in LDS in FP64 for the solve.
#include <algorithm>
#include <climits>

#include "common.hpp"
#include "cpqr.hpp"
#include "prof.hpp"

namespace miid {

constexpr int kBThreads = 1024;
constexpr int kBWaves = kBThreads / kWave;
constexpr int kBMaxM = 256;
constexpr int kBMaxN = 1024;
constexpr int kBMaxK = 64;
constexpr int kBRows = kBMaxM / kWave;  // rows per lane
constexpr int kBLdsBytes = 88 * 1024;   // LDS for a whole block when it fits
constexpr uint32_t kBlockUnsupported = 16u;

// Sort block indices by decreasing m * n (ties by index) into order[]:
// bitonic sort of (size, index) keys in LDS by one workgroup.
__global__ void __launch_bounds__(1024) k_lpt_order(const int32_t* __restrict__ m, const int32_t* __restrict__ n,
                                                    int32_t nblk, int32_t* __restrict__ order) {
    __shared__ uint64_t key[8192];
    int P = 1;
    while (P < nblk) P <<= 1;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        if (i < nblk) {
            const uint64_t sz = (uint64_t)(int64_t)m[i] * (uint64_t)(int64_t)n[i];
            // larger size first: sort ascending on (~size, index)
            key[i] = ((~sz & 0xFFFFFFFFull) << 32) | (uint64_t)(uint32_t)i;
        } else {
            key[i] = ~0ull;
        }
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int ixj = i ^ jj;
                if (ixj > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t a = key[i], b = key[ixj];
                    if ((a > b) == up) {
                        key[i] = b;
                        key[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) order[i] = (int32_t)(key[i] & 0xFFFFFFFFull);
}

__global__ void k_iota(int32_t* __restrict__ order, int32_t nblk, int32_t* __restrict__ queue) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nblk; i += gridDim.x * blockDim.x) order[i] = i;
    if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0;
}

__global__ void k_zero_queue(int32_t* __restrict__ queue) {
    if (threadIdx.x == 0) *queue = 0;
}

template <typename T>
struct BLds {
    static constexpr int elems = kBLdsBytes / (int)sizeof(T);
};

template <typename T>
__global__ void __launch_bounds__(kBThreads) k_batched(const T* __restrict__ A, const int64_t* __restrict__ a_off,
                                                       const int32_t* __restrict__ mv, const int32_t* __restrict__ nv,
                                                       int32_t nblk, double eps, int32_t kmax,
                                                       int32_t* __restrict__ J, const int64_t* __restrict__ j_off,
                                                       T* __restrict__ Z, const int64_t* __restrict__ z_off,
                                                       miid_info* __restrict__ info,
                                                       const int32_t* __restrict__ order, int32_t* __restrict__ queue,
                                                       T* __restrict__ slabs, int64_t slab_elems) {
    constexpr int kBLdsElems = BLds<T>::elems;
    __shared__ __align__(16) T sW[kBLdsElems];   // the block when it fits
    __shared__ double sR[kBMaxK * (kBMaxK + 1)];
    __shared__ double nu[kBMaxN];
    __shared__ T sv[kBMaxM];
    __shared__ double w_best[kBWaves], w_sum[kBWaves];
    __shared__ int32_t w_idx[kBWaves];
    __shared__ int32_t s_blk;
    __shared__ int32_t s_sel[kBMaxK];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    T* slab = slabs + (int64_t)blockIdx.x * slab_elems;

    for (;;) {
        if (tid == 0) s_blk = atomicAdd(queue, 1);
        __syncthreads();
        const int32_t q = s_blk;
        __syncthreads();
        if (q >= nblk) break;  // every wave leaves here once the queue is drained
        const int32_t b = order[q];
        const int m = mv[b], n = nv[b];
        const int kb = min(min(m, n), kmax);
        if (m < 1 || n < 1 || m > kBMaxM || n > kBMaxN || m > n || kb > kBMaxK) {
            if (tid == 0) info[b] = miid_info{0, kBlockUnsupported, 0.0, 0.0, 0, 0};
            continue;
        }
        const T* Ab = A + a_off[b];
        T* W = ((int64_t)m * n <= kBLdsElems) ? sW : slab;  // flat pointer: LDS or global
        for (int64_t e = tid; e < (int64_t)m * n; e += kBThreads) W[e] = Ab[e];
        __syncthreads();
        // exact column norms (FP64 accumulation) and ||A_b||_F
        double fro = 0.0;
        for (int c = wave; c < n; c += kBWaves) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < kBRows; ++t) {
                const int r = lane + kWave * t;
                if (r < m) {
                    const double x = (double)W[(int64_t)c * m + r];
                    s += x * x;
                }
            }
            s = wave_sum(s);
            if (lane == 0) nu[c] = sqrt(s);
            fro += s;
        }
        if (lane == 0) w_sum[wave] = fro;
        __syncthreads();
        double a2 = 0.0;
        for (int w = 0; w < kBWaves; ++w) a2 += w_sum[w];
        const double a_norm = sqrt(a2);
        const double stop_abs = eps * a_norm;
        __syncthreads();

        int k = 0;
        uint32_t status = 0;
        double resid = a_norm;
        const bool nonfinite = !(a_norm <= 1.0e300);
        if (nonfinite) status |= MIID_NONFINITE;
        while (!nonfinite) {
            // pivot: largest residual norm among the alive columns (one per thread)
            ArgMax best{-1.0, INT32_MAX};
            double ss = 0.0;
            for (int c = tid; c < n; c += kBThreads) {
                const double v = nu[c];
                if (v >= 0.0) {
                    if (argmax_better(v, c, best.v, best.i)) best = {v, c};
                    ss += v * v;
                }
            }
            best = wave_argmax(best);
            ss = wave_sum(ss);
            if (lane == 0) {
                w_best[wave] = best.v;
                w_idx[wave] = best.i;
                w_sum[wave] = ss;
            }
            __syncthreads();
            best = ArgMax{w_best[0], w_idx[0]};
            ss = w_sum[0];
            for (int w = 1; w < kBWaves; ++w) {
                if (argmax_better(w_best[w], w_idx[w], best.v, best.i)) best = {w_best[w], w_idx[w]};
                ss += w_sum[w];
            }
            resid = sqrt(ss);
            __syncthreads();
            if (resid <= stop_abs) break;
            if (k >= kb) {
                status |= MIID_KMAX_HIT;
                break;
            }
            if (!(best.v > 0.0)) {
                status |= MIID_RANK_DEFICIENT;
                break;
            }
            const int p = best.i;
            const int j = k;
            // Householder reflector of W[j:, p]
            T* wp = W + (int64_t)p * m;
            if (wave == 0) {
                double xs = 0.0;
#pragma unroll
                for (int t = 0; t < kBRows; ++t) {
                    const int r = lane + kWave * t;
                    if (r > j && r < m) {
                        const double x = (double)wp[r];
                        xs += x * x;
                    }
                }
                xs = wave_sum(xs);
                if (lane == 0) w_sum[0] = xs;
            }
            __syncthreads();
            const double x0 = (double)wp[j];
            const double alpha = sqrt(x0 * x0 + w_sum[0]);
            const double beta = x0 >= 0.0 ? -alpha : alpha;
            const double tau = (beta - x0) / beta;
            const double scale = 1.0 / (x0 - beta);
            for (int r = tid; r < m; r += kBThreads)
                sv[r] = r < j ? T(0) : (r == j ? T(1) : (T)((double)wp[r] * scale));
            __syncthreads();
            if (tid == 0) {
                wp[j] = (T)beta;
                nu[p] = -1.0;
                s_sel[j] = p;
            }
            double vr[kBRows];
#pragma unroll
            for (int t = 0; t < kBRows; ++t) {
                const int r = lane + kWave * t;
                vr[t] = r < m ? (double)sv[r] : 0.0;
            }
            // apply H = I - tau v v^T to the other alive columns, two at a
            // time per wave, and recompute their residual norms exactly
            for (int c0 = wave * 2; c0 < n; c0 += 2 * kBWaves) {
                int cc[2];
                bool act[2];
                double x[2][kBRows], d[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    cc[u] = c0 + u;
                    act[u] = cc[u] < n && cc[u] != p && nu[cc[u]] >= 0.0;
                    d[u] = 0.0;
#pragma unroll
                    for (int t = 0; t < kBRows; ++t) {
                        const int r = lane + kWave * t;
                        x[u][t] = (act[u] && r >= j && r < m) ? (double)W[(int64_t)cc[u] * m + r] : 0.0;
                        d[u] += x[u][t] * vr[t];
                    }
                }
                d[0] = tau * wave_sum(d[0]);
                d[1] = tau * wave_sum(d[1]);
                double s2[2] = {0.0, 0.0};
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (!act[u]) continue;
#pragma unroll
                    for (int t = 0; t < kBRows; ++t) {
                        const int r = lane + kWave * t;
                        if (r >= j && r < m) {
                            const T y = (T)(x[u][t] - d[u] * vr[t]);
                            W[(int64_t)cc[u] * m + r] = y;
                            if (r > j) s2[u] += (double)y * (double)y;
                        }
                    }
                }
                s2[0] = wave_sum(s2[0]);
                s2[1] = wave_sum(s2[1]);
                if (lane == 0) {
                    if (act[0]) nu[cc[0]] = sqrt(s2[0]);
                    if (act[1]) nu[cc[1]] = sqrt(s2[1]);
                }
            }
            ++k;
            __syncthreads();
        }

        // triangular solve: Z[:, c] = R11^{-1} R[:, c] in FP64, Z[:, J[i]] = e_i
        for (int e = tid; e < k * k; e += kBThreads) {
            const int a = e % k, c = e / k;
            sR[a * (kBMaxK + 1) + c] = a <= c ? (double)W[(int64_t)s_sel[c] * m + a] : 0.0;
        }
        __syncthreads();
        T* Zb = Z + z_off[b];
        int32_t* Jb = J + j_off[b];
        for (int i = tid; i < kb; i += kBThreads) Jb[i] = i < k ? s_sel[i] : -1;
        // one wave per column, lane i holds z_i (k <= 64): right-looking
        // substitution, z_t broadcast by a shuffle
        for (int c = wave; c < n; c += kBWaves) {
            T* zc = Zb + (int64_t)c * kb;
            if (nu[c] < 0.0) {
                int sidx = 0;
                for (int i = 0; i < k; ++i)
                    if (s_sel[i] == c) sidx = i;
                if (lane < kb) zc[lane] = (T)(lane == sidx ? 1.0 : 0.0);
                continue;
            }
            double z = lane < k ? (double)W[(int64_t)c * m + lane] : 0.0;
            for (int t = k - 1; t >= 0; --t) {
                const double zt = __shfl(z, t, kWave) / sR[t * (kBMaxK + 1) + t];
                if (lane == t) z = zt;
                if (lane < t) z -= sR[lane * (kBMaxK + 1) + t] * zt;
            }
            if (lane < kb) zc[lane] = (T)(lane < k ? z : 0.0);
        }
        if (tid == 0) info[b] = miid_info{k, status, a_norm, resid, 0, k};
        __syncthreads();
    }
}

}  // namespace miid

using namespace miid;

namespace {
struct BPlan {
    int grid;
    size_t oOrder, oQueue, oSlab, total;
    int64_t slab_elems;
};

BPlan batched_plan(int32_t nblk, size_t esz) {
    BPlan P;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    P.grid = std::max(1, std::min(nblk, cus));
    P.slab_elems = (int64_t)kBMaxM * kBMaxN;
    size_t off = 0;
    P.oOrder = off;
    off = align_up(off + (size_t)std::max(nblk, 1) * 4, 256);
    P.oQueue = off;
    off = align_up(off + 4, 256);
    P.oSlab = off;
    off = align_up(off + (size_t)P.grid * P.slab_elems * esz, 256);
    P.total = off;
    return P;
}
}  // namespace

extern "C" {

size_t miid_batched_workspace(int32_t nblk, miid_dtype dtype) {
    if (nblk < 1 || (dtype != MIID_F32 && dtype != MIID_F64)) return 0;
    return batched_plan(nblk, dtype == MIID_F64 ? 8 : 4).total;
}

int id_batched(int32_t nblk, const void* A, const int64_t* a_off, const int32_t* m, const int32_t* n,
               miid_dtype dtype, double eps, int32_t kmax, int32_t* J, const int64_t* j_off, void* Z,
               const int64_t* z_off, miid_info* info, void* ws, size_t ws_bytes, void* stream) {
    if (nblk < 1) return -1;
    if (!A) return -2;
    if (!a_off) return -3;
    if (!m) return -4;
    if (!n) return -5;
    if (dtype != MIID_F32 && dtype != MIID_F64) return -6;
    if (!(eps >= 0.0)) return -7;
    if (kmax < 1 || kmax > kBMaxK) return -8;
    if (!J) return -9;
    if (!j_off) return -10;
    if (!Z) return -11;
    if (!z_off) return -12;
    if (!info) return -13;
    if (!ws) return -14;
    const size_t esz = dtype == MIID_F64 ? 8 : 4;
    const BPlan P = batched_plan(nblk, esz);
    if (ws_bytes < P.total) return MIID_E_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    int32_t* order = reinterpret_cast<int32_t*>(w + P.oOrder);
    int32_t* queue = reinterpret_cast<int32_t*>(w + P.oQueue);
    if (nblk <= 8192) {
        hipLaunchKernelGGL(k_lpt_order, dim3(1), dim3(1024), 0, s, m, n, nblk, order);
        hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, s, queue);
    } else {
        hipLaunchKernelGGL(k_iota, dim3(64), dim3(256), 0, s, order, nblk, queue);
    }
    const int pr = prof_take(MIID_K_BATCHED, 0, nblk, 0);
    if (dtype == MIID_F64) {
        MIID_LAUNCH(pr, k_batched<double>, dim3(P.grid), dim3(kBThreads), 0, s, (const double*)A, a_off, m, n,
                           nblk, eps, kmax, J, j_off, (double*)Z, z_off, info, order, queue,
                           reinterpret_cast<double*>(w + P.oSlab), P.slab_elems);
    } else {
        MIID_LAUNCH(pr, k_batched<float>, dim3(P.grid), dim3(kBThreads), 0, s, (const float*)A, a_off, m, n, nblk,
                           eps, kmax, J, j_off, (float*)Z, z_off, info, order, queue,
                           reinterpret_cast<float*>(w + P.oSlab), P.slab_elems);
    }
    MIID_HIP(hipGetLastError());
    return 0;
}

}  // extern "C"
