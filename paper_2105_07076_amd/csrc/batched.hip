// batched.hip -- many independent small IDs in one persistent launch.
//
// Paper: Advani & O'Hagan, Section 2.1 (column-pivoted QR selects C, Z from
// the triangular solves), Section 4.1 (stop the QR once enough columns are
// chosen), Definition 1 (Z[:, J] = I).  Here each block stops at the smallest
// k whose residual ||R22||_F <= eps ||A_b||_F.
//
// Design: one workgroup works on one block at a time and takes the next block
// from an atomic queue over the blocks sorted by decreasing m * n (longest
// first), so uneven sizes balance across the chip.  Each Householder step
// applies the reflector to every remaining column and recomputes that
// column's residual norm exactly (FP64 accumulation) in the same pass -- at
// eps = 1e-6 in FP32 downdated norms would have lost all their digits.  The
// working copy W of the block stays in LDS when it fits; otherwise it lives
// in a per-workgroup scratch and every pass streams it through two LDS column
// tiles (the next tile's loads in flight while the current one is updated,
// the updated one written back behind it).  A column is handled by a 16-lane
// group (lane l16 takes rows l16 + 16 t; DPP row sums).  R stays in W's
// first k rows and is copied row by row into Z's storage (no column swaps);
// the k x k triangle is staged in LDS in FP64 for the solve, which then
// overwrites Z in place.
#include <algorithm>
#include <cmath>
#include <climits>

#include "common.hpp"
#include "cpqr.hpp"
#include "prof.hpp"

namespace miid {

constexpr int kBThreads = 512;
constexpr int kBWaves = kBThreads / kWave;
// dynamic LDS (V, then the block or its column tiles): what the 160 KB of a
// CU leave beside the kernel's static arrays
constexpr int bdyn_bytes(int) { return 148 * 1024; }
constexpr int kBTileBytes = 24 * 1024;  // default streamed column tile (the rest of LDS keeps columns resident)
constexpr int kBMaxM = 256;
constexpr int kBMaxN = 1024;
constexpr int kBMaxK = 64;
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

// Block-wide (value, index) argmax and sum: wave results through LDS, read
// back in wave order (identical in every thread).
__device__ __forceinline__ void block_argmax_sum(ArgMax& best, double& sum, ArgMax* w_best, double* w_sum) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    best = wave_argmax_dpp(best);
    sum = wave_sum_dpp(sum);
    if (lane == 0) {
        w_best[wave] = best;
        w_sum[wave] = sum;
    }
    lds_barrier();
    best = w_best[0];
    sum = w_sum[0];
    for (int w = 1; w < kBWaves; ++w) {
        if (argmax_better(w_best[w].v, w_best[w].i, best.v, best.i)) best = w_best[w];
        sum += w_sum[w];
    }
    lds_barrier();
}

__device__ __forceinline__ double block_sum(double v, double* w_sum) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    v = wave_sum_dpp(v);
    if (lane == 0) w_sum[wave] = v;
    lds_barrier();
    double t = 0.0;
    for (int w = 0; w < kBWaves; ++w) t += w_sum[w];
    lds_barrier();
    return t;
}

// Persistent kernel: one block at a time per workgroup (8 waves, one per CU).
typedef __attribute__((address_space(3))) uint32_t lds_u32;

template <typename T>
__global__ void __launch_bounds__(kBThreads) k_batched(const T* __restrict__ A, const int64_t* __restrict__ a_off,
                                                       const int32_t* __restrict__ mv, const int32_t* __restrict__ nv,
                                                       int32_t nblk, double eps, int32_t kmax,
                                                       int32_t* __restrict__ J, const int64_t* __restrict__ j_off,
                                                       T* __restrict__ Z, const int64_t* __restrict__ z_off,
                                                       miid_info* __restrict__ info,
                                                       const int32_t* __restrict__ order, int32_t* __restrict__ queue,
                                                       T* __restrict__ Wscr, int tile_bytes) {
    constexpr int kDyn = bdyn_bytes((int)sizeof(T)) / (int)sizeof(T);
    constexpr int kRT = kBMaxM / 16;              // rows per lane of a column group
    constexpr int kGroups = kBWaves * 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    __shared__ double snu[kBMaxN];
    __shared__ double s_v[kBMaxM];  // the reflector (v_j = 1, zero above j)
    __shared__ ArgMax w_best[kBWaves];
    __shared__ double w_sum[kBWaves];
    __shared__ int32_t s_sel[kBMaxK];
    __shared__ int32_t s_blk;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int l16 = lane & 15, grp = lane >> 4;
    const int cgroup = wave * 4 + grp;  // 16-lane column group
    T* Wb = Wscr + (int64_t)blockIdx.x * kBMaxM * kBMaxN;  // W when it does not fit in LDS

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
        T* Zb = Z + z_off[b];
        // LDS: the first cres columns stay resident for the whole block; the
        // other ns columns (if any) stream through two tiles of TC columns
        const bool resident = m * n <= kDyn;
        const int TC = resident ? 1 : max(1, min(n, min(kDyn / 2, tile_bytes / (int)sizeof(T)) / m));
        const int cres = resident ? n : min(n, max(0, (kDyn - 2 * TC * m) / m));
        const int ns = n - cres;
        const int nt = (ns + TC - 1) / TC;
        T* res = lds;
        T* buf0 = lds + cres * m;
        T* buf1 = buf0 + TC * m;
        if (cres > 0) {  // the resident columns straight into LDS
            const int cntw = cres * m * (int)(sizeof(T) / 4);
            const uint32_t* s32 = reinterpret_cast<const uint32_t*>(Ab);
            lds_u32* d32 = (lds_u32*)smem_raw;
            for (int e0 = 0; e0 < cntw; e0 += kBThreads) {
                const int e = e0 + tid;
                if (e < cntw) __builtin_amdgcn_global_load_lds((const void*)(s32 + e), d32 + (e - lane), 4, 0, 0);
            }
            __syncthreads();
        }

        // one pass over W: fn(l, column in LDS) for every column; the
        // streamed columns' tiles come from src (A on the first pass, the
        // scratch afterwards) and go back to the scratch when write is set
        auto pass = [&](const T* src, bool write, auto&& fn) {
            for (int l = cgroup; l < cres; l += kGroups) fn(l, res + l * m);
            if (ns == 0) {
                lds_barrier();
                return;
            }
            // a tile is a contiguous range of src; it goes straight from
            // global memory into LDS (global_load_lds: no registers, the
            // next tile's copy in flight while the current one is updated)
            auto issue = [&](int t) {
                const int c0 = cres + t * TC;
                const int cntw = min(TC, n - c0) * m * (int)(sizeof(T) / 4);
                const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src + (int64_t)c0 * m);
                lds_u32* d32 = (lds_u32*)smem_raw + (cres + ((t & 1) ? TC : 0)) * m * (int)(sizeof(T) / 4);
                for (int e0 = 0; e0 < cntw; e0 += kBThreads) {
                    const int e = e0 + tid;
                    if (e < cntw) __builtin_amdgcn_global_load_lds((const void*)(s32 + e), d32 + (e - lane), 4, 0, 0);
                }
            };
            issue(0);
            __syncthreads();
            for (int t = 0; t < nt; ++t) {
                if (t + 1 < nt) issue(t + 1);
                const int c0 = cres + t * TC, c1 = min(n, c0 + TC);
                T* cur = (t & 1) ? buf1 : buf0;
                for (int l = c0 + cgroup; l < c1; l += kGroups) fn(l, cur + (l - c0) * m);
                lds_barrier();
                if (write) {
                    const int cnt = (c1 - c0) * m;
                    T* d0 = Wb + (int64_t)c0 * m;
                    for (int e = tid; e < cnt; e += kBThreads) d0[e] = cur[e];
                }
                __syncthreads();  // the next tile has landed; this one is written back
            }
        };

        // exact column norms (FP64) and ||A_b||_F; a streamed block is copied
        // to the scratch on the way
        double fro = 0.0;
        pass(Ab, ns > 0, [&](int l, T* col) {
            double ss = 0.0;
#pragma unroll
            for (int t = 0; t < kRT; ++t) {
                const int r = l16 + 16 * t;
                if (r < m) {
                    const double x = (double)col[r];
                    ss += x * x;
                }
            }
            ss = row16_sum(ss);
            if (l16 == 0) {
                snu[l] = sqrt(ss);
                fro += ss;
            }
        });
        const double a2 = block_sum(fro, w_sum);
        const double a_norm = sqrt(a2);
        const double stop_abs = eps * a_norm;
        // W (the scratch writes of the copy) complete before it is read
        __syncthreads();

        int k = 0;
        uint32_t status = 0;
        double resid = a_norm;
        const bool nonfinite = !(a_norm <= 1.0e300);
        if (nonfinite) status |= MIID_NONFINITE;
        while (!nonfinite) {
            // pivot: largest residual norm among the alive columns
            ArgMax best{-1.0, INT32_MAX};
            double ss = 0.0;
            for (int l = tid; l < n; l += kBThreads) {
                const double v = snu[l];
                if (v >= 0.0) {
                    if (argmax_better(v, l, best.v, best.i)) best = {v, l};
                    ss += v * v;
                }
            }
            block_argmax_sum(best, ss, w_best, w_sum);
            resid = sqrt(ss);
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
            // Householder reflector of W[j:, p] (one thread per row)
            const T* colp = p < cres ? res + p * m : Wb + (int64_t)p * m;
            const double x = (tid < m && tid >= j) ? (double)colp[tid] : 0.0;
            const double s0 = block_sum(tid > j && tid < m ? x * x : 0.0, w_sum);
            if (tid == j) s_v[kBMaxM - 1] = x;  // x0 (row j) parked in the last slot
            lds_barrier();
            const double x0 = tid == j ? x : s_v[kBMaxM - 1];
            lds_barrier();
            const double alpha = sqrt(x0 * x0 + s0);
            if (!(alpha > 0.0)) {
                status |= MIID_RANK_DEFICIENT;
                break;
            }
            const double beta = x0 >= 0.0 ? -alpha : alpha;
            const double tau = (beta - x0) / beta;
            const double scale = 1.0 / (x0 - beta);
            if (tid < kBMaxM) s_v[tid] = (tid < j || tid >= m) ? 0.0 : (tid == j ? 1.0 : (double)(T)(x * scale));
            if (tid == 0) {
                s_sel[j] = p;
                snu[p] = -1.0;
                Zb[j + (int64_t)p * kb] = (T)beta;
            }
            lds_barrier();
            // apply H = I - tau v v^T to the alive columns, row j of R, exact
            // new norms of rows j+1..m-1
            pass(Wb, ns > 0, [&](int l, T* col) {
                if (!(snu[l] >= 0.0)) return;  // dead column (uniform over the group)
                double xr[kRT];
                double d = 0.0;
#pragma unroll
                for (int t = 0; t < kRT; ++t) {
                    const int r = l16 + 16 * t;
                    xr[t] = (r >= j && r < m) ? (double)col[r] : 0.0;
                    d += xr[t] * s_v[r < kBMaxM ? r : 0];
                }
                d = tau * row16_sum(d);
                double s2 = 0.0;
#pragma unroll
                for (int t = 0; t < kRT; ++t) {
                    const int r = l16 + 16 * t;
                    if (r >= j && r < m) {
                        const T y = (T)(xr[t] - d * s_v[r]);
                        col[r] = y;
                        if (r == j) Zb[j + (int64_t)l * kb] = y;
                        if (r > j) s2 += (double)y * (double)y;
                    }
                }
                s2 = row16_sum(s2);
                if (l16 == 0) snu[l] = sqrt(s2);
            });
            ++k;
            __syncthreads();  // R rows and the scratch writes of step j are complete
        }

        // triangular solve: Z[:, l] = R11^{-1} R[:, l] in FP64, Z[:, J[i]] = e_i
        double* sR = reinterpret_cast<double*>(smem_raw);  // reuses the dynamic LDS: k x (kBMaxK + 1)
        __syncthreads();
        for (int e = tid; e < k * k; e += kBThreads) {
            const int a = e % k, c = e / k;
            sR[a * (kBMaxK + 1) + c] = a <= c ? (double)Zb[a + (int64_t)s_sel[c] * kb] : 0.0;
        }
        __syncthreads();
        int32_t* Jb = J + j_off[b];
        for (int i = tid; i < kb; i += kBThreads) Jb[i] = i < k ? s_sel[i] : -1;
        // four lanes per column (a quad), lane c of the quad holds z_q for
        // q = 4 i + c: back substitution with the solved z_t broadcast from
        // its owner inside the quad (DPP quad permutes)
        for (int l0 = tid / 4; l0 < n; l0 += kBThreads / 4) {
            const int l = l0;
            const int c = tid % 4;
            T* zc = Zb + (int64_t)l * kb;
            const bool dead = snu[l] < 0.0;
            double z[kBMaxK / 4];
#pragma unroll
            for (int i = 0; i < kBMaxK / 4; ++i) {
                const int qq = 4 * i + c;
                z[i] = (!dead && qq < k) ? (double)zc[qq] : 0.0;
            }
#pragma unroll
            for (int i = kBMaxK / 4 - 1; i >= 0; --i) {
#pragma unroll
                for (int r = 3; r >= 0; --r) {
                    const int t = 4 * i + r;
                    if (t >= k) continue;  // uniform
                    double zt = z[i] / sR[t * (kBMaxK + 1) + t];
                    zt = r == 0 ? dpp_f64<0x00>(zt) : (r == 1 ? dpp_f64<0x55>(zt) : (r == 2 ? dpp_f64<0xAA>(zt) : dpp_f64<0xFF>(zt)));
                    if (c == r) z[i] = zt;
#pragma unroll
                    for (int i2 = 0; i2 <= i; ++i2) {
                        const int qq = 4 * i2 + c;
                        if (qq < t) z[i2] -= sR[qq * (kBMaxK + 1) + t] * zt;
                    }
                }
            }
            int sidx = -1;
            if (dead)
                for (int i = 0; i < k; ++i)
                    if (s_sel[i] == l) sidx = i;
#pragma unroll
            for (int i = 0; i < kBMaxK / 4; ++i) {
                const int qq = 4 * i + c;
                if (qq < kb) zc[qq] = dead ? (T)(qq == sidx ? 1.0 : 0.0) : (T)(qq < k ? z[i] : 0.0);
            }
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
    size_t oOrder, oQueue, oW, total;
};

// One workgroup per CU (8 waves; LDS: the block or two column tiles of it).
BPlan batched_plan(int32_t nblk, size_t esz) {
    BPlan P;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    P.grid = std::max(1, std::min(nblk, cus));
    size_t off = 0;
    P.oOrder = off;
    off = align_up(off + (size_t)std::max(nblk, 1) * 4, 256);
    P.oQueue = off;
    off = align_up(off + 4, 256);
    P.oW = off;
    off = align_up(off + (size_t)P.grid * kBMaxM * kBMaxN * esz, 256);
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
               miid_dtype dtype, const miid_opts* opts, int32_t* J, const int64_t* j_off, void* Z,
               const int64_t* z_off, miid_info* info, void* ws, size_t ws_bytes, void* stream) {
    if (nblk < 1) return -1;
    if (!A) return -2;
    if (!a_off) return -3;
    if (!m) return -4;
    if (!n) return -5;
    if (dtype != MIID_F32 && dtype != MIID_F64) return -6;
    if (!opts || !(opts->eps >= 0.0) || opts->kmax < 1 || opts->kmax > kBMaxK) return -7;
    if (!J) return -8;
    if (!j_off) return -9;
    if (!Z) return -10;
    if (!z_off) return -11;
    if (!info) return -12;
    if (!ws) return -13;
    const double eps = opts->eps;
    const int32_t kmax = opts->kmax;
    const int tile_hint = (int)((opts->flags >> MIID_HINT_TILE_SHIFT) & 15u);
    const int tile_bytes = tile_hint >= 1 ? tile_hint * 8 * 1024 : kBTileBytes;
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
    const size_t shmem = (size_t)bdyn_bytes((int)esz);
    if (dtype == MIID_F64) {
        static bool attr64 = false;
        if (!attr64) {
            MIID_HIP(hipFuncSetAttribute((const void*)k_batched<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         bdyn_bytes(8)));
            attr64 = true;
        }
        MIID_LAUNCH(pr, k_batched<double>, dim3(P.grid), dim3(kBThreads), shmem, s, (const double*)A, a_off, m, n,
                    nblk, eps, kmax, J, j_off, (double*)Z, z_off, info, order, queue,
                    reinterpret_cast<double*>(w + P.oW), tile_bytes);
    } else {
        static bool attr32 = false;
        if (!attr32) {
            MIID_HIP(hipFuncSetAttribute((const void*)k_batched<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         bdyn_bytes(4)));
            attr32 = true;
        }
        MIID_LAUNCH(pr, k_batched<float>, dim3(P.grid), dim3(kBThreads), shmem, s, (const float*)A, a_off, m, n,
                    nblk, eps, kmax, J, j_off, (float*)Z, z_off, info, order, queue,
                    reinterpret_cast<float*>(w + P.oW), tile_bytes);
    }
    MIID_HIP(hipGetLastError());
    return 0;
}

}  // extern "C"
