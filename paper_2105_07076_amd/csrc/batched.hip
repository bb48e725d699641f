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
// eps = 1e-6 in FP32 downdated norms would have lost all their digits.  A
// column is handled by a 16-lane group (lane l16 takes rows l16 + 16 t; DPP
// row sums), with the rows per lane fitted to m.  The working copy W of the
// block is spread over the chip: its first columns in registers, the next in
// LDS, and whatever does not fit in a per-workgroup scratch that every pass
// streams through two LDS column tiles (the next tile's loads in flight while
// the current one is updated, the updated one written back behind it).  The
// waves stage their best columns at the end of a pass and every lane forms
// the next reflector itself, so a step costs two workgroup barriers and no
// serial section.  R stays in W's first k rows and is copied row by row into Z's
// storage (no column swaps); the k x k triangle is staged in LDS in FP64 for
// the solve, which then overwrites Z in place.
#include <algorithm>
#include <cmath>
#include <climits>

#include "common.hpp"
#include "cpqr.hpp"
#include "prof.hpp"

namespace miid {

constexpr int kBThreads = 512;
constexpr int kBWaves = kBThreads / kWave;
// dynamic LDS (the block's LDS columns and tiles, later the triangle of the
// solve): what the 160 KB of a CU leave beside the kernel's static arrays
// (residual norms, the waves' staged columns, a few scalars)
constexpr int bdyn_bytes(int esz) { return 160 * 1024 - 9 * 1024 - 8 * 256 * esz; }
constexpr int kBTileBytes = 24 * 1024;  // default streamed column tile (the rest of LDS keeps columns resident)
constexpr int kBMaxM = 256;
constexpr int kBMaxN = 1024;
constexpr int kBMaxK = 64;
constexpr uint32_t kBlockUnsupported = 16u;

// Order the blocks by decreasing size for the queue (longest first): a
// counting sort of one workgroup on the coarse key m n / 256 (1024 buckets
// cover every admissible block; the order inside a bucket is whatever the
// LDS atomics give -- it only affects which workgroup takes a block, not its
// result).  Also zeroes the queue.
constexpr int kLptBuckets = 1024;

__global__ void __launch_bounds__(1024) k_lpt_order(const int32_t* __restrict__ m, const int32_t* __restrict__ n,
                                                    int32_t nblk, int32_t* __restrict__ order,
                                                    int32_t* __restrict__ queue) {
    __shared__ int32_t cnt[kLptBuckets];
    __shared__ int32_t scan[kLptBuckets];
    const int tid = threadIdx.x;
    auto bucket = [&](int i) {
        const int64_t sz = (int64_t)max(m[i], 0) * (int64_t)max(n[i], 0);
        return kLptBuckets - 1 - (int)min<int64_t>(sz >> 8, kLptBuckets - 1);  // larger first
    };
    for (int b = tid; b < kLptBuckets; b += blockDim.x) cnt[b] = 0;
    __syncthreads();
    for (int i = tid; i < nblk; i += blockDim.x) atomicAdd(&cnt[bucket(i)], 1);
    __syncthreads();
    // exclusive prefix sum over the buckets (one per thread, Hillis-Steele)
    const int v = tid < kLptBuckets ? cnt[tid] : 0;
    if (tid < kLptBuckets) scan[tid] = v;
    __syncthreads();
    for (int d = 1; d < kLptBuckets; d <<= 1) {
        const int t = (tid < kLptBuckets && tid >= d) ? scan[tid - d] : 0;
        __syncthreads();
        if (tid < kLptBuckets) scan[tid] += t;
        __syncthreads();
    }
    if (tid < kLptBuckets) cnt[tid] = scan[tid] - v;  // start of the bucket
    __syncthreads();
    for (int i = tid; i < nblk; i += blockDim.x) order[atomicAdd(&cnt[bucket(i)], 1)] = i;
    if (tid == 0) *queue = 0;
}


typedef __attribute__((address_space(3))) uint32_t lds_u32;

// Columns of a block kept in registers, per 16-lane group: what the pass
// leaves free of the 256 VGPRs a lane has at two waves per SIMD (FP64
// columns take twice the registers and the pass's FP64 state more too).
template <typename T, int RT>
constexpr int breg_cols() {
    return sizeof(T) == 4 ? (RT == 2 ? 32 : (RT == 4 ? 40 : 48)) / RT
                          : (RT == 16 ? 0 : 16 / (2 * RT));
}

// a * b + c with one rounding, in the working precision
__device__ __forceinline__ float fma_w(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_w(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The kernel's static LDS, handed to the per-block factorisation.
template <typename T>
struct BShared {
    double* snu;     // residual norm of every column (-1: chosen)
    ArgMax* w_best;  // per wave
    double* w_sum;   // per wave
    T* w_col;        // per wave its best column (kBMaxM rows)
    int32_t* s_sel;  // chosen columns in order
};

struct BResult {
    int k;
    uint32_t status;
    double a_norm, resid;
};

// Pivoted Householder QR of one block, stopped by the tolerance.  A column
// belongs to the 16-lane group (column mod 32); lane l16 holds rows
// l16 + 16 t, t < RT (RT = ceil(m / 16) rounded up to 2, 4, 8 or 16).  The
// first 32 NR columns live in registers, the next cres in LDS, the rest in
// the workgroup's scratch Wb, streamed through two LDS tiles of TC columns
// per pass.  Columns in LDS and in the scratch are stored with the row count
// padded to mp = a multiple of 16 (zeros below row m), so whole slices t are
// either in the column or not and no per-row bounds are needed.
//
// A step: at the end of the previous pass each wave stages its best column
// (and its residual norm and sum) in LDS; after one barrier every lane picks
// the pivot from the eight wave entries and forms the reflector itself from
// the staged column -- alpha is the pivot's residual norm from the pass (its
// rows j.. are what the reflector annihilates), so only x0 = x[j] is read --
// and after a second barrier (the staging area is reused) the pass applies
// H = I - tau v v^T to every alive column, writes row j of R into Zb and
// recomputes the residual norms exactly (FP64 accumulation of the stored
// values).
template <typename T, int RT>
__device__ __forceinline__ BResult factor_block(const T* __restrict__ Ab, T* __restrict__ Zb, T* __restrict__ Wb,
                                                int m, int n, int kb, double eps, int tile_bytes,
                                                unsigned char* smem_raw, BShared<T> sh) {
    constexpr int NR = breg_cols<T, RT>();
    constexpr int kDyn = bdyn_bytes((int)sizeof(T)) / (int)sizeof(T);
    constexpr int kGroups = kBWaves * 4;
    const int tid = threadIdx.x;
    const int lane = tid % kWave;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    int l16 = lane & 15;
    // opaque to the optimiser: what is derived from it is formed here, per
    // block, instead of being hoisted out of the persistent loop for every
    // RT instance and held in registers throughout
    asm volatile("" : "+v"(l16));
    const int cgroup = tid / 16;  // 16-lane column group, 0..31
    T* lds = reinterpret_cast<T*>(smem_raw);

    const int mp = (m + 15) & ~15;
    const int ntv = mp / 16;  // slices t inside a padded column
    const int nreg = min(n, kGroups * NR);
    const int nrest = n - nreg;
    const bool resident = nrest * mp <= kDyn;
    const int TC = resident ? 1 : max(1, min(nrest, min(kDyn / 2, tile_bytes / (int)sizeof(T)) / mp));
    const int cres = resident ? nrest : min(nrest, max(0, (kDyn - 2 * TC * mp) / mp));
    const int c_str = nreg + cres;  // first streamed column
    const int ns = n - c_str;
    const int nt = (ns + TC - 1) / TC;
    T* buf0 = lds + cres * mp;
    T* buf1 = buf0 + TC * mp;
    // home of column l >= nreg: LDS or the scratch
    auto home = [&](int l) { return l < c_str ? lds + (l - nreg) * mp : Wb + (int64_t)l * mp; };

    T rc[NR > 0 ? NR : 1][RT];  // register-resident columns cgroup + 32 c (zero below row m)
    T sv[RT];      // v at this lane's rows (v is rounded to T, so exact)
    ArgMax gb{-1.0, INT32_MAX};  // the group's best (the same in its 16 lanes)
    double acc = 0.0;            // the group's sum (the same in its 16 lanes)

    // a column's new residual norm: the group's best and sum, branch-free
    auto consider = [&](int l, double nu, double add) {
        acc += add;
        const bool bt = argmax_better(nu, l, gb.v, gb.i);
        gb.v = bt ? nu : gb.v;
        gb.i = bt ? l : gb.i;
    };
    // the wave's best of its four groups (row leaders, fixed order), staged
    // with its column; a streamed column is read back from the scratch
    // (written there by other lanes: device scope, past this CU's L1)
    auto publish = [&]() {
        ArgMax wbst{-1.0, INT32_MAX};
        double wsum = 0.0;
        int wrow = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t bits = __builtin_bit_cast(int64_t, gb.v);
            const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffff), 16 * r);
            const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), 16 * r);
            const double v = __builtin_bit_cast(double, ((int64_t)hi << 32) | (uint32_t)lo);
            const int32_t i = __builtin_amdgcn_readlane(gb.i, 16 * r);
            const int64_t abits = __builtin_bit_cast(int64_t, acc);
            const int alo = __builtin_amdgcn_readlane((int)(abits & 0xffffffff), 16 * r);
            const int ahi = __builtin_amdgcn_readlane((int)(abits >> 32), 16 * r);
            wsum += __builtin_bit_cast(double, ((int64_t)ahi << 32) | (uint32_t)alo);
            if (argmax_better(v, i, wbst.v, wbst.i)) {
                wbst = {v, i};
                wrow = r;
            }
        }
        const int q = wbst.i;  // wave-uniform
        if ((lane >> 4) == wrow && wbst.v >= 0.0) {
            T* slot = sh.w_col + wave * kBMaxM;
            if (q < nreg) {
                // one uniform branch per register column (a select chain
                // over c would be turned into an indexed, memory-held array)
                const int cq = q / kGroups;
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    if (c == cq) {
#pragma unroll
                        for (int t = 0; t < RT; ++t) slot[l16 + 16 * t] = rc[c][t];
                    }
                }
            } else if (q < c_str) {
                const T* col = lds + (q - nreg) * mp;
#pragma unroll
                for (int t = 0; t < RT; ++t) slot[l16 + 16 * t] = t < ntv ? col[l16 + 16 * t] : T(0);
            } else {
                const T* col = Wb + (int64_t)q * mp;
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    const int r = l16 + 16 * t;
                    slot[r] = t < ntv ? __hip_atomic_load(col + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : T(0);
                }
            }
        }
        if (lane == 0) {
            sh.w_best[wave] = wbst;
            sh.w_sum[wave] = wsum;
        }
    };

    // copy the streamed tile t of the scratch into its LDS buffer (no registers)
    auto issue = [&](int t) {
        const int c0 = c_str + t * TC;
        const int cntw = min(TC, n - c0) * mp * (int)(sizeof(T) / 4);
        const uint32_t* s32 = reinterpret_cast<const uint32_t*>(Wb + (int64_t)c0 * mp);
        lds_u32* d32 = (lds_u32*)smem_raw + (cres + ((t & 1) ? TC : 0)) * mp * (int)(sizeof(T) / 4);
        for (int e0 = 0; e0 < cntw; e0 += kBThreads) {
            const int e = e0 + tid;
            if (e < cntw) __builtin_amdgcn_global_load_lds((const void*)(s32 + e), d32 + (e - lane), 4, 0, 0);
        }
    };

    // ---- first pass: every column from A_b to its home, exact norms --------
    auto first_norm = [&](int l, double ss) {
        ss = row16_sum(ss);
        const double nu = sqrt(ss);
        if (l16 == 0) sh.snu[l] = nu;
        consider(l, nu, ss);
    };
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        const int l = cgroup + kGroups * c;
        const bool have = l < nreg;
        double ss = 0.0;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int r = l16 + 16 * t;
            const T x = (have && r < m) ? Ab[(int64_t)l * m + r] : T(0);
            rc[c][t] = x;
            ss += (double)x * (double)x;
        }
        if (have) first_norm(l, ss);
    }
    // the other columns CB at a time per group, all their loads in flight
    // before the first is stored
    constexpr int CB = RT >= 16 ? 2 : (RT >= 8 ? 4 : 8);
    for (int l0 = nreg + cgroup; l0 < n; l0 += kGroups * CB) {
        T xv[CB][RT];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int l = l0 + kGroups * cb;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int r = l16 + 16 * t;
                xv[cb][t] = (l < n && t < ntv && r < m) ? Ab[(int64_t)l * m + r] : T(0);
            }
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int l = l0 + kGroups * cb;
            if (l >= n) break;  // uniform over the group
            T* col = home(l);
            double ss = 0.0;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                if (t < ntv) {
                    col[l16 + 16 * t] = xv[cb][t];
                    ss += (double)xv[cb][t] * (double)xv[cb][t];
                }
            }
            first_norm(l, ss);
        }
    }
    if (ns > 0) {
        __syncthreads();  // the scratch holds the streamed columns
        issue(0);         // the first tile of the first step's pass
    }
    publish();

    int k = 0;
    uint32_t status = 0;
    double a_norm = 0.0, resid = 0.0, stop_abs = 0.0;
    for (;;) {
        lds_barrier();
        // ---- the pivot: best of the eight wave entries ----------------------
        ArgMax e[kBWaves];
        double sm[kBWaves];
#pragma unroll
        for (int w = 0; w < kBWaves; ++w) {
            e[w] = sh.w_best[w];
            sm[w] = sh.w_sum[w];
        }
        ArgMax best = e[0];
        double ss = sm[0];
        int bw = 0;
#pragma unroll
        for (int w = 1; w < kBWaves; ++w) {
            if (argmax_better(e[w].v, e[w].i, best.v, best.i)) {
                best = e[w];
                bw = w;
            }
            ss += sm[w];
        }
        const T* pc = sh.w_col + bw * kBMaxM;  // the pivot column
        if (k == 0) {
            a_norm = sqrt(ss);
            stop_abs = eps * a_norm;
            resid = a_norm;
            if (!(a_norm <= 1.0e300)) {
                status |= MIID_NONFINITE;
                break;
            }
        } else {
            resid = sqrt(ss);
        }
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
        const int jt = j >> 4, jl = j & 15;
        // ---- the reflector, in every lane ------------------------------------
        const double alpha = best.v;
        const double x0 = (double)pc[j];
        const double beta = x0 >= 0.0 ? -alpha : alpha;
        const double tau = (beta - x0) / beta;
        const double scale = 1.0 / (x0 - beta);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            T v = (T)((double)pc[l16 + 16 * t] * scale);
            if (t < jt) v = T(0);
            if (t == jt) v = l16 < jl ? T(0) : (l16 == jl ? T(1) : v);
            sv[t] = v;
        }
        if (tid == 0) {
            sh.s_sel[j] = p;
            sh.snu[p] = -1.0;
            Zb[j + (int64_t)p * kb] = (T)beta;
        }
        lds_barrier();  // the staged entries are read before the pass restages them

        // ---- the pass: H = I - tau v v^T on every alive column -------------
        gb = {-1.0, INT32_MAX};
        acc = 0.0;
        // s2 over rows > j and the store of row j, from slice t of y
        auto tail = [&](int t, T y, double& s2, int l, bool alive) {
            if (t > jt) s2 += (double)y * (double)y;
            if (t == jt) {
                if (l16 > jl) s2 += (double)y * (double)y;
                if (l16 == jl && alive) Zb[j + (int64_t)l * kb] = y;
            }
        };
        auto track = [&](int l, double s2) {
            s2 = row16_sum(s2);
            const double nu = sqrt(s2);
            if (l16 == 0) sh.snu[l] = nu;
            consider(l, nu, nu * nu);
        };
        // register columns, branch-free (a chosen or missing column gets
        // tau = 0, which leaves it unchanged)
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            if (kGroups * c >= nreg) break;  // uniform: no group has column c
            const int l = cgroup + kGroups * c;
            const bool alive = l < nreg && sh.snu[l < nreg ? l : 0] >= 0.0;
            double d = 0.0;
#pragma unroll
            for (int t = 0; t < RT; ++t) d += (double)rc[c][t] * (double)sv[t];
            d = row16_sum(d);
            // the update itself in the working precision (the dot product
            // above and the norm below accumulate in FP64)
            const T tc = alive ? (T)(tau * d) : T(0);
            double s2 = 0.0;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const T y = fma_w(-tc, sv[t], rc[c][t]);
                rc[c][t] = y;
                tail(t, y, s2, l, alive);
            }
            if (alive) track(l, s2);
        }
        // a column read from src (LDS) and written to dst (the same LDS
        // column, or its scratch home for a streamed tile)
        auto col_step = [&](int l, const T* src, T* dst) {
            if (!(sh.snu[l] >= 0.0)) return;  // chosen column (uniform over the group)
            T x[RT];
            double d = 0.0;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                x[t] = t < ntv ? src[l16 + 16 * t] : T(0);
                d += (double)x[t] * (double)sv[t];
            }
            const T dw = (T)(tau * row16_sum(d));
            double s2 = 0.0;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                x[t] = fma_w(-dw, sv[t], x[t]);
                if (t < ntv) dst[l16 + 16 * t] = x[t];
                tail(t, x[t], s2, l, true);
            }
            track(l, s2);
        };
        for (int l = nreg + cgroup; l < c_str; l += kGroups) {
            T* col = lds + (l - nreg) * mp;
            col_step(l, col, col);
        }
        if (ns > 0) {
            // streamed columns: tile t + 1 in flight while tile t is updated
            // and stored straight back to the scratch
            __syncthreads();  // tile 0 has landed
            for (int t = 0; t < nt; ++t) {
                if (t + 1 < nt) issue(t + 1);
                const int c0 = c_str + t * TC, c1 = min(n, c0 + TC);
                const T* cur = (t & 1) ? buf1 : buf0;
                for (int l = c0 + cgroup; l < c1; l += kGroups) col_step(l, cur + (l - c0) * mp, Wb + (int64_t)l * mp);
                __syncthreads();  // the next tile has landed, this one is stored and no longer read
            }
            issue(0);  // the first tile of the next step's pass
        }
        ++k;
        publish();
    }
    if (ns > 0) __syncthreads();  // no tile copy left in flight
    return BResult{k, status, a_norm, resid};
}

// Persistent kernel: one block at a time per workgroup (8 waves, one per CU).
template <typename T>
__global__ void __launch_bounds__(kBThreads) k_batched(const T* __restrict__ A, const int64_t* __restrict__ a_off,
                                                       const int32_t* __restrict__ mv, const int32_t* __restrict__ nv,
                                                       int32_t nblk, double eps, int32_t kmax,
                                                       int32_t* __restrict__ J, const int64_t* __restrict__ j_off,
                                                       T* __restrict__ Z, const int64_t* __restrict__ z_off,
                                                       miid_info* __restrict__ info,
                                                       const int32_t* __restrict__ order, int32_t* __restrict__ queue,
                                                       T* __restrict__ Wscr, int tile_bytes) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double snu[kBMaxN];
    __shared__ ArgMax w_best[kBWaves];
    __shared__ double w_sum[kBWaves];
    __shared__ T w_col[kBWaves * kBMaxM];
    __shared__ int32_t s_sel[kBMaxK];
    __shared__ int32_t s_blk;
    const int tid = threadIdx.x;
    T* Wb = Wscr + (int64_t)blockIdx.x * kBMaxM * kBMaxN;  // W when it does not fit on chip
    const BShared<T> sh{snu, w_best, w_sum, w_col, s_sel};

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
        BResult res;
        if (m <= 32)
            res = factor_block<T, 2>(Ab, Zb, Wb, m, n, kb, eps, tile_bytes, smem_raw, sh);
        else if (m <= 64)
            res = factor_block<T, 4>(Ab, Zb, Wb, m, n, kb, eps, tile_bytes, smem_raw, sh);
        else if (m <= 128)
            res = factor_block<T, 8>(Ab, Zb, Wb, m, n, kb, eps, tile_bytes, smem_raw, sh);
        else
            res = factor_block<T, 16>(Ab, Zb, Wb, m, n, kb, eps, tile_bytes, smem_raw, sh);
        const int k = res.k;

        // triangular solve: Z[:, l] = R11^{-1} R[:, l] in FP64, Z[:, J[i]] = e_i.
        // The strict upper triangle of R11 goes to sR (zeros elsewhere, up to
        // k rounded to 4), the reciprocals of its diagonal to sDi: the updates
        // below then need no bounds tests and no divisions.
        constexpr int kSR = kBMaxK + 1;
        double* sR = reinterpret_cast<double*>(smem_raw);  // reuses the dynamic LDS
        double* sDi = sR + kBMaxK * kSR;  // reciprocals of the diagonal
        const int kq4 = (k + 3) & ~3;
        __syncthreads();
        for (int e = tid; e < kq4 * kq4; e += kBThreads) {
            const int a = e % kq4, c = e / kq4;
            sR[a * kSR + c] = (a < c && c < k) ? (double)Zb[a + (int64_t)s_sel[c] * kb] : 0.0;
        }
        for (int t = tid; t < k; t += kBThreads) sDi[t] = 1.0 / (double)Zb[t + (int64_t)s_sel[t] * kb];
        __syncthreads();
        int32_t* Jb = J + j_off[b];
        for (int i = tid; i < kb; i += kBThreads) Jb[i] = i < k ? s_sel[i] : -1;
        // four lanes per column (a quad), lane c of the quad holds z_q for
        // q = 4 i + c: back substitution with the solved z_t broadcast from
        // its owner inside the quad (DPP quad permutes)
        int cq = tid % 4;
        asm volatile("" : "+v"(cq));  // as in factor_block: no hoisting out of the block loop
        for (int l0 = tid / 4; l0 < n; l0 += kBThreads / 4) {
            const int l = l0;
            const int c = cq;
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
                if (4 * i >= k) continue;  // uniform
#pragma unroll
                for (int r = 3; r >= 0; --r) {
                    const int t = 4 * i + r;
                    if (t >= k) continue;  // uniform
                    double zt = z[i] * sDi[t];
                    zt = r == 0 ? dpp_f64<0x00>(zt) : (r == 1 ? dpp_f64<0x55>(zt) : (r == 2 ? dpp_f64<0xAA>(zt) : dpp_f64<0xFF>(zt)));
                    if (c == r) z[i] = zt;
                    // rows q < t take R[q, t] z_t; sR is zero on and below
                    // the diagonal, so the other rows are left as they are
#pragma unroll
                    for (int i2 = 0; i2 <= i; ++i2) z[i2] -= sR[(4 * i2 + c) * kSR + t] * zt;
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
        if (tid == 0) info[b] = miid_info{k, res.status, res.a_norm, res.resid, 0, k};
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
    hipLaunchKernelGGL(k_lpt_order, dim3(1), dim3(1024), 0, s, m, n, nblk, order, queue);
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
