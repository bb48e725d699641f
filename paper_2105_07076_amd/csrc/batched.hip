// batched.hip -- many independent small IDs in one persistent launch.
//
// Paper: Advani & O'Hagan, Section 2.1 (column-pivoted QR selects C, Z from
// the triangular solves), Section 4.1 (stop the QR once enough columns are
// chosen), Definition 1 (Z[:, J] = I).  Here each block stops at the smallest
// k whose residual ||R22||_F <= eps ||A_b||_F.
//
// Design.  One 512-lane workgroup factors one block at a time and takes the
// next block from an atomic queue over the blocks sorted by decreasing m n
// (longest first).  Unlike a GEMV-style layout (many lanes per column and a
// cross-lane sum for every dot product), a column here belongs to a group of
// L lanes (L = 1, 2, 4 or 8, the largest that fits n L <= 512), so each
// lane's share of the Householder step -- the dot product v^T x, the update
// x - tau (v^T x) v and the new residual norm -- is a serial loop over the
// rows it holds, and the only cross-lane work per column is an L-lane DPP
// sum.  Rows are dealt to the L lanes in chunks of four (lane q holds rows
// 4 (q + L t) + i), so every lane of the group touches the same number of
// rows at every step.  Columns are dealt round-robin over the eight waves so
// the four SIMDs get equal work.
//
// Storage: a lane's rows ("virtual rows", the column's rows chunk by chunk;
// for n > 512 a lane holds two columns, one after the other) live in
// registers first, then in an LDS slab indexed [row][lane] (conflict-free),
// and only what fits in neither in a per-workgroup global scratch with the
// same layout.  In FP32 every block with n <= 512 stays on chip.
//
// A step: each wave reduces the residual norms of its columns to the best
// (value, column) and the sum of squares and writes them to LDS; barrier;
// every lane folds the eight entries (the same result everywhere), applies
// the stopping tests, and the pivot column's lanes copy its rows into an LDS
// stage; barrier; every lane forms the reflector from the staged column and
// applies H = I - tau v v^T to its columns: the dot products and the squared
// norms as four-row sums in the working precision accumulated in FP64, the
// update in the working precision; row j of R goes to the block's Z storage
// and leaves the register file.  R stays in place (no column swaps); the
// solve then reads R11 into LDS in FP64 and overwrites Z.
//
// Blocks outside the size limits never enter the queue (the ordering kernel
// writes their info); a block holding a NaN or an infinity stops before its
// first step with k = 0.  Every branch that contains a barrier depends only
// on values that are the same in every thread of the workgroup, and the step
// loop is bounded by kmax.
#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "handle.hpp"
#include "cpqr.hpp"
#include "prof.hpp"

namespace miid {

constexpr int kBThreads = 512;
constexpr int kBWaves = kBThreads / kWave;
constexpr int kBMaxM = 256;
constexpr int kBMaxN = 1024;
constexpr int kBMaxK = 64;
constexpr int kBLdsBytes = 160 * 1024;  // the whole LDS of a CU, carved by hand
// the staged pivot column: L x VS entries (at most 264 for an admissible block)
constexpr int kBSlot = 264;
// the end of LDS: staged columns (working precision), the waves' entries of
// both step parities, the selected columns, the queue slot; the rest holds
// block rows
template <typename T>
struct BLds {
    static constexpr int kOffStW = 0;
    static constexpr int kOffPBest = kOffStW + kBSlot * (int)sizeof(T);
    static constexpr int kOffPSum = kOffPBest + 2 * kBWaves * 8;
    static constexpr int kOffPIdx = kOffPSum + 2 * kBWaves * 8;
    static constexpr int kOffSel = kOffPIdx + 2 * kBWaves * 4;
    static constexpr int kOffBlk = kOffSel + kBMaxK * 4;
    static constexpr int kMiscBytes = (kOffBlk + 4 + 255) / 256 * 256;
    static constexpr int kMiscOff = kBLdsBytes - kMiscBytes;
};
constexpr int kSolveLd = kBMaxK + 2;  // column stride of R11 in the solve (even: 16-byte aligned columns)
static_assert(kBMaxK * kSolveLd * 8 + kBMaxK * 8 <= BLds<float>::kMiscOff, "solve arrays");

// Block rows a lane keeps in registers (multiples of 4): at most kRegRows
// with one column per lane, kRegRowsC2 with two (what the 256 VGPRs of a lane
// at two waves per SIMD leave beside the step's own values); then LDS rows.
template <typename T>
struct BCfg;
template <>
struct BCfg<float> {
    static constexpr int kRegRows = 168;
    static constexpr int kRegRowsC2 = 64;
};
template <>
struct BCfg<double> {
    static constexpr int kRegRows = 80;
    static constexpr int kRegRowsC2 = 48;
};
template <typename T>
constexpr int b_lds_rows() {
    return (BLds<T>::kMiscOff / (kBThreads * (int)sizeof(T))) & ~3;
}
// virtual rows of a lane at most: one column of 256 rows, or two
constexpr int kBMaxVRows = kBMaxM;
constexpr int kBMaxVRowsC2 = 2 * kBMaxM;
template <typename T>
constexpr int b_glob_rows() {
    const int r1 = kBMaxVRows - BCfg<T>::kRegRows - b_lds_rows<T>();
    const int r2 = kBMaxVRowsC2 - BCfg<T>::kRegRowsC2 - b_lds_rows<T>();
    const int r = r1 > r2 ? r1 : r2;
    return r > 0 ? r : 0;
}

// Order the admissible blocks by decreasing size for the queue (longest
// first): a counting sort of one workgroup on the coarse key m n / 256 (1024
// buckets cover every admissible block; the order inside a bucket is
// whatever the LDS atomics give -- it only affects which workgroup takes a
// block, not its result).  A block outside the limits, or one that needs more
// scratch rows per lane than the rg each workgroup has, gets its info here
// (k_out = 0, MIID_BLOCK_UNSUPPORTED) and is left out of the order; queue[1]
// receives the number of admissible blocks, queue[0] the queue head (0).
constexpr int kLptBuckets = 1024;

__device__ __forceinline__ bool block_ok(int m, int n) {
    return m >= 1 && n >= 1 && m <= kBMaxM && n <= kBMaxN && m <= n;
}

// How an admissible m x n block is spread over the workgroup: two columns
// per lane when n > 512, else L lanes per column (as many as n L <= 512 and
// the cap lmax allow); nq4 chunks of four rows per lane and column, nvc
// chunks per lane in all.
struct BShape {
    bool c2;
    int L, nq4, nvc;
};
__device__ __forceinline__ BShape b_shape(int m, int n, int lmax) {
    BShape s;
    s.c2 = n > kBThreads;
    s.L = 1;
    if (!s.c2) {
        while (s.L < 8 && s.L < lmax && n * (2 * s.L) <= kBThreads) s.L *= 2;
    }
    s.nq4 = ((m + 3) / 4 + s.L - 1) / s.L;
    s.nvc = (s.c2 ? 2 : 1) * s.nq4;
    return s;
}

// Rows per lane of such a block that fit neither the registers nor the LDS
// and go to the workgroup's scratch rows (at most b_glob_rows<T>()).
template <typename T>
__device__ __forceinline__ int b_block_glob_rows(int m, int n, int lmax) {
    const BShape s = b_shape(m, n, lmax);
    const int ncr = (s.c2 ? BCfg<T>::kRegRowsC2 : BCfg<T>::kRegRows) / 4;
    const int chunks = s.nvc - ncr - b_lds_rows<T>() / 4;
    return chunks > 0 ? 4 * chunks : 0;
}

template <typename T>
__global__ void __launch_bounds__(1024) k_lpt_order(const int32_t* __restrict__ m, const int32_t* __restrict__ n,
                                                    int32_t nblk, int lmax, int rg, int32_t* __restrict__ order,
                                                    int32_t* __restrict__ queue, miid_info* __restrict__ info) {
    __shared__ int32_t cnt[kLptBuckets];
    __shared__ int32_t scan[kLptBuckets];
    const int tid = threadIdx.x;
    auto admissible = [&](int i) {
        const int mi = m[i], ni = n[i];
        return block_ok(mi, ni) && b_block_glob_rows<T>(mi, ni, lmax) <= rg;
    };
    auto bucket = [&](int i) {
        const int64_t sz = (int64_t)m[i] * (int64_t)n[i];
        return kLptBuckets - 1 - (int)min<int64_t>(sz >> 8, kLptBuckets - 1);  // larger first
    };
    for (int b = tid; b < kLptBuckets; b += blockDim.x) cnt[b] = 0;
    __syncthreads();
    for (int i = tid; i < nblk; i += blockDim.x) {
        if (admissible(i))
            atomicAdd(&cnt[bucket(i)], 1);
        else
            info[i] = miid_info{0, MIID_BLOCK_UNSUPPORTED, 0.0, 0.0, 0, 0};
    }
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
    if (tid == kLptBuckets - 1) {
        queue[0] = 0;
        queue[1] = scan[tid];  // admissible blocks
    }
    __syncthreads();
    for (int i = tid; i < nblk; i += blockDim.x)
        if (admissible(i)) order[atomicAdd(&cnt[bucket(i)], 1)] = i;
}

// a * b + c with one rounding, in the working precision
__device__ __forceinline__ float fma_w(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_w(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Sum over the L lanes of a column group (L = 1, 2, 4, 8; groups aligned to
// L): butterflies, so every lane of the group ends with the same value.
__device__ __forceinline__ double group_sum(double v, int L) {
    if (L >= 2) v += dpp_f64<kDppXor1>(v);
    if (L >= 4) v += dpp_f64<kDppXor2>(v);
    if (L >= 8) v += dpp_f64<kDppHalfMirror>(v);
    return v;
}

// wave-uniform copies of values the compiler cannot prove uniform (LDS
// loads): branches on them become scalar branches
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
    const int64_t b = __builtin_bit_cast(int64_t, v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((int64_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ float readlane_w(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double readlane_w(double v, int l) {
    const int64_t b = __builtin_bit_cast(int64_t, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((int64_t)hi << 32) | (uint32_t)lo);
}

// four-term sums in the working precision, as two pairs (a shorter
// dependence chain than a running sum)
template <typename T>
__device__ __forceinline__ T dot4w(const T (&a)[4], const T (&b)[4]) {
    const T p = fma_w(a[1], b[1], a[0] * b[0]);
    const T r = fma_w(a[3], b[3], a[2] * b[2]);
    return p + r;
}
template <typename T>
__device__ __forceinline__ T sumsq4(const T (&a)[4]) { return dot4w(a, a); }

// one element through a buffer resource (zero when out of range)
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int voff);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0));
}

// four consecutive entries of the pivot column buffers
__device__ __forceinline__ void ld4(const float* p, float (&v)[4]) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
__device__ __forceinline__ void ld4(const double* p, double (&v)[4]) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void st4(float* p, const float (&v)[4]) {
    *reinterpret_cast<float4*>(p) = float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4(double* p, const double (&v)[4]) {
    *reinterpret_cast<double2*>(p) = double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = double2(v[2], v[3]);
}

// Geometry of one block and this lane's place in it (all but the lane fields
// are the same in every thread of the workgroup).
struct BGeo {
    int m, n, kb;
    int L;      // lanes per column
    int P;      // columns per slot (512 / L)
    int nq4;    // chunks of four rows per lane and column
    int nvc;    // virtual chunks of a lane (C nq4)
    int VS;     // stride of the pivot buffers per lane of a group
    int tlmax;  // chunks per lane the pivot buffers hold (v is zero beyond the column)
    // lane
    int tid, lane, wave, q, gi;
    int col0, col1;
    bool valid0, valid1;
};

struct BRes {
    int k;
    uint32_t status;
    double a_norm, resid;
    int step0, step1;  // per lane: the step at which its columns were chosen (-1: not chosen)
};

// Pivoted Householder QR of one block, stopped by the tolerance.  NCR
// register chunks (four rows each) per lane; with NCR at its maximum the
// lane's further chunks live in LDS and then in the global scratch.  C2: two
// columns per lane (n > 512).
//
// Every register chunk is processed at every step, straight-line: the staged
// pivot column is zero above row j (finished rows of R are set to zero in the
// register file once written out) and beyond the column, so the dot products
// and the update leave those rows exactly as they are and the residual norm is
// the plain sum over the lane's rows.  (A chunk range that depends on j would
// make the register array conditional and the compiler would keep two copies
// of it.)
//
// A step: at the end of a pass every wave writes its best column's residual
// norm, index and its sum of squared norms to LDS; after a barrier every lane
// folds the eight entries (the same result everywhere) and the pivot column's
// lanes copy its rows into the stage; after a second barrier every lane reads
// x_j from the stage and forms beta, tau and the scale of the reflector
// itself: v = (x scaled, 1 at row j, 0 above).  The dot products run on the
// staged x and are corrected for v_j = 1.
template <typename T, int NCR, bool C2>
__device__ __forceinline__ BRes factor_block(const BGeo& G, const T* __restrict__ Ab, T* __restrict__ Zb,
                                             T* __restrict__ gsc, unsigned char* smem, double eps) {
    // only the largest classes keep rows in LDS / scratch
    constexpr bool kTiers = C2 || NCR == BCfg<T>::kRegRows / 4;
    constexpr int RLMAX = b_lds_rows<T>();
    using L_ = BLds<T>;
    T* lds_rows = reinterpret_cast<T*>(smem);
    unsigned char* misc = smem + L_::kMiscOff;
    T* st_w = reinterpret_cast<T*>(misc + L_::kOffStW);  // staged columns
    double* p_best = reinterpret_cast<double*>(misc + L_::kOffPBest);
    double* p_sum = reinterpret_cast<double*>(misc + L_::kOffPSum);
    int32_t* p_idx = reinterpret_cast<int32_t*>(misc + L_::kOffPIdx);
    int32_t* s_sel = reinterpret_cast<int32_t*>(misc + L_::kOffSel);

    const int m = G.m, kb = G.kb, L = G.L, P = G.P, nq4 = G.nq4, nvc = kTiers ? G.nvc : NCR;
    // chunks [NCR, vcL1) in LDS, [vcL1, nvc) in the scratch
    const int vcL1 = NCR + min(max(nvc - NCR, 0), RLMAX / 4);
    const int q = G.q, lane = G.lane, wave = G.wave;
    const int tid = G.tid;
    auto lds_at = [&](int vc, int i) -> T* { return lds_rows + (4 * (vc - NCR) + i) * kBThreads + tid; };
    auto glob_at = [&](int vc, int i) -> T* {
        return gsc + (int64_t)(4 * (vc - vcL1) + i) * kBThreads + tid;
    };
    // slot of virtual chunk vc (which of the lane's two columns)
    auto slot_of = [&](int vc) { return (C2 && vc >= nq4) ? 1 : 0; };

    // four rows per vector register tuple (keeps the chunks in contiguous
    // registers; scalar arrays were allocated interleaved with other values)
    typedef T T4 __attribute__((ext_vector_type(4)));
    T4 rc[NCR];

    // ---- first pass: the block into registers / LDS / scratch, exact norms -
    double s2a = 0.0, s2b = 0.0;
    T yn0 = T(0), yn1 = T(0);  // this lane's entry at the next pivot row's place (row 0 now)
    // the block through a bounds-checked buffer resource: loads past the
    // block return zero (columns >= n), rows >= m of a column are zeroed
    // below; one 32-bit offset per load instead of a 64-bit address
    const int nbytes = m * G.n * (int)sizeof(T);
    const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc((void*)Ab, (short)0, nbytes, 0x00020000);
    const int off0 = G.valid0 ? (G.col0 * m + 4 * q) * (int)sizeof(T) : nbytes;
    const int off1 = G.valid1 ? (G.col1 * m + 4 * q) * (int)sizeof(T) : nbytes;
    auto raw_chunk = [&](int vc, T (&x)[4]) {
        const int s = slot_of(vc);
        const int tl = vc - s * nq4;
        const int voff = (s ? off1 : off0) + 4 * L * tl * (int)sizeof(T);
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = buf_load<T>(rsA, voff + i * (int)sizeof(T));
    };
    // rows >= m zeroed, the norm contributions
    auto finish_chunk = [&](int vc, T (&x)[4]) {
        const int s = slot_of(vc);
        const int tl = vc - s * nq4;
        const int rlim = m - 4 * L * tl;  // rows 4 q + i of this chunk exist when 4 q + i < rlim
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = 4 * q + i < rlim ? x[i] : T(0);
        const double ss = (double)sumsq4(x);
        // selects, not branches on s (a branch would make the compiler index a
        // two-element array in memory)
        s2a += s ? 0.0 : ss;
        s2b += s ? ss : 0.0;
        yn0 = (!s && tl == 0) ? x[0] : yn0;
        yn1 = (s && tl == 0) ? x[0] : yn1;
    };
    auto load_chunk = [&](int vc, T (&x)[4]) {
        raw_chunk(vc, x);
        finish_chunk(vc, x);
    };
    // every register chunk's loads go out before any of them is used (the
    // loads of one chunk at a time would each wait for memory)
#pragma unroll
    for (int vc = 0; vc < NCR; ++vc) {
        T x[4];
        raw_chunk(vc, x);
#pragma unroll
        for (int i = 0; i < 4; ++i) rc[vc][i] = x[i];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int vc = 0; vc < NCR; ++vc) {
        T x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = rc[vc][i];
        finish_chunk(vc, x);
#pragma unroll
        for (int i = 0; i < 4; ++i) rc[vc][i] = x[i];
    }
    if constexpr (kTiers) {
        for (int vc = NCR; vc < min(nvc, vcL1); ++vc) {
            T x[4];
            load_chunk(vc, x);
#pragma unroll
            for (int i = 0; i < 4; ++i) *lds_at(vc, i) = x[i];
        }
        for (int vc = vcL1; vc < nvc; ++vc) {
            T x[4];
            load_chunk(vc, x);
#pragma unroll
            for (int i = 0; i < 4; ++i) *glob_at(vc, i) = x[i];
        }
    }
    double nu0 = sqrt(group_sum(s2a, L));
    double nu1 = sqrt(group_sum(s2b, L));
    bool alive0 = G.valid0, alive1 = G.valid1;
    int step0 = -1, step1 = -1;  // the step at which this lane's column was chosen

    // with two columns per lane the stage past a column (read by the passes
    // over the padding chunks) holds zeros for the whole block and staging
    // never writes there; with one, staging writes every chunk
    if constexpr (C2) {
        const int per = 4 * (G.tlmax - nq4);
        for (int e = tid; e < L * per; e += kBThreads) {
            const int qq = e / per, r = e - qq * per;
            st_w[qq * G.VS + 4 * nq4 + r] = T(0);
        }
    }

    // (A): the wave's best alive column and its sum of squared norms into the
    // entries of parity par; the column itself staged into slot `slot`
    auto publish = [&](int par) {
        ArgMax cand{-1.0, INT32_MAX};
        double sum = 0.0;
        if (alive0) {
            cand = ArgMax{nu0, G.col0};
            if (q == 0) sum += nu0 * nu0;
        }
        if (C2 && alive1) {
            if (argmax_better(nu1, G.col1, cand.v, cand.i)) cand = ArgMax{nu1, G.col1};
            if (q == 0) sum += nu1 * nu1;
        }
        cand = wave_argmax_dpp(cand);
        sum = wave_sum_dpp(sum);
        if (lane == 0) {
            p_best[par * kBWaves + wave] = cand.v;
            p_idx[par * kBWaves + wave] = cand.i;
            p_sum[par * kBWaves + wave] = sum;
        }
    };
    // the pivot column's lanes copy all its chunks into the stage (rows above
    // the pivot row are zero in the register file by now)
    auto stage = [&](int p) {
        const int sb = (C2 && p >= P) ? 1 : 0;
        const int lcp = p - sb * P;
        if (wave == (lcp & (kBWaves - 1)) && G.gi == lcp / kBWaves) {
            int qo = q;  // through an empty asm: the addresses below are formed
            asm volatile("" : "+v"(qo));  // here, not kept per chunk
            T* dw = st_w + qo * G.VS;
            const int cs = sb * nq4;
            auto put = [&](int tl, const T (&x)[4]) { st4(dw + 4 * tl, x); };
#pragma unroll
            for (int vc = 0; vc < NCR; ++vc) {
                // one column per lane: every register chunk, the ones past
                // the column being zeros (no per-chunk test); two: the slot's
                // chunks
                if (!C2 || (vc >= cs && vc < cs + nq4)) {
                    T x[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) x[i] = rc[vc][i];
                    put(vc - cs, x);
                }
            }
            if constexpr (kTiers) {
                for (int vc = max(cs, NCR); vc < min(cs + nq4, vcL1); ++vc) {
                    T x[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) x[i] = *lds_at(vc, i);
                    put(vc - cs, x);
                }
                for (int vc = max(cs, vcL1); vc < cs + nq4; ++vc) {
                    T x[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) x[i] = *glob_at(vc, i);
                    put(vc - cs, x);
                }
            }
        }
    };
    publish(0);

    int k = 0;
    uint32_t status = 0;
    double a_norm = 0.0, stop_abs = 0.0, stop2 = 0.0, ss_last = 0.0;
    for (;;) {
        const int par = k & 1;
        lds_barrier();  // the waves' entries are in LDS
        ArgMax best;
        double ss;
        {
            double bv[kBWaves], bs[kBWaves];
            int32_t bi[kBWaves];
#pragma unroll
            for (int w = 0; w < kBWaves; ++w) {
                bv[w] = p_best[par * kBWaves + w];
                bs[w] = p_sum[par * kBWaves + w];
                bi[w] = p_idx[par * kBWaves + w];
            }
            best = ArgMax{bv[0], bi[0]};
            ss = bs[0];
#pragma unroll
            for (int w = 1; w < kBWaves; ++w) {
                if (argmax_better(bv[w], bi[w], best.v, best.i)) best = ArgMax{bv[w], bi[w]};
                ss += bs[w];
            }
            best = ArgMax{uni(best.v), uni(best.i)};
            ss = uni(ss);
        }
        if (k == 0) {
            a_norm = sqrt(ss);
            stop_abs = eps * a_norm;
            stop2 = stop_abs * stop_abs;
        }
        ss_last = ss;
        // one exit (several would give the compiler's structurizer more
        // paths to merge the register array over)
        const uint32_t why = (k == 0 && !(a_norm <= 1.0e300)) ? MIID_NONFINITE
                             : ss <= stop2                   ? 0x100u
                             : k >= kb                        ? MIID_KMAX_HIT
                             : !(best.v > 0.0)                ? MIID_RANK_DEFICIENT
                                                              : 0u;
        if (why != 0u) {
            status |= why & 0xffu;
            break;
        }

        // ---- the reflector, from the staged pivot column ------------------
        const int j = k;
        const int p = best.i;
        const int sp = (C2 && p >= P) ? 1 : 0;
        const int gj = j >> 2;
        const int qj = gj & (L - 1), tj = gj / L, ij = j & 3;
        stage(p);
        if (tid == 0) s_sel[j] = p;
        if (sp ? G.col1 == p : G.col0 == p) {  // this lane's column is the pivot
            if (sp) {
                alive1 = false;
                step1 = j;
            } else {
                alive0 = false;
                step0 = j;
            }
        }
        lds_barrier();  // the pivot column is staged
        const double x0 = (double)st_w[qj * G.VS + 4 * tj + ij];
        const double alpha = best.v;
        const double beta = x0 >= 0.0 ? -alpha : alpha;
        // 1 / (x0 - beta) and 1 / beta: hardware reciprocal and two Newton
        // steps (each doubles the correct bits; the IEEE division sequence is
        // several times longer)
        auto recip = [](double a) {
            double r = __builtin_amdgcn_rcp(a);
            r = __builtin_fma(__builtin_fma(-a, r, 1.0), r, r);
            r = __builtin_fma(__builtin_fma(-a, r, 1.0), r, r);
            return r;
        };
        const double scale = recip(x0 - beta);
        const double tau = (beta - x0) * recip(beta);
        if (tid == 0) Zb[j + (int64_t)p * kb] = (T)beta;

        // ---- H = I - tau v v^T on every column -----------------------------
        const bool own = q == qj;  // this lane holds row j (of each of its columns)
        bool mj[4];  // this lane's element i of the boundary chunk is row j
#pragma unroll
        for (int i = 0; i < 4; ++i) mj[i] = own && i == ij;
        // x^T y over all rows with the staged x (zero above row j); v^T y =
        // scale (x^T y - x_j y_j) + y_j = scale (x^T y - beta y_j).  Each
        // chunk's four products are summed in the working precision (one
        // rounding per term of a four-term sum) and the chunk sums in FP64:
        // the accuracy of a four-term dot product for one conversion per four
        // rows (a conversion costs about two FMAs)
        double da[2] = {0.0, 0.0}, db[2] = {0.0, 0.0};
        // y_j (row j before the update) where this lane holds it: kept from
        // the previous step's update
        const T yja = yn0, yjb = yn1;
        const T* pv_w = st_w;
        auto pw_at = [&](int vc) { return pv_w + q * G.VS + 4 * (vc - slot_of(vc) * nq4); };
        auto dot4v = [&](int vc, const T (&x)[4], const T (&xs)[4]) {
            const int s = slot_of(vc);
            const T c = dot4w(xs, x);
            if constexpr (C2) {
                da[vc & 1] += s ? 0.0 : (double)c;
                db[vc & 1] += s ? (double)c : 0.0;
            } else {
                da[vc & 1] += (double)c;
            }
        };
        auto dot4 = [&](int vc, const T (&x)[4]) {
            T xs[4];
            ld4(pw_at(vc), xs);
            dot4v(vc, x, xs);
        };
        {
            // register chunks, the staged x of the chunk after next loaded
            // while this one is used
            T xs0[4], xs1[4], xs2[4];
            ld4(pw_at(0), xs0);
            if (NCR > 1) ld4(pw_at(1), xs1);
#pragma unroll
            for (int vc = 0; vc < NCR; ++vc) {
                if (vc + 2 < NCR) ld4(pw_at(vc + 2), xs2);
                T x[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) x[i] = rc[vc][i];
                dot4v(vc, x, xs0);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    xs0[i] = xs1[i];
                    xs1[i] = xs2[i];
                }
                // one chunk at a time: the scheduler would otherwise start many
                // chunks' loads and products at once and run out of registers
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if constexpr (kTiers) {
            for (int vc = NCR; vc < min(nvc, vcL1); ++vc) {
                T x[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) x[i] = *lds_at(vc, i);
                dot4(vc, x);
            }
            for (int vc = vcL1; vc < nvc; ++vc) {
                T x[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) x[i] = *glob_at(vc, i);
                dot4(vc, x);
            }
        }
        // lane sums, corrected by the lane holding row j, then the group sum
        const bool hasj = mj[0] | mj[1] | mj[2] | mj[3];
        const double ca = (da[0] + da[1]) - (hasj ? beta * (double)yja : 0.0);
        const double d0 = scale * group_sum(ca, L);
        const T wa = (T)(tau * d0), wva = (T)(tau * d0 * scale);
        T wb = T(0), wvb = T(0);
        if (C2) {
            const double cb = (db[0] + db[1]) - (hasj ? beta * (double)yjb : 0.0);
            const double d1 = scale * group_sum(cb, L);
            wb = (T)(tau * d1);
            wvb = (T)(tau * d1 * scale);
        }
        // the update in the working precision (y - (tau d scale) x, and
        // y_j - tau d for row j, written out and zeroed); the residual norms
        // over what is left, chunk sums of squares in the working precision
        // accumulated in FP64 (relative error of a four-term sum)
        double na[2] = {0.0, 0.0}, nb[2] = {0.0, 0.0};
        const int tj1 = ((j + 1) >> 2) / L, ij1 = (j + 1) & 3;
        T yna = yn0, ynb = yn1;
        auto upd4v = [&](int vc, T (&x)[4], const T (&xw)[4]) {
            const int s = slot_of(vc);
            const int tl = vc - s * nq4;
            const T wv = s ? wvb : wva;
#pragma unroll
            for (int i = 0; i < 4; ++i) x[i] = fma_w(-wv, xw[i], x[i]);
            if (tl == tj) {  // uniform: row j of R leaves the register file
#pragma unroll
                for (int i = 0; i < 4; ++i) x[i] = mj[i] ? T(0) : x[i];
            }
            if (tl == tj1) {  // uniform: keep the entry at row j + 1's place
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    ynb = (s && i == ij1) ? x[i] : ynb;
                    yna = (!s && i == ij1) ? x[i] : yna;
                }
            }
            const T c = sumsq4(x);
            if constexpr (C2) {
                na[vc & 1] += s ? 0.0 : (double)c;
                nb[vc & 1] += s ? (double)c : 0.0;
            } else {
                na[vc & 1] += (double)c;
            }
        };
        auto upd4 = [&](int vc, T (&x)[4]) {
            T xw[4];
            ld4(pw_at(vc), xw);
            upd4v(vc, x, xw);
        };
        {
            T xs0[4], xs1[4], xs2[4];
            ld4(pw_at(0), xs0);
            if (NCR > 1) ld4(pw_at(1), xs1);
#pragma unroll
            for (int vc = 0; vc < NCR; ++vc) {
                if (vc + 2 < NCR) ld4(pw_at(vc + 2), xs2);
                T x[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) x[i] = rc[vc][i];
                upd4v(vc, x, xs0);
#pragma unroll
                for (int i = 0; i < 4; ++i) rc[vc][i] = x[i];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    xs0[i] = xs1[i];
                    xs1[i] = xs2[i];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if constexpr (kTiers) {
            for (int vc = NCR; vc < min(nvc, vcL1); ++vc) {
                T x[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) x[i] = *lds_at(vc, i);
                upd4(vc, x);
#pragma unroll
                for (int i = 0; i < 4; ++i) *lds_at(vc, i) = x[i];
            }
            for (int vc = vcL1; vc < nvc; ++vc) {
                T x[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) x[i] = *glob_at(vc, i);
                upd4(vc, x);
#pragma unroll
                for (int i = 0; i < 4; ++i) *glob_at(vc, i) = x[i];
            }
        }
        if (own && alive0) Zb[j + (int64_t)G.col0 * kb] = yja - wa;
        if (C2 && own && alive1) Zb[j + (int64_t)G.col1 * kb] = yjb - wb;
        yn0 = yna;
        yn1 = ynb;
        nu0 = sqrt(group_sum(na[0] + na[1], L));
        if (C2) nu1 = sqrt(group_sum(nb[0] + nb[1], L));
        ++k;
        publish(k & 1);
    }
    return BRes{k, status, a_norm, sqrt(ss_last), step0, step1};
}

// Register chunks for a block of nvc chunks per lane: the smallest class
// that holds them (the largest keeps the rest in LDS / scratch).
template <typename T>
__device__ __forceinline__ int reg_class(int nvc);
template <>
__device__ __forceinline__ int reg_class<float>(int nvc) {
    return nvc <= 2 ? 2 : nvc <= 4 ? 4 : nvc <= 6 ? 6 : nvc <= 8 ? 8 : nvc <= 10 ? 10 : nvc <= 12 ? 12
           : nvc <= 14 ? 14 : nvc <= 16 ? 16 : nvc <= 20 ? 20 : nvc <= 24 ? 24 : nvc <= 28 ? 28
           : nvc <= 32 ? 32 : nvc <= 36 ? 36 : BCfg<float>::kRegRows / 4;
}
template <>
__device__ __forceinline__ int reg_class<double>(int nvc) {
    return nvc <= 2 ? 2 : nvc <= 4 ? 4 : nvc <= 8 ? 8 : nvc <= 12 ? 12 : BCfg<double>::kRegRows / 4;
}

// Persistent kernel: one block at a time per workgroup (one workgroup per CU).
template <typename T>
__global__ void __launch_bounds__(kBThreads) k_batched(const T* __restrict__ A, const int64_t* __restrict__ a_off,
                                                       const int32_t* __restrict__ mv, const int32_t* __restrict__ nv,
                                                       double eps, int32_t kmax, int lmax,
                                                       int32_t* __restrict__ J, const int64_t* __restrict__ j_off,
                                                       T* __restrict__ Z, const int64_t* __restrict__ z_off,
                                                       miid_info* __restrict__ info,
                                                       const int32_t* __restrict__ order, int32_t* __restrict__ queue,
                                                       T* __restrict__ Wscr, int rg) {
    constexpr int NCRMAX = BCfg<T>::kRegRows / 4;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char* misc = smem + BLds<T>::kMiscOff;
    int32_t* s_sel = reinterpret_cast<int32_t*>(misc + BLds<T>::kOffSel);
    int32_t* s_blk = reinterpret_cast<int32_t*>(misc + BLds<T>::kOffBlk);

    BGeo G;
    G.tid = threadIdx.x;
    G.lane = G.tid & (kWave - 1);
    G.wave = __builtin_amdgcn_readfirstlane(G.tid >> 6);
    const int tid = G.tid;
    T* gsc = Wscr + (int64_t)blockIdx.x * rg * kBThreads;  // this workgroup's rg scratch rows per lane
    const int nvalid = uni(queue[1]);

    for (;;) {
        if (tid == 0) *s_blk = atomicAdd(&queue[0], 1);
        __syncthreads();
        const int32_t qi = uni(*s_blk);
        __syncthreads();
        if (qi >= nvalid) break;  // the same in every thread
        const int32_t b = uni(order[qi]);
        const int m = uni(mv[b]), n = uni(nv[b]);
        const int kb = min(min(m, n), kmax);
        T* __restrict__ Zb = Z + z_off[b];

        // ---- geometry (uniform) ----------------------------------------
        const BShape sh = b_shape(m, n, lmax);
        const bool c2 = sh.c2;  // two columns per lane
        const int L = sh.L;
        G.m = m;
        G.n = n;
        G.kb = kb;
        G.L = L;
        G.P = kBThreads / L;
        G.nq4 = sh.nq4;
        G.nvc = sh.nvc;
        G.q = G.lane & (L - 1);
        G.gi = G.lane / L;
        const int lc = G.gi * kBWaves + G.wave;
        G.col0 = lc;
        G.col1 = G.P + lc;
        G.valid0 = lc < n;
        G.valid1 = c2 && G.col1 < n;

        BRes res;
        const T* __restrict__ Ab = A + a_off[b];
        constexpr int NCRC2 = BCfg<T>::kRegRowsC2 / 4;
        const int cls = c2 ? NCRC2 : reg_class<T>(G.nvc);
        // the pivot buffers cover every chunk a pass touches (local chunk
        // index within the chunk's column)
        G.tlmax = c2 ? max(G.nq4, cls - G.nq4) : max(G.nvc, cls);
        G.VS = 4 * G.tlmax + 4;
        if (c2) {
            res = factor_block<T, NCRC2, true>(G, Ab, Zb, gsc, smem, eps);
        } else if (cls == NCRMAX) {
            res = factor_block<T, NCRMAX, false>(G, Ab, Zb, gsc, smem, eps);
        } else if constexpr (sizeof(T) == 4) {
            switch (cls) {
                case 2: res = factor_block<T, 2, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 4: res = factor_block<T, 4, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 6: res = factor_block<T, 6, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 8: res = factor_block<T, 8, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 10: res = factor_block<T, 10, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 12: res = factor_block<T, 12, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 14: res = factor_block<T, 14, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 16: res = factor_block<T, 16, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 20: res = factor_block<T, 20, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 24: res = factor_block<T, 24, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 28: res = factor_block<T, 28, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 32: res = factor_block<T, 32, false>(G, Ab, Zb, gsc, smem, eps); break;
                default: res = factor_block<T, 36, false>(G, Ab, Zb, gsc, smem, eps); break;
            }
        } else {
            switch (cls) {
                case 2: res = factor_block<T, 2, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 4: res = factor_block<T, 4, false>(G, Ab, Zb, gsc, smem, eps); break;
                case 8: res = factor_block<T, 8, false>(G, Ab, Zb, gsc, smem, eps); break;
                default: res = factor_block<T, 12, false>(G, Ab, Zb, gsc, smem, eps); break;
            }
        }
        const int k = res.k;

        // ---- triangular solve: Z[:, l] = R11^{-1} R[:, l] in FP64, Z[:, J[i]] = e_i
        // the R rows written to Z above are visible to the whole workgroup
        // after a workgroup barrier (its waves share one CU's vector cache; a
        // device-scope fence would write back the whole L2 instead)
        __syncthreads();
        double* sR = reinterpret_cast<double*>(smem);  // column-major, reuses the row slab
        double* sDi = sR + kBMaxK * kSolveLd;            // reciprocals of the diagonal
        // the strict upper triangle of R11 (only its entries are read)
        for (int e = tid; e < k * k; e += kBThreads) {
            const int a = e % k, c = e / k;
            if (a < c) sR[c * kSolveLd + a] = (double)Zb[a + (int64_t)s_sel[c] * kb];
        }
        for (int t = tid; t < k; t += kBThreads) sDi[t] = 1.0 / (double)Zb[t + (int64_t)s_sel[t] * kb];
        int32_t* Jb = J + j_off[b];
        for (int i = tid; i < kb; i += kBThreads) Jb[i] = i < k ? s_sel[i] : -1;
        __syncthreads();
        // one lane per column (the first lane of the column's group): back
        // substitution with z in registers, R11's columns read from LDS by every
        // lane at the same address; a chosen column gets its unit vector
        const __amdgpu_buffer_rsrc_t rsZ =
            __builtin_amdgcn_make_buffer_rsrc((void*)Zb, (short)0, kb * n * (int)sizeof(T), 0x00020000);
        auto solve_col = [&](int c, int step) {
            T* zc = Zb + (int64_t)c * kb;
            if (step >= 0) {
                for (int i = 0; i < kb; ++i) zc[i] = i == step ? T(1) : T(0);
                return;
            }
            // eight loads at a time through the block's bounds-checked resource
            // (one guard per eight: a guard per load would make each wait for
            // memory); entries past k are zeroed
            double z[kBMaxK];
            const int zoff = c * kb * (int)sizeof(T);
#pragma unroll
            for (int g = 0; g < kBMaxK / 8; ++g) {
                if (8 * g < k) {  // uniform
#pragma unroll
                    for (int i = 8 * g; i < 8 * g + 8; ++i) {
                        const T v = buf_load<T>(rsZ, zoff + i * (int)sizeof(T));
                        z[i] = i < k ? (double)v : 0.0;
                    }
                } else {
#pragma unroll
                    for (int i = 8 * g; i < 8 * g + 8; ++i) z[i] = 0.0;
                }
            }
#pragma unroll
            for (int t = kBMaxK - 1; t >= 0; --t) {
                if (t < k) {  // uniform
                    const double zt = z[t] * sDi[t];
                    z[t] = zt;
                    const double* rcol = sR + t * kSolveLd;
#pragma unroll
                    for (int i = 0; i < t; ++i) z[i] = __builtin_fma(-rcol[i], zt, z[i]);
                }
            }
#pragma unroll
            for (int i = 0; i < kBMaxK; ++i)
                if (i < kb) zc[i] = i < k ? (T)z[i] : T(0);
        };
        if (G.q == 0) {
            if (G.valid0) solve_col(G.col0, res.step0);
            if (G.valid1) solve_col(G.col1, res.step1);
        }
        if (tid == 0) info[b] = miid_info{k, res.status, res.a_norm, res.resid, 0, k};
        __syncthreads();  // LDS is reused by the next block
    }
}

}  // namespace miid

using namespace miid;

// Scratch of the allocation-free entry point, one copy per GPU (each GPU the
// library runs on holds it until the process ends): the queue order of at
// most kNaMaxBlocks blocks, the queue head and count, then the scratch rows
// of the workgroups.  Host code uses the address hipGetSymbolAddress gives
// for the current device, never the array's name.
constexpr size_t kNaBytes = size_t(64) << 20;
constexpr int kNaMaxBlocks = 1 << 18;
constexpr size_t kNaOffQueue = size_t(kNaMaxBlocks) * 4;
constexpr size_t kNaOffRows = kNaOffQueue + 256;
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {
struct BPlan {
    int grid;
    size_t oOrder, oQueue, oW, total;
};

// One workgroup per CU (the whole LDS); global rows only for what fits
// neither registers nor LDS.
BPlan batched_plan(int32_t nblk, size_t esz) {
    BPlan P;
    P.grid = std::max(1, std::min(nblk, dev_info().cus));
    const int grows = esz == 8 ? b_glob_rows<double>() : b_glob_rows<float>();
    size_t off = 0;
    P.oOrder = off;
    off = align_up(off + (size_t)std::max(nblk, 1) * 4, 256);
    P.oQueue = off;
    off = align_up(off + 8, 256);
    P.oW = off;
    off = align_up(off + (size_t)P.grid * grows * kBThreads * esz, 256);
    P.total = off;
    return P;
}

// The checks shared by id_batched and id_batched_noalloc (argument numbers
// counted from nblk); returns 0 or the code.
int batched_args(int32_t nblk, const void* A, const int64_t* a_off, const int32_t* m, const int32_t* n,
                 miid_dtype dtype, const miid_opts* opts, int32_t* J, const int64_t* j_off, void* Z,
                 const int64_t* z_off, miid_info* info) {
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
    return 0;
}

int lanes_cap(const miid_opts* opts) {
    const int h = (int)((opts->flags >> MIID_HINT_LPC_SHIFT) & 15u);
    return (h == 1 || h == 2 || h == 4 || h == 8) ? h : 8;
}

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current) and kept.
constexpr int kNaDevices = 64;
std::mutex g_na_mu;
void* g_na_ptr[kNaDevices] = {};

int na_scratch(void** out) {
    int dev = -1;
    MIID_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaDevices) return MIID_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        MIID_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_na_ptr[dev] = p;
    }
    *out = g_na_ptr[dev];
    return 0;
}

// Scratch rows per lane each of `grid` workgroups gets from the static
// scratch (a multiple of 4, at most what any admissible block needs).
template <typename T>
int na_rows(int grid) {
    const size_t per = (size_t)grid * kBThreads * sizeof(T);
    const size_t r = ((kNaBytes - kNaOffRows) / per) & ~size_t(3);
    return (int)std::min<size_t>(r, (size_t)b_glob_rows<T>());
}

// The ordering kernel, then the persistent kernel on `grid` workgroups with
// rg scratch rows per lane each at Wscr (order, queue and Wscr: device
// memory of the caller's workspace or of the static scratch).
template <typename T>
int enqueue_batched(int32_t nblk, const T* A, const int64_t* a_off, const int32_t* m, const int32_t* n,
                    const miid_opts* opts, int32_t* J, const int64_t* j_off, T* Z, const int64_t* z_off,
                    miid_info* info, int32_t* order, int32_t* queue, T* Wscr, int grid, int rg, hipStream_t s) {
    const int lmax = lanes_cap(opts);
    hipLaunchKernelGGL(k_lpt_order<T>, dim3(1), dim3(1024), 0, s, m, n, nblk, lmax, rg, order, queue, info);
    MIID_HIP(hipGetLastError());
    MIID_HIP(lds_limit_once((const void*)k_batched<T>, kBLdsBytes));
    const int pr = prof_take(MIID_K_BATCHED, 0, nblk, 0);
    MIID_LAUNCH(pr, k_batched<T>, dim3(grid), dim3(kBThreads), (size_t)kBLdsBytes, s, A, a_off, m, n, opts->eps,
                opts->kmax, lmax, J, j_off, Z, z_off, info, order, queue, Wscr, rg);
    MIID_HIP(hipGetLastError());
    return 0;
}
}  // namespace

namespace miid {
int batched_noalloc_setup() {
    void* p = nullptr;
    return na_scratch(&p);
}
}  // namespace miid

extern "C" {

static size_t batched_workspace_body(int32_t nblk, miid_dtype dtype) {
    if (nblk < 1 || (dtype != MIID_F32 && dtype != MIID_F64)) return 0;
    return batched_plan(nblk, dtype == MIID_F64 ? 8 : 4).total;
}

static int batched_body(int32_t nblk, const void* A, const int64_t* a_off, const int32_t* m, const int32_t* n,
                        miid_dtype dtype, const miid_opts* opts, int32_t* J, const int64_t* j_off, void* Z,
                        const int64_t* z_off, miid_info* info, void* ws, size_t ws_bytes, void* stream) {
    if (const int rc = batched_args(nblk, A, a_off, m, n, dtype, opts, J, j_off, Z, z_off, info)) return rc;
    if (!ws) return -13;
    const size_t esz = dtype == MIID_F64 ? 8 : 4;
    const BPlan P = batched_plan(nblk, esz);
    if (ws_bytes < P.total) return MIID_E_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    int32_t* order = reinterpret_cast<int32_t*>(w + P.oOrder);
    int32_t* queue = reinterpret_cast<int32_t*>(w + P.oQueue);
    if (dtype == MIID_F64)
        return enqueue_batched<double>(nblk, (const double*)A, a_off, m, n, opts, J, j_off, (double*)Z, z_off, info,
                                       order, queue, reinterpret_cast<double*>(w + P.oW), P.grid,
                                       b_glob_rows<double>(), s);
    return enqueue_batched<float>(nblk, (const float*)A, a_off, m, n, opts, J, j_off, (float*)Z, z_off, info, order,
                                  queue, reinterpret_cast<float*>(w + P.oW), P.grid, b_glob_rows<float>(), s);
}

// ---- entry points: the handle resolved, then the bodies above -----------
size_t miid_batched_workspace(miid_handle h, int32_t nblk, miid_dtype dtype) {
    if (check_handle(h) != 0) return 0;
    return batched_workspace_body(nblk, dtype);
}

int id_batched(miid_handle h, int32_t nblk, const void* A, const int64_t* a_off, const int32_t* m, const int32_t* n,
               miid_dtype dtype, const miid_opts* opts, int32_t* J, const int64_t* j_off, void* Z,
               const int64_t* z_off, miid_info* info, void* ws, size_t ws_bytes, void* stream) {
    miid_opts o;
    if (resolve_opts(h, kTuneBatched, dtype, nblk, 0, opts ? opts->kmax : 0, opts, &o) != 0) return -1;
    return shift_arg(batched_body(nblk, A, a_off, m, n, dtype, opts ? &o : nullptr, J, j_off, Z, z_off, info, ws,
                                  ws_bytes, stream));
}

int id_batched_noalloc(miid_handle h, int32_t nblk, const void* A, const int64_t* a_off, const int32_t* m,
                       const int32_t* n, miid_dtype dtype, const miid_opts* opts, int32_t* J, const int64_t* j_off,
                       void* Z, const int64_t* z_off, miid_info* info, void* stream) {
    miid_opts o;
    if (resolve_opts(h, kTuneBatched, dtype, nblk, 0, opts ? opts->kmax : 0, opts, &o) != 0) return -1;
    const miid_opts* op = opts ? &o : nullptr;
    if (const int rc = batched_args(nblk, A, a_off, m, n, dtype, op, J, j_off, Z, z_off, info)) return shift_arg(rc);
    if (nblk > kNaMaxBlocks) return MIID_E_UNSUPPORTED;
    void* base = nullptr;
    if (const int rc = na_scratch(&base)) return rc;
    unsigned char* w = reinterpret_cast<unsigned char*>(base);
    int32_t* order = reinterpret_cast<int32_t*>(w);
    int32_t* queue = reinterpret_cast<int32_t*>(w + kNaOffQueue);
    const int grid = std::max(1, std::min(nblk, dev_info().cus));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (dtype == MIID_F64)
        return enqueue_batched<double>(nblk, (const double*)A, a_off, m, n, op, J, j_off, (double*)Z, z_off, info,
                                       order, queue, reinterpret_cast<double*>(w + kNaOffRows), grid,
                                       na_rows<double>(grid), s);
    return enqueue_batched<float>(nblk, (const float*)A, a_off, m, n, op, J, j_off, (float*)Z, z_off, info, order,
                                  queue, reinterpret_cast<float*>(w + kNaOffRows), grid, na_rows<float>(grid), s);
}

}  // extern "C"
