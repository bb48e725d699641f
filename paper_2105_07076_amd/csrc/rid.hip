// rid.hip -- randomized ID with a Gaussian row sketch on gfx950.
//
// Paper: Advani & O'Hagan, Section 2.2 (the randomized method runs the same
// column-pivoted QR on a smaller matrix and maps the chosen columns back to
// A) and Section 2.2.1 (the key is a smaller matrix with which to compute the
// ID).  The smaller matrix here is the row sketch Y = Omega A (l x n) with a
// Gaussian Omega; the CPQR of Y (the driver shared with id_cpqr, FP32 with
// FP64 norms and an FP64 triangular solve) gives J and T, and C = A[:, J].
//
// The sketch runs on the matrix cores: v_mfma_f32_32x32x16_bf16, Omega exact
// in bfloat16, A rounded to bfloat16 once (mode 0), split as hi + mid with
// hi = bf16(a), mid = bf16(a - hi) (mode 1, two passes: |a - hi - mid| <=
// 2^-16 |a|, bfloat16's unit roundoff being 2^-8), or as hi + mid + lo
// (mode 2, three passes: 2^-24 |a|, FP32's own rounding), FP32 accumulation;
// the differences a - hi and a - hi - mid are exact in FP32.
#include <algorithm>

#include "common.hpp"
#include "handle.hpp"
#include "cpqr.hpp"
#include "prof.hpp"

namespace miid {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f16v_t __attribute__((ext_vector_type(16)));

constexpr int kSkK = 16;  // K of one v_mfma_f32_32x32x16_bf16

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

// Y = Omega A on the matrix cores, 32 x 32 tiles of Y (v_mfma_f32_32x32x16_bf16:
// 32 x 16 by 16 x 32, FP32 accumulation).  A workgroup of WR x WC waves owns
// 32 WC columns of Y and every row tile: wave (wr, wc) accumulates row tiles
// RT wr .. RT wr + RT - 1 of the 32 columns starting at 32 wc.  Operand
// layout of the instruction: lane l holds row l % 32 and k = 8 (l / 32) + e
// (e < 8) of the Omega operand, and k = 8 (l / 32) + e of column l % 32 of the
// A operand; accumulator element r of lane l is row 8 (r / 4) + 4 (l / 32) +
// r % 4, column l % 32.
//
// K runs in chunks of 32.  A chunk's Omega rows (64 bytes each) and A
// columns (128 bytes each) go straight from memory into an NS-stage ring in
// LDS (global_load_lds / buffer_load ... lds, 1 KiB per wave instruction, no
// registers), NS - 1 chunks ahead of the one being multiplied; each wave
// waits only for its own copies of the current chunk (an exact count of
// outstanding loads) before the one barrier per chunk.  Within a row or a
// column the 16-byte segments are stored XOR-permuted, so that the lanes that
// read the same segment of consecutive rows or columns hit different banks.
// A is read through a buffer resource based at the workgroup's first column
// (loads past its last element return zero); the last chunk, when m is not a
// multiple of 32, is copied through registers with the rows >= m zeroed.
// A is split into NSPLIT bfloat16 parts (1: hi = bf16(a); 2: hi + mid with
// mid = bf16(a - hi); 3: hi + mid + lo with lo = bf16(a - hi - mid)), one
// product per part and Omega operand.  Rows lpad .. ldw - 1 of S are written
// as zeros.
typedef __attribute__((address_space(3))) void lds_void_t;

constexpr int kSkKC = 32;  // K per chunk
constexpr int64_t kSkMaxLda = (int64_t)1 << 23;  // 128 columns of A within 32-bit byte offsets

// segment permutations (Omega rows: 4 segments, A columns: 8)
__device__ __forceinline__ int om_swz(int row) { return ((row >> 1) ^ (row >> 3)) & 3; }
__device__ __forceinline__ int a_swz(int col) { return (col ^ (col >> 3)) & 7; }

// wait until at most N vector-memory operations of this wave are outstanding
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}

// Workgroup barrier after this wave's LDS writes are done.  Written as one
// asm statement: the compiler's own barrier would also wait for every
// outstanding copy into LDS (later chunks included).
__device__ __forceinline__ void ring_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

typedef int v4i_t __attribute__((ext_vector_type(4)));

// The LDS reads of one MFMA step: RT Omega tiles at aw + 2048 t and the two
// A segments at aa0, aa1 (LDS byte addresses), issued together and waited
// for in the same asm statement.
template <int RT>
struct StepReads;
#define MIID_SK_RD(i) "ds_read_b128 %" #i ", %[aw] offset:" #i "*2048\n\t"
template <>
struct StepReads<3> {
    __device__ __forceinline__ static void run(uint32_t aw, uint32_t aa0, uint32_t aa1, v4i_t (&w)[3], v4i_t& a0,
                                               v4i_t& a1) {
        asm volatile(MIID_SK_RD(0) MIID_SK_RD(1) MIID_SK_RD(2)
                     "ds_read_b128 %[a0], %[aa0]\n\tds_read_b128 %[a1], %[aa1]\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(w[0]), "=&v"(w[1]), "=&v"(w[2]), [a0] "=&v"(a0), [a1] "=&v"(a1)
                     : [aw] "v"(aw), [aa0] "v"(aa0), [aa1] "v"(aa1)
                     : "memory");
    }
};
template <>
struct StepReads<5> {
    __device__ __forceinline__ static void run(uint32_t aw, uint32_t aa0, uint32_t aa1, v4i_t (&w)[5], v4i_t& a0,
                                               v4i_t& a1) {
        asm volatile(MIID_SK_RD(0) MIID_SK_RD(1) MIID_SK_RD(2) MIID_SK_RD(3) MIID_SK_RD(4)
                     "ds_read_b128 %[a0], %[aa0]\n\tds_read_b128 %[a1], %[aa1]\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(w[0]), "=&v"(w[1]), "=&v"(w[2]), "=&v"(w[3]), "=&v"(w[4]), [a0] "=&v"(a0),
                       [a1] "=&v"(a1)
                     : [aw] "v"(aw), [aa0] "v"(aa0), [aa1] "v"(aa1)
                     : "memory");
    }
};
template <>
struct StepReads<6> {
    __device__ __forceinline__ static void run(uint32_t aw, uint32_t aa0, uint32_t aa1, v4i_t (&w)[6], v4i_t& a0,
                                               v4i_t& a1) {
        asm volatile(MIID_SK_RD(0) MIID_SK_RD(1) MIID_SK_RD(2) MIID_SK_RD(3) MIID_SK_RD(4) MIID_SK_RD(5)
                     "ds_read_b128 %[a0], %[aa0]\n\tds_read_b128 %[a1], %[aa1]\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(w[0]), "=&v"(w[1]), "=&v"(w[2]), "=&v"(w[3]), "=&v"(w[4]), "=&v"(w[5]), [a0] "=&v"(a0),
                       [a1] "=&v"(a1)
                     : [aw] "v"(aw), [aa0] "v"(aa0), [aa1] "v"(aa1)
                     : "memory");
    }
};
template <>
struct StepReads<8> {
    __device__ __forceinline__ static void run(uint32_t aw, uint32_t aa0, uint32_t aa1, v4i_t (&w)[8], v4i_t& a0,
                                               v4i_t& a1) {
        asm volatile(MIID_SK_RD(0) MIID_SK_RD(1) MIID_SK_RD(2) MIID_SK_RD(3) MIID_SK_RD(4) MIID_SK_RD(5)
                         MIID_SK_RD(6) MIID_SK_RD(7)
                     "ds_read_b128 %[a0], %[aa0]\n\tds_read_b128 %[a1], %[aa1]\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(w[0]), "=&v"(w[1]), "=&v"(w[2]), "=&v"(w[3]), "=&v"(w[4]), "=&v"(w[5]), "=&v"(w[6]),
                       "=&v"(w[7]), [a0] "=&v"(a0), [a1] "=&v"(a1)
                     : [aw] "v"(aw), [aa0] "v"(aa0), [aa1] "v"(aa1)
                     : "memory");
    }
};
template <>
struct StepReads<9> {
    __device__ __forceinline__ static void run(uint32_t aw, uint32_t aa0, uint32_t aa1, v4i_t (&w)[9], v4i_t& a0,
                                               v4i_t& a1) {
        asm volatile(MIID_SK_RD(0) MIID_SK_RD(1) MIID_SK_RD(2) MIID_SK_RD(3) MIID_SK_RD(4) MIID_SK_RD(5)
                         MIID_SK_RD(6) MIID_SK_RD(7) MIID_SK_RD(8)
                     "ds_read_b128 %[a0], %[aa0]\n\tds_read_b128 %[a1], %[aa1]\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(w[0]), "=&v"(w[1]), "=&v"(w[2]), "=&v"(w[3]), "=&v"(w[4]), "=&v"(w[5]), "=&v"(w[6]),
                       "=&v"(w[7]), "=&v"(w[8]), [a0] "=&v"(a0), [a1] "=&v"(a1)
                     : [aw] "v"(aw), [aa0] "v"(aa0), [aa1] "v"(aa1)
                     : "memory");
    }
};
#undef MIID_SK_RD

template <int NSPLIT, int RT, int WR, int WC, int NS, int KG>
__global__ void __launch_bounds__(64 * WR * WC * KG) k_sketch(const float* __restrict__ A, int64_t lda, int64_t m,
                                                         int64_t n, const uint16_t* __restrict__ Wt, int64_t mpad,
                                                         int rt_total, float* __restrict__ S, int64_t ldw,
                                                         float* __restrict__ Yout, int64_t ldy, int l) {
    constexpr int NW = WR * WC;            // waves of one K group
    constexpr int ROWS = WR * RT * 32;     // Omega rows of the workgroup
    constexpr int COLS = 32 * WC;          // columns of the workgroup
    constexpr int OM_BYTES = ROWS * 64;    // Omega chunk: ROWS x 32 bf16
    constexpr int A_BYTES = COLS * 128;    // A chunk: COLS x 32 floats
    constexpr int STAGE = OM_BYTES + A_BYTES;
    constexpr int OM_INS = OM_BYTES / 1024, A_INS = A_BYTES / 1024, INS = OM_INS + A_INS;
    constexpr int BASE = INS / NW, REM = INS % NW;  // copy instructions per wave and stage
    constexpr int KS = kSkKC / kSkK;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x;
    const int wave_all = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int kg = wave_all / NW;          // K group: chunks kg, kg + KG, kg + 2 KG, ...
    const int wave = wave_all % NW;        // the wave within its group
    const int wr = wave % WR, wc = wave / WR;
    const int rt0 = wr * RT;
    const int nrt = min(RT, rt_total - rt0);  // this wave's row tiles (may be <= 0)
    const int rows_st = rt_total * 32;        // rows of Wt
    const int64_t col0 = (int64_t)blockIdx.x * COLS;
    const int ncv = (int)min<int64_t>(COLS, n - col0);
    const uint32_t arec = (uint32_t)min<int64_t>(((int64_t)(ncv - 1) * lda + m) * 4, (int64_t)0x7FFFFFF0);
    const __amdgpu_buffer_rsrc_t rsA =
        __builtin_amdgcn_make_buffer_rsrc((void*)(A + col0 * lda), (short)0, (int)arec, 0x00020000);
    const int nfull = (int)(m / kSkKC);       // chunks with every row < m
    const int nch = (int)(mpad / kSkKC);      // all chunks (mpad = m rounded up to 32)
    const int nit = (nch + KG - 1) / KG;      // iterations: one chunk per K group each
    unsigned char* const ring = smem_raw + kg * NS * STAGE;  // this group's ring
    // the chunk of iteration i for this wave's group (>= nch: none)
    auto chunk_of = [&](int i) { return KG * i + kg; };

    // stage i % NS of the group's ring: Omega rows and A columns of the
    // chunk of iteration i
    auto issue = [&](int i) {
        unsigned char* sb = ring + (i % NS) * STAGE;
        const int c = chunk_of(i);
        const int64_t k0 = (int64_t)c * kSkKC;
        const bool tail = c >= nfull;
        for (int ins = wave; ins < INS; ins += NW) {
            if (ins < OM_INS) {
                const int row = 16 * ins + lane / 4;
                const int q = (lane % 4) ^ om_swz(row);
                const int srow = row < rows_st ? row : 0;  // rows past Wt: any valid row (never read)
                __builtin_amdgcn_global_load_lds((const void*)(Wt + (int64_t)srow * mpad + k0 + 8 * q),
                                                 (lds_void_t*)(sb + ins * 1024), 16, 0, 0);
            } else {
                const int ia = ins - OM_INS;
                const int c_ = 8 * ia + lane / 8;
                const int q = (lane % 8) ^ a_swz(c_);
                const uint32_t voff = (uint32_t)(((int64_t)c_ * lda + k0 + 4 * q) * 4);
                if (!tail) {
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsA, (lds_void_t*)(sb + OM_BYTES + ia * 1024), 16,
                                                             voff, 0, 0, 0);
                } else {
                    // the last chunk: rows >= m (the caller's padding or the
                    // next column) are zeroed
                    float4 v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rsA, voff, 0, 0));
                    const int64_t kr = k0 + 4 * q;
                    if (kr + 0 >= m) v.x = 0.f;
                    if (kr + 1 >= m) v.y = 0.f;
                    if (kr + 2 >= m) v.z = 0.f;
                    if (kr + 3 >= m) v.w = 0.f;
                    *reinterpret_cast<float4*>(sb + OM_BYTES + ia * 1024 + lane * 16) = v;
                }
            }
        }
    };

    f16v_t acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;

    const int cl = wc * 32 + lane % 32;  // this lane's A column within the workgroup
    const int ga = a_swz(cl);
    const int h = lane / 32;
    // LDS byte addresses: the ring, this lane's first Omega row (tile t is
    // 2048 t further; every tile's rows share the row's segment permutation)
    // and this lane's A column
    const uint32_t lds0 = (uint32_t)(uintptr_t)(lds_void_t*)smem_raw;
    const int row0 = rt0 * 32 + lane % 32;
    const uint32_t woff = (uint32_t)(row0 * 64);
    const int sw = om_swz(row0);
    const uint32_t aoff = (uint32_t)(OM_BYTES + cl * 128);
#pragma unroll
    for (int i = 0; i < NS - 1; ++i)
        if (chunk_of(i) < nch) issue(i);
    for (int i = 0; i < nit; ++i) {
        // this wave's copies of iteration i's chunk are done once only those
        // of the NS - 2 later (full) chunks of its group can be outstanding
        if (NS > 2 && chunk_of(i + NS - 2) < nfull) {
            if (REM != 0 && wave < REM)
                wait_vm<(BASE + 1) * (NS > 2 ? NS - 2 : 0)>();
            else
                wait_vm<BASE * (NS > 2 ? NS - 2 : 0)>();
        } else {
            wait_vm<0>();
        }
        // every group's copies of iteration i are in LDS; iteration i - 1's
        // buffers are free
        ring_barrier();
        if (chunk_of(i + NS - 1) < nch) issue(i + NS - 1);
        if (chunk_of(i) >= nch) continue;  // the last iteration of a group without a chunk (uniform per wave)
        const uint32_t sb = lds0 + (uint32_t)(kg * NS * STAGE + (i % NS) * STAGE);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int q0 = 4 * ks + 2 * h;
            v4i_t wv[RT], av0, av1;
            StepReads<RT>::run(sb + woff + 16 * ((2 * ks + h) ^ sw), sb + aoff + 16 * (q0 ^ ga),
                               sb + aoff + 16 * ((q0 + 1) ^ ga), wv, av0, av1);
            const float4 a0 = __builtin_bit_cast(float4, av0);
            const float4 a1 = __builtin_bit_cast(float4, av1);
            const float x[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
            // a = hi + mid + lo: each part the bfloat16 rounding of what the
            // earlier parts leave (exact differences in FP32)
            bf16x8_t hi, mid, lo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const __bf16 hh = (__bf16)x[e];
                hi[e] = hh;
                const float r1 = x[e] - (float)hh;
                const __bf16 mm = (__bf16)r1;
                mid[e] = mm;
                lo[e] = (__bf16)(r1 - (float)mm);
            }
            // the hi products of every tile, then the lo products: a tile's
            // second product comes RT instructions after its first (back to
            // back they would wait for each other).  Tiles past the last row
            // tile multiply rows of the stage that are never stored (no
            // branches: a predicate per tile would make the compiler copy the
            // accumulators around it)
#pragma unroll
            for (int t = 0; t < RT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, wv[t]), hi, acc[t], 0,
                                                                  0, 0);
            if (NSPLIT >= 2) {
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, wv[t]), mid,
                                                                      acc[t], 0, 0, 0);
            }
            if (NSPLIT >= 3) {
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, wv[t]), lo,
                                                                      acc[t], 0, 0, 0);
            }
        }
    }
    if constexpr (KG == 2) {
        // the second group's sums into the first group's (one addition per
        // element, the same order everywhere): through LDS, laid out
        // [wave][tile][element][lane] over the ring, which no copy targets any
        // more (every issued chunk was waited for)
        float* red = reinterpret_cast<float*>(smem_raw);
        __syncthreads();
        if (kg == 1) {
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int r = 0; r < 16; ++r) red[((wave * RT + t) * 16 + r) * kWave + lane] = acc[t][r];
        }
        __syncthreads();
        if (kg == 1) return;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[t][r] += red[((wave * RT + t) * 16 + r) * kWave + lane];
    }
    const int64_t col = col0 + cl;
    if (col >= n) return;
    // accumulator elements 4 q .. 4 q + 3 are four consecutive rows of the
    // column: one 16-byte store each into S (ldw is a multiple of 64)
    float* sc = S + col * ldw;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        if (t < nrt) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = (int64_t)(rt0 + t) * 32 + 8 * q + 4 * h;
                if (row < ldw)
                    *reinterpret_cast<float4*>(sc + row) = float4(acc[t][4 * q], acc[t][4 * q + 1],
                                                                 acc[t][4 * q + 2], acc[t][4 * q + 3]);
                if (Yout) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (row + e < l) Yout[row + e + col * ldy] = acc[t][4 * q + e];
                }
            }
        }
    }
    // the rows below the last tile, zero (the CPQR reads ldw rows)
    if (wr == 0) {
        for (int64_t row = (int64_t)rt_total * 32 + 4 * h; row < ldw; row += 8)
            *reinterpret_cast<float4*>(sc + row) = float4(0.f, 0.f, 0.f, 0.f);
    }
}

// LDS bytes of a k_sketch instantiation (a ring per K group)
constexpr size_t sketch_lds(int rt, int wr, int wc, int ns, int kg) {
    return (size_t)kg * ns * ((size_t)wr * rt * 32 * 64 + (size_t)32 * wc * 128);
}

template <int NSPLIT, int RT, int WR, int WC, int NS, int KG = 1>
static hipError_t launch_sketch(int pr, hipStream_t s, int64_t n, int rt_total, const float* A, int64_t lda, int64_t m,
                                const uint16_t* Wt, int64_t mpad, float* S, int64_t ldw, float* Y, int64_t ldy,
                                int l) {
    constexpr size_t lds = sketch_lds(RT, WR, WC, NS, KG);
    static_assert(lds <= 160 * 1024, "LDS of a CU");
    static_assert(KG == 1 || KG == 2, "one or two K groups");
    // the second group's accumulators pass through the first group's ring
    static_assert(KG == 1 || (size_t)WR * WC * RT * 16 * kWave * 4 <= lds, "reduction fits the ring");
    {
        const hipError_t e = lds_limit_once((const void*)k_sketch<NSPLIT, RT, WR, WC, NS, KG>, (int)lds);
        if (e != hipSuccess) return e;
    }
    dim3 grid((unsigned)((n + 32 * WC - 1) / (32 * WC)));
    MIID_LAUNCH(pr, (k_sketch<NSPLIT, RT, WR, WC, NS, KG>), grid, dim3(64 * WR * WC * KG), lds, s, A, lda, m, n, Wt, mpad,
                rt_total, S, ldw, Y, ldy, l);
    return hipGetLastError();
}

// Workgroup shape from the 32-row tiles of Y: two waves along the rows with
// 5 or 9 tiles each up to 18 tiles (576 rows), four with 8 tiles beyond (at
// most 32 tiles: l <= 1024); four waves along the columns when that still
// gives two workgroups per CU, else two.  The ring depth fills the LDS.  Up
// to 9 tiles with fewer than two 128-column workgroups per CU (one wave per
// SIMD in the shape above), three waves of 3 tiles along the rows, two along
// the columns, and two K groups, each with its own ring, taking alternate
// chunks of K: three waves per SIMD on the same 64 columns.
template <int NSPLIT>
static hipError_t launch_sketch_shape(int pr, hipStream_t s, int64_t n, int rt_total, const float* A, int64_t lda,
                                      int64_t m, const uint16_t* Wt, int64_t mpad, float* S, int64_t ldw, float* Y,
                                      int64_t ldy, int l) {
    const bool wide = (n + 127) / 128 >= 2 * (int64_t)dev_info().cus;
    if (rt_total <= 9 && !wide)
        return launch_sketch<NSPLIT, 3, 3, 2, 3, 2>(pr, s, n, rt_total, A, lda, m, Wt, mpad, S, ldw, Y, ldy, l);
    if (rt_total <= 10)
        return wide ? launch_sketch<NSPLIT, 5, 2, 4, 4>(pr, s, n, rt_total, A, lda, m, Wt, mpad, S, ldw, Y, ldy, l)
                    : launch_sketch<NSPLIT, 5, 2, 2, 4>(pr, s, n, rt_total, A, lda, m, Wt, mpad, S, ldw, Y, ldy, l);
    if (rt_total <= 18)
        return wide ? launch_sketch<NSPLIT, 6, 3, 4, 3>(pr, s, n, rt_total, A, lda, m, Wt, mpad, S, ldw, Y, ldy, l)
                    : launch_sketch<NSPLIT, 9, 2, 2, 3>(pr, s, n, rt_total, A, lda, m, Wt, mpad, S, ldw, Y, ldy, l);
    return launch_sketch<NSPLIT, 8, 4, 2, 2>(pr, s, n, rt_total, A, lda, m, Wt, mpad, S, ldw, Y, ldy, l);
}

struct RidPlan {
    IdPlan id;
    int lpad;        // rows of Wt (32-row tiles)
    int rt_total;    // 32-row tiles of Y
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
    R->rt_total = (l + 31) / 32;
    R->lpad = R->rt_total * 32;
    if (R->lpad > R->id.ldw) return MIID_E_UNSUPPORTED;
    R->mpad = (int64_t)align_up((size_t)m, 32);
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
    // the sketch addresses a workgroup's 128 columns of A with 32-bit offsets
    if (lda > kSkMaxLda) return MIID_E_UNSUPPORTED;
    if (ldo < l) return -7;
    if (mode < 0 || mode > 2) return -8;
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

    {
        dim3 grid((unsigned)((R.mpad + 63) / 64), (unsigned)((R.lpad + 63) / 64));
        hipLaunchKernelGGL(k_omega_t, grid, dim3(256), 0, s, Omega, l, m, ldo, Wt, R.lpad, R.mpad);
    }
    {
        const int pr = prof_take(MIID_K_SKETCH, 0, m, n);
        hipError_t e;
        if (mode == 2)
            e = launch_sketch_shape<3>(pr, s, n, R.rt_total, A, lda, m, Wt, R.mpad, S, ldw, Y, ldy, l);
        else if (mode == 1)
            e = launch_sketch_shape<2>(pr, s, n, R.rt_total, A, lda, m, Wt, R.mpad, S, ldw, Y, ldy, l);
        else
            e = launch_sketch_shape<1>(pr, s, n, R.rt_total, A, lda, m, Wt, R.mpad, S, ldw, Y, ldy, l);
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
