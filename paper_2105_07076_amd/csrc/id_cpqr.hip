// id_cpqr.hip -- deterministic ID on gfx950: rank-k truncated column-pivoted
// Householder QR (Businger-Golub pivoting with norm downdating and exact
// recomputation), blocked in panels, followed by the FP64 triangular solve
// T = R11^{-1} R12 that gives Z = [I T] P^T.
//
// Paper: Advani & O'Hagan, Section 2.1 (C = A P_k from the pivoted QR; Z from
// the least-squares problem, reduced to triangular solves), Section 4.1 (stop
// the QR after k columns), Definition 1 (Z[:, J] = I), Section 2 footnote
// (m > n: work on A^T).
//
// Design (one GPU, HBM-bound):
//  * Columns are never swapped.  A selected column is marked dead (nu < 0)
//    and the rows of R are stored in a k x n buffer indexed by the original
//    column, so Z = R11^{-1} R comes out directly in original column order.
//  * Blocked right-looking QR with a lazily updated panel (compact-WY form):
//    inside a panel the trailing matrix S is stale; step j reads it once
//    (the F-GEMV) and keeps V (Householder vectors) and F = S^T V T.  At the
//    end of a panel S -= V F^T is applied in one pass.
//  * Each step is two launches: a small row-parallel kernel that updates the
//    pivot column and forms the reflector's partial sums, and a
//    column-parallel kernel that finishes the reflector (every workgroup
//    redundantly, from the same partials, so no atomics are needed), streams
//    the trailing matrix once for the F column, updates row j of R,
//    downdates the column norms and writes per-workgroup argmax partials for
//    the next step.
//  * Column norms are FP64.  When the downdate cancels (the test of Drmac &
//    Bujanovic, LAPACK Working Note 176) the norm is recomputed exactly
//    from the lazily updated column, inside the same kernel, without ending
//    the panel; so the host's launch sequence is fixed.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include <type_traits>

#include "common.hpp"
#include "handle.hpp"
#include "cpqr.hpp"
#include "prof.hpp"

namespace miid {

constexpr int kThreads = 256;
constexpr int kRowsPerChunk = 256; // rows per workgroup of the pivot-column kernel
constexpr int kMaxNb = 64;
constexpr int kPartAStride = kMaxNb + 1;
constexpr int kMaxK = 1024;
constexpr size_t kMaxVecLds = 131072;  // bytes of LDS for the reflector in the GEMV


// ---------------------------------------------------------------------------
// a1: staging.  S (ldw x n, padded rows zero) <- A (inside the first norm
// pass, k_norms<T, true>), or A^T for the dual ID.
// ---------------------------------------------------------------------------
// S[r, c] = A[c, r] (A is n x m with leading dimension lda), 64 x 64 tiles.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_stage_transpose(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                              T* __restrict__ S, int64_t ldw) {
    __shared__ T tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.x * 64;  // rows of S = columns of A
    const int64_t c0 = (int64_t)blockIdx.y * 64;  // columns of S = rows of A
    const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
    for (int e = ty; e < 64; e += 4) {
        const int64_t ar = c0 + tx, ac = r0 + e;  // A[ar, ac]
        tile[e][tx] = (ar < n && ac < m) ? A[ar + ac * lda] : T(0);
    }
    __syncthreads();
    for (int e = ty; e < 64; e += 4) {
        const int64_t sr = r0 + tx, sc = c0 + e;  // S[sr, sc] = A[sc, sr]
        if (sc < n && sr < ldw) S[sr + sc * ldw] = tile[tx][e];
    }
}

// Column norms of S with FP64 accumulation; sel = -1; argmax partials.
// Workgroup b owns columns [4 cpw b, 4 cpw (b + 1)), wave w the cpw columns
// starting at 4 cpw b + w cpw (the same partition as k_gemv).  With STAGE
// the columns come from A (m x n, leading dimension lda) and are written to
// S on the way (a1 and the first norms in one pass over A).
template <typename T, bool STAGE>
__global__ void __launch_bounds__(kThreads) k_norms(const T* __restrict__ A, int64_t lda, int64_t m,
                                                    T* __restrict__ S, int64_t ldw, int64_t n, int cpw,
                                                    double* __restrict__ nu, double* __restrict__ nuref,
                                                    int32_t* __restrict__ sel, ColPartial* __restrict__ part,
                                                    int32_t* __restrict__ recomp) {
    __shared__ double s_best[4], s_sum[4];
    __shared__ int32_t s_idx[4], s_nf[4];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    ArgMax best{-1.0, INT32_MAX};
    double sum = 0.0;
    int nf = 0;
    for (int c = 0; c < cpw; ++c) {
        const int64_t col = ((int64_t)blockIdx.x * 4 + wave) * cpw + c;
        if (col >= n) break;
        double acc = 0.0;
        if (STAGE) {
            // A's columns need not be 16-byte aligned: element loads, four
            // in flight per lane
            const T* a = A + col * lda;
            T* sc = S + col * ldw;
            int64_t r = lane;
            for (; r + 3 * kWave < ldw; r += 4 * kWave) {
                T x[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) x[q] = r + q * kWave < m ? a[r + q * kWave] : T(0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    sc[r + q * kWave] = x[q];
                    acc += (double)x[q] * (double)x[q];
                }
            }
            for (; r < ldw; r += kWave) {
                const T x = r < m ? a[r] : T(0);
                sc[r] = x;
                acc += (double)x * (double)x;
            }
        }
        // 16-byte loads, four in flight per lane (ldw is a multiple of 64)
        using VT = typename Vec16<T>::type;
        constexpr int VEC = Vec16<T>::n;
        const VT* s = reinterpret_cast<const VT*>(S + col * ldw);
        const int64_t ng = STAGE ? 0 : ldw / VEC;
        int64_t g = lane;
        for (; g + 3 * kWave < ng; g += 4 * kWave) {
            VT v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = s[g + q * kWave];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc += (double)get(v[q], e) * (double)get(v[q], e);
        }
        for (; g < ng; g += kWave) {
            const VT v = s[g];
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc += (double)get(v, e) * (double)get(v, e);
        }
        acc = wave_sum(acc);
        const double v = sqrt(acc);
        if (!is_finite_d(v)) nf = 1;
        if (lane == 0) {
            nu[col] = v;
            nuref[col] = v;
            sel[col] = -1;
        }
        if (argmax_better(v, (int32_t)col, best.v, best.i)) best = {v, (int32_t)col};
        sum += acc;
    }
    if (lane == 0) {
        s_best[wave] = best.v;
        s_idx[wave] = best.i;
        s_sum[wave] = sum;
        s_nf[wave] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ArgMax b{s_best[0], s_idx[0]};
        double t = s_sum[0];
        int f = s_nf[0];
        for (int w = 1; w < 4; ++w) {
            if (argmax_better(s_best[w], s_idx[w], b.v, b.i)) b = {s_best[w], s_idx[w]};
            t += s_sum[w];
            f |= s_nf[w];
        }
        part[blockIdx.x] = ColPartial{b.v, b.i, f, t, 0.0};
        recomp[blockIdx.x] = 0;
    }
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t count, T value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ---------------------------------------------------------------------------
// a2 + a3 + first half of a4: pivot search, lazy update of the pivot column,
// partial sums for the reflector.  One thread per row, 256 rows per workgroup;
// NBT >= nb bounds the unrolled loops over the panel.
// ---------------------------------------------------------------------------
template <typename T, int NBT>
__global__ void __launch_bounds__(kThreads) k_pivot_col(const T* __restrict__ S, int64_t ldw, int64_t m,
                                                        const T* __restrict__ V, const T* __restrict__ F, int nb,
                                                        T* __restrict__ u, const ColPartial* __restrict__ part,
                                                        int npart, double* __restrict__ partA,
                                                        DevState* __restrict__ st, int32_t* __restrict__ J, int j,
                                                        int i, int tol_mode, double eps) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double s_F[kMaxNb];
    __shared__ double s_red[kThreads / 32][kPartAStride];
    __shared__ double w_best[4], w_sum[4];
    __shared__ int32_t w_idx[4], w_nf[4];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int64_t r = (int64_t)blockIdx.x * kRowsPerChunk + tid;
    const bool active = r >= j && r < m;
    const int stop_in = st->stop;
    const double a_prev = st->a_norm;

    // a2: pivot = argmax of the per-workgroup column partials (same order in
    // every workgroup, no atomics).  The first kPU per thread are all issued
    // before anything else, so one memory round trip covers them.
    ArgMax best{-1.0, INT32_MAX};
    double sumsq = 0.0;
    int nf = 0;
    constexpr int kPU = 16;
    ColPartial cp[kPU];
#pragma unroll
    for (int k = 0; k < kPU; ++k) {
        const int q = tid + k * kThreads;
        cp[k] = q < npart ? part[q] : ColPartial{-1.0, INT32_MAX, 0, 0.0, 0.0};
    }
    // row r of the panel's reflectors does not depend on the pivot: its loads
    // go out now, behind the partials (so waiting for those does not wait
    // for these)
    // (columns q >= i load column i - 1 again, a cache hit, so that the
    // loads need no branch and the traffic stays i columns).  Beyond 32
    // columns the rest is loaded with the pivot column, once the partials no
    // longer hold registers.
    constexpr int NLO = NBT > 32 ? 32 : NBT;
    double vr[NBT];
    const int64_t rv = r < ldw ? r : 0;
    const int qlast = i > 0 ? i - 1 : 0;
    auto load_vr = [&](int q) {
        vr[q] = (double)load_or(V, r + (int64_t)q * ldw, active && q < i, rv + (int64_t)min(q, qlast) * ldw, T(0));
    };
#pragma unroll
    for (int q = 0; q < NLO; ++q) load_vr(q);
#pragma unroll
    for (int k = 0; k < kPU; ++k) {
        if (argmax_better(cp[k].best, cp[k].idx, best.v, best.i)) best = {cp[k].best, cp[k].idx};
        sumsq += cp[k].sumsq;
        nf |= cp[k].nonfinite;
    }
    for (int q = tid + kPU * kThreads; q < npart; q += kThreads) {  // more than kPU per thread: rare
        const ColPartial cp = part[q];
        if (argmax_better(cp.best, cp.idx, best.v, best.i)) best = {cp.best, cp.idx};
        sumsq += cp.sumsq;
        nf |= cp.nonfinite;
    }
    if (stop_in) return;
    best = wave_argmax(best);
    sumsq = wave_sum(sumsq);
    nf = __any(nf) ? 1 : 0;
    if (lane == 0) {
        w_best[wave] = best.v;
        w_idx[wave] = best.i;
        w_sum[wave] = sumsq;
        w_nf[wave] = nf;
    }
    __syncthreads();
    fold_waves<4>(w_best, w_idx, w_sum, w_nf, best, sumsq, nf);

    const double a_norm = (j == 0) ? sqrt(sumsq) : a_prev;
    uint32_t status = 0;
    bool stop = false;
    if (nf) {
        stop = true;
        status = MIID_NONFINITE;
    } else if (!(best.v > 0.0) || best.i == INT32_MAX) {
        stop = true;
        status = MIID_RANK_DEFICIENT;
    } else if (tol_mode && sqrt(sumsq) <= eps * a_norm) {
        stop = true;
    }
    if (blockIdx.x == 0 && tid == 0) {
        if (j == 0) st->a_norm = a_norm;
        if (stop) {
            st->k_out = j;
            st->status |= status;
            st->stop = 1;
        } else {
            J[j] = best.i;
        }
    }
    if (stop) return;
    const int64_t p = best.i;
#pragma unroll
    for (int q = NLO; q < NBT; ++q) load_vr(q);
    const double spr = (double)load_or(S, r + p * ldw, active, p * ldw, T(0));
    const double fp = (double)load_or(F, p * nb + tid, tid < i, p * nb, T(0));
    if (tid < i) s_F[tid] = fp;
    __syncthreads();

    // a3: lazily updated pivot column u = S[:, p] - V F[p, :]^T (rows j..m-1),
    // the sum over the panel in four interleaved chains
    double ua[4] = {spr, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NBT; ++q)
        if (q < i) ua[q & 3] -= vr[q] * s_F[q];
    const double ur = (ua[0] + ua[1]) + (ua[2] + ua[3]);
    const T ut = (T)ur;
    // u[j] is kept apart (u[ldw]) so that u is zero at and above row j and the
    // GEMV can use it directly: v = e_j + scale * u.
    if (r < ldw) u[r] = (active && r != j) ? ut : T(0);
    if (r == j) u[ldw] = ut;
    // a4 partial sums over the chunk's rows: sum_{r>j} u_r^2 and
    // V[j+1:, q]^T u[j+1:], q < i.  Each thread's i + 1 products go to a row
    // of sP; 32-row slices of every column are then summed in parallel and
    // the eight slice sums in a fixed order (no chain of i wave reductions).
    const double w = (active && r > j) ? (double)ut : 0.0;
    const int ncol = i + 1;
    double* sP = reinterpret_cast<double*>(smem_raw);  // kThreads x (nb + 1)
    const int ldp = nb + 1;
    sP[tid * ldp] = w * w;
#pragma unroll
    for (int q = 0; q < NBT; ++q)
        if (q < i) sP[tid * ldp + 1 + q] = vr[q] * w;
    __syncthreads();
    for (int c = tid % 32; c < ncol; c += 32) {
        const int h = tid / 32;  // slice of 32 rows
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int rr = 0; rr < 32; ++rr) a[rr & 3] += sP[(h * 32 + rr) * ldp + c];
        s_red[h][c] = (a[0] + a[1]) + (a[2] + a[3]);
    }
    __syncthreads();
    if (tid < ncol) {
        double t = 0.0;
#pragma unroll
        for (int h = 0; h < kThreads / 32; ++h) t += s_red[h][tid];
        partA[(int64_t)blockIdx.x * kPartAStride + tid] = t;
    }

}

// ---------------------------------------------------------------------------
// a5 + a6 (+ a8 when flagged): F-GEMV over the stale trailing matrix, row j of
// R, norm downdate / exact recompute, argmax partials for the next step.
// C columns per wave, 4 waves per workgroup, lanes over rows with 16-byte
// loads.  The reflector is v = e_j + scale * u with u read from L2 (zero at
// rows <= j), so the stream starts without waiting on any reduction.
// ---------------------------------------------------------------------------
constexpr int kPrefetchA = 4;  // partial-sum entries prefetched per thread

template <typename T, int C>
__global__ void __launch_bounds__(kThreads) k_gemv(const T* __restrict__ S, int64_t ldw, int64_t m, int64_t n,
                                                   T* __restrict__ V, T* __restrict__ F, int nb,
                                                   const T* __restrict__ u, const double* __restrict__ partA, int NA,
                                                   DevState* __restrict__ st, const int32_t* __restrict__ J,
                                                   T* __restrict__ R, double* __restrict__ nu,
                                                   double* __restrict__ nuref, int32_t* __restrict__ sel,
                                                   ColPartial* __restrict__ part, int32_t* __restrict__ recomp, int j,
                                                   int i, double tol) {
    using VT = typename Vec16<T>::type;
    constexpr int VEC = Vec16<T>::n;
    constexpr int U = C >= 4 ? 4 : (C == 2 ? 4 : 8);  // 16-byte loads in flight per column per lane
    __shared__ double s_y[kMaxNb], s_vj[kMaxNb];
    __shared__ double s_pa[kPrefetchA * kThreads];
    __shared__ double s_red[kPartAStride];
    __shared__ double s_best[4], s_sum[4];
    __shared__ int32_t s_idx[4], s_nrec[4];

    const int tid = threadIdx.x;
    // Serpentine sweep: odd steps walk the columns from the far end, so the
    // part of the matrix read last in one step (still in the memory-side
    // cache) is read first in the next.
    const int wg = (j & 1) ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int64_t col0 = ((int64_t)wg * 4 + wave) * C;
    const int stop = st->stop;
    const int64_t p = J[j];  // meaningful only when !stop
    // the pivot kernel's partial sums (sum u^2, V^T u per row chunk), u[j]
    // and V[j, 0:i]: loaded now, used after the stream, so that their latency
    // hides behind it
    const int na = NA * (i + 1);
    double pa[kPrefetchA];
#pragma unroll
    for (int k = 0; k < kPrefetchA; ++k) {
        const int e = tid + k * kThreads;
        pa[k] = load_or(partA, (int64_t)(e / (i + 1)) * kPartAStride + e % (i + 1), e < na, 0, 0.0);
    }
    const double u0 = (double)u[ldw];
    const double vjq = (double)load_or(V, j + (int64_t)tid * ldw, tid < i, 0, T(0));

    // per-column scalars, loaded together before the stream (on the range
    // only: none of these loads waits for another; reading the dead columns
    // too, to spare the stream the wait for their norms, cost more)
    bool alive[C];
    double fq[C], nuc[C], nrf[C], sjc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t col = col0 + c;
        const bool in = col < n;
        const double nv = load_or(nu, col, in, 0, -1.0);
        nrf[c] = load_or(nuref, col, in, 0, 1.0);
        fq[c] = (double)load_or(F, col * nb + lane, in && lane < i, 0, T(0));
        sjc[c] = (double)load_or(S, col * ldw + j, in, 0, T(0));
        nuc[c] = nv;
        alive[c] = in && col != p && nv >= 0.0;
    }

    // a5: acc_c = S[j0:, col_c] . u  (u is zero at rows <= j and >= m).  j0
    // is j rounded down to a 128-byte line, so that no line is split between
    // two of a wave's loads (nontemporal loads would fetch it twice)
    const int64_t j0 = (int64_t)j & ~(int64_t)(128 / sizeof(T) - 1);
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    const int64_t ngroups = (ldw - j0) / VEC;
    const VT* up = reinterpret_cast<const VT*>(u + j0);
    const VT* sp[C];
#pragma unroll
    for (int c = 0; c < C; ++c) sp[c] = reinterpret_cast<const VT*>(S + (col0 + c) * ldw + j0);
    // the stream over S; NTL: loads marked nontemporal.  Every pass issues
    // its U loads per column together, the last one masked per lane at the
    // end of the column (a remainder loop of single loads would wait a full
    // memory round trip per 64 groups).
    auto stream = [&](auto ntl) {
        constexpr bool NTL = decltype(ntl)::value;
        for (int64_t g = lane; g < ngroups; g += U * kWave) {
            VT sv[C][U], uv[U];
#pragma unroll
            for (int q = 0; q < U; ++q) uv[q] = g + q * kWave < ngroups ? up[g + q * kWave] : VT{};
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (alive[c]) {
#pragma unroll
                    for (int q = 0; q < U; ++q) {
                        const int64_t gq = g + q * kWave;
                        sv[c][q] = gq < ngroups ? (NTL ? load_nt(&sp[c][gq]) : sp[c][gq]) : VT{};
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if (alive[c]) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) acc[c] += (double)get(sv[c][q], e) * (double)get(uv[q], e);
                    }
                }
            }
        }
    };
    // FP64: the first third of the workgroups in dispatch order (the columns
    // the previous step read last, still in the memory-side cache) load
    // nontemporally, so that re-reading them does not push out what the rest
    // of this step brings in -- the part the next step, sweeping back, reads
    // first.  FP32 steps (half the bytes) nearly fit that cache and stay
    // ordinary.  Measured on the 4096 x 16384 FP64 ID with 64-wide panels:
    // 26.4 ms with no nontemporal loads, 25.6 with the first third, 26.8 with
    // two thirds, 27.0 with all of them.
    if (sizeof(T) == 8 && 3 * (int64_t)blockIdx.x < (int64_t)gridDim.x)
        stream(std::true_type{});
    else
        stream(std::false_type{});
    if (stop) return;

    // a4 (second half): the reflector, identical in every workgroup
#pragma unroll
    for (int k = 0; k < kPrefetchA; ++k) s_pa[tid + k * kThreads] = pa[k];
    __syncthreads();
    if (tid <= i) {
        double t = 0.0;
        if (na <= kPrefetchA * kThreads) {
            for (int c = 0; c < NA; ++c) t += s_pa[c * (i + 1) + tid];
        } else {
            for (int c = 0; c < NA; ++c) t += partA[(int64_t)c * kPartAStride + tid];
        }
        s_red[tid] = t;
    }
    __syncthreads();
    const double alpha = sqrt(u0 * u0 + s_red[0]);
    if (!(alpha > 0.0)) {  // the pivot column vanished: rank(A) == j
        if (blockIdx.x == 0 && tid == 0) {
            st->k_out = j;
            st->status |= MIID_RANK_DEFICIENT;
            st->stop = 1;
        }
        return;
    }
    const double beta = u0 >= 0.0 ? -alpha : alpha;
    const double tau = (beta - u0) / beta;
    const double scale = 1.0 / (u0 - beta);
    if (tid < i) {
        s_vj[tid] = vjq;
        s_y[tid] = vjq + scale * s_red[1 + tid];
    }
    if (blockIdx.x == 0) {
        for (int64_t r = tid; r < ldw; r += kThreads)
            V[r + (int64_t)i * ldw] = r < j ? T(0) : (r == j ? T(1) : (T)((double)u[r] * scale));
        if (tid == 0) {
            R[(int64_t)j * n + p] = (T)beta;
            sel[p] = j;
        }
    }
    if (tid == 0 && p / (4 * C) == wg) nu[p] = -1.0;
    __syncthreads();

    // a6: F column, row j of R, norm downdate (a8: exact recompute if flagged)
    ArgMax best{-1.0, INT32_MAX};
    double sumsq = 0.0;
    int nrec = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (!alive[c]) continue;
        const int64_t col = col0 + c;
        const double dot = sjc[c] + scale * wave_sum(acc[c]);
        const double t1 = wave_sum(lane < i ? fq[c] * s_y[lane] : 0.0);
        const double t2 = wave_sum(lane < i ? fq[c] * s_vj[lane] : 0.0);
        const T fT = (T)(tau * (dot - t1));
        const double f = (double)fT;
        const double rjl = sjc[c] - t2 - f;
        if (lane == 0) {
            F[col * nb + i] = fT;
            R[(int64_t)j * n + col] = (T)rjl;
        }
        double nnew = nuc[c];
        bool rec = false;
        if (nuc[c] > 0.0) {
            double t = fabs(rjl) / nuc[c];
            t = fmax(0.0, (1.0 - t) * (1.0 + t));
            const double ratio = nuc[c] / nrf[c];
            if (t * ratio * ratio <= tol)
                rec = true;
            else
                nnew = nuc[c] * sqrt(t);
        }
        if (rec) {
            // exact norm of the lazily updated column, rows j+1..m-1
            double ss = 0.0;
            for (int64_t r = j + 1 + lane; r < m; r += kWave) {
                double x = (double)S[col * ldw + r] - scale * (double)u[r] * f;
                for (int q = 0; q < i; ++q) x -= (double)V[r + (int64_t)q * ldw] * (double)F[col * nb + q];
                ss += x * x;
            }
            ss = wave_sum(ss);
            nnew = sqrt(ss);
            ++nrec;
            if (lane == 0) nuref[col] = nnew;
        }
        if (lane == 0) nu[col] = nnew;
        if (argmax_better(nnew, (int32_t)col, best.v, best.i)) best = {nnew, (int32_t)col};
        sumsq += nnew * nnew;
    }
    if (lane == 0) {
        s_best[wave] = best.v;
        s_idx[wave] = best.i;
        s_sum[wave] = sumsq;
        s_nrec[wave] = nrec;
    }
    __syncthreads();
    if (tid == 0) {
        ArgMax b2{s_best[0], s_idx[0]};
        double t = s_sum[0];
        int nr = s_nrec[0];
        for (int w = 1; w < 4; ++w) {
            if (argmax_better(s_best[w], s_idx[w], b2.v, b2.i)) b2 = {s_best[w], s_idx[w]};
            t += s_sum[w];
            nr += s_nrec[w];
        }
        part[wg] = ColPartial{b2.v, b2.i, 0, t, 0.0};
        recomp[wg] += nr;
    }
}

// ---------------------------------------------------------------------------
// a2-a6 (+ a8) in one launch per step for short matrices (the sketch Y of the
// randomized ID, short IDs: at most 576 rows in FP32, 320 in FP64, panels of
// at most 32).  The working matrix then sits in the L2 caches and the step is
// latency-bound: the separate pivot kernel's launch and its reduction over
// thousands of partials cost more than the GEMV.  Here every workgroup (8
// waves, one per CU)
//   1. reduces the previous step's per-workgroup partials to the pivot p, the
//      residual sum of squares and the stop decision, while the panel's V
//      columns are staged into LDS and its first column chunk is in flight;
//   2. forms the lazily updated pivot column u = S[:, p] - V F[p, :]^T and
//      the reflector (identical in every workgroup: same inputs, same order);
//   3. runs the F-GEMV over its own columns (16 lanes per column) and V^T v
//      from LDS, then the row of R, the norm downdate and the exact recompute
//      of flagged columns, and writes its partial.
// The partials ping-pong between two buffers (step j reads buffer j & 1 and
// writes the other), because every workgroup reads all of them.  Column
// partition: workgroup b owns 32 NP consecutive columns, wave w the 4 NP
// starting at 32 NP b + 4 NP w.
// ---------------------------------------------------------------------------
constexpr int kFusedWaves = 8;
constexpr int kFusedThreads = kFusedWaves * kWave;
constexpr int kFusedMaxNb = 32;
constexpr int kFusedMaxRows = 576;

// sum over the 16 lanes of a row group (every lane of the group ends with it)
__device__ __forceinline__ double group16_sum(double v) { return row16_sum(v); }

// One column's rows j0..ldw-1 as seen by lane l16 of its 16-lane group:
// 16-byte groups l16, l16 + 16, ... (GL of them at most), loaded together.
template <typename T, int GL>
struct ColChunk {
    using VT = typename Vec16<T>::type;
    VT v[GL];
    // base: the column's row j0 where ok, else any valid element
    __device__ __forceinline__ void load(const T* base, bool ok, int64_t ngroups, int l16) {
#pragma unroll
        for (int t = 0; t < GL; ++t) {
            const int64_t g = l16 + 16 * t;
            v[t] = load_or(reinterpret_cast<const VT*>(base), g, ok && g < ngroups, 0, VT{});
        }
    }
    // sum over this lane's rows of x_r * u_r (u in LDS, indexed from j0)
    __device__ __forceinline__ double dot(const double* su, int64_t ngroups, int l16) const {
        constexpr int VEC = Vec16<T>::n;
        double a = 0.0;
#pragma unroll
        for (int t = 0; t < GL; ++t) {
            const int64_t g = l16 + 16 * t;
            if (g < ngroups) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) a += (double)get(v[t], e) * su[g * VEC + e];
            }
        }
        return a;
    }
};

template <typename T, int NP, int GL>
__global__ void __launch_bounds__(kFusedThreads) k_step_fused(const T* __restrict__ S, int64_t ldw, int64_t m,
                                                              int64_t n, T* __restrict__ V, T* __restrict__ F, int nb,
                                                              const ColPartial* __restrict__ part_in,
                                                              ColPartial* __restrict__ part_out, int npart,
                                                              DevState* __restrict__ st, int32_t* __restrict__ J,
                                                              T* __restrict__ R, double* __restrict__ nu,
                                                              double* __restrict__ nuref, int32_t* __restrict__ sel,
                                                              int32_t* __restrict__ recomp, int j, int i,
                                                              int tol_mode, double eps, double tol) {
    using VT = typename Vec16<T>::type;
    constexpr int VEC = Vec16<T>::n;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sV = reinterpret_cast<T*>(smem_raw);  // V[:, 0:i], column q at sV + q ldw
    __shared__ double s_u[kFusedMaxRows];
    __shared__ double s_F[kFusedMaxNb], s_y[kFusedMaxNb], s_vj[kFusedMaxNb], s_g[kFusedMaxNb];
    __shared__ double w_best[kFusedWaves], w_sum[kFusedWaves];
    __shared__ int32_t w_idx[kFusedWaves], w_nf[kFusedWaves], w_nrec[kFusedWaves];
    __shared__ double s_x0;
    __shared__ double s_fg[kFusedWaves * 4][kFusedMaxNb];  // F[col, 0:i] of a group's recomputed column

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int l16 = lane & 15, grp = lane >> 4;
    const int wg = blockIdx.x;
    const int stop_in = st->stop;
    const double a_prev = st->a_norm;
    // rows from j rounded down to a 128-byte line (u is zero at rows <= j)
    const int64_t j0 = (int64_t)j & ~(int64_t)(128 / sizeof(T) - 1);
    const int64_t ngroups = (ldw - j0) / VEC;  // VEC-row groups from j0

    // the previous step's partials first: the loads below are independent of
    // them and of each other, so one memory round trip covers them all
    // (npart <= kFusedThreads partials: one per thread)
    const ColPartial cp0 = load_or(part_in, tid, tid < npart, 0, ColPartial{-1.0, INT32_MAX, 0, 0.0, 0.0});

    // this wave's columns and their per-column data, independent of the pivot
    // (loaded whatever the column's state; used only for alive columns).
    // Up to four passes per wave the data is loaded here, in flight with the
    // partials; with eight (one workgroup per CU over the widest matrices),
    // or four over columns of nine or ten 16-byte groups per lane, it is
    // loaded after the dot products, when the column chunks no longer hold
    // registers.
    constexpr bool kLate = NP > 4 || (NP == 4 && GL >= 9);
    int64_t col[NP];
    bool in[NP];
    double nuc[NP], nrf[NP], sjc[NP], fq[NP][kFusedMaxNb / 16];
#pragma unroll
    for (int ps = 0; ps < NP; ++ps) {
        col[ps] = (int64_t)wg * 32 * NP + (int64_t)wave * 4 * NP + ps * 4 + grp;
        in[ps] = col[ps] < n;
    }
    auto load_cols = [&]() {
#pragma unroll
        for (int ps = 0; ps < NP; ++ps) {
            nuc[ps] = load_or(nu, col[ps], in[ps], 0, -1.0);
            nrf[ps] = load_or(nuref, col[ps], in[ps], 0, 1.0);
            sjc[ps] = (double)load_or(S, col[ps] * ldw + j, in[ps], 0, T(0));
#pragma unroll
            for (int s = 0; s < kFusedMaxNb / 16; ++s) {
                const int q = l16 + 16 * s;
                fq[ps][s] = (double)load_or(F, col[ps] * nb + q, in[ps] && q < i, 0, T(0));
            }
        }
    };
    if (!kLate) load_cols();
    // the first two column chunks and V[:, 0:i] (GL 16-byte groups per
    // thread at most: i ldw / VEC <= 32 * 16 GL) are in flight while the
    // pivot is found
    ColChunk<T, GL> buf[2];
#pragma unroll
    for (int ps = 0; ps < (NP < 2 ? NP : 2); ++ps) buf[ps].load(in[ps] ? S + col[ps] * ldw + j0 : S, in[ps], ngroups, l16);
    const int64_t vtot = (ldw / VEC) * i;
    VT vst[GL];
#pragma unroll
    for (int k = 0; k < GL; ++k) {
        const int64_t e = tid + (int64_t)k * kFusedThreads;
        vst[k] = load_or(reinterpret_cast<const VT*>(V), e, e < vtot, 0, VT{});
    }

    // 1. pivot from the previous step's partials
    ArgMax best{-1.0, INT32_MAX};
    double sumsq = 0.0;
    int nf = 0;
    if (argmax_better(cp0.best, cp0.idx, best.v, best.i)) best = {cp0.best, cp0.idx};
    sumsq += cp0.sumsq;
    nf |= cp0.nonfinite;
    for (int q = tid + kFusedThreads; q < npart; q += kFusedThreads) {
        const ColPartial cp = part_in[q];
        if (argmax_better(cp.best, cp.idx, best.v, best.i)) best = {cp.best, cp.idx};
        sumsq += cp.sumsq;
        nf |= cp.nonfinite;
    }
    if (stop_in) return;
    best = wave_argmax_dpp(best);
    sumsq = wave_sum_dpp(sumsq);
    nf = __any(nf) ? 1 : 0;
    if (lane == 0) {
        w_best[wave] = best.v;
        w_idx[wave] = best.i;
        w_sum[wave] = sumsq;
        w_nf[wave] = nf;
    }
    lds_barrier();
    fold_waves<kFusedWaves>(w_best, w_idx, w_sum, w_nf, best, sumsq, nf);
    const double a_norm = (j == 0) ? sqrt(sumsq) : a_prev;
    {
        uint32_t status = 0;
        bool stop = false;
        if (nf) {
            stop = true;
            status = MIID_NONFINITE;
        } else if (!(best.v > 0.0) || best.i == INT32_MAX) {
            stop = true;
            status = MIID_RANK_DEFICIENT;
        } else if (tol_mode && sqrt(sumsq) <= eps * a_norm) {
            stop = true;
        }
        if (wg == 0 && tid == 0) {
            if (j == 0) st->a_norm = a_norm;
            if (stop) {
                st->k_out = j;
                st->status |= status;
                st->stop = 1;
            } else {
                J[j] = best.i;
            }
        }
        if (stop) return;
    }
    const int64_t p = best.i;

    // 2. u = S[:, p] - V F[p, :]^T (rows j..m-1), the reflector; the pivot
    // column's rows (two per thread at most: ldw <= 2 x 512) and F[p, 0:i]
    // are loaded together
    static_assert(kFusedMaxRows <= 2 * kFusedThreads, "two pivot-column rows per thread at most");
    double spc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t r = tid + (int64_t)h * kFusedThreads;
        spc[h] = (double)load_or(S, r + p * ldw, r >= j && r < m, p * ldw, T(0));
    }
    const double fp = (double)load_or(F, p * nb + tid, tid < i, p * nb, T(0));
    if (tid < i) s_F[tid] = fp;
#pragma unroll
    for (int k = 0; k < GL; ++k) {
        const int64_t e = tid + (int64_t)k * kFusedThreads;
        if (e < vtot) reinterpret_cast<VT*>(sV)[e] = vst[k];
    }
    lds_barrier();  // s_F, sV (and the w_* reads above are done)
    if (tid < i) s_vj[tid] = (double)sV[j + (int64_t)tid * ldw];
    double ss = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t r = tid + (int64_t)h * kFusedThreads;
        if (r >= ldw) break;
        double x = 0.0;
        if (r >= j && r < m) {
            x = spc[h];
#pragma unroll 8
            for (int q = 0; q < i; ++q) x -= (double)sV[r + (int64_t)q * ldw] * s_F[q];
            x = (double)(T)x;
        }
        if (r == j) s_x0 = x;
        s_u[r] = r > j ? x : 0.0;
        ss += r > j ? x * x : 0.0;
    }
    ss = wave_sum_dpp(ss);
    if (lane == 0) w_sum[wave] = ss;
    lds_barrier();
    const double x0 = s_x0;
    double s0 = 0.0;
    for (int w = 0; w < kFusedWaves; ++w) s0 += w_sum[w];
    const double alpha = sqrt(x0 * x0 + s0);
    if (!(alpha > 0.0)) {  // the pivot column vanished: rank(A) == j
        if (wg == 0 && tid == 0) {
            st->k_out = j;
            st->status |= MIID_RANK_DEFICIENT;
            st->stop = 1;
        }
        return;
    }
    const double beta = x0 >= 0.0 ? -alpha : alpha;
    const double tau = (beta - x0) / beta;
    const double scale = 1.0 / (x0 - beta);
    if (wg == 0) {
        for (int64_t r = tid; r < ldw; r += kFusedThreads)
            V[r + (int64_t)i * ldw] = r < j ? T(0) : (r == j ? T(1) : (T)(s_u[r] * scale));
        if (tid == 0) {
            R[(int64_t)j * n + p] = (T)beta;
            sel[p] = j;
        }
    }
    if (tid == 0 && p / (32 * NP) == wg) nu[p] = -1.0;

    // 3a. dots with u: the wave's NP columns (one chunk loaded ahead of the
    // one in use), then V^T u from LDS (column q = 4 wave + group)
    const double* su = s_u + j0;
    double acc[NP];
#pragma unroll
    for (int ps = 0; ps < NP; ++ps) {
        // (kLate: every column in range; the dead ones' sums go unused)
        const bool alive = kLate ? in[ps] : (in[ps] && col[ps] != p && nuc[ps] >= 0.0);
        acc[ps] = alive ? buf[ps & 1].dot(su, ngroups, l16) : 0.0;
        if (ps + 2 < NP) buf[ps & 1].load(in[ps + 2] ? S + col[ps + 2] * ldw + j0 : S, in[ps + 2], ngroups, l16);
    }
    if (kLate) load_cols();
    {
        const int q = 4 * wave + grp;
        double a = 0.0;
        if (q < i) {
            const T* vq = sV + (int64_t)q * ldw + j0;
            for (int64_t g = l16; g < ngroups; g += 16) {
                const VT vv = *reinterpret_cast<const VT*>(vq + g * VEC);
#pragma unroll
                for (int e = 0; e < VEC; ++e) a += (double)get(vv, e) * su[g * VEC + e];
            }
        }
        a = group16_sum(a);
        if (q < i && l16 == 0) s_g[q] = a;
    }
#pragma unroll
    for (int ps = 0; ps < NP; ++ps) acc[ps] = group16_sum(acc[ps]);
    lds_barrier();
    if (tid < i) s_y[tid] = s_vj[tid] + scale * s_g[tid];
    lds_barrier();

    // 3b. F column, row j of R, downdate / recompute, partials
    ArgMax b2{-1.0, INT32_MAX};
    double sum2 = 0.0;
    int nrec = 0;
#pragma unroll
    for (int ps = 0; ps < NP; ++ps) {
        const bool alive = in[ps] && col[ps] != p && nuc[ps] >= 0.0;
        if (!alive) continue;  // uniform over the 16-lane group
        double t1 = 0.0, t2 = 0.0;
#pragma unroll
        for (int s = 0; s < kFusedMaxNb / 16; ++s) {
            const int q = l16 + 16 * s;
            if (q < i) {
                t1 += fq[ps][s] * s_y[q];
                t2 += fq[ps][s] * s_vj[q];
            }
        }
        t1 = group16_sum(t1);
        t2 = group16_sum(t2);
        const double dot = sjc[ps] + scale * acc[ps];
        const T fT = (T)(tau * (dot - t1));
        const double f = (double)fT;
        const double rjl = sjc[ps] - t2 - f;
        if (l16 == 0) {
            F[col[ps] * nb + i] = fT;
            R[(int64_t)j * n + col[ps]] = (T)rjl;
        }
        double nnew = nuc[ps];
        bool rec = false;
        if (nuc[ps] > 0.0) {
            double t = fabs(rjl) / nuc[ps];
            t = fmax(0.0, (1.0 - t) * (1.0 + t));
            const double ratio = nuc[ps] / nrf[ps];
            if (t * ratio * ratio <= tol)
                rec = true;
            else
                nnew = nuc[ps] * sqrt(t);
        }
        if (rec) {
            // exact norm of the lazily updated column, rows j+1..m-1; the
            // column's F row goes through the group's LDS slot
            double* fg = s_fg[wave * 4 + grp];
#pragma unroll
            for (int s = 0; s < kFusedMaxNb / 16; ++s) {
                const int q = l16 + 16 * s;
                if (q < i) fg[q] = fq[ps][s];
            }
            double s2 = 0.0;
            for (int64_t r = j + 1 + l16; r < m; r += 16) {
                double x = (double)S[col[ps] * ldw + r] - scale * s_u[r] * f;
                for (int q = 0; q < i; ++q) x -= (double)sV[r + (int64_t)q * ldw] * fg[q];
                s2 += x * x;
            }
            nnew = sqrt(group16_sum(s2));
            if (l16 == 0) {
                ++nrec;
                nuref[col[ps]] = nnew;
            }
        }
        if (l16 == 0) {
            nu[col[ps]] = nnew;
            if (argmax_better(nnew, (int32_t)col[ps], b2.v, b2.i)) b2 = {nnew, (int32_t)col[ps]};
            sum2 += nnew * nnew;
        }
    }
    b2 = wave_argmax_dpp(b2);
    sum2 = wave_sum_dpp(sum2);
    nrec = (int)wave_sum_dpp((double)nrec);
    if (lane == 0) {
        w_best[wave] = b2.v;
        w_idx[wave] = b2.i;
        w_sum[wave] = sum2;
        w_nrec[wave] = nrec;
    }
    lds_barrier();
    if (tid == 0) {
        ArgMax b3{w_best[0], w_idx[0]};
        double t = w_sum[0];
        int nr = w_nrec[0];
        for (int w = 1; w < kFusedWaves; ++w) {
            if (argmax_better(w_best[w], w_idx[w], b3.v, b3.i)) b3 = {w_best[w], w_idx[w]};
            t += w_sum[w];
            nr += w_nrec[w];
        }
        part_out[wg] = ColPartial{b3.v, b3.i, 0, t, 0.0};
        if (nr) recomp[wg] += nr;
    }
}

// ---------------------------------------------------------------------------
// a7: trailing update at the end of a panel, S[r0:, :] -= V[r0:, 0:w] F[:, 0:w]^T,
// on the matrix cores.  64 x 64 tile per workgroup, 32 x 32 per wave (2 x 2
// blocks of 16 x 16), K = w in steps of 4 (v_mfma_{f64,f32}_16x16x4).
// Operands: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16].  Output
// element e of lane l is column l % 16 and row 4 (l / 16) + e for f32 but
// row l / 16 + 4 e for f64 (measured on gfx950).
// ---------------------------------------------------------------------------
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
template <typename T> struct Acc4;
template <> struct Acc4<double> {
    using type = d4_t;
    static __device__ __forceinline__ int row(int lg, int e) { return lg + 4 * e; }
};
template <> struct Acc4<float> {
    using type = f4_t;
    static __device__ __forceinline__ int row(int lg, int e) { return 4 * lg + e; }
};

__device__ __forceinline__ d4_t mfma16x16x4(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma16x16x4(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T, int W>
__global__ void __launch_bounds__(kThreads) k_trail(T* __restrict__ S, int64_t ldw, int64_t n,
                                                    const T* __restrict__ V, const T* __restrict__ F, int nb, int w,
                                                    int64_t r0, const DevState* __restrict__ st) {
    // D = F_tile V_tile^T, so the MFMA's row index runs over columns of S and
    // its column index over rows of S: one accumulator element of 16
    // neighbouring lanes is 16 consecutive rows of one column of S.
    using A4 = typename Acc4<T>::type;
    if (st->stop) return;
    const int64_t rbase = (r0 & ~(int64_t)63) + (int64_t)blockIdx.x * 64;
    const int64_t cbase = (int64_t)blockIdx.y * 64;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;  // wave's 32 rows x 32 columns
    const int l16 = lane % 16, lg = lane / 16;
    A4 acc[2][2];  // [column block][row block]
#pragma unroll
    for (int bc = 0; bc < 2; ++bc)
#pragma unroll
        for (int br = 0; br < 2; ++br) {
            const int64_t row = rbase + wr + br * 16 + l16;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t col = cbase + wc + bc * 16 + Acc4<T>::row(lg, e);
                acc[bc][br][e] = col < n ? S[row + col * ldw] : T(0);
            }
        }
    if (W > 0) {
        // the whole panel's F and V operands in flight at once, then the
        // W / 4 MFMA steps
        constexpr int KS = W > 0 ? W / 4 : 1;
        T a[KS][2], b[KS][2];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int q = 4 * ks + lg;
#pragma unroll
            for (int bc = 0; bc < 2; ++bc) {
                const int64_t col = cbase + wc + bc * 16 + l16;
                a[ks][bc] = col < n ? F[col * nb + q] : T(0);
            }
#pragma unroll
            for (int br = 0; br < 2; ++br) {
                const int64_t row = rbase + wr + br * 16 + l16;
                b[ks][br] = -V[row + (int64_t)q * ldw];
            }
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int bc = 0; bc < 2; ++bc)
#pragma unroll
                for (int br = 0; br < 2; ++br) acc[bc][br] = mfma16x16x4(a[ks][bc], b[ks][br], acc[bc][br]);
    } else {
        for (int k0 = 0; k0 < w; k0 += 4) {
            const int q = k0 + lg;
            T a[2], b[2];
#pragma unroll
            for (int bc = 0; bc < 2; ++bc) {
                const int64_t col = cbase + wc + bc * 16 + l16;
                a[bc] = (q < w && col < n) ? F[col * nb + q] : T(0);
            }
#pragma unroll
            for (int br = 0; br < 2; ++br) {
                const int64_t row = rbase + wr + br * 16 + l16;
                b[br] = q < w ? -V[row + (int64_t)q * ldw] : T(0);
            }
#pragma unroll
            for (int bc = 0; bc < 2; ++bc)
#pragma unroll
                for (int br = 0; br < 2; ++br) acc[bc][br] = mfma16x16x4(a[bc], b[br], acc[bc][br]);
        }
    }
#pragma unroll
    for (int bc = 0; bc < 2; ++bc)
#pragma unroll
        for (int br = 0; br < 2; ++br) {
            const int64_t row = rbase + wr + br * 16 + l16;
            if (row < r0) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t col = cbase + wc + bc * 16 + Acc4<T>::row(lg, e);
                if (col < n) S[row + col * ldw] = acc[bc][br][e];
            }
        }
}

// ---------------------------------------------------------------------------
// a9: R11 (FP64, pivot order, kpad x kpad column-major, kpad = kmax rounded up
// to the diagonal block) gathered from the rows of R; the identity pads it
// beyond the K rows/columns that exist.
// ---------------------------------------------------------------------------
constexpr int kTB = 32;  // diagonal block of the triangular solve

template <typename T>
__global__ void k_gather_r11(const T* __restrict__ R, int64_t n, const int32_t* __restrict__ J, int kmax, int kpad,
                             const DevState* __restrict__ st, int ksteps, double* __restrict__ R11s,
                             double* __restrict__ R11out, int64_t ldr) {
    const int kout = st->stop ? st->k_out : ksteps;
    const int64_t total = (int64_t)kpad * kpad;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(e % kpad), b = (int)(e / kpad);
        double val;
        if (a < kout && b < kout)
            val = a <= b ? (double)R[(int64_t)a * n + J[b]] : 0.0;
        else
            val = a == b ? 1.0 : 0.0;
        R11s[e] = val;
        if (R11out && a < kmax && b < kmax) R11out[a + (int64_t)b * ldr] = (a < kout && b < kout) ? val : 0.0;
    }
}

// Inverses of the kTB x kTB diagonal blocks of R11 (upper triangular), one
// workgroup per block: thread t solves D x = e_t by back substitution, so
// column t of D^{-1} is exact up to the rounding of that substitution.
__global__ void __launch_bounds__(kTB) k_trsm_dinv(const double* __restrict__ R11s, int kpad,
                                                   double* __restrict__ Dinv) {
    __shared__ double sD[kTB][kTB + 1];
    __shared__ double sx[kTB][kTB + 1];  // sx[row][t]
    const int b = blockIdx.x, t = threadIdx.x;
    const int64_t r0 = (int64_t)b * kTB;
    double d[kTB];
#pragma unroll
    for (int c = 0; c < kTB; ++c) d[c] = R11s[(r0 + t) + (r0 + c) * kpad];  // all loads in flight
#pragma unroll
    for (int c = 0; c < kTB; ++c) sD[t][c] = d[c];
    __syncthreads();
    for (int r = kTB - 1; r >= 0; --r) {
        double x = 0.0;
        if (r <= t) {
            double acc = (r == t) ? 1.0 : 0.0;
#pragma unroll 8
            for (int c = r + 1; c <= t; ++c) acc -= sD[r][c] * sx[c][t];
            x = acc / sD[r][r];
        }
        sx[r][t] = x;
    }
    for (int r = 0; r < kTB; ++r) Dinv[(int64_t)b * kTB * kTB + r + (int64_t)t * kTB] = sx[r][t];
}

// Z[:, cols] = R11^{-1} R[:, cols] in FP64 for NC columns per workgroup, by
// block back substitution with the inverted diagonal blocks: the columns'
// right-hand sides stay in LDS (kpad x NC); for row block b (bottom up)
//   T = X_b - sum_{c > b} R11[b, c] X_c,   X_b = D_b^{-1} T.
// The refinement sweep (one step of iterative refinement, residual in FP64)
// runs the same recursion on the residual and overwrites X in place:
//   X_b += D_b^{-1} (B_b - sum_{c >= b} R11[b, c] X_c)
// where the X_c (c > b) are already refined -- in exact arithmetic the same
// correction as solving R11 d = B - R11 X and adding d.
// Both products run on the FP64 matrix cores (v_mfma_f64_16x16x4): wave w
// owns the 16 x 16 tile (rows 16 (w % 2), columns 16 (w / 2)) of the
// kTB x NC block; A operand lane l = R11[row l % 16][k l / 16] (from L2),
// B operand lane l = X[k l / 16][col l % 16] (LDS), output element e of
// lane l = row l / 16 + 4 e, column l % 16.
// Z[:, J[c]] = e_c exactly; rows >= K are zero.
// SEMI: the right-hand sides are first replaced by R11^{-T} B with the same
// machinery read transposed (top-down over the row blocks, the transposed
// diagonal-block inverses), so that Z = R11^{-1} R11^{-T} B -- the solution of
// R11^T R11 Z = B (no refinement sweep in this form).
// JMODE 0: the columns marked in sel (sel[c] = step index) are written as
// exact unit vectors (Z[:, J] = I); JMODE 1: their right-hand sides are read
// as zero (the solution's columns come out zero).  The right-hand side
// element (q, c) is R[q rs + c cs] (rows of R: rs = n, cs = 1).
// KG = 2 (back substitution only): two groups of NC / 8 waves on the same
// columns, group g taking the R11 slices g, g + 2, ... of each row block's
// product; the second group's sums reach the first through LDS (added in
// the same order in every run) and the first finishes the block.  Where
// the right-hand sides fill the LDS (one workgroup per CU) this doubles the
// waves per SIMD.
template <typename T, int NC, bool SEMI = false, int JMODE = 0, int KG = 1>
__global__ void __launch_bounds__(8 * NC * KG) k_trsm_blk(const T* __restrict__ R, int64_t n,
                                                     const double* __restrict__ R11s, int kpad,
                                                     const double* __restrict__ Dinv,
                                                     const DevState* __restrict__ st, int ksteps,
                                                     const int32_t* __restrict__ sel, T* __restrict__ Z,
                                                     int64_t ldz, int kmax, int refine, int64_t rs,
                                                     int64_t cs) {
    static_assert(KG == 1 || (KG == 2 && !SEMI), "K groups in the back substitution only");
    constexpr int NT = 8 * NC * KG;
    constexpr int NCP = NC + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* sX = reinterpret_cast<double*>(smem_raw);  // [kpad][NCP]
    __shared__ double sT[kTB][NCP];
    __shared__ double sT1[KG == 2 ? kTB : 1][NCP];  // the second group's sums
    const int K = st->stop ? st->k_out : ksteps;
    const int nbk = (K + kTB - 1) / kTB;
    const int kend = nbk * kTB;
    const int tid = threadIdx.x;
    const int wave_all = tid / kWave, lane = tid % kWave;
    const int kgi = wave_all / (NC / 8);  // K group
    const int wave = wave_all % (NC / 8);
    const int tr = 16 * (wave % 2), tc = 16 * (wave / 2);
    const int l16 = lane % 16, lq = lane / 16;
    const int64_t c0 = (int64_t)blockIdx.x * NC;
    const int64_t col = c0 + tc + l16;  // this lane's output column
    // the workgroup's columns' selection marks (one load per column)
    __shared__ int32_t s_sel[NC];
    for (int cc = tid; cc < NC; cc += NT) s_sel[cc] = c0 + cc < n ? sel[c0 + cc] : -1;
    __syncthreads();
    // the right-hand sides into LDS, eight loads per thread in flight
    for (int e0 = tid; e0 < kend * NC; e0 += 8 * NT) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * NT;
            const int q = e / NC, c = e % NC;
            const bool zc = JMODE == 1 && e < kend * NC && s_sel[c] >= 0;
            v[u] = (double)load_or(R, (int64_t)q * rs + (c0 + c) * cs, e < kend * NC && q < K && c0 + c < n && !zc, 0,
                                   T(0));
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * NT;
            if (e < kend * NC) sX[(e / NC) * NCP + e % NC] = v[u];
        }
    }
    __syncthreads();
    if (SEMI) {
        // Y = R11^{-T} B: for row block b top-down, T = B_b - sum_{c < b}
        // R11[c, b]^T Y_c, Y_b = (D_b^{-1})^T T
        for (int b = 0; b < nbk; ++b) {
            const int r0 = b * kTB;
            d4_t acc;
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = sX[(r0 + tr + lq + 4 * e) * NCP + tc + l16];
            const double* Db = Dinv + (int64_t)b * kTB * kTB;
            const double* ap = R11s + lq + (int64_t)(r0 + tr + l16) * kpad;  // R11[k][row] = (R11^T)[row][k]
            for (int k0 = 0; k0 < r0; k0 += kTB) {
                double av[kTB / 4], xv[kTB / 4];
#pragma unroll
                for (int q = 0; q < kTB / 4; ++q) av[q] = ap[k0 + 4 * q];
#pragma unroll
                for (int q = 0; q < kTB / 4; ++q) xv[q] = sX[(k0 + 4 * q + lq) * NCP + tc + l16];
#pragma unroll
                for (int q = 0; q < kTB / 4; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[q], xv[q], acc, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) sT[tr + lq + 4 * e][tc + l16] = acc[e];
            __syncthreads();
            d4_t out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k0 = 0; k0 < kTB; k0 += 4) {
                const double av = Db[(k0 + lq) + (tr + l16) * kTB];  // (D_b^{-1})^T
                const double xv = sT[k0 + lq][tc + l16];
                out = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xv, out, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) sX[(r0 + tr + lq + 4 * e) * NCP + tc + l16] = out[e];
            __syncthreads();
        }
    }
    for (int sweep = 0; sweep < (refine && !SEMI ? 2 : 1); ++sweep) {
        for (int b = nbk - 1; b >= 0; --b) {
            const int r0 = b * kTB;
            d4_t acc;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = r0 + tr + lq + 4 * e;
                if (kgi != 0)
                    acc[e] = 0.0;
                else if (sweep == 0)
                    acc[e] = sX[row * NCP + tc + l16];
                else
                    acc[e] = (double)load_or(R, (int64_t)row * rs + col * cs, row < K && col < n, 0, T(0));
            }
            // one kTB-deep slice of R11 at a time (kend - kstart is a
            // multiple of kTB): its eight operand loads are all in flight
            // before the first product waits on them
            const int kstart = sweep == 0 ? r0 + kTB : r0;
            const double* ap = R11s + (r0 + tr + l16) + (int64_t)lq * kpad;
            for (int k0 = kstart + kgi * kTB; k0 < kend; k0 += KG * kTB) {
                double av[kTB / 4], xv[kTB / 4];
#pragma unroll
                for (int q = 0; q < kTB / 4; ++q) av[q] = ap[(int64_t)(k0 + 4 * q) * kpad];
#pragma unroll
                for (int q = 0; q < kTB / 4; ++q) xv[q] = sX[(k0 + 4 * q + lq) * NCP + tc + l16];
#pragma unroll
                for (int q = 0; q < kTB / 4; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[q], xv[q], acc, 0, 0, 0);
            }
            if constexpr (KG == 2) {
                if (kgi == 1) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) sT1[tr + lq + 4 * e][tc + l16] = acc[e];
                }
                __syncthreads();
                if (kgi == 0) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        sT[tr + lq + 4 * e][tc + l16] = acc[e] + sT1[tr + lq + 4 * e][tc + l16];
                }
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) sT[tr + lq + 4 * e][tc + l16] = acc[e];
            }
            __syncthreads();
            if (kgi == 0) {
                const double* Db = Dinv + (int64_t)b * kTB * kTB;
                d4_t out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k0 = 0; k0 < kTB; k0 += 4) {
                    const double av = Db[(tr + l16) + (k0 + lq) * kTB];
                    const double xv = sT[k0 + lq][tc + l16];
                    out = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xv, out, 0, 0, 0);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    double* xp = &sX[(r0 + tr + lq + 4 * e) * NCP + tc + l16];
                    *xp = sweep == 0 ? out[e] : *xp + out[e];
                }
            }
            __syncthreads();
        }
    }
    // Z, column by column of the workgroup's NC
    for (int e = tid; e < kmax * NC; e += NT) {
        const int q = e % kmax, cc = e / kmax;
        const int64_t c = c0 + cc;
        if (c >= n) continue;
        const int s = s_sel[cc];
        double val;
        if (JMODE == 0 && s >= 0 && s < K)
            val = (q == s) ? 1.0 : 0.0;
        else
            val = q < K ? sX[q * NCP + cc] : 0.0;
        Z[q + c * ldz] = (T)val;
    }
}

// a10: C = A[:, J] (or A[J, :]^T), info, J tail = -1.
template <typename T>
__global__ void k_gather_c(const T* __restrict__ A, int64_t lda, int trans, int64_t mrows,
                           const int32_t* __restrict__ J, const DevState* __restrict__ st, int ksteps,
                           T* __restrict__ C, int64_t ldc) {
    const int K = st->stop ? st->k_out : ksteps;
    const int cidx = blockIdx.y;
    if (cidx >= K) return;
    const int64_t src = J[cidx];
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < mrows; r += (int64_t)gridDim.x * blockDim.x)
        C[r + (int64_t)cidx * ldc] = trans ? A[src + r * lda] : A[r + src * lda];
}

// part_alt > 0: the partials ping-pong between part and part + part_alt and
// the last ones written after K steps are in the buffer of parity K; after
// zero steps they are the npart0 partials of the norm pass.
__global__ void k_finalize(const DevState* __restrict__ st, const ColPartial* __restrict__ part, int npart,
                           int part_alt, int npart0, const int32_t* __restrict__ recomp, int32_t* __restrict__ J,
                           int kmax, int ksteps, int tol_mode, double eps, int trans, miid_info* __restrict__ info) {
    __shared__ double s_sum[kThreads];
    __shared__ int32_t s_rec[kThreads];
    const int t = threadIdx.x;
    const int Kd = st->stop ? st->k_out : ksteps;
    if (part_alt > 0 && (Kd & 1)) part += part_alt;
    const int np = (part_alt > 0 && Kd == 0) ? npart0 : npart;
    double s = 0.0;
    int rc = 0;
#pragma unroll 8
    for (int q = t; q < np; q += kThreads) s += part[q].sumsq;
#pragma unroll 8
    for (int q = t; q < npart; q += kThreads) rc += recomp[q];
    s_sum[t] = s;
    s_rec[t] = rc;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            s_sum[t] += s_sum[t + h];
            s_rec[t] += s_rec[t + h];
        }
        __syncthreads();
    }
    const int K = st->stop ? st->k_out : ksteps;
    for (int q = K + t; q < kmax; q += kThreads) J[q] = -1;
    if (t == 0) {
        miid_info o;
        o.k_out = K;
        uint32_t status = st->status;
        const double r22 = sqrt(s_sum[0]);
        if (trans) status |= MIID_TRANSPOSED;
        if (tol_mode && !st->stop && !(r22 <= eps * st->a_norm)) status |= MIID_KMAX_HIT;
        o.status = status;
        o.a_norm = st->a_norm;
        o.r22_norm = (status & (MIID_NONFINITE)) ? NAN : r22;
        o.n_recompute = s_rec[0];
        o.n_steps = K;
        *info = o;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// Columns per wave of the F-GEMV (1, 2 or 4): the CPW hint, else one (timed
// fastest for 4096-row matrices in both precisions: more columns per wave
// mean fewer, longer workgroups and a longer ragged end of each launch).
static int gemv_cols_per_wave(uint32_t flags) {
    const int h = (int)((flags >> MIID_HINT_CPW_SHIFT) & 15u);
    if (h == 1 || h == 2 || h == 4) return h;
    return 1;
}

// The fused path is taken where eligible unless the PATH hint asks for the
// blocked one; the NP hint, else one workgroup per CU, sets the column passes
// per wave.
static bool fused_enabled(uint32_t flags) {
    const int h = (int)((flags >> MIID_HINT_PATH_SHIFT) & 15u);
    return h != 1;
}

static int fused_np(int64_t n, uint32_t flags) {
    const int h = (int)((flags >> MIID_HINT_NP_SHIFT) & 15u);
    if (h == 1 || h == 2 || h == 4 || h == 8) return h;
    for (int v = 1; v <= 8; v *= 2)
        if (n <= (int64_t)256 * 32 * v) return v;  // one workgroup per CU
    return 8;
}

int make_plan(int64_t M, int64_t N, miid_dtype dtype, const miid_opts* o, IdPlan* P) {
    if (M < 1) return -2;
    if (N < 1) return -3;
    if (dtype != MIID_F32 && dtype != MIID_F64) return -5;
    if (!o || o->k < 0 || (o->k == 0 && (o->kmax < 1 || !(o->eps >= 0.0))) || o->nb < 0) return -6;
    P->M = M;
    P->N = N;
    P->trans = M > N && !(o->flags & MIID_KEEP_COLUMNS);
    P->m = P->trans ? N : M;
    P->n = P->trans ? M : N;
    P->tol = o->k == 0;
    P->kmax = P->tol ? o->kmax : o->k;
    P->eps = o->eps;
    // panel width: the caller's, else 32
    P->nb = o->nb != 0 ? o->nb : 32;
    P->refine = !(o->flags & MIID_NO_REFINE);
    if (P->nb > kMaxNb || P->kmax > P->m || P->kmax > P->n || P->kmax > kMaxK) return MIID_E_UNSUPPORTED;
    P->esz = dtype == MIID_F64 ? 8 : 4;
    P->ldw = (int64_t)align_up((size_t)P->m, 64);
    if ((size_t)P->ldw * P->esz > kMaxVecLds) return MIID_E_UNSUPPORTED;
    P->cpw = gemv_cols_per_wave(o->flags);
    P->npart = (int)((P->n + 4 * P->cpw - 1) / (4 * P->cpw));
    P->NA = (int)((P->ldw + kRowsPerChunk - 1) / kRowsPerChunk);
    P->fnp = fused_np(P->n, o->flags);
    P->fnpart = (int)((P->n + 32 * P->fnp - 1) / (32 * P->fnp));
    {
        // 16-byte row groups per lane of a 16-lane column group
        const int64_t ng = P->ldw * (int64_t)P->esz / 16;  // 16-byte groups in a column
        const int64_t per_lane = (ng + 15) / 16;
        // (ten only in FP64: up to 320 rows; FP32 reaches 576 rows with nine)
        P->fgl = per_lane <= 5 ? 5 : (per_lane <= 9 ? 9 : (per_lane <= 10 && P->esz == 8 ? 10 : 0));
    }
    P->fused = P->ldw <= kFusedMaxRows && P->fgl > 0 && P->nb <= kFusedMaxNb && fused_enabled(o->flags);
    // 32 also timed fastest on the blocked path for 4096 x 16384 IDs in both
    // precisions (FP64 with 64: 26.3 against 25.8 ms -- four fewer trailing
    // updates, but the pivot kernel's few workgroups read twice the panel
    // rows per step; FP32 with 16: 13.8 against 13.7 ms); on the fused path
    // it is also the fewest roundings of the eagerly updated trailing matrix
    // for the same time
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o2 = off;
        off = align_up(off + bytes, 256);
        return o2;
    };
    P->oS = take((size_t)P->ldw * P->n * P->esz);
    P->oV = take((size_t)P->ldw * P->nb * P->esz);
    P->oF = take((size_t)P->n * P->nb * P->esz);
    P->ou = take((size_t)(P->ldw + 64) * P->esz);
    P->onu = take((size_t)P->n * 8);
    P->onuref = take((size_t)P->n * 8);
    P->oR = take((size_t)P->kmax * P->n * P->esz);
    P->osel = take((size_t)P->n * 4);
    P->opart = take((size_t)std::max(P->npart, 16 * P->fnpart) * sizeof(ColPartial));
    P->opartA = take((size_t)P->NA * kPartAStride * 8);
    P->kpad = (int)align_up((size_t)P->kmax, kTB);
    P->oR11 = take((size_t)P->kpad * P->kpad * 8);
    P->oDinv = take((size_t)P->kpad * kTB * 8);
    P->ostate = take(sizeof(DevState));
    P->orec = take((size_t)std::max(P->npart, 8 * P->fnpart) * 4);
    P->total = off;
    return 0;
}

template <typename T, int NP, int GL>
static hipError_t launch_fused_k(const IdPlan& P, int pr, hipStream_t stream, T* S, T* V, T* F, ColPartial* pin,
                                 ColPartial* pout, int npin, DevState* st, int32_t* J, T* R, double* nu,
                                 double* nuref, int32_t* sel, int32_t* recomp, int j, int i, double tol) {
    const size_t shmem = (size_t)P.ldw * kFusedMaxNb * P.esz;
    {
        const hipError_t e = lds_limit_once((const void*)k_step_fused<T, NP, GL>,
                                            kFusedMaxRows * kFusedMaxNb * (int)sizeof(T));
        if (e != hipSuccess) return e;
    }
    MIID_LAUNCH(pr, (k_step_fused<T, NP, GL>), dim3(P.fnpart), dim3(kFusedThreads), shmem, stream, S, P.ldw, P.m,
                P.n, V, F, P.nb, pin, pout, npin, st, J, R, nu, nuref, sel, recomp, j, i, (int)P.tol, P.eps, tol);
    return hipGetLastError();
}

template <typename T, int NP>
static hipError_t launch_fused_np(const IdPlan& P, int pr, hipStream_t stream, T* S, T* V, T* F, ColPartial* pin,
                                  ColPartial* pout, int npin, DevState* st, int32_t* J, T* R, double* nu,
                                  double* nuref, int32_t* sel, int32_t* recomp, int j, int i, double tol) {
    if (P.fgl == 5)
        return launch_fused_k<T, NP, 5>(P, pr, stream, S, V, F, pin, pout, npin, st, J, R, nu, nuref, sel, recomp, j,
                                        i, tol);
    if constexpr (sizeof(T) == 8) {
        if (P.fgl == 10)
            return launch_fused_k<T, NP, 10>(P, pr, stream, S, V, F, pin, pout, npin, st, J, R, nu, nuref, sel, recomp,
                                             j, i, tol);
    }
    return launch_fused_k<T, NP, 9>(P, pr, stream, S, V, F, pin, pout, npin, st, J, R, nu, nuref, sel, recomp, j, i,
                                    tol);
}

template <typename T>
static hipError_t launch_fused(const IdPlan& P, int pr, hipStream_t stream, T* S, T* V, T* F, ColPartial* pin,
                               ColPartial* pout, int npin, DevState* st, int32_t* J, T* R, double* nu, double* nuref,
                               int32_t* sel, int32_t* recomp, int j, int i, double tol) {
    switch (P.fnp) {
        case 8:
            return launch_fused_np<T, 8>(P, pr, stream, S, V, F, pin, pout, npin, st, J, R, nu, nuref, sel, recomp,
                                         j, i, tol);
        case 4:
            return launch_fused_np<T, 4>(P, pr, stream, S, V, F, pin, pout, npin, st, J, R, nu, nuref, sel, recomp,
                                         j, i, tol);
        case 2:
            return launch_fused_np<T, 2>(P, pr, stream, S, V, F, pin, pout, npin, st, J, R, nu, nuref, sel, recomp,
                                         j, i, tol);
        default:
            return launch_fused_np<T, 1>(P, pr, stream, S, V, F, pin, pout, npin, st, J, R, nu, nuref, sel, recomp,
                                         j, i, tol);
    }
}

template <typename T>
int run_id(const IdPlan& P, const T* A, int64_t lda, int32_t* J, T* Z, int64_t ldz, double* R11out, int64_t ldr, T* C,
           int64_t ldc, miid_info* info, unsigned char* ws, hipStream_t stream, bool staged, const T* Csrc,
           int64_t ldcsrc, int64_t crows) {
    T* S = reinterpret_cast<T*>(ws + P.oS);
    T* V = reinterpret_cast<T*>(ws + P.oV);
    T* F = reinterpret_cast<T*>(ws + P.oF);
    T* u = reinterpret_cast<T*>(ws + P.ou);
    double* nu = reinterpret_cast<double*>(ws + P.onu);
    double* nuref = reinterpret_cast<double*>(ws + P.onuref);
    T* R = reinterpret_cast<T*>(ws + P.oR);
    int32_t* sel = reinterpret_cast<int32_t*>(ws + P.osel);
    ColPartial* part = reinterpret_cast<ColPartial*>(ws + P.opart);
    double* partA = reinterpret_cast<double*>(ws + P.opartA);
    double* R11s = reinterpret_cast<double*>(ws + P.oR11);
    DevState* st = reinterpret_cast<DevState*>(ws + P.ostate);
    int32_t* recomp = reinterpret_cast<int32_t*>(ws + P.orec);
    const int64_t m = P.m, n = P.n, ldw = P.ldw;
    const int nb = P.nb;

    // dynamic LDS above 64 KB (once per device): the right-hand sides of the
    // solve (the largest kpad of each variant: 256, 512, 1024 rows of NC + 1
    // doubles) and the pivot kernel's per-row products (kThreads x (nb + 1))
    MIID_HIP(lds_limit_once((const void*)k_trsm_blk<T, 64>, 256 * 65 * 8));
    MIID_HIP(lds_limit_once((const void*)k_trsm_blk<T, 32, false, 0, 2>, 512 * 33 * 8));
    MIID_HIP(lds_limit_once((const void*)k_trsm_blk<T, 16>, 1024 * 17 * 8));
    MIID_HIP(lds_limit_once((const void*)k_trsm_blk<T, 64, true>, 256 * 65 * 8));
    MIID_HIP(lds_limit_once((const void*)k_trsm_blk<T, 32, true>, 512 * 33 * 8));
    MIID_HIP(lds_limit_once((const void*)k_trsm_blk<T, 16, true>, 1024 * 17 * 8));
    MIID_HIP(lds_limit_once((const void*)k_pivot_col<T, 16>, kThreads * (16 + 1) * 8));
    MIID_HIP(lds_limit_once((const void*)k_pivot_col<T, 32>, kThreads * (32 + 1) * 8));
    MIID_HIP(lds_limit_once((const void*)k_pivot_col<T, kMaxNb>, kThreads * (kMaxNb + 1) * 8));

    // control block, R rows
    hipLaunchKernelGGL(k_fill<unsigned char>, dim3(1), dim3(64), 0, stream, reinterpret_cast<unsigned char*>(st),
                       (int64_t)sizeof(DevState), (unsigned char)0);
    {
        const int64_t cnt = (int64_t)P.kmax * n;
        const int blocks = (int)std::min<int64_t>((cnt + 255) / 256, 8192);
        hipLaunchKernelGGL(k_fill<T>, dim3(blocks), dim3(256), 0, stream, R, cnt, T(0));
    }
    // a1: stage + norms
    if (staged) {
        // S was filled by the caller (the sketch Y = Omega A)
    } else if (P.trans) {
        dim3 grid((unsigned)((ldw + 63) / 64), (unsigned)((n + 63) / 64));
        hipLaunchKernelGGL(k_stage_transpose<T>, grid, dim3(kThreads), 0, stream, A, lda, m, n, S, ldw);
    }
    // a1 for a plain A happens inside the first norm pass
    const bool stage_in_norms = !staged && !P.trans;
    auto launch_norms = [&](int grid, int cpw) {
        if (stage_in_norms)
            hipLaunchKernelGGL((k_norms<T, true>), dim3(grid), dim3(kThreads), 0, stream, A, lda, m, S, ldw, n, cpw, nu,
                               nuref, sel, part, recomp);
        else
            hipLaunchKernelGGL((k_norms<T, false>), dim3(grid), dim3(kThreads), 0, stream, (const T*)nullptr,
                               (int64_t)0, m, S, ldw, n, cpw, nu, nuref, sel, part, recomp);
    };

    const double tol = sizeof(T) == 8 ? sqrt(2.220446049250313e-16) : sqrt(1.1920928955078125e-07);
    int ksteps = P.kmax;
    int32_t host_stop = 0;
    ColPartial* fin_part = part;
    int fin_npart = P.npart;
    int fin_alt = 0;
    if (P.fused) {
    // the norm pass writes 8 fnpart partials (four-wave workgroups of NP
    // columns per wave) into buffer 0; the steps write fnpart
    fin_npart = P.fnpart;
    fin_alt = 8 * P.fnpart;
    launch_norms(8 * P.fnpart, P.fnp);
    for (int j = 0; j < P.kmax; ++j) {
        const int jb = (j / nb) * nb;
        const int i = j - jb;
        ColPartial* pin = part + (j & 1) * fin_alt;
        ColPartial* pout = part + ((j + 1) & 1) * fin_alt;
        const int npin = j == 0 ? 8 * P.fnpart : P.fnpart;
        const int pr = prof_take(MIID_K_STEP, j, m - j, n - j);
        MIID_HIP(launch_fused<T>(P, pr, stream, S, V, F, pin, pout, npin, st, J, R, nu, nuref, sel, recomp, j, i,
                                 tol));
        if (i == nb - 1 && j + 1 < P.kmax) {
            const int64_t r0 = j + 1;
            const int64_t rbase = r0 & ~(int64_t)63;
            dim3 grid((unsigned)((ldw - rbase + 63) / 64), (unsigned)((n + 63) / 64));
            const int pt = prof_take(MIID_K_TRAIL, j / nb, m - r0, n);
            if (nb == 32)
                MIID_LAUNCH(pt, (k_trail<T, 32>), grid, dim3(kThreads), 0, stream, S, ldw, n, V, F, nb, nb, r0, st);
            else if (nb == 16)
                MIID_LAUNCH(pt, (k_trail<T, 16>), grid, dim3(kThreads), 0, stream, S, ldw, n, V, F, nb, nb, r0, st);
            else
                MIID_LAUNCH(pt, (k_trail<T, 0>), grid, dim3(kThreads), 0, stream, S, ldw, n, V, F, nb, nb, r0, st);
        }
        if (P.tol && (j % 8 == 7) && j + 1 < P.kmax) {
            MIID_HIP(hipMemcpyAsync(&host_stop, &st->stop, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
            MIID_HIP(hipStreamSynchronize(stream));
            if (host_stop) {
                ksteps = j + 1;
                break;
            }
        }
    }
    } else {
    launch_norms(P.npart, P.cpw);
    for (int j = 0; j < P.kmax; ++j) {
        const int jb = (j / nb) * nb;
        const int i = j - jb;
        int pr = prof_take(MIID_K_PIVOT, j, m - j, 1);
        {
            const size_t lds = (size_t)kThreads * (nb + 1) * 8;
            if (nb <= 16)
                MIID_LAUNCH(pr, (k_pivot_col<T, 16>), dim3(P.NA), dim3(kThreads), lds, stream, S, ldw, m, V, F, nb, u,
                            part, P.npart, partA, st, J, j, i, (int)P.tol, P.eps);
            else if (nb <= 32)
                MIID_LAUNCH(pr, (k_pivot_col<T, 32>), dim3(P.NA), dim3(kThreads), lds, stream, S, ldw, m, V, F, nb, u,
                            part, P.npart, partA, st, J, j, i, (int)P.tol, P.eps);
            else
                MIID_LAUNCH(pr, (k_pivot_col<T, kMaxNb>), dim3(P.NA), dim3(kThreads), lds, stream, S, ldw, m, V, F, nb,
                            u, part, P.npart, partA, st, J, j, i, (int)P.tol, P.eps);
        }
        pr = prof_take(MIID_K_GEMV, j, m - j, n - j);
        switch (P.cpw) {
            case 4:
                MIID_LAUNCH(pr, (k_gemv<T, 4>), dim3(P.npart), dim3(kThreads), 0, stream, S, ldw, m, n, V, F, nb, u,
                            partA, P.NA, st, J, R, nu, nuref, sel, part, recomp, j, i, tol);
                break;
            case 2:
                MIID_LAUNCH(pr, (k_gemv<T, 2>), dim3(P.npart), dim3(kThreads), 0, stream, S, ldw, m, n, V, F, nb, u,
                            partA, P.NA, st, J, R, nu, nuref, sel, part, recomp, j, i, tol);
                break;
            default:
                MIID_LAUNCH(pr, (k_gemv<T, 1>), dim3(P.npart), dim3(kThreads), 0, stream, S, ldw, m, n, V, F, nb, u,
                            partA, P.NA, st, J, R, nu, nuref, sel, part, recomp, j, i, tol);
        }
        const bool panel_end = (i == nb - 1);
        if (panel_end && j + 1 < P.kmax) {
            const int64_t r0 = j + 1;
            const int64_t rbase = r0 & ~(int64_t)63;
            dim3 grid((unsigned)((ldw - rbase + 63) / 64), (unsigned)((n + 63) / 64));
            pr = prof_take(MIID_K_TRAIL, j / nb, m - r0, n);
            if (nb == 32)
                MIID_LAUNCH(pr, (k_trail<T, 32>), grid, dim3(kThreads), 0, stream, S, ldw, n, V, F, nb, nb, r0, st);
            else if (nb == 16)
                MIID_LAUNCH(pr, (k_trail<T, 16>), grid, dim3(kThreads), 0, stream, S, ldw, n, V, F, nb, nb, r0, st);
            else if (nb == 64)
                MIID_LAUNCH(pr, (k_trail<T, 64>), grid, dim3(kThreads), 0, stream, S, ldw, n, V, F, nb, nb, r0, st);
            else
                MIID_LAUNCH(pr, (k_trail<T, 0>), grid, dim3(kThreads), 0, stream, S, ldw, n, V, F, nb, nb, r0, st);
        }
        if (P.tol && (j % 8 == 7) && j + 1 < P.kmax) {
            MIID_HIP(hipMemcpyAsync(&host_stop, &st->stop, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
            MIID_HIP(hipStreamSynchronize(stream));
            if (host_stop) {
                ksteps = j + 1;
                break;
            }
        }
    }
    }
    MIID_HIP(hipGetLastError());
    // a9: triangular solve
    {
        double* Dinv = reinterpret_cast<double*>(ws + P.oDinv);
        const int64_t total = (int64_t)P.kpad * P.kpad;
        const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
        hipLaunchKernelGGL(k_gather_r11<T>, dim3(blocks), dim3(256), 0, stream, R, n, J, P.kmax, P.kpad, st, ksteps,
                           R11s, R11out, ldr);
        hipLaunchKernelGGL(k_trsm_dinv, dim3((unsigned)(P.kpad / kTB)), dim3(kTB), 0, stream, R11s, P.kpad, Dinv);
        const int pr = prof_take(MIID_K_TRSM, 0, P.kmax, n);
        if (P.kpad <= 256) {
            MIID_LAUNCH(pr, (k_trsm_blk<T, 64>), dim3((unsigned)((n + 63) / 64)), dim3(8 * 64),
                        (size_t)P.kpad * 65 * 8, stream, R, n, R11s, P.kpad, Dinv, st, ksteps, sel, Z, ldz, P.kmax,
                        (int)P.refine, n, (int64_t)1);
        } else if (P.kpad <= 512) {
            // the right-hand sides fill the LDS: two K groups (eight waves)
            MIID_LAUNCH(pr, (k_trsm_blk<T, 32, false, 0, 2>), dim3((unsigned)((n + 31) / 32)), dim3(8 * 32 * 2),
                        (size_t)P.kpad * 33 * 8, stream, R, n, R11s, P.kpad, Dinv, st, ksteps, sel, Z, ldz, P.kmax,
                        (int)P.refine, n, (int64_t)1);
        } else {
            MIID_LAUNCH(pr, (k_trsm_blk<T, 16>), dim3((unsigned)((n + 15) / 16)), dim3(8 * 16),
                        (size_t)P.kpad * 17 * 8, stream, R, n, R11s, P.kpad, Dinv, st, ksteps, sel, Z, ldz, P.kmax,
                        (int)P.refine, n, (int64_t)1);
        }
    }
    // a10: C, info
    if (C) {
        dim3 grid((unsigned)std::min<int64_t>((crows + 255) / 256, 64), (unsigned)P.kmax);
        hipLaunchKernelGGL(k_gather_c<T>, grid, dim3(256), 0, stream, Csrc, ldcsrc, (int)P.trans, crows, J, st, ksteps,
                           C, ldc);
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, stream, st, fin_part, fin_npart, fin_alt, 8 * P.fnpart, recomp, J, P.kmax,
                       ksteps, (int)P.tol, P.eps, (int)P.trans, info);
    MIID_HIP(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------------------
// The paper's randomized ID by column sampling (Section 2.2, the Optim RID
// listing): CPQR of A_S = A[:, idx] (m x p) for J, then Z from
// R_k^T R_k Z = C^T A over the full A (eq. final_eq).
// ---------------------------------------------------------------------------

// A_S[:, c] = A[:, idx[c]] (an index outside [0, n) gives a zero column)
template <typename T>
__global__ void k_gather_cols(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                              const int32_t* __restrict__ idx, T* __restrict__ As) {
    const int c = blockIdx.y;
    const int64_t src = idx[c];
    const bool ok = src >= 0 && src < n;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x)
        As[r + (int64_t)c * m] = ok ? A[r + src * lda] : T(0);
}

// J[i] = idx[J_S[i]]; sel[J[i]] = i (sel was filled with -1)
__global__ void k_map_idx(const int32_t* __restrict__ Js, const int32_t* __restrict__ idx, int k, int64_t n,
                          int32_t* __restrict__ J, int32_t* __restrict__ sel) {
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const int s = Js[i];
        const int32_t g = s >= 0 ? idx[s] : -1;
        J[i] = g;
        if (g >= 0 && g < n) sel[g] = i;
    }
}

// G (k x n, row-major: G[i n + l]) = C^T A, C m x k (ldc), A m x n (lda),
// on the matrix cores.  Workgroup tile 128 x 128, wave tile 64 x 64 (4 x 4
// blocks of 16 x 16: sixteen products per eight operand loads), K = m in
// batches of 16; the operands of the next batch are loaded while the current
// one is multiplied.  Operand lane l: C^T[row l % 16][k] (= C[k][row],
// contiguous in k) and A[k][column l % 16].  Scalar form: the u-th product
// of a batch takes k = k0 + 4 u + l / 16.  VEC form (16-byte aligned columns):
// lane group g = l / 16 loads the four consecutive k0 + 4 g .. k0 + 4 g + 3 as
// one vector and the u-th product takes k = k0 + 4 g + u -- the same sixteen
// k of the batch, paired identically in both operands.  Split over K:
// workgroup z takes rows [z mz, (z + 1) mz) of C and A and writes the
// partial product to G + z k n.
constexpr int kGtB = 4;  // 16 x 16 blocks per wave side
constexpr int kGtU = 4;  // K steps (of 4) per batch of loads (2: the same, 8: slower)
static_assert(kGtU == 4, "the vector form loads four consecutive k per lane");

template <typename T>
struct Vec4K;
template <>
struct Vec4K<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec4K<double> {
    typedef double type __attribute__((ext_vector_type(4)));
};

template <typename T, bool VEC>
__global__ void __launch_bounds__(kThreads) k_gemm_tn(const T* __restrict__ C, int64_t ldc, const T* __restrict__ A,
                                                      int64_t lda, int64_t m, int k, int64_t n, T* __restrict__ G,
                                                      int64_t mz) {
    using A4 = typename Acc4<T>::type;
    using V4 = typename Vec4K<T>::type;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int i0 = blockIdx.x * 128 + (wave & 1) * 64;               // this wave's rows of G
    const int64_t j0 = (int64_t)blockIdx.y * 128 + (wave >> 1) * 64;  // and columns
    const int l16 = lane % 16, lg = lane / 16;
    {
        const int64_t kb = (int64_t)blockIdx.z * mz;
        C += kb;
        A += kb;
        m = std::min<int64_t>(m - kb, mz);
        G += (int64_t)blockIdx.z * k * n;
    }
    A4 acc[kGtB][kGtB];
#pragma unroll
    for (int br = 0; br < kGtB; ++br)
#pragma unroll
        for (int bc = 0; bc < kGtB; ++bc)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[br][bc][e] = T(0);
    const T* cp[kGtB];
    const T* ap[kGtB];
    bool rok[kGtB], cok[kGtB];
#pragma unroll
    for (int h = 0; h < kGtB; ++h) {
        const int row = i0 + h * 16 + l16;
        const int64_t col = j0 + h * 16 + l16;
        rok[h] = row < k;
        cok[h] = col < n;
        cp[h] = C + (int64_t)(rok[h] ? row : 0) * ldc;
        ap[h] = A + (cok[h] ? col : 0) * lda;
    }
    auto load = [&](int64_t k0, T (&a)[kGtU][kGtB], T (&b)[kGtU][kGtB]) {
        if constexpr (VEC) {
#pragma unroll
            for (int h = 0; h < kGtB; ++h) {
                const V4 va = rok[h] ? *reinterpret_cast<const V4*>(cp[h] + k0 + 4 * lg) : V4(T(0));
                const V4 vb = cok[h] ? *reinterpret_cast<const V4*>(ap[h] + k0 + 4 * lg) : V4(T(0));
#pragma unroll
                for (int u = 0; u < kGtU; ++u) {
                    a[u][h] = va[u];
                    b[u][h] = vb[u];
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < kGtU; ++u)
#pragma unroll
                for (int h = 0; h < kGtB; ++h) {
                    a[u][h] = rok[h] ? cp[h][k0 + 4 * u + lg] : T(0);
                    b[u][h] = cok[h] ? ap[h][k0 + 4 * u + lg] : T(0);
                }
        }
    };
    auto mul = [&](const T (&a)[kGtU][kGtB], const T (&b)[kGtU][kGtB]) {
#pragma unroll
        for (int u = 0; u < kGtU; ++u)
#pragma unroll
            for (int br = 0; br < kGtB; ++br)
#pragma unroll
                for (int bc = 0; bc < kGtB; ++bc) acc[br][bc] = mfma16x16x4(a[u][br], b[u][bc], acc[br][bc]);
    };
    constexpr int KB = 4 * kGtU;  // K per batch
    const int64_t kfull = m > 0 ? m / KB * KB : 0;
    if (kfull > 0) {
        T a0[kGtU][kGtB], b0[kGtU][kGtB], a1[kGtU][kGtB], b1[kGtU][kGtB];
        load(0, a0, b0);
        int64_t k0 = 0;
        for (; k0 + 2 * KB <= kfull; k0 += 2 * KB) {
            load(k0 + KB, a1, b1);
            mul(a0, b0);
            if (k0 + 2 * KB < kfull) load(k0 + 2 * KB, a0, b0);
            mul(a1, b1);
        }
        if (k0 < kfull) mul(a0, b0);  // an odd number of batches: the last one is in a0
    }
    for (int64_t k0 = kfull; k0 < m; k0 += 4) {  // the ragged end of K
        const int64_t kk = k0 + lg;
        T a[kGtB], b[kGtB];
#pragma unroll
        for (int h = 0; h < kGtB; ++h) {
            a[h] = (rok[h] && kk < m) ? cp[h][kk] : T(0);
            b[h] = (cok[h] && kk < m) ? ap[h][kk] : T(0);
        }
#pragma unroll
        for (int br = 0; br < kGtB; ++br)
#pragma unroll
            for (int bc = 0; bc < kGtB; ++bc) acc[br][bc] = mfma16x16x4(a[br], b[bc], acc[br][bc]);
    }
    // output element e of lane l: row Acc4::row(l / 16, e), column l % 16
#pragma unroll
    for (int br = 0; br < kGtB; ++br)
#pragma unroll
        for (int bc = 0; bc < kGtB; ++bc)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = i0 + br * 16 + Acc4<T>::row(lg, e);
                const int64_t col = j0 + bc * 16 + l16;
                if (row < k && col < n) G[(int64_t)row * n + col] = acc[br][bc][e];
            }
}

// G (+ z k n for split z) = C^T A over the row slices of mz rows; the vector
// form when both operands' columns are 16-byte (FP32) / 32-byte (FP64) aligned
template <typename T>
static void gemm_tn(const T* C, int64_t ldc, const T* A, int64_t lda, int64_t m, int k, int64_t n, T* G, int splits,
                    hipStream_t s) {
    const int64_t mz = splits > 1 ? (int64_t)align_up((size_t)((m + splits - 1) / splits), 16) : m;
    const int gz = (int)((m + mz - 1) / mz);
    const uintptr_t va = 4 * sizeof(T) - 1;
    const bool vec = ((reinterpret_cast<uintptr_t>(C) | reinterpret_cast<uintptr_t>(A)) & va) == 0 && ldc % 4 == 0 &&
                     lda % 4 == 0;
    const dim3 grid((unsigned)((k + 127) / 128), (unsigned)((n + 127) / 128), (unsigned)gz);
    if (vec)
        hipLaunchKernelGGL((k_gemm_tn<T, true>), grid, dim3(kThreads), 0, s, C, ldc, A, lda, m, k, n, G, mz);
    else
        hipLaunchKernelGGL((k_gemm_tn<T, false>), grid, dim3(kThreads), 0, s, C, ldc, A, lda, m, k, n, G, mz);
}

struct RsPlan {
    IdPlan id;  // the CPQR of A_S (its workspace comes first)
    size_t oAs, oZs, oJs, oC, oG, oSel, total;
};

static int rs_plan(int64_t m, int64_t n, int32_t p, miid_dtype dtype, const miid_opts* o, RsPlan* Q) {
    if (p < 1 || p > n) return -7;
    if (!o || o->k < 1) return -8;  // fixed rank only
    miid_opts oo = *o;
    oo.flags |= MIID_KEEP_COLUMNS;
    const int rc = make_plan(m, p, dtype, &oo, &Q->id);
    if (rc != 0) return rc == -3 ? -7 : (rc == -6 ? -8 : rc);
    const size_t esz = dtype == MIID_F64 ? 8 : 4;
    const int k = Q->id.kmax;
    size_t off = Q->id.total;
    auto take = [&](size_t bytes) {
        const size_t o2 = off;
        off = align_up(off + bytes, 256);
        return o2;
    };
    Q->oAs = take((size_t)m * p * esz);
    Q->oZs = take((size_t)k * p * esz);
    Q->oJs = take((size_t)k * 4);
    Q->oC = take((size_t)m * k * esz);
    Q->oG = take((size_t)k * n * esz);
    Q->oSel = take((size_t)n * 4);
    Q->total = off;
    return 0;
}

template <typename T>
static int run_rid_sample(const RsPlan& Q, const T* A, int64_t m, int64_t n, int64_t lda, const int32_t* idx, int p,
                          int32_t* J, T* Z, int64_t ldz, double* R11, int64_t ldr, T* C, int64_t ldc,
                          miid_info* info, unsigned char* w, hipStream_t s) {
    const IdPlan& P = Q.id;
    const int k = P.kmax;
    T* As = reinterpret_cast<T*>(w + Q.oAs);
    T* Zs = reinterpret_cast<T*>(w + Q.oZs);
    int32_t* Js = reinterpret_cast<int32_t*>(w + Q.oJs);
    T* Cx = C ? C : reinterpret_cast<T*>(w + Q.oC);
    const int64_t ldcx = C ? ldc : m;
    T* G = reinterpret_cast<T*>(w + Q.oG);
    int32_t* sel = reinterpret_cast<int32_t*>(w + Q.oSel);
    hipLaunchKernelGGL(k_gather_cols<T>, dim3((unsigned)std::min<int64_t>((m + 255) / 256, 64), (unsigned)p), dim3(256),
                       0, s, A, lda, m, n, idx, As);
    // the CPQR of A_S (its own column ID, no transpose): J_S, R_k (also
    // left, padded, with its diagonal-block inverses, in the CPQR's
    // workspace), C = A_S[:, J_S], info
    const int rc = run_id<T>(P, As, m, Js, Zs, k, R11, ldr, Cx, ldcx, info, w, s, false, As, m, m);
    if (rc != 0) return rc;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, s, sel, n,
                       (int32_t)-1);
    hipLaunchKernelGGL(k_map_idx, dim3(1), dim3(256), 0, s, Js, idx, k, n, J, sel);
    // C^T A, then Z = R_k^{-1} R_k^{-T} (C^T A) with Z[:, J] = I
    gemm_tn<T>(Cx, ldcx, A, lda, m, k, n, G, 1, s);
    const double* R11s = reinterpret_cast<const double*>(w + P.oR11);
    const double* Dinv = reinterpret_cast<const double*>(w + P.oDinv);
    const DevState* st = reinterpret_cast<const DevState*>(w + P.ostate);
    if (P.kpad <= 256)
        hipLaunchKernelGGL((k_trsm_blk<T, 64, true>), dim3((unsigned)((n + 63) / 64)), dim3(8 * 64),
                           (size_t)P.kpad * 65 * 8, s, G, n, R11s, P.kpad, Dinv, st, k, sel, Z, ldz, k, 0, n,
                           (int64_t)1);
    else if (P.kpad <= 512)
        hipLaunchKernelGGL((k_trsm_blk<T, 32, true>), dim3((unsigned)((n + 31) / 32)), dim3(8 * 32),
                           (size_t)P.kpad * 33 * 8, s, G, n, R11s, P.kpad, Dinv, st, k, sel, Z, ldz, k, 0, n,
                           (int64_t)1);
    else
        hipLaunchKernelGGL((k_trsm_blk<T, 16, true>), dim3((unsigned)((n + 15) / 16)), dim3(8 * 16),
                           (size_t)P.kpad * 17 * 8, s, G, n, R11s, P.kpad, Dinv, st, k, sel, Z, ldz, k, 0, n,
                           (int64_t)1);
    MIID_HIP(hipGetLastError());
    return 0;
}

// R11s (kpad x kpad, column-major) = R11 (upper triangle) padded with the
// identity
__global__ void k_pad_r11(const double* __restrict__ R11, int64_t ldr, int k, int kpad, double* __restrict__ R11s) {
    const int64_t total = (int64_t)kpad * kpad;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(e % kpad), b = (int)(e / kpad);
        R11s[e] = (a < k && b < k) ? (a <= b ? R11[a + (int64_t)b * ldr] : 0.0) : (a == b ? 1.0 : 0.0);
    }
}

size_t semi_solve_workspace(int k) {
    const size_t kpad = align_up((size_t)k, kTB);
    return align_up(kpad * kpad * 8, 256) + align_up(kpad * kTB * 8, 256) + align_up(sizeof(DevState), 256);
}

template <typename T, int JMODE>
static hipError_t semi_solve_attr() {
    {
        hipError_t e = lds_limit_once((const void*)k_trsm_blk<T, 64, true, JMODE>, 256 * 65 * 8);
        if (e == hipSuccess) e = lds_limit_once((const void*)k_trsm_blk<T, 32, true, JMODE>, 512 * 33 * 8);
        if (e == hipSuccess) e = lds_limit_once((const void*)k_trsm_blk<T, 16, true, JMODE>, 1024 * 17 * 8);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int JMODE>
static void semi_solve_launch(int kpad, const T* B, int64_t n, const double* R11s, const double* Dinv,
                              const DevState* st, int k, const int32_t* sel, T* M, int64_t ldm, int64_t rs, int64_t cs,
                              hipStream_t s) {
    if (kpad <= 256)
        hipLaunchKernelGGL((k_trsm_blk<T, 64, true, JMODE>), dim3((unsigned)((n + 63) / 64)), dim3(8 * 64),
                           (size_t)kpad * 65 * 8, s, B, n, R11s, kpad, Dinv, st, k, sel, M, ldm, k, 0, rs, cs);
    else if (kpad <= 512)
        hipLaunchKernelGGL((k_trsm_blk<T, 32, true, JMODE>), dim3((unsigned)((n + 31) / 32)), dim3(8 * 32),
                           (size_t)kpad * 33 * 8, s, B, n, R11s, kpad, Dinv, st, k, sel, M, ldm, k, 0, rs, cs);
    else
        hipLaunchKernelGGL((k_trsm_blk<T, 16, true, JMODE>), dim3((unsigned)((n + 15) / 16)), dim3(8 * 16),
                           (size_t)kpad * 17 * 8, s, B, n, R11s, kpad, Dinv, st, k, sel, M, ldm, k, 0, rs, cs);
}

template <typename T>
int semi_solve(const double* R11, int64_t ldr, int k, const T* B, int64_t rs, int64_t cs, int64_t n,
               const int32_t* sel, int jmode, T* M, int64_t ldm, unsigned char* ws, hipStream_t s) {
    const int kpad = (int)align_up((size_t)k, kTB);
    double* R11s = reinterpret_cast<double*>(ws);
    double* Dinv = reinterpret_cast<double*>(ws + align_up((size_t)kpad * kpad * 8, 256));
    DevState* st = reinterpret_cast<DevState*>(ws + align_up((size_t)kpad * kpad * 8, 256) +
                                                align_up((size_t)kpad * kTB * 8, 256));
    const hipError_t ea = jmode ? semi_solve_attr<T, 1>() : semi_solve_attr<T, 0>();
    MIID_HIP(ea);
    hipLaunchKernelGGL(k_fill<unsigned char>, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned char*>(st),
                       (int64_t)sizeof(DevState), (unsigned char)0);  // not stopped: K = k
    const int64_t total = (int64_t)kpad * kpad;
    hipLaunchKernelGGL(k_pad_r11, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 4096)), dim3(256), 0, s, R11, ldr,
                       k, kpad, R11s);
    hipLaunchKernelGGL(k_trsm_dinv, dim3((unsigned)(kpad / kTB)), dim3(kTB), 0, s, R11s, kpad, Dinv);
    if (jmode)
        semi_solve_launch<T, 1>(kpad, B, n, R11s, Dinv, st, k, sel, M, ldm, rs, cs, s);
    else
        semi_solve_launch<T, 0>(kpad, B, n, R11s, Dinv, st, k, sel, M, ldm, rs, cs, s);
    MIID_HIP(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------------------
// Least-squares coefficients over the full A for a given skeleton: Z = C^+ A,
// C = A[:, J], from the normal equations C^T C Z = C^T A (the paper forms the
// randomized ID's Z this way, Section 2.2, eq. final_eq) with R the Cholesky
// factor of C^T C (R^T R = C^T C, upper triangular, positive diagonal): the
// Gram matrix in FP64 on the matrix cores, a blocked right-looking Cholesky,
// C^T A on the matrix cores, then the FP64 two-sided triangular solve.
// ---------------------------------------------------------------------------
constexpr int kChB = 32;  // Cholesky panel width

// v of lane l (l a wave-uniform constant)
__device__ inline double readlane_f64(double v, int l) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// C64[:, c] = A[:, J[c]] in FP64 (an index outside [0, n) gives a zero column)
template <typename T>
__global__ void k_gather_f64(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n, const int32_t* __restrict__ J,
                             double* __restrict__ C64) {
    const int c = blockIdx.y;
    const int64_t src = J[c];
    const bool ok = src >= 0 && src < n;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x)
        C64[r + (int64_t)c * m] = ok ? (double)A[r + src * lda] : 0.0;
}

// R[0:k, 0:k] = 0 (leading dimension ldr; nothing outside the block is touched)
__global__ void k_zero_block(double* __restrict__ R, int64_t ldr, int k) {
    const int64_t total = (int64_t)k * k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        R[e % k + (e / k) * ldr] = 0.0;
}

// sel[J[i]] = i (sel was filled with -1)
__global__ void k_sel_of(const int32_t* __restrict__ J, int k, int64_t n, int32_t* __restrict__ sel) {
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const int32_t g = J[i];
        if (g >= 0 && g < n) sel[g] = i;
    }
}

// Panel r0 of the Cholesky of G (k x k; the upper triangle, element (i, c) at
// G[i k + c], is read and kept up to date): the 32 x 32 diagonal block is
// factored by one wave in registers, then the panel's rows of R beyond it follow by forward
// substitution with the block's transpose (one column per thread).  Columns
// from K = kinfo->k_out on (a skeleton cut short) become unit rows of R; a
// pivot that is not positive sets *flag and is replaced by 1.
__global__ void __launch_bounds__(256) k_chol_panel(const double* __restrict__ G, int k, int r0,
                                                     const miid_info* __restrict__ kinfo, double* __restrict__ R,
                                                     int64_t ldr, uint32_t* __restrict__ flag) {
    __shared__ double D[kChB][kChB + 1];
    const int K = kinfo ? min(kinfo->k_out, k) : k;
    const int nb = min(kChB, k - r0);
    const int tid = threadIdx.x;
    for (int e = tid; e < kChB * kChB; e += blockDim.x) {
        const int i = e / kChB, c = e % kChB;
        D[i][c] = (i < nb && c < nb && i <= c) ? G[(int64_t)(r0 + i) * k + (r0 + c)] : 0.0;
    }
    __syncthreads();
    if (tid < kWave) {
        // one wave factors the block in registers: lane c holds column c;
        // row j of the step's factor is read lane by lane (the lane index is
        // a constant of the unrolled loops)
        double d[kChB];
#pragma unroll
        for (int i = 0; i < kChB; ++i) d[i] = tid < kChB ? D[i][tid] : 0.0;
#pragma unroll
        for (int j = 0; j < kChB; ++j) {
            if (j < nb) {
                const double djj = readlane_f64(d[j], j);
                double piv;
                if (r0 + j >= K) {
                    piv = 0.0;  // unit row
                } else if (djj > 0.0) {
                    piv = sqrt(djj);
                } else {
                    if (tid == 0) flag[0] = 1u;
                    piv = 1.0;
                }
                if (tid > j) d[j] = piv > 0.0 ? d[j] / piv : 0.0;
                if (tid == j) d[j] = piv > 0.0 ? piv : 1.0;
#pragma unroll
                for (int i = j + 1; i < kChB; ++i) {
                    const double rji = readlane_f64(d[j], i);
                    if (i <= tid) d[i] = fma(-rji, d[j], d[i]);
                }
            }
        }
        if (tid < kChB) {
#pragma unroll
            for (int i = 0; i < kChB; ++i) D[i][tid] = d[i];
        }
    }
    __syncthreads();
    for (int e = tid; e < nb * nb; e += blockDim.x) {
        const int i = e % nb, c = e / nb;
        R[(r0 + i) + (int64_t)(r0 + c) * ldr] = i <= c ? D[i][c] : 0.0;
    }
    for (int c = r0 + nb + tid; c < k; c += blockDim.x) {
        double x[kChB];
#pragma unroll
        for (int j = 0; j < kChB; ++j) x[j] = j < nb ? G[(int64_t)(r0 + j) * k + c] : 0.0;
#pragma unroll
        for (int j = 0; j < kChB; ++j) {
            double v = x[j];
#pragma unroll
            for (int q = 0; q < j; ++q) v -= D[q][j] * x[q];
            x[j] = (j < nb && r0 + j < K) ? v / D[j][j] : 0.0;
            // keep the block's LDS reads to one row of the recursion at a
            // time (hoisting all of them would need ~1000 registers)
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int j = 0; j < kChB; ++j)
            if (j < nb) R[(r0 + j) + (int64_t)c * ldr] = x[j];
    }
}

// The trailing update after panel r0: G[i, c] -= sum_j R[r0 + j, i] R[r0 + j, c]
// for r0 + 32 <= i <= c < k; 64 x 64 tiles of the upper triangle, 4 x 4
// elements per thread, the panel's rows of R staged in LDS.
__global__ void __launch_bounds__(256) k_chol_update(double* __restrict__ G, int k, int r0, const double* __restrict__ R,
                                                     int64_t ldr) {
    const int bi = blockIdx.x, bc = blockIdx.y;
    if (bi > bc) return;  // tiles below the diagonal (uniform per workgroup)
    const int t0 = r0 + kChB;
    const int i0 = t0 + bi * 64, c0 = t0 + bc * 64;
    __shared__ double sRi[kChB][65], sRc[kChB][65];
    // both tiles' loads in flight together, then into LDS
    constexpr int kPer = kChB * 64 / 256;
    static_assert(kChB * 64 % 256 == 0, "whole passes of the tile copy");
    double ri[kPer], rc[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int e = threadIdx.x + 256 * t;
        const int j = e % kChB, x = e / kChB;
        ri[t] = load_or(R, (r0 + j) + (int64_t)(i0 + x) * ldr, i0 + x < k, 0, 0.0);
        rc[t] = load_or(R, (r0 + j) + (int64_t)(c0 + x) * ldr, c0 + x < k, 0, 0.0);
    }
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int e = threadIdx.x + 256 * t;
        sRi[e % kChB][e / kChB] = ri[t];
        sRc[e % kChB][e / kChB] = rc[t];
    }
    __syncthreads();
    const int ti = (threadIdx.x % 16) * 4, tc = (threadIdx.x / 16) * 4;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
#pragma unroll 4
    for (int j = 0; j < kChB; ++j) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = sRi[j][ti + u];
            b[u] = sRc[j][tc + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    // the sixteen G loads together, then the stores
    double g[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + ti + u, c = c0 + tc + v;
            g[u][v] = load_or(G, (int64_t)i * k + c, i < k && c < k && i <= c, 0, 0.0);
        }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + ti + u, c = c0 + tc + v;
            if (i < k && c < k && i <= c) G[(int64_t)i * k + c] = g[u][v] - acc[u][v];
        }
}

// out[e] = sum over z of part[z count + e], z in order
__global__ void k_sum_parts(const double* __restrict__ part, int nz, int64_t count, double* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int z = 0; z < nz; ++z) v += part[(int64_t)z * count + e];
        out[e] = v;
    }
}

int ls_plan(int64_t m, int64_t n, int k, size_t esz, LsPlan* L) {
    if (m < 1 || n < 1 || k < 1 || k > m || k > n || k > 1024) return MIID_E_UNSUPPORTED;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    // the Gram's split over rows: about 512 workgroups, slices of >= 64 rows
    const int64_t tiles = (int64_t)((k + 127) / 128) * ((k + 127) / 128);
    L->gz = (int)std::max<int64_t>(1, std::min<int64_t>(512 / tiles, m / 64));
    {
        const int64_t mz = L->gz > 1 ? (int64_t)align_up((size_t)((m + L->gz - 1) / L->gz), 16) : m;
        L->gzr = (int)((m + mz - 1) / mz);  // slices actually launched
    }
    L->oC64 = take((size_t)m * k * 8);
    L->oGram = take((size_t)k * k * 8);
    L->oGp = take(L->gz > 1 ? (size_t)L->gzr * k * k * 8 : 8);
    L->oR = take((size_t)k * k * 8);
    L->oCT = take((size_t)m * k * esz);
    L->oB = take((size_t)k * n * esz);
    L->oSel = take((size_t)n * 4);
    L->oFlag = take(4);
    L->oSemi = take(semi_solve_workspace(k));
    L->total = off;
    return 0;
}

template <typename T>
int run_lstsq(const LsPlan& L, const T* A, int64_t m, int64_t n, int64_t lda, const int32_t* J, int k,
              const miid_info* kinfo, T* Z, int64_t ldz, double* R11, int64_t ldr, unsigned char* w, hipStream_t s) {
    double* C64 = reinterpret_cast<double*>(w + L.oC64);
    double* Gram = reinterpret_cast<double*>(w + L.oGram);
    double* R = R11 ? R11 : reinterpret_cast<double*>(w + L.oR);
    const int64_t ldR = R11 ? ldr : k;
    T* B = reinterpret_cast<T*>(w + L.oB);
    int32_t* sel = reinterpret_cast<int32_t*>(w + L.oSel);
    uint32_t* flag = reinterpret_cast<uint32_t*>(w + L.oFlag);
    // C gathered here, not taken from the caller: its columns beyond a
    // skeleton cut short (J = -1) must be zero so that Z's rows there are
    const dim3 ggrid((unsigned)std::min<int64_t>((m + 255) / 256, 64), (unsigned)k);
    T* CT = reinterpret_cast<T*>(w + L.oCT);
    hipLaunchKernelGGL(k_gather_cols<T>, ggrid, dim3(256), 0, s, A, lda, m, n, J, CT);
    hipLaunchKernelGGL(k_gather_f64<T>, ggrid, dim3(256), 0, s, A, lda, m, n, J, C64);
    // C^T C (symmetric: row- and column-major alike), split over the rows
    // into L.gz partial products summed in a fixed order
    double* Gp = reinterpret_cast<double*>(w + L.oGp);
    gemm_tn<double>(C64, m, C64, m, m, k, (int64_t)k, L.gz > 1 ? Gp : Gram, L.gz, s);
    if (L.gz > 1) {
        const int64_t kk = (int64_t)k * k;
        hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)std::min<int64_t>((kk + 255) / 256, 4096)), dim3(256), 0, s, Gp,
                           L.gzr, kk, Gram);
    }
    hipLaunchKernelGGL(k_zero_block, dim3((unsigned)std::min<int64_t>(((int64_t)k * k + 255) / 256, 4096)), dim3(256), 0,
                       s, R, ldR, k);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(64), 0, s, flag, (int64_t)1, 0u);
    for (int r0 = 0; r0 < k; r0 += kChB) {
        hipLaunchKernelGGL(k_chol_panel, dim3(1), dim3(256), 0, s, Gram, k, r0, kinfo, R, ldR, flag);
        const int rest = k - r0 - kChB;
        if (rest > 0) {
            const unsigned nt = (unsigned)((rest + 63) / 64);
            hipLaunchKernelGGL(k_chol_update, dim3(nt, nt), dim3(256), 0, s, Gram, k, r0, R, ldR);
        }
    }
    // C^T A (k x n, row-major), then Z = R^{-1} R^{-T} C^T A with Z[:, J] = I
    gemm_tn<T>(CT, m, A, lda, m, k, n, B, 1, s);
    hipLaunchKernelGGL(k_fill<int32_t>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, s, sel, n,
                       (int32_t)-1);
    hipLaunchKernelGGL(k_sel_of, dim3(1), dim3(256), 0, s, J, k, n, sel);
    MIID_HIP(hipGetLastError());
    return semi_solve<T>(R, ldR, k, B, n, (int64_t)1, n, sel, 0, Z, ldz, w + L.oSemi, s);
}

template int run_lstsq<float>(const LsPlan&, const float*, int64_t, int64_t, int64_t, const int32_t*, int,
                              const miid_info*, float*, int64_t, double*, int64_t, unsigned char*, hipStream_t);
template int run_lstsq<double>(const LsPlan&, const double*, int64_t, int64_t, int64_t, const int32_t*, int,
                               const miid_info*, double*, int64_t, double*, int64_t, unsigned char*, hipStream_t);

template int semi_solve<float>(const double*, int64_t, int, const float*, int64_t, int64_t, int64_t, const int32_t*,
                               int, float*, int64_t, unsigned char*, hipStream_t);
template int semi_solve<double>(const double*, int64_t, int, const double*, int64_t, int64_t, int64_t,
                                const int32_t*, int, double*, int64_t, unsigned char*, hipStream_t);

template int run_id<float>(const IdPlan&, const float*, int64_t, int32_t*, float*, int64_t, double*, int64_t, float*,
                           int64_t, miid_info*, unsigned char*, hipStream_t, bool, const float*, int64_t, int64_t);
template int run_id<double>(const IdPlan&, const double*, int64_t, int32_t*, double*, int64_t, double*, int64_t,
                            double*, int64_t, miid_info*, unsigned char*, hipStream_t, bool, const double*, int64_t,
                            int64_t);

}  // namespace miid

using namespace miid;

extern "C" {

static size_t rid_sample_workspace_body(int64_t m, int64_t n, int32_t p, miid_dtype dtype, const miid_opts* opts) {
    RsPlan Q;
    if (m < 1 || n < 1 || rs_plan(m, n, p, dtype, opts, &Q) != 0) return 0;
    return Q.total;
}

static int rid_sample_body(const void* A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype, const int32_t* idx, int32_t p,
                    const miid_opts* opts, int32_t* J, void* Z, int64_t ldz, double* R11, int64_t ldr, void* C,
                    int64_t ldc, miid_info* info, void* ws, size_t ws_bytes, void* stream) {
    if (!A) return -1;
    if (m < 1) return -2;
    if (n < 1) return -3;
    if (lda < m) return -4;
    if (dtype != MIID_F32 && dtype != MIID_F64) return -5;
    if (!idx) return -6;
    RsPlan Q;
    const int rc = rs_plan(m, n, p, dtype, opts, &Q);
    if (rc != 0) return rc;
    const int k = Q.id.kmax;
    if (!J) return -9;
    if (!Z) return -10;
    if (ldz < k) return -11;
    if (R11 && ldr < k) return -13;
    if (C && ldc < m) return -15;
    if (!info) return -16;
    if (!ws) return -17;
    if (ws_bytes < Q.total) return MIID_E_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    if (dtype == MIID_F64)
        return run_rid_sample<double>(Q, (const double*)A, m, n, lda, idx, p, J, (double*)Z, ldz, R11, ldr, (double*)C,
                                      ldc, info, w, s);
    return run_rid_sample<float>(Q, (const float*)A, m, n, lda, idx, p, J, (float*)Z, ldz, R11, ldr, (float*)C, ldc,
                                 info, w, s);
}

static size_t id_workspace_body(int64_t m, int64_t n, miid_dtype dtype, const miid_opts* opts) {
    IdPlan P;
    if (make_plan(m, n, dtype, opts, &P) != 0) return 0;
    return P.total;
}

static int id_cpqr_body(const void* A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype, const miid_opts* opts, int32_t* J,
            void* Z, int64_t ldz, double* R11, int64_t ldr, void* C, int64_t ldc, miid_info* info, void* ws,
            size_t ws_bytes, void* stream) {
    if (!A) return -1;
    IdPlan P;
    const int rc = make_plan(m, n, dtype, opts, &P);
    if (rc != 0) return rc;
    if (lda < m) return -4;
    if (!J) return -7;
    if (!Z) return -8;
    if (ldz < P.kmax) return -9;
    if (R11 && ldr < P.kmax) return -11;
    if (C && ldc < P.m) return -13;
    if (!info) return -14;
    if (!ws) return -15;
    if (ws_bytes < P.total) return MIID_E_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    if (dtype == MIID_F64)
        return run_id<double>(P, (const double*)A, lda, J, (double*)Z, ldz, R11, ldr, (double*)C, ldc, info, w, s, false,
                              (const double*)A, lda, P.m);
    return run_id<float>(P, (const float*)A, lda, J, (float*)Z, ldz, R11, ldr, (float*)C, ldc, info, w, s, false,
                         (const float*)A, lda, P.m);
}

// ---- entry points: the handle resolved, then the bodies above -----------
size_t miid_rid_sample_workspace(miid_handle h, int64_t m, int64_t n, int32_t p, miid_dtype dtype,
                                 const miid_opts* opts) {
    miid_opts o;
    if (resolve_opts(h, kTuneRidSample, dtype, m, n, opts ? opts->k : 0, opts, &o) != 0) return 0;
    return rid_sample_workspace_body(m, n, p, dtype, opts ? &o : nullptr);
}

int rid_sample_cpqr(miid_handle h, const void* A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype,
                    const int32_t* idx, int32_t p, const miid_opts* opts, int32_t* J, void* Z, int64_t ldz,
                    double* R11, int64_t ldr, void* C, int64_t ldc, miid_info* info, void* ws, size_t ws_bytes,
                    void* stream) {
    miid_opts o;
    if (resolve_opts(h, kTuneRidSample, dtype, m, n, opts ? opts->k : 0, opts, &o) != 0) return -1;
    return shift_arg(rid_sample_body(A, m, n, lda, dtype, idx, p, opts ? &o : nullptr, J, Z, ldz, R11, ldr, C, ldc,
                                     info, ws, ws_bytes, stream));
}

size_t miid_id_workspace(miid_handle h, int64_t m, int64_t n, miid_dtype dtype, const miid_opts* opts) {
    miid_opts o;
    if (resolve_opts(h, kTuneId, dtype, m, n, opts ? opts->k : 0, opts, &o) != 0) return 0;
    return id_workspace_body(m, n, dtype, opts ? &o : nullptr);
}

int id_cpqr(miid_handle h, const void* A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype, const miid_opts* opts,
            int32_t* J, void* Z, int64_t ldz, double* R11, int64_t ldr, void* C, int64_t ldc, miid_info* info,
            void* ws, size_t ws_bytes, void* stream) {
    miid_opts o;
    if (resolve_opts(h, kTuneId, dtype, m, n, opts ? opts->k : 0, opts, &o) != 0) return -1;
    return shift_arg(id_cpqr_body(A, m, n, lda, dtype, opts ? &o : nullptr, J, Z, ldz, R11, ldr, C, ldc, info, ws,
                                  ws_bytes, stream));
}

}  // extern "C"
