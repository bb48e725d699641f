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
#include <cstring>

#include "common.hpp"
#include "prof.hpp"

namespace miid {

constexpr int kThreads = 256;
constexpr int kColsPerWave = 4;
constexpr int kColsPerWG = 16;     // 4 waves x 4 columns
constexpr int kRowsPerChunk = 256; // rows per workgroup of the pivot-column kernel
constexpr int kMaxNb = 64;
constexpr int kPartAStride = kMaxNb + 1;
constexpr int kMaxK = 1024;
constexpr size_t kMaxVecLds = 131072;  // bytes of LDS for the reflector in the GEMV

static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// a1: staging.  S (ldw x n, padded rows zero) <- A, or A^T for the dual ID.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads) k_stage_copy(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                         T* __restrict__ S, int64_t ldw) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int c = 0; c < kColsPerWave; ++c) {
        const int64_t col = (int64_t)blockIdx.x * kColsPerWG + wave * kColsPerWave + c;
        if (col >= n) break;
        const T* a = A + col * lda;
        T* s = S + col * ldw;
        for (int64_t r = lane; r < ldw; r += kWave) s[r] = r < m ? a[r] : T(0);
    }
}

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
template <typename T>
__global__ void __launch_bounds__(kThreads) k_norms(const T* __restrict__ S, int64_t ldw, int64_t n,
                                                    double* __restrict__ nu, double* __restrict__ nuref,
                                                    int32_t* __restrict__ sel, ColPartial* __restrict__ part,
                                                    int32_t* __restrict__ recomp) {
    __shared__ double s_best[4], s_sum[4];
    __shared__ int32_t s_idx[4], s_nf[4];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    ArgMax best{-1.0, INT32_MAX};
    double sum = 0.0;
    int nf = 0;
    for (int c = 0; c < kColsPerWave; ++c) {
        const int64_t col = (int64_t)blockIdx.x * kColsPerWG + wave * kColsPerWave + c;
        if (col >= n) break;
        const T* s = S + col * ldw;
        double acc = 0.0;
        for (int64_t r = lane; r < ldw; r += kWave) {
            const double x = (double)s[r];
            acc += x * x;
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

// Reduce the per-workgroup column partials (identical result in every
// workgroup: fixed order, no atomics).  Returns best (value, index), the sum
// of squares, and the non-finite flag through shared memory.
__device__ void reduce_partials(const ColPartial* __restrict__ part, int npart, ArgMax* out_best, double* out_sum,
                                int* out_nf) {
    __shared__ double r_best[kThreads], r_sum[kThreads];
    __shared__ int32_t r_idx[kThreads], r_nf[kThreads];
    const int t = threadIdx.x;
    ArgMax b{-1.0, INT32_MAX};
    double s = 0.0;
    int nf = 0;
    for (int q = t; q < npart; q += kThreads) {
        const ColPartial cp = part[q];
        if (argmax_better(cp.best, cp.idx, b.v, b.i)) b = {cp.best, cp.idx};
        s += cp.sumsq;
        nf |= cp.nonfinite;
    }
    r_best[t] = b.v;
    r_idx[t] = b.i;
    r_sum[t] = s;
    r_nf[t] = nf;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            if (argmax_better(r_best[t + h], r_idx[t + h], r_best[t], r_idx[t])) {
                r_best[t] = r_best[t + h];
                r_idx[t] = r_idx[t + h];
            }
            r_sum[t] += r_sum[t + h];
            r_nf[t] |= r_nf[t + h];
        }
        __syncthreads();
    }
    *out_best = ArgMax{r_best[0], r_idx[0]};
    *out_sum = r_sum[0];
    *out_nf = r_nf[0];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// a2 + a3 + first half of a4: pivot search, lazy update of the pivot column,
// partial sums for the reflector.  One thread per row, 256 rows per workgroup.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads) k_pivot_col(const T* __restrict__ S, int64_t ldw, int64_t m,
                                                        const T* __restrict__ V, const T* __restrict__ F, int nb,
                                                        T* __restrict__ u, const ColPartial* __restrict__ part,
                                                        int npart, double* __restrict__ partA,
                                                        DevState* __restrict__ st, int32_t* __restrict__ J, int j,
                                                        int i, int tol_mode, double eps) {
    __shared__ double s_F[kMaxNb];
    __shared__ double s_red[4][kPartAStride];
    if (st->stop) return;
    ArgMax best;
    double sumsq;
    int nf;
    reduce_partials(part, npart, &best, &sumsq, &nf);
    const double a_norm = (j == 0) ? sqrt(sumsq) : st->a_norm;
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
    if (blockIdx.x == 0 && threadIdx.x == 0) {
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
    if (threadIdx.x < i) s_F[threadIdx.x] = (double)F[p * nb + threadIdx.x];
    __syncthreads();

    const int64_t r = (int64_t)blockIdx.x * kRowsPerChunk + threadIdx.x;
    const bool active = r >= j && r < m;
    double vr[kMaxNb];
    double ur = 0.0;
    if (active) {
        ur = (double)S[r + p * ldw];
#pragma unroll
        for (int q = 0; q < kMaxNb; ++q) {
            if (q < i) {
                vr[q] = (double)V[r + q * ldw];
                ur -= vr[q] * s_F[q];
            } else {
                vr[q] = 0.0;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < kMaxNb; ++q) vr[q] = 0.0;
    }
    const T ut = (T)ur;
    if (r < ldw) u[r] = active ? ut : T(0);
    const double w = (active && r > j) ? (double)ut : 0.0;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    double s0 = wave_sum(w * w);
    if (lane == 0) s_red[wave][0] = s0;
#pragma unroll
    for (int q = 0; q < kMaxNb; ++q) {
        if (q < i) {
            const double pq = wave_sum(vr[q] * w);
            if (lane == 0) s_red[wave][1 + q] = pq;
        }
    }
    __syncthreads();
    if (threadIdx.x <= i) {
        const int t = threadIdx.x;
        partA[(int64_t)blockIdx.x * kPartAStride + t] = s_red[0][t] + s_red[1][t] + s_red[2][t] + s_red[3][t];
    }
}

// ---------------------------------------------------------------------------
// second half of a4 + a5 + a6 (+ a8 when flagged): reflector, F-GEMV over the
// stale trailing matrix, row j of R, norm downdate / exact recompute, argmax
// partials.  4 columns per wave, 16 per workgroup; the reflector v lives in
// LDS (rows j0..ldw).
// ---------------------------------------------------------------------------
template <typename T>
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
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* v = reinterpret_cast<T*>(smem_raw);
    __shared__ double s_red[kPartAStride];
    __shared__ double s_y[kMaxNb], s_vj[kMaxNb + 1];
    __shared__ double s_best[4], s_sum[4];
    __shared__ int32_t s_idx[4], s_nrec[4];

    if (st->stop) return;
    const int tid = threadIdx.x;
    const int64_t p = J[j];
    if (tid <= i) {
        double acc = 0.0;
        for (int c = 0; c < NA; ++c) acc += partA[(int64_t)c * kPartAStride + tid];
        s_red[tid] = acc;
    }
    __syncthreads();
    const double u0 = (double)u[j];
    const double alpha = sqrt(u0 * u0 + s_red[0]);
    if (!(alpha > 0.0)) {
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
        const double vjq = (double)V[j + (int64_t)tid * ldw];
        s_vj[tid] = vjq;
        s_y[tid] = vjq + scale * s_red[1 + tid];
    }
    const int64_t j0 = (int64_t)j & ~(int64_t)(VEC - 1);
    for (int64_t r = j0 + tid; r < ldw; r += kThreads) {
        const T x = r < j ? T(0) : (r == j ? T(1) : (r < m ? (T)((double)u[r] * scale) : T(0)));
        v[r - j0] = x;
    }
    if (blockIdx.x == 0) {
        for (int64_t r = tid; r < ldw; r += kThreads) {
            const T x = r < j ? T(0) : (r == j ? T(1) : (r < m ? (T)((double)u[r] * scale) : T(0)));
            V[r + (int64_t)i * ldw] = x;
        }
        if (tid == 0) {
            R[(int64_t)j * n + p] = (T)beta;
            sel[p] = j;
        }
    }
    if (tid == 0 && p / kColsPerWG == blockIdx.x) nu[p] = -1.0;
    __syncthreads();

    const int wave = tid / kWave, lane = tid % kWave;
    const int64_t col0 = (int64_t)blockIdx.x * kColsPerWG + wave * kColsPerWave;
    bool alive[kColsPerWave];
    double acc[kColsPerWave];
#pragma unroll
    for (int c = 0; c < kColsPerWave; ++c) {
        const int64_t col = col0 + c;
        alive[c] = col < n && col != p && nu[col] >= 0.0;
        acc[c] = 0.0;
    }
    const int64_t ngroups = (ldw - j0) / VEC;
    for (int64_t g = lane; g < ngroups; g += kWave) {
        const VT vv = *reinterpret_cast<const VT*>(v + g * VEC);
#pragma unroll
        for (int c = 0; c < kColsPerWave; ++c) {
            if (alive[c]) {
                const VT sv = *reinterpret_cast<const VT*>(S + (col0 + c) * ldw + j0 + g * VEC);
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[c] += (double)get(sv, e) * (double)get(vv, e);
            }
        }
    }

    ArgMax best{-1.0, INT32_MAX};
    double sumsq = 0.0;
    int nrec = 0;
#pragma unroll
    for (int c = 0; c < kColsPerWave; ++c) {
        if (!alive[c]) continue;
        const int64_t col = col0 + c;
        const double dot = wave_sum(acc[c]);
        const double fq = lane < i ? (double)F[col * nb + lane] : 0.0;
        const double t1 = wave_sum(lane < i ? fq * s_y[lane] : 0.0);
        const double t2 = wave_sum(lane < i ? fq * s_vj[lane] : 0.0);
        const T fT = (T)(tau * (dot - t1));
        const double f = (double)fT;
        const double rjl = (double)S[col * ldw + j] - t2 - f;
        if (lane == 0) {
            F[col * nb + i] = fT;
            R[(int64_t)j * n + col] = (T)rjl;
        }
        const double nuc = nu[col];
        double nnew = nuc;
        bool rec = false;
        if (nuc > 0.0) {
            double t = fabs(rjl) / nuc;
            t = fmax(0.0, (1.0 - t) * (1.0 + t));
            const double ratio = nuc / nuref[col];
            if (t * ratio * ratio <= tol)
                rec = true;
            else
                nnew = nuc * sqrt(t);
        }
        if (rec) {
            double ss = 0.0;
            for (int64_t r = j + 1 + lane; r < m; r += kWave) {
                double x = (double)S[col * ldw + r] - (double)v[r - j0] * f;
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
        ArgMax b{s_best[0], s_idx[0]};
        double t = s_sum[0];
        int nr = s_nrec[0];
        for (int w = 1; w < 4; ++w) {
            if (argmax_better(s_best[w], s_idx[w], b.v, b.i)) b = {s_best[w], s_idx[w]};
            t += s_sum[w];
            nr += s_nrec[w];
        }
        part[blockIdx.x] = ColPartial{b.v, b.i, 0, t, 0.0};
        recomp[blockIdx.x] += nr;
    }
}

// ---------------------------------------------------------------------------
// a7: trailing update at the end of a panel, S[r0:, :] -= V[r0:, 0:w] F[:, 0:w]^T.
// 64 x 64 tiles; each thread owns one row and 16 columns.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads) k_trail(T* __restrict__ S, int64_t ldw, int64_t n,
                                                    const T* __restrict__ V, const T* __restrict__ F, int nb, int w,
                                                    int64_t r0, const DevState* __restrict__ st) {
    __shared__ T sV[64][kMaxNb + 1];
    __shared__ T sF[kMaxNb][64];
    if (st->stop) return;
    const int64_t rbase = (r0 & ~(int64_t)63) + (int64_t)blockIdx.x * 64;
    const int64_t cbase = (int64_t)blockIdx.y * 64;
    const int tid = threadIdx.x;
    for (int e = tid; e < 64 * w; e += kThreads) {
        const int rr = e % 64, q = e / 64;
        sV[rr][q] = V[rbase + rr + (int64_t)q * ldw];
    }
    for (int e = tid; e < 64 * w; e += kThreads) {
        const int q = e % w, cc = e / w;
        const int64_t col = cbase + cc;
        sF[q][cc] = col < n ? F[col * nb + q] : T(0);
    }
    __syncthreads();
    const int rr = tid % 64, cg = tid / 64;
    const int64_t row = rbase + rr;
    if (row < r0 || row >= ldw) return;
    double acc[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t col = cbase + cg * 16 + e;
        acc[e] = col < n ? (double)S[row + col * ldw] : 0.0;
    }
    for (int q = 0; q < w; ++q) {
        const double vq = (double)sV[rr][q];
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] -= vq * (double)sF[q][cg * 16 + e];
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t col = cbase + cg * 16 + e;
        if (col < n) S[row + col * ldw] = (T)acc[e];
    }
}

// ---------------------------------------------------------------------------
// a9: R11 (FP64, pivot order) gathered from the rows of R.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_gather_r11(const T* __restrict__ R, int64_t n, const int32_t* __restrict__ J, int kmax,
                             const DevState* __restrict__ st, int ksteps, double* __restrict__ R11s,
                             double* __restrict__ R11out, int64_t ldr) {
    const int kout = st->stop ? st->k_out : ksteps;
    const int64_t total = (int64_t)kmax * kmax;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(e % kmax), b = (int)(e / kmax);
        double val;
        if (a < kout && b < kout)
            val = a <= b ? (double)R[(int64_t)a * n + J[b]] : 0.0;
        else
            val = a == b ? 1.0 : 0.0;
        R11s[e] = val;
        if (R11out) R11out[a + (int64_t)b * ldr] = (a < kout && b < kout) ? val : 0.0;
    }
}

// Right-looking back substitution of R11 x = b for NCOL columns held in LDS
// (work[k][NCOL]); thread (g, c) owns column c and rows q = g (mod G).
template <int NCOL>
__device__ void lds_backsolve(double* work, const double* __restrict__ R11s, int kmax, int K) {
    constexpr int G = kThreads / NCOL;
    const int c = threadIdx.x % NCOL, g = threadIdx.x / NCOL;
    for (int i = K - 1; i >= 0; --i) {
        if (g == i % G) work[i * NCOL + c] /= R11s[i + (int64_t)i * kmax];
        __syncthreads();
        const double zi = work[i * NCOL + c];
        const double* col = R11s + (int64_t)i * kmax;
        for (int q = g; q < i; q += G) work[q * NCOL + c] -= col[q] * zi;
    }
    __syncthreads();
}

// Z[:, cols] = R11^{-1} R[:, cols] in FP64 with one refinement step;
// Z[:, J[c]] = e_c exactly; rows >= k_out are zero.
template <typename T, int NCOL>
__global__ void __launch_bounds__(kThreads) k_trsm(const T* __restrict__ R, int64_t n,
                                                   const double* __restrict__ R11s, int kmax,
                                                   const DevState* __restrict__ st, int ksteps,
                                                   const int32_t* __restrict__ sel, T* __restrict__ Z, int64_t ldz,
                                                   int refine) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* z = reinterpret_cast<double*>(smem_raw);  // [kmax][NCOL]
    double* work = z + (int64_t)kmax * NCOL;          // [kmax][NCOL]
    constexpr int G = kThreads / NCOL;
    const int K = st->stop ? st->k_out : ksteps;
    const int64_t c0 = (int64_t)blockIdx.x * NCOL;
    const int c = threadIdx.x % NCOL, g = threadIdx.x / NCOL;
    const int64_t col = c0 + c;
    for (int q = g; q < K; q += G) work[q * NCOL + c] = col < n ? (double)R[(int64_t)q * n + col] : 0.0;
    __syncthreads();
    lds_backsolve<NCOL>(work, R11s, kmax, K);
    for (int q = g; q < K; q += G) z[q * NCOL + c] = work[q * NCOL + c];
    if (refine) {
        __syncthreads();
        for (int q = g; q < K; q += G) {
            double e = col < n ? (double)R[(int64_t)q * n + col] : 0.0;
            for (int t = q; t < K; ++t) e -= R11s[q + (int64_t)t * kmax] * z[t * NCOL + c];
            work[q * NCOL + c] = e;
        }
        __syncthreads();
        lds_backsolve<NCOL>(work, R11s, kmax, K);
        for (int q = g; q < K; q += G) z[q * NCOL + c] += work[q * NCOL + c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kmax * NCOL; e += kThreads) {
        const int q = e % kmax, cc = e / kmax;
        const int64_t cl = c0 + cc;
        if (cl >= n) continue;
        const int s = sel[cl];
        double val;
        if (s >= 0 && s < K)
            val = (q == s) ? 1.0 : 0.0;
        else
            val = q < K ? z[q * NCOL + cc] : 0.0;
        Z[q + cl * ldz] = (T)val;
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

__global__ void k_finalize(const DevState* __restrict__ st, const ColPartial* __restrict__ part, int npart,
                           const int32_t* __restrict__ recomp, int32_t* __restrict__ J, int kmax, int ksteps,
                           int tol_mode, double eps, int trans, miid_info* __restrict__ info) {
    __shared__ double s_sum[kThreads];
    __shared__ int32_t s_rec[kThreads];
    const int t = threadIdx.x;
    double s = 0.0;
    int rc = 0;
    for (int q = t; q < npart; q += kThreads) {
        s += part[q].sumsq;
        rc += recomp[q];
    }
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
struct IdPlan {
    int64_t M, N;  // caller's shape
    int64_t m, n;  // working shape, m <= n
    bool trans;
    int64_t ldw;
    int kmax, nb;
    bool tol;
    double eps;
    bool refine;
    size_t esz;
    int npart, NA;
    size_t oS, oV, oF, ou, onu, onuref, oR, osel, opart, opartA, oR11, ostate, orec, total;
};

static int make_plan(int64_t M, int64_t N, miid_dtype dtype, const miid_opts* o, IdPlan* P) {
    if (M < 1) return -2;
    if (N < 1) return -3;
    if (dtype != MIID_F32 && dtype != MIID_F64) return -5;
    if (!o || o->k < 0 || (o->k == 0 && (o->kmax < 1 || !(o->eps >= 0.0))) || o->nb < 0) return -6;
    P->M = M;
    P->N = N;
    P->trans = M > N;
    P->m = P->trans ? N : M;
    P->n = P->trans ? M : N;
    P->tol = o->k == 0;
    P->kmax = P->tol ? o->kmax : o->k;
    P->eps = o->eps;
    P->nb = o->nb == 0 ? 32 : o->nb;
    P->refine = !(o->flags & MIID_NO_REFINE);
    if (P->nb > kMaxNb || P->kmax > P->m || P->kmax > kMaxK) return MIID_E_UNSUPPORTED;
    P->esz = dtype == MIID_F64 ? 8 : 4;
    P->ldw = (int64_t)align_up((size_t)P->m, 64);
    if ((size_t)P->ldw * P->esz > kMaxVecLds) return MIID_E_UNSUPPORTED;
    P->npart = (int)((P->n + kColsPerWG - 1) / kColsPerWG);
    P->NA = (int)((P->ldw + kRowsPerChunk - 1) / kRowsPerChunk);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o2 = off;
        off = align_up(off + bytes, 256);
        return o2;
    };
    P->oS = take((size_t)P->ldw * P->n * P->esz);
    P->oV = take((size_t)P->ldw * P->nb * P->esz);
    P->oF = take((size_t)P->n * P->nb * P->esz);
    P->ou = take((size_t)P->ldw * P->esz);
    P->onu = take((size_t)P->n * 8);
    P->onuref = take((size_t)P->n * 8);
    P->oR = take((size_t)P->kmax * P->n * P->esz);
    P->osel = take((size_t)P->n * 4);
    P->opart = take((size_t)P->npart * sizeof(ColPartial));
    P->opartA = take((size_t)P->NA * kPartAStride * 8);
    P->oR11 = take((size_t)P->kmax * P->kmax * 8);
    P->ostate = take(sizeof(DevState));
    P->orec = take((size_t)P->npart * 4);
    P->total = off;
    return 0;
}

template <typename T>
static int run_id(const IdPlan& P, const T* A, int64_t lda, int32_t* J, T* Z, int64_t ldz, double* R11out,
                  int64_t ldr, T* C, int64_t ldc, miid_info* info, unsigned char* ws, hipStream_t stream) {
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

    static bool attr_done = false;
    if (!attr_done) {
        // dynamic LDS above 64 KB: the reflector (k_gemv) and the solve tiles (k_trsm)
        MIID_HIP(hipFuncSetAttribute((const void*)k_gemv<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxVecLds));
        MIID_HIP(hipFuncSetAttribute((const void*)k_trsm<T, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
        MIID_HIP(hipFuncSetAttribute((const void*)k_trsm<T, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
        attr_done = true;
    }

    // control block, R rows
    hipLaunchKernelGGL(k_fill<unsigned char>, dim3(1), dim3(64), 0, stream, reinterpret_cast<unsigned char*>(st),
                       (int64_t)sizeof(DevState), (unsigned char)0);
    {
        const int64_t cnt = (int64_t)P.kmax * n;
        const int blocks = (int)std::min<int64_t>((cnt + 255) / 256, 8192);
        hipLaunchKernelGGL(k_fill<T>, dim3(blocks), dim3(256), 0, stream, R, cnt, T(0));
    }
    // a1: stage + norms
    if (P.trans) {
        dim3 grid((unsigned)((ldw + 63) / 64), (unsigned)((n + 63) / 64));
        hipLaunchKernelGGL(k_stage_transpose<T>, grid, dim3(kThreads), 0, stream, A, lda, m, n, S, ldw);
    } else {
        hipLaunchKernelGGL(k_stage_copy<T>, dim3(P.npart), dim3(kThreads), 0, stream, A, lda, m, n, S, ldw);
    }
    hipLaunchKernelGGL(k_norms<T>, dim3(P.npart), dim3(kThreads), 0, stream, S, ldw, n, nu, nuref, sel, part, recomp);

    const double tol = sizeof(T) == 8 ? sqrt(2.220446049250313e-16) : sqrt(1.1920928955078125e-07);
    int ksteps = P.kmax;
    int32_t host_stop = 0;
    for (int j = 0; j < P.kmax; ++j) {
        const int jb = (j / nb) * nb;
        const int i = j - jb;
        int pr = prof_open(MIID_K_PIVOT, j, m - j, 1, stream);
        hipLaunchKernelGGL(k_pivot_col<T>, dim3(P.NA), dim3(kThreads), 0, stream, S, ldw, m, V, F, nb, u, part,
                           P.npart, partA, st, J, j, i, (int)P.tol, P.eps);
        prof_close(pr, stream);
        const int64_t j0 = (int64_t)j & ~(int64_t)(Vec16<T>::n - 1);
        const size_t lds = (size_t)(ldw - j0) * sizeof(T);
        pr = prof_open(MIID_K_GEMV, j, m - j, n - j, stream);
        hipLaunchKernelGGL(k_gemv<T>, dim3(P.npart), dim3(kThreads), lds, stream, S, ldw, m, n, V, F, nb, u, partA,
                           P.NA, st, J, R, nu, nuref, sel, part, recomp, j, i, tol);
        prof_close(pr, stream);
        const bool panel_end = (i == nb - 1);
        if (panel_end && j + 1 < P.kmax) {
            const int64_t r0 = j + 1;
            const int64_t rbase = r0 & ~(int64_t)63;
            dim3 grid((unsigned)((ldw - rbase + 63) / 64), (unsigned)((n + 63) / 64));
            pr = prof_open(MIID_K_TRAIL, j / nb, m - r0, n, stream);
            hipLaunchKernelGGL(k_trail<T>, grid, dim3(kThreads), 0, stream, S, ldw, n, V, F, nb, nb, r0, st);
            prof_close(pr, stream);
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
    MIID_HIP(hipGetLastError());
    // a9: triangular solve
    {
        const int64_t total = (int64_t)P.kmax * P.kmax;
        const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
        hipLaunchKernelGGL(k_gather_r11<T>, dim3(blocks), dim3(256), 0, stream, R, n, J, P.kmax, st, ksteps, R11s,
                           R11out, ldr);
        const int pr = prof_open(MIID_K_TRSM, 0, P.kmax, n, stream);
        if (P.kmax <= 512) {
            const size_t lds = (size_t)2 * P.kmax * 16 * 8;
            hipLaunchKernelGGL((k_trsm<T, 16>), dim3((unsigned)((n + 15) / 16)), dim3(kThreads), lds, stream, R, n,
                               R11s, P.kmax, st, ksteps, sel, Z, ldz, (int)P.refine);
        } else {
            const size_t lds = (size_t)2 * P.kmax * 8 * 8;
            hipLaunchKernelGGL((k_trsm<T, 8>), dim3((unsigned)((n + 7) / 8)), dim3(kThreads), lds, stream, R, n, R11s,
                               P.kmax, st, ksteps, sel, Z, ldz, (int)P.refine);
        }
        prof_close(pr, stream);
    }
    // a10: C, info
    if (C) {
        dim3 grid((unsigned)std::min<int64_t>((m + 255) / 256, 64), (unsigned)P.kmax);
        hipLaunchKernelGGL(k_gather_c<T>, grid, dim3(256), 0, stream, A, lda, (int)P.trans, m, J, st, ksteps, C, ldc);
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, stream, st, part, P.npart, recomp, J, P.kmax, ksteps,
                       (int)P.tol, P.eps, (int)P.trans, info);
    MIID_HIP(hipGetLastError());
    return 0;
}

}  // namespace miid

using namespace miid;

extern "C" {

size_t miid_id_workspace(int64_t m, int64_t n, miid_dtype dtype, const miid_opts* opts) {
    IdPlan P;
    if (make_plan(m, n, dtype, opts, &P) != 0) return 0;
    return P.total;
}

int id_cpqr(const void* A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype, const miid_opts* opts, int32_t* J,
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
        return run_id<double>(P, (const double*)A, lda, J, (double*)Z, ldz, R11, ldr, (double*)C, ldc, info, w, s);
    return run_id<float>(P, (const float*)A, lda, J, (float*)Z, ldz, R11, ldr, (float*)C, ldc, info, w, s);
}

}  // extern "C"
