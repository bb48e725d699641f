// two_sided.hip -- two-sided ID, A ~ W A[I, J] Z.
//
// The paper treats the one-sided ID and credits the two-sided variant to
// Cheng et al. (footnote to the ID's definition, Section 1.2).  Built from
// the paper's own pieces: the column ID of A (Section 2.1, truncated at k per
// Section 4.1) gives J and Z; the row ID of its skeleton C = A[:, J] -- the
// dual ID of Section 2's footnote, i.e. the column ID of C^T -- gives the
// skeleton rows I and W (m x k, W[I, :] = I_k).  Both stages run the blocked
// CPQR and triangular-solve kernels of the one-sided path; C^T is gathered
// straight from A (k x m, FP64 or FP32 as A), and W is the transpose of the
// second stage's Z.
#include <algorithm>

#include "common.hpp"
#include "handle.hpp"
#include "cpqr.hpp"

namespace miid {

// Ct (k x m, column-major, ld k) = A[:, J]^T; J[q] outside [0, n) gives a zero
// row.  64 x 64 tiles through LDS: reads along the columns of A, writes along
// the columns of Ct.
template <typename T>
__global__ void __launch_bounds__(256) k_gather_ct(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                   const int32_t* __restrict__ J, int k, T* __restrict__ Ct) {
    __shared__ T tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int q0 = blockIdx.y * 64;
    const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
    for (int qq = ty; qq < 64; qq += 4) {
        const int q = q0 + qq;
        const int64_t src = q < k ? J[q] : -1;
        const int64_t r = r0 + tx;
        tile[qq][tx] = (src >= 0 && src < n && r < m) ? A[r + src * lda] : T(0);
    }
    __syncthreads();
    for (int rr = ty; rr < 64; rr += 4) {
        const int64_t r = r0 + rr;
        const int q = q0 + tx;
        if (r < m && q < k) Ct[q + r * k] = tile[tx][rr];
    }
}

// W (m x k, ldw) = Z2^T, Z2 k x m (ld k)
template <typename T>
__global__ void __launch_bounds__(256) k_transpose_w(const T* __restrict__ Z2, int k, int64_t m, T* __restrict__ W,
                                                     int64_t ldw) {
    __shared__ T tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int q0 = blockIdx.y * 64;
    const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
    for (int rr = ty; rr < 64; rr += 4) {
        const int64_t r = r0 + rr;
        const int q = q0 + tx;
        tile[rr][tx] = (r < m && q < k) ? Z2[q + r * k] : T(0);
    }
    __syncthreads();
    for (int qq = ty; qq < 64; qq += 4) {
        const int q = q0 + qq;
        const int64_t r = r0 + tx;
        if (r < m && q < k) W[r + (int64_t)q * ldw] = tile[tx][qq];
    }
}

struct TsPlan {
    IdPlan cols, rows;  // the column ID of A (m x n), the column ID of C^T (k x m)
    size_t oRows, oCt, oZ2, total;
};

static int ts_plan(int64_t m, int64_t n, miid_dtype dtype, const miid_opts* o, TsPlan* P) {
    if (!o || o->k < 1) return o ? MIID_E_UNSUPPORTED : -6;  // fixed rank only
    miid_opts o1 = *o;
    o1.flags |= MIID_KEEP_COLUMNS;
    int rc = make_plan(m, n, dtype, &o1, &P->cols);
    if (rc != 0) return rc;
    const int k = P->cols.kmax;
    miid_opts o2 = o1;
    o2.k = k;
    rc = make_plan(k, m, dtype, &o2, &P->rows);
    if (rc != 0) return rc == -3 ? -2 : rc;
    const size_t esz = dtype == MIID_F64 ? 8 : 4;
    size_t off = align_up(P->cols.total, 256);
    P->oRows = off;
    off = align_up(off + P->rows.total, 256);
    P->oCt = off;
    off = align_up(off + (size_t)k * m * esz, 256);
    P->oZ2 = off;
    off = align_up(off + (size_t)k * m * esz, 256);
    P->total = off;
    return 0;
}

template <typename T>
static int run_two_sided(const TsPlan& P, const T* A, int64_t m, int64_t n, int64_t lda, int32_t* J, T* Z,
                         int64_t ldz, int32_t* I, T* W, int64_t ldw, miid_info* info, miid_info* info_rows,
                         unsigned char* w, hipStream_t s) {
    const int k = P.cols.kmax;
    T* Ct = reinterpret_cast<T*>(w + P.oCt);
    T* Z2 = reinterpret_cast<T*>(w + P.oZ2);
    int rc = run_id<T>(P.cols, A, lda, J, Z, ldz, nullptr, 0, nullptr, 0, info, w, s, false, A, lda, m);
    if (rc != 0) return rc;
    const dim3 tg((unsigned)((m + 63) / 64), (unsigned)((k + 63) / 64));
    hipLaunchKernelGGL(k_gather_ct<T>, tg, dim3(256), 0, s, A, lda, m, n, J, k, Ct);
    rc = run_id<T>(P.rows, Ct, (int64_t)k, I, Z2, (int64_t)k, nullptr, 0, nullptr, 0, info_rows, w + P.oRows, s, false,
                   Ct, (int64_t)k, (int64_t)k);
    if (rc != 0) return rc;
    hipLaunchKernelGGL(k_transpose_w<T>, tg, dim3(256), 0, s, Z2, k, m, W, ldw);
    MIID_HIP(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------------------
// CUR form: C = A[:, J], R = A[I, :], U = Z R^+ (k x k), the least-squares
// solution of U R ~ Z.  Transposed, U^T = (R^T)^+ Z^T is the least-squares
// coefficient matrix of [R^T | Z^T] (n x 2k) for its first k columns, which
// the least-squares pass of the randomized ID computes (Gram in FP64,
// Cholesky, two-sided solve): its output is [I | U^T].
// ---------------------------------------------------------------------------

// Mt[:, 0:k] = A[I, :]^T (n x k, ld n); I[q] outside [0, m) gives a zero column
template <typename T>
__global__ void __launch_bounds__(256) k_gather_rows_t(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                       const int32_t* __restrict__ I, int k, T* __restrict__ Mt) {
    const int q = blockIdx.y;
    const int64_t src = I[q];
    const bool ok = src >= 0 && src < m;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        Mt[c + (int64_t)q * n] = ok ? A[src + c * lda] : T(0);
}

__global__ void k_iota_i32(int32_t* __restrict__ J, int k) {
    for (int i = threadIdx.x; i < k; i += blockDim.x) J[i] = i;
}

// a breakdown of the least-squares pass's Cholesky into the row stage's status
__global__ void k_cur_status(miid_info* __restrict__ info_rows, const uint32_t* __restrict__ flag) {
    if (threadIdx.x == 0 && flag[0]) info_rows->status |= MIID_LSTSQ_BREAKDOWN;
}

struct CurPlan {
    TsPlan ts;
    LsPlan ls;
    size_t oZ, oW, oMt, oJid, oZls, oLs, total;
};

static int cur_plan(int64_t m, int64_t n, miid_dtype dtype, const miid_opts* o, CurPlan* P) {
    int rc = ts_plan(m, n, dtype, o, &P->ts);
    if (rc != 0) return rc;
    const int k = P->ts.cols.kmax;
    const size_t esz = dtype == MIID_F64 ? 8 : 4;
    rc = ls_plan(n, 2 * (int64_t)k, k, esz, &P->ls);
    if (rc != 0) return rc;
    size_t off = P->ts.total;
    auto take = [&](size_t bytes) {
        const size_t o2 = off;
        off = align_up(off + bytes, 256);
        return o2;
    };
    P->oZ = take((size_t)k * n * esz);
    P->oW = take((size_t)m * k * esz);
    P->oMt = take((size_t)n * 2 * k * esz);
    P->oJid = take((size_t)k * 4);
    P->oZls = take((size_t)k * 2 * k * esz);
    P->oLs = take(P->ls.total);
    P->total = off;
    return 0;
}

template <typename T>
static int run_cur(const CurPlan& P, const T* A, int64_t m, int64_t n, int64_t lda, int32_t* J, int32_t* I, T* U,
                   int64_t ldu, miid_info* info, miid_info* info_rows, unsigned char* w, hipStream_t s) {
    const int k = P.ts.cols.kmax;
    T* Z = reinterpret_cast<T*>(w + P.oZ);
    T* W = reinterpret_cast<T*>(w + P.oW);
    T* Mt = reinterpret_cast<T*>(w + P.oMt);
    int32_t* Jid = reinterpret_cast<int32_t*>(w + P.oJid);
    T* Zls = reinterpret_cast<T*>(w + P.oZls);
    unsigned char* wl = w + P.oLs;
    int rc = run_two_sided<T>(P.ts, A, m, n, lda, J, Z, (int64_t)k, I, W, m, info, info_rows, w, s);
    if (rc != 0) return rc;
    hipLaunchKernelGGL(k_gather_rows_t<T>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64), (unsigned)k),
                       dim3(256), 0, s, A, lda, m, n, I, k, Mt);
    hipLaunchKernelGGL(k_transpose_w<T>, dim3((unsigned)((n + 63) / 64), (unsigned)((k + 63) / 64)), dim3(256), 0, s,
                       Z, k, n, Mt + (int64_t)k * n, n);
    hipLaunchKernelGGL(k_iota_i32, dim3(1), dim3(256), 0, s, Jid, k);
    // rows of the skeleton beyond the row stage's k_out are absent
    rc = run_lstsq<T>(P.ls, Mt, n, 2 * (int64_t)k, n, Jid, k, info_rows, Zls, (int64_t)k, nullptr, 0, wl, s);
    if (rc != 0) return rc;
    hipLaunchKernelGGL(k_cur_status, dim3(1), dim3(64), 0, s, info_rows,
                       reinterpret_cast<const uint32_t*>(wl + P.ls.oFlag));
    // U = (U^T)^T, U^T = Zls[:, k:2k]
    const dim3 tg((unsigned)((k + 63) / 64), (unsigned)((k + 63) / 64));
    hipLaunchKernelGGL(k_transpose_w<T>, tg, dim3(256), 0, s, Zls + (int64_t)k * k, k, (int64_t)k, U, ldu);
    MIID_HIP(hipGetLastError());
    return 0;
}

}  // namespace miid

using namespace miid;

extern "C" {

static size_t two_sided_workspace_body(int64_t m, int64_t n, miid_dtype dtype, const miid_opts* opts) {
    TsPlan P;
    if (m < 1 || n < 1 || ts_plan(m, n, dtype, opts, &P) != 0) return 0;
    return P.total;
}

static int two_sided_body(const void* A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype, const miid_opts* opts,
                 int32_t* J, void* Z, int64_t ldz, int32_t* I, void* W, int64_t ldw, miid_info* info,
                 miid_info* info_rows, void* ws, size_t ws_bytes, void* stream) {
    if (!A) return -1;
    if (m < 1) return -2;
    if (n < 1) return -3;
    if (lda < m) return -4;
    if (dtype != MIID_F32 && dtype != MIID_F64) return -5;
    TsPlan P;
    const int rc = ts_plan(m, n, dtype, opts, &P);
    if (rc != 0) return rc;
    const int k = P.cols.kmax;
    if (!J) return -7;
    if (!Z) return -8;
    if (ldz < k) return -9;
    if (!I) return -10;
    if (!W) return -11;
    if (ldw < m) return -12;
    if (!info) return -13;
    if (!info_rows) return -14;
    if (!ws) return -15;
    if (ws_bytes < P.total) return MIID_E_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    if (dtype == MIID_F64)
        return run_two_sided<double>(P, (const double*)A, m, n, lda, J, (double*)Z, ldz, I, (double*)W, ldw, info,
                                     info_rows, w, s);
    return run_two_sided<float>(P, (const float*)A, m, n, lda, J, (float*)Z, ldz, I, (float*)W, ldw, info, info_rows,
                                w, s);
}

static size_t cur_workspace_body(int64_t m, int64_t n, miid_dtype dtype, const miid_opts* opts) {
    CurPlan P;
    if (m < 1 || n < 1 || cur_plan(m, n, dtype, opts, &P) != 0) return 0;
    return P.total;
}

static int cur_body(const void* A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype, const miid_opts* opts, int32_t* J,
           int32_t* I, void* U, int64_t ldu, miid_info* info, miid_info* info_rows, void* ws, size_t ws_bytes,
           void* stream) {
    if (!A) return -1;
    if (m < 1) return -2;
    if (n < 1) return -3;
    if (lda < m) return -4;
    if (dtype != MIID_F32 && dtype != MIID_F64) return -5;
    CurPlan P;
    const int rc = cur_plan(m, n, dtype, opts, &P);
    if (rc != 0) return rc;
    const int k = P.ts.cols.kmax;
    if (!J) return -7;
    if (!I) return -8;
    if (!U) return -9;
    if (ldu < k) return -10;
    if (!info) return -11;
    if (!info_rows) return -12;
    if (!ws) return -13;
    if (ws_bytes < P.total) return MIID_E_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    if (dtype == MIID_F64)
        return run_cur<double>(P, (const double*)A, m, n, lda, J, I, (double*)U, ldu, info, info_rows, w, s);
    return run_cur<float>(P, (const float*)A, m, n, lda, J, I, (float*)U, ldu, info, info_rows, w, s);
}

// ---- entry points: the handle resolved, then the bodies above -----------
size_t miid_two_sided_workspace(miid_handle h, int64_t m, int64_t n, miid_dtype dtype, const miid_opts* opts) {
    miid_opts o;
    if (resolve_opts(h, kTuneTwoSided, dtype, m, n, opts ? opts->k : 0, opts, &o) != 0) return 0;
    return two_sided_workspace_body(m, n, dtype, opts ? &o : nullptr);
}

int id_two_sided(miid_handle h, const void* A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype,
                 const miid_opts* opts, int32_t* J, void* Z, int64_t ldz, int32_t* I, void* W, int64_t ldw,
                 miid_info* info, miid_info* info_rows, void* ws, size_t ws_bytes, void* stream) {
    miid_opts o;
    if (resolve_opts(h, kTuneTwoSided, dtype, m, n, opts ? opts->k : 0, opts, &o) != 0) return -1;
    return shift_arg(two_sided_body(A, m, n, lda, dtype, opts ? &o : nullptr, J, Z, ldz, I, W, ldw, info, info_rows,
                                    ws, ws_bytes, stream));
}

size_t miid_cur_workspace(miid_handle h, int64_t m, int64_t n, miid_dtype dtype, const miid_opts* opts) {
    miid_opts o;
    if (resolve_opts(h, kTuneCur, dtype, m, n, opts ? opts->k : 0, opts, &o) != 0) return 0;
    return cur_workspace_body(m, n, dtype, opts ? &o : nullptr);
}

int id_cur(miid_handle h, const void* A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype, const miid_opts* opts,
           int32_t* J, int32_t* I, void* U, int64_t ldu, miid_info* info, miid_info* info_rows, void* ws,
           size_t ws_bytes, void* stream) {
    miid_opts o;
    if (resolve_opts(h, kTuneCur, dtype, m, n, opts ? opts->k : 0, opts, &o) != 0) return -1;
    return shift_arg(cur_body(A, m, n, lda, dtype, opts ? &o : nullptr, J, I, U, ldu, info, info_rows, ws, ws_bytes,
                              stream));
}

}  // extern "C"
