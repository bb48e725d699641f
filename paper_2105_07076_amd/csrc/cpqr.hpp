// cpqr.hpp -- the blocked column-pivoted QR + triangular-solve driver shared
// by the deterministic ID (id_cpqr) and the randomized ID (rid_sketch_cpqr).
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace miid {

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

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
    int cpw;   // columns per wave in the column passes (k_norms, k_gemv)
    int npart, NA;
    // fused one-launch-per-step path (at most 1024 rows): NP passes of four
    // columns per wave, fnpart workgroups
    bool fused;
    int fnp, fnpart, fgl;  // fgl: 16-byte row groups per lane (5, 9 or 16)
    // resident path (few rows): rows per lane, grid, columns per workgroup
    bool res_ok;
    int res_rpl, res_grid, res_cpb;
    int kpad;  // kmax rounded up to the triangular solve's diagonal block
    size_t oS, oV, oF, ou, onu, onuref, oR, osel, opart, opartA, oR11, oDinv, ostate, orec, total;
    size_t oPart2, oPartF, oSlots, oBar;
};

// Validates the shape/options and lays out the workspace (returns 0 or a
// negative MIID code).
int make_plan(int64_t M, int64_t N, miid_dtype dtype, const miid_opts* o, IdPlan* P);

// Enqueues the whole factorisation.  With staged = true the working matrix S
// (ldw x n, rows >= m zero) already holds the matrix to factor and the
// staging kernels are skipped; C is gathered from Csrc (crows x n, ldcsrc).
template <typename T>
int run_id(const IdPlan& P, const T* A, int64_t lda, int32_t* J, T* Z, int64_t ldz, double* R11out, int64_t ldr, T* C,
           int64_t ldc, miid_info* info, unsigned char* ws, hipStream_t stream, bool staged, const T* Csrc,
           int64_t ldcsrc, int64_t crows);

// The column-sampling randomized ID: the CPQR of A_S = A[:, idx] (m x p,
// its own column ID) picks J = idx[J_S] and R_k; Z solves
// R_k^T R_k Z = C^T A over the full A (Z[:, J] = I).
struct RsPlan {
    IdPlan id;  // the CPQR of A_S (its workspace comes first)
    size_t oAs, oZs, oJs, oC, oG, oSel, total;
};
int rs_plan(int64_t m, int64_t n, int32_t p, miid_dtype dtype, const miid_opts* o, RsPlan* Q);
template <typename T>
int run_rid_sample(const RsPlan& Q, const T* A, int64_t m, int64_t n, int64_t lda, const int32_t* idx, int p,
                   int32_t* J, T* Z, int64_t ldz, double* R11, int64_t ldr, T* C, int64_t ldc, miid_info* info,
                   unsigned char* w, hipStream_t s);

// M = R11^{-1} R11^{-T} B on the matrix cores (the solution of
// R11^T R11 M = B), R11 k x k FP64 upper triangular (ldr), B and M k x n
// column-major (ldb, ldm); the columns marked in sel (sel[c] >= 0) are
// treated as zero right-hand sides.  ws holds semi_solve_workspace(k) bytes.
size_t semi_solve_workspace(int k);
template <typename T>
int semi_solve(const double* R11, int64_t ldr, int k, const T* B, int64_t ldb, int64_t n, const int32_t* sel, T* M,
               int64_t ldm, unsigned char* ws, hipStream_t s);

}  // namespace miid
