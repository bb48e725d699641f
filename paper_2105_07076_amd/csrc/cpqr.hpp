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
    // fused one-launch-per-step path (at most 576 rows): NP passes of four
    // columns per wave, fnpart workgroups
    bool fused;
    int fnp, fnpart, fgl;  // fgl: 16-byte row groups per lane (5, 9 or 10)
    int kpad;  // kmax rounded up to the triangular solve's diagonal block
    size_t oS, oV, oF, ou, onu, onuref, oR, osel, opart, opartA, oR11, oDinv, ostate, orec, total;
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

// M = R11^{-1} R11^{-T} B on the matrix cores (the solution of
// R11^T R11 M = B), R11 k x k FP64 upper triangular (ldr); B is k x n with
// element (q, c) at B[q rs + c cs]; M is k x n column-major (ldm).  jmode 1:
// the columns marked in sel (sel[c] >= 0) are zero right-hand sides; jmode 0:
// they come out as the unit vectors e_sel[c].  ws holds
// semi_solve_workspace(k) bytes.
size_t semi_solve_workspace(int k);
template <typename T>
int semi_solve(const double* R11, int64_t ldr, int k, const T* B, int64_t rs, int64_t cs, int64_t n,
               const int32_t* sel, int jmode, T* M, int64_t ldm, unsigned char* ws, hipStream_t s);

// Z = C^+ A (k x n, ldz) for the skeleton J (k entries; -1 gathers a zero
// column, whose row of Z comes out zero), C = A[:, J] gathered into the
// workspace, by the normal equations with the Cholesky factor R of C^T C,
// written to R11 (k x k FP64, ldr) when given.  With kinfo, columns from
// kinfo->k_out on are treated as absent.  A pivot of the Cholesky that is not
// positive (C's columns dependent in FP64) sets the workspace flag at oFlag.
struct LsPlan {
    int gz, gzr;  // the Gram's split over rows (planned, launched)
    size_t oC64, oGram, oGp, oR, oCT, oB, oSel, oFlag, oSemi, total;
};
int ls_plan(int64_t m, int64_t n, int k, size_t esz, LsPlan* L);
template <typename T>
int run_lstsq(const LsPlan& L, const T* A, int64_t m, int64_t n, int64_t lda, const int32_t* J, int k,
              const miid_info* kinfo, T* Z, int64_t ldz, double* R11, int64_t ldr, unsigned char* w, hipStream_t s);

}  // namespace miid
