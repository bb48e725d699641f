/*
 * miid.h -- C ABI of the MI355X (gfx950) interpolative-decomposition library.
 *
 * Paper: R. Advani and S. O'Hagan, "Efficient Algorithms for Constructing an
 * Interpolative Decomposition" (arXiv 2105.07076).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are column-major.  "ld" arguments are leading dimensions in
 *    elements.  Indices are 0-based int32.
 *  - Every matrix/vector argument is a DEVICE pointer owned by the caller
 *    (the library never allocates device memory); option structs are HOST
 *    pointers.  `ws` is a caller-owned device workspace of at least the size
 *    returned by the matching *_workspace() query; its contents on entry are
 *    irrelevant and on return are unspecified.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously; results (including `info`, a DEVICE pointer) are valid
 *    once the stream has been synchronised.  Tolerance mode (opts.k == 0)
 *    synchronises the stream a few times to stop early.
 *  - The return value only reports problems the host can see at call time:
 *      0                 success (launches enqueued)
 *      -i                argument i (1-based; the handle is argument 1) is
 *                        invalid (LAPACK convention)
 *      MIID_E_WORKSPACE  ws_bytes is smaller than the workspace query
 *      MIID_E_HIP        a HIP call failed (miid_last_hip_error() tells which)
 *      MIID_E_UNSUPPORTED shape or option outside the documented limits
 *    Numerical outcomes are written to `info` on the device.
 *  - Calls that share a workspace must not overlap in time.
 */
#ifndef MIID_H
#define MIID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MIID_E_WORKSPACE (-100)
#define MIID_E_HIP (-101)
#define MIID_E_UNSUPPORTED (-102)

/* element type of A, Z, C (and of the gradients in id_backward) */
typedef enum { MIID_F32 = 0, MIID_F64 = 1 } miid_dtype;

/* status bits written to miid_info.status */
#define MIID_RANK_DEFICIENT 1u /* a residual became exactly zero: k_out < k   */
#define MIID_NONFINITE 2u      /* A holds a NaN or an infinity: outputs unspecified */
#define MIID_TRANSPOSED 4u     /* m > n: the dual ID of A^T was computed      */
#define MIID_KMAX_HIT 8u       /* tolerance mode stopped at kmax, not at eps  */
#define MIID_BLOCK_UNSUPPORTED 16u /* id_batched: block outside the size limits */
#define MIID_LSTSQ_BREAKDOWN 32u   /* rid_sketch_cpqr with MIID_LSTSQ_Z: C^T C is not
                                      positive definite in FP64 (C's columns
                                      numerically dependent): Z unspecified */

/* option flags */
#define MIID_NO_REFINE 1u      /* skip the refinement step of the triangular solve */
#define MIID_KEEP_COLUMNS 2u   /* id_cpqr: column ID even when m > n (no dual ID of A^T);
                                  then k <= n is required                           */
#define MIID_LSTSQ_Z 4u        /* rid_sketch_cpqr, fixed rank only: Z = C^+ A over the
                                  full A instead of T from the sketch             */

/* Tuning hints, 4-bit fields of miid_opts.flags (0 = library default).  They
 * change launch shapes only, never the arithmetic's definition; the
 * autotuner of the Python package picks them by timing.
 *  CPW   id_cpqr/rid: columns per wave of the two-launch blocked path's
 *        F-GEMV (1, 2 or 4)
 *  NP    id_cpqr/rid: column passes per wave of the one-launch fused path
 *        for short matrices (1, 2, 4 or 8; default: the fewest that give
 *        one workgroup per CU)
 *  PATH  id_cpqr/rid: 1 = blocked two-launch path, 2 = fused path (taken
 *        only where eligible: at most 576 rows in FP32 / 320 in FP64,
 *        panels of at most 32)
 *  LPC   id_batched: cap on the lanes that share one column of a block
 *        (1, 2, 4 or 8; default 8: as many as n L <= 512 allows).  It
 *        changes the order of the per-lane partial sums, so results can
 *        differ in the last bits between settings                       */
#define MIID_HINT_CPW_SHIFT 8
#define MIID_HINT_NP_SHIFT 12
#define MIID_HINT_PATH_SHIFT 16
#define MIID_HINT_LPC_SHIFT 20
#define MIID_HINT(field_shift, value) (((uint32_t)(value) & 15u) << (field_shift))

typedef struct {
    int32_t k;      /* > 0: fixed rank.  0: tolerance mode: the smallest k with
                       ||R22||_F <= eps * ||A||_F (estimated from the downdated
                       column norms), at most kmax                       */
    int32_t kmax;   /* tolerance mode cap (ignored when k > 0); rows of Z/J */
    double eps;     /* relative tolerance for tolerance mode             */
    int32_t nb;     /* panel width of the blocked QR, 0 = library default */
    uint32_t flags; /* MIID_NO_REFINE | MIID_HINT(...) fields            */
} miid_opts;

typedef struct {
    int32_t k_out;       /* number of columns selected                      */
    uint32_t status;     /* MIID_* status bits                              */
    double a_norm;       /* ||A||_F                                          */
    double r22_norm;     /* ||R22||_F estimate from the downdated norms      */
    int32_t n_recompute; /* column norms recomputed after cancellation       */
    int32_t n_steps;     /* pivot steps executed                             */
} miid_info;

/* Instrumentation (host): kernel timing with HIP events recorded on the
 * stream each kernel is launched on.  miid_prof_begin(e) samples every e-th
 * launch of each kernel (e = 0 switches it off); miid_prof_end() waits for
 * the recorded events, copies up to max_records records and returns their
 * number.  Kernel ids: */
#define MIID_K_GEMV 1      /* F-GEMV + row update + downdate, one per pivot step */
#define MIID_K_PIVOT 2     /* pivot search + pivot column, one per pivot step     */
#define MIID_K_TRAIL 3     /* trailing update, one per panel                      */
#define MIID_K_SKETCH 4    /* sketch GEMM Y = Omega A                             */
#define MIID_K_BATCHED 5   /* persistent batched ID kernel                        */
#define MIID_K_BWD_GEMM 6  /* adjoint GEMMs                                       */
#define MIID_K_TRSM 7      /* triangular solve                                    */
#define MIID_K_STEP 8      /* fused pivot step (matrices of <= 1024 rows)         */
typedef struct {
    int32_t kernel; /* MIID_K_* */
    int32_t step;   /* launch index (pivot step for per-step kernels)     */
    int64_t rows;   /* rows of the operand streamed by this launch        */
    int64_t cols;   /* columns of that operand                            */
    float ms;       /* elapsed time between the two events                */
} miid_prof_record;
int miid_prof_begin(int sample_every);
int miid_prof_end(miid_prof_record *out, int max_records);

/* library version string (host) */
const char *miid_version(void);
/* HIP error code of the last MIID_E_HIP return on this thread */
int miid_last_hip_error(void);

/* ------------------------------------------------------------------------
 * Library handle, the first argument of every entry point below.
 *
 * A handle belongs to the device that is current when miid_create runs and
 * holds a read-only table of tuned launch shapes.  Passing it while another
 * device is current returns -1 (argument 1 invalid).  NULL is accepted
 * everywhere and means "no table".  The facts the library keeps per device
 * -- its compute-unit count, the kernels whose LDS limit has been raised --
 * are queried once per device whether or not a handle is used.  A handle
 * created with no visible device serves the workspace queries only.  The
 * paper's problem statement (Section 2) fixes the arguments, A, k (or a
 * tolerance), J and Z; the handle only changes launch shapes, never what is
 * computed.
 *
 *  out            receives the handle (release it with miid_destroy)
 *  autotune_path  nullable: a text file with one row per line ('#' starts a
 *                 comment line):
 *                     routine dtype m n k nb hints
 *                 routine  id | rid | rid_sample | two_sided | cur | batched
 *                 dtype    f32 | f64 (rid: f32)
 *                 m n k    the call's m, n and opts.k (batched: nblk, 0 and
 *                          opts.kmax); 0 matches any value
 *                 nb       panel width (0 = the library's)
 *                 hints    MIID_HINT fields, decimal or 0x hex
 *                 A call whose opts leave nb = 0 and every hint field 0
 *                 runs with the most specific matching row; the workspace
 *                 queries apply the same rule.
 * Returns 0; -1 if out is NULL; -2 if the file cannot be read or a row is
 * malformed (no handle is created); MIID_E_UNSUPPORTED if host memory for
 * the handle cannot be allocated.
 * ---------------------------------------------------------------------- */
typedef struct miid_handle_s *miid_handle;
int miid_create(miid_handle *out, const char *autotune_path);
void miid_destroy(miid_handle h);
/* device ordinal the handle belongs to (-1: none visible at creation) */
int miid_handle_device(miid_handle h);
/* number of rows in the handle's tuning table */
int miid_handle_rows(miid_handle h);

/* ------------------------------------------------------------------------
 * Deterministic ID (Section 2.1; truncated QR of Section 4.1).
 *
 * Column-pivoted Householder QR A P = Q R with Businger-Golub pivoting on the
 * residual column norms (largest norm first, ties to the smallest column
 * index), stopped after k steps; C = A P_k (= A[:, J]) and
 * Z = [I  R11^{-1} R12] P^T, the least-squares solution of min ||A - C Z||_F
 * (Section 2.1, eq. final_eq solved by triangular solves).
 * If m > n the dual ID of A^T is computed (footnote to Section 2): J then
 * indexes rows of A, Z is k x m and A ~ Z^T A[J, :]; status gets
 * MIID_TRANSPOSED.
 *
 *  A     (2)  m x n, leading dimension lda >= m, read only
 *  J     (8)  kmax int32 (kmax = opts.k when k > 0): selected indices in
 *             pivot order; entries >= k_out are -1
 *  Z     (9)  kmax x N (N = max(m, n)), ldz >= kmax, dtype: Z[:, J[c]] is
 *             exactly the c-th unit vector, the other columns hold T, rows
 *             >= k_out are zero; columns in ORIGINAL order
 *  R11   (11) nullable, kmax x kmax FP64, ldr >= kmax: the triangular factor
 *             in pivot order (upper triangle; needed by id_backward)
 *  C     (13) nullable, M x kmax (M = min(m, n)), ldc >= M, dtype: A[:, J]
 *             (or A[J, :]^T when transposed); columns >= k_out unspecified
 *  info  (15) device pointer to one miid_info
 * Limits: 1 <= kmax <= min(m, n, 1024); nb in [1, 64].
 * ---------------------------------------------------------------------- */
size_t miid_id_workspace(miid_handle h, int64_t m, int64_t n, miid_dtype dtype, const miid_opts *opts);
int id_cpqr(miid_handle h, const void *A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype,
            const miid_opts *opts, int32_t *J, void *Z, int64_t ldz,
            double *R11, int64_t ldr, void *C, int64_t ldc, miid_info *info,
            void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Randomized ID with a Gaussian row sketch.  The paper's randomized method
 * (Section 2.2) runs the same CPQR on a smaller matrix; here that smaller
 * matrix is Y = Omega A (l x n), computed on the matrix cores in bfloat16
 * with FP32 accumulation.  The CPQR of Y (FP32, FP64 norms, FP64 triangular
 * solve) gives J and T; C = A[:, J].
 *
 *  A      (2)  m x n FP32, lda >= m, m <= n (else MIID_E_UNSUPPORTED)
 *  Omega  (6)  l x m bfloat16 bit patterns, column-major, ldo >= l
 *  mode   (9)  0: A rounded once to bfloat16 (one matrix-core pass,
 *                 |a - hi| <= 2^-8 |a|);
 *              1: A split as hi + mid, both bfloat16 (two passes,
 *                 |a - hi - mid| <= 2^-16 |a|);
 *              2: A split as hi + mid + lo (three passes, 2^-24 |a|: the
 *                 sketch as accurate as FP32 accumulation allows)
 *  J, Z, C, R11, info: as in id_cpqr with dtype FP32; Z is kmax x n
 *  Y      (16) nullable, l x n FP32, ldy >= l: the sketch
 * With MIID_LSTSQ_Z in opts.flags (fixed rank, k <= m) Z is instead the
 * least-squares coefficient matrix over the full A, Z = C^+ A, the paper's
 * way of forming the randomized ID's Z (Section 2.2, eq. final_eq), for the
 * skeleton J the sketch selected (same J, same order): R11 is then the
 * Cholesky factor of C^T C (computed in FP64, R11^T R11 = C^T C, positive
 * diagonal) and Z solves R11^T R11 Z = C^T A with Z[:, J] = I.  info still
 * describes the CPQR of Y, plus MIID_LSTSQ_BREAKDOWN.
 * Limits: k <= l <= min(n, 1024) (kmax <= l in tolerance mode), m <= n,
 * lda <= 2^23.
 * ---------------------------------------------------------------------- */
size_t miid_rid_workspace(miid_handle h, int64_t m, int64_t n, int32_t l, const miid_opts *opts);
int rid_sketch_cpqr(miid_handle h, const float *A, int64_t m, int64_t n, int64_t lda,
                    const uint16_t *Omega, int32_t l, int64_t ldo, int32_t mode,
                    const miid_opts *opts, int32_t *J, float *Z, int64_t ldz,
                    float *C, int64_t ldc, float *Y, int64_t ldy,
                    double *R11, int64_t ldr, miid_info *info,
                    void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * The paper's randomized ID by column sampling (Section 2.2 and its Optim
 * RID listing).  The column-pivoted QR of A_S = A[:, idx] (m x p: the p
 * sampled columns; the paper samples p = k + floor(0.2 k) without
 * replacement -- the sample is an input here) selects k of them, so
 * J = idx[selected] and C = A_S P_k = A[:, J]; Z is the least-squares
 * solution over the FULL A, R_k^T R_k Z = C^T A (eq. final_eq), R_k the
 * leading k x k triangle of A_S's factor, solved as Z = R_k^{-1} R_k^{-T}
 * (C^T A) in FP64 (C^T A on the matrix cores in the working precision).
 * Z[:, J[c]] is set to the c-th unit vector exactly (Definition 1).
 *
 *  A     (2)  m x n, lda >= m, dtype, read only
 *  idx   (7)  device int32[p]: the sampled column indices (distinct, in
 *             [0, n); an index outside gives a zero column of A_S)
 *  p     (8)  1 <= p <= n
 *  opts  (9)  fixed rank only: k >= 1, k <= min(m, p, 1024); nb, flags as
 *             for id_cpqr (MIID_KEEP_COLUMNS is implied, MIID_NO_REFINE has
 *             no effect on the least-squares solve)
 *  J     (10) k int32; entries >= k_out are -1
 *  Z     (11) k x n, ldz >= k, dtype, columns in original order; rows
 *             >= k_out zero
 *  R11   (13) nullable: R_k, k x k FP64, ldr >= k
 *  C     (15) nullable: m x k, ldc >= m, dtype: A[:, J]
 *  info  (17) device miid_info of the CPQR of A_S (a_norm, r22_norm refer to
 *             A_S)
 * ---------------------------------------------------------------------- */
size_t miid_rid_sample_workspace(miid_handle h, int64_t m, int64_t n, int32_t p, miid_dtype dtype,
                                 const miid_opts *opts);
int rid_sample_cpqr(miid_handle h, const void *A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype,
                    const int32_t *idx, int32_t p, const miid_opts *opts,
                    int32_t *J, void *Z, int64_t ldz, double *R11, int64_t ldr,
                    void *C, int64_t ldc, miid_info *info,
                    void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Two-sided ID, A ~ W A[I, J] Z (the variant the paper credits to Cheng et
 * al., footnote to the ID's definition, Section 1.2): the column ID of A
 * (Section 2.1, a column ID whatever the shape: MIID_KEEP_COLUMNS is
 * implied) gives J and Z, then the row ID of its skeleton C = A[:, J] --
 * the dual ID of Section 2's footnote, the column ID of C^T -- gives I and
 * W.  Both stages are the blocked CPQR + triangular solve of id_cpqr.
 *
 *  A          (2)  m x n, lda >= m, dtype, read only
 *  opts       (7)  fixed rank only: 1 <= k <= min(m, n, 1024); nb, flags as
 *                  for id_cpqr (else MIID_E_UNSUPPORTED)
 *  J          (8)  k int32: skeleton columns; entries >= k_out are -1
 *  Z          (9)  k x n, ldz >= k, dtype: Z[:, J[c]] = e_c
 *  I          (11) k int32: skeleton rows (of the skeleton C, i.e. of A);
 *                  entries >= the row stage's k_out are -1
 *  W          (12) m x k, ldw >= m, dtype: W[I[c], :] = e_c^T
 *  info       (14) device miid_info of the column stage (norms refer to A)
 *  info_rows  (15) device miid_info of the row stage (norms refer to C)
 * ---------------------------------------------------------------------- */
size_t miid_two_sided_workspace(miid_handle h, int64_t m, int64_t n, miid_dtype dtype, const miid_opts *opts);
int id_two_sided(miid_handle h, const void *A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype,
                 const miid_opts *opts, int32_t *J, void *Z, int64_t ldz,
                 int32_t *I, void *W, int64_t ldw, miid_info *info, miid_info *info_rows,
                 void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * CUR form of the two-sided ID: A ~ C U R with C = A[:, J], R = A[I, :]
 * (J, I from id_two_sided) and U = Z R^+ (k x k), the least-squares
 * solution of U R ~ Z (so C U R ~ C Z), computed like the least-squares Z
 * of rid_sketch_cpqr (FP64 Gram of R, Cholesky, two-sided solve).  Not in
 * the paper; it completes the two-sided form.
 *
 *  A, opts, J, I: as for id_two_sided; U (10) k x k, ldu >= k, dtype
 *  info, info_rows: as for id_two_sided; info_rows also gets
 *                   MIID_LSTSQ_BREAKDOWN if R R^T is not positive definite in
 *                   FP64
 * ---------------------------------------------------------------------- */
size_t miid_cur_workspace(miid_handle h, int64_t m, int64_t n, miid_dtype dtype, const miid_opts *opts);
int id_cur(miid_handle h, const void *A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype,
           const miid_opts *opts, int32_t *J, int32_t *I, void *U, int64_t ldu,
           miid_info *info, miid_info *info_rows, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Batched tolerance-mode IDs of many independent small blocks (for instance
 * the off-diagonal blocks of a hierarchical kernel-matrix compression), in
 * one persistent launch.  Block b is m[b] x n[b] (column-major, leading
 * dimension m[b]) at A + a_off[b]; its rank is the smallest k with
 * ||R22||_F <= eps ||A_b||_F (exact residual norms), at most
 * kmax_b = min(m[b], n[b], kmax).
 *
 *  A      (3)  packed blocks, dtype
 *  a_off, m, n (4-6) device int64 / int32 / int32 arrays of length nblk
 *  opts   (8)  host: eps, kmax and flags (MIID_HINT(MIID_HINT_LPC_SHIFT, l));
 *              k and nb are ignored
 *  J      (9)  packed int32: block b owns kmax_b entries at j_off[b]
 *  Z      (11) packed dtype: block b owns a kmax_b x n[b] column-major
 *              matrix (leading dimension kmax_b) at z_off[b]; rows >= k_out
 *              are zero
 *  info   (13) nblk miid_info entries
 * Limits: 1 <= m[b] <= 256, m[b] <= n[b] <= 1024, 1 <= kmax <= 64.  A block
 * outside them is skipped with k_out = 0 and status MIID_BLOCK_UNSUPPORTED;
 * the others are unaffected (likewise a block holding a NaN only gets its
 * own MIID_NONFINITE).  Blocks are processed largest first (by m n).
 * ---------------------------------------------------------------------- */
size_t miid_batched_workspace(miid_handle h, int32_t nblk, miid_dtype dtype);
int id_batched(miid_handle h, int32_t nblk, const void *A, const int64_t *a_off, const int32_t *m,
               const int32_t *n, miid_dtype dtype, const miid_opts *opts,
               int32_t *J, const int64_t *j_off, void *Z, const int64_t *z_off,
               miid_info *info, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * id_batched for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * The same kernels and the same results as id_batched (arguments 1-13 as
 * there; no workspace), with the library's own static scratch instead of
 * `ws`: 64 MiB of device memory per GPU, reserved when the library is
 * loaded and held until the process ends.  This call allocates nothing;
 * the scratch's address is looked up once per device, by miid_create or by
 * the first call on that device.
 * Limits: nblk <= 262144 (else MIID_E_UNSUPPORTED).  Rows of a block that
 * fit neither the registers nor the LDS get
 *     rg = min(floor((64 MiB - 1 MiB - 256 B) / (G * 512 * esz)) rounded
 *              down to a multiple of 4, the most any block needs)
 * rows per lane, G = min(nblk, compute units), esz = 4 (FP32) or 8 (FP64);
 * a block that needs more gets k_out = 0 and MIID_BLOCK_UNSUPPORTED like a
 * block outside the size limits.  With 256 compute units every FP32 block
 * with n <= 512 fits, and in FP64 those with n <= 256; the blocks that can
 * exceed rg are the widest and tallest ones (n > 256 in FP64 or n > 512 in
 * FP32, m near 256).
 * Every call on a GPU uses that GPU's one copy of the scratch: calls that
 * overlap in time on one GPU (two streams, two threads) race and must not
 * be issued; calls in stream order are fine.
 * ---------------------------------------------------------------------- */
int id_batched_noalloc(miid_handle h, int32_t nblk, const void *A, const int64_t *a_off,
                       const int32_t *m, const int32_t *n, miid_dtype dtype,
                       const miid_opts *opts, int32_t *J, const int64_t *j_off, void *Z,
                       const int64_t *z_off, miid_info *info, void *stream);

/* ------------------------------------------------------------------------
 * Adjoint of the ID with the pivots held fixed (the paper has no
 * derivatives; this is the derivative of T = C^+ A_rest, C = A[:, J]).
 * Given upstream gradients gC (of C) and gZ (of Z), with M = (C^T C)^{-1} Gz
 * where Gz is gZ with its J columns zeroed and C^T C = R11^T R11:
 *     gA          = C M
 *     gA[:, J]   += gC + A M^T - C (Z M^T + M Z^T)
 *
 *  A   (2)   m x n, lda, dtype (the forward input; m <= n)
 *  J   (7)   k int32, R11 (9): k x k FP64 from id_cpqr, ldr
 *  Z   (11)  k x n, ldz, dtype, from id_cpqr
 *  gC  (13)  nullable m x k, ldgc;  gZ (15) nullable k x n, ldgz
 *  gA  (17)  m x n, ldga, written (not accumulated)
 * Limits: 1 <= k <= min(m, n, 1024).
 * ---------------------------------------------------------------------- */
size_t miid_backward_workspace(miid_handle h, int64_t m, int64_t n, int32_t k, miid_dtype dtype);
int id_backward(miid_handle h, const void *A, int64_t m, int64_t n, int64_t lda, miid_dtype dtype,
                const int32_t *J, int32_t k, const double *R11, int64_t ldr,
                const void *Z, int64_t ldz, const void *gC, int64_t ldgc,
                const void *gZ, int64_t ldgz, void *gA, int64_t ldga,
                void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MIID_H */
