"""Plain FP64 CPU oracle for the interpolative decomposition (ID) hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
It shares no code with the GPU library.  The arithmetic lives in
``oracle.c`` (unblocked Householder QR with exact per-step Businger-Golub
pivoting, back substitution, plain matrix product); this module only
marshals numpy arrays to it and adds the derivative formula, written in numpy.

Paper: Advani & O'Hagan, "Efficient Algorithms for Constructing an
Interpolative Decomposition".  Section 2 (A is m x n, m <= n, else work on
A^T; rank k), Section 2.1 (CPQR selects C = A P_k; Z from the least-squares
problem min ||A - C Z||_F, reduced to triangular solves), Definition 1
(k columns of Z form the identity), Section 4.1 (stop the QR after k
columns).  Beside the ID: ``rid`` (the same CPQR on an exact FP64 sketch),
``rid_sample`` (Section 2.2's column sampling with the normal-equation Z
over the full A), ``two_sided`` (the column ID followed by the dual ID of
its skeleton) and ``cur`` (its CUR form), ``batched`` (tolerance mode per block) and ``id_vjp`` (the
adjoint with the pivots held fixed).

Parity unpinned: none of the functions; only the intermediate rounding of
downdated column norms is internal to the GPU path and has no counterpart
here (the oracle recomputes exact norms every step).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, portable x86-64 code)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_id.restype = ctypes.c_int
        lib.oracle_id.argtypes = [P, I64, I64, I64, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                  P, ctypes.c_int, P, P, P, P, P, P, P]
        lib.oracle_matmul.restype = None
        lib.oracle_matmul.argtypes = [P, I64, P, I64, P, I64, I64, I64, I64]
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class IDResult:
    """Result of one oracle ID.  Z is k x n in original column order with
    Z[:, J] = I; R holds the first k rows of the triangular factor in
    original column order (R[:, J] = R11)."""
    J: np.ndarray
    Z: np.ndarray
    R: np.ndarray
    k: int
    transposed: bool
    nu1: np.ndarray = field(repr=False)
    nu2: np.ndarray = field(repr=False)
    nuo: np.ndarray = field(repr=False)
    resid: np.ndarray = field(repr=False)
    a_norm: float = 0.0

    @property
    def margins(self) -> np.ndarray:
        """mu_j = (nu_(1) - nu_(2)) / nu_(1) per step."""
        with np.errstate(divide="ignore", invalid="ignore"):
            return (self.nu1[: self.k] - self.nu2[: self.k]) / self.nu1[: self.k]

    @property
    def rho(self) -> np.ndarray:
        """rho_j = chosen residual norm / original norm of that column."""
        with np.errstate(divide="ignore", invalid="ignore"):
            return self.nu1[: self.k] / self.nuo[: self.k]

    @property
    def r22(self) -> float:
        """||R22||_F after k steps (residual Frobenius norm)."""
        return float(self.resid[self.k])

    @property
    def T(self) -> np.ndarray:
        """T = R11^{-1} R12 in original column order of the non-selected columns."""
        mask = np.ones(self.Z.shape[1], dtype=bool)
        mask[self.J[: self.k]] = False
        return self.Z[: self.k][:, mask]


def id(A: np.ndarray, k: int | None = None, eps: float | None = None, kmax: int | None = None,
       force: np.ndarray | None = None) -> IDResult:
    """Deterministic ID of A (Section 2.1, truncated at k per Section 4.1).

    Exactly one of ``k`` (fixed rank) or ``eps`` (smallest k with
    ||R22||_F <= eps ||A||_F, capped at ``kmax``) is given.  When m > n the
    ID of A^T is returned (``transposed`` = True): J then indexes rows and
    A ~ Z^T A[J, :] (the dual ID of the footnote to Section 2).
    ``force`` fixes the first pivots (original indices).
    """
    A = np.asarray(A, dtype=np.float64)
    transposed = A.shape[0] > A.shape[1]
    return _id_of(np.asfortranarray(A.T if transposed else A), transposed, k, eps, kmax, force)


def _id_of(W: np.ndarray, transposed: bool, k, eps, kmax, force) -> IDResult:
    """The column ID of W as given (m x n, any shape with k <= min(m, n))."""
    m, n = W.shape
    if (k is None) == (eps is None):
        raise ValueError("give exactly one of k or eps")
    if k is not None:
        kk, e, km = int(k), 0.0, int(k)
        if kk <= 0:
            raise ValueError("k must be positive")
    else:
        km = int(kmax) if kmax is not None else min(m, n)
        kk, e = 0, float(eps)
    km = min(km, m, n)
    J = np.full(max(km, 1), -1, dtype=np.int32)
    Z = np.zeros((max(km, 1), n), dtype=np.float64, order="F")
    R = np.zeros((max(km, 1), n), dtype=np.float64, order="F")
    nu1 = np.zeros(max(km, 1))
    nu2 = np.zeros(max(km, 1))
    nuo = np.zeros(max(km, 1))
    resid = np.zeros(max(km, 1) + 1)
    f = None
    nf = 0
    if force is not None:
        f = np.ascontiguousarray(force, dtype=np.int32)
        nf = len(f)
    kk = min(kk, km) if k is not None else 0
    kout = _load().oracle_id(_ptr(W), m, n, m, kk, e, max(km, 1), _ptr(f), nf, _ptr(J), _ptr(Z), _ptr(R),
                             _ptr(nu1), _ptr(nu2), _ptr(nuo), _ptr(resid))
    Z = Z[:km]
    R = R[:km]
    return IDResult(J=J[:kout].copy(), Z=np.asfortranarray(Z[:kout]), R=np.asfortranarray(R[:kout]), k=kout,
                    transposed=transposed, nu1=nu1, nu2=nu2, nuo=nuo, resid=resid,
                    a_norm=float(np.linalg.norm(W)))


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (for timing; results do not
    depend on it)."""
    _load().oracle_set_threads(int(n))


def threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().oracle_threads())


def matmul(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Plain FP64 product X @ Y computed by oracle.c."""
    X = np.asfortranarray(X, dtype=np.float64)
    Y = np.asfortranarray(Y, dtype=np.float64)
    m, p = X.shape
    p2, n = Y.shape
    assert p == p2
    out = np.zeros((m, n), order="F")
    _load().oracle_matmul(_ptr(X), max(m, 1), _ptr(Y), max(p, 1), _ptr(out), max(m, 1), m, p, n)
    return out


def skeleton(A: np.ndarray, res: IDResult) -> np.ndarray:
    """C = A[:, J] (or A[J, :]^T for the dual ID)."""
    W = np.asarray(A, dtype=np.float64)
    W = W.T if res.transposed else W
    return np.asfortranarray(W[:, res.J])


def error(A: np.ndarray, J: np.ndarray, Z: np.ndarray, transposed: bool = False) -> float:
    """||A - C Z||_F computed directly in FP64 (C = A[:, J])."""
    W = np.asarray(A, dtype=np.float64)
    W = W.T if transposed else W
    C = np.asfortranarray(W[:, np.asarray(J)])
    return float(np.linalg.norm(W - matmul(C, np.asarray(Z, dtype=np.float64))))


def rid(A: np.ndarray, Omega: np.ndarray, k: int) -> tuple[IDResult, np.ndarray]:
    """Randomized ID with a Gaussian row sketch: Y = Omega A in FP64, the ID
    oracle on Y picks J and T (from Y's R), and C = A[:, J].  Returns the
    ID result on Y and Y itself.  (The paper's Section 2.2 samples columns
    instead; this is the sketched variant whose CPQR stage is the same.)"""
    Y = matmul(np.asarray(Omega, dtype=np.float64), np.asarray(A, dtype=np.float64))
    return id(Y, k=k), Y


def rid_sample(A: np.ndarray, idx: np.ndarray, k: int) -> tuple[np.ndarray, np.ndarray, IDResult]:
    """The paper's randomized ID by column sampling (Section 2.2 and its
    Optim RID listing), with the random sample ``idx`` (p distinct column
    indices) an input: A_S = A[:, idx]; the column-pivoted QR of A_S,
    truncated after k steps (Section 4.1), selects k of its columns (no
    transpose, A_S is usually tall); cols = idx[selected], C = A[:, cols];
    R_k is the leading k x k triangle of A_S's factor, and Z solves
    R_k^T R_k Z = C^T A (eq. final_eq, over the full A): a forward
    substitution with the lower triangle R_k^T, then a back substitution with
    R_k (the paper hands R_k^T R_k to a symmetric-indefinite solver; the
    solution is the same).  Returns (cols, Z, the ID result of A_S)."""
    import scipy.linalg as sla
    A = np.asarray(A, dtype=np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    AS = np.asfortranarray(A[:, idx])
    res = _id_of(AS, False, k, None, None, None)
    cols = idx[res.J]
    Rk = res.R[:, res.J]          # R holds the rows in original order: R[:, J] = R11
    C = np.asfortranarray(A[:, cols])
    Y = sla.solve_triangular(Rk, matmul(C.T, A), trans="T", lower=False)   # R_k^T Y = C^T A
    Z = sla.solve_triangular(Rk, Y, lower=False)                           # R_k Z = Y
    return cols.astype(np.int32), Z, res


def two_sided(A: np.ndarray, k: int, force_J: np.ndarray | None = None, force_I: np.ndarray | None = None):
    """Two-sided ID, A ~ W A[I, J] Z (the variant the paper credits to Cheng
    et al. in its footnote to the ID's definition, Section 1.2): the column ID
    of A (Section 2.1, a column ID whatever the shape) gives J and Z; the row
    ID of its skeleton C = A[:, J] -- the paper's dual ID (Section 2's
    footnote), i.e. the column ID of C^T -- gives I and W = Z_2^T (m x k,
    W[I, :] = I_k).  ``force_J`` / ``force_I`` fix the pivots of the two
    stages (as ``force`` does for :func:`id`).  Returns (I, J, W, Z,
    column-stage result, row-stage result)."""
    A = np.asarray(A, dtype=np.float64)
    cres = _id_of(np.asfortranarray(A), False, k, None, None, force_J)
    C = A[:, cres.J]
    rres = _id_of(np.asfortranarray(C.T), False, k, None, None, force_I)
    return rres.J.copy(), cres.J.copy(), np.asfortranarray(rres.Z.T), cres.Z, cres, rres


def cur(A: np.ndarray, k: int, force_J: np.ndarray | None = None, force_I: np.ndarray | None = None):
    """CUR form of the two-sided ID: C = A[:, J], R = A[I, :] and U = Z R^+
    (the k x k matrix with U R closest to Z in the Frobenius norm, so that
    C U R ~ C Z), from the normal equations (R R^T) U^T = R Z^T solved by
    numpy's LAPACK solve.  ``force_J`` / ``force_I`` fix the two stages'
    pivots.  Returns (I, J, U)."""
    I, J, _, Z, _, _ = two_sided(A, k, force_J, force_I)
    R = np.asarray(A, dtype=np.float64)[I, :]
    Ut = np.linalg.solve(matmul(R, R.T), matmul(R, Z.T))
    return I, J, Ut.T


def batched(blocks, eps: float) -> list[IDResult]:
    """Tolerance-mode ID of every block (kmax = min(m_b, n_b))."""
    out = []
    for b in range(len(blocks.m)):
        out.append(id(blocks.block(b), eps=eps))
    return out


def id_vjp(A: np.ndarray, J: np.ndarray, Z: np.ndarray, gC: np.ndarray | None, gZ: np.ndarray | None) -> np.ndarray:
    """Gradient of a loss L(C, Z) with respect to A with the pivots J held
    fixed, C = A[:, J] and Z = C^+ A (so Z[:, J] = I, T = C^+ A_rest).

    With M = (C^T C)^{-1} Gz where Gz = gZ with its J columns zeroed:
        gA         = C M                      (all columns)
        gA[:, J]  += gC + A M^T - C (Z M^T + M Z^T)
    (the paper has no derivatives; this is the adjoint of the least-squares
    map, derived by differentiating T = (C^T C)^{-1} C^T A_rest).
    (C^T C)^{-1} is applied through the triangular factor of a QR of C.
    """
    A = np.asarray(A, dtype=np.float64)
    J = np.asarray(J)
    k = len(J)
    m, n = A.shape
    C = A[:, J]
    Gz = np.zeros((k, n)) if gZ is None else np.array(gZ, dtype=np.float64, copy=True)
    Gz[:, J] = 0.0
    import scipy.linalg as sla
    Rc = np.linalg.qr(C, mode="r")
    M = sla.solve_triangular(Rc, sla.solve_triangular(Rc, Gz, trans="T"))
    gA = C @ M
    extra = A @ M.T - C @ (Z @ M.T + M @ Z.T)
    if gC is not None:
        extra = extra + gC
    gA[:, J] += extra
    return gA
