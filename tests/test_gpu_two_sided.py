"""GPU parity of id_two_sided (A ~ W A[I, J] Z: the column ID of A, then the
row ID of its skeleton) against the oracle's ``two_sided``.

Per case: J margin-aware against the oracle's column stage; I margin-aware
against the oracle's row stage run on the GPU's own skeleton; Z and W within
the precision's bar of the oracle's (following the GPU's pivots); exact
identities W[I, :] and Z[:, J]; the two-sided error against the oracle's.
"""
from __future__ import annotations

import numpy as np
import pytest

import idgen
import oracle
from gpu_helpers import U32, U64, pivot_parity, rel, t_part, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _miid():
    import paper_2105_07076_amd as miid
    miid.load()
    return miid


def _col_parity(A64, J, k, u):
    """Column-stage parity on A as a column ID whatever its shape (a tall A
    is padded with zero columns so that the oracle does not take the dual)."""
    m, n = A64.shape
    W = np.hstack([A64, np.zeros((m, m - n))]) if m > n else A64
    return pivot_parity(W, J, k, u)


def _check(A64, r, k, u, tol):
    J, I = to_np(r.J), to_np(r.I)
    Z = to_np(r.Z).astype(np.float64)
    W = to_np(r.W).astype(np.float64)
    assert r.k == k and r.k_rows == k
    refc, _ = _col_parity(A64, J, k, u)
    assert np.array_equal(Z[:, J], np.eye(k))
    assert rel(t_part(Z, J), t_part(refc.Z[:, :A64.shape[1]], J)) <= tol(refc)
    # the row stage on the GPU's skeleton (the oracle's column ID of C^T)
    Ct = np.asfortranarray(A64[:, J].T)
    refr, _ = pivot_parity(Ct, I, k, u)
    assert np.array_equal(W[I, :], np.eye(k))
    assert rel(t_part(W.T, I), t_part(refr.Z, I)) <= tol(refr)
    # the two-sided error against the oracle's on the same index sets
    e = np.linalg.norm(A64 - W @ A64[np.ix_(I, J)] @ Z)
    e_ref = np.linalg.norm(A64 - refr.Z.T @ A64[np.ix_(I, J)] @ refc.Z[:, :A64.shape[1]])
    a = np.linalg.norm(A64)
    assert abs(e - e_ref) <= max(1e-10, 1e3 * u) * a, f"error {e:.6e} vs oracle {e_ref:.6e}"
    return e


@pytest.mark.parametrize("m,n,k", [(60, 300, 12), (300, 80, 20), (64, 64, 64), (257, 1000, 70), (33, 40, 33)])
def test_two_sided_fp64(m, n, k):
    miid = _miid()
    g = idgen.rng(m * 3 + n)
    A = g.standard_normal((m, n)) @ np.diag(0.97 ** np.arange(n))
    A = np.asfortranarray(np.diag(0.98 ** np.arange(m)) @ A)
    r = miid.two_sided(torch.tensor(A, device="cuda"), k)
    torch.cuda.synchronize()
    _check(A, r, k, U64, lambda ref: 1e-10)
    # against the oracle's own two-sided ID end to end, its two stages
    # following the GPU's pivots (equal to its own wherever the margins are
    # not declared near-ties, which _check asserted)
    Jg, Ig = to_np(r.J), to_np(r.I)
    I, J, W, Z, _, _ = oracle.two_sided(A, k, force_J=Jg, force_I=Ig)
    assert np.array_equal(J, Jg) and np.array_equal(I, Ig)
    assert rel(to_np(r.W), W) <= 1e-10 and rel(to_np(r.Z), Z) <= 1e-10


def test_two_sided_fp32():
    miid = _miid()
    g = idgen.rng(44)
    A = g.standard_normal((200, 700)) @ np.diag(0.98 ** np.arange(700))
    A_t = torch.tensor(A, dtype=torch.float32, device="cuda")
    A32 = A_t.double().cpu().numpy()
    r = miid.two_sided(A_t, 40)
    torch.cuda.synchronize()
    _check(A32, r, 40, U32, lambda ref: max(1e-5, 8.0 * U32 * np.linalg.cond(ref.R[:, ref.J])))


def test_two_sided_exact_rank_k():
    """A rank-k integer matrix: W A[I, J] Z reproduces it."""
    miid = _miid()
    A = idgen.integer_lowrank(8, 90, 150, 10)
    r = miid.two_sided(torch.tensor(A, device="cuda"), 10)
    torch.cuda.synchronize()
    J, I = to_np(r.J), to_np(r.I)
    M = to_np(r.W) @ A[np.ix_(I, J)] @ to_np(r.Z)
    assert np.linalg.norm(A - M) <= 1e-10 * np.linalg.norm(A)


def test_two_sided_rejects_tolerance_mode():
    import ctypes
    from paper_2105_07076_amd import _abi, api
    lib = _abi.load()
    opts = api._opts(None, 1e-3, 8, 0, True)
    assert lib.miid_two_sided_workspace(None, 16, 40, _abi.MIID_F64, ctypes.byref(opts)) == 0


def test_two_sided_4096x16384_k256():
    """The metric's matrix (FP64, 4096 x 16384, k = 256): J exactly the
    oracle's, I margin-aware on the GPU's skeleton, W against the oracle's row
    stage; C = A[:, J] has rank k, so its row ID is exact and the two-sided
    error equals the column stage's (checked on 256 sampled columns)."""
    miid = _miid()
    A_t = idgen.lowrank_plus_noise_device(2, 4096, 16384, np.exp(-np.arange(4096) / 64.0), 1e-8,
                                          dtype=torch.float64)
    r = miid.two_sided(A_t, 256)
    torch.cuda.synchronize()
    assert r.k == 256 and r.k_rows == 256
    J, I = to_np(r.J), to_np(r.I)
    A64 = A_t.cpu().numpy()
    ref = oracle.id(A64, k=256)
    assert np.array_equal(J, ref.J)
    Ct = np.asfortranarray(A64[:, J].T)
    refr, _ = pivot_parity(Ct, I, 256, U64)
    W = to_np(r.W)
    assert np.array_equal(W[I, :], np.eye(256))
    assert rel(t_part(W.T, I), t_part(refr.Z, I)) <= 1e-10
    g = idgen.rng(81)
    cols = np.sort(g.choice(16384, 256, replace=False))
    Z = to_np(r.Z)
    e2 = np.linalg.norm(A64[:, cols] - W @ A64[np.ix_(I, J)] @ Z[:, cols])
    e1 = np.linalg.norm(A64[:, cols] - A64[:, J] @ Z[:, cols])
    assert abs(e2 - e1) <= 1e-8 * np.linalg.norm(A64[:, cols])


# --------------------------------------------------------------------------
# CUR form: U = Z R^+ with R = A[I, :]
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,k", [(60, 300, 12), (300, 80, 20), (257, 1000, 70)])
def test_cur_fp64(m, n, k):
    """I, J as the two-sided ID's; U against the oracle's normal-equation U
    (bar c u kappa(R)^2); the CUR error against the oracle's."""
    miid = _miid()
    g = idgen.rng(m * 3 + n)
    A = g.standard_normal((m, n)) @ np.diag(0.97 ** np.arange(n))
    A = np.asfortranarray(np.diag(0.98 ** np.arange(m)) @ A)
    A_t = torch.tensor(A, device="cuda")
    I, J, U, st, st_rows = miid.cur(A_t, k)
    t = miid.two_sided(A_t, k)
    torch.cuda.synchronize()
    assert st == 0 and st_rows == 0
    assert torch.equal(I, t.I) and torch.equal(J, t.J)
    I, J, U = to_np(I), to_np(J), to_np(U)
    R = A[I, :]
    # the oracle's CUR with its stages following the GPU's pivots (the
    # two-sided test asserts those pivots margin-aware)
    oI, oJ, oU = oracle.cur(A, k, force_J=J, force_I=I)
    assert np.array_equal(I, oI) and np.array_equal(J, oJ)
    bar = max(1e-12, 256.0 * U64 * np.linalg.cond(R) ** 2)
    assert rel(U, oU) <= bar, f"U error {rel(U, oU):.3e} > {bar:.3e}"
    e = np.linalg.norm(A - A[:, J] @ U @ R)
    e_ref = np.linalg.norm(A - A[:, oJ] @ oU @ A[oI, :])
    assert abs(e - e_ref) <= 1e-9 * np.linalg.norm(A)


def test_cur_exact_rank_k_fp32():
    """A rank-k integer matrix in FP32: C U R reproduces it to FP32 rounding."""
    miid = _miid()
    A = idgen.integer_lowrank(9, 120, 200, 8)
    A_t = torch.tensor(A, dtype=torch.float32, device="cuda")
    I, J, U, st, st_rows = miid.cur(A_t, 8)
    torch.cuda.synchronize()
    I, J, U = to_np(I), to_np(J), to_np(U).astype(np.float64)
    M = A[:, J] @ U @ A[I, :]
    assert np.linalg.norm(A - M) <= 1e-4 * np.linalg.norm(A)
