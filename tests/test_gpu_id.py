"""GPU parity of id_cpqr (deterministic ID) against the FP64 oracle.

Bar: pivots identical to the oracle (margin-aware in FP32, see
gpu_helpers.pivot_parity); Z[:, J] exactly the identity; T within 1e-12
(FP64) / 1e-5 (FP32) relative in the Frobenius norm; C = A[:, J] exactly.
"""
from __future__ import annotations

import numpy as np
import pytest

import idgen
import oracle
from gpu_helpers import U32, U64, pivot_parity, rel, t_part, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}
UW = {torch.float64: U64, torch.float32: U32}


def kappa_tol(ref, dtype, floor):
    """Bar for T: the fixed tolerance, widened to 8 u kappa_2(R11) when R11 is
    ill conditioned (a backward-stable QR + triangular solve has forward
    error ~ u kappa in T).  The 4096 x 16384 workload keeps the fixed bar."""
    R11 = ref.R[:, ref.J]
    kap = np.linalg.cond(R11) if ref.k > 0 else 1.0
    return max(floor, 8.0 * UW[dtype] * kap)


@pytest.fixture(params=["fused", "blocked"])
def path(request):
    """The PATH hint for the call: matrices of at most 576 rows (FP32) / 320
    (FP64) take the fused one-launch-per-step kernel unless the hint asks for
    the two-launch blocked path."""
    from paper_2105_07076_amd import _abi
    return _abi.hint(_abi.MIID_HINT_PATH_SHIFT, 2 if request.param == "fused" else 1)


def _miid():
    import paper_2105_07076_amd as miid
    miid.load()
    return miid


def _check_id(A_np, k, dtype, nb=0, exact_pivots=True, tol=None, refine=True, hints=0):
    miid = _miid()
    A_t = torch.tensor(A_np, dtype=dtype, device="cuda")
    A64 = A_t.double().cpu().numpy()          # exactly the numbers the GPU factors
    r = miid.id(A_t, k=k, nb=nb, refine=refine, hints=hints)
    torch.cuda.synchronize()
    J = to_np(r.J)
    Z = to_np(r.Z).astype(np.float64)
    assert r.k == min(k, *A64.shape)
    if exact_pivots:
        ref = oracle.id(A64, k=k)
        assert list(J) == list(ref.J)
        ties = 0
    else:
        ref, ties = pivot_parity(A64.T if r.transposed else A64, J, k, UW[dtype])
    assert np.array_equal(Z[:, J], np.eye(r.k))
    e = rel(t_part(Z, J), t_part(ref.Z, J))
    bar = kappa_tol(ref, dtype, tol or TOL[dtype])
    assert e <= bar, f"T relative error {e:.3e} > {bar:.3e}"
    C = to_np(r.C)
    W = A64.T if r.transposed else A64
    assert np.array_equal(C.astype(np.float64), W[:, J])
    return r, ref, ties


def test_cfg1_fp64(path):
    A, k = idgen.cfg1()
    r, ref, _ = _check_id(A, k, torch.float64, hints=path)
    # the last steps' residuals (~2^-16 of the columns' norms) cancel in the
    # downdate: those norms are recomputed, and the pivots still equal the
    # oracle's exact-norm pivots
    assert r.n_recompute > 0
    e_gpu = oracle.error(A, to_np(r.J), to_np(r.Z))
    e_ora = oracle.error(A, ref.J, ref.Z)
    assert abs(e_gpu - e_ora) <= 1e-6 * e_ora
    assert r.r22_norm == pytest.approx(ref.r22, rel=1e-3)
    assert r.a_norm == pytest.approx(np.linalg.norm(A), rel=1e-12)


@pytest.mark.parametrize("nb", [1, 5, 32, 64])
def test_cfg1_panel_widths(nb, path):
    A, k = idgen.cfg1()
    _check_id(A, k, torch.float64, nb=nb, hints=path)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,n,k,nb", [(37, 101, 9, 4), (128, 128, 40, 16), (200, 1000, 64, 32),
                                      (300, 700, 100, 64), (65, 4099, 30, 8)])
def test_planted(dtype, m, n, k, nb, path):
    A, planted, U, perm = idgen.planted_id(100 + m, m, n, k, r=0.9)
    r, ref, _ = _check_id(A, k, dtype, nb=nb, hints=path)
    assert list(to_np(r.J)) == list(planted)
    T = to_np(r.Z).astype(np.float64)[:, perm[k:]]
    assert rel(T, U) <= (1e-10 if dtype == torch.float64 else kappa_tol(ref, dtype, 1e-5))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (1, 9, 1), (2, 3, 2), (63, 64, 20), (64, 64, 64),
                                   (65, 130, 33), (257, 511, 70), (129, 2000, 128)])
def test_random_shapes(dtype, m, n, k, path):
    g = idgen.rng(7 * m + n)
    A = g.standard_normal((m, n)) * (0.97 ** np.arange(n))[None, :]
    _check_id(A, k, dtype, exact_pivots=False, hints=path)


@pytest.mark.parametrize("m", [289, 320])
def test_fp64_fused_tallest(m, path):
    # 289..320 rows in FP64: ten 16-byte groups per lane of a column group on
    # the fused path; planted so that the pivots are exact
    A, planted, U, perm = idgen.planted_id(11 + m, m, 1500, 96, r=0.93)
    r, ref, _ = _check_id(A, 96, torch.float64, hints=path)
    assert list(to_np(r.J)) == list(planted)


@pytest.mark.parametrize("dtype,m", [(torch.float32, 400), (torch.float64, 300)])
def test_fused_four_passes_tall_columns(dtype, m, path):
    # 20000 columns: four column passes per wave on the fused path; 400 FP32
    # rows (nine 16-byte groups per lane) and 300 FP64 rows (ten) load their
    # per-column data after the dot products
    A, planted, U, perm = idgen.planted_id(31 + m, m, 20000, 64, r=0.95)
    r, ref, _ = _check_id(A, 64, dtype, hints=path)
    assert list(to_np(r.J)) == list(planted)


def test_dual_tall_matrix(path):
    g = idgen.rng(9)
    A = g.standard_normal((300, 120)) @ np.diag(0.93 ** np.arange(120))
    r, ref, _ = _check_id(A, 40, torch.float64, hints=path)
    assert r.transposed
    assert ref.transposed


def test_full_rank():
    g = idgen.rng(6)
    A = g.standard_normal((48, 100))
    r, ref, _ = _check_id(A, 48, torch.float64, exact_pivots=False)
    assert oracle.error(A, to_np(r.J), to_np(r.Z)) <= 1e-12 * np.linalg.norm(A)


def test_rank_deficient_stops(path):
    miid = _miid()
    A = idgen.diag_case(np.array([5.0, 0.0, 3.0, 0.0, 2.0, 0.0]), 10)
    A[:, 7] = 2.0 * A[:, 0]
    r = miid.id(torch.tensor(A, device="cuda"), k=6, hints=path)
    assert r.k == 3
    assert r.status & 1
    assert list(to_np(r.J)) == [7, 2, 4]


def test_nonfinite_input(path):
    miid = _miid()
    A = np.ones((20, 30))
    A[3, 4] = np.nan
    r = miid.id(torch.tensor(A, device="cuda"), k=5, hints=path)
    assert r.k == 0
    assert r.status & 2


def test_tolerance_mode(path):
    miid = _miid()
    A, _ = idgen.cfg1()
    a = np.linalg.norm(A)
    for eps in [1e-1, 1e-3, 1e-6]:
        r = miid.id(torch.tensor(A, device="cuda"), eps=eps, kmax=64, hints=path)
        ref = oracle.id(A, eps=eps, kmax=64)
        assert abs(r.k - ref.k) <= 1
        if r.k != ref.k:   # only where the oracle's residual sits within 1% of eps ||A||
            kk = min(r.k, ref.k)
            assert abs(ref.resid[kk] - eps * a) <= 0.01 * eps * a
        assert oracle.error(A, to_np(r.J), to_np(r.Z)) <= 1.01 * eps * a


def test_deterministic_repeat():
    miid = _miid()
    A, k = idgen.cfg1()
    A_t = torch.tensor(A, device="cuda")
    outs = [miid.id(A_t, k=k) for _ in range(3)]
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert torch.equal(o.J, outs[0].J)
        assert torch.equal(o.Z, outs[0].Z)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_cfg2_reduced(dtype, path):
    A, k = idgen.cfg2(m=1024, n=4096)
    _check_id(A, k, dtype, exact_pivots=(dtype == torch.float64), hints=path)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_cfg2_full_size(dtype):
    """4096 x 16384, k = 256: the benchmarked launch configuration."""
    A_t = idgen.lowrank_plus_noise_device(2, 4096, 16384, np.exp(-np.arange(4096) / 64.0), 1e-8,
                                          dtype=dtype)
    A64 = A_t.double().cpu().numpy()
    miid = _miid()
    r = miid.id(A_t, k=256)
    torch.cuda.synchronize()
    J = to_np(r.J)
    Z = to_np(r.Z).astype(np.float64)
    ref, ties = pivot_parity(A64, J, 256, UW[dtype])
    if dtype == torch.float64:
        assert ties == 0
    assert np.array_equal(Z[:, J], np.eye(256))
    T_gpu, T_ora = t_part(Z, J), t_part(ref.Z, J)
    e = rel(T_gpu, T_ora)
    assert e <= TOL[dtype], f"T relative error {e:.3e}"
    # element by element: no entry off by more than the bar relative to T's
    # largest entry
    emax = float(np.max(np.abs(T_gpu - T_ora)) / np.max(np.abs(T_ora)))
    assert emax <= TOL[dtype], f"largest entry error {emax:.3e} of max|T|"


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_exact_tie_lowest_index(dtype, path):
    """Columns 1 and 3 have exactly the same norm (5): the pivot is the lower
    index.  Then the same for a batched block."""
    miid = _miid()
    A = np.array([[1.0, 3.0, 0.0, 4.0], [0.0, 4.0, 1.0, 3.0]])
    r = miid.id(torch.tensor(A, dtype=dtype, device="cuda"), k=1, hints=path)
    torch.cuda.synchronize()
    assert list(to_np(r.J)) == [1]
    assert list(oracle.id(A, k=1).J) == [1]
    packed = torch.tensor(np.asfortranarray(A).T.reshape(-1), dtype=dtype, device="cuda")
    rb = miid.batched(packed, [0], [2], [4], 0.0, 1)
    assert rb.k[0] == 1 and list(rb.block(0)[0]) == [1]
