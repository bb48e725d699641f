"""GPU parity of rid_sample_cpqr (the paper's randomized ID by column
sampling: CPQR of A[:, idx], Z by the normal equations over the full A)
against the FP64 oracle's ``rid_sample``.

Per case: the selected columns are the oracle's (inputs with separated
column norms), Z[:, J] is exactly the identity, and Z agrees with the
oracle's within the bar of the normal equations, c u kappa(R_k)^2 (they
square the condition number of C, in both implementations).
"""
from __future__ import annotations

import numpy as np
import pytest

import idgen
import oracle
from gpu_helpers import U32, U64, rel, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _miid():
    import paper_2105_07076_amd as miid
    miid.load()
    return miid


def _decaying(seed, m, n, q):
    g = idgen.rng(seed)
    return np.asfortranarray(g.standard_normal((m, n)) @ np.diag(q ** np.arange(n)))


def _z_bar(Rk, u):
    return max(1e-12, 256.0 * u * np.linalg.cond(Rk) ** 2)


@pytest.mark.parametrize("m,n,k", [(60, 300, 12), (200, 777, 40), (96, 130, 64), (33, 1000, 5)])
def test_rid_sample_fp64_matches_oracle(m, n, k):
    miid = _miid()
    A = _decaying(m + n + k, m, n, 0.97)
    idx = idgen.column_sample(m + k, n, k)
    r = miid.rid_sample(torch.tensor(A, device="cuda"), idx, k, want_R11=True)
    torch.cuda.synchronize()
    cols, Zref, res = oracle.rid_sample(A, idx, k)
    J = to_np(r.J)
    Z = to_np(r.Z)
    assert r.k == k
    assert list(J) == list(cols)
    assert np.array_equal(Z[:, J], np.eye(k))
    Rk = res.R[:, res.J]
    assert rel(to_np(r.R11), Rk) <= 1e-12
    assert rel(Z, Zref) <= _z_bar(Rk, U64), f"Z error {rel(Z, Zref):.3e}"
    # C = A[:, J] exactly
    assert np.array_equal(to_np(r.C), A[:, J])


def test_rid_sample_full_sample_equals_id():
    """Sampling every column reproduces the GPU's deterministic ID."""
    miid = _miid()
    A = _decaying(5, 64, 200, 0.9)
    A_t = torch.tensor(A, device="cuda")
    r = miid.rid_sample(A_t, np.arange(200), 16)
    d = miid.id(A_t, k=16)
    torch.cuda.synchronize()
    assert torch.equal(r.J, d.J)
    assert rel(to_np(r.Z), to_np(d.Z)) <= 1e-10


def test_rid_sample_fp32():
    miid = _miid()
    A = _decaying(7, 128, 600, 0.9)
    idx = idgen.column_sample(8, 600, 24)
    A_t = torch.tensor(A, dtype=torch.float32, device="cuda")
    r = miid.rid_sample(A_t, idx, 24)
    torch.cuda.synchronize()
    A32 = A_t.double().cpu().numpy()
    cols, Zref, res = oracle.rid_sample(A32, idx, 24)
    J = to_np(r.J)
    assert list(J) == list(cols)
    Z = to_np(r.Z).astype(np.float64)
    assert np.array_equal(Z[:, J], np.eye(24))
    assert rel(Z, Zref) <= _z_bar(res.R[:, res.J], U32)


def test_rid_sample_rank_deficient_sample():
    """A sample holding fewer nonzero columns than k: the CPQR of A_S stops
    (MIID_RANK_DEFICIENT) at k_out = 3; J beyond k_out is -1 and Z's rows
    there are zero; C Z reproduces A (its only nonzero columns are sampled)."""
    miid = _miid()
    g = idgen.rng(9)
    B = np.zeros((40, 90))
    keep = [5, 17, 33]
    B[:, keep] = g.standard_normal((40, 3))
    idx = np.array([60, 5, 71, 17, 2, 33], dtype=np.int32)
    r = miid.rid_sample(torch.tensor(B, device="cuda"), idx, 5)
    torch.cuda.synchronize()
    assert r.k == 3
    assert r.status & 1
    cols, Zref, _ = oracle.rid_sample(B, idx, 3)
    J = to_np(r.J)
    assert list(J) == list(cols)
    Zall = to_np(r.Z)
    assert np.linalg.norm(B - B[:, J] @ Zall[:3]) <= 1e-12 * np.linalg.norm(B)
    assert rel(Zall[:3], Zref) <= 1e-12


@pytest.mark.timeout(170)
def test_rid_sample_4096x16384_k256():
    """The FP64 4096 x 16384 workload with the paper's p = k + 0.2 k = 307:
    pivots against the oracle's CPQR of the sample; Z on 64 sampled columns
    against the oracle's normal equations for those columns."""
    miid = _miid()
    m, n, k = 4096, 16384, 256
    A_t = idgen.lowrank_plus_noise_device(2, m, n, np.exp(-np.arange(m) / 64.0), 1e-8, dtype=torch.float64)
    idx = idgen.column_sample(12, n, k)
    r = miid.rid_sample(A_t, idx, k)
    torch.cuda.synchronize()
    S = np.random.default_rng(13).choice(n, 64, replace=False)
    cat = np.concatenate([idx.astype(np.int64), S])
    A_small = A_t[:, torch.tensor(cat, device="cuda")].cpu().numpy()
    cols_s, Zs, res = oracle.rid_sample(A_small, np.arange(len(idx)), k)
    J = to_np(r.J)
    assert list(J) == [int(idx[c]) for c in cols_s]
    Z = to_np(r.Z)
    assert rel(Z[:, S], Zs[:, len(idx):]) <= _z_bar(res.R[:, res.J], U64)
    assert np.array_equal(Z[:, J], np.eye(k))
