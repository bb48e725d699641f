"""The paper's experiments reshaped as GPU parity sweeps (Section 3 and
Appendix A): the synthetic Boolean, Gaussian and Uniform 784 x 1000 datasets
over k = 10, 30, ..., 470, through the deterministic ID (FP64) and the
column-sampling randomized ID (FP64, p = k + floor(0.2 k)), against the
oracle step by step; at k = 190 also against the values the paper prints
(Table 2's relative errors, Table 1's max |Z|).  The sparse datasets are
stand-ins with the paper's shapes and nonzero counts (the matrices are not
available), checked for parity and for the bound on Z the paper reports for
the deterministic ID (entries at most 2).
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import idgen
import oracle
from gpu_helpers import U64, pivot_parity, rel, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KS = list(range(10, 471, 20))
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables_synthetic.json")


def _miid():
    import paper_2105_07076_amd as miid
    miid.load()
    return miid


def _table():
    with open(GOLDEN) as f:
        return json.load(f)


def _column_parity(W, J_pos, k):
    """Margin-aware parity of the column CPQR of W (any shape): padded with
    zero columns to at least as many columns as rows, so that the oracle takes
    the column ID; a zero column is never picked ahead of a nonzero residual."""
    m, n = W.shape
    Wp = np.hstack([W, np.zeros((m, max(0, m - n)))]) if n < m else W
    return pivot_parity(Wp, J_pos, k, U64)


@pytest.mark.parametrize("name", ["boolean", "gaussian", "uniform"])
def test_sweep_deterministic_id(name):
    """Every k of the sweep: pivots margin-aware against the oracle (the
    Boolean set has exact ties in its column norms), the ID's error equal to
    the oracle's residual norm at k, Z[:, J] = I; at k = 190 the paper's
    Table 2 error and Table 1 max |Z| = 1."""
    miid = _miid()
    tab = _table()
    A = idgen.paper_dataset(name, seed=0)
    A_t = torch.tensor(A, device="cuda")
    a = np.linalg.norm(A)
    ties_total = 0
    for k in KS:
        r = miid.id(A_t, k=k)
        torch.cuda.synchronize()
        J = to_np(r.J)
        Z = to_np(r.Z)
        assert r.k == k
        ref, ties = pivot_parity(A, J, k, U64)
        ties_total += ties
        assert np.array_equal(Z[:, J], np.eye(k))
        e = oracle.error(A, J, Z)
        assert abs(e - ref.resid[k]) <= 1e-10 * a, f"k={k}: error {e:.12e} vs oracle {ref.resid[k]:.12e}"
        if k == tab["k"]:
            assert abs(e / a - tab["rows"][name]["id_rel_error"]) <= tab["abs_tol"]
            assert np.abs(Z).max() <= tab["rows"][name]["id_max_abs_Z"] * (1.0 + 1e-12)
    if name != "boolean":
        assert ties_total == 0


@pytest.mark.parametrize("name", ["boolean", "gaussian", "uniform"])
def test_sweep_column_sampling_rid(name):
    """Every k of the sweep with a fresh sample: the selected columns margin-
    aware against the oracle's CPQR of A[:, idx], Z against FP64 least squares
    on the GPU's skeleton, the error against the oracle's for that skeleton."""
    miid = _miid()
    A = idgen.paper_dataset(name, seed=0)
    A_t = torch.tensor(A, device="cuda")
    a = np.linalg.norm(A)
    for k in KS:
        idx = idgen.column_sample(1000 + k, A.shape[1], k)
        r = miid.rid_sample(A_t, idx, k)
        torch.cuda.synchronize()
        J = to_np(r.J)
        Z = to_np(r.Z)
        assert r.k == k
        pos = np.array([int(np.where(idx == j)[0][0]) for j in J], dtype=np.int32)
        ref, _ = _column_parity(A[:, idx], pos, k)
        assert np.array_equal(Z[:, J], np.eye(k))
        C = A[:, J]
        Zref = np.linalg.lstsq(C, A, rcond=None)[0]
        Rk = ref.R[:, ref.J]
        bar = max(1e-12, 256.0 * U64 * np.linalg.cond(Rk) ** 2)
        assert rel(Z, Zref) <= bar, f"k={k}: Z error {rel(Z, Zref):.3e} > {bar:.3e}"
        e = oracle.error(A, J, Z)
        e_ref = oracle.error(A, J, Zref)
        assert abs(e - e_ref) <= 1e-10 * a


@pytest.mark.parametrize("name", ["boolean", "gaussian", "uniform"])
def test_table_k190_optim_rid(name):
    """Table 2's Optim RID error and Table 1's max |Z| at k = 190: means over
    the paper's 10 runs, each run on the GPU."""
    miid = _miid()
    tab = _table()
    row = tab["rows"][name]
    k = tab["k"]
    A = idgen.paper_dataset(name, seed=0)
    A_t = torch.tensor(A, device="cuda")
    errs, zmax = [], []
    for run in range(tab["rid_runs"]):
        idx = idgen.column_sample(100 + run, A.shape[1], k)
        r = miid.rid_sample(A_t, idx, k)
        torch.cuda.synchronize()
        Z = to_np(r.Z)
        errs.append(oracle.error(A, to_np(r.J), Z) / np.linalg.norm(A))
        zmax.append(np.abs(Z).max())
    assert abs(np.mean(errs) - row["rid_rel_error"]) <= tab["abs_tol"]
    assert abs(np.mean(zmax) - row["rid_max_abs_Z"]) <= 5e-4


@pytest.mark.parametrize("name", ["sparse1", "sparse2", "sparse3"])
def test_sparse_standins(name):
    """k = 190 on the sparse stand-ins: deterministic ID in parity with the
    oracle and its Z bounded by 2 (the paper's observation for its ID on every
    dataset); the column-sampling RID in parity with the oracle on the same
    sample (its Z is not bounded by 1 in general on sparse inputs)."""
    miid = _miid()
    A = idgen.sparse_standin(name, seed=0)
    A_t = torch.tensor(A, device="cuda")
    k = 190
    r = miid.id(A_t, k=k)
    torch.cuda.synchronize()
    J, Z = to_np(r.J), to_np(r.Z)
    ref, _ = pivot_parity(A, J, k, U64)
    assert abs(oracle.error(A, J, Z) - ref.resid[k]) <= 1e-10 * np.linalg.norm(A)
    assert np.abs(Z).max() <= 2.0
    idx = idgen.column_sample(7, A.shape[1], k)
    rs = miid.rid_sample(A_t, idx, k)
    torch.cuda.synchronize()
    Js, Zs = to_np(rs.J), to_np(rs.Z)
    pos = np.array([int(np.where(idx == j)[0][0]) for j in Js], dtype=np.int32)
    ref_s, _ = _column_parity(A[:, idx], pos, k)
    Zref = np.linalg.lstsq(A[:, Js], A, rcond=None)[0]
    bar = max(1e-12, 256.0 * U64 * np.linalg.cond(ref_s.R[:, ref_s.J]) ** 2)
    assert rel(Zs, Zref) <= bar
