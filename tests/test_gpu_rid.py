"""GPU parity of rid_sketch_cpqr (randomized ID with a bfloat16 Gaussian row
sketch on the matrix cores) against the FP64 oracle.

Three checks per case:
  * the sketch: Y_gpu vs Y64 = Omega A in FP64 on the same (bf16-exact)
    Omega and the same FP32 A, normwise;
  * the CPQR stage: the oracle run on the GPU's own Y (promoted) must give the
    same pivots (margin-aware, FP32) and T within the FP32 bar;
  * end to end: ||A - C Z||_F in FP64 against the oracle's randomized ID with
    an exact FP64 sketch (split form within 1e-5 relative).
"""
from __future__ import annotations

import numpy as np
import pytest

import idgen
import oracle
from gpu_helpers import U32, pivot_parity, rel, t_part, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# bf16 hi+lo represents a to ~2^-17 relative; FP32 accumulation over m terms
# adds ~sqrt(m) 2^-24.  A single bf16 rounding is ~2^-9.
# normwise relative error of Y against the FP64 product: mode 0 rounds A to
# bfloat16 once (2^-8 per entry), mode 1 splits it in two parts (2^-16), mode
# 2 in three (2^-24, FP32's unit roundoff: what is left is the FP32
# accumulation over K terms, about sqrt(K) u32 <= 8e-6 for K <= 16384)
SKETCH_TOL = {2: 1e-5, 1: 3e-5, 0: 6e-3}


def _miid():
    import paper_2105_07076_amd as miid
    miid.load()
    return miid


def _run(A_np, l, k, mode, seed=77, nb=0, hints=0):
    miid = _miid()
    m, n = A_np.shape
    A_t = torch.tensor(A_np, dtype=torch.float32, device="cuda")
    A64 = A_t.double().cpu().numpy()
    Om = idgen.omega_bf16(seed, l, m)
    Om_t = torch.tensor(Om, dtype=torch.bfloat16, device="cuda")
    r = miid.rid(A_t, Om_t, k=k, mode=mode, want_Y=True, nb=nb, hints=hints)
    torch.cuda.synchronize()
    return r, A64, Om.astype(np.float64)


def _check(A_np, l, k, mode, e2e_tol=None, nb=0, hints=0):
    r, A64, Om = _run(A_np, l, k, mode, nb=nb, hints=hints)
    Y = to_np(r.Y).astype(np.float64)
    Y64 = oracle.matmul(Om, A64)
    ey = rel(Y, Y64)
    assert ey <= SKETCH_TOL[mode], f"sketch error {ey:.3e}"
    J = to_np(r.J)
    Z = to_np(r.Z).astype(np.float64)
    assert r.k == k
    # CPQR stage on the GPU's own Y
    ref, ties = pivot_parity(Y, J, k, U32)
    assert np.array_equal(Z[:, J], np.eye(k))
    R11 = ref.R[:, ref.J]
    bar = max(1e-5, 8.0 * U32 * np.linalg.cond(R11))
    et = rel(t_part(Z, J), t_part(ref.Z, J))
    assert et <= bar, f"T error {et:.3e} > {bar:.3e}"
    # C = A[:, J] exactly
    assert np.array_equal(to_np(r.C).astype(np.float64), A64[:, J])
    # end to end against the exact-sketch oracle
    e_gpu = oracle.error(A64, J, Z)
    if e2e_tol is not None:
        ore, _ = oracle.rid(A64, Om, k)
        e_ora = oracle.error(A64, ore.J, ore.Z)
        assert abs(e_gpu - e_ora) <= e2e_tol * e_ora, f"e2e {e_gpu:.6e} vs {e_ora:.6e}"
    return r, e_gpu, ties


@pytest.mark.parametrize("mode", [2, 1, 0])
@pytest.mark.parametrize("m,n,l,k", [(64, 200, 26, 16), (100, 333, 50, 40), (257, 1000, 74, 64),
                                     (33, 65, 33, 20),
                                     # one 32-row chunk of K (the second K group has none), a
                                     # ragged one, 9 row tiles exactly (two K groups), 10 (one
                                     # group, five tiles per wave) and 19 (eight per wave)
                                     (5, 40, 5, 3), (31, 90, 12, 8), (300, 1200, 288, 200),
                                     (320, 1000, 300, 250), (640, 1400, 600, 400),
                                     # 13 row tiles on two-by-two waves of nine; at least 65409
                                     # columns (two 128-column workgroups per CU) with 2 tiles
                                     (600, 2000, 400, 300), (64, 65536, 40, 30)])
def test_rid_small(mode, m, n, l, k):
    g = idgen.rng(m * 7 + n)
    A = g.standard_normal((m, n)) @ np.diag(0.97 ** np.arange(n))
    _check(A, l, k, mode, e2e_tol={2: 1e-5, 1: 1e-4}.get(mode))


def test_rid_exact_for_rank_k():
    A = idgen.integer_lowrank(5, 80, 300, 12).astype(np.float32).astype(np.float64)
    r, e, _ = _check(A, 22, 12, 1)
    assert e <= 1e-4 * np.linalg.norm(A)


def test_rid_planted_rank_k():
    """A planted rank-k input: a random sketch does not keep the planted pivot
    order, but any k columns it picks reconstruct A (rank k, k <= l)."""
    A, planted, U, perm = idgen.planted_id(9, 120, 500, 20, r=0.9)
    r, e, ties = _check(A, 30, 20, 1)
    assert e <= 1e-4 * np.linalg.norm(A)


def test_rid_unaligned_lda():
    """A column-major view with an odd leading dimension takes the scalar path."""
    miid = _miid()
    g = idgen.rng(3)
    big = torch.tensor(g.standard_normal((101, 400)), dtype=torch.float32, device="cuda")
    A_t = big.t().contiguous().t()[:99]          # 99 x 400, lda = 101
    Om = torch.tensor(idgen.omega_bf16(4, 30, 99), dtype=torch.bfloat16, device="cuda")
    r = miid.rid(A_t, Om, k=20, want_Y=True)
    A64 = A_t.double().cpu().numpy()
    Y64 = oracle.matmul(Om.double().cpu().numpy(), A64)
    assert rel(to_np(r.Y).astype(np.float64), Y64) <= SKETCH_TOL[1]


@pytest.mark.parametrize("mode", [2, 1])
@pytest.mark.parametrize("path", [2, 1])
def test_rid_cfg2_reduced(path, mode):
    """cfg2 construction at 1024 x 4096, k = 256, l = k + 10, through the
    fused one-launch-per-step CPQR (default for the sketch, PATH hint 2) and
    the blocked two-launch one (PATH hint 1).  End to end against the
    exact-sketch oracle: within 1e-5 with the three-part split (mode 2), whose
    sketch is as accurate as FP32 accumulation; with the two-part split (mode
    1) the ID's error moves with the sketch's own perturbation, checked at the
    sketch's error bar."""
    from paper_2105_07076_amd import _abi
    A, k = idgen.cfg2(m=1024, n=4096)
    _check(A, k + 10, k, mode, e2e_tol=1e-5 if mode == 2 else SKETCH_TOL[1],
           hints=_abi.hint(_abi.MIID_HINT_PATH_SHIFT, path))


def test_rid_cfg2_full_size():
    """4096 x 16384, k = 256, l = 266, split sketch: the benchmarked launch."""
    miid = _miid()
    A_t = idgen.lowrank_plus_noise_device(2, 4096, 16384, np.exp(-np.arange(4096) / 64.0), 1e-8,
                                          dtype=torch.float32)
    Om = idgen.omega_bf16(77, 266, 4096)
    Om_t = torch.tensor(Om, dtype=torch.bfloat16, device="cuda")
    r = miid.rid(A_t, Om_t, k=256, mode=1, want_Y=True)
    torch.cuda.synchronize()
    A64 = A_t.double().cpu().numpy()
    Y = to_np(r.Y).astype(np.float64)
    Y64 = oracle.matmul(Om.astype(np.float64), A64)
    assert rel(Y, Y64) <= SKETCH_TOL[1]
    J = to_np(r.J)
    Z = to_np(r.Z).astype(np.float64)
    ref, ties = pivot_parity(Y, J, 256, U32)
    T_gpu, T_ora = t_part(Z, J), t_part(ref.Z, J)
    assert rel(T_gpu, T_ora) <= 1e-5
    # element by element, relative to T's largest entry: the forward error of
    # a backward-stable QR + triangular solve, ~ u kappa_2(R11), with the
    # normwise bar as its floor
    bar = max(1e-5, 8.0 * U32 * np.linalg.cond(ref.R[:, ref.J]))
    emax = float(np.max(np.abs(T_gpu - T_ora)) / np.max(np.abs(T_ora)))
    assert emax <= bar, f"largest entry error {emax:.3e} of max|T|, bar {bar:.3e}"
    ore, _ = oracle.rid(A64, Om.astype(np.float64), 256)
    e_gpu = oracle.error(A64, J, Z)
    e_ora = oracle.error(A64, ore.J, ore.Z)
    assert abs(e_gpu - e_ora) <= 1e-5 * e_ora


@pytest.mark.timeout(900)
def test_rid_16384x65536_k512():
    """The large randomized workload: A 16384 x 65536 FP32 (s_i = exp(-i/128),
    4096 singular triplets, noise 1e-8), Omega 522 x 16384, k = 512, split
    sketch.  Sampled sketch entries against FP64 dot products; the CPQR stage
    against the oracle on the GPU's own Y; end to end against the exact-sketch
    oracle: Y64 = Omega A in FP64 built on the host in column chunks (the
    oracle's randomized ID is the ID of that Y), pivots margin-aware at the
    sketch's error level, and the error on 256 sampled columns within 1e-5
    (relative) of the oracle's."""
    import time
    miid = _miid()
    m, n, l, k = 16384, 65536, 522, 512
    A_t = idgen.lowrank_plus_noise_device(3, m, n, np.exp(-np.arange(4096) / 128.0), 1e-8, r=4096,
                                          dtype=torch.float32)
    Om = idgen.omega_bf16(78, l, m)
    Om_t = torch.tensor(Om, dtype=torch.bfloat16, device="cuda")
    r = miid.rid(A_t, Om_t, k=k, mode=1, want_Y=True)
    torch.cuda.synchronize()
    assert r.k == k
    Y = to_np(r.Y).astype(np.float64)
    g = idgen.rng(79)
    cols = np.sort(g.choice(n, 256, replace=False))
    Acols = A_t[:, torch.tensor(cols, device="cuda")].double().cpu().numpy()
    Om64 = Om.astype(np.float64)
    assert rel(Y[:, cols], Om64 @ Acols) <= SKETCH_TOL[1]
    J = to_np(r.J)
    Z = to_np(r.Z).astype(np.float64)
    ref, ties = pivot_parity(Y, J, k, U32)
    R11 = ref.R[:, ref.J]
    bar = max(1e-5, 8.0 * U32 * np.linalg.cond(R11))
    assert rel(t_part(Z, J), t_part(ref.Z, J)) <= bar
    C = A_t[:, torch.tensor(J.astype(np.int64), device="cuda")].double().cpu().numpy()
    err = np.linalg.norm(Acols - C @ Z[:, cols]) / np.linalg.norm(Acols)
    tail = np.exp(-k / 128.0)
    assert 0.5 * tail <= err <= 10.0 * tail, f"sampled relative error {err:.3e}, tail {tail:.3e}"
    # the exact sketch: Omega's entries are bfloat16 and A's FP32, so each
    # product is exact in FP64; numpy's product (pinned to oracle.matmul)
    t0 = time.time()
    Y64 = np.empty((l, n))
    for c0 in range(0, n, 4096):
        Y64[:, c0:c0 + 4096] = Om64 @ A_t[:, c0:c0 + 4096].double().cpu().numpy()
    ora = oracle.id(Y64, k=k)
    t1 = time.time()
    # pivots: margin-aware against the exact sketch, at the split sketch's
    # error level (its normwise bound stands in for the working precision)
    _, ties64 = pivot_parity(Y64, J, k, SKETCH_TOL[1])
    Co = A_t[:, torch.tensor(ora.J.astype(np.int64), device="cuda")].double().cpu().numpy()
    e_ora = np.linalg.norm(Acols - Co @ ora.Z[:, cols]) / np.linalg.norm(Acols)
    same = len(set(int(x) for x in J) & set(int(x) for x in ora.J))
    print(f"\n[cfg3] sampled error gpu {err:.6e} oracle {e_ora:.6e} (rel diff {abs(err - e_ora) / e_ora:.2e}); "
          f"{same}/{k} columns shared, {ties64} declared near-ties vs the exact sketch; host oracle "
          f"{t1 - t0:.1f} s", flush=True)
    assert abs(err - e_ora) <= 1e-5 * e_ora, f"sampled error {err:.6e} vs oracle {e_ora:.6e}"


# --------------------------------------------------------------------------
# least-squares Z over the full A (MIID_LSTSQ_Z): the sketch's skeleton as the
# column sample of the paper's Z construction, Z = C^+ A
# --------------------------------------------------------------------------
def _lstsq_pair(A_t, Om_t, k, mode=1):
    miid = _miid()
    rs = miid.rid(A_t, Om_t, k=k, mode=mode)
    rl = miid.rid(A_t, Om_t, k=k, mode=mode, lstsq=True, want_R11=True)
    torch.cuda.synchronize()
    return rs, rl


def _check_lstsq_against_oracle(A64, Js, rl, k, cols=None):
    """The least-squares pass for the sketch's skeleton Js: the same J in the
    same order, R11 the Cholesky factor of C^T C (R11^T R11 = C^T C, upper
    triangular, positive diagonal), Z = C^+ A against the oracle's
    column-sampling RID run with Js as its whole sample (the paper's
    normal-equation Z; its rows follow its own pivot order, mapped back here)
    within the normal equations' bar c u kappa(C)^2."""
    J = to_np(rl.J)
    assert np.array_equal(J, Js)
    m, n = A64.shape
    S = np.arange(n) if cols is None else np.asarray(cols)
    C = A64[:, J]
    R = to_np(rl.R11)
    assert np.array_equal(R, np.triu(R)) and np.all(np.diag(R) > 0)
    assert rel(R.T @ R, C.T @ C) <= 1e-12
    kap = np.linalg.cond(C)
    # the oracle on the columns J followed by the checked ones: Z restricted
    # to a set of columns is the same least-squares solve
    Wc = np.hstack([C, A64[:, S]])
    oc, Zo, _ = oracle.rid_sample(Wc, np.arange(k), k)
    Zref = np.empty((k, len(S)))
    Zref[np.asarray(oc)] = Zo[:, k:]
    Z = to_np(rl.Z).astype(np.float64)
    assert np.array_equal(Z[:, J], np.eye(k))
    bar = max(1e-5, 256.0 * U32 * kap ** 2)
    assert rel(Z[:, S], Zref) <= bar, f"Z error {rel(Z[:, S], Zref):.3e} > {bar:.3e}"


@pytest.mark.parametrize("m,n,l,k", [(64, 200, 26, 16), (100, 333, 50, 40), (257, 1000, 74, 64)])
def test_rid_lstsq_matches_oracle(m, n, l, k):
    g = idgen.rng(m * 5 + n)
    A = g.standard_normal((m, n)) @ np.diag(0.97 ** np.arange(n))
    A_t = torch.tensor(A, dtype=torch.float32, device="cuda")
    A64 = A_t.double().cpu().numpy()
    Om_t = torch.tensor(idgen.omega_bf16(m + 3, l, m), dtype=torch.bfloat16, device="cuda")
    rs, rl = _lstsq_pair(A_t, Om_t, k)
    assert rl.k == k
    Js = to_np(rs.J)
    _check_lstsq_against_oracle(A64, Js, rl, k)
    # C = A[:, J] exactly, and Z is the best for this skeleton: no larger
    # error than T from the sketch, column by column
    J = to_np(rl.J)
    assert np.array_equal(to_np(rl.C).astype(np.float64), A64[:, J])
    el = np.linalg.norm(A64 - A64[:, J] @ to_np(rl.Z).astype(np.float64), axis=0)
    es = np.linalg.norm(A64 - A64[:, Js] @ to_np(rs.Z).astype(np.float64), axis=0)
    _no_worse(el, es, np.linalg.norm(A64, axis=0))


def _no_worse(el, es, anorm):
    """Least squares is optimal for the skeleton: no larger error than T from
    the sketch, in total and column by column up to FP32 rounding."""
    assert np.linalg.norm(el) <= np.linalg.norm(es) * (1.0 + 1e-4)
    assert np.all(el <= es + 1e-3 * anorm)


def test_rid_lstsq_rejects_tolerance_mode():
    miid = _miid()
    A_t = torch.ones((16, 40), dtype=torch.float32, device="cuda")
    Om_t = torch.ones((8, 16), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(ValueError):
        miid.rid(A_t, Om_t, eps=1e-3, lstsq=True)


def test_rid_lstsq_cfg2_full_size():
    """4096 x 16384, k = 256, l = 266 with Z = C^+ A: Z on 64 sampled columns
    against FP64 least squares on the GPU's skeleton; per-column errors on 256
    sampled columns no larger than with T from the sketch."""
    A_t = idgen.lowrank_plus_noise_device(2, 4096, 16384, np.exp(-np.arange(4096) / 64.0), 1e-8,
                                          dtype=torch.float32)
    Om_t = torch.tensor(idgen.omega_bf16(77, 266, 4096), dtype=torch.bfloat16, device="cuda")
    rs, rl = _lstsq_pair(A_t, Om_t, 256)
    assert rl.k == 256
    A64 = A_t.double().cpu().numpy()
    g = idgen.rng(80)
    cols = np.sort(g.choice(16384, 256, replace=False))
    _check_lstsq_against_oracle(A64, to_np(rs.J), rl, 256, cols=cols[:64])
    J, Js = to_np(rl.J), to_np(rs.J)
    el = np.linalg.norm(A64[:, cols] - A64[:, J] @ to_np(rl.Z).astype(np.float64)[:, cols], axis=0)
    es = np.linalg.norm(A64[:, cols] - A64[:, Js] @ to_np(rs.Z).astype(np.float64)[:, cols], axis=0)
    _no_worse(el, es, np.linalg.norm(A64[:, cols], axis=0))


def test_rid_lstsq_skeleton_cut_short():
    """Five nonzero columns and k = 8: the sketch's CPQR stops at k_out = 5
    (MIID_RANK_DEFICIENT), the rest of the skeleton is absent, the Cholesky
    treats it as unit rows, and C Z reproduces A."""
    miid = _miid()
    g = idgen.rng(21)
    m, n = 40, 120
    cols = [3, 17, 50, 77, 101]
    A = np.zeros((m, n))
    A[:, cols] = g.standard_normal((m, 5))
    A_t = torch.tensor(A, dtype=torch.float32, device="cuda")
    A64 = A_t.double().cpu().numpy()
    Om_t = torch.tensor(idgen.omega_bf16(22, 16, m), dtype=torch.bfloat16, device="cuda")
    r = miid.rid(A_t, Om_t, k=8, lstsq=True, want_R11=True)
    torch.cuda.synchronize()
    assert r.k == 5
    assert r.status & 1 and not r.status & 32
    J = to_np(r.J)
    assert sorted(J.tolist()) == cols
    Z = to_np(r.Z).astype(np.float64)
    assert np.array_equal(Z[:, J], np.eye(5))
    assert rel(A64[:, J] @ Z, A64) <= 1e-5
    R = to_np(r.R11)
    C = A64[:, J]
    assert rel(R.T @ R, C.T @ C) <= 1e-12
    # the full k x n output: rows beyond k_out are zero, J there is -1
    from paper_2105_07076_amd import api
    raw = api.rid_raw(A_t, Om_t, k=8, lstsq=True)
    torch.cuda.synchronize()
    assert np.all(to_np(raw["J"])[5:] == -1)
    assert np.all(to_np(raw["Z"])[5:] == 0.0)


def test_rid_lstsq_r11_leading_dimension():
    """A caller's R11 inside a taller buffer (ldr = k + 5): the k x k block is
    written, the rows below it are left as they were."""
    import ctypes
    from paper_2105_07076_amd import _abi, api
    _miid()
    g = idgen.rng(23)
    m, n, l, k = 96, 300, 50, 40
    A = g.standard_normal((m, n)) @ np.diag(0.97 ** np.arange(n))
    A_t = torch.tensor(A, dtype=torch.float32, device="cuda")
    Om_t = torch.tensor(idgen.omega_bf16(24, l, m), dtype=torch.bfloat16, device="cuda")
    big = torch.full((k, k + 5), 7.0, dtype=torch.float64, device="cuda").t()  # (k + 5) x k, column-major
    out = {
        "J": torch.empty(k, dtype=torch.int32, device="cuda"),
        "Z": torch.empty((n, k), dtype=torch.float32, device="cuda").t(),
        "C": None, "Y": None, "R11": big[:k],
        "info": torch.empty(ctypes.sizeof(_abi.MiidInfo), dtype=torch.uint8, device="cuda"),
    }
    assert out["R11"].stride() == (1, k + 5)
    api.rid_raw(A_t, Om_t, k=k, mode=1, lstsq=True, out=out)
    torch.cuda.synchronize()
    assert torch.all(big[k:] == 7.0)
    R = to_np(big[:k])
    J = to_np(out["J"])
    C = A_t.double().cpu().numpy()[:, J]
    assert np.array_equal(R, np.triu(R))
    assert rel(R.T @ R, C.T @ C) <= 1e-12
