"""GPU parity of id_backward (the adjoint of the ID with the pivots held fixed)
against the FP64 oracle's closed form, finite differences and torch autograd
through a dense least-squares reference."""
from __future__ import annotations

import numpy as np
import pytest

import idgen
import oracle
from gpu_helpers import rel, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _miid():
    import paper_2105_07076_amd as miid
    miid.load()
    return miid


def _forward(A_np, k, dtype):
    miid = _miid()
    A_t = torch.tensor(A_np, dtype=dtype, device="cuda")
    r = miid.id(A_t, k=k, want_R11=True)
    torch.cuda.synchronize()
    return miid, A_t, r


def _loss_parts(A, B, J):
    C = A[:, J]
    Z = np.linalg.lstsq(C, A, rcond=None)[0]
    M = C @ Z
    return M, B - M, C, Z


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 2e-4)])
@pytest.mark.parametrize("m,n,k", [(30, 80, 8), (64, 300, 40), (100, 1000, 77), (17, 17, 17)])
def test_backward_matches_oracle(dtype, tol, m, n, k):
    g = idgen.rng(m + n + k)
    A = g.standard_normal((m, n)) @ np.diag(0.98 ** np.arange(n))
    miid, A_t, r = _forward(A, k, dtype)
    A64 = A_t.double().cpu().numpy()
    J = to_np(r.J)
    gC = g.standard_normal((m, k))
    gZ = g.standard_normal((k, n))
    gA = miid.id_backward(A_t, r.J, r.R11, r.Z, torch.tensor(gC, dtype=dtype, device="cuda"),
                          torch.tensor(gZ, dtype=dtype, device="cuda"))
    torch.cuda.synchronize()
    ref_fwd = oracle.id(A64, k=k, force=J)
    ref = oracle.id_vjp(A64, J, ref_fwd.Z, gC, gZ)
    assert rel(to_np(gA).astype(np.float64), ref) <= tol


def test_backward_without_gC():
    g = idgen.rng(5)
    A = g.standard_normal((40, 120)) @ np.diag(0.97 ** np.arange(120))
    miid, A_t, r = _forward(A, 12, torch.float64)
    gZ = g.standard_normal((12, 120))
    gA = miid.id_backward(A_t, r.J, r.R11, r.Z, None, torch.tensor(gZ, device="cuda"))
    J = to_np(r.J)
    ref = oracle.id_vjp(A, J, oracle.id(A, k=12, force=J).Z, None, gZ)
    assert rel(to_np(gA), ref) <= 1e-10


def test_autograd_function_full_rank_closed_form():
    """k = m: C Z = A, so the gradient of ||B - C Z||^2 is -2 (B - A)."""
    miid = _miid()
    g = idgen.rng(6)
    A = torch.tensor(g.standard_normal((24, 60)), device="cuda", requires_grad=True)
    B = torch.tensor(g.standard_normal((24, 60)), device="cuda")
    C, Z = miid.IDFunction.apply(A, 24)
    loss = ((B - C @ Z) ** 2).sum()
    loss.backward()
    ref = -2.0 * (B - A.detach())
    assert torch.linalg.norm(A.grad - ref) <= 1e-8 * torch.linalg.norm(ref)


def test_autograd_function_vs_dense_lstsq():
    """Gradient through IDFunction vs torch autograd through a dense FP64
    least-squares solve on the CPU with the same pivots."""
    miid = _miid()
    g = idgen.rng(7)
    A_np = g.standard_normal((50, 200)) @ np.diag(0.96 ** np.arange(200))
    B_np = g.standard_normal((50, 200))
    A = torch.tensor(A_np, device="cuda", requires_grad=True)
    C, Z = miid.IDFunction.apply(A, 15)
    loss = ((torch.tensor(B_np, device="cuda") - C @ Z) ** 2).sum()
    loss.backward()
    J = torch.tensor(to_np(miid.id(A.detach(), k=15).J), dtype=torch.long)
    Ac = torch.tensor(A_np, requires_grad=True)
    Cc = Ac[:, J]
    Zc = torch.linalg.pinv(Cc) @ Ac
    lc = ((torch.tensor(B_np) - Cc @ Zc) ** 2).sum()
    lc.backward()
    assert rel(to_np(A.grad), Ac.grad.numpy()) <= 1e-8


def _loss_parts_dev(X, B, J):
    """M = C C^+ X (the projection of X onto span C, C = X[:, J]) and the
    residual B - M, in FP64 on the device through a Householder QR of C."""
    Q, _ = torch.linalg.qr(X[:, J], mode="reduced")
    M = Q @ (Q.T @ X)
    return M, B - M


@pytest.mark.timeout(170)
def test_backward_cfg5_fp32():
    """2048 x 8192, s_i = exp(-i/32), noise 1e-6, k = 128, L = ||B - C Z||^2:
    the FP32 adjoint against the FP64 closed form (<= 1e-4 relative) and
    central finite differences in FP64 (h = 1e-6) on 64 random directions
    (the perturbed losses evaluated in FP64 by torch on the device)."""
    miid = _miid()
    A_np, B_np, k = idgen.cfg5()
    miid_, A_t, r = _forward(A_np, k, torch.float32)
    A64 = A_t.double().cpu().numpy()
    J = to_np(r.J)
    M, G, C, Z = _loss_parts(A64, B_np, J)
    gC = -2.0 * G @ Z.T
    gZ = -2.0 * C.T @ G
    gA = miid.id_backward(A_t, r.J, r.R11, r.Z, torch.tensor(gC, dtype=torch.float32, device="cuda"),
                          torch.tensor(gZ, dtype=torch.float32, device="cuda"))
    gA = to_np(gA).astype(np.float64)
    ref = oracle.id_vjp(A64, J, Z, gC, gZ)
    assert rel(gA, ref) <= 1e-4
    Ad = torch.tensor(A64, device="cuda")
    Bd = torch.tensor(B_np, device="cuda")
    Jd = torch.tensor(J.astype(np.int64), device="cuda")
    gAd = torch.tensor(gA, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(55)
    h = 1e-6
    bound = 1e-4 * float(np.linalg.norm(ref))
    for _ in range(64):
        D = torch.randn(Ad.shape, generator=gen, device="cuda", dtype=torch.float64)
        D /= torch.linalg.norm(D)
        Mp, Gp = _loss_parts_dev(Ad + h * D, Bd, Jd)
        Mm, Gm = _loss_parts_dev(Ad - h * D, Bd, Jd)
        fd = float(-torch.sum((Gp + Gm) * (Mp - Mm)) / (2.0 * h))
        an = float(torch.sum(gAd * D))
        assert abs(fd - an) <= bound + 1e-6 * abs(fd), f"directional derivative {an:.6e} vs FD {fd:.6e}"
