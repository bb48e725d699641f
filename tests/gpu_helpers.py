"""Shared helpers of the GPU parity tests (not collected as tests)."""
from __future__ import annotations

import numpy as np

import oracle

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def to_np(x):
    return None if x is None else x.detach().cpu().numpy()


def pivot_parity(A64: np.ndarray, J_gpu, k: int, u_work: float):
    """Margin-aware pivot parity.

    The GPU must pick the oracle's pivot at every step that is not a declared
    near-tie.  Step j is a declared near-tie when the oracle's relative margin
    mu_j = (nu_(1) - nu_(2)) / nu_(1) is at most beta_j = 16 u (1 / rho_j)^2
    (rho_j = chosen residual / original norm: downdated norms carry error
    amplified by (||a|| / nu)^2).  There the GPU may pick any column whose
    residual is within (1 - beta_j) of the largest; the oracle then follows
    the GPU's choice.  Returns (oracle result following the GPU, ties)."""
    J_gpu = [int(x) for x in J_gpu]
    res = oracle.id(A64, k=k)
    ties = 0
    for j in range(len(J_gpu)):
        assert j < res.k, f"GPU selected more columns ({len(J_gpu)}) than the oracle ({res.k})"
        if int(res.J[j]) == J_gpu[j]:
            continue
        mu = float(res.margins[j])
        rho = float(res.rho[j])
        beta = 16.0 * u_work / (rho * rho)
        assert mu <= beta, (f"undeclared pivot mismatch at step {j}: gpu {J_gpu[j]} oracle {res.J[j]} "
                            f"mu={mu:.3e} beta={beta:.3e}")
        res = oracle.id(A64, k=k, force=np.array(J_gpu[: j + 1], dtype=np.int32))
        assert res.nu1[j] >= (1.0 - beta) * res.nu2[j], f"step {j}: GPU pivot not within beta of the best"
        ties += 1
    return res, ties


def t_part(Z: np.ndarray, J) -> np.ndarray:
    mask = np.ones(Z.shape[1], dtype=bool)
    mask[np.asarray(J)] = False
    return Z[:, mask]


def rel(a: np.ndarray, b: np.ndarray) -> float:
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))
