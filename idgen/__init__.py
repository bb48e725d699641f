"""Seeded synthetic inputs for the interpolative-decomposition (ID) hot path.

This module holds only input construction: random matrices of the shapes,
spectra and structure described for the workloads, drawn from seeded
generators.  It contains none of the method's arithmetic (no pivoting, no
QR of the input, no solves) and is imported both by the tests that drive the
GPU path and by the tests that drive the CPU oracle, so that both sides see
the same numbers.

Random numbers that the randomized ID draws (the Gaussian sketch Omega) are
produced here and passed in as inputs.

Haar-distributed orthonormal frames are built the standard way: QR of a
Gaussian matrix with the columns of Q multiplied by sign(diag R)
(Mezzadri, "How to generate random matrices from the classical compact
groups", 2007).  That QR is part of building the input, not of the method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng", "haar", "lowrank_plus_noise", "cfg1", "cfg2", "cfg3_factors", "cfg5",
    "paper_dataset", "omega_bf16", "bf16_round", "batched_blocks", "BatchedBlocks",
    "planted_id", "integer_lowrank", "diag_case",
]


def rng(seed: int) -> np.random.Generator:
    """PCG64 generator for a fixed integer seed."""
    return np.random.Generator(np.random.PCG64(int(seed)))


def haar(g: np.random.Generator, m: int, r: int) -> np.ndarray:
    """m x r matrix with orthonormal columns, Haar-distributed (r <= m)."""
    X = g.standard_normal((m, r))
    Q, R = np.linalg.qr(X, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return np.asfortranarray(Q * d[None, :])


def lowrank_plus_noise(seed: int, m: int, n: int, s: np.ndarray, noise: float,
                       r: int | None = None) -> np.ndarray:
    """A = U diag(s) V^T + noise * G, float64, column-major.

    U (m x r) and V (n x r) are Haar frames, G is standard Gaussian.  ``r``
    defaults to min(m, n, len(s)); terms beyond ``r`` are dropped.
    """
    g = rng(seed)
    r = min(m, n, len(s)) if r is None else r
    U = haar(g, m, r)
    V = haar(g, n, r)
    G = g.standard_normal((m, n))
    A = (U * np.asarray(s[:r])[None, :]) @ V.T + noise * G
    return np.asfortranarray(A)


def cfg1(seed: int = 1) -> tuple[np.ndarray, int]:
    """Small FP64 workload: 256 x 512, s_i = 2^(-i/2) for i < 32 else 0,
    noise 1e-10, rank k = 32."""
    m, n = 256, 512
    s = np.zeros(256)
    s[:32] = 2.0 ** (-np.arange(32) / 2.0)
    return lowrank_plus_noise(seed, m, n, s, 1e-10), 32


def cfg2(seed: int = 2, m: int = 4096, n: int = 16384, r: int | None = None) -> tuple[np.ndarray, int]:
    """Deterministic-ID-at-scale workload: m x n, s_i = exp(-i/64), noise 1e-8,
    rank k = 256.  ``m``/``n`` can be reduced for quick tests; ``r`` caps the
    number of singular triplets (terms with s_i below ~1e-14 of s_0 are far
    below the 1e-8 noise)."""
    s = np.exp(-np.arange(min(m, n)) / 64.0)
    return lowrank_plus_noise(seed, m, n, s, 1e-8, r=r), 256


def cfg5(seed: int = 5, m: int = 2048, n: int = 8192) -> tuple[np.ndarray, np.ndarray, int]:
    """Differentiable-ID workload: A (m x n) with s_i = exp(-i/32), noise 1e-6,
    rank k = 128, and a Gaussian target B of the same shape."""
    s = np.exp(-np.arange(min(m, n)) / 32.0)
    A = lowrank_plus_noise(seed, m, n, s, 1e-6)
    B = np.asfortranarray(rng(seed + 1000).standard_normal((m, n)))
    return A, B, 128


def cfg3_factors(seed: int = 3, m: int = 16384, n: int = 65536, r: int = 4096):
    """Factors of the randomized-ID workload A = U diag(s) V^T + 1e-8 G with
    s_i = exp(-i/128), truncated to r terms (s_i <= e^-32 beyond r=4096).
    Returns (U, s, V); the caller forms A on whatever device it uses."""
    g = rng(seed)
    U = haar(g, m, r)
    V = haar(g, n, r)
    s = np.exp(-np.arange(r) / 128.0)
    return U, s, V


def paper_dataset(name: str, seed: int = 0, m: int = 784, n: int = 1000) -> np.ndarray:
    """The synthetic dense datasets of the paper's appendix: 784 x 1000 with
    entries drawn from {0,1} ("boolean"), N(0,1) ("gaussian") or U[0,1)
    ("uniform")."""
    g = rng(seed)
    if name == "boolean":
        A = g.integers(0, 2, size=(m, n)).astype(np.float64)
    elif name == "gaussian":
        A = g.standard_normal((m, n))
    elif name == "uniform":
        A = g.random((m, n))
    else:
        raise ValueError(name)
    return np.asfortranarray(A)


# shapes and nonzero counts of the paper's three sparse datasets (its table
# of sparse dataset information); the matrices themselves are not available
SPARSE_SHAPES = {"sparse1": (1138, 4054), "sparse2": (846, 10894), "sparse3": (531, 7422)}


def sparse_standin(name: str, seed: int = 0) -> np.ndarray:
    """A stand-in for one of the paper's sparse datasets, stored densely as
    the paper did: a random symmetric n x n matrix with the dataset's shape
    and nonzero count, a nonzero diagonal plus symmetric off-diagonal pairs at
    uniformly random positions, values uniform in (0, 1] (weighted graphs)."""
    n, nnz = SPARSE_SHAPES[name]
    g = rng(seed)
    A = np.zeros((n, n))
    A[np.arange(n), np.arange(n)] = 1.0 - g.random(n)
    pairs = (nnz - n) // 2
    placed = 0
    while placed < pairs:
        i = g.integers(0, n, size=pairs - placed)
        j = g.integers(0, n, size=pairs - placed)
        for a, b in zip(i, j):
            if a != b and A[a, b] == 0.0 and placed < pairs:
                v = 1.0 - g.random()
                A[a, b] = A[b, a] = v
                placed += 1
    return np.asfortranarray(A)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even); returns
    float32 values that are exactly representable in bfloat16."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).reshape(f.shape)


def omega_bf16(seed: int, l: int, m: int) -> np.ndarray:
    """Gaussian sketch matrix Omega (l x m), entries N(0,1) rounded to
    bfloat16 so that the same values are exact in bfloat16 and float64.
    Returned as float32, column-major."""
    g = rng(seed)
    return np.asfortranarray(bf16_round(g.standard_normal((l, m))))


def column_sample(seed: int, n: int, k: int, p: int | None = None) -> np.ndarray:
    """The random column sample of the column-sampling randomized ID: p
    distinct indices of range(n) drawn uniformly without replacement; p
    defaults to the paper's k + floor(0.2 k).  int32, in draw order."""
    if p is None:
        p = k + int(0.2 * k)
    return rng(seed).choice(n, size=p, replace=False).astype(np.int32)


def bf16_bits(x_bf16_exact: np.ndarray) -> np.ndarray:
    """uint16 bit patterns of float32 values that are exact bfloat16."""
    f = np.asarray(x_bf16_exact, dtype=np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


@dataclass
class BatchedBlocks:
    """Packed column-major blocks: block b is m[b] x n[b] starting at a_off[b]."""
    A: np.ndarray          # packed values (float64)
    m: np.ndarray          # int32
    n: np.ndarray          # int32
    a_off: np.ndarray      # int64

    def block(self, b: int) -> np.ndarray:
        mb, nb = int(self.m[b]), int(self.n[b])
        o = int(self.a_off[b])
        return self.A[o:o + mb * nb].reshape((nb, mb)).T


def batched_blocks(seed: int = 4, nblk: int = 4096, mmin: int = 32, mmax: int = 256,
                   sep: float = 4.0) -> BatchedBlocks:
    """Kernel-matrix blocks A_b[i, j] = 1 / ||x_i - y_j||: x uniform in the unit
    cube, y uniform in the unit cube shifted by ``sep`` box widths along the
    first axis.  m_b is uniform on [mmin, mmax] and n_b uniform on
    [m_b, 2 m_b] (inclusive).  Entries are computed in float64."""
    g = rng(seed)
    ms = g.integers(mmin, mmax + 1, size=nblk).astype(np.int32)
    ns = np.array([g.integers(mb, 2 * mb + 1) for mb in ms], dtype=np.int32)
    return _kernel_blocks(g, ms, ns, sep)


def kernel_blocks_sized(seed: int, ms, ns, sep: float = 4.0) -> BatchedBlocks:
    """The same kernel-matrix blocks with the given sizes (m[b], n[b])."""
    g = rng(seed)
    return _kernel_blocks(g, np.asarray(ms, dtype=np.int32), np.asarray(ns, dtype=np.int32), sep)


def _kernel_blocks(g, ms: np.ndarray, ns: np.ndarray, sep: float) -> BatchedBlocks:
    nblk = len(ms)
    sizes = ms.astype(np.int64) * ns.astype(np.int64)
    off = np.zeros(nblk, dtype=np.int64)
    off[1:] = np.cumsum(sizes)[:-1]
    A = np.empty(int(sizes.sum()), dtype=np.float64)
    shift = np.array([sep, 0.0, 0.0])
    for b in range(nblk):
        x = g.random((ms[b], 3))
        y = g.random((ns[b], 3)) + shift
        d = np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(-1))
        A[off[b]:off[b] + sizes[b]] = (1.0 / d).T.reshape(-1)  # column-major
    return BatchedBlocks(A=A, m=ms, n=ns, a_off=off)


def planted_id(seed: int, m: int, n: int, k: int, r: float = 0.9, eta: float = 0.0):
    """Input with a known pivot sequence.

    A has k 'skeleton' columns Q diag(d) (Q orthonormal m x k, d_i = r^i)
    and n-k columns Q diag(d) U + eta*N with |U_il| bounded so that every
    non-skeleton column stays strictly behind the skeleton column of the
    same step.  Columns are shuffled by a seeded permutation.
    Returns (A, planted_order, U, perm) where planted_order[i] is the column
    index of skeleton column i.
    """
    g = rng(seed)
    Q = haar(g, m, k)
    d = r ** np.arange(k)
    bound = (1.0 - r) * math.sqrt(1.0 - r * r) / math.sqrt(k)
    U = g.uniform(-bound, bound, size=(k, n - k))
    S = Q * d[None, :]
    rest = S @ U
    if eta > 0:
        rest = rest + eta * g.standard_normal((m, n - k))
    full = np.concatenate([S, rest], axis=1)
    perm = g.permutation(n)           # full column c goes to position perm[c]
    A = np.empty_like(full)
    A[:, perm] = full
    return np.asfortranarray(A), perm[:k].copy(), U, perm


def integer_lowrank(seed: int, m: int, n: int, k: int, lo: int = -3, hi: int = 3) -> np.ndarray:
    """A = B W with small-integer B (m x k) and W (k x n): rank <= k, exact in
    floating point."""
    g = rng(seed)
    B = g.integers(lo, hi + 1, size=(m, k)).astype(np.float64)
    W = g.integers(lo, hi + 1, size=(k, n)).astype(np.float64)
    return np.asfortranarray(B @ W)


def diag_case(d: np.ndarray, n: int) -> np.ndarray:
    """A = [diag(d) 0] (len(d) x n)."""
    m = len(d)
    A = np.zeros((m, n))
    A[np.arange(m), np.arange(m)] = d
    return np.asfortranarray(A)


def lowrank_plus_noise_device(seed: int, m: int, n: int, s, noise: float, r: int | None = None,
                              device: str = "cuda", dtype=None):
    """Device-side version of :func:`lowrank_plus_noise` for the large
    workloads: the same construction (Haar U, V from QR of seeded Gaussians
    with the sign fix, A = U diag(s) V^T + noise G) drawn with torch's
    seeded generator on ``device`` (not bit-identical to the numpy recipe).
    Returns a column-major (m, n) tensor (stride (1, m))."""
    import torch
    dtype = torch.float64 if dtype is None else dtype
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    r = min(m, n, len(s)) if r is None else r

    def haar_t(rows, cols):
        X = torch.randn(rows, cols, generator=g, device=device, dtype=torch.float64)
        Q, R = torch.linalg.qr(X, mode="reduced")
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        return Q * d[None, :]

    U = haar_t(m, r)
    V = haar_t(n, r)
    sv = torch.as_tensor(np.asarray(s[:r], dtype=np.float64), device=device)
    At = (V * sv[None, :]) @ U.T                      # (n, m) row-major = A column-major
    At += noise * torch.randn(n, m, generator=g, device=device, dtype=torch.float64)
    del U, V
    return At.to(dtype).t()
