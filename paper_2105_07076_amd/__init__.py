"""miid: interpolative decompositions on AMD MI355X (gfx950).

Hot path of Advani & O'Hagan, "Efficient Algorithms for Constructing an
Interpolative Decomposition": rank-k truncated column-pivoted Householder
QR (Businger-Golub pivoting) on A (deterministic ID) or on a Gaussian sketch
Y = Omega A (randomized ID), then Z = [I R11^{-1} R12] P^T and C = A[:, J].
Every step runs in the HIP kernels of libmiid.so behind the C ABI of
include/miid.h; this package only marshals arguments (torch supplies device
memory and the stream).
"""
from ._abi import MiidError, load  # noqa: F401
from .api import (IDResult, BatchedResult, TwoSidedResult, id, rid, rid_sample, two_sided, cur,  # noqa: F401
                  batched, id_backward, IDFunction, handle, set_tuning_table)
from . import autotune  # noqa: F401

__all__ = ["IDResult", "id", "rid", "batched", "id_backward", "IDFunction", "MiidError", "load", "autotune",
           "handle", "set_tuning_table"]
