"""torch-facing wrappers of the miid C ABI.

torch provides device memory (outputs, workspace) and the current HIP stream;
all arithmetic runs in libmiid.so.  Matrices cross the boundary column-major:
a torch tensor ``A`` of shape (m, n) is passed as is when it is column-major
(``A.t().is_contiguous()``), otherwise a column-major copy is made first.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _abi

_DT = {torch.float32: _abi.MIID_F32, torch.float64: _abi.MIID_F64}


def colmajor(x: torch.Tensor) -> torch.Tensor:
    """Column-major view/copy of a 2-D tensor (stride(0) == 1)."""
    if x.dim() != 2:
        raise ValueError("expected a matrix")
    if x.stride(0) == 1 and x.stride(1) >= max(1, x.shape[0]):
        return x
    return x.t().contiguous().t()


def empty_colmajor(m: int, n: int, dtype, device) -> torch.Tensor:
    return torch.empty((n, m), dtype=dtype, device=device).t()


def _ptr(x: torch.Tensor | None):
    return None if x is None else ctypes.c_void_p(x.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ld(x: torch.Tensor) -> int:
    return max(1, x.stride(1))


@dataclass
class IDResult:
    """J: selected indices (k_out); Z: k_out x N with Z[:, J] = I; C: A[:, J];
    R11: FP64 triangular factor in pivot order (k_out x k_out) or None."""
    J: torch.Tensor
    Z: torch.Tensor
    C: torch.Tensor | None
    R11: torch.Tensor | None
    k: int
    status: int
    a_norm: float
    r22_norm: float
    n_recompute: int
    Y: torch.Tensor | None = None

    @property
    def transposed(self) -> bool:
        return bool(self.status & _abi.MIID_TRANSPOSED)


class Workspace:
    """Grow-only device workspace (one per device and purpose)."""

    def __init__(self):
        self.buf: dict = {}

    def get(self, key, nbytes: int, device) -> torch.Tensor:
        b = self.buf.get((key, device))
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
            self.buf[(key, device)] = b
        return b


_WS = Workspace()

# one miid_handle per device, all created with the same tuning table
_HANDLES: dict = {}
_TABLE_PATH: str | None = None


def set_tuning_table(path: str | None) -> None:
    """Run later calls with the native tuning table at ``path`` (rows
    "routine dtype m n k nb hints", as written by autotune.Table.export_native);
    None drops it.  Calls that pass nb or hints themselves are unaffected."""
    global _TABLE_PATH
    for h in _HANDLES.values():
        h.close()
    _HANDLES.clear()
    _TABLE_PATH = path


def handle(device: int | None = None) -> _abi.Handle:
    """The miid_handle of ``device`` (default: the current device)."""
    dev = torch.cuda.current_device() if device is None else int(device)
    h = _HANDLES.get(dev)
    if h is None:
        with torch.cuda.device(dev):
            h = _abi.Handle(_TABLE_PATH)
        _HANDLES[dev] = h
    return h


def _h():
    return ctypes.c_void_p(handle().ptr)


def _read_info(info_dev: torch.Tensor) -> _abi.MiidInfo:
    host = info_dev.cpu().numpy().tobytes()
    return _abi.MiidInfo.from_buffer_copy(host)


def _opts(k, eps, kmax, nb, refine, hints: int = 0) -> _abi.MiidOpts:
    o = _abi.MiidOpts()
    if (k is None) == (eps is None):
        raise ValueError("give exactly one of k or eps")
    o.k = int(k) if k is not None else 0
    o.kmax = int(kmax) if kmax is not None else 0
    o.eps = float(eps) if eps is not None else 0.0
    o.nb = int(nb)
    o.flags = (0 if refine else _abi.MIID_NO_REFINE) | int(hints)
    return o


def id_raw(A: torch.Tensor, k: int | None = None, eps: float | None = None, kmax: int | None = None,
           nb: int = 0, refine: bool = True, want_C: bool = True, want_R11: bool = False,
           out: dict | None = None, hints: int = 0):
    """Enqueue id_cpqr without synchronising.  Returns a dict of device
    tensors (J, Z, C, R11, info) sized for kmax; ``out`` reuses buffers;
    ``hints`` are MIID_HINT fields (see :mod:`.autotune`)."""
    lib = _abi.load()
    if A.dtype not in _DT or not A.is_cuda:
        raise TypeError("A must be a float32/float64 CUDA tensor")
    A = colmajor(A)
    M, N = A.shape
    mw, nw = min(M, N), max(M, N)
    if kmax is None:
        kmax = min(M, N) if k is None else k
    kk = k if k is not None else kmax
    opts = _opts(k, eps, kmax, nb, refine, hints)
    dt = _DT[A.dtype]
    ws_bytes = lib.miid_id_workspace(_h(), M, N, dt, ctypes.byref(opts))
    if ws_bytes == 0:
        _abi.check(_abi.MIID_E_UNSUPPORTED, "miid_id_workspace")
    ws = _WS.get("id", ws_bytes, A.device)
    dev = A.device
    if out is None:
        out = {
            "J": torch.empty(kk, dtype=torch.int32, device=dev),
            "Z": empty_colmajor(kk, nw, A.dtype, dev),
            "C": empty_colmajor(mw, kk, A.dtype, dev) if want_C else None,
            "R11": empty_colmajor(kk, kk, torch.float64, dev) if want_R11 else None,
            "info": torch.empty(ctypes.sizeof(_abi.MiidInfo), dtype=torch.uint8, device=dev),
        }
    Z, C, R11 = out["Z"], out["C"], out["R11"]
    rc = lib.id_cpqr(_h(), _ptr(A), M, N, _ld(A), dt, ctypes.byref(opts), _ptr(out["J"]), _ptr(Z), _ld(Z),
                     _ptr(R11), _ld(R11) if R11 is not None else 1, _ptr(C), _ld(C) if C is not None else 1,
                     _ptr(out["info"]), _ptr(ws), ws_bytes, _stream())
    _abi.check(rc, "id_cpqr")
    return out


def _finish(out: dict, Y=None) -> IDResult:
    info = _read_info(out["info"])
    k = info.k_out
    J = out["J"][:k]
    Z = out["Z"][:k]
    C = out["C"][:, :k] if out.get("C") is not None else None
    R11 = out["R11"][:k, :k] if out.get("R11") is not None else None
    return IDResult(J=J, Z=Z, C=C, R11=R11, k=k, status=info.status, a_norm=info.a_norm,
                    r22_norm=info.r22_norm, n_recompute=info.n_recompute, Y=Y)


def id(A: torch.Tensor, k: int | None = None, eps: float | None = None, kmax: int | None = None,
       nb: int = 0, refine: bool = True, want_C: bool = True, want_R11: bool = False,
       hints: int = 0) -> IDResult:
    """Deterministic ID of A (m x n, float32/float64, on the GPU).

    Fixed rank ``k``, or tolerance mode ``eps`` (relative, on ||R22||_F) with
    cap ``kmax``.  m > n gives the dual ID of A^T (``transposed``).  ``nb``
    and ``hints`` set launch shapes only (see :mod:`.autotune`)."""
    out = id_raw(A, k=k, eps=eps, kmax=kmax, nb=nb, refine=refine, want_C=want_C, want_R11=want_R11,
                 hints=hints)
    return _finish(out)


def rid_sample_raw(A: torch.Tensor, idx, k: int, nb: int = 0, want_C: bool = True, want_R11: bool = False,
                   out: dict | None = None, hints: int = 0):
    """Enqueue rid_sample_cpqr without synchronising (see :func:`rid_sample`)."""
    lib = _abi.load()
    if A.dtype not in _DT or not A.is_cuda:
        raise TypeError("A must be a float32/float64 CUDA tensor")
    A = colmajor(A)
    m, n = A.shape
    idx_t = torch.as_tensor(idx, dtype=torch.int32, device=A.device).contiguous()
    p = int(idx_t.numel())
    opts = _opts(k, None, k, nb, True, hints)
    dt = _DT[A.dtype]
    ws_bytes = lib.miid_rid_sample_workspace(_h(), m, n, p, dt, ctypes.byref(opts))
    if ws_bytes == 0:
        _abi.check(_abi.MIID_E_UNSUPPORTED, "miid_rid_sample_workspace")
    ws = _WS.get("rid_sample", ws_bytes, A.device)
    dev = A.device
    if out is None:
        out = {
            "J": torch.empty(k, dtype=torch.int32, device=dev),
            "Z": empty_colmajor(k, n, A.dtype, dev),
            "C": empty_colmajor(m, k, A.dtype, dev) if want_C else None,
            "R11": empty_colmajor(k, k, torch.float64, dev) if want_R11 else None,
            "info": torch.empty(ctypes.sizeof(_abi.MiidInfo), dtype=torch.uint8, device=dev),
        }
    out["idx"] = idx_t
    Z, C, R11 = out["Z"], out["C"], out["R11"]
    rc = lib.rid_sample_cpqr(_h(), _ptr(A), m, n, _ld(A), dt, _ptr(idx_t), p, ctypes.byref(opts), _ptr(out["J"]),
                             _ptr(Z), _ld(Z), _ptr(R11), _ld(R11) if R11 is not None else 1, _ptr(C),
                             _ld(C) if C is not None else 1, _ptr(out["info"]), _ptr(ws), ws_bytes, _stream())
    _abi.check(rc, "rid_sample_cpqr")
    return out


def rid_sample(A: torch.Tensor, idx, k: int, nb: int = 0, want_C: bool = True, want_R11: bool = False,
               hints: int = 0) -> IDResult:
    """The paper's randomized ID by column sampling (its Optim RID): the
    column-pivoted QR of A[:, idx] picks k of the sampled columns
    (J = idx[selected], C = A[:, J]) and Z solves R_k^T R_k Z = C^T A over the
    full A.  ``idx`` holds the sample (the paper draws p = k + floor(0.2 k)
    distinct columns; the random numbers are an input; a device int32
    tensor is used as it is, anything else is copied to the device on each
    call, which graph capture does not allow).  ``a_norm`` and ``r22_norm``
    of the result refer to A[:, idx]."""
    out = rid_sample_raw(A, idx, k, nb=nb, want_C=want_C, want_R11=want_R11, hints=hints)
    return _finish(out)


@dataclass
class TwoSidedResult:
    """A ~ W A[I, J] Z: I (k_rows skeleton rows), J (k skeleton columns),
    W (m x k_rows, W[I, :] = identity), Z (k x n, Z[:, J] = identity)."""
    I: torch.Tensor
    J: torch.Tensor
    W: torch.Tensor
    Z: torch.Tensor
    k: int
    k_rows: int
    status: int
    status_rows: int


def two_sided_raw(A: torch.Tensor, k: int, nb: int = 0, out: dict | None = None, hints: int = 0):
    """Enqueue id_two_sided without synchronising (see :func:`two_sided`)."""
    lib = _abi.load()
    if A.dtype not in _DT or not A.is_cuda:
        raise TypeError("A must be a float32/float64 CUDA tensor")
    A = colmajor(A)
    m, n = A.shape
    opts = _opts(k, None, k, nb, True, hints)
    dt = _DT[A.dtype]
    ws_bytes = lib.miid_two_sided_workspace(_h(), m, n, dt, ctypes.byref(opts))
    if ws_bytes == 0:
        _abi.check(_abi.MIID_E_UNSUPPORTED, "miid_two_sided_workspace")
    ws = _WS.get("two_sided", ws_bytes, A.device)
    dev = A.device
    if out is None:
        isz = ctypes.sizeof(_abi.MiidInfo)
        out = {
            "J": torch.empty(k, dtype=torch.int32, device=dev),
            "Z": empty_colmajor(k, n, A.dtype, dev),
            "I": torch.empty(k, dtype=torch.int32, device=dev),
            "W": empty_colmajor(m, k, A.dtype, dev),
            "info": torch.empty(isz, dtype=torch.uint8, device=dev),
            "info_rows": torch.empty(isz, dtype=torch.uint8, device=dev),
        }
    rc = lib.id_two_sided(_h(), _ptr(A), m, n, _ld(A), dt, ctypes.byref(opts), _ptr(out["J"]), _ptr(out["Z"]),
                          _ld(out["Z"]), _ptr(out["I"]), _ptr(out["W"]), _ld(out["W"]), _ptr(out["info"]),
                          _ptr(out["info_rows"]), _ptr(ws), ws_bytes, _stream())
    _abi.check(rc, "id_two_sided")
    return out


def two_sided(A: torch.Tensor, k: int, nb: int = 0, hints: int = 0) -> TwoSidedResult:
    """Two-sided ID A ~ W A[I, J] Z (fixed rank k): the column ID of A, then
    the row (dual) ID of its skeleton C = A[:, J]."""
    out = two_sided_raw(A, k, nb=nb, hints=hints)
    ic = _read_info(out["info"])
    ir = _read_info(out["info_rows"])
    kc, kr = ic.k_out, ir.k_out
    return TwoSidedResult(I=out["I"][:kr], J=out["J"][:kc], W=out["W"][:, :kr], Z=out["Z"][:kc], k=kc, k_rows=kr,
                          status=ic.status, status_rows=ir.status)


def cur_raw(A: torch.Tensor, k: int, nb: int = 0, out: dict | None = None, hints: int = 0):
    """Enqueue id_cur without synchronising (see :func:`cur`)."""
    lib = _abi.load()
    if A.dtype not in _DT or not A.is_cuda:
        raise TypeError("A must be a float32/float64 CUDA tensor")
    A = colmajor(A)
    m, n = A.shape
    opts = _opts(k, None, k, nb, True, hints)
    dt = _DT[A.dtype]
    ws_bytes = lib.miid_cur_workspace(_h(), m, n, dt, ctypes.byref(opts))
    if ws_bytes == 0:
        _abi.check(_abi.MIID_E_UNSUPPORTED, "miid_cur_workspace")
    ws = _WS.get("cur", ws_bytes, A.device)
    dev = A.device
    if out is None:
        isz = ctypes.sizeof(_abi.MiidInfo)
        out = {
            "J": torch.empty(k, dtype=torch.int32, device=dev),
            "I": torch.empty(k, dtype=torch.int32, device=dev),
            "U": empty_colmajor(k, k, A.dtype, dev),
            "info": torch.empty(isz, dtype=torch.uint8, device=dev),
            "info_rows": torch.empty(isz, dtype=torch.uint8, device=dev),
        }
    rc = lib.id_cur(_h(), _ptr(A), m, n, _ld(A), dt, ctypes.byref(opts), _ptr(out["J"]), _ptr(out["I"]), _ptr(out["U"]),
                    _ld(out["U"]), _ptr(out["info"]), _ptr(out["info_rows"]), _ptr(ws), ws_bytes, _stream())
    _abi.check(rc, "id_cur")
    return out


def cur(A: torch.Tensor, k: int, nb: int = 0, hints: int = 0):
    """CUR form of the two-sided ID (fixed rank k): returns (I, J, U, status,
    status_rows) with A ~ A[:, J] U A[I, :] and U = Z R^+."""
    out = cur_raw(A, k, nb=nb, hints=hints)
    ic = _read_info(out["info"])
    ir = _read_info(out["info_rows"])
    return out["I"], out["J"], out["U"], ic.status, ir.status


def rid_raw(A: torch.Tensor, omega: torch.Tensor, k: int | None = None, eps: float | None = None,
            kmax: int | None = None, mode: int = 1, nb: int = 0, refine: bool = True, want_C: bool = True,
            want_Y: bool = False, want_R11: bool = False, out: dict | None = None, hints: int = 0,
            lstsq: bool = False):
    """Enqueue rid_sketch_cpqr without synchronising (see :func:`rid`)."""
    lib = _abi.load()
    if A.dtype != torch.float32 or not A.is_cuda:
        raise TypeError("A must be a float32 CUDA tensor")
    if omega.dtype != torch.bfloat16 or not omega.is_cuda:
        raise TypeError("omega must be a bfloat16 CUDA tensor (l x m)")
    A = colmajor(A)
    om = colmajor(omega)
    m, n = A.shape
    l = om.shape[0]
    if om.shape[1] != m:
        raise ValueError("omega must be l x m")
    if kmax is None:
        kmax = l if k is None else k
    kk = k if k is not None else kmax
    opts = _opts(k, eps, kmax, nb, refine, hints)
    if lstsq:
        if k is None:
            raise ValueError("lstsq needs a fixed rank k")
        opts.flags |= _abi.MIID_LSTSQ_Z
    ws_bytes = lib.miid_rid_workspace(_h(), m, n, l, ctypes.byref(opts))
    if ws_bytes == 0:
        _abi.check(_abi.MIID_E_UNSUPPORTED, "miid_rid_workspace")
    ws = _WS.get("rid", ws_bytes, A.device)
    dev = A.device
    if out is None:
        out = {
            "J": torch.empty(kk, dtype=torch.int32, device=dev),
            "Z": empty_colmajor(kk, n, torch.float32, dev),
            "C": empty_colmajor(m, kk, torch.float32, dev) if want_C else None,
            "Y": empty_colmajor(l, n, torch.float32, dev) if want_Y else None,
            "R11": empty_colmajor(kk, kk, torch.float64, dev) if want_R11 else None,
            "info": torch.empty(ctypes.sizeof(_abi.MiidInfo), dtype=torch.uint8, device=dev),
        }
    Z, C, Y, R11 = out["Z"], out["C"], out["Y"], out["R11"]
    rc = lib.rid_sketch_cpqr(_h(), _ptr(A), m, n, _ld(A), _ptr(om), l, _ld(om), int(mode), ctypes.byref(opts),
                             _ptr(out["J"]), _ptr(Z), _ld(Z), _ptr(C), _ld(C) if C is not None else 1,
                             _ptr(Y), _ld(Y) if Y is not None else 1, _ptr(R11), _ld(R11) if R11 is not None else 1,
                             _ptr(out["info"]), _ptr(ws), ws_bytes, _stream())
    _abi.check(rc, "rid_sketch_cpqr")
    return out


def rid(A: torch.Tensor, omega: torch.Tensor, k: int | None = None, eps: float | None = None,
        kmax: int | None = None, mode: int = 1, nb: int = 0, refine: bool = True, want_C: bool = True,
        want_Y: bool = False, want_R11: bool = False, hints: int = 0, lstsq: bool = False) -> IDResult:
    """Randomized ID of A (m x n float32, m <= n) with the Gaussian row sketch
    Y = omega A computed on the matrix cores.

    ``omega`` is an l x m bfloat16 tensor (the random numbers the method
    draws are an input).  ``mode`` 1 splits A as hi + mid bfloat16 (two
    passes, 2^-16 relative per entry), 2 as hi + mid + lo (three passes,
    2^-24), 0 rounds it once.  J and T come from the CPQR of Y; C = A[:, J].
    With ``lstsq`` (fixed rank) Z is instead C^+ A over the full A, the
    paper's way of forming the randomized ID's Z, for the same J: R11 is then
    the Cholesky factor of C^T C.
    ``a_norm``/``r22_norm`` in the result refer to Y."""
    out = rid_raw(A, omega, k=k, eps=eps, kmax=kmax, mode=mode, nb=nb, refine=refine, want_C=want_C,
                  want_Y=want_Y, want_R11=want_R11, hints=hints, lstsq=lstsq)
    return _finish(out, Y=out["Y"])


@dataclass
class BatchedResult:
    """Packed outputs of :func:`batched`: block b selected k[b] columns
    J[j_off[b]: j_off[b] + k[b]] and owns the kmax_b x n_b matrix
    Z[z_off[b]: z_off[b] + kmax_b * n_b] (column-major, rows >= k[b] zero)."""
    J: torch.Tensor
    Z: torch.Tensor
    k: "np.ndarray"
    status: "np.ndarray"
    a_norm: "np.ndarray"
    r22_norm: "np.ndarray"
    kmax_b: "np.ndarray"
    j_off: "np.ndarray"
    z_off: "np.ndarray"
    n: "np.ndarray"

    def block(self, b: int):
        """(J_b, Z_b) of block b as host numpy arrays (Z_b is k_b x n_b)."""
        kb, kk, nb = int(self.kmax_b[b]), int(self.k[b]), int(self.n[b])
        Jh = self.J[int(self.j_off[b]): int(self.j_off[b]) + kk].cpu().numpy()
        Zh = self.Z[int(self.z_off[b]): int(self.z_off[b]) + kb * nb].cpu().numpy().reshape(nb, kb).T[:kk]
        return Jh, Zh


def batched_raw(A: torch.Tensor, a_off, m, n, eps: float, kmax: int = 64, out: dict | None = None,
                hints: int = 0, noalloc: bool = False):
    """Enqueue id_batched without synchronising.  ``A`` is the packed blocks
    (1-D float32/float64 CUDA tensor), ``a_off``/``m``/``n`` host sequences.
    ``noalloc`` calls id_batched_noalloc, which uses the library's static
    scratch instead of a workspace."""
    import numpy as np
    lib = _abi.load()
    if A.dtype not in _DT or not A.is_cuda:
        raise TypeError("A must be a float32/float64 CUDA tensor")
    dev = A.device
    if out is None:
        mh = np.asarray(m, dtype=np.int32)
        nh = np.asarray(n, dtype=np.int32)
        kb = np.minimum(np.minimum(mh, nh), kmax).astype(np.int64)
        j_off = np.zeros(len(mh), dtype=np.int64)
        j_off[1:] = np.cumsum(kb)[:-1]
        z_off = np.zeros(len(mh), dtype=np.int64)
        z_off[1:] = np.cumsum(kb * nh)[:-1]
        nblk = len(mh)
        out = {
            "nblk": nblk, "kmax_b": kb, "j_off_h": j_off, "z_off_h": z_off, "n_h": nh,
            "a_off": torch.as_tensor(np.asarray(a_off, dtype=np.int64), device=dev),
            "m": torch.as_tensor(mh, device=dev), "n": torch.as_tensor(nh, device=dev),
            "j_off": torch.as_tensor(j_off, device=dev), "z_off": torch.as_tensor(z_off, device=dev),
            "J": torch.empty(int(kb.sum()), dtype=torch.int32, device=dev),
            "Z": torch.empty(int((kb * nh).sum()), dtype=A.dtype, device=dev),
            "info": torch.empty(nblk * ctypes.sizeof(_abi.MiidInfo), dtype=torch.uint8, device=dev),
        }
    dt = _DT[A.dtype]
    opts = _abi.MiidOpts()
    opts.k, opts.kmax, opts.eps, opts.nb, opts.flags = 0, int(kmax), float(eps), 0, int(hints)
    if noalloc:
        rc = lib.id_batched_noalloc(_h(), out["nblk"], _ptr(A), _ptr(out["a_off"]), _ptr(out["m"]), _ptr(out["n"]),
                                    dt, ctypes.byref(opts), _ptr(out["J"]), _ptr(out["j_off"]), _ptr(out["Z"]),
                                    _ptr(out["z_off"]), _ptr(out["info"]), _stream())
        _abi.check(rc, "id_batched_noalloc")
        return out
    ws_bytes = lib.miid_batched_workspace(_h(), out["nblk"], dt)
    ws = _WS.get("batched", ws_bytes, dev)
    rc = lib.id_batched(_h(), out["nblk"], _ptr(A), _ptr(out["a_off"]), _ptr(out["m"]), _ptr(out["n"]), dt,
                        ctypes.byref(opts), _ptr(out["J"]), _ptr(out["j_off"]), _ptr(out["Z"]),
                        _ptr(out["z_off"]), _ptr(out["info"]), _ptr(ws), ws_bytes, _stream())
    _abi.check(rc, "id_batched")
    return out


def batched(A: torch.Tensor, a_off, m, n, eps: float, kmax: int = 64, hints: int = 0,
            noalloc: bool = False) -> BatchedResult:
    """Tolerance-mode IDs of many independent blocks in one launch: block b is
    m[b] x n[b] (column-major) at A[a_off[b]:]; its rank is the smallest k with
    ||R22||_F <= eps ||A_b||_F, at most min(m_b, n_b, kmax).  ``noalloc``: the
    allocation-free entry point (id_batched_noalloc)."""
    out = batched_raw(A, a_off, m, n, eps, kmax, hints=hints, noalloc=noalloc)
    return batched_result(out)


def batched_result(out: dict) -> BatchedResult:
    """The BatchedResult of a finished batched_raw call (reads info)."""
    import numpy as np
    raw = out["info"].cpu().numpy().tobytes()
    sz = ctypes.sizeof(_abi.MiidInfo)
    infos = [_abi.MiidInfo.from_buffer_copy(raw[i * sz:(i + 1) * sz]) for i in range(out["nblk"])]
    return BatchedResult(J=out["J"], Z=out["Z"], k=np.array([x.k_out for x in infos]),
                         status=np.array([x.status for x in infos]), a_norm=np.array([x.a_norm for x in infos]),
                         r22_norm=np.array([x.r22_norm for x in infos]), kmax_b=out["kmax_b"],
                         j_off=out["j_off_h"], z_off=out["z_off_h"], n=out["n_h"])


def id_backward(A: torch.Tensor, J: torch.Tensor, R11: torch.Tensor, Z: torch.Tensor,
                gC: torch.Tensor | None, gZ: torch.Tensor | None) -> torch.Tensor:
    """Gradient of a loss on (C, Z) with respect to A, pivots J fixed
    (C = A[:, J], Z = C^+ A).  R11 (k x k FP64) and Z come from the forward
    :func:`id` of the same A.  Enqueued on the current stream."""
    lib = _abi.load()
    if A.dtype not in _DT or not A.is_cuda:
        raise TypeError("A must be a float32/float64 CUDA tensor")
    A = colmajor(A)
    m, n = A.shape
    k = int(J.numel())
    J = J.to(torch.int32).contiguous()
    R11 = colmajor(R11.to(torch.float64))
    Z = colmajor(Z.to(A.dtype))
    gCc = colmajor(gC.to(A.dtype)) if gC is not None else None
    gZc = colmajor(gZ.to(A.dtype)) if gZ is not None else None
    dt = _DT[A.dtype]
    ws_bytes = lib.miid_backward_workspace(_h(), m, n, k, dt)
    if ws_bytes == 0:
        _abi.check(_abi.MIID_E_UNSUPPORTED, "miid_backward_workspace")
    ws = _WS.get("bwd", ws_bytes, A.device)
    gA = empty_colmajor(m, n, A.dtype, A.device)
    rc = lib.id_backward(_h(), _ptr(A), m, n, _ld(A), dt, _ptr(J), k, _ptr(R11), _ld(R11), _ptr(Z), _ld(Z),
                         _ptr(gCc), _ld(gCc) if gCc is not None else 1, _ptr(gZc), _ld(gZc) if gZc is not None else 1,
                         _ptr(gA), _ld(gA), _ptr(ws), ws_bytes, _stream())
    _abi.check(rc, "id_backward")
    return gA


class IDFunction(torch.autograd.Function):
    """(C, Z) = ID(A) at rank k with the pivots fixed in the forward pass;
    the backward pass runs id_backward.  A is m x n with m <= n."""

    @staticmethod
    def forward(ctx, A, k):
        r = id(A.detach(), k=int(k), want_C=True, want_R11=True)
        if r.transposed:
            raise ValueError("IDFunction needs m <= n")
        ctx.save_for_backward(A.detach(), r.J, r.R11, r.Z)
        return r.C, r.Z

    @staticmethod
    def backward(ctx, gC, gZ):
        A, J, R11, Z = ctx.saved_tensors
        gA = id_backward(A, J, R11, Z, gC, gZ)
        return gA, None
