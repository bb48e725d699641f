"""ctypes binding of the miid C ABI (include/miid.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libmiid.so.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmiid.so")

MIID_F32 = 0
MIID_F64 = 1
MIID_E_WORKSPACE = -100
MIID_E_HIP = -101
MIID_E_UNSUPPORTED = -102

MIID_RANK_DEFICIENT = 1
MIID_NONFINITE = 2
MIID_TRANSPOSED = 4
MIID_KMAX_HIT = 8
MIID_LSTSQ_BREAKDOWN = 32

MIID_NO_REFINE = 1
MIID_KEEP_COLUMNS = 2
MIID_LSTSQ_Z = 4

# every symbol declared in include/miid.h
EXPORTED = [
    "miid_version", "miid_last_hip_error",
    "miid_create", "miid_destroy", "miid_handle_device", "miid_handle_rows",
    "miid_id_workspace", "id_cpqr",
    "miid_rid_workspace", "rid_sketch_cpqr",
    "miid_rid_sample_workspace", "rid_sample_cpqr",
    "miid_two_sided_workspace", "id_two_sided",
    "miid_cur_workspace", "id_cur",
    "miid_batched_workspace", "id_batched", "id_batched_noalloc",
    "miid_backward_workspace", "id_backward",
]


# tuning-hint fields of miid_opts.flags (4 bits each, 0 = library default)
MIID_HINT_CPW_SHIFT = 8
MIID_HINT_NP_SHIFT = 12
MIID_HINT_PATH_SHIFT = 16
MIID_HINT_LPC_SHIFT = 20


def hint(shift: int, value: int) -> int:
    """One tuning-hint field of miid_opts.flags."""
    return (int(value) & 15) << shift


class MiidOpts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("kmax", ctypes.c_int32), ("eps", ctypes.c_double),
                ("nb", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class MiidInfo(ctypes.Structure):
    _fields_ = [("k_out", ctypes.c_int32), ("status", ctypes.c_uint32), ("a_norm", ctypes.c_double),
                ("r22_norm", ctypes.c_double), ("n_recompute", ctypes.c_int32), ("n_steps", ctypes.c_int32)]


class MiidError(RuntimeError):
    pass


_lib = None


def load(path: str = LIB_PATH):
    """Load libmiid.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2105_07076_amd/build.py "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    OPTS = ctypes.POINTER(MiidOpts)
    lib.miid_version.restype = ctypes.c_char_p
    lib.miid_version.argtypes = []
    lib.miid_last_hip_error.restype = ctypes.c_int
    lib.miid_last_hip_error.argtypes = []
    H = ctypes.c_void_p  # miid_handle, the first argument of every entry point
    lib.miid_create.restype = ctypes.c_int
    lib.miid_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_char_p]
    lib.miid_destroy.restype = None
    lib.miid_destroy.argtypes = [H]
    lib.miid_handle_device.restype = ctypes.c_int
    lib.miid_handle_device.argtypes = [H]
    lib.miid_handle_rows.restype = ctypes.c_int
    lib.miid_handle_rows.argtypes = [H]
    lib.miid_id_workspace.restype = SZ
    lib.miid_id_workspace.argtypes = [H, I64, I64, ctypes.c_int, OPTS]
    lib.id_cpqr.restype = ctypes.c_int
    lib.id_cpqr.argtypes = [H, P, I64, I64, I64, ctypes.c_int, OPTS, P, P, I64, P, I64, P, I64, P, P, SZ, P]
    lib.miid_rid_sample_workspace.restype = SZ
    lib.miid_rid_sample_workspace.argtypes = [H, I64, I64, I32, ctypes.c_int, OPTS]
    lib.rid_sample_cpqr.restype = ctypes.c_int
    lib.rid_sample_cpqr.argtypes = [H, P, I64, I64, I64, ctypes.c_int, P, I32, OPTS, P, P, I64, P, I64, P, I64, P,
                                    P, SZ, P]
    lib.miid_two_sided_workspace.restype = SZ
    lib.miid_two_sided_workspace.argtypes = [H, I64, I64, ctypes.c_int, OPTS]
    lib.id_two_sided.restype = ctypes.c_int
    lib.id_two_sided.argtypes = [H, P, I64, I64, I64, ctypes.c_int, OPTS, P, P, I64, P, P, I64, P, P, P, SZ, P]
    lib.miid_cur_workspace.restype = SZ
    lib.miid_cur_workspace.argtypes = [H, I64, I64, ctypes.c_int, OPTS]
    lib.id_cur.restype = ctypes.c_int
    lib.id_cur.argtypes = [H, P, I64, I64, I64, ctypes.c_int, OPTS, P, P, P, I64, P, P, P, SZ, P]
    lib.miid_rid_workspace.restype = SZ
    lib.miid_rid_workspace.argtypes = [H, I64, I64, I32, OPTS]
    lib.rid_sketch_cpqr.restype = ctypes.c_int
    lib.rid_sketch_cpqr.argtypes = [H, P, I64, I64, I64, P, I32, I64, I32, OPTS, P, P, I64, P, I64, P, I64,
                                    P, I64, P, P, SZ, P]
    lib.miid_batched_workspace.restype = SZ
    lib.miid_batched_workspace.argtypes = [H, I32, ctypes.c_int]
    lib.id_batched.restype = ctypes.c_int
    lib.id_batched.argtypes = [H, I32, P, P, P, P, ctypes.c_int, OPTS, P, P, P, P, P, P, SZ, P]
    lib.id_batched_noalloc.restype = ctypes.c_int
    lib.id_batched_noalloc.argtypes = [H, I32, P, P, P, P, ctypes.c_int, OPTS, P, P, P, P, P, P]
    lib.miid_backward_workspace.restype = SZ
    lib.miid_backward_workspace.argtypes = [H, I64, I64, I32, ctypes.c_int]
    lib.id_backward.restype = ctypes.c_int
    lib.id_backward.argtypes = [H, P, I64, I64, I64, ctypes.c_int, P, I32, P, I64, P, I64, P, I64, P, I64,
                                P, I64, P, SZ, P]
    _lib = lib
    return lib


class Handle:
    """A miid_handle: the device current at creation and, optionally, a
    tuning table (text rows "routine dtype m n k nb hints")."""

    def __init__(self, autotune_path: str | None = None):
        lib = load()
        h = ctypes.c_void_p()
        rc = lib.miid_create(ctypes.byref(h), autotune_path.encode() if autotune_path else None)
        if rc != 0:
            raise MiidError(f"miid_create: rc={rc}" + (f" (cannot read {autotune_path})" if rc == -2 else ""))
        self.ptr = h.value
        self.path = autotune_path

    @property
    def device(self) -> int:
        return load().miid_handle_device(self.ptr)

    @property
    def rows(self) -> int:
        return load().miid_handle_rows(self.ptr)

    def close(self) -> None:
        if self.ptr:
            load().miid_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def check(rc: int, what: str) -> None:
    if rc == 0:
        return
    if rc == MIID_E_HIP:
        raise MiidError(f"{what}: HIP error {load().miid_last_hip_error()}")
    names = {MIID_E_WORKSPACE: "workspace too small", MIID_E_UNSUPPORTED: "unsupported shape/options"}
    raise MiidError(f"{what}: {names.get(rc, f'invalid argument {-rc}')} (rc={rc})")
