"""CPU checks of the C ABI: the built library loads without a GPU, exports
every function include/miid.h declares, its struct layouts match the ctypes
mirrors, and argument validation returns the documented codes before any
device work (no compute calls are made here)."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "miid.h")


def _lib():
    from paper_2105_07076_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2105_07076_amd import build
        build.build()
    return _abi, _abi.load()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for must in ["id_cpqr", "rid_sketch_cpqr", "id_batched", "id_backward"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    _abi, lib = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s+(\S+)", out))
    missing = [n for n in _declared_functions() if n not in exported]
    assert not missing, missing
    for n in _declared_functions():
        assert hasattr(lib, n)
    assert set(_abi.EXPORTED) <= exported


def test_struct_layouts():
    _abi, _ = _lib()
    assert ctypes.sizeof(_abi.MiidOpts) == 24
    assert ctypes.sizeof(_abi.MiidInfo) == 32
    assert _abi.MiidInfo.r22_norm.offset == 16


def test_version_string():
    _, lib = _lib()
    assert lib.miid_version().startswith(b"miid")


def test_argument_validation_before_any_device_work():
    _abi, lib = _lib()
    hd = _abi.Handle()
    h = ctypes.c_void_p(hd.ptr)
    o = _abi.MiidOpts()
    o.k = 4
    P = ctypes.c_void_p
    dummy = P(0x1000)  # never dereferenced: validation fails first
    # A null -> -2 (the handle is argument 1)
    assert lib.id_cpqr(h, None, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1, dummy, dummy,
                       1 << 30, None) == -2
    # lda < m -> -5
    assert lib.id_cpqr(h, dummy, 10, 20, 9, 1, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1, dummy, dummy,
                       1 << 30, None) == -5
    # bad dtype -> -6
    assert lib.id_cpqr(h, dummy, 10, 20, 10, 7, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1, dummy, dummy,
                       1 << 30, None) == -6
    # ldz < k -> -10
    assert lib.id_cpqr(h, dummy, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, 3, None, 1, None, 1, dummy, dummy,
                       1 << 30, None) == -10
    # workspace too small
    assert lib.id_cpqr(h, dummy, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1, dummy, dummy,
                       16, None) == _abi.MIID_E_WORKSPACE
    # k above min(m, n) -> unsupported
    o.k = 11
    assert lib.id_cpqr(h, dummy, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, 11, None, 1, None, 1, dummy, dummy,
                       1 << 30, None) == _abi.MIID_E_UNSUPPORTED
    assert lib.miid_id_workspace(h, 10, 20, 1, ctypes.byref(o)) == 0
    o.k = 4
    assert lib.miid_id_workspace(h, 10, 20, 1, ctypes.byref(o)) > 0
    # randomized ID: m > n unsupported, bad mode -> -9
    assert lib.rid_sketch_cpqr(h, dummy, 30, 20, 30, dummy, 8, 8, 1, ctypes.byref(o), dummy, dummy, 4, None, 1, None,
                               1, None, 1, dummy, dummy, 1 << 30, None) == _abi.MIID_E_UNSUPPORTED
    assert lib.rid_sketch_cpqr(h, dummy, 10, 20, 10, dummy, 8, 8, 3, ctypes.byref(o), dummy, dummy, 4, None, 1, None,
                               1, None, 1, dummy, dummy, 1 << 30, None) == -9
    # batched: kmax out of range in the options -> -8
    ob = _abi.MiidOpts()
    ob.k, ob.kmax, ob.eps, ob.nb, ob.flags = 0, 65, 1e-6, 0, 0
    assert lib.id_batched(h, 4, dummy, dummy, dummy, dummy, 0, ctypes.byref(ob), dummy, dummy, dummy, dummy, dummy,
                          dummy, 1 << 30, None) == -8
    ob.kmax = 16
    ob.eps = -1.0
    assert lib.id_batched(h, 4, dummy, dummy, dummy, dummy, 0, ctypes.byref(ob), dummy, dummy, dummy, dummy, dummy,
                          dummy, 1 << 30, None) == -8
    # backward: k > m -> -8
    assert lib.id_backward(h, dummy, 10, 20, 10, 0, dummy, 11, dummy, 11, dummy, 11, None, 1, None, 1, dummy, 10,
                           dummy, 1 << 30, None) == -8


def test_argument_validation_of_the_sampled_two_sided_and_cur_entry_points():
    _abi, lib = _lib()
    h = None  # NULL handle: no tuning table
    P = ctypes.c_void_p
    dummy = P(0x1000)  # never dereferenced: validation fails first
    big = 1 << 30
    o = _abi.MiidOpts()
    o.k = 4
    tol = _abi.MiidOpts()
    tol.eps, tol.kmax = 1e-3, 4
    # column-sampling RID: idx null -> -7, p > n -> -8, tolerance mode -> -9
    assert lib.rid_sample_cpqr(h, dummy, 10, 20, 10, 1, None, 6, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1,
                               dummy, dummy, big, None) == -7
    assert lib.rid_sample_cpqr(h, dummy, 10, 20, 10, 1, dummy, 21, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1,
                               dummy, dummy, big, None) == -8
    assert lib.rid_sample_cpqr(h, dummy, 10, 20, 10, 1, dummy, 6, ctypes.byref(tol), dummy, dummy, 4, None, 1, None, 1,
                               dummy, dummy, big, None) == -9
    assert lib.miid_rid_sample_workspace(h, 10, 20, 6, 1, ctypes.byref(o)) > 0
    # two-sided ID: fixed rank only; any shape (the column stage keeps columns)
    assert lib.miid_two_sided_workspace(h, 10, 20, 1, ctypes.byref(o)) > 0
    assert lib.miid_two_sided_workspace(h, 30, 20, 1, ctypes.byref(o)) > 0
    assert lib.miid_two_sided_workspace(h, 10, 20, 1, ctypes.byref(tol)) == 0
    # ldw < m -> -13
    assert lib.id_two_sided(h, dummy, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, 4, dummy, dummy, 9, dummy, dummy,
                            dummy, big, None) == -13
    # CUR: ldu < k -> -11
    assert lib.miid_cur_workspace(h, 10, 20, 1, ctypes.byref(o)) > 0
    assert lib.id_cur(h, dummy, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, dummy, 3, dummy, dummy, dummy, big,
                      None) == -11
    # sketch RID with the least-squares Z: more workspace; fixed rank only
    ol = _abi.MiidOpts()
    ol.k, ol.flags = 4, _abi.MIID_LSTSQ_Z
    assert lib.miid_rid_workspace(h, 10, 20, 8, ctypes.byref(ol)) > lib.miid_rid_workspace(h, 10, 20, 8, ctypes.byref(o))
    tol.flags = _abi.MIID_LSTSQ_Z
    assert lib.miid_rid_workspace(h, 10, 20, 8, ctypes.byref(tol)) == 0


def test_handle_create_destroy_and_workspace_queries(tmp_path):
    """miid_create without a visible device gives a handle for the workspace
    queries (device -1); the tuning table's rows change the launch shape a
    call runs with, and so its workspace, only when the caller leaves nb and
    the hint fields at 0; a malformed table creates no handle."""
    _abi, lib = _lib()
    o = _abi.MiidOpts()
    o.k = 4
    plain = _abi.Handle()
    assert plain.rows == 0
    assert plain.device == -1  # no GPU in this process
    hp = ctypes.c_void_p(plain.ptr)
    w_null = lib.miid_id_workspace(None, 100, 300, 1, ctypes.byref(o))
    assert w_null > 0
    assert lib.miid_id_workspace(hp, 100, 300, 1, ctypes.byref(o)) == w_null
    # a row for this shape with panel width 64 (the library's default is 32):
    # the panel-sized parts of the workspace grow
    table = tmp_path / "tune.txt"
    table.write_text("# routine dtype m n k nb hints\n"
                     "id f64 100 300 4 64 0x10000\n"
                     "id f64 0 0 0 16 0\n"
                     "batched f32 0 0 0 0 0x400000\n")
    tuned = _abi.Handle(str(table))
    assert tuned.rows == 3
    ht = ctypes.c_void_p(tuned.ptr)
    w_tuned = lib.miid_id_workspace(ht, 100, 300, 1, ctypes.byref(o))
    o64 = _abi.MiidOpts()
    o64.k, o64.nb = 4, 64
    assert w_tuned == lib.miid_id_workspace(None, 100, 300, 1, ctypes.byref(o64))
    assert w_tuned > w_null
    # another shape takes the wildcard row (nb = 16)
    o16 = _abi.MiidOpts()
    o16.k, o16.nb = 4, 16
    assert (lib.miid_id_workspace(ht, 100, 400, 1, ctypes.byref(o))
            == lib.miid_id_workspace(None, 100, 400, 1, ctypes.byref(o16)))
    # the caller's own nb wins over the table
    o.nb = 32
    assert lib.miid_id_workspace(ht, 100, 300, 1, ctypes.byref(o)) == w_null
    # FP32 rows do not apply to FP64 calls
    o.nb = 0
    assert lib.miid_id_workspace(ht, 100, 300, 0, ctypes.byref(o)) == lib.miid_id_workspace(None, 100, 300, 0,
                                                                                            ctypes.byref(o))
    # batched workspace through a handle
    assert lib.miid_batched_workspace(ht, 64, 0) == lib.miid_batched_workspace(None, 64, 0) > 0
    tuned.close()
    plain.close()
    # errors: NULL out, unreadable file, malformed rows
    assert lib.miid_create(None, None) == -1
    hh = ctypes.c_void_p()
    assert lib.miid_create(ctypes.byref(hh), str(tmp_path / "missing.txt").encode()) == -2
    for bad in ["id f64 1 2 3\n", "qr f64 0 0 0 0 0\n", "id f16 0 0 0 0 0\n", "id f64 0 0 0 65 0\n",
                "id f64 0 0 0 0 0x1\n", "id f64 0 0 0 0 0 extra\n"]:
        table.write_text(bad)
        hh = ctypes.c_void_p()
        assert lib.miid_create(ctypes.byref(hh), str(table).encode()) == -2, bad
        assert not hh.value
    lib.miid_destroy(None)  # a no-op
