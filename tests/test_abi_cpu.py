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
    o = _abi.MiidOpts()
    o.k = 4
    P = ctypes.c_void_p
    dummy = P(0x1000)  # never dereferenced: validation fails first
    # A null -> -1
    assert lib.id_cpqr(None, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1, dummy, dummy,
                       1 << 30, None) == -1
    # lda < m -> -4
    assert lib.id_cpqr(dummy, 10, 20, 9, 1, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1, dummy, dummy,
                       1 << 30, None) == -4
    # bad dtype -> -5
    assert lib.id_cpqr(dummy, 10, 20, 10, 7, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1, dummy, dummy,
                       1 << 30, None) == -5
    # ldz < k -> -9
    assert lib.id_cpqr(dummy, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, 3, None, 1, None, 1, dummy, dummy,
                       1 << 30, None) == -9
    # workspace too small
    assert lib.id_cpqr(dummy, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1, dummy, dummy,
                       16, None) == _abi.MIID_E_WORKSPACE
    # k above min(m, n) -> unsupported
    o.k = 11
    assert lib.id_cpqr(dummy, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, 11, None, 1, None, 1, dummy, dummy,
                       1 << 30, None) == _abi.MIID_E_UNSUPPORTED
    assert lib.miid_id_workspace(10, 20, 1, ctypes.byref(o)) == 0
    o.k = 4
    assert lib.miid_id_workspace(10, 20, 1, ctypes.byref(o)) > 0
    # randomized ID: m > n unsupported, bad mode -> -8
    assert lib.rid_sketch_cpqr(dummy, 30, 20, 30, dummy, 8, 8, 1, ctypes.byref(o), dummy, dummy, 4, None, 1, None,
                               1, None, 1, dummy, dummy, 1 << 30, None) == _abi.MIID_E_UNSUPPORTED
    assert lib.rid_sketch_cpqr(dummy, 10, 20, 10, dummy, 8, 8, 2, ctypes.byref(o), dummy, dummy, 4, None, 1, None,
                               1, None, 1, dummy, dummy, 1 << 30, None) == -8
    # batched: kmax out of range in the options -> -7
    ob = _abi.MiidOpts()
    ob.k, ob.kmax, ob.eps, ob.nb, ob.flags = 0, 65, 1e-6, 0, 0
    assert lib.id_batched(4, dummy, dummy, dummy, dummy, 0, ctypes.byref(ob), dummy, dummy, dummy, dummy, dummy,
                          dummy, 1 << 30, None) == -7
    ob.kmax = 16
    ob.eps = -1.0
    assert lib.id_batched(4, dummy, dummy, dummy, dummy, 0, ctypes.byref(ob), dummy, dummy, dummy, dummy, dummy,
                          dummy, 1 << 30, None) == -7
    # backward: k > m -> -7
    assert lib.id_backward(dummy, 10, 20, 10, 0, dummy, 11, dummy, 11, dummy, 11, None, 1, None, 1, dummy, 10,
                           dummy, 1 << 30, None) == -7


def test_argument_validation_of_the_sampled_two_sided_and_cur_entry_points():
    _abi, lib = _lib()
    P = ctypes.c_void_p
    dummy = P(0x1000)  # never dereferenced: validation fails first
    big = 1 << 30
    o = _abi.MiidOpts()
    o.k = 4
    tol = _abi.MiidOpts()
    tol.eps, tol.kmax = 1e-3, 4
    # column-sampling RID: idx null -> -6, p > n -> -7, tolerance mode -> -8
    assert lib.rid_sample_cpqr(dummy, 10, 20, 10, 1, None, 6, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1,
                               dummy, dummy, big, None) == -6
    assert lib.rid_sample_cpqr(dummy, 10, 20, 10, 1, dummy, 21, ctypes.byref(o), dummy, dummy, 4, None, 1, None, 1,
                               dummy, dummy, big, None) == -7
    assert lib.rid_sample_cpqr(dummy, 10, 20, 10, 1, dummy, 6, ctypes.byref(tol), dummy, dummy, 4, None, 1, None, 1,
                               dummy, dummy, big, None) == -8
    assert lib.miid_rid_sample_workspace(10, 20, 6, 1, ctypes.byref(o)) > 0
    # two-sided ID: fixed rank only; any shape (the column stage keeps columns)
    assert lib.miid_two_sided_workspace(10, 20, 1, ctypes.byref(o)) > 0
    assert lib.miid_two_sided_workspace(30, 20, 1, ctypes.byref(o)) > 0
    assert lib.miid_two_sided_workspace(10, 20, 1, ctypes.byref(tol)) == 0
    # ldw < m -> -12
    assert lib.id_two_sided(dummy, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, 4, dummy, dummy, 9, dummy, dummy,
                            dummy, big, None) == -12
    # CUR: ldu < k -> -10
    assert lib.miid_cur_workspace(10, 20, 1, ctypes.byref(o)) > 0
    assert lib.id_cur(dummy, 10, 20, 10, 1, ctypes.byref(o), dummy, dummy, dummy, 3, dummy, dummy, dummy, big,
                      None) == -10
    # sketch RID with the least-squares Z: more workspace; fixed rank only
    ol = _abi.MiidOpts()
    ol.k, ol.flags = 4, _abi.MIID_LSTSQ_Z
    assert lib.miid_rid_workspace(10, 20, 8, ctypes.byref(ol)) > lib.miid_rid_workspace(10, 20, 8, ctypes.byref(o))
    tol.flags = _abi.MIID_LSTSQ_Z
    assert lib.miid_rid_workspace(10, 20, 8, ctypes.byref(tol)) == 0
