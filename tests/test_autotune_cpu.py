"""Host-side pieces of the autotuner: hint encoding, candidate lists, the
JSON table (no GPU)."""
from __future__ import annotations

import pytest

torch = pytest.importorskip("torch")

from paper_2105_07076_amd import _abi, autotune  # noqa: E402


def test_hint_fields_match_header():
    hdr = open(__import__("os").path.join(__import__("os").path.dirname(__file__), "..", "include", "miid.h")).read()
    for name in ["MIID_HINT_CPW_SHIFT", "MIID_HINT_NP_SHIFT", "MIID_HINT_PATH_SHIFT", "MIID_HINT_LPC_SHIFT"]:
        line = next(l for l in hdr.splitlines() if l.startswith(f"#define {name} "))
        assert int(line.split()[2]) == getattr(_abi, name)
    assert _abi.hint(_abi.MIID_HINT_NP_SHIFT, 4) == 4 << 12
    assert _abi.hint(_abi.MIID_HINT_LPC_SHIFT, 17) == 1 << 20   # 4-bit field


def test_id_candidates():
    # 266-row FP32 sketch: fused candidates present; 4096-row FP64 ID: blocked only
    c1 = autotune.id_candidates(266, 16384, torch.float32, for_rid=True)
    assert any(lbl.startswith("fused") for lbl, _, _ in c1)
    c2 = autotune.id_candidates(4096, 16384, torch.float64)
    assert all(lbl.startswith("blocked") for lbl, _, _ in c2)
    assert {nb for _, nb, _ in c2} == {16, 32, 48, 64}
    # FP64: 320 rows (ten 16-byte groups per lane) still fused, 321 not
    c3 = autotune.id_candidates(300, 1000, torch.float64)
    assert any(lbl.startswith("fused") for lbl, _, _ in c3)
    c4 = autotune.id_candidates(321, 1000, torch.float64)
    assert all(lbl.startswith("blocked") for lbl, _, _ in c4)
    # FP32 reaches 576 rows
    assert any(lbl.startswith("fused") for lbl, _, _ in autotune.id_candidates(576, 4096, torch.float32))
    assert all(lbl.startswith("blocked") for lbl, _, _ in autotune.id_candidates(577, 4096, torch.float32))
    assert len(autotune.batched_candidates()) == 4


def test_table_roundtrip(tmp_path):
    t = autotune.Table(str(tmp_path / "tune.json"))
    k = autotune.key("id", torch.float64, (4096, 16384, 256), device="MI355X")
    assert k == "MI355X|id|float64|4096x16384x256"
    assert t.get(k) is None
    t.put(k, autotune.Choice(nb=32, hints=autotune.H(_abi.MIID_HINT_CPW_SHIFT, 1), ms=29.6, label="x",
                             timings={"x": 29.6}))
    t.save()
    t2 = autotune.Table(str(tmp_path / "tune.json"))
    c = t2.get(k)
    assert c.nb == 32 and c.hints == 1 << 8 and c.label == "x"


def test_table_exports_the_native_rows(tmp_path):
    """The JSON table's entries for one device become rows the library's
    miid_create accepts; the exported panel width reaches the workspace."""
    import ctypes
    t = autotune.Table()
    t.put(autotune.key("id", torch.float64, (100, 300, 4), device="dev0"),
          autotune.Choice(nb=64, hints=autotune.H(_abi.MIID_HINT_PATH_SHIFT, 1), ms=1.0, label="x"))
    t.put(autotune.key("batched", torch.float32, (4096, 0, 64), device="dev0"),
          autotune.Choice(nb=0, hints=autotune.H(_abi.MIID_HINT_LPC_SHIFT, 4), ms=1.0, label="y"))
    t.put(autotune.key("id", torch.float64, (8, 8, 2), device="other"),
          autotune.Choice(nb=16, hints=0, ms=1.0, label="z"))
    path = str(tmp_path / "native.txt")
    assert t.export_native(path, device="dev0") == 2
    text = open(path).read()
    assert "id f64 100 300 4 64 0x10000" in text
    assert "batched f32 4096 0 64 0 0x400000" in text
    lib = _abi.load()
    h = _abi.Handle(path)
    assert h.rows == 2
    o = _abi.MiidOpts()
    o.k = 4
    o64 = _abi.MiidOpts()
    o64.k, o64.nb = 4, 64
    hp = ctypes.c_void_p(h.ptr)
    assert (lib.miid_id_workspace(hp, 100, 300, 1, ctypes.byref(o))
            == lib.miid_id_workspace(None, 100, 300, 1, ctypes.byref(o64)))
    h.close()
