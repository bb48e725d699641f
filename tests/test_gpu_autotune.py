"""The autotuner on the GPU: it times real candidates, and what it returns is
a launch shape only -- the tuned call computes the same ID as the default."""
from __future__ import annotations

import numpy as np
import pytest

import idgen
from gpu_helpers import rel, t_part, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mods():
    import paper_2105_07076_amd as miid
    from paper_2105_07076_amd import autotune, api
    miid.load()
    return miid, autotune, api


def test_tune_id_same_result():
    miid, autotune, api = _mods()
    A = idgen.lowrank_plus_noise_device(21, 1024, 4096, np.exp(-np.arange(1024) / 64.0), 1e-8,
                                        dtype=torch.float64)
    cands = [c for c in autotune.id_candidates(1024, 4096, torch.float64) if c[1] in (16, 32)]
    ch = autotune.tune_id(1024, 4096, 128, torch.float64, A=A, reps=2, candidates=cands)
    assert ch.label in ch.timings and ch.ms == min(ch.timings.values()) and len(ch.timings) == len(cands)
    r0 = miid.id(A, k=128)
    r1 = miid.id(A, k=128, nb=ch.nb, hints=ch.hints)
    J0, J1 = to_np(r0.J), to_np(r1.J)
    assert np.array_equal(J0, J1)
    assert rel(t_part(to_np(r1.Z), J1), t_part(to_np(r0.Z), J0)) <= 1e-12


def test_tune_rid_paths_agree():
    """Fused and blocked candidates of the sketch's CPQR give the same pivots."""
    miid, autotune, api = _mods()
    A = idgen.lowrank_plus_noise_device(22, 1024, 4096, np.exp(-np.arange(1024) / 64.0), 1e-8,
                                        dtype=torch.float32)
    Om = torch.tensor(idgen.omega_bf16(23, 138, 1024), dtype=torch.bfloat16, device="cuda")
    cands = autotune.id_candidates(138, 4096, torch.float32, for_rid=True)
    cands = [c for c in cands if c[1] == 32]
    ch = autotune.tune_rid(A, Om, 128, reps=2, candidates=cands)
    assert any(l.startswith("fused") for l in ch.timings) and any(l.startswith("blocked") for l in ch.timings)
    ref = miid.rid(A, Om, k=128)
    for label, nb, hints in cands:
        r = miid.rid(A, Om, k=128, nb=nb, hints=hints)
        assert np.array_equal(to_np(r.J), to_np(ref.J)), label
        assert rel(to_np(r.Z).astype(np.float64), to_np(ref.Z).astype(np.float64)) <= 1e-5, label


def test_tune_batched_lane_caps_same_ids():
    """The lanes-per-column cap changes the launch shape and the order of
    the partial sums only: in FP64 every candidate selects the same columns
    and its Z agrees to rounding."""
    miid, autotune, api = _mods()
    blocks = idgen.batched_blocks(seed=46, nblk=200)
    A = torch.tensor(blocks.A, dtype=torch.float64, device="cuda")
    ch = autotune.tune_batched(A, blocks.a_off, blocks.m, blocks.n, 1e-6, 64, reps=2)
    assert len(ch.timings) == len(autotune.batched_candidates())
    ref = miid.batched(A, blocks.a_off, blocks.m, blocks.n, 1e-6, 64)
    for label, _, hints in autotune.batched_candidates():
        r = miid.batched(A, blocks.a_off, blocks.m, blocks.n, 1e-6, 64, hints=hints)
        assert np.array_equal(r.k, ref.k), label
        assert torch.equal(r.J, ref.J), label
        assert rel(to_np(r.Z), to_np(ref.Z)) <= 1e-10, label


def test_native_table_applies_to_calls(tmp_path):
    """A handle created with a tuning table runs a call that leaves nb and the
    hints at 0 with the matching row's launch shape: the same bits as the
    call that passes that shape itself."""
    miid, autotune, api = _mods()
    from paper_2105_07076_amd import _abi
    A = idgen.lowrank_plus_noise_device(22, 512, 3000, np.exp(-np.arange(512) / 64.0), 1e-8,
                                        dtype=torch.float64)
    hints = _abi.hint(_abi.MIID_HINT_PATH_SHIFT, 1) | _abi.hint(_abi.MIID_HINT_CPW_SHIFT, 4)
    path = tmp_path / "tune.txt"
    path.write_text(f"id f64 512 3000 96 16 {hints:#x}\n")
    try:
        api.set_tuning_table(str(path))
        h = api.handle()
        assert h.rows == 1 and h.device == torch.cuda.current_device()
        r_tab = miid.id(A, k=96)
    finally:
        api.set_tuning_table(None)
    r_exp = miid.id(A, k=96, nb=16, hints=hints)
    r_def = miid.id(A, k=96)
    assert torch.equal(r_tab.J, r_exp.J) and torch.equal(r_tab.Z, r_exp.Z)
    assert torch.equal(r_tab.J, r_def.J)
    assert rel(t_part(to_np(r_tab.Z), to_np(r_tab.J)), t_part(to_np(r_def.Z), to_np(r_def.J))) <= 1e-12
