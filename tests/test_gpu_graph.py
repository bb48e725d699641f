"""The ID entry points under HIP graph capture: id_cpqr (fixed rank),
rid_sketch_cpqr (also with the least-squares Z), rid_sample_cpqr,
id_two_sided and id_batched are enqueued on the capturing stream with
caller-owned buffers and no host synchronisation, so torch.cuda.CUDAGraph can
record them.  Every replay (with eager work and synchronisations between the
replays) must reproduce the eager result bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

import idgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _miid():
    import paper_2105_07076_amd as miid
    miid.load()
    return miid


def _capture_and_check(run, outputs):
    """run() enqueues the call on the current stream writing into the
    tensors of `outputs`; the eager result is compared with three replays."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()  # warm-up: workspace allocation and one-time kernel attributes
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref = [o.clone() for o in outputs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    torch.cuda.synchronize()
    for rep in range(3):
        for o in outputs:
            o.zero_()
        junk = torch.randn(1024, 1024, device="cuda") @ torch.randn(1024, 1024, device="cuda")
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outputs, ref):
            assert torch.equal(o, r), f"replay {rep} differs from the eager result"
        del junk


def test_graph_id_fixed_rank():
    miid = _miid()
    from paper_2105_07076_amd import api
    A = idgen.lowrank_plus_noise_device(12, 512, 2048, np.exp(-np.arange(512) / 32.0), 1e-8,
                                        dtype=torch.float64)
    out = api.id_raw(A, k=64, want_R11=True)
    torch.cuda.synchronize()
    _capture_and_check(lambda: api.id_raw(A, k=64, want_R11=True, out=out),
                       [out["J"], out["Z"], out["C"], out["R11"], out["info"]])


def test_graph_rid():
    miid = _miid()
    from paper_2105_07076_amd import api
    A = idgen.lowrank_plus_noise_device(13, 1024, 4096, np.exp(-np.arange(1024) / 64.0), 1e-8,
                                        dtype=torch.float32)
    Om = torch.tensor(idgen.omega_bf16(14, 138, 1024), dtype=torch.bfloat16, device="cuda").t().contiguous().t()
    out = api.rid_raw(A, Om, k=128, mode=1)
    torch.cuda.synchronize()
    _capture_and_check(lambda: api.rid_raw(A, Om, k=128, mode=1, out=out),
                       [out["J"], out["Z"], out["info"]])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_graph_batched(dtype):
    """The batched launch (LPT ordering, queue reset and the persistent
    kernel) replayed from one graph."""
    miid = _miid()
    from paper_2105_07076_amd import api
    blocks = idgen.batched_blocks(seed=45, nblk=300)
    A = torch.tensor(blocks.A, dtype=dtype, device="cuda")
    out = api.batched_raw(A, blocks.a_off, blocks.m, blocks.n, 1e-6, 64)
    torch.cuda.synchronize()
    _capture_and_check(lambda: api.batched_raw(A, blocks.a_off, blocks.m, blocks.n, 1e-6, 64, out=out),
                       [out["J"], out["Z"], out["info"]])


def test_graph_rid_sample_and_lstsq_and_two_sided():
    """The column-sampling RID, the sketch RID with the least-squares Z and
    the two-sided ID under capture (the same kernels plus the Gram, Cholesky
    and transposes)."""
    miid = _miid()
    from paper_2105_07076_amd import api
    A = idgen.lowrank_plus_noise_device(15, 384, 1500, np.exp(-np.arange(384) / 32.0), 1e-8,
                                        dtype=torch.float64)
    idx = torch.tensor(idgen.column_sample(16, 1500, 48), dtype=torch.int32, device="cuda")  # no copy in capture
    out = api.rid_sample_raw(A, idx, 48, want_R11=True)
    torch.cuda.synchronize()
    _capture_and_check(lambda: api.rid_sample_raw(A, idx, 48, want_R11=True, out=out),
                       [out["J"], out["Z"], out["C"], out["R11"], out["info"]])
    A32 = A.to(torch.float32)
    Om = torch.tensor(idgen.omega_bf16(17, 58, 384), dtype=torch.bfloat16, device="cuda").t().contiguous().t()
    out2 = api.rid_raw(A32, Om, k=48, mode=1, lstsq=True, want_R11=True)
    torch.cuda.synchronize()
    _capture_and_check(lambda: api.rid_raw(A32, Om, k=48, mode=1, lstsq=True, want_R11=True, out=out2),
                       [out2["J"], out2["Z"], out2["R11"], out2["info"]])
    out3 = api.two_sided_raw(A, 40)
    torch.cuda.synchronize()
    _capture_and_check(lambda: api.two_sided_raw(A, 40, out=out3),
                       [out3["J"], out3["Z"], out3["I"], out3["W"], out3["info"], out3["info_rows"]])
