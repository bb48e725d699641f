"""id_batched_noalloc (the allocation-free batched entry point) against
id_batched on the same inputs: the same kernels, so every block the static
scratch can hold gets bit-identical J, Z and info; a block that needs more
scratch rows per lane than the call's share gets k_out = 0 and
MIID_BLOCK_UNSUPPORTED.  Two calls in a row, the second with a smaller input
(and another element type), then a third, so that what the scratch holds
from one call cannot leak into the next."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import idgen
from gpu_helpers import to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = 1e-6
UNSUPPORTED = 16

# The kernel's storage of a block, restated for the test: rows per lane in
# registers (one column per lane / two), rows per lane in LDS, and the
# largest count of scratch rows any admissible block needs.
REG_ROWS = {4: (168, 64), 8: (80, 48)}
LDS_ROWS = {4: 76, 8: 36}
GLOB_MAX = {4: 372, 8: 428}
SCRATCH = 64 << 20


def _glob_rows(m: int, n: int, esz: int) -> int:
    c2 = n > 512
    L = 1
    if not c2:
        while L < 8 and n * 2 * L <= 512:
            L *= 2
    nq4 = ((m + 3) // 4 + L - 1) // L
    nvc = (2 if c2 else 1) * nq4
    ncr = (REG_ROWS[esz][1] if c2 else REG_ROWS[esz][0]) // 4
    return max(0, 4 * (nvc - ncr - LDS_ROWS[esz] // 4))


def _rg(nblk: int, esz: int) -> int:
    grid = min(nblk, torch.cuda.get_device_properties(0).multi_processor_count)
    r = ((SCRATCH - (1 << 20) - 256) // (grid * 512 * esz)) & ~3
    return min(r, GLOB_MAX[esz])


def _infos(raw: torch.Tensor, nblk: int):
    from paper_2105_07076_amd import _abi
    b = raw.cpu().numpy().tobytes()
    sz = ctypes.sizeof(_abi.MiidInfo)
    return [_abi.MiidInfo.from_buffer_copy(b[i * sz:(i + 1) * sz]) for i in range(nblk)]


def _compare(blocks, dtype):
    """Both entry points on the same blocks; returns the number of blocks the
    allocation-free call left out."""
    from paper_2105_07076_amd import api
    esz = 8 if dtype == torch.float64 else 4
    A = torch.tensor(blocks.A, dtype=dtype, device="cuda")
    ref = api.batched_raw(A, blocks.a_off, blocks.m, blocks.n, EPS, 64)
    out = api.batched_raw(A, blocks.a_off, blocks.m, blocks.n, EPS, 64, noalloc=True)
    torch.cuda.synchronize()
    nblk = len(blocks.m)
    iref, iout = _infos(ref["info"], nblk), _infos(out["info"], nblk)
    rg = _rg(nblk, esz)
    Jr, Jo, Zr, Zo = to_np(ref["J"]), to_np(out["J"]), to_np(ref["Z"]), to_np(out["Z"])
    left_out = 0
    for b in range(nblk):
        m, n = int(blocks.m[b]), int(blocks.n[b])
        if _glob_rows(m, n, esz) > rg:
            left_out += 1
            assert iout[b].k_out == 0 and iout[b].status == UNSUPPORTED, f"block {b} ({m}x{n})"
            continue
        assert iout[b].k_out == iref[b].k_out and iout[b].status == iref[b].status, f"block {b}"
        assert iout[b].a_norm == iref[b].a_norm and iout[b].r22_norm == iref[b].r22_norm, f"block {b}"
        jo, kb = int(ref["j_off_h"][b]), int(ref["kmax_b"][b])
        assert np.array_equal(Jo[jo:jo + kb], Jr[jo:jo + kb]), f"block {b}"
        zo = int(ref["z_off_h"][b])
        assert np.array_equal(Zo[zo:zo + kb * n], Zr[zo:zo + kb * n]), f"block {b}"
    return left_out


def test_noalloc_matches_id_batched_on_consecutive_calls():
    import paper_2105_07076_amd as miid
    miid.load()
    # 1: the 4096-block FP32 workload (every block fits the static scratch)
    big = idgen.batched_blocks(seed=4, nblk=4096)
    assert _compare(big, torch.float32) == 0
    # 2: a smaller FP64 batch with wide blocks; the two tallest wide ones need
    # more scratch rows than this call's share and are left out
    ms = [8, 40, 100, 256, 256, 200, 64, 128] + list(idgen.rng(51).integers(32, 257, size=62))
    ns = [513, 600, 777, 1024, 700, 1000, 64, 200] + [int(idgen.rng(52 + i).integers(m, 2 * m + 1))
                                                     for i, m in enumerate(ms[8:])]
    wide = idgen.kernel_blocks_sized(50, ms, ns)
    assert _compare(wide, torch.float64) >= 2
    # 3: smaller again, FP32
    small = idgen.batched_blocks(seed=53, nblk=12, mmin=1, mmax=64)
    assert _compare(small, torch.float32) == 0


def test_noalloc_rejects_too_many_blocks():
    from paper_2105_07076_amd import _abi, api
    lib = _abi.load()
    opts = _abi.MiidOpts()
    opts.kmax, opts.eps = 8, EPS
    d = torch.empty(16, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(d.data_ptr())
    rc = lib.id_batched_noalloc(ctypes.c_void_p(api.handle().ptr), (1 << 18) + 1, p, p, p, p, _abi.MIID_F64,
                                ctypes.byref(opts), p, p, p, p, p, None)
    assert rc == _abi.MIID_E_UNSUPPORTED
