"""Autotuner for the launch shapes of the ID kernels.

The library's tuning knobs change launch shapes only, never what is computed:
the panel width nb and the MIID_HINT fields of miid_opts.flags (columns per
wave of the blocked path's F-GEMV, column passes per wave of the fused
short-matrix path, the path itself, and the lanes per column of the
batched kernel).  :func:`tune_id` and :func:`tune_batched` time every
candidate on the caller's own data (or a seeded synthetic matrix of the given
shape) with HIP events and return the fastest; :class:`Table` keeps results
in a JSON file keyed by device, routine, dtype and shape, so a tuned shape is
looked up instead of re-timed, and exports them as the library's own tuning
table, which a miid_handle applies to calls that leave the knobs at 0.
"""
from __future__ import annotations

import itertools
import json
import os
from dataclasses import asdict, dataclass, field

import torch

from . import _abi
from . import api

H = _abi.hint


@dataclass
class Choice:
    """A tuned launch configuration and its measured time."""
    nb: int
    hints: int
    ms: float
    label: str
    timings: dict = field(default_factory=dict)


def _time(fn, reps: int) -> float:
    fn()  # warm-up (workspace, one-time kernel attributes)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def id_candidates(m: int, n: int, dtype: torch.dtype, for_rid: bool = False):
    """(label, nb, hints) candidates for an ID whose CPQR works on m x n
    (m <= n after the transpose rule).  The fused path exists for at most
    576 rows in FP32 (320 in FP64) and panels of at most 32."""
    esz = 4 if (for_rid or dtype == torch.float32) else 8
    ldw = (m + 63) // 64 * 64
    fused_ok = ldw <= 576 and (ldw * esz // 16 + 15) // 16 <= (10 if esz == 8 else 9)
    out = []
    for nb, cpw in itertools.product((16, 32, 48, 64), (1, 2, 4)):
        out.append((f"blocked nb={nb} cpw={cpw}", nb,
                    H(_abi.MIID_HINT_PATH_SHIFT, 1) | H(_abi.MIID_HINT_CPW_SHIFT, cpw)))
    if fused_ok:
        for nb, np_ in itertools.product((16, 32), (1, 2, 4, 8)):
            out.append((f"fused nb={nb} np={np_}", nb,
                        H(_abi.MIID_HINT_PATH_SHIFT, 2) | H(_abi.MIID_HINT_NP_SHIFT, np_)))
    return out


def _synthetic(m: int, n: int, dtype: torch.dtype, seed: int = 0) -> torch.Tensor:
    """A seeded m x n column-major matrix with a decaying spectrum."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    r = min(m, n)
    U = torch.linalg.qr(torch.randn(m, r, generator=g, device="cuda", dtype=torch.float64))[0]
    V = torch.linalg.qr(torch.randn(n, r, generator=g, device="cuda", dtype=torch.float64))[0]
    s = torch.exp(-torch.arange(r, device="cuda", dtype=torch.float64) / max(1.0, r / 64.0))
    A = (V * s) @ U.T + 1e-8 * torch.randn(n, m, generator=g, device="cuda", dtype=torch.float64)
    return A.to(dtype).t()


def tune_id(m: int, n: int, k: int, dtype: torch.dtype = torch.float64, A: torch.Tensor | None = None,
            reps: int = 3, candidates=None) -> Choice:
    """Fastest (nb, hints) for a fixed-rank ID of an m x n matrix."""
    if A is None:
        A = _synthetic(m, n, dtype)
    mw, nw = min(m, n), max(m, n)
    cands = candidates or id_candidates(mw, nw, dtype)
    out = api.id_raw(A, k=k)
    timings = {}
    for label, nb, hints in cands:
        if k > mw:
            continue
        timings[label] = _time(lambda: api.id_raw(A, k=k, nb=nb, hints=hints, out=out), reps)
    best = min(timings, key=timings.get)
    nb, hints = next((c[1], c[2]) for c in cands if c[0] == best)
    return Choice(nb=nb, hints=hints, ms=timings[best], label=best, timings=timings)


def tune_rid(A: torch.Tensor, omega: torch.Tensor, k: int, mode: int = 1, reps: int = 3,
             candidates=None) -> Choice:
    """Fastest (nb, hints) for a fixed-rank randomized ID of A with sketch omega."""
    l, n = omega.shape[0], A.shape[1]
    cands = candidates or id_candidates(l, n, torch.float32, for_rid=True)
    out = api.rid_raw(A, omega, k=k, mode=mode)
    timings = {}
    for label, nb, hints in cands:
        timings[label] = _time(lambda: api.rid_raw(A, omega, k=k, mode=mode, nb=nb, hints=hints, out=out),
                               reps)
    best = min(timings, key=timings.get)
    nb, hints = next((c[1], c[2]) for c in cands if c[0] == best)
    return Choice(nb=nb, hints=hints, ms=timings[best], label=best, timings=timings)


def batched_candidates():
    """Caps on the lanes per column of the batched kernel (1, 2, 4, 8)."""
    return [(f"lanes<={l}", 0, H(_abi.MIID_HINT_LPC_SHIFT, l)) for l in (1, 2, 4, 8)]


def tune_batched(A: torch.Tensor, a_off, m, n, eps: float, kmax: int = 64, reps: int = 3,
                 candidates=None) -> Choice:
    """Fastest lanes-per-column cap for one batch of blocks (the caller's own
    blocks)."""
    cands = candidates or batched_candidates()
    out = api.batched_raw(A, a_off, m, n, eps, kmax)
    timings = {}
    for label, _, hints in cands:
        timings[label] = _time(lambda: api.batched_raw(A, a_off, m, n, eps, kmax, out=out, hints=hints), reps)
    best = min(timings, key=timings.get)
    hints = next(c[2] for c in cands if c[0] == best)
    return Choice(nb=0, hints=hints, ms=timings[best], label=best, timings=timings)


def key(routine: str, dtype, shape, device=None) -> str:
    """Table key: device name | routine | dtype | shape."""
    if device is None:
        device = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    dt = str(dtype).replace("torch.", "")
    return "|".join([device, routine, dt, "x".join(str(int(v)) for v in shape)])


class Table:
    """Tuned configurations in a JSON file: key -> {nb, hints, ms, label}."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.entries: dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, k: str) -> Choice | None:
        e = self.entries.get(k)
        return Choice(nb=e["nb"], hints=e["hints"], ms=e["ms"], label=e["label"]) if e else None

    def put(self, k: str, c: Choice) -> None:
        d = asdict(c)
        d.pop("timings", None)
        self.entries[k] = d

    def save(self, path: str | None = None) -> None:
        p = path or self.path
        if not p:
            raise ValueError("no path for the table")
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, p)

    def export_native(self, path: str, device: str | None = None) -> int:
        """Write the entries of ``device`` (default: the current GPU's name)
        as the library's own tuning table -- rows "routine dtype m n k nb
        hints" that miid_create reads (api.set_tuning_table) -- and return
        the number of rows.  A batched entry's shape is (nblk, 0, kmax)."""
        if device is None:
            device = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
        dts = {"float32": "f32", "float64": "f64"}
        rows = []
        for k, e in sorted(self.entries.items()):
            dev, routine, dt, shape = k.split("|")
            if dev != device or dt not in dts:
                continue
            dims = [int(v) for v in shape.split("x")] + [0, 0, 0]
            rows.append(f"{routine} {dts[dt]} {dims[0]} {dims[1]} {dims[2]} {int(e['nb'])} {int(e['hints']):#x}")
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            f.write("# routine dtype m n k nb hints\n")
            f.writelines(r + "\n" for r in rows)
        os.replace(tmp, path)
        return len(rows)

    def id_config(self, m: int, n: int, k: int, dtype, tune_if_missing: bool = False, **kw) -> Choice | None:
        """The stored choice for an ID of this shape; tuned (and stored) on a
        miss when tune_if_missing."""
        kk = key("id", dtype, (m, n, k))
        c = self.get(kk)
        if c is None and tune_if_missing:
            c = tune_id(m, n, k, dtype, **kw)
            self.put(kk, c)
        return c
