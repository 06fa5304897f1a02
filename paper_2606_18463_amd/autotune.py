"""Autotuner for the s-step fit.

For a fixed mini-batch size b the iterate does not depend on s (the s-step
block is an exact rewrite of s SGD steps), so the tuner only maximises SGD
updates per second over the launch choices the library exposes:

  * s (outer block size; s*b <= 4096),
  * execution mode: the fused persistent launch (variant 1: every workgroup
    runs the recurrence; variant 2: one workgroup runs it while the others
    build the next Gram matrix; variant 3: the chain and helper workgroups
    run it while the others build the next Gram matrix) or the
    stream-ordered kernel sequence,
  * the fused launch's grid size,
  * the Gram work unit (64-row units whose waves split K, or 128 x 128
    LDS-staged tiles) for s > 1.

Candidates a shape does not support (variant 3 needs b in {16, 32, 64, 128}
and s > 1) are skipped. Results persist in a JSON table keyed by (dtype, b,
n bucket, m bucket) with power-of-two buckets, so similar shapes reuse one
measurement.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import asdict, dataclass

import paper_2606_18463_amd as cg

S_GRID = (1, 2, 4, 8, 16, 32, 64)
# (exec_mode, fused_variant): 0 = fused persistent launch, 2 = stream-ordered
MODES = ((0, 1), (0, 2), (0, 3), (2, 0))


@dataclass
class Choice:
    s: int
    exec_mode: int
    variant: int
    grid_blocks: int
    updates_per_s: float
    gram_tile: int = 0    # 0 automatic, 64 or 128


def _bucket(v: int) -> int:
    return 1 << max(0, math.ceil(math.log2(max(1, v))))


def key(m: int, n: int, dtype: int, b: int) -> str:
    return f"{dtype}:{b}:{_bucket(n)}:{_bucket(m)}"


def _time_fit(X, y, b, s, eta, lam, seed, o, budget_s: float) -> float:
    """Seconds per outer iteration, measured with events on the current stream."""
    import torch
    x = torch.zeros(X.n, device="cuda")
    ws = cg.workspace(cg.casgd_workspace_size(X, b, s))
    cg.casgd_fit(X, y, x, eta, lam, b, s, seed, 0, 2, opts=o, ws=ws)   # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_outer = 4
    while True:
        e0.record()
        cg.casgd_fit(X, y, x, eta, lam, b, s, seed, 2, n_outer, opts=o, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        if t >= budget_s or n_outer >= 1 << 16:
            cg.casgd_check(ws)
            return t / n_outer
        n_outer *= max(2, min(16, int(budget_s / max(t, 1e-6))))


def tune(X, y, b: int, eta: float = 0.5, lam: float = 1e-5, seed: int = 0,
         s_grid=S_GRID, modes=MODES, grids=(0,), tiles=(64, 128), budget_s: float = 0.02,
         verbose: bool = False, results: list | None = None) -> Choice:
    """Measure every candidate on (X, y) and return the fastest (every
    measured candidate is appended to `results` when given). `tiles`: Gram
    unit kinds tried for s > 1."""
    best = None
    for s in s_grid:
        if s * b > 4096:
            continue
        for em, var in modes:
            for gb in (grids if em == 0 else (0,)):
                for gt in (tiles if s > 1 else (0,)):
                    o = cg.opts(exec_mode=em, fused_variant=var, grid_blocks=gb, gram_tile=gt)
                    what = f"s={s} mode={em}/{var} grid={gb} tile={gt}"
                    try:
                        t = _time_fit(X, y, b, s, eta, lam, seed, o, budget_s)
                    except cg.CasgdError as e:
                        if verbose:
                            print(f"{what}: {e}")
                        continue
                    ups = s / t   # SGD updates (mini-batches) per second
                    c = Choice(s, em, var, gb, ups, gt)
                    if results is not None:
                        results.append(c)
                    if verbose:
                        print(f"{what}: {ups:.0f} updates/s")
                    if best is None or ups > best.updates_per_s:
                        best = c
    if best is None:
        raise RuntimeError("no candidate ran")
    return best


class Table:
    """Persistent tuning table (JSON)."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.entries: dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, m: int, n: int, dtype: int, b: int) -> Choice | None:
        e = self.entries.get(key(m, n, dtype, b))
        return Choice(**e) if e else None

    def lookup_or_tune(self, X, y, b: int, **kw) -> Choice:
        c = self.get(X.m, X.n, X.dtype, b)
        if c is None:
            c = tune(X, y, b, **kw)
            self.entries[key(X.m, X.n, X.dtype, b)] = asdict(c)
            self.save()
        return c

    def save(self) -> None:
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.entries, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)

    def opts(self, c: Choice, **kw):
        return cg.opts(exec_mode=c.exec_mode, fused_variant=c.variant,
                       grid_blocks=c.grid_blocks, gram_tile=c.gram_tile, **kw)
