"""Autotuner for the plan parameters that set the factorization's tile
shapes: the column-block width of the supernodal panels (16, 32 or 64
columns per block, hence per tile and per diagonal triangle) and whether
fundamental supernodes are amalgamated into wider panels.

Exhaustive over a small space: each candidate is analysed, bound and its
factorization timed on the GPU (HIP events on the current stream, median
of `reps` runs after one warm-up), for one value set or a whole batch.
The fastest candidate wins; the full table is returned so that a caller
(or a learned model) can be judged against it.
"""
from __future__ import annotations

import numpy as np

from .binding import Analysis, Batch

SPACE = tuple({"block_width": b, "amalgamate": a} for b in (16, 32, 64) for a in (True, False))


def _time_ms(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return float(np.median(out))


def tune(n, Ap, Ai, values, ordering="nd", precision="f64", space=SPACE, reps: int = 3):
    """values: float64 CUDA tensor of shape (nnz,) or (m, nnz).  Returns
    (best candidate dict, table of every candidate with its factor time
    in ms and its analysis statistics)."""
    table = []
    for cand in space:
        an = Analysis(n, Ap, Ai, ordering=ordering, precision=precision, **cand)
        an.bind(values.device)
        if values.dim() == 1:
            ms = _time_ms(lambda: an.factor(values), reps)
            ok = an.status() == 0
        else:
            bt = Batch(an, values.shape[0])
            ms = _time_ms(lambda: bt.factor(values), reps)
            ok = bool((bt.status() == 0).all())
            bt.close()
        table.append({**cand, "ms": ms, "ok": ok, "flops": an.stat("flops"),
                      "stored_lower": an.stat("stored_lower"), "nsuper": an.stat("ndsuper")})
        an.close()
    best = min((t for t in table if t["ok"]), key=lambda t: t["ms"])
    return {k: best[k] for k in space[0]}, table
