"""Autotuner for the plan parameters that set the factorization's tile
shapes and work split: the column-block width of the supernodal panels
(16, 32 or 64 columns per block, hence per tile and per diagonal triangle),
whether fundamental supernodes are amalgamated into wider panels, and the
split share (how finely long external-update tiles are cut into parts:
a part holds about max(64, level cost / share) units).

Two stages, each exhaustive: block width x amalgamation at the default
share, then the share for the winner.  Each candidate is analysed, bound
and its factorization timed on the GPU (HIP events on the current stream,
median of `reps` runs after one warm-up), for one value set or a whole
batch.  The fastest candidate wins; the full table is returned so that a
caller (or a learned model) can be measured against it.
"""
from __future__ import annotations

import numpy as np

from .binding import Analysis, Batch

SPACE = tuple({"block_width": b, "amalgamate": a} for b in (16, 32, 64) for a in (True, False))
SHARES = (6144, 24576)          # second stage; the default share is 12288


def label(t) -> str:
    """Short name of a table row: B<width>[a][/s<share>]."""
    s = f"B{t['block_width']}{'a' if t['amalgamate'] else ''}"
    return s + (f"/s{t['split_share']}" if t.get("split_share") else "")


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


def tune(n, Ap, Ai, values, ordering="nd", precision="f64", space=SPACE, reps: int = 3,
         shares=SHARES):
    """values: float64 CUDA tensor of shape (nnz,) or (m, nnz).  Returns
    (best candidate dict, table of every candidate with its factor time
    in ms and its analysis statistics)."""
    best, table = _search(n, Ap, Ai, values, ordering, precision, space, reps)
    if shares:
        best2, table2 = _search(n, Ap, Ai, values, ordering, precision,
                                tuple({**best, "split_share": s} for s in shares), reps)
        table += table2
        fastest = min((t for t in table if t["ok"]), key=lambda t: t["ms"])
        best = {k: fastest[k] for k in ("block_width", "amalgamate")}
        if fastest.get("split_share"):
            best["split_share"] = fastest["split_share"]
    return best, table


def _search(n, Ap, Ai, values, ordering, precision, space, reps):
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
