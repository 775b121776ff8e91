#!/usr/bin/env python3
"""Benchmark of the numeric phase on one MI355X: FP64 supernodal Cholesky
followed by the triangular solves, on the 3-D 7-point weighted Laplacian of
a 64^3 grid (n = 262144; weights log-uniform in [0.1, 10]; diagonal = row
sum + 1e-6), ordered by the library's own nested dissection.

One step = one pass of the whole numeric path over the input already
resident in HBM: scatter A into the supernodal panels, factor P A P^T =
L L^T, a full solve A x = b with a dense right-hand side (permute, forward
sweep, backward sweep, permute back) and a reach-pruned forward solve with a
sparse right-hand side of 1% random nonzeros.

Prints ONE JSON line.  `value` is the step's FP64 arithmetic (sum_j |L_j|^2
for the factor plus 2 flops per stored entry of L per sweep) per second.
Extra fields give each part separately; `roofline` covers the dominant
kernel of the factor, timed with HIP events on the library's stream around
every launch of the last timed step's factorization (read after the timed
loop, so that no step waits for the host); `cpu_baseline` is the CPU oracle
timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 (matrix and vector)
HBM_PEAK_GBPS = 8000.0       # MI355X HBM3E


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def leading_sample(w, perm, Lp, Li, target_flops: float):
    """The benchmark matrix's leading principal submatrix C[:k, :k] of
    C = P A P^T (P: the benchmark's ordering): its Cholesky factor is
    L[:k, :k], so factoring it is exactly the first k columns' share of the
    benchmark's factorization (their rows below k left out).  k is the
    largest multiple of n/64 whose flops, sum over j < k of |L_j rows < k|^2,
    stay within target_flops.  Returns (k, flops, Ap, Ai, Ax) in the new
    numbering (identity ordering)."""
    import numpy as np
    n = w.n
    best = (0, 0.0)
    for q in range(1, 65):
        k = n * q // 64
        m = Li[:Lp[k]] < k
        cnt = np.add.reduceat(m.astype(np.int64), Lp[:k]) if k > 0 else np.zeros(0, np.int64)
        fl = float((cnt.astype(np.float64) ** 2).sum())
        if fl > target_flops:
            break
        best = (k, fl)
    k, fl = best
    pinv = np.empty(n, np.int64)
    pinv[perm] = np.arange(n)
    cols = np.repeat(np.arange(n), np.diff(w.Ap))
    a, b = pinv[w.Ai.astype(np.int64)], pinv[cols]
    keep = (a < k) & (b < k)
    hi, lo, val = np.maximum(a, b)[keep], np.minimum(a, b)[keep], w.Ax[keep]
    order = np.lexsort((hi, lo))
    Ap = np.zeros(k + 1, np.int64)
    np.add.at(Ap, lo + 1, 1)
    return k, fl, np.cumsum(Ap), hi[order].astype(np.int32), val[order]


def cpu_baseline(w, perm, Lp, Li, target_flops: float = 5e10):
    """The oracle (plain C, one thread) on a bounded sample of the benchmark
    workload itself: the leading principal submatrix of the 64^3 matrix in
    the benchmark's ordering (see leading_sample), about 10-30 s of CPU
    work."""
    import numpy as np
    import oracle
    k, fl, Ap, Ai, Ax = leading_sample(w, perm, Lp, Li, target_flops)
    t0 = time.perf_counter()
    f = oracle.factor(k, Ap, Ai, Ax, np.arange(k, dtype=np.int32))
    dt = time.perf_counter() - t0
    assert f["info"] == 0 and f["flops"] == fl
    return {"value": round(f["flops"] / dt / 1e9, 3), "unit": "GFLOP/s", "cores": 1,
            "kind": "oracle",
            "sample": f"column Cholesky of the leading {k} x {k} principal submatrix of the "
                      f"benchmark's permuted 64^3 matrix (its factor is the first {k} of "
                      f"{w.n} columns of L, rows below {k} left out; {fl:.3e} flops), {dt:.1f} s",
            "host_cpu": _host_cpu(), "host_threads": os.cpu_count()}


def attainable_factor_ms(an, w) -> float:
    """Sum over supernodes of max(flops / FP64 peak, compulsory bytes / HBM
    bandwidth): flops = sum of c_j^2 over its columns; bytes = its L
    entries and A entries (8 B each) and its row indices (4 B each)."""
    import numpy as np
    sptr = an.get("super").astype(np.int64)
    cc = an.get("colcount").astype(np.float64)
    pinv = np.empty(w.n, np.int64)
    pinv[an.get("perm").astype(np.int64)] = np.arange(w.n)
    cols = np.repeat(np.arange(w.n), np.diff(w.Ap))
    pc = np.minimum(pinv[w.Ai.astype(np.int64)], pinv[cols])
    a_per_col = np.bincount(pc, minlength=w.n).astype(np.float64)
    seg = sptr[:-1]
    flops = np.add.reduceat(cc * cc, seg)
    lent = np.add.reduceat(cc, seg)
    aent = np.add.reduceat(a_per_col, seg)
    rows = cc[seg]
    nbytes = 8.0 * lent + 8.0 * aent + 4.0 * rows
    t = np.maximum(flops / (FP64_PEAK_TFLOPS * 1e12), nbytes / (HBM_PEAK_GBPS * 1e9))
    return float(t.sum() * 1e3)


def cold_sweep_ms(torch, an, b, ys, reps: int = 5) -> float:
    """Forward sweep with L2 and the Infinity Cache evicted first (a 1 GiB
    device copy before each timed run); median."""
    import numpy as np
    src = torch.empty(1 << 27, dtype=torch.float64, device=b.device)
    dst = torch.empty_like(src)
    out = []
    for _ in range(reps):
        dst.copy_(src)
        e0, e1 = _events(torch)
        e0.record()
        an.solve_lower(b, out=ys)
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    del src, dst
    return float(np.median(out))


def small_case(dev, reps: int = 10):
    """The 64 x 64 2-D 5-point case (n = 4096): latency, not bandwidth, bounds
    it (L is 0.8 MB and stays in cache); medians in microseconds."""
    import numpy as np
    import torch

    import paper_1705_06575_amd as S
    import workloads as W
    w = W.config1()
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm)
    an.bind(dev)
    rng = np.random.default_rng(20260001)
    Ax = torch.from_numpy(w.Ax).to(dev)
    b = torch.from_numpy(W.dense_rhs(w.n, rng)).to(dev)
    pos, val = W.sparse_rhs(w.n, 8, rng)
    rp = an.rhs_analyze(pos).bind(dev)
    bv = torch.from_numpy(val).to(dev)
    x = torch.empty_like(b)
    ys = torch.empty_like(b)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            e0, e1 = _events(torch)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1) * 1e3)
        return round(float(np.median(out)), 1)

    res = {"workload": f"laplace2d_5pt_64x64 (n={w.n}, nnz(L)={int(an.stat('nnzL'))})",
           "factor_us": timed(lambda: an.factor(Ax)),
           "fwd_dense_us": timed(lambda: an.solve_lower(b, out=ys)),
           "full_solve_us": timed(lambda: (x.copy_(b), an.solve_(x))),
           "fwd_sparse_8_us": timed(lambda: an.solve_lower_sparse(rp, bv, out=ys)),
           "full_solve_sparse_8_us": timed(lambda: an.solve_sparse(rp, bv, out=x)),
           "note": "latency-bound (L cache-resident); no bandwidth fraction reported"}
    assert an.status() == 0
    return res


def mixed_ir(dev, m: int = 80, reps: int = 3):
    """Time to a normwise backward error <= 1e-12 on the mixed-precision
    workload (3-D 27-point weighted Laplacian on an m^3 grid, weights
    log-uniform in [1e-3, 1e3], diagonal = row sum * (1 + 1e-6), geometric
    nested dissection): FP64 factor + solve (+ refinement if needed) against
    FP32 factors (FP32 update products, or bfloat16 / IEEE-half update
    products with per-supernode scaling) + FP64 iterative refinement, all on
    this GPU."""
    import numpy as np
    import torch

    import paper_1705_06575_amd as S
    import workloads as W
    w = W.config3(m)
    Ax = torch.from_numpy(w.Ax).to(dev)
    b = torch.from_numpy(W.dense_rhs(w.n, np.random.default_rng(20260003))).to(dev)
    x = torch.empty_like(b)
    out = {"workload": f"grid3d_27pt_{m}^3 weighted Laplacian (n={w.n}), geometric ND",
           "tol": 1e-12}
    for prec, method in (("f64", "ir"), ("f32", "ir"), ("f32", "pcg"), ("bf16", "pcg"),
                         ("f16", "pcg")):
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, precision=prec)
        an.bind(dev)
        flops = an.stat("flops")
        an.factor(Ax)
        an.refine(Ax, b, tol=1e-12, maxit=200, out=x, method=method)      # warm-up
        torch.cuda.synchronize()
        times, tf = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            an.factor(Ax)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, iters, eta = an.refine(Ax, b, tol=1e-12, maxit=200, out=x, method=method)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            times.append((t2 - t0) * 1e3)
            tf.append((t1 - t0) * 1e3)
        ms = float(np.median(times))
        key = prec if prec == "f64" else f"{prec}_{method}"
        out[key] = {"ms_to_1e-12": round(ms, 2), "factor_ms": round(float(np.median(tf)), 2),
                    "refine": method, "refine_iters": iters, "eta_inf": eta,
                    "pivots_perturbed": an.pivots_perturbed(),
                    "gflops_fp64_equiv": round(flops / (ms * 1e-3) / 1e9, 1),
                    "factor_gflops": round(flops / (float(np.median(tf)) * 1e-3) / 1e9, 1)}
        out["factor_flops"] = flops
        del an
        torch.cuda.empty_cache()
    best = min(("f32_ir", "f32_pcg", "bf16_pcg", "f16_pcg"), key=lambda k: out[k]["ms_to_1e-12"])
    out["mixed_best"] = best
    out["speedup_mixed_vs_fp64"] = round(out["f64"]["ms_to_1e-12"] / out[best]["ms_to_1e-12"], 3)
    return out


# the factor kernels, the schedule they run (tasks, splits, items) and the
# ordering and defaults that shape it
FACTOR_SOURCES = [os.path.join(ROOT, "paper_1705_06575_amd", "csrc", f)
                  for f in ("factor.hip", "symbolic.cpp", "plan.hpp", "ordering.cpp", "capi.cpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_factor_grid3d_7pt_64.json")
FACTOR_KERNELS = ("k_external", "k_internal", "k_trsm")


def _source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for path in FACTOR_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def copy_probe(nbytes: int, reps: int = 3):
    """A plain device copy of known size: the calibration run for the HBM
    byte counters (each counter is scaled by what it reads for this copy)."""
    import torch
    n = nbytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "reps": reps}))


def _counter_rows(path: str, counter: str):
    """(kernel name, value) per dispatch of a rocprofv3 counter CSV."""
    import csv
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                out.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return out


def write_traffic(fetch_csv: str, write_csv: str, copy_fetch_csv: str, copy_write_csv: str,
                  copy_bytes: int, out_path: str = TRAFFIC_FILE):
    """HBM bytes per launch of each factor kernel from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled so that the calibration copy
    of copy_bytes reads copy_bytes fetched and copy_bytes written."""
    def copy_kib(path, counter):
        vals = [v for k, v in _counter_rows(path, counter) if "copyBuffer" in k]
        return max(vals)

    scale_f = copy_bytes / (copy_kib(copy_fetch_csv, "FETCH_SIZE") * 1024.0)
    scale_w = copy_bytes / (copy_kib(copy_write_csv, "WRITE_SIZE") * 1024.0)
    res = {"source_sha256": _source_digest(), "copy_bytes": copy_bytes,
           "scale_fetch": scale_f, "scale_write": scale_w, "kernels": {}}
    for kern in FACTOR_KERNELS:
        fv = [v for k, v in _counter_rows(fetch_csv, "FETCH_SIZE") if kern + "<double" in k]
        wv = [v for k, v in _counter_rows(write_csv, "WRITE_SIZE") if kern + "<double" in k]
        if not fv or not wv:
            continue
        res["kernels"][kern] = {
            "launches": len(fv),
            "fetch_bytes_per_launch": sum(fv) / len(fv) * 1024.0 * scale_f,
            "write_bytes_per_launch": sum(wv) / len(wv) * 1024.0 * scale_w}
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


MFMA_FILE = os.path.join(ROOT, "profiles", "mfma_busy_factor_grid3d_7pt_64.json")


def write_mfma_busy(sq_csv: str, out_path: str = MFMA_FILE):
    """Matrix-core busy share of each factor kernel from a rocprofv3 SQ
    counter run: SQ_VALU_MFMA_BUSY_CYCLES / (4 x SQ_BUSY_CU_CYCLES), summed
    over the kernel's FP64 dispatches."""
    res = {"source_sha256": _source_digest(), "kernels": {}}
    for kern in FACTOR_KERNELS:
        busy = sum(v for k, v in _counter_rows(sq_csv, "SQ_VALU_MFMA_BUSY_CYCLES") if kern + "<double" in k)
        cu = sum(v for k, v in _counter_rows(sq_csv, "SQ_BUSY_CU_CYCLES") if kern + "<double" in k)
        if cu > 0:
            res["kernels"][kern] = {"mfma_busy": busy / (4.0 * cu)}
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def stored_mfma_busy(kernel: str):
    """The stored matrix-core busy share of `kernel`, or None when there is
    none or the factor sources changed since it was measured."""
    try:
        with open(MFMA_FILE) as f:
            res = json.load(f)
    except (OSError, ValueError):
        return None
    if res.get("source_sha256") != _source_digest() or kernel not in res.get("kernels", {}):
        return None
    return round(res["kernels"][kernel]["mfma_busy"], 4)


def stored_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the stored counter runs, or
    None when there are none or the kernel source changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            res = json.load(f)
    except (OSError, ValueError):
        return None
    if res.get("source_sha256") != _source_digest() or kernel not in res.get("kernels", {}):
        return None
    k = res["kernels"][kernel]
    return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]


def batched(dev, steps: int = 4, reps: int = 3, tune_m: int = 4):
    """The batched workload: 512 value sets on the 2-D 9-point 128^2 pattern
    plus 64 each on the 3-D 7-point 24^3 and 40^3 patterns (per-instance
    weights log-uniform in [1e-2, 1e2], A = L_G(w) + 1e-3 I), FP32 factors
    + `steps` FP64 refinement steps for every instance, captured in one HIP
    graph and timed per replay.  The three patterns run as one: the
    block-diagonal union of eight 9-point grids, one 24^3 and one 40^3 grid,
    with 64 value sets, so every launch of the schedule covers all
    instances of all three patterns.  Block width, amalgamation and split
    share are picked by the autotuner (timed on tune_m value sets)."""
    import numpy as np
    import torch

    import paper_1705_06575_amd as S
    from paper_1705_06575_amd import autotune
    import workloads as W
    n, Ap, Ai, X, perm, offsets = W.config4_union(64, 8)
    m = X.shape[0]
    vals = torch.from_numpy(X).to(dev)
    best, table = autotune.tune(n, Ap, Ai, vals[:tune_m].contiguous(), ordering=perm,
                                precision="f32", reps=2)
    an = S.Analysis(n, Ap, Ai, ordering=perm, precision="f32", **best)
    an.bind(dev)
    bt = S.Batch(an, m)
    B = torch.from_numpy(np.random.default_rng(20261000).uniform(-1.0, 1.0, (m, n))).to(dev)
    Xs = torch.empty_like(B)
    flops = m * an.stat("flops")
    out = {"workload": "512 x grid2d_9pt_128^2 + 64 x grid3d_7pt_24^3 + 64 x grid3d_7pt_40^3 as 64 value "
                       "sets of their block-diagonal union (n=%d), FP32 factor + FP64 refinement, one graph" % n,
           "steps": steps, "value_sets": m, "n": n, "nnz_L": int(an.stat("nnzL")),
           "factor_launches": int(an.stat("nphases")) + 3, "tuned": best,
           "tune_ms": {autotune.label(t): round(t["ms"], 3) for t in table}}

    def run():
        bt.factor(vals)
        bt.refine(vals, B, Xs, steps)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run()
    graph.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = _events(torch)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    # the factor alone, eagerly, for the split
    tf = []
    for _ in range(reps):
        e0, e1 = _events(torch)
        e0.record()
        bt.factor(vals)
        e1.record()
        torch.cuda.synchronize()
        tf.append(e0.elapsed_time(e1))
    eta = bt.eta(vals, B, Xs)
    bad = int((bt.status() != 0).sum())
    out.update({"graph_ms": round(ms, 2), "factor_ms": round(float(np.median(tf)), 2),
                "factor_flops": flops, "gflops_fp64_equiv": round(flops / (ms * 1e-3) / 1e9, 1),
                "factor_gflops": round(flops / (float(np.median(tf)) * 1e-3) / 1e9, 1),
                "max_eta_inf": float(eta.max()), "failed_instances": bad})
    bt.close()
    return out


def costmodel(dev, rounds: int = 6):
    """The learned part on the k-NN family (50 seeded graphs of 20k to
    200k vertices; k = 13 union-symmetrised neighbours of uniform points
    in the unit cube, 3 dofs per vertex, random SPD 3x3 blocks): the
    shipped model, trained on eleven instances of the family, chooses the
    per-supernode kernel variants of the held-out benchmark instance.  Its
    end-to-end factor time is compared with the default variant's and with
    the exhaustive per-supernode best (from summed workgroup times under
    every variant), interleaved over `rounds` rounds; the noise is the
    relative difference between the default's odd- and even-round
    medians."""
    import numpy as np
    import torch

    import paper_1705_06575_amd as S
    from paper_1705_06575_amd import costmodel as cm
    import workloads as W
    model = cm.load()
    split = W.knn_split()
    k = split["bench"]
    w = W.knn_instance(k)
    Ax = torch.from_numpy(w.Ax).to(dev)
    t0 = time.perf_counter()
    runs = {name: S.Analysis(w.n, w.Ap, w.Ai, ordering="nd") for name in ("default", "mlp", "exhaustive")}
    analyze_s = (time.perf_counter() - t0) / 3
    nds = int(runs["default"].stat("ndsuper"))
    t0 = time.perf_counter()
    choice = model.choose(runs["default"].get("super_feat"))
    choose_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    T = cm.measure_variants(runs["exhaustive"], Ax)
    measure_s = time.perf_counter() - t0
    best = np.argmin(T, axis=1).astype(np.uint8)
    runs["mlp"].set_variants(choice)
    runs["exhaustive"].set_variants(best)
    for an in runs.values():
        an.factor(Ax)
    torch.cuda.synchronize()
    times = {name: [] for name in runs}
    for _ in range(rounds):
        for name, an in runs.items():
            e0, e1 = _events(torch)
            e0.record()
            an.factor(Ax)
            e1.record()
            torch.cuda.synchronize()
            times[name].append(e0.elapsed_time(e1))
    med = {name: float(np.median(v)) for name, v in times.items()}
    d = np.asarray(times["default"])
    r = cm.regret(T, choice)
    gain_x = med["default"] - med["exhaustive"]
    out = {"workload": f"k-NN family (50 seeded graphs, 20k-200k vertices, k=13, 3 dofs): held-out "
                       f"instance {k}, {W.knn_size(k)} vertices (n={w.n}); model trained on instances "
                       f"{split['train']}",
           "supernodes": nds, "factor_flops": runs["default"].stat("flops"),
           "margin": model.margin if np.isfinite(model.margin) else "none (validation kept the default)",
           "variants_chosen": np.bincount(choice, minlength=cm.NVAR).tolist(),
           "variants_exhaustive": np.bincount(best, minlength=cm.NVAR).tolist(),
           "factor_ms": {name: round(v, 3) for name, v in med.items()},
           "gain_vs_default": round(1.0 - med["mlp"] / med["default"], 4),
           "noise": round(float(abs(np.median(d[0::2]) - np.median(d[1::2])) / med["default"]), 4),
           "share_of_exhaustive_gain": round((med["default"] - med["mlp"]) / gain_x, 3) if gain_x > 0 else None,
           "summed_wg_ms": {"mlp": round(r["chosen_us"] / 1e3, 2), "default": round(r["default_us"] / 1e3, 2),
                            "exhaustive": round(r["best_us"] / 1e3, 2)},
           "analyze_s": round(analyze_s, 1), "choose_s": round(choose_s, 2),
           "exhaustive_measure_s": round(measure_s, 1)}
    for an in runs.values():
        an.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--m", type=int, default=64, help="grid side (64 = the benchmark workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP64 vs FP32+refinement comparison")
    ap.add_argument("--mixed-m", type=int, default=80, help="grid side of the mixed-precision workload")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched graph workload")
    ap.add_argument("--no-costmodel", action="store_true", help="skip the learned cost model")
    ap.add_argument("--no-small-case", action="store_true", help="skip the small latency-bound case")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device copy of BYTES (byte-counter calibration)")
    ap.add_argument("--write-mfma-busy", metavar="SQ_CSV",
                    help="only turn a rocprofv3 SQ counter run into the stored matrix-core busy "
                         "share of the factor kernels")
    ap.add_argument("--write-traffic", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                        "COPY_WRITE_CSV", "COPY_BYTES"),
                    help="only turn rocprofv3 FETCH_SIZE / WRITE_SIZE runs into the stored "
                         "per-launch HBM bytes of the factor kernels")
    args = ap.parse_args()
    if args.write_mfma_busy:
        write_mfma_busy(args.write_mfma_busy)
        return
    if args.write_traffic:
        a = args.write_traffic
        write_traffic(a[0], a[1], a[2], a[3], int(a[4]))
        return
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the path runs on a single MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1705_06575_amd as S
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = W.config2(args.m)
    t0 = time.perf_counter()
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd")
    analyze_s = time.perf_counter() - t0
    an.bind(dev)
    rng = np.random.default_rng(20260002)
    Ax = torch.from_numpy(w.Ax).to(dev)
    b = torch.from_numpy(W.dense_rhs(w.n, rng)).to(dev)
    pos, val = W.sparse_rhs(w.n, w.n // 100, rng)
    rp = an.rhs_analyze(pos).bind(dev)
    bv = torch.from_numpy(val).to(dev)
    x = torch.empty_like(b)
    ys = torch.empty_like(b)

    flops_factor = an.stat("flops")
    nnzL = an.stat("nnzL")
    perm_bench = an.get("perm")
    Lp_bench = an.get("Lp") if not args.no_cpu_baseline else None
    Li_bench = an.get("Li") if not args.no_cpu_baseline else None
    reach = rp.reach()
    colcount = an.get("colcount")
    nnzL_reach = float(colcount[reach].sum())
    flops_solve = 2.0 * 2.0 * nnzL            # forward + backward sweeps
    flops_sparse = 2.0 * nnzL_reach
    flops_step = flops_factor + flops_solve + flops_sparse

    def step():
        an.factor(Ax)
        x.copy_(b)
        an.solve_(x)
        an.solve_lower_sparse(rp, bv, out=ys)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    an.profile(True)                           # creates the events
    an.profile(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        if i == args.steps - 1:
            an.profile(True)                   # events around the last step's launches
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-launch event times of the last timed step's factorization (read
    # after the loop, so that no step waits for the host)
    prof_ms, prof_n, kflops = an.profile_read()
    an.profile(False)
    assert an.status() == 0
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    # parts, timed separately with events (median of the same step count)
    def timed(fn, reps):
        out = []
        for _ in range(reps):
            e0, e1 = _events(torch)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out))

    reps = max(3, args.steps)
    t_factor = timed(lambda: an.factor(Ax), reps)
    t_fwd = timed(lambda: an.solve_lower(b, out=ys), reps)
    t_solve = timed(lambda: (x.copy_(b), an.solve_(x)), reps)
    t_sparse = timed(lambda: an.solve_lower_sparse(rp, bv, out=ys), reps)
    t_fwd_cold = cold_sweep_ms(torch, an, b, ys)
    t_attain = attainable_factor_ms(an, w)

    # SpTRSV algorithmic bytes (one forward sweep): L's values, each touched
    # block's row indices, and 16 bytes per solved column (read + write of y)
    blocks = an.get("blocks")
    col2blk = np.repeat(np.arange(blocks.size - 1), np.diff(blocks))
    rows_per_block = colcount[blocks[:-1]]
    bytes_fwd = 8.0 * nnzL + 4.0 * float(rows_per_block.sum()) + 16.0 * w.n
    touched = np.unique(col2blk[reach])
    bytes_sparse = 8.0 * nnzL_reach + 4.0 * float(rows_per_block[touched].sum()) + 16.0 * reach.size

    # dominant kernel of the factor, from the live events of the last timed step
    dom = max((k for k in prof_ms if k != "scatter"), key=lambda k: prof_ms[k])
    dom_ms_per_launch = prof_ms[dom] / max(prof_n[dom], 1)
    dom_flops_per_launch = kflops[dom] / max(prof_n[dom], 1)
    achieved = dom_flops_per_launch / (dom_ms_per_launch * 1e-3) / 1e12

    out = {
        "metric": "supernodal Cholesky GFLOP/s, FP64 vs mixed+IR to 1e-12 bwd err; SpTRSV GB/s",
        "value": round(flops_step / (ms_per_step * 1e-3) / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"grid3d_7pt_{args.m}^3 weighted Laplacian (n={w.n}), "
                               f"library nested dissection; factor + dense full solve + "
                               f"1% sparse forward solve",
                   "n": w.n, "nnz_A_lower": w.nnz, "nnz_L": int(nnzL),
                   "factor_flops": flops_factor, "sparse_rhs_nnz": int(pos.size),
                   "reach": int(reach.size)},
        "factor_ms": round(t_factor, 3),
        "factor_gflops": round(flops_factor / (t_factor * 1e-3) / 1e9, 2),
        "factor_frac_fp64_peak": round(flops_factor / (t_factor * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
        "sptrsv_fwd_dense_ms": round(t_fwd, 4),
        "sptrsv_fwd_dense_gbps": round(bytes_fwd / (t_fwd * 1e-3) / 1e9, 2),
        "sptrsv_fwd_dense_frac_hbm": round(bytes_fwd / (t_fwd * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "factor_attainable_ms": round(t_attain, 3),
        "factor_frac_attainable": round(t_attain / t_factor, 4),
        "sptrsv_fwd_dense_cold_ms": round(t_fwd_cold, 4),
        "sptrsv_fwd_dense_cold_gbps": round(bytes_fwd / (t_fwd_cold * 1e-3) / 1e9, 2),
        "sptrsv_fwd_sparse_ms": round(t_sparse, 4),
        "sptrsv_fwd_sparse_gbps": round(bytes_sparse / (t_sparse * 1e-3) / 1e9, 2),
        "sptrsv_fwd_sparse_frac_hbm": round(bytes_sparse / (t_sparse * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "sptrsv_algorithmic_bytes": {"fwd_dense": bytes_fwd, "fwd_sparse": bytes_sparse},
        "full_solve_ms": round(t_solve, 4),
        "analyze_s": round(analyze_s, 3),
        "factor_kernels_ms_per_step": {k: round(v, 3) for k, v in prof_ms.items()},
        "factor_launches_per_step": dict(prof_n),
        "roofline": {"kernel": f"factor {dom} update (k_{dom})", "bound": "mfma",
                     "achieved": round(achieved, 4), "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 5),
                     "traffic": stored_traffic(f"k_{dom}"),
                     "mfma_busy": stored_mfma_busy(f"k_{dom}"),
                     "mfma_busy_note": "matrix-core busy cycles / (4 SIMDs x busy CU cycles), "
                                       "rocprofv3 SQ counters of the same kernel (profiles/); "
                                       "null once the factor sources changed since",
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated)",
                     "algorithmic_flops_per_launch": dom_flops_per_launch},
    }
    if not args.no_small_case:
        out["small_case"] = small_case(dev)
    if not args.no_mixed:
        del an, rp
        torch.cuda.empty_cache()
        out["mixed_ir"] = mixed_ir(dev, args.mixed_m)
    if not args.no_batched:
        torch.cuda.empty_cache()
        out["batched"] = batched(dev)
    if not args.no_costmodel:
        torch.cuda.empty_cache()
        out["costmodel"] = costmodel(dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, perm_bench, Lp_bench, Li_bench)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
