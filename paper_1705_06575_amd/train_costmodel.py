"""Train the cost model the package ships (costmodel.DEFAULT_MODEL).

The training graphs are the k-NN family's training instances
(workloads.knn_split()["train"]: eleven seeded graphs of 21.9k to 200k
vertices, 3 dofs each, the library's nested-dissection ordering).  For
each, the external-update time of every device supernode is measured
under every kernel variant (costmodel.measure_variants, on the GPU); the
ensemble is then fit to those rows and its decision margin chosen by
leave-one-graph-out validation (costmodel.train).  The held-out instances
of the split are never measured here.

Run from the repository root on a machine with the GPU:

    python -m paper_1705_06575_amd.train_costmodel [--out FILE] [--data FILE]
    python -m paper_1705_06575_amd.train_costmodel --from-data FILE [--out FILE]

--data writes the raw measurements (features and times per graph) to an
.npz file; --from-data refits from such a file without measuring again.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def measure_training_set(ks, dev, say=_say):
    """[(features, T), ...] for k-NN instances ks (see costmodel.measure_variants)."""
    import torch

    import workloads as W
    from . import costmodel as cm
    from .binding import Analysis
    out = []
    for i, k in enumerate(ks):
        t0 = time.perf_counter()
        w = W.knn_instance(k)
        an = Analysis(w.n, w.Ap, w.Ai, ordering="nd")
        say(f"graph {i + 1}/{len(ks)}: instance {k}, n={w.n}, analysed in {time.perf_counter() - t0:.1f} s")
        Ax = torch.from_numpy(w.Ax).to(dev)
        T = cm.measure_variants(an, Ax, say=lambda s: say("  " + s))
        out.append((an.get("super_feat"), T))
        say(f"  summed external-update time per variant (ms): {np.round(T.sum(axis=0) / 1e3, 2).tolist()}")
        an.close()
        del Ax
        torch.cuda.empty_cache()
    return out


def main(argv=None):
    import torch

    import workloads as W
    from . import costmodel as cm
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=cm.DEFAULT_MODEL)
    ap.add_argument("--data", default=None, help="write the raw measurements here (.npz)")
    ap.add_argument("--from-data", default=None, help="refit from measurements written by --data")
    ap.add_argument("--epochs", type=int, default=400)
    a = ap.parse_args(argv)
    ks = W.knn_split()["train"]
    if a.from_data:
        z = np.load(a.from_data, allow_pickle=False)
        ks = z["instances"].tolist()
        measured = [(z[f"feat{i}"], z[f"T{i}"]) for i in range(len(ks))]
    else:
        measured = measure_training_set(ks, torch.device("cuda:0"))
        if a.data:
            np.savez(a.data, instances=np.asarray(ks),
                     **{f"feat{i}": f for i, (f, _) in enumerate(measured)},
                     **{f"T{i}": T for i, (_, T) in enumerate(measured)})
    t0 = time.perf_counter()
    model, min_work, hist, rows = cm.train(measured, epochs=a.epochs)
    _say(f"fit: {rows} rows, loss {hist[-1]:.4f}, margin {model.margin}, work floor {min_work:.3g} "
         f"flops, {time.perf_counter() - t0:.1f} s")
    for k, (f, T) in zip(ks, measured):
        r = cm.regret(T, model.choose(f))
        gain = r["default_us"] - r["best_us"]
        share = (r["default_us"] - r["chosen_us"]) / gain if gain > 0 else 0.0
        _say(f"  instance {k}: in-sample share of the exhaustive gain {share:.2f} "
             f"(default {r['default_us'] / 1e3:.1f} ms, chosen {r['chosen_us'] / 1e3:.1f} ms, "
             f"best {r['best_us'] / 1e3:.1f} ms summed)")
    model.save(a.out, instances=np.asarray(ks), loss=np.asarray(hist))
    _say(f"wrote {a.out}")


if __name__ == "__main__":
    main()
