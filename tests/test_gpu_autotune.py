"""GPU: the autotuner times every candidate, returns the fastest, and the
chosen plan factors correctly (against the oracle)."""
import sys

import numpy as np
import pytest
import torch  # noqa: F401

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_autotune_picks_fastest_and_is_correct(orc, torch_cuda):
    torch = torch_cuda
    import paper_1705_06575_amd as S
    from paper_1705_06575_amd import autotune
    n, Ap, Ai, X, perm = W.config4_batch("7pt24", 4)
    vals = torch.from_numpy(X).cuda()
    best, table = autotune.tune(n, Ap, Ai, vals, ordering=perm, precision="f64", reps=2)
    print("case autotune:", [(t["block_width"], t["amalgamate"], round(t["ms"], 3)) for t in table],
          "best", best, flush=True)
    sys.stdout.flush()
    assert len(table) == len(autotune.SPACE) + len(autotune.SHARES)
    assert all(t["ok"] for t in table)
    fastest = min(table, key=lambda t: t["ms"])
    want = {"block_width": fastest["block_width"], "amalgamate": fastest["amalgamate"]}
    if fastest.get("split_share"):
        want["split_share"] = fastest["split_share"]
    assert best == want
    # the second stage varied only the split share, around the first stage's winner
    first = min(table[:len(autotune.SPACE)], key=lambda t: t["ms"])
    for t in table[len(autotune.SPACE):]:
        assert (t["block_width"], t["amalgamate"]) == (first["block_width"], first["amalgamate"])
    # every candidate has the same method flop count (amalgamation adds stored zeros only)
    assert len({t["flops"] for t in table}) == 1
    an = S.Analysis(n, Ap, Ai, ordering=perm, precision="f64", **best)
    an.factor(vals[1].contiguous())
    f = orc.factor(n, Ap, Ai, X[1], perm)
    Lx = an.export_factor()
    e = np.linalg.norm(Lx - f["Lx"]) / np.linalg.norm(f["Lx"])
    assert e <= 1e-12
