"""GPU: batches of value sets sharing one analysis, and their capture in a
HIP graph.

Every instance of a batch runs the same factor kernels in the same order as
a single factorization of its values, so its factor is the single one bit
for bit; the triangular sweeps add contributions with atomics in an order
that varies from run to run, so solutions agree to rounding (relative
1e-12 here, far above the ~1e-15 such reorderings cause and far below any
real error).  Graph replays are held to the same bound against eager runs
on the same inputs, checked after every replay with eager work between.
"""
import sys

import numpy as np
import pytest
import torch  # noqa: F401

import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def S():
    import paper_1705_06575_amd as S
    S.load_library()
    return S


def _instances(kind_shape, m, seed0):
    """m value sets on one grid pattern (weights drawn per instance)."""
    ws = [W.weighted_grid(kind_shape, len(kind_shape) == 2, 1e-2, 1e2, "shift1e-3",
                          np.random.default_rng(seed0 + k), f"g#{k}") for k in range(m)]
    for w in ws[1:]:
        assert np.array_equal(w.Ap, ws[0].Ap) and np.array_equal(w.Ai, ws[0].Ai)
    return ws


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_factor_equals_single_factors(S, orc, torch_cuda, precision):
    torch = torch_cuda
    ws = _instances((20, 20), 5, 300)
    w0 = ws[0]
    an = S.Analysis(w0.n, w0.Ap, w0.Ai, ordering="nd", precision=precision)
    Axb = torch.from_numpy(np.stack([w.Ax for w in ws])).cuda()
    bt = S.Batch(an, len(ws))
    bt.factor(Axb)
    assert (bt.status() == 0).all()
    B = torch.from_numpy(np.stack([W.dense_rhs(w0.n, np.random.default_rng(7 + k))
                                   for k in range(len(ws))])).cuda()
    Xb = B.clone()
    bt.solve_(Xb)
    perm = an.get("perm")
    for k, w in enumerate(ws):
        single = S.Analysis(w.n, w.Ap, w.Ai, ordering=perm, precision=precision)
        single.factor(torch.from_numpy(w.Ax).cuda())
        x1 = single.solve(B[k])
        d = float(torch.linalg.norm(x1 - Xb[k]) / torch.linalg.norm(x1))
        _say(f"case batch {precision} instance {k}: rel diff to single solve {d:.1e}")
        assert d <= 1e-12
        if k == 0 and precision == "f64":
            f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, perm)
            xr = orc.solve(w.n, perm, f["Lp"], f["Li"], f["Lx"], B[k].cpu().numpy())
            e = np.linalg.norm(Xb[k].cpu().numpy() - xr) / np.linalg.norm(xr)
            _say(f"case batch vs oracle: rel diff {e:.2e}")
            assert e <= 1e-10


def test_batch_refine_reaches_1e12(S, orc, torch_cuda):
    """FP32 batch factor + fixed FP64 refinement steps: every instance's
    backward error (library and oracle) <= 1e-12."""
    torch = torch_cuda
    ws = _instances((24, 24), 6, 500)
    w0 = ws[0]
    an = S.Analysis(w0.n, w0.Ap, w0.Ai, ordering="nd", precision="f32")
    Axb = torch.from_numpy(np.stack([w.Ax for w in ws])).cuda()
    B = torch.from_numpy(np.stack([W.dense_rhs(w0.n, np.random.default_rng(20 + k))
                                   for k in range(len(ws))])).cuda()
    X = torch.empty_like(B)
    bt = S.Batch(an, len(ws))
    bt.factor(Axb)
    bt.refine(Axb, B, X, steps=4)
    eta = bt.eta(Axb, B, X)
    _say(f"case batch refine: eta {eta}")
    assert (eta <= 1e-12).all()
    for k in (0, len(ws) - 1):
        e_orc = orc.eta_inf(w0.n, ws[k].Ap, ws[k].Ai, ws[k].Ax, X[k].cpu().numpy(), B[k].cpu().numpy())
        assert e_orc <= 1e-12 and abs(e_orc - eta[k]) <= 1e-3 * e_orc + 1e-15


def test_graph_capture_of_uneven_batches(S, torch_cuda):
    """Two patterns of different size, each a batch, factored and refined
    in one captured graph; replays (with new values copied in between and
    eager work on the stream) match the eager results."""
    torch = torch_cuda
    groups = []
    for shape, m, seed in (((16, 16), 4, 700), ((8, 8, 8), 3, 800)):
        ws = _instances(shape, m, seed)
        an = S.Analysis(ws[0].n, ws[0].Ap, ws[0].Ai, ordering="nd", precision="f32")
        Ax = torch.from_numpy(np.stack([w.Ax for w in ws])).cuda()
        B = torch.from_numpy(np.stack([W.dense_rhs(ws[0].n, np.random.default_rng(seed + k))
                                       for k in range(m)])).cuda()
        bt = S.Batch(an, m)
        groups.append(dict(an=an, bt=bt, Ax=Ax, Ax_in=Ax.clone(), B=B, X=torch.empty_like(B)))
    torch.cuda.synchronize()

    def run():
        for g in groups:
            g["bt"].factor(g["Ax_in"])
            g["bt"].refine(g["Ax_in"], g["B"], g["X"], steps=3)

    # warm-up outside the capture, then capture on a side stream
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run()
    torch.cuda.synchronize()
    for rep in range(3):
        # new values: a per-replay scaling (SPD kept), copied into the captured input
        for g in groups:
            g["Ax_in"].copy_(g["Ax"] * (1.0 + 0.25 * rep))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [g["X"].clone() for g in groups]
        run()                                   # eager reference on the same inputs
        torch.cuda.synchronize()
        for gi, g in enumerate(groups):
            d = float(torch.linalg.norm(got[gi] - g["X"]) / torch.linalg.norm(g["X"]))
            eta = g["bt"].eta(g["Ax_in"], g["B"], got[gi])
            _say(f"case graph replay {rep} group {gi}: rel diff to eager {d:.1e}, max eta {eta.max():.1e}")
            assert d <= 1e-12
            assert (eta <= 1e-12).all()
            assert (g["bt"].status() == 0).all()


def test_batch_refuses_stale_plan(S, torch_cuda):
    """After the analysis is rebound (here: new kernel variants, which
    rebuild its schedule) a batch bound before holds stale device pointers:
    its calls fail with SYM_ESTATE until it is bound again."""
    from paper_1705_06575_amd import SymError
    torch = torch_cuda
    ws = _instances((12, 12), 2, 500)
    w0 = ws[0]
    an = S.Analysis(w0.n, w0.Ap, w0.Ai, ordering="nd")
    Axb = torch.from_numpy(np.stack([w.Ax for w in ws])).cuda()
    bt = S.Batch(an, 2)
    bt.factor(Axb)
    assert (bt.status() == 0).all()
    an.set_variants(np.zeros(int(an.stat("ndsuper")), np.uint8))
    an.bind()
    with pytest.raises(SymError) as e:
        bt.factor(Axb)
    assert e.value.name == "SYM_ESTATE"
    bt2 = S.Batch(an, 2)
    bt2.factor(Axb)
    assert (bt2.status() == 0).all()
