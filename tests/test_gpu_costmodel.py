"""GPU: the cost model's network kernels against the FP64 oracle, the
per-supernode kernel variants against the factor oracle, the training
pipeline, and the shipped model's choice on a held-out k-NN graph against
the default variant (end-to-end time, beyond measured noise) and against
exhaustive measurement (regret).

Tolerances: the network runs in FP32 (u = 6e-8); outputs and gradients of
this size (64-wide layers, 500 samples) agree with the FP64 oracle to a
few hundred u in norm, so 1e-4 relative is the bound.  Factors under any
variant equal the oracle to the FP64 factor bound of the parity tests.
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


@pytest.mark.parametrize("n", [37, 500])
def test_network_forward_and_gradient_match_oracle(torch_cuda, n):
    torch = torch_cuda
    from oracle import mlp as omlp
    from paper_1705_06575_amd import costmodel as cm
    from paper_1705_06575_amd.binding import _dev_ptr, _stream, load_library
    L = load_library()
    rng = np.random.default_rng(11)
    D = cm.D_IN
    p = rng.normal(0.0, 0.2, omlp.param_count(D)).astype(np.float32)
    X = rng.normal(0.0, 1.0, (n, D)).astype(np.float32)
    t = rng.normal(0.0, 1.0, n).astype(np.float32)
    pd, Xd, td = (torch.from_numpy(a).cuda() for a in (p, X, t))
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    assert L.sym_mlp_forward(_dev_ptr(pd, "torch.float32"), _dev_ptr(Xd, "torch.float32"), n, D,
                             _dev_ptr(y, "torch.float32"), _stream()) == 0
    g = torch.empty_like(pd)
    from paper_1705_06575_amd.binding import mlp_work_size
    work = torch.empty(mlp_work_size(n, D), dtype=torch.float32, device="cuda")
    assert L.sym_mlp_backward(_dev_ptr(pd, "torch.float32"), _dev_ptr(Xd, "torch.float32"),
                              _dev_ptr(td, "torch.float32"), n, D, _dev_ptr(g, "torch.float32"),
                              _dev_ptr(work, "torch.float32"), _stream()) == 0
    y_ref = omlp.forward(p.astype(np.float64), X.astype(np.float64), D)
    g_ref = omlp.grad(p.astype(np.float64), X.astype(np.float64), t.astype(np.float64), D)
    ey = np.linalg.norm(y.cpu().numpy() - y_ref) / np.linalg.norm(y_ref)
    eg = np.linalg.norm(g.cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
    _say(f"case mlp n={n}: forward rel err {ey:.1e}, gradient rel err {eg:.1e}")
    assert ey <= 1e-4 and eg <= 1e-4
    # reproducible: a second backward gives the same bits
    g2 = torch.empty_like(pd)
    L.sym_mlp_backward(_dev_ptr(pd, "torch.float32"), _dev_ptr(Xd, "torch.float32"),
                       _dev_ptr(td, "torch.float32"), n, D, _dev_ptr(g2, "torch.float32"),
                       _dev_ptr(work, "torch.float32"), _stream())
    assert torch.equal(g, g2)


def test_training_fits_a_smooth_function(torch_cuda):
    from paper_1705_06575_amd import costmodel as cm
    rng = np.random.default_rng(3)
    X = rng.normal(0.0, 1.0, (2000, cm.D_IN))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] + 0.1 * X[:, 3]
    model = cm.CostModel(seed=1)
    hist = model.fit(X, t, epochs=300, lr=3e-3)
    _say(f"case mlp training loss {hist}")
    assert hist[-1] < 0.1 * np.var(t)


def test_every_variant_factors_correctly(orc, torch_cuda):
    torch = torch_cuda
    import paper_1705_06575_amd as S
    w = W.knn_instance(2, nv=900)
    f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm)
    nds = int(an.stat("ndsuper"))
    rng = np.random.default_rng(5)
    Ax = torch.from_numpy(w.Ax).cuda()
    for name, var in (("all 0", np.zeros(nds)), ("all 1", np.ones(nds)), ("all 2", np.full(nds, 2)),
                      ("all 3", np.full(nds, 3)), ("mixed", rng.integers(0, 4, nds))):
        an.set_variants(var.astype(np.uint8))
        assert np.array_equal(an.get("variant"), var.astype(np.uint8))
        an.factor(Ax)
        assert an.status() == 0
        Lx = an.export_factor()
        e = np.linalg.norm(Lx - f["Lx"]) / np.linalg.norm(f["Lx"])
        _say(f"case variants {name}: rel diff {e:.1e}")
        assert e <= 1e-13


def test_training_pipeline_round_trip(torch_cuda, tmp_path):
    """Measure two small k-NN patterns, fit, save and load: the loaded
    model predicts the same bits and makes the same choices."""
    torch = torch_cuda
    import paper_1705_06575_amd as S
    from paper_1705_06575_amd import costmodel as cm
    measured = []
    for k in (10, 11):
        w = W.knn_instance(k, nv=4000)
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd")
        T = cm.measure_variants(an, torch.from_numpy(w.Ax).cuda())
        assert T.shape == (int(an.stat("ndsuper")), cm.NVAR) and (T >= 0).all()
        measured.append((an.get("super_feat"), T))
    model, min_work, hist, rows = cm.train(measured, min_us=10.0, epochs=100)
    assert rows > 0 and np.isfinite(hist[-1])
    path = str(tmp_path / "cm.npz")
    model.save(path)
    back = cm.load(path)
    f = measured[0][0]
    X = cm.encode(f, np.zeros(len(f) // cm.NFEAT, dtype=np.int64))
    assert np.array_equal(model.predict(X), back.predict(X))
    assert back.margin == model.margin and back.min_work == min_work
    assert np.array_equal(model.choose(f), back.choose(f))


def _factor_times(torch, runs, Ax, rounds):
    """Interleaved end-to-end factor times (ms) of several bound analyses:
    one run of each per round, after one warm-up."""
    for an in runs.values():
        an.factor(Ax)
    torch.cuda.synchronize()
    out = {k: [] for k in runs}
    for _ in range(rounds):
        for k, an in runs.items():
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            an.factor(Ax)
            e1.record()
            torch.cuda.synchronize()
            out[k].append(e0.elapsed_time(e1))
    return {k: np.asarray(v) for k, v in out.items()}


def test_shipped_model_gains_on_held_out_graph(torch_cuda):
    """The shipped model (trained on the k-NN family's training instances)
    chooses the variants of the held-out test instance.  Its end-to-end
    factor time must beat the default variant's by more than the run-to-run
    noise measured in the same run: the relative difference between the
    medians of the default's odd and even rounds.  Regret against the
    exhaustive per-supernode choice (from summed workgroup times) is
    reported; every choice factors to the same result."""
    torch = torch_cuda
    import paper_1705_06575_amd as S
    from paper_1705_06575_amd import costmodel as cm
    model = cm.load()
    k = W.knn_split()["test"]
    assert k not in W.knn_split()["train"]
    w = W.knn_instance(k)
    Ax = torch.from_numpy(w.Ax).cuda()
    runs = {name: S.Analysis(w.n, w.Ap, w.Ai, ordering="nd") for name in ("default", "mlp", "exhaustive")}
    feat = runs["default"].get("super_feat")
    choice = model.choose(feat)
    T = cm.measure_variants(runs["exhaustive"], Ax)
    best = np.argmin(T, axis=1).astype(np.uint8)
    runs["mlp"].set_variants(choice)
    runs["exhaustive"].set_variants(best)
    t = _factor_times(torch, runs, Ax, rounds=10)
    med = {name: float(np.median(v)) for name, v in t.items()}
    d = t["default"]
    noise = abs(np.median(d[0::2]) - np.median(d[1::2])) / med["default"]
    gain = 1.0 - med["mlp"] / med["default"]
    gain_x = 1.0 - med["exhaustive"] / med["default"]
    r = cm.regret(T, choice)
    _say(f"case held-out instance {k} (n={w.n}): factor ms default {med['default']:.3f}, "
         f"mlp {med['mlp']:.3f}, exhaustive {med['exhaustive']:.3f}; gain {gain:.4f} "
         f"(exhaustive {gain_x:.4f}), noise {noise:.4f}; variants {np.bincount(choice, minlength=cm.NVAR)}; "
         f"summed regret {r['regret_us'] / 1e3:.1f} ms vs default's {r['default_regret_us'] / 1e3:.1f} ms")
    ref = None
    for name, an in runs.items():
        assert an.status() == 0
        Lx = an.export_factor()
        if ref is None:
            ref = Lx
        assert np.linalg.norm(Lx - ref) <= 1e-13 * np.linalg.norm(ref), name
    assert gain > noise and gain > 0.0
