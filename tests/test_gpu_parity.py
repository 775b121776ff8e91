"""GPU parity: the HIP factor and solves, called through the C ABI, against
the CPU oracle on the same seeded inputs.

Tolerances (FP64, unit roundoff u = 1.1e-16):
  - factor, elementwise:  ||L_gpu - L_orc||_F / ||L_orc||_F <= 1e-13.  Both
    are backward stable factorizations that differ only in summation order;
    on these inputs (kappa(A) <= ~1e4 after diagonal scaling) the difference
    is a few hundred u at most.
  - invariants: ||L L^T - P A P^T||_F / ||A||_F <= 1e-13 and
    ||L y - P b|| / ||b|| <= 1e-13 (the bound stated for the method); for
    the transposed sweep L^T z = y, whose solution norm grows with
    kappa(L), the normwise backward error
    ||L^T z - y||_inf / (||L^T||_inf ||z||_inf + ||y||_inf) <= 1e-15.
  - solutions, elementwise: ||x_gpu - x_orc|| / ||x_orc|| <= 1e-13 on
    well-conditioned inputs; on the Laplacian grids the forward error of a
    solve scales with kappa(A), so the bound there is 1e3 * kappa * u,
    derived from the smallest eigenvalue of the Dirichlet Laplacian.
  - structure: reach sets and the zero pattern of a pruned solve exactly.
"""
import sys

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside the per-test time limit)

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


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _gpu_factor(S, torch, w, ordering, **kw):
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering=ordering, **kw)
    Ax = torch.from_numpy(w.Ax).cuda()
    an.factor(Ax)
    info = an.status()
    return an, info


def _check_against_oracle(S, orc, torch, w, block_width=64, tol_L=1e-13, tol_x=1e-13):
    _say(f"case {w.name} n={w.n} B={block_width}")
    an, info = _gpu_factor(S, torch, w, w.perm, block_width=block_width)
    assert info == 0
    f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    assert f["info"] == 0
    assert np.array_equal(an.get("Lp"), f["Lp"]) and np.array_equal(an.get("Li"), f["Li"])
    Lx = an.export_factor()
    eL = _rel(Lx, f["Lx"])
    res = orc.llt_residual(w.n, f["Cp"], f["Ci"], f["Cx"], f["Lp"], f["Li"], Lx)
    _say(f"  factor rel diff {eL:.3e}  llt residual {res:.3e}")
    assert eL <= tol_L
    assert res <= 1e-13
    # full solve, dense RHS
    rng = np.random.default_rng(11)
    b = W.dense_rhs(w.n, rng)
    x = an.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    x_ref = orc.solve(w.n, w.perm, f["Lp"], f["Li"], f["Lx"], b)
    ex = _rel(x, x_ref)
    _say(f"  solve rel diff {ex:.3e}")
    assert ex <= tol_x
    # forward sweep alone: residual ||L y - P b|| / ||b||
    y = an.solve_lower(torch.from_numpy(b).cuda()).cpu().numpy()
    ry = _rel(orc.lmul(w.n, f["Lp"], f["Li"], Lx, y), b[w.perm])
    ey = _rel(y, orc.fwd(w.n, f["Lp"], f["Li"], f["Lx"], b[w.perm]))
    _say(f"  forward residual {ry:.3e}  forward rel diff {ey:.3e}")
    assert ry <= 1e-13 and ey <= tol_x
    # backward sweep alone: normwise backward error of L^T z = y (the
    # residual relative to ||y|| alone grows with kappa(L) because ||z|| does)
    z = an.solve_upper_(torch.from_numpy(y.copy()).cuda()).cpu().numpy()
    rz = orc.ltmul(w.n, f["Lp"], f["Li"], Lx, z) - y
    lt_norm = orc.lmul(w.n, f["Lp"], f["Li"], np.abs(Lx), np.ones(w.n)).max(initial=0.0)
    den = lt_norm * np.abs(z).max(initial=0.0) + np.abs(y).max(initial=0.0)
    bz = np.abs(rz).max(initial=0.0) / (den if den > 0 else 1.0)
    _say(f"  backward sweep backward error {bz:.3e}  residual/||y|| {_rel(rz + y, y):.3e}")
    assert bz <= 1e-15
    return an, f, Lx


def test_small_random_matrices(S, orc, torch_cuda):
    rng = np.random.default_rng(23)
    for t in range(40):
        n = int(rng.integers(1, 120))
        dens = float(rng.choice([0.02, 0.08, 0.3, 0.9]))
        w = W.random_spd(n, dens, np.random.default_rng(4000 + t))
        _check_against_oracle(S, orc, torch_cuda, w)


@pytest.mark.parametrize("amalgamate", [False, True])
def test_amalgamation_modes(S, orc, torch_cuda, amalgamate):
    """The factor and solves with and without explicit-zero amalgamation."""
    torch = torch_cuda
    for w in [W.config2(14), W.knn_instance(5, nv=900)]:
        _say(f"case {w.name} amalgamate={amalgamate}")
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, amalgamate=amalgamate)
        an.factor(torch.from_numpy(w.Ax).cuda())
        assert an.status() == 0
        f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        Lx = an.export_factor()
        eL = _rel(Lx, f["Lx"])
        res = orc.llt_residual(w.n, f["Cp"], f["Ci"], f["Cx"], f["Lp"], f["Li"], Lx)
        _say(f"  factor rel diff {eL:.3e} llt residual {res:.3e}")
        assert res <= 1e-13 and eL <= 1e-10


@pytest.mark.parametrize("max_width", [7, 40])
def test_cut_supernodes(S, orc, torch_cuda, max_width):
    """Device supernodes cut into pieces of at most max_width columns (the
    rule that keeps the kernels' 16-bit widths and 32-bit panel offsets in
    range, forced here at small widths): factor and solve against the
    oracle as for the uncut plan."""
    torch = torch_cuda
    for w in [W.random_spd(200, 1.0, np.random.default_rng(6)), W.config2(14)]:
        _say(f"case {w.name} max_super_width={max_width}")
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, max_super_width=max_width)
        an.factor(torch.from_numpy(w.Ax).cuda())
        assert an.status() == 0
        f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        Lx = an.export_factor()
        eL = _rel(Lx, f["Lx"])
        res = orc.llt_residual(w.n, f["Cp"], f["Ci"], f["Cx"], f["Lp"], f["Li"], Lx)
        b = W.dense_rhs(w.n, np.random.default_rng(12))
        x = an.solve(torch.from_numpy(b).cuda()).cpu().numpy()
        xr = orc.solve(w.n, w.perm, f["Lp"], f["Li"], f["Lx"], b)
        ex = _rel(x, xr)
        _say(f"  factor rel diff {eL:.3e} llt residual {res:.3e} solve rel diff {ex:.3e}")
        assert res <= 1e-13 and eL <= 1e-10 and ex <= 1e-9


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16"])
def test_staged_external_updates(S, orc, torch_cuda, precision):
    """Every device supernode on the staged external-update path (variant
    3: each incidence's rows staged in LDS once per tile, in chunks of 16
    inner indices): the factor against the oracle as for the default
    variant, in FP64, FP32 and with bfloat16 update products."""
    torch = torch_cuda
    tol = {"f64": 1e-13, "f32": 1e-5, "bf16": None}[precision]
    for w in [W.random_spd(200, 1.0, np.random.default_rng(6)), W.config2(14),
              W.knn_instance(3, nv=900)]:
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, precision=precision)
        an.set_variants(np.full(int(an.stat("ndsuper")), 3, np.uint8))
        an.factor(torch.from_numpy(w.Ax).cuda())
        assert an.status() == 0
        f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        Lx = an.export_factor()
        eL = _rel(Lx, f["Lx"])
        res = orc.llt_residual(w.n, f["Cp"], f["Ci"], f["Cx"], f["Lp"], f["Li"], Lx)
        _say(f"case staged {precision} {w.name}: factor rel diff {eL:.3e} llt residual {res:.3e}")
        if tol is None:
            assert res <= 4.0 * 2.0 ** -8
        else:
            assert res <= (1e-13 if precision == "f64" else 1e-5)
            if not w.name.startswith("grid3d"):
                assert eL <= tol


def test_dense_multi_block_multi_tile(S, orc, torch_cuda):
    """Fully dense 200 x 200: one supernode cut into 4 blocks of <= 64
    columns with up to 4 row tiles each (exercises the off-diagonal tile
    solves and the dense descendant updates)."""
    w = W.random_spd(200, 1.0, np.random.default_rng(6))
    for B in (64, 32, 16):
        _check_against_oracle(S, orc, torch_cuda, w, block_width=B)


def test_config1_full(S, orc, torch_cuda):
    w = W.config1()
    # Dirichlet 5-point on 64 x 64: kappa = lambda_max / lambda_min
    lmin = 4 - 4 * np.cos(np.pi / 65)
    kappa = (4 + 4 * np.cos(np.pi / 65)) / lmin
    tol_x = 1e3 * kappa * 1.1e-16
    an, f, Lx = _check_against_oracle(S, orc, torch_cuda, w, tol_x=tol_x)
    torch = torch_cuda
    # sparse RHS with 8 nonzeros: reach set, zero pattern and values
    rng = np.random.default_rng(12)
    pinv = np.empty(w.n, np.int64)
    pinv[w.perm] = np.arange(w.n)
    for nb in (8, 1, 64):
        pos, val = W.sparse_rhs(w.n, nb, rng)
        r = an.rhs_analyze(pos)
        ref_reach = orc.reach(w.n, f["Lp"], f["Li"], np.sort(pinv[pos]).astype(np.int32))
        assert np.array_equal(r.reach(), ref_reach)
        y = an.solve_lower_sparse(r, torch.from_numpy(val).cuda()).cpu().numpy()
        b = np.zeros(w.n)
        b[pinv[pos]] = val
        y_ref = orc.fwd_pruned(w.n, f["Lp"], f["Li"], f["Lx"], ref_reach, b)
        outside = np.ones(w.n, bool)
        outside[ref_reach] = False
        assert (y[outside] == 0.0).all()
        e = _rel(y, y_ref)
        _say(f"  sparse rhs nb={nb} reach={ref_reach.size} rel diff {e:.3e}")
        assert e <= tol_x
        assert _rel(orc.lmul(w.n, f["Lp"], f["Li"], Lx, y), b) <= 1e-13
        # the full solve with the same sparse right-hand side (pruned forward
        # sweep, full backward sweep), original ordering, against the
        # oracle's dense solve of that b
        bo = np.zeros(w.n)
        bo[pos] = val
        x = an.solve_sparse(r, torch.from_numpy(val).cuda()).cpu().numpy()
        x_ref = orc.solve(w.n, w.perm, f["Lp"], f["Li"], f["Lx"], bo)
        ex = _rel(x, x_ref)
        _say(f"  full solve, sparse rhs nb={nb}: rel diff {ex:.3e}")
        assert ex <= tol_x


def test_indefinite_reports_first_pivot(S, orc, torch_cuda):
    rng = np.random.default_rng(31)
    for t in range(8):
        w = W.random_spd(int(rng.integers(20, 150)), 0.1, np.random.default_rng(700 + t))
        Ax = w.Ax.copy()
        col = int(rng.integers(0, w.n))
        Ax[w.Ap[col]] = -Ax[w.Ap[col]]
        w2 = W.Workload(w.name, w.n, w.Ap, w.Ai, Ax, w.perm)
        f = orc.factor(w.n, w.Ap, w.Ai, Ax, w.perm)
        assert f["info"] > 0
        an, info = _gpu_factor(S, torch_cuda, w2, w.perm)
        expect = 1 + int(w.perm[f["info"] - 1])
        _say(f"case indefinite {t}: oracle col {expect}, gpu {info}")
        assert info == expect


def test_factor_is_bitwise_deterministic(S, torch_cuda):
    w = W.config2(20)
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd")
    Ax = torch_cuda.from_numpy(w.Ax).cuda()
    an.factor(Ax)
    L1 = an.export_factor()
    an.factor(Ax)
    L2 = an.export_factor()
    assert np.array_equal(L1.view(np.uint64), L2.view(np.uint64))


@pytest.mark.parametrize("prec,B", [("f64", 64), ("f32", 64), ("bf16", 64), ("f64", 32)])
def test_chain_launch_matches_step_launches(S, orc, torch_cuda, prec, B):
    """The persistent per-level chain launch (tasks waiting for the tiles
    they read, device-coherent handoffs) gives the step launches' factor
    bit for bit, on a pattern with wide supernodes (several blocks); a
    batch's solves agree to rounding; the FP64 factor equals the oracle."""
    torch = torch_cuda
    w = W.config2(24)
    Ax = torch.from_numpy(w.Ax).cuda()
    out = {}
    for chain in (False, True):
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, precision=prec, block_width=B, chain_launch=chain)
        an.factor(Ax)
        assert an.status() == 0
        out[chain] = (an.export_factor(), int(an.stat("nphases")))
        X = np.stack([w.Ax, 2.0 * w.Ax, w.Ax + 1.0 * (w.Ai == np.repeat(np.arange(w.n), np.diff(w.Ap)))])
        bt = S.Batch(an, 3)
        bt.factor(torch.from_numpy(X).cuda())
        assert (bt.status() == 0).all()
        R = torch.from_numpy(np.random.default_rng(8).uniform(-1.0, 1.0, (3, w.n))).cuda()
        out[(chain, "batch")] = bt.solve_(R).cpu().numpy()
        bt.close()
    _say(f"case chain {prec} B{B}: launches {out[False][1]} -> {out[True][1]}")
    assert out[True][1] < out[False][1]
    assert np.array_equal(out[True][0], out[False][0])
    # the sweeps add with atomics (order not fixed), so the batch's solves
    # agree to rounding, not bit for bit
    xb, xs = out[(True, "batch")], out[(False, "batch")]
    assert np.linalg.norm(xb - xs) <= 1e-10 * np.linalg.norm(xs)
    if prec == "f64":
        f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        assert np.linalg.norm(out[True][0] - f["Lx"]) <= 1e-12 * np.linalg.norm(f["Lx"])


@pytest.mark.parametrize("prec,B", [("f64", 64), ("f32", 64), ("bf16", 64), ("f64", 32)])
def test_update_depth_same_factor(S, orc, torch_cuda, prec, B):
    """Grouping a supernode's internal updates (one product over up to 16
    source blocks per target tile) keeps each entry's accumulation sequence,
    so the factor is bit for bit that of one block at a time; the FP64
    factor equals the oracle."""
    torch = torch_cuda
    w = W.config2(24)
    Ax = torch.from_numpy(w.Ax).cuda()
    out = {}
    for depth in (1, 2, 4, 16):
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, precision=prec, block_width=B, update_depth=depth)
        an.factor(Ax)
        assert an.status() == 0
        out[depth] = an.export_factor()
        an.close()
    _say(f"case update depth {prec} B{B}: {len(out)} depths")
    for depth in (2, 4, 16):
        assert np.array_equal(out[depth].view(np.uint64), out[1].view(np.uint64))
    if prec == "f64":
        f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        assert np.linalg.norm(out[4] - f["Lx"]) <= 1e-12 * np.linalg.norm(f["Lx"])


def test_backward_walkers_match_standard_schedule(S, orc, torch_cuda):
    """The backward sweep with walkers (one value set: the widest
    supernodes' diagonal chains walked by one workgroup each) and the
    standard schedule (a batch of value sets x walkers > 128) give the same
    solution to rounding, and the oracle's."""
    torch = torch_cuda
    w = W.config2(24)
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm)
    nwalk = int(an.stat("walkers"))
    assert nwalk > 0
    Ax = torch.from_numpy(w.Ax).cuda()
    an.factor(Ax)
    b = W.dense_rhs(w.n, np.random.default_rng(12))
    x1 = an.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    m = 128 // nwalk + 1
    bt = S.Batch(an, m)
    bt.factor(Ax.repeat(m, 1).contiguous())
    xb = bt.solve_(torch.from_numpy(np.tile(b, (m, 1))).cuda()).cpu().numpy()
    bt.close()
    f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    x_ref = orc.solve(w.n, w.perm, f["Lp"], f["Li"], f["Lx"], b)
    d = np.linalg.norm(x1 - xb[m - 1]) / np.linalg.norm(xb[m - 1])
    e = np.linalg.norm(x1 - x_ref) / np.linalg.norm(x_ref)
    eta = orc.eta_inf(w.n, w.Ap, w.Ai, w.Ax, x1, b)
    _say(f"case walkers: {nwalk} walkers, batch of {m} on the standard schedule; rel diff {d:.1e}, "
         f"vs oracle {e:.1e}, eta {eta:.1e}")
    # same factor; the sweeps' atomic sums differ in order only
    assert d <= 1e-10 and e <= 1e-9 and eta <= 1e-14


@pytest.mark.parametrize("m", [12, 24])
def test_grid3d_scaled(S, orc, torch_cuda, m):
    w = W.config2(m)
    # weighted Laplacian + 1e-6 shift: kappa up to ~1e7 * m^2 scale; check
    # the factor elementwise and the solve by its residual only
    an, f, Lx = _check_against_oracle(S, orc, torch_cuda, w, tol_x=np.inf)
    torch = torch_cuda
    b = W.dense_rhs(w.n, np.random.default_rng(3))
    x = an.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    eta = orc.eta_inf(w.n, w.Ap, w.Ai, w.Ax, x, b)
    _say(f"  eta_inf {eta:.3e}")
    assert eta <= 1e-14


def test_own_ordering_solution_matches(S, orc, torch_cuda):
    """The solution of A x = b does not depend on the ordering: the GPU path
    with the library's own nested dissection against the oracle with the
    geometric one."""
    torch = torch_cuda
    for w in [W.config1(), W.knn_instance(2, nv=3000)]:
        an, info = _gpu_factor(S, torch, w, "nd")
        assert info == 0
        f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        b = W.dense_rhs(w.n, np.random.default_rng(5))
        x = an.solve(torch.from_numpy(b).cuda()).cpu().numpy()
        x_ref = orc.solve(w.n, w.perm, f["Lp"], f["Li"], f["Lx"], b)
        e = _rel(x, x_ref)
        _say(f"case own-ordering {w.name}: rel diff {e:.3e}")
        assert e <= 1e-11
        assert orc.eta_inf(w.n, w.Ap, w.Ai, w.Ax, x, b) <= 1e-15 * 20


def test_config2_full_size_invariants(S, orc, torch_cuda):
    """The benchmark workload (3-D 7-point, 64^3, library ordering):
    properties that hold at any size, computed by the oracle's products."""
    torch = torch_cuda
    w = W.config2()
    _say(f"case {w.name} full size")
    an, info = _gpu_factor(S, torch, w, "nd")
    assert info == 0
    p = an.get("perm").astype(np.int64)
    Cp, Ci, Cx = orc.permute(w.n, w.Ap, w.Ai, w.Ax, p)
    Lp, Li = an.get("Lp"), an.get("Li")
    Lx = an.export_factor()
    rng = np.random.default_rng(19)
    for k in range(4):
        v = rng.standard_normal(w.n)
        lhs = orc.lmul(w.n, Lp, Li, Lx, orc.ltmul(w.n, Lp, Li, Lx, v))
        rhs = orc.symv(w.n, Cp, Ci, Cx, v)
        e = _rel(lhs, rhs)
        _say(f"  Freivalds probe {k}: {e:.3e}")
        assert e <= 1e-13
    b = W.dense_rhs(w.n, rng)
    y = an.solve_lower(torch.from_numpy(b).cuda()).cpu().numpy()
    ry = _rel(orc.lmul(w.n, Lp, Li, Lx, y), b[p])
    _say(f"  forward residual {ry:.3e}")
    assert ry <= 1e-13
    x = an.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    eta = orc.eta_inf(w.n, w.Ap, w.Ai, w.Ax, x, b)
    _say(f"  eta_inf {eta:.3e}")
    assert eta <= 1e-14
    # sparse RHS, 1 % of n
    pos, val = W.sparse_rhs(w.n, w.n // 100, rng)
    r = an.rhs_analyze(pos)
    reach = r.reach()
    pinv = np.empty(w.n, np.int64)
    pinv[p] = np.arange(w.n)
    beta = np.sort(pinv[pos]).astype(np.int32)
    assert np.array_equal(reach, orc.reach(w.n, Lp, Li, beta))
    ys = an.solve_lower_sparse(r, torch.from_numpy(val).cuda()).cpu().numpy()
    bb = np.zeros(w.n)
    bb[beta] = val[np.argsort(pinv[pos])]
    outside = np.ones(w.n, bool)
    outside[reach] = False
    assert (ys[outside] == 0.0).all()
    rs = _rel(orc.lmul(w.n, Lp, Li, Lx, ys), bb)
    _say(f"  sparse forward residual {rs:.3e} reach {reach.size}/{w.n}")
    assert rs <= 1e-13
    # element by element against the oracle's pruned substitution over the
    # same reach with the same factor (summation order differs only)
    y_ref = orc.fwd_pruned(w.n, Lp, Li, Lx, reach, bb)
    es = _rel(ys, y_ref)
    _say(f"  sparse forward vs oracle's pruned substitution {es:.3e}")
    assert es <= 1e-13
    assert (y_ref[outside] == 0.0).all()
