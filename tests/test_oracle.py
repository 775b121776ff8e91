"""Pins for the CPU oracle: brute force, library routines, closed forms and
invariants that do not depend on the oracle itself.  CPU only."""
import numpy as np
import pytest
from scipy.linalg import lapack

import workloads as W


def _perm_dense(w):
    A = W.to_dense(w)
    p = w.perm.astype(np.int64)
    return A[np.ix_(p, p)]


def _pattern_from_dense_chol(C):
    """L's structural pattern as computed by LAPACK on generic values:
    with random values there is no exact cancellation."""
    L, info = lapack.dpotrf(C, lower=1)
    assert info == 0
    L = np.tril(L)
    n = C.shape[0]
    Lp = [0]
    Li = []
    for j in range(n):
        rows = np.nonzero(L[j:, j])[0] + j
        Li.extend(rows.tolist())
        Lp.append(len(Li))
    return np.array(Lp, np.int64), np.array(Li, np.int32), L


def _random_cases(count=120, nmax=48):
    rng = np.random.default_rng(7)
    cases = []
    for t in range(count):
        n = int(rng.integers(1, nmax + 1))
        dens = float(rng.choice([0.02, 0.05, 0.1, 0.2, 0.4]))
        cases.append(W.random_spd(n, dens, np.random.default_rng(1000 + t)))
    return cases


# ---------------------------------------------------------------- symbolic


def test_bool_elim_matches_eq1_random(orc):
    for w in _random_cases():
        Cp, Ci, _ = orc.permute(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        Lp1, Li1 = orc.bool_elim(w.n, Cp, Ci)
        Lp2, Li2, par = orc.symbolic_eq1(w.n, Cp, Ci)
        assert np.array_equal(Lp1, Lp2) and np.array_equal(Li1, Li2)
        assert np.array_equal(par, orc.etree_from_pattern(w.n, Lp1, Li1))


def test_pattern_matches_lapack_fill(orc):
    """Fill pattern and elimination tree against the nonzeros of LAPACK's
    dense Cholesky factor on generic values."""
    for w in _random_cases(60, 40):
        C = _perm_dense(w)
        Lp_ref, Li_ref, _ = _pattern_from_dense_chol(C)
        Cp, Ci, _ = orc.permute(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        Lp, Li, par = orc.symbolic_eq1(w.n, Cp, Ci)
        assert np.array_equal(Lp, Lp_ref) and np.array_equal(Li, Li_ref)
        for j in range(w.n):
            below = Li_ref[Lp_ref[j]:Lp_ref[j + 1]]
            below = below[below > j]
            assert par[j] == (below.min() if below.size else -1)


def test_pattern_config1_bool_elim(orc):
    w = W.config1()
    Cp, Ci, _ = orc.permute(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    Lp1, Li1 = orc.bool_elim(w.n, Cp, Ci)
    Lp2, Li2, par = orc.symbolic_eq1(w.n, Cp, Ci)
    assert np.array_equal(Lp1, Lp2) and np.array_equal(Li1, Li2)
    # structural invariants of a filled graph
    for j in range(w.n):
        col = Li2[Lp2[j]:Lp2[j + 1]]
        assert col[0] == j
        if par[j] >= 0:
            assert par[j] > j
            pc = set(Li2[Lp2[par[j]]:Lp2[par[j] + 1]].tolist())
            assert set(col[1:].tolist()) <= pc


def _sym_from_lower_edges(n, edges, diag=4.0):
    rows = list(range(n)) + [max(e) for e in edges]
    cols = list(range(n)) + [min(e) for e in edges]
    vals = [diag] * n + [-1.0] * len(edges)
    order = np.lexsort((rows, cols))
    rows = np.array(rows)[order]
    cols = np.array(cols)[order]
    vals = np.array(vals)[order]
    Ap = np.zeros(n + 1, np.int64)
    np.add.at(Ap, cols + 1, 1)
    return np.cumsum(Ap), rows.astype(np.int32), vals


@pytest.mark.parametrize("kind", ["diag", "tridiag", "dense", "arrow_down", "arrow_up", "blocks"])
def test_structured_special_cases(orc, kind):
    n = 9
    if kind == "diag":
        edges = []
    elif kind == "tridiag":
        edges = [(j + 1, j) for j in range(n - 1)]
    elif kind == "dense":
        edges = [(i, j) for j in range(n) for i in range(j + 1, n)]
    elif kind == "arrow_down":       # dense last row
        edges = [(n - 1, j) for j in range(n - 1)]
    elif kind == "arrow_up":         # dense first column -> complete fill
        edges = [(i, 0) for i in range(1, n)]
    else:                            # two disconnected dense blocks
        edges = [(i, j) for j in range(4) for i in range(j + 1, 4)] + \
                [(i, j) for j in range(4, n) for i in range(j + 1, n)]
    Ap, Ai, Ax = _sym_from_lower_edges(n, edges, diag=float(n + 1))
    Lp, Li, par = orc.symbolic_eq1(n, Ap, Ai)
    cc = orc.colcounts(Lp)
    sp = orc.supernodes(n, par, cc)
    if kind == "diag":
        assert (par == -1).all() and (cc == 1).all() and len(sp) - 1 == n
    elif kind == "tridiag":
        assert np.array_equal(par, np.r_[np.arange(1, n), -1])
        assert len(sp) - 1 == n - 1            # only the last two columns merge
    elif kind in ("dense", "arrow_up"):
        assert np.array_equal(cc, np.arange(n, 0, -1)) and len(sp) - 1 == 1
    elif kind == "arrow_down":
        assert np.array_equal(par, np.r_[np.full(n - 1, n - 1), -1])
        # column n-1 has n-1 children, so no column merges into it
        assert (cc[:-1] == 2).all() and len(sp) - 1 == n
    else:
        assert (par == np.r_[1, 2, 3, -1, 5, 6, 7, 8, -1]).all()   # a forest
        assert len(sp) - 1 == 2
    # a dense solve recovers the same pattern
    Lp_ref, Li_ref, _ = _pattern_from_dense_chol(W.to_dense(W.Workload("", n, Ap, Ai, Ax, np.arange(n))))
    assert np.array_equal(Lp, Lp_ref) and np.array_equal(Li, Li_ref)


def test_supernodes_have_nested_patterns(orc):
    """Within a fundamental supernode, column j's pattern is column j-1's
    minus its diagonal, and the supernode's columns form a chain."""
    for w in _random_cases(60, 48) + [W.config1()]:
        Cp, Ci, _ = orc.permute(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        Lp, Li, par = orc.symbolic_eq1(w.n, Cp, Ci)
        sp = orc.supernodes(w.n, par, orc.colcounts(Lp))
        assert sp[0] == 0 and sp[-1] == w.n and (np.diff(sp) > 0).all()
        for s in range(len(sp) - 1):
            for j in range(sp[s] + 1, sp[s + 1]):
                prev = Li[Lp[j - 1] + 1:Lp[j]]
                cur = Li[Lp[j]:Lp[j + 1]]
                assert np.array_equal(prev, cur)
                assert par[j - 1] == j


def test_reach_closed_form_and_dense_solve(orc):
    """Reach_L(beta) equals the union of elimination-tree paths from beta to
    the roots, and the set of nonzeros of a solve with random values."""
    rng = np.random.default_rng(3)
    for w in _random_cases(50, 40):
        Cp, Ci, Cx = orc.permute(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        Lp, Li, par = orc.symbolic_eq1(w.n, Cp, Ci)
        for nb in (1, 2, 5):
            beta = np.sort(rng.choice(w.n, size=min(nb, w.n), replace=False)).astype(np.int32)
            r = orc.reach(w.n, Lp, Li, beta)
            path = set()
            for b in beta:
                j = int(b)
                while j >= 0 and j not in path:
                    path.add(j)
                    j = int(par[j])
            assert set(r.tolist()) == path
            # numeric: L with random values, b nonzero exactly on beta
            Lx = rng.uniform(0.5, 1.5, Lp[-1])
            bvec = np.zeros(w.n)
            bvec[beta] = rng.uniform(1, 2, beta.size)
            x = orc.fwd(w.n, Lp, Li, Lx, bvec)
            assert set(np.nonzero(x)[0].tolist()) == path


# ---------------------------------------------------------------- numeric


def test_chol_matches_lapack(orc):
    for w in _random_cases(80, 48):
        C = _perm_dense(w)
        Lref, info = lapack.dpotrf(C, lower=1)
        assert info == 0
        Lref = np.tril(Lref)
        f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        assert f["info"] == 0
        L = np.zeros((w.n, w.n))
        for j in range(w.n):
            L[f["Li"][f["Lp"][j]:f["Lp"][j + 1]], j] = f["Lx"][f["Lp"][j]:f["Lp"][j + 1]]
        assert np.linalg.norm(L - Lref) <= 1e-13 * np.linalg.norm(Lref)
        cc = orc.colcounts(f["Lp"])
        assert f["flops"] == float((cc.astype(np.float64) ** 2).sum())


def test_chol_closed_forms(orc):
    # diagonal: L = sqrt(A)
    n = 17
    d = np.linspace(0.5, 9.0, n)
    Ap = np.arange(n + 1, dtype=np.int64)
    Ai = np.arange(n, dtype=np.int32)
    Lp, Li, _ = orc.symbolic_eq1(n, Ap, Ai)
    Lx, info, _ = orc.chol_column(n, Ap, Ai, d, Lp, Li)
    assert info == 0 and np.array_equal(Lx, np.sqrt(d))
    # 1-D Laplacian tridiag(-1, 2, -1) in natural order
    n = 200
    Ap, Ai, Ax = _sym_from_lower_edges(n, [(j + 1, j) for j in range(n - 1)], diag=2.0)
    Lp, Li, _ = orc.symbolic_eq1(n, Ap, Ai)
    Lx, info, _ = orc.chol_column(n, Ap, Ai, Ax, Lp, Li)
    assert info == 0
    j = np.arange(n)
    diag = Lx[Lp[:-1]]
    sub = Lx[Lp[:-2] + 1]
    np.testing.assert_allclose(diag, np.sqrt((j + 2) / (j + 1)), rtol=1e-14)
    np.testing.assert_allclose(sub, -np.sqrt((j[:-1] + 1) / (j[:-1] + 2)), rtol=1e-14)


def test_chol_residual_invariant(orc):
    for w in _random_cases(30, 48) + [W.config1()]:
        f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        r = orc.llt_residual(w.n, f["Cp"], f["Ci"], f["Cx"], f["Lp"], f["Li"], f["Lx"])
        assert r <= 1e-13


def test_llt_residual_detects_error(orc):
    """The residual invariant is not vacuous: a perturbed factor fails it."""
    w = W.random_spd(30, 0.2, np.random.default_rng(11))
    f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    Lx = f["Lx"].copy()
    Lx[len(Lx) // 2] *= 1.0 + 1e-9
    r = orc.llt_residual(w.n, f["Cp"], f["Ci"], f["Cx"], f["Lp"], f["Li"], Lx)
    assert r > 1e-12


def test_info_matches_lapack(orc):
    """A forced-indefinite matrix stops at the same column as LAPACK."""
    rng = np.random.default_rng(5)
    for t in range(40):
        w = W.random_spd(int(rng.integers(3, 40)), 0.15, np.random.default_rng(500 + t))
        Ax = w.Ax.copy()
        col = int(rng.integers(0, w.n))
        dpos = w.Ap[col]                         # diagonal is first (rows sorted, i >= j)
        assert w.Ai[dpos] == col
        Ax[dpos] = -Ax[dpos]
        w2 = W.Workload("", w.n, w.Ap, w.Ai, Ax, w.perm)
        C = _perm_dense(w2)
        _, info_ref = lapack.dpotrf(C, lower=1)
        f = orc.factor(w.n, w.Ap, w.Ai, Ax, w.perm)
        assert info_ref > 0 and f["info"] == info_ref


def test_solve_laplace2d_eigenvectors(orc):
    """Dirichlet 5-point Laplacian on 64 x 64: A v_kl = lambda_kl v_kl with
    v_kl(i, j) = sin(k pi (i+1)/65) sin(l pi (j+1)/65) and
    lambda_kl = 4 - 2 cos(k pi / 65) - 2 cos(l pi / 65)."""
    w = W.config1()
    f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    i = np.arange(64)[:, None]
    j = np.arange(64)[None, :]
    for k, l in [(1, 1), (3, 7), (20, 2), (64 - 1, 64 - 1)]:
        v = (np.sin(k * np.pi * (i + 1) / 65) * np.sin(l * np.pi * (j + 1) / 65)).ravel()
        lam = 4 - 2 * np.cos(k * np.pi / 65) - 2 * np.cos(l * np.pi / 65)
        x = orc.solve(w.n, w.perm, f["Lp"], f["Li"], f["Lx"], v)
        # forward error bounded by kappa * u with a modest constant (kappa ~ 1.7e3)
        assert np.linalg.norm(x - v / lam) <= 1e-11 * np.linalg.norm(v / lam)


def test_solve_round_trip_and_residual(orc):
    rng = np.random.default_rng(9)
    for w in _random_cases(20, 48) + [W.config1()]:
        f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        xt = np.where(rng.random(w.n) < 0.3, rng.uniform(-1, 1, w.n), 0.0)
        b = orc.lmul(w.n, f["Lp"], f["Li"], f["Lx"], xt)
        x = orc.fwd(w.n, f["Lp"], f["Li"], f["Lx"], b)
        assert np.linalg.norm(x - xt) <= 1e-13 * max(np.linalg.norm(xt), 1e-300)
        bt = orc.ltmul(w.n, f["Lp"], f["Li"], f["Lx"], xt)
        x = orc.bwd(w.n, f["Lp"], f["Li"], f["Lx"], bt)
        assert np.linalg.norm(x - xt) <= 1e-13 * max(np.linalg.norm(xt), 1e-300)
        b = W.dense_rhs(w.n, rng)
        y = orc.fwd(w.n, f["Lp"], f["Li"], f["Lx"], b)
        assert np.linalg.norm(orc.lmul(w.n, f["Lp"], f["Li"], f["Lx"], y) - b) <= 1e-13 * np.linalg.norm(b)


def test_pruned_forward_equals_full(orc):
    """The reach-pruned forward solve gives the full forward solve's result
    and leaves every entry outside the reach set exactly zero."""
    w = W.config1()
    f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    rng = np.random.default_rng(4)
    pinv = np.empty(w.n, np.int64)
    pinv[w.perm] = np.arange(w.n)
    for nb in (1, 8, 40):
        pos, val = W.sparse_rhs(w.n, nb, rng)
        b = np.zeros(w.n)
        b[pinv[pos]] = val
        r = orc.reach(w.n, f["Lp"], f["Li"], np.sort(pinv[pos]).astype(np.int32))
        xp = orc.fwd_pruned(w.n, f["Lp"], f["Li"], f["Lx"], r, b)
        xf = orc.fwd(w.n, f["Lp"], f["Li"], f["Lx"], b)
        outside = np.ones(w.n, bool)
        outside[r] = False
        assert (xp[outside] == 0.0).all()
        assert np.array_equal(xp, xf)
        assert r.size < w.n


def test_eta_inf_small(orc):
    w = W.config1()
    f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    b = W.dense_rhs(w.n, np.random.default_rng(1))
    x = orc.solve(w.n, w.perm, f["Lp"], f["Li"], f["Lx"], b)
    assert orc.eta_inf(w.n, w.Ap, w.Ai, w.Ax, x, b) < 1e-15 * 10
    # the backward error sees a perturbed solution
    assert orc.eta_inf(w.n, w.Ap, w.Ai, w.Ax, x * (1 + 1e-8), b) > 1e-12


def test_planted_mistakes_fail_pins(orc, monkeypatch):
    """Plant plausible mistakes in the oracle (on the CPU) and check that the
    pins above would catch them: a dropped update term and a transposed
    permutation."""
    w = W.random_spd(24, 0.25, np.random.default_rng(21))
    C = _perm_dense(w)
    Lref = np.tril(lapack.dpotrf(C, lower=1)[0])
    # (1) drop the update of the last earlier column
    f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    Lp, Li = f["Lp"], f["Li"]
    Cp, Ci, Cx = f["Cp"], f["Ci"], f["Cx"]
    Lx = np.zeros(Lp[-1])
    for j in range(w.n):                  # numpy re-run of the column method, one term dropped
        wv = np.zeros(w.n)
        wv[Ci[Cp[j]:Cp[j + 1]]] += Cx[Cp[j]:Cp[j + 1]]
        ks = [k for k in range(j) if j in Li[Lp[k]:Lp[k + 1]]]
        for k in ks[:-1]:
            rows = Li[Lp[k]:Lp[k + 1]]
            vals = Lx[Lp[k]:Lp[k + 1]]
            ljk = vals[rows == j][0]
            sel = rows >= j
            wv[rows[sel]] -= vals[sel] * ljk
        Lx[Lp[j]] = np.sqrt(wv[j])
        Lx[Lp[j] + 1:Lp[j + 1]] = wv[Li[Lp[j] + 1:Lp[j + 1]]] / Lx[Lp[j]]
    L = np.zeros((w.n, w.n))
    for j in range(w.n):
        L[Li[Lp[j]:Lp[j + 1]], j] = Lx[Lp[j]:Lp[j + 1]]
    assert np.linalg.norm(L - Lref) > 1e-6 * np.linalg.norm(Lref)
    assert orc.llt_residual(w.n, Cp, Ci, Cx, Lp, Li, Lx) > 1e-10
    # (2) using perm^-1 in place of perm changes the matrix factored
    pinv = np.empty(w.n, np.int64)
    pinv[w.perm] = np.arange(w.n)
    if not np.array_equal(pinv, w.perm):
        g = orc.factor(w.n, w.Ap, w.Ai, w.Ax, pinv)
        Lg = np.zeros((w.n, w.n))
        for j in range(w.n):
            Lg[g["Li"][g["Lp"][j]:g["Lp"][j + 1]], j] = g["Lx"][g["Lp"][j]:g["Lp"][j + 1]]
        assert np.linalg.norm(Lg - Lref) > 1e-6 * np.linalg.norm(Lref)


def test_llt_residual_equals_dense_definition(orc):
    """||L L^T - C||_F / ||C||_F written out with dense numpy matrices (the
    full symmetric C, off-diagonal entries counted twice) equals the
    oracle's sparse evaluation, for exact and for perturbed factors."""
    rng = np.random.default_rng(23)
    for t in range(20):
        n = int(rng.integers(3, 60))
        w = W.random_spd(n, float(rng.choice([0.05, 0.2, 0.6])), np.random.default_rng(4100 + t))
        f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        Cd = np.zeros((n, n))
        for j in range(n):
            for p in range(f["Cp"][j], f["Cp"][j + 1]):
                Cd[f["Ci"][p], j] = Cd[j, f["Ci"][p]] = f["Cx"][p]
        for scale in (0.0, 1e-3, 0.3):
            Lx = f["Lx"] * (1.0 + scale * rng.standard_normal(f["Lx"].size))
            Ld = np.zeros((n, n))
            for j in range(n):
                Ld[f["Li"][f["Lp"][j]:f["Lp"][j + 1]], j] = Lx[f["Lp"][j]:f["Lp"][j + 1]]
            ref = np.linalg.norm(Ld @ Ld.T - Cd) / np.linalg.norm(Cd)
            got = orc.llt_residual(n, f["Cp"], f["Ci"], f["Cx"], f["Lp"], f["Li"], Lx)
            assert abs(got - ref) <= 1e-12 * max(ref, 1e-3), (n, scale, got, ref)
