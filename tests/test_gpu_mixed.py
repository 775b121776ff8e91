"""GPU: FP32 factor and FP64 iterative refinement against the oracle.

Tolerances: the FP32 factor differs from the FP64 oracle factor by the FP32
rounding of a backward-stable factorization, a few hundred times
u32 = 6e-8 on these well-conditioned inputs, so the elementwise bound is
1e-5 relative and the FP64-evaluated residual ||L L^T - A||_F/||A||_F is
bounded by 1e-5 (for the ill-conditioned grid only the residual is gated:
its factor's forward error grows with kappa).  Refinement must reach the requested normwise backward
error, evaluated independently by the oracle (eta_inf <= 1e-12), and its
solution must match the oracle's FP64 solution to kappa * 1e-12.
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


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def test_fp32_factor_matches_oracle(S, orc, torch_cuda):
    torch = torch_cuda
    rng = np.random.default_rng(41)
    cases = [W.random_spd(int(rng.integers(5, 150)), float(rng.choice([0.05, 0.3, 1.0])),
                          np.random.default_rng(900 + t)) for t in range(12)]
    cases += [W.config1(), W.config3(12)]
    for w in cases:
        # the weighted 27-point grid has kappa ~ 1e6: its factor's forward
        # error is kappa-amplified, so only the backward residual is gated
        well_conditioned = not w.name.startswith("grid3d")
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, precision="f32")
        an.factor(torch.from_numpy(w.Ax).cuda())
        assert an.status() == 0
        f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
        Lx = an.export_factor()
        e = _rel(Lx, f["Lx"])
        res = orc.llt_residual(w.n, f["Cp"], f["Ci"], f["Cx"], f["Lp"], f["Li"], Lx)
        _say(f"case fp32 {w.name}: rel diff {e:.2e} llt residual {res:.2e}")
        assert res <= 1e-5
        if well_conditioned:
            assert e <= 1e-5


@pytest.mark.parametrize("method", ["ir", "pcg"])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_refinement_reaches_1e12(S, orc, torch_cuda, precision, method):
    """3-D 27-point weighted Laplacian (the mixed-precision workload's
    recipe, 20^3): FP32 or FP64 factor, FP64 refinement (classical or
    conjugate-gradient accelerated) to eta <= 1e-12."""
    torch = torch_cuda
    w = W.config3(20)
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd", precision=precision)
    Ax = torch.from_numpy(w.Ax).cuda()
    an.factor(Ax)
    assert an.status() == 0
    b = W.dense_rhs(w.n, np.random.default_rng(7))
    x, iters, eta = an.refine(Ax, torch.from_numpy(b).cuda(), tol=1e-12, maxit=30, method=method)
    x = x.cpu().numpy()
    eta_orc = orc.eta_inf(w.n, w.Ap, w.Ai, w.Ax, x, b)
    f = orc.factor(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    x_ref = orc.solve(w.n, w.perm, f["Lp"], f["Li"], f["Lx"], b)
    e = _rel(x, x_ref)
    _say(f"case refine {method} {precision} {w.name}: iters {iters} eta {eta:.2e} (oracle {eta_orc:.2e}) "
         f"x rel diff {e:.2e}")
    assert eta <= 1e-12 and eta_orc <= 1e-12
    # the two residuals differ by summation order: at most rounding noise,
    # about n_row * u relative to ||A|| ||x|| (1e-15 here)
    assert abs(eta - eta_orc) <= 1e-3 * eta_orc + 1e-15
    if precision == "f64":
        assert iters <= 1
    else:
        assert 1 <= iters <= 30
    # solution error of a backward-stable result: at most kappa * eta; the
    # recipe's kappa (row-sum scaled) is ~1e6, so 1e6 * 1e-12 bounds it
    assert e <= 1e-5


def test_pcg_needs_fewer_corrections_than_ir(S, torch_cuda):
    """On the ill-conditioned recipe the conjugate-gradient form reaches
    1e-12 with fewer applications of the FP32 factor than classical
    refinement (both from the same factor and right-hand side)."""
    torch = torch_cuda
    w = W.config3(24)
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd", precision="f32")
    Ax = torch.from_numpy(w.Ax).cuda()
    an.factor(Ax)
    b = torch.from_numpy(W.dense_rhs(w.n, np.random.default_rng(9))).cuda()
    _, it_ir, eta_ir = an.refine(Ax, b, tol=1e-12, maxit=60, method="ir")
    _, it_cg, eta_cg = an.refine(Ax, b, tol=1e-12, maxit=60, method="pcg")
    _say(f"case ir vs pcg: ir {it_ir} ({eta_ir:.1e}), pcg {it_cg} ({eta_cg:.1e})")
    assert eta_ir <= 1e-12 and eta_cg <= 1e-12
    assert it_cg <= it_ir


def test_refinement_reports_stagnation(S, torch_cuda):
    """A shifted Laplacian with kappa * u32 > 1: FP32 refinement need not
    converge; the call returns after maxit corrections with the honest eta."""
    torch = torch_cuda
    w = W.config2(16)
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd", precision="f32")
    Ax = torch.from_numpy(w.Ax).cuda()
    an.factor(Ax)
    b = torch.from_numpy(W.dense_rhs(w.n, np.random.default_rng(8))).cuda()
    x, iters, eta = an.refine(Ax, b, tol=1e-30, maxit=3)
    _say(f"case stagnation: iters {iters} eta {eta:.2e}")
    assert iters == 3 and eta > 0.0


def test_fp32_indefinite_reports_pivot(S, orc, torch_cuda):
    torch = torch_cuda
    w = W.random_spd(80, 0.1, np.random.default_rng(77))
    Ax = w.Ax.copy()
    col = 33
    Ax[w.Ap[col]] = -Ax[w.Ap[col]]
    f = orc.factor(w.n, w.Ap, w.Ai, Ax, w.perm)
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, precision="f32")
    an.factor(torch.from_numpy(Ax).cuda())
    assert an.status() == 1 + int(w.perm[f["info"] - 1])


@pytest.mark.parametrize("method", ["ir", "pcg"])
def test_refinement_on_failed_factor_is_an_error(S, orc, torch_cuda, method):
    """An indefinite matrix: the FP32 factor records a non-positive pivot and
    its solves fill x with NaN.  Refinement must not report a small backward
    error for that: the call fails with SYM_ENUMERIC and eta is not <= tol."""
    from paper_1705_06575_amd import SymError
    torch = torch_cuda
    w = W.random_spd(80, 0.1, np.random.default_rng(78))
    Ax = w.Ax.copy()
    col = 21
    Ax[w.Ap[col]] = -Ax[w.Ap[col]]
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, precision="f32")
    Axd = torch.from_numpy(Ax).cuda()
    an.factor(Axd)
    assert an.status() != 0
    b = torch.from_numpy(W.dense_rhs(w.n, np.random.default_rng(5))).cuda()
    with pytest.raises(SymError) as e:
        an.refine(Axd, b, tol=1e-12, maxit=5, method=method)
    _say(f"case refine {method} on failed factor: {e.value.name}")
    assert e.value.name == "SYM_ENUMERIC"
