"""GPU: factors whose Schur-complement update products run on the 16-bit
matrix cores (SYM_BF16, SYM_F16), against the FP64 oracle, and FP64
refinement with them to a normwise backward error of 1e-12.

Bound on the factor.  The update products take their operands rounded to
16 bits (unit roundoff u16 = 2^-8 for bfloat16, 2^-11 for IEEE half) and
accumulate in FP32; to first order an entry of a Schur-complement update,
sum_k l_ik l_jk, is then off by at most 2 u16 sum_k |l_ik| |l_jk| (each
product of two rounded operands is off by at most 2 u16 of its size), and
the FP32 and FP64 parts of the factorization add far less.  So the computed
factor satisfies |L L^T - A| <= c u16 |L| |L^T| entrywise with c a small
constant; the test takes c = 4 in the Frobenius norm, with ||L L^T - A||_F
evaluated by the oracle in FP64 and || |L| |L^T| ||_F from the exported
factor.  The per-supernode scaling is exact (powers of two), and the export
undoes it, so the bound is on the factor of P A P^T itself.

Refinement is gated as for the FP32 factor: eta_inf <= 1e-12 by the
library and, independently, by the oracle.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import torch  # noqa: F401

import workloads as W

pytestmark = pytest.mark.gpu

U16 = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}


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


def _abs_product_norm(n, Lp, Li, Lx):
    """|| |L| |L^T| ||_F for L in CSC."""
    L = sp.csc_matrix((np.abs(Lx), Li, Lp), shape=(n, n))
    return float(sp.linalg.norm(L @ L.T))


def _check_factor(S, orc, torch, w, precision, Ax=None):
    Ax = w.Ax if Ax is None else Ax
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, precision=precision)
    an.factor(torch.from_numpy(Ax).cuda())
    assert an.status() == 0
    f = orc.factor(w.n, w.Ap, w.Ai, Ax, w.perm)
    Lx = an.export_factor()
    res = orc.llt_residual(w.n, f["Cp"], f["Ci"], f["Cx"], f["Lp"], f["Li"], Lx)
    anorm = float(np.linalg.norm(f["Cx"]) * np.sqrt(2.0))     # ||A||_F from its lower triangle, roughly
    cnorm = np.sqrt(2.0 * np.sum(f["Cx"] ** 2) - np.sum(f["Cx"][f["Cp"][:-1]] ** 2))
    bound = 4.0 * U16[precision] * _abs_product_norm(w.n, f["Lp"], f["Li"], Lx) / cnorm
    pert = an.pivots_perturbed()
    _say(f"case {precision} {w.name} n={w.n}: llt residual {res:.2e} bound {bound:.2e} "
         f"perturbed pivots {pert}")
    del anorm
    assert np.isfinite(res) and res <= bound
    return an, pert


@pytest.mark.parametrize("precision", ["bf16", "f16"])
def test_16bit_factor_within_rounding_bound(S, orc, torch_cuda, precision):
    torch = torch_cuda
    rng = np.random.default_rng(51)
    cases = [W.random_spd(int(rng.integers(20, 200)), float(rng.choice([0.05, 0.3, 1.0])),
                          np.random.default_rng(950 + t)) for t in range(8)]
    cases += [W.config1(), W.config3(12), W.config2(14)]
    for w in cases:
        _, pert = _check_factor(S, orc, torch, w, precision)
        if not w.name.startswith("grid3d"):
            assert pert == 0


def test_f16_scaling_keeps_wide_ranges_finite(S, orc, torch_cuda):
    """A well-conditioned SPD matrix under a two-sided diagonal scaling whose
    entries span 2^-30 .. 2^30: unscaled, its entries (up to ~1e18) overflow
    IEEE half (largest 65504).  The per-supernode scaling brings every
    device supernode's largest diagonal entry to [1/2, 2), so the factor
    stays finite and within the rounding bound."""
    torch = torch_cuda
    w = W.random_spd(160, 0.3, np.random.default_rng(13))
    e = np.random.default_rng(14).integers(-15, 16, w.n).astype(np.float64)
    d = 2.0 ** e
    cols = np.repeat(np.arange(w.n), np.diff(w.Ap))
    Ax = w.Ax * d[w.Ai] * d[cols]
    assert Ax.max() > 1e8
    _check_factor(S, orc, torch, w, "f16", Ax=Ax)


@pytest.mark.parametrize("precision", ["bf16", "f16"])
def test_16bit_refinement_reaches_1e12(S, orc, torch_cuda, precision):
    """The mixed-precision recipe (3-D 27-point, weights log-uniform in
    [1e-3, 1e3], kappa ~ 1e6) at 20^3: CG refinement with the 16-bit-update
    factor as preconditioner reaches eta_inf <= 1e-12."""
    torch = torch_cuda
    w = W.config3(20)
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, precision=precision)
    Ax = torch.from_numpy(w.Ax).cuda()
    an.factor(Ax)
    assert an.status() == 0
    b = W.dense_rhs(w.n, np.random.default_rng(17))
    x, iters, eta = an.refine(Ax, torch.from_numpy(b).cuda(), tol=1e-12, maxit=200, method="pcg")
    x = x.cpu().numpy()
    eta_orc = orc.eta_inf(w.n, w.Ap, w.Ai, w.Ax, x, b)
    _say(f"case refine pcg {precision} {w.name}: iters {iters} eta {eta:.2e} (oracle {eta_orc:.2e}) "
         f"perturbed pivots {an.pivots_perturbed()}")
    assert eta <= 1e-12 and eta_orc <= 1e-12
    assert abs(eta - eta_orc) <= 1e-3 * eta_orc + 1e-15


def test_16bit_batch_equals_single_factors(S, torch_cuda):
    """A batch of bf16-update factors: each instance has its own scaling
    (from its own diagonal); every instance's solve matches a single
    factorization of its values to rounding."""
    torch = torch_cuda
    ws = [W.weighted_grid((16, 16), True, 1e-2, 1e2, "shift1e-3", np.random.default_rng(700 + k),
                          f"g#{k}") for k in range(3)]
    w0 = ws[0]
    an = S.Analysis(w0.n, w0.Ap, w0.Ai, ordering="nd", precision="bf16")
    Axb = torch.from_numpy(np.stack([w.Ax for w in ws])).cuda()
    bt = S.Batch(an, len(ws))
    bt.factor(Axb)
    assert (bt.status() == 0).all()
    B = torch.from_numpy(np.stack([W.dense_rhs(w0.n, np.random.default_rng(80 + k))
                                   for k in range(len(ws))])).cuda()
    Xb = B.clone()
    bt.solve_(Xb)
    perm = an.get("perm")
    for k, w in enumerate(ws):
        single = S.Analysis(w.n, w.Ap, w.Ai, ordering=perm, precision="bf16")
        single.factor(torch.from_numpy(w.Ax).cuda())
        x1 = single.solve(B[k])
        dd = float(torch.linalg.norm(x1 - Xb[k]) / torch.linalg.norm(x1))
        _say(f"case bf16 batch instance {k}: rel diff to single solve {dd:.1e}")
        assert dd <= 1e-12
