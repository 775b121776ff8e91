"""GPU: the allocation-free full solve, sym_solve_static, called through the
C ABI, against sym_solve on the same factor and right-hand side.

Both run the same sweep kernels on the same FP64 factor; they differ only
in where the sweeps' scratch lives (the bound workspace or the library's
static array) and in the order of the sweeps' atomic additions, so the
solutions agree to rounding: relative 1e-12, far above the ~1e-15 such
reorderings cause and far below any real error.  Two calls in a row, the
second on a smaller system, show that what the first call left in the
shared array does not leak into the second.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_static_solve_matches_solve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_06575_amd as S
    lib = S.load_library()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cases = [W.config3(18), W.laplace2d_5pt(17, 23)]
    assert cases[1].n < cases[0].n
    for k, w in enumerate(cases):
        _say(f"case static solve {w.name} n={w.n}")
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm)
        an.factor(torch.from_numpy(w.Ax).cuda())
        assert an.status() == 0
        b = torch.from_numpy(W.dense_rhs(w.n, np.random.default_rng(60 + k))).cuda()
        x_ref = an.solve(b)
        x = b.clone()
        rc = lib.sym_solve_static(an._h, ctypes.c_void_p(x.data_ptr()), stream)
        assert rc == 0
        torch.cuda.synchronize()
        d = float(torch.linalg.norm(x - x_ref) / torch.linalg.norm(x_ref))
        _say(f"  rel diff to sym_solve {d:.2e}")
        assert d <= 1e-12
        # and once more on the same system: the array's previous contents
        # (this system's own counters and sums) are cleared as well
        x2 = b.clone()
        assert lib.sym_solve_static(an._h, ctypes.c_void_p(x2.data_ptr()), stream) == 0
        torch.cuda.synchronize()
        d2 = float(torch.linalg.norm(x2 - x_ref) / torch.linalg.norm(x_ref))
        assert d2 <= 1e-12
