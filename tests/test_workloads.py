"""The batched generator reproduces the per-instance recipe exactly."""
import numpy as np

import workloads as W


def test_config4_batch_matches_instances():
    for kind in ("9pt128", "7pt24"):
        n, Ap, Ai, X, perm = W.config4_batch(kind, 3, k0=5)
        for j in range(3):
            w = W.config4_instance(kind, 5 + j)
            assert w.n == n and np.array_equal(w.Ap, Ap) and np.array_equal(w.Ai, Ai)
            assert np.allclose(X[j], w.Ax, rtol=1e-15, atol=0.0)
            assert np.array_equal(np.sort(perm), np.arange(n))


def test_config4_union_is_the_batch_side_by_side():
    """The union pattern holds the three batched families side by side:
    value set i carries 9-point instances 8 i .. 8 i + 7 and instance i of
    each 3-D family, with the per-family patterns shifted along the
    diagonal and their orderings placed one after another."""
    n, Ap, Ai, X, perm, off = W.config4_union(m=3, copies_9pt=2)
    assert X.shape[0] == 3 and np.array_equal(np.sort(perm), np.arange(n))
    fams = [W.config4_batch("9pt128", 6), W.config4_batch("7pt24", 3), W.config4_batch("7pt40", 3)]
    blocks = [(fams[0], lambda i: 2 * i), (fams[0], lambda i: 2 * i + 1), (fams[1], lambda i: i),
              (fams[2], lambda i: i)]
    for b, ((nb, Apb, Aib, Xb, pb), inst) in enumerate(blocks):
        o = off[b]
        cols = slice(o, o + nb)
        ps = Ap[o]
        assert np.array_equal(Ap[cols.start:cols.stop + 1] - ps, Apb)
        assert np.array_equal(Ai[ps:ps + Apb[-1]], Aib + o)
        assert np.array_equal(perm[o:o + nb], pb + o)
        for i in range(3):
            assert np.array_equal(X[i, ps:ps + Apb[-1]], Xb[inst(i)])
