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
