"""Learned cost model for per-supernode kernel variants.

Each device supernode's external update can run in one of three variants
(sym_set_variants: every incidence on the per-wavefront path, or the ones
of at least 32 / 16 rows, columns and inner indices on the workgroup's LDS
path).  The autotuner's measurements -- the workgroup time of every
external-update task of a profiled factorization, summed per supernode,
under each variant -- train a small network (the library's FP32 2 x 64
MLP, trained on the GPU by its own forward, backward and Adam kernels) to
predict a supernode's time from its features and a variant; the model then
picks each supernode's variant.  Exhaustive measurement of all variants
stays the fallback and the judge: `regret` compares a choice with the
per-supernode best.

Argument marshalling only: the network's arithmetic runs in the library's
kernels (sym_mlp_forward / sym_mlp_backward / sym_mlp_adam).
"""
from __future__ import annotations

import ctypes

import numpy as np

from .binding import _check, _dev_ptr, _stream, load_library

NVAR = 3                 # kernel variants
NFEAT = 8                # features per device supernode (SYM_GET_SUPER_FEAT)
D_IN = NFEAT + NVAR      # network inputs: transformed features + one-hot variant


def encode(feat: np.ndarray, variant: np.ndarray) -> np.ndarray:
    """Network inputs for supernodes with features feat (k x 8) run in
    `variant` (k): logs of the sizes, counts and flops, the two flop
    fractions as they are, and the variant one-hot."""
    f = np.asarray(feat, dtype=np.float64).reshape(-1, NFEAT)
    x = np.empty((f.shape[0], D_IN))
    x[:, 0:5] = np.log1p(f[:, 0:5])
    x[:, 5:7] = f[:, 5:7]
    x[:, 7] = np.log1p(f[:, 7])
    x[:, 8:] = 0.0
    x[np.arange(f.shape[0]), 8 + np.asarray(variant, dtype=np.int64)] = 1.0
    return x


def measure_variants(an, Ax, reps: int = 2) -> np.ndarray:
    """Measured time (us) of every device supernode's external update under
    each variant: T[s, v] = sum of its tasks' workgroup times, the median
    over `reps` profiled factorizations.  Leaves `an` with variant 1."""
    nds = int(an.stat("ndsuper"))
    T = np.zeros((nds, NVAR))
    for v in range(NVAR):
        an.set_variants(np.full(nds, v, dtype=np.uint8))
        an.factor(Ax)                                # binds, warms up
        runs = []
        an.profile(True)
        for _ in range(reps):
            an.factor(Ax)
            an.profile_read()
            ts = an.task_times()
            owner = an.get("task_super")
            per = np.zeros(nds)
            m = owner >= 0
            np.add.at(per, owner[m], ts[m])
            runs.append(per)
        an.profile(False)
        T[:, v] = np.median(np.stack(runs), axis=0)
    an.set_variants(np.full(nds, 1, dtype=np.uint8))
    return T


class CostModel:
    """The network plus the input/target standardization it was fit with.
    Targets are log(time in us)."""

    def __init__(self, seed: int = 0, device="cuda"):
        import torch
        L = load_library()
        self._lib = L
        cnt = ctypes.c_int64()
        _check("sym_mlp_param_count", L.sym_mlp_param_count(D_IN, ctypes.byref(cnt)))
        self.count = cnt.value
        rng = np.random.default_rng(seed)
        H = 64
        parts = [rng.normal(0, np.sqrt(2.0 / D_IN), H * D_IN), np.zeros(H),
                 rng.normal(0, np.sqrt(2.0 / H), H * H), np.zeros(H),
                 rng.normal(0, np.sqrt(1.0 / H), H), np.zeros(1)]
        p = np.concatenate(parts).astype(np.float32)
        assert p.size == self.count
        self.device = device
        self.params = torch.from_numpy(p).to(device)
        self.mu = np.zeros(D_IN)
        self.sd = np.ones(D_IN)

    def _inputs(self, X):
        import torch
        Z = ((np.asarray(X, dtype=np.float64) - self.mu) / self.sd).astype(np.float32)
        return torch.from_numpy(np.ascontiguousarray(Z)).to(self.device)

    def predict(self, X) -> np.ndarray:
        import torch
        Xd = self._inputs(X)
        n = Xd.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=self.device)
        _check("sym_mlp_forward", self._lib.sym_mlp_forward(
            _dev_ptr(self.params, "torch.float32"), _dev_ptr(Xd, "torch.float32"), n, D_IN,
            _dev_ptr(y, "torch.float32"), _stream()))
        return y.cpu().numpy().astype(np.float64)

    def fit(self, X, t, epochs: int = 400, lr: float = 3e-3) -> list:
        """Full-batch Adam on the mean squared error of log-times.  Returns
        the training loss every 50 epochs."""
        import torch
        X = np.asarray(X, dtype=np.float64)
        self.mu = X.mean(axis=0)
        self.sd = X.std(axis=0)
        self.sd[self.sd == 0] = 1.0
        Xd = self._inputs(X)
        n = Xd.shape[0]
        td = torch.from_numpy(np.asarray(t, dtype=np.float32)).to(self.device)
        grad = torch.zeros(self.count, dtype=torch.float32, device=self.device)
        m = torch.zeros_like(grad)
        v = torch.zeros_like(grad)
        work = torch.empty(n * (4 * 64 + 1), dtype=torch.float32, device=self.device)
        hist = []
        for ep in range(1, epochs + 1):
            _check("sym_mlp_backward", self._lib.sym_mlp_backward(
                _dev_ptr(self.params, "torch.float32"), _dev_ptr(Xd, "torch.float32"),
                _dev_ptr(td, "torch.float32"), n, D_IN, _dev_ptr(grad, "torch.float32"),
                _dev_ptr(work, "torch.float32"), _stream()))
            _check("sym_mlp_adam", self._lib.sym_mlp_adam(
                _dev_ptr(self.params, "torch.float32"), _dev_ptr(grad, "torch.float32"),
                _dev_ptr(m, "torch.float32"), _dev_ptr(v, "torch.float32"), self.count, ep,
                ctypes.c_float(lr), _stream()))
            if ep % 50 == 0 or ep == epochs:
                y = self.predict(X)
                hist.append(float(np.mean((y - np.asarray(t)) ** 2)))
        return hist

    def choose(self, feat) -> np.ndarray:
        """Variant with the smallest predicted time for every supernode."""
        f = np.asarray(feat).reshape(-1, NFEAT)
        k = f.shape[0]
        pred = np.stack([self.predict(encode(f, np.full(k, v))) for v in range(NVAR)], axis=1)
        return np.argmin(pred, axis=1).astype(np.uint8)


def dataset(feat, T):
    """Training rows (inputs, log-time targets) from measured T[s, v]."""
    f = np.asarray(feat).reshape(-1, NFEAT)
    k = f.shape[0]
    X = np.concatenate([encode(f, np.full(k, v)) for v in range(NVAR)])
    t = np.concatenate([np.log(np.maximum(T[:, v], 1e-3)) for v in range(NVAR)])
    return X, t


def regret(T, choice) -> dict:
    """Per-supernode measured cost of a choice against the exhaustive best
    and against the default variant 1 (sums over supernodes, us)."""
    T = np.asarray(T)
    k = np.arange(T.shape[0])
    best = float(T.min(axis=1).sum())
    return {"chosen_us": float(T[k, choice].sum()), "best_us": best,
            "default_us": float(T[:, 1].sum()),
            "regret_us": float(T[k, choice].sum()) - best,
            "default_regret_us": float(T[:, 1].sum()) - best}
