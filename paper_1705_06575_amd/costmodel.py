"""Learned cost model for per-supernode kernel variants.

Each device supernode's external update can run in one of three variants
(sym_set_variants: every incidence on the per-wavefront path, or the ones
of at least 64 / 32 rows, columns and inner indices on the workgroup's LDS
path; variant 1 is the default).  The autotuner's measurements -- the
workgroup time of every external-update task of a profiled factorization,
summed per supernode, under each variant -- train small networks (the
library's FP32 2 x 64 MLP, trained on the GPU by its own forward, backward
and Adam kernels; four from different initial weights, averaged) to
predict, from a supernode's features and a variant v != 1,
log(T_v / T_1): how much faster or slower v is than the default.  The
ratio rather than the time itself is learned because the choice depends
only on differences between variants, which are small next to the times.
Supernodes whose default time is below `min_us` are left out of training
(their ratios are mostly noise and their share of the time negligible)
and keep the default; a variant replaces the default only when its
predicted gain exceeds a margin chosen by leave-one-pattern-out
validation on the training patterns (no replacement at all when no
margin pays there).  Exhaustive measurement of all variants stays the
fallback and the judge: `regret` compares a choice with the per-supernode
best.

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


class _Chooser:
    """Variant choice from predicted log-ratios (needs `predict` and
    `margin`)."""

    def choose(self, feat, margin: float | None = None, min_work: float = 0.0) -> np.ndarray:
        """Per supernode: the variant with the smallest predicted log-ratio
        to the default, if that beats the default by more than `margin`
        (log scale; the model's own, set by `train`, when None), else the
        default.  Supernodes with fewer than `min_work` update flops keep
        the default."""
        if margin is None:
            margin = self.margin
        f = np.asarray(feat).reshape(-1, NFEAT)
        k = f.shape[0]
        r = np.zeros((k, NVAR))
        for v in (0, 2):
            r[:, v] = self.predict(encode(f, np.full(k, v)))
        v = np.argmin(r, axis=1)
        keep = (r[np.arange(k), v] > -margin) | (f[:, 4] < min_work)
        v[keep] = 1
        return v.astype(np.uint8)


class CostModel(_Chooser):
    """The network plus the input standardization it was fit with.
    Targets are log-ratios of a variant's time to the default's."""

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
        self.margin = 0.02

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

MARGINS = (0.02, 0.05, 0.1, 0.2)


class Ensemble(_Chooser):
    """Networks fit from different initial weights to the same rows; the
    prediction is their mean, which is steadier than any one of them."""

    def __init__(self, members):
        self.members = list(members)
        self.margin = 0.02

    def predict(self, X) -> np.ndarray:
        return np.mean([m.predict(X) for m in self.members], axis=0)


MEMBERS = 4


def _fit(measured, min_us: float, epochs: int, seed: int, members: int = MEMBERS):
    X = np.concatenate([dataset(f, T, min_us)[0] for f, T in measured])
    t = np.concatenate([dataset(f, T, min_us)[1] for f, T in measured])
    flops = np.concatenate([np.asarray(f).reshape(-1, NFEAT)[np.asarray(T)[:, 1] >= min_us, 4]
                            for f, T in measured])
    nets, hist = [], []
    for i in range(members):
        net = CostModel(seed=seed + i)
        hist.append(net.fit(X, t, epochs=epochs))
        nets.append(net)
    hist = np.mean(np.asarray(hist), axis=0).tolist()
    return Ensemble(nets), float(np.percentile(flops, 5)), hist, X.shape[0]


def select_margin(measured, min_us: float = 10.0, epochs: int = 400, seed: int = 0,
                  margins=MARGINS) -> float:
    """The decision margin by leave-one-pattern-out validation: for each
    training pattern, a model fit to the others chooses its variants under
    every candidate margin, scored by that pattern's measured times.  The
    margin with the smallest time summed over the patterns wins; if even
    that one is not below the default variant's sum, the result is
    infinite, i.e. the model never overrides the default."""
    cost = np.zeros(len(margins))
    base = 0.0
    for i, (f, T) in enumerate(measured):
        rest = [m for j, m in enumerate(measured) if j != i]
        model, min_work, _, _ = _fit(rest, min_us, epochs, seed)
        T = np.asarray(T)
        k = np.arange(T.shape[0])
        base += float(T[:, 1].sum())
        for c, mg in enumerate(margins):
            cost[c] += float(T[k, model.choose(f, margin=mg, min_work=min_work)].sum())
    best = int(np.argmin(cost))
    return float(margins[best]) if cost[best] < base else float("inf")


def train(measured, min_us: float = 10.0, epochs: int = 400, seed: int = 0):
    """An ensemble of MEMBERS networks fit to [(features, T), ...]
    measured on training patterns, and the update-flop floor below which
    its choices keep the default (the 5th percentile of the training
    supernodes').  With two or more patterns the decision margin comes
    from `select_margin`."""
    model, min_work, hist, rows = _fit(measured, min_us, epochs, seed)
    if len(measured) >= 2:
        model.margin = select_margin(measured, min_us, epochs, seed)
    return model, min_work, hist, rows


def dataset(feat, T, min_us: float = 10.0):
    """Training rows from measured T[s, v]: inputs for variants 0 and 2 of
    every supernode whose default time is at least min_us, targets
    log(T[s, v] / T[s, 1])."""
    f = np.asarray(feat).reshape(-1, NFEAT)
    T = np.asarray(T)
    sel = T[:, 1] >= min_us
    fs = f[sel]
    k = fs.shape[0]
    X = np.concatenate([encode(fs, np.full(k, v)) for v in (0, 2)])
    t = np.concatenate([np.log(np.maximum(T[sel, v], 1e-3) / T[sel, 1]) for v in (0, 2)])
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
