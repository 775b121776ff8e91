"""Learned cost model for per-supernode kernel variants.

Each device supernode's external update can run in one of four variants
(sym_set_variants): every incidence on the per-wavefront path (0); the
ones of at least 64 (1, the default) or 32 (2) rows, columns and inner
indices on the workgroup's LDS path; or every incidence as LDS-staged
chunks (3).  Measured times -- the workgroup time of every external-update
task of a profiled factorization, summed per supernode, under each variant
-- train small networks (the library's FP32 2 x 64 MLP, trained on the GPU
by its own forward, backward and Adam kernels; four from different initial
weights, averaged) to predict, from a supernode's features and a variant
v != 1, log(T_v / T_1): how much faster or slower v is than the default.
The ratio rather than the time itself is learned because the choice depends
only on differences between variants, which are small next to the times.

The features are the supernode's own (width, rows, update tiles,
incidences, update flops and their size mix, level) and its level's
context: the level's update flops, supernode count and update tiles, and
the supernode's share of them.  The context matters: the same supernode
favours the workgroup path when its launch is crowded and the per-wavefront
path when it has the device to itself.

Only supernodes whose default time is at least `min_us` (1 ms) train the
model: a few dozen supernodes per graph hold almost all of the external
update's time, and rows of the thousands of small ones would otherwise
dominate the fit while their ratios are mostly noise.  At choice time,
supernodes with fewer update flops than the smallest training supernode
keep the default; a variant replaces the default only when its predicted
gain exceeds a margin chosen by leave-one-pattern-out validation on the
training patterns (no replacement at all when no margin pays there).
Exhaustive measurement of all variants stays the fallback and the yardstick:
`regret` compares a choice with the per-supernode best.  A trained model
is saved to and loaded from an .npz file (`Ensemble.save`, `load`); the
package ships one trained on the k-NN family (`DEFAULT_MODEL`, written by
`train_costmodel`).

Argument marshalling only: the network's arithmetic runs in the library's
kernels (sym_mlp_forward / sym_mlp_backward / sym_mlp_adam).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .binding import _check, _dev_ptr, _stream, load_library, mlp_work_size

NVAR = 4                 # kernel variants
DEFAULT = 1              # the library's default variant
ALT = (0, 2, 3)          # the variants the model weighs against the default
NFEAT = 12               # features per device supernode (SYM_GET_SUPER_FEAT)
D_IN = NFEAT + NVAR      # network inputs: transformed features + one-hot variant
DEFAULT_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "costmodel_knn13.npz")


def encode(feat: np.ndarray, variant: np.ndarray) -> np.ndarray:
    """Network inputs for supernodes with features feat (k x 12) run in
    `variant` (k): logs of the sizes, counts, flops and the level, the
    flop fractions as they are, and the variant one-hot."""
    f = np.asarray(feat, dtype=np.float64).reshape(-1, NFEAT)
    x = np.empty((f.shape[0], D_IN))
    x[:, 0:5] = np.log1p(f[:, 0:5])
    x[:, 5:7] = f[:, 5:7]
    x[:, 7:11] = np.log1p(f[:, 7:11])
    x[:, 11] = f[:, 11]
    x[:, NFEAT:] = 0.0
    x[np.arange(f.shape[0]), NFEAT + np.asarray(variant, dtype=np.int64)] = 1.0
    return x


def measure_variants(an, Ax, reps: int = 2, say=None) -> np.ndarray:
    """Measured time (us) of every device supernode's external update under
    each variant: T[s, v] = sum of its tasks' workgroup times, the median
    over `reps` profiled factorizations.  Leaves `an` with variant 1.
    `say`, if given, is called with a line of progress per variant."""
    nds = int(an.stat("ndsuper"))
    T = np.zeros((nds, NVAR))
    for v in range(NVAR):
        if say:
            say(f"measure variant {v} of {NVAR} ({nds} supernodes)")
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
    an.set_variants(np.full(nds, DEFAULT, dtype=np.uint8))
    return T


class _Chooser:
    """Variant choice from predicted log-ratios (needs `predict` and
    `margin`)."""

    def choose(self, feat, margin: float | None = None, min_work: float | None = None) -> np.ndarray:
        """Per supernode: the variant with the smallest predicted log-ratio
        to the default, if that beats the default by more than `margin`
        (log scale), else the default.  Supernodes with fewer than
        `min_work` update flops keep the default.  Either left None takes
        the model's own (set by `train` or `load`)."""
        if margin is None:
            margin = self.margin
        if min_work is None:
            min_work = getattr(self, "min_work", 0.0)
        f = np.asarray(feat).reshape(-1, NFEAT)
        k = f.shape[0]
        r = np.zeros((k, NVAR))
        for v in ALT:
            r[:, v] = self.predict(encode(f, np.full(k, v)))
        v = np.argmin(r, axis=1)
        keep = (r[np.arange(k), v] > -margin) | (f[:, 4] < min_work)
        v[keep] = DEFAULT
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
        work = torch.empty(mlp_work_size(n, D_IN), dtype=torch.float32, device=self.device)
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

MARGINS = (0.0, 0.02, 0.05, 0.1)
MIN_US = 1000.0          # training supernodes: default external-update time of at least 1 ms


class Ensemble(_Chooser):
    """Networks fit from different initial weights to the same rows; the
    prediction is their mean, which is steadier than any one of them."""

    def __init__(self, members):
        self.members = list(members)
        self.margin = 0.02
        self.min_work = 0.0

    def predict(self, X) -> np.ndarray:
        return np.mean([m.predict(X) for m in self.members], axis=0)

    def save(self, path, **meta) -> None:
        """Write the members' weights and input standardization, the margin
        and the work floor to an .npz file (plus any `meta` arrays)."""
        np.savez(path, params=np.stack([m.params.cpu().numpy() for m in self.members]),
                 mu=np.stack([m.mu for m in self.members]), sd=np.stack([m.sd for m in self.members]),
                 margin=np.float64(self.margin), min_work=np.float64(self.min_work),
                 nfeat=np.int64(NFEAT), nvar=np.int64(NVAR), **meta)


def load(path: str | None = None, device="cuda") -> Ensemble:
    """The ensemble saved at `path` (DEFAULT_MODEL when None)."""
    import torch
    z = np.load(DEFAULT_MODEL if path is None else path, allow_pickle=False)
    if int(z["nfeat"]) != NFEAT or int(z["nvar"]) != NVAR:
        raise ValueError("cost model file was written for other features or variants")
    nets = []
    for i in range(z["params"].shape[0]):
        net = CostModel(seed=0, device=device)
        if z["params"].shape[1] != net.count:
            raise ValueError("cost model file has the wrong parameter count")
        net.params = torch.from_numpy(np.ascontiguousarray(z["params"][i])).to(device)
        net.mu, net.sd = z["mu"][i].copy(), z["sd"][i].copy()
        nets.append(net)
    ens = Ensemble(nets)
    ens.margin = float(z["margin"])
    ens.min_work = float(z["min_work"])
    return ens


MEMBERS = 4


def _fit(measured, min_us: float, epochs: int, seed: int, members: int = MEMBERS):
    X = np.concatenate([dataset(f, T, min_us)[0] for f, T in measured])
    t = np.concatenate([dataset(f, T, min_us)[1] for f, T in measured])
    flops = np.concatenate([np.asarray(f).reshape(-1, NFEAT)[np.asarray(T)[:, DEFAULT] >= min_us, 4]
                            for f, T in measured])
    nets, hist = [], []
    for i in range(members):
        net = CostModel(seed=seed + i)
        hist.append(net.fit(X, t, epochs=epochs))
        nets.append(net)
    hist = np.mean(np.asarray(hist), axis=0).tolist()
    return Ensemble(nets), float(np.min(flops)), hist, X.shape[0]


def select_margin(measured, min_us: float = MIN_US, epochs: int = 400, seed: int = 0,
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
        base += float(T[:, DEFAULT].sum())
        for c, mg in enumerate(margins):
            cost[c] += float(T[k, model.choose(f, margin=mg, min_work=min_work)].sum())
    best = int(np.argmin(cost))
    return float(margins[best]) if cost[best] < base else float("inf")


def train(measured, min_us: float = MIN_US, epochs: int = 400, seed: int = 0):
    """An ensemble of MEMBERS networks fit to [(features, T), ...]
    measured on training patterns, and the update-flop floor below which
    its choices keep the default (the smallest training supernode's).  With
    two or more patterns the decision margin comes from `select_margin`."""
    model, min_work, hist, rows = _fit(measured, min_us, epochs, seed)
    model.min_work = min_work
    if len(measured) >= 2:
        model.margin = select_margin(measured, min_us, epochs, seed)
    return model, min_work, hist, rows


def dataset(feat, T, min_us: float = MIN_US):
    """Training rows from measured T[s, v]: inputs for every variant v other
    than the default, for every supernode whose default time is at least
    min_us, targets log(T[s, v] / T[s, 1])."""
    f = np.asarray(feat).reshape(-1, NFEAT)
    T = np.asarray(T)
    sel = T[:, DEFAULT] >= min_us
    fs = f[sel]
    k = fs.shape[0]
    X = np.concatenate([encode(fs, np.full(k, v)) for v in ALT])
    t = np.concatenate([np.log(np.maximum(T[sel, v], 1e-3) / T[sel, DEFAULT]) for v in ALT])
    return X, t


def regret(T, choice) -> dict:
    """Per-supernode measured cost of a choice against the exhaustive best
    and against the default variant 1 (sums over supernodes, us)."""
    T = np.asarray(T)
    k = np.arange(T.shape[0])
    best = float(T.min(axis=1).sum())
    return {"chosen_us": float(T[k, choice].sum()), "best_us": best,
            "default_us": float(T[:, DEFAULT].sum()),
            "regret_us": float(T[k, choice].sum()) - best,
            "default_regret_us": float(T[:, DEFAULT].sum()) - best}
