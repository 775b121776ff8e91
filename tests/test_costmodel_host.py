"""Host logic of the learned variant choice (no device needed): the margin
rule of `choose` and the leave-one-pattern-out margin selection, with
stand-in models whose predictions are fixed by the features."""
import numpy as np
import pytest

from paper_1705_06575_amd import costmodel as cm


class _Fixed(cm._Chooser):
    """Predicts log(T_0/T_1) = -log1p(f0), log(T_2/T_1) = -log1p(f1) and
    log(T_3/T_1) = 1 (variant 3 always slower)."""

    def __init__(self, margin=0.02):
        self.margin = margin

    def predict(self, X):
        X = np.asarray(X)
        return np.where(X[:, cm.NFEAT] == 1.0, -X[:, 0],
                        np.where(X[:, cm.NFEAT + 3] == 1.0, 1.0, -X[:, 1]))


def _feat(gain0, gain2, work=1e9):
    f = np.zeros((len(gain0), cm.NFEAT))
    f[:, 0] = np.expm1(gain0)
    f[:, 1] = np.expm1(gain2)
    f[:, 4] = work
    return f


def test_choose_applies_margin_and_work_floor():
    f = _feat([0.10, 0.00, 0.010, -0.3], [-0.05, 0.30, 0.015, -0.2])
    m = _Fixed()
    # gains 0.10 (v0), 0.30 (v2), 0.015 (< margin), none
    assert m.choose(f).tolist() == [0, 2, 1, 1]
    assert m.choose(f, margin=0.2).tolist() == [1, 2, 1, 1]
    assert m.choose(f, margin=float("inf")).tolist() == [1, 1, 1, 1]
    f[1, 4] = 10.0
    assert m.choose(f, min_work=100.0).tolist() == [0, 1, 1, 1]


@pytest.fixture
def fixed_fit(monkeypatch):
    monkeypatch.setattr(cm, "_fit", lambda measured, min_us, epochs, seed: (_Fixed(), 0.0, [0.0], 0))


def test_select_margin_keeps_default_when_predicted_gains_are_losses(fixed_fit):
    f = _feat([0.05] * 6, [-1.0] * 6)
    T = np.column_stack([np.full(6, 2.0), np.ones(6), np.full(6, 5.0), np.full(6, 9.0)])
    assert cm.select_margin([(f, T), (f, T)]) == float("inf")


def test_select_margin_takes_real_gains(fixed_fit):
    f = _feat([0.3] * 6, [-1.0] * 6)
    T = np.column_stack([np.full(6, 0.5), np.ones(6), np.full(6, 5.0), np.full(6, 9.0)])
    assert cm.select_margin([(f, T), (f, T)]) == cm.MARGINS[0]


def test_select_margin_separates_real_from_false_gains(fixed_fit):
    # predicted gains 0.07 are real, predicted gains 0.03 are losses:
    # only a margin between them pays best
    f = _feat([0.07] * 4 + [0.03] * 4, [-1.0] * 8)
    T = np.column_stack([[0.5] * 4 + [3.0] * 4, np.ones(8), np.full(8, 5.0), np.full(8, 9.0)])
    assert cm.select_margin([(f, T), (f, T)]) == 0.05


def test_encode_layout():
    f = np.arange(1, 2 * cm.NFEAT + 1, dtype=np.float64).reshape(2, cm.NFEAT)
    f[:, 5:7] = 0.25
    f[:, 11] = 0.5
    X = cm.encode(f, np.array([0, 3]))
    assert X.shape == (2, cm.D_IN)
    assert np.allclose(X[:, 0:5], np.log1p(f[:, 0:5])) and np.allclose(X[:, 7:11], np.log1p(f[:, 7:11]))
    assert (X[:, 5:7] == 0.25).all() and (X[:, 11] == 0.5).all()
    assert X[0, cm.NFEAT:].tolist() == [1, 0, 0, 0] and X[1, cm.NFEAT:].tolist() == [0, 0, 0, 1]
