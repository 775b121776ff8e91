"""Host side of the library, on the CPU: the C ABI's exports and error
codes, and its symbolic analysis against the oracle, bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def S():
    import paper_1705_06575_amd as S
    S.load_library()
    return S


def test_exports_match_header(S):
    hdr = open(os.path.join(ROOT, "include", "sym.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void)\s+(sym_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 20
    lib = S.load_library()
    for name in declared:
        assert hasattr(lib, name), name
    from paper_1705_06575_amd.binding import EXPORTS
    assert set(EXPORTS) == declared


def _check_symbolic(S, orc, w, perm):
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering=perm)
    Cp, Ci, _ = orc.permute(w.n, w.Ap, w.Ai, w.Ax, perm)
    Lp, Li, par = orc.symbolic_eq1(w.n, Cp, Ci)
    assert np.array_equal(an.get("perm"), np.asarray(perm, np.int32))
    assert np.array_equal(an.get("parent"), par)
    assert np.array_equal(an.get("colcount"), np.diff(Lp))
    assert np.array_equal(an.get("Lp"), Lp)
    assert np.array_equal(an.get("Li"), Li)
    sp = orc.supernodes(w.n, par, np.diff(Lp))
    assert np.array_equal(an.get("super"), sp)
    assert an.stat("nnzL") == Lp[-1]
    assert an.stat("flops") == float((np.diff(Lp).astype(float) ** 2).sum())
    return an, Lp, Li


def test_symbolic_matches_oracle_random(S, orc):
    rng = np.random.default_rng(17)
    for t in range(150):
        n = int(rng.integers(0, 70))
        w = W.random_spd(n, float(rng.choice([0.03, 0.1, 0.3, 0.6])), np.random.default_rng(3000 + t))
        _check_symbolic(S, orc, w, w.perm)


def test_symbolic_matches_bool_elim_config1(S, orc):
    w = W.config1()
    an, Lp, Li = _check_symbolic(S, orc, w, w.perm)
    Cp, Ci, _ = orc.permute(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    Lp1, Li1 = orc.bool_elim(w.n, Cp, Ci)
    assert np.array_equal(Lp1, Lp) and np.array_equal(Li1, Li)


@pytest.mark.parametrize("cfg", ["grid3d_7pt_16", "grid3d_27pt_12", "grid2d_9pt_40", "knn_small"])
def test_symbolic_matches_oracle_families(S, orc, cfg):
    if cfg == "grid3d_7pt_16":
        w = W.config2(16)
    elif cfg == "grid3d_27pt_12":
        w = W.config3(12)
    elif cfg == "grid2d_9pt_40":
        w = W.weighted_grid((40, 40), True, 1e-2, 1e2, "shift1e-3", np.random.default_rng(1), "g")
    else:
        w = W.knn_instance(0, nv=1500)
    _check_symbolic(S, orc, w, w.perm)


def test_own_ordering_is_valid_and_consistent(S, orc):
    """The library's own nested dissection: a permutation whose symbolic
    analysis agrees with the oracle's on the same permutation."""
    for w in [W.config1(), W.config2(12), W.knn_instance(1, nv=800),
              W.random_spd(60, 0.05, np.random.default_rng(2))]:
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd")
        p = an.get("perm")
        assert np.array_equal(np.sort(p), np.arange(w.n))
        an2, _, _ = _check_symbolic(S, orc, w, p)
        assert an2.stat("nnzL") == an.stat("nnzL")


def test_reach_matches_oracle_dfs(S, orc):
    w = W.config1()
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm)
    Cp, Ci, _ = orc.permute(w.n, w.Ap, w.Ai, w.Ax, w.perm)
    Lp, Li, _ = orc.symbolic_eq1(w.n, Cp, Ci)
    pinv = np.empty(w.n, np.int64)
    pinv[w.perm] = np.arange(w.n)
    rng = np.random.default_rng(8)
    for nb in (0, 1, 8, 100, w.n):
        pos = np.sort(rng.choice(w.n, size=nb, replace=False)).astype(np.int32)
        r = an.rhs_analyze(pos)
        ref = orc.reach(w.n, Lp, Li, np.sort(pinv[pos]).astype(np.int32))
        assert np.array_equal(r.reach(), ref)


def _lower(n, entries):
    entries = sorted(entries, key=lambda e: (e[1], e[0]))
    Ap = np.zeros(n + 1, np.int64)
    for i, j in entries:
        Ap[j + 1] += 1
    Ap = np.cumsum(Ap)
    Ai = np.array([i for i, j in entries], np.int32)
    return Ap, Ai


def test_error_codes(S):
    from paper_1705_06575_amd import SymError
    # entry above the diagonal
    Ap, Ai = _lower(3, [(0, 0), (1, 1), (2, 2)])
    Ai_bad = Ai.copy()
    Ai_bad[1] = 0                      # column 1 holds row 0 < 1
    with pytest.raises(SymError) as e:
        S.Analysis(3, Ap, Ai_bad)
    assert e.value.name == "SYM_EPATTERN"
    # row out of range
    Ai_bad = Ai.copy()
    Ai_bad[2] = 3
    with pytest.raises(SymError) as e:
        S.Analysis(3, Ap, Ai_bad)
    assert e.value.name == "SYM_EPATTERN"
    # duplicate entry
    Ap2 = np.array([0, 2, 3, 4], np.int64)
    Ai2 = np.array([1, 1, 1, 2], np.int32)
    with pytest.raises(SymError) as e:
        S.Analysis(3, Ap2, Ai2)
    assert e.value.name == "SYM_EPATTERN"
    # bad user permutation
    with pytest.raises(SymError) as e:
        S.Analysis(3, Ap, Ai, ordering=np.array([0, 0, 1], np.int32))
    assert e.value.name == "SYM_EINVAL"
    # bad block width
    with pytest.raises(SymError) as e:
        S.Analysis(3, Ap, Ai, block_width=24)
    assert e.value.name == "SYM_EINVAL"
    # negative n through the raw ABI
    lib = S.load_library()
    h = ctypes.c_void_p()
    assert lib.sym_analyze(-1, None, None, None, ctypes.byref(h)) == -1
    # unsorted rows and a missing diagonal are accepted
    Ap3 = np.array([0, 2, 3, 3], np.int64)
    Ai3 = np.array([2, 0, 2], np.int32)
    an = S.Analysis(3, Ap3, Ai3, ordering="natural")
    assert an.stat("nnzL") == 5


def test_state_errors_without_device(S):
    """Calls that need a bound workspace fail with SYM_ESTATE before any
    device work (no GPU needed)."""
    lib = S.load_library()
    w = W.config1()
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm)
    assert lib.sym_factor(an._h, ctypes.c_void_p(16), None) == -5
    assert lib.sym_solve(an._h, ctypes.c_void_p(16), None) == -5
    info = ctypes.c_int64()
    assert lib.sym_status(an._h, ctypes.byref(info)) == -5
    sz = ctypes.c_size_t()
    assert lib.sym_workspace(an._h, ctypes.byref(sz)) == 0 and sz.value > 0
    # misaligned workspace
    assert lib.sym_bind(an._h, ctypes.c_void_p(4096 + 8), sz, None) == -6
    assert lib.sym_bind(an._h, ctypes.c_void_p(4096), ctypes.c_size_t(sz.value - 1), None) == -6
    # a batch on an unbound analysis, or itself unbound, runs nothing
    b = ctypes.c_void_p()
    assert lib.sym_batch_create(an._h, 2, ctypes.byref(b)) == 0
    assert lib.sym_batch_workspace(b, ctypes.byref(sz)) == 0 and sz.value > 0
    assert lib.sym_batch_bind(b, ctypes.c_void_p(4096), sz, None) == -5
    p = ctypes.c_void_p(16)
    assert lib.sym_batch_factor(b, p, None) == -5
    assert lib.sym_batch_solve(b, p, None) == -5
    assert lib.sym_batch_refine(b, p, p, ctypes.c_void_p(32), 1, None) == -5
    eta = np.zeros(2)
    assert lib.sym_batch_eta(b, p, p, p, eta.ctypes.data_as(ctypes.c_void_p), None) == -5
    info2 = np.zeros(2, np.int64)
    assert lib.sym_batch_status(b, info2.ctypes.data_as(ctypes.c_void_p)) == -5
    lib.sym_batch_destroy(b)
    # refinement before a factorization
    it, e = ctypes.c_int32(), ctypes.c_double()
    assert lib.sym_refine(an._h, p, p, ctypes.c_void_p(32), 1e-12, 5, None,
                          ctypes.byref(it), ctypes.byref(e)) == -5


def test_static_solve_rejects_oversized_systems(S):
    """sym_solve_static's scratch holds n up to SYM_STATIC_MAX_N: larger
    systems are refused with SYM_EWORKSPACE before any device work."""
    lib = S.load_library()
    n = 524288 + 1
    Ap = np.arange(n + 1, dtype=np.int64)
    Ai = np.arange(n, dtype=np.int32)
    an = S.Analysis(n, Ap, Ai, ordering="natural")
    assert lib.sym_solve_static(an._h, ctypes.c_void_p(256), None) == -6
    assert lib.sym_solve_static(None, ctypes.c_void_p(256), None) == -1
    small = W.config1()
    an2 = S.Analysis(small.n, small.Ap, small.Ai, ordering=small.perm)
    assert lib.sym_solve_static(an2._h, ctypes.c_void_p(256), None) == -5


def test_empty_matrix(S):
    an = S.Analysis(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert an.stat("nnzL") == 0 and an.stat("nblocks") == 0


def test_block_structure(S, orc):
    """Device blocks tile each (fundamental, without amalgamation) supernode
    into pieces of at most B columns."""
    for B in (16, 32, 64):
        w = W.random_spd(150, 0.9, np.random.default_rng(4))
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, block_width=B, amalgamate=False)
        sp = an.get("super")
        bp = an.get("blocks")
        assert set(sp.tolist()) <= set(bp.tolist())
        assert (np.diff(bp) <= B).all() and bp[-1] == w.n
        lv = an.get("blevel")
        assert lv.max() + 1 == an.stat("nlevels")


def test_amalgamation_keeps_reported_structure(S, orc):
    """Relaxed amalgamation changes only the device panels: the reported
    fundamental supernodes and L pattern are unchanged, every device
    supernode boundary is a fundamental one, and the stored lower trapezoid
    covers nnz(L) plus explicit zeros."""
    for w in [W.config1(), W.config2(16), W.knn_instance(4, nv=1000)]:
        a0 = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, amalgamate=False)
        a1 = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, amalgamate=True)
        for k in ("parent", "colcount", "Lp", "Li", "super"):
            assert np.array_equal(a0.get(k), a1.get(k))
        assert set(a1.get("blocks").tolist()) <= set(a0.get("blocks").tolist()) | set(range(w.n + 1))
        assert a1.stat("ndsuper") <= a0.stat("ndsuper") == a0.stat("nsuper")
        assert a0.stat("stored_lower") == a0.stat("nnzL")
        assert a1.stat("stored_lower") >= a1.stat("nnzL")
        assert a1.stat("flops") == a0.stat("flops")


def test_kind_flops_partition_the_method_count(S):
    """The arithmetic attributed to the factor's launch kinds adds up to
    sum_j |L_j|^2 exactly (a check on the schedule covering every update)."""
    for w in [W.config1(), W.config2(20), W.random_spd(200, 1.0, np.random.default_rng(6)),
              W.knn_instance(3, nv=1200)]:
        for B in (16, 64):
            an = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd", block_width=B)
            kf = an.kind_flops()
            assert sum(kf.values()) == an.stat("flops")


def test_chain_launch_schedule(S):
    """With the per-level chain launch the analysis checks on the host that
    the launch's tasks, run one after another in their order, never wait
    (it fails with SYM_ESCHED otherwise); the schedule then has one launch
    per level where the step launches have one per step and kind, and the
    same method flop count."""
    for w in [W.config2(20), W.knn_instance(3, nv=2500), W.random_spd(300, 1.0, np.random.default_rng(4))]:
        for B in (16, 32, 64):
            a = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd", block_width=B)
            c = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd", block_width=B, chain_launch=True)
            assert c.stat("nphases") <= a.stat("nphases")
            assert c.stat("flops") == a.stat("flops")
            assert c.kind_flops() == a.kind_flops()


def test_update_depth_option(S):
    """update_depth groups the internal updates inside a supernode; the
    launch count and the method's flops do not depend on it, and values
    outside 0..16 are rejected."""
    w = W.config2(20)
    ref = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd", update_depth=1)
    for depth in (0, 2, 4, 16):
        a = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd", update_depth=depth)
        assert a.stat("nphases") == ref.stat("nphases")
        assert a.stat("flops") == ref.stat("flops")
    for bad in (-1, 17):
        with pytest.raises(RuntimeError):
            S.Analysis(w.n, w.Ap, w.Ai, ordering="nd", update_depth=bad)


def test_supernode_features(S):
    """The cost model's features: sizes match the device supernodes, the
    update flops (whole tile products, so at least the external-update
    share of the method count) cover that share, the flop fractions lie in
    [0, 1], and the level context is the level's sums of the supernodes'
    own features."""
    w = W.knn_instance(4, nv=1500)
    an = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd")
    f = an.get("super_feat").reshape(-1, 12)
    nds = int(an.stat("ndsuper"))
    assert f.shape[0] == nds
    assert f[:, 0].sum() == w.n and (f[:, 0] >= 1).all() and (f[:, 1] >= f[:, 0]).all()
    assert ((f[:, 5] >= 0) & (f[:, 5] <= f[:, 6]) & (f[:, 6] <= 1)).all()
    assert f[:, 4].sum() >= an.kind_flops()["external"] > 0
    for lv in np.unique(f[:, 7]):
        m = f[:, 7] == lv
        assert np.allclose(f[m, 8], f[m, 4].sum()) and (f[m, 9] == m.sum()).all()
        assert (f[m, 10] == f[m, 2].sum()).all()
        share = f[m, 4] / f[m, 4].sum() if f[m, 4].sum() > 0 else np.zeros(m.sum())
        assert np.allclose(f[m, 11], share)


class _Pat:
    """A pattern with dummy values, for the symbolic comparisons."""

    def __init__(self, name, n, Ap, Ai, perm):
        self.name, self.n, self.Ap, self.Ai, self.perm = name, n, Ap, Ai, perm
        self.Ax = np.ones(Ai.size)


@pytest.mark.slow
@pytest.mark.parametrize("cfg", ["grid3d_7pt_64_library_nd", "grid3d_27pt_80", "batch_9pt128",
                                 "batch_7pt24", "batch_7pt40"])
def test_symbolic_matches_oracle_full_size(S, orc, cfg):
    """The benchmark workloads' full patterns, bit for bit against O2 (Eq.
    (1) with explicit sets): elimination tree, column counts, L's pattern
    and the fundamental supernodes.  The 64^3 7-point grid in the library's
    own nested-dissection order (the benchmark's), the 80^3 27-point grid in
    its geometric order (the mixed-precision workload's), and the three
    batched patterns in their grid orders."""
    if cfg == "grid3d_7pt_64_library_nd":
        w = W.config2(64)
        perm = S.Analysis(w.n, w.Ap, w.Ai, ordering="nd").get("perm")
    elif cfg == "grid3d_27pt_80":
        w = W.config3(80)
        perm = w.perm
    else:
        n, Ap, Ai, _, perm = W.config4_batch(cfg.split("_")[1], 1)
        w = _Pat(cfg, n, Ap, Ai, perm)
    _check_symbolic(S, orc, w, perm)


def test_wide_supernodes_are_cut_into_pieces(S, orc):
    """Device supernodes wider than max_super_width are cut into pieces of
    consecutive columns: the reported (fundamental) structure is unchanged,
    every device block stays within one piece's width limit, and the
    schedule still covers the method's arithmetic exactly."""
    w = W.config2(16)
    base = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm)
    assert max(np.diff(base.get("blocks"))) == 64
    for mw in (1, 7, 40):
        an = S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, max_super_width=mw)
        for k in ("parent", "colcount", "Lp", "Li", "super"):
            assert np.array_equal(an.get(k), base.get(k))
        assert an.stat("ndsuper") > base.stat("ndsuper")
        assert max(np.diff(an.get("blocks"))) <= mw
        assert sum(an.kind_flops().values()) == an.stat("flops")
    with pytest.raises(Exception):
        S.Analysis(w.n, w.Ap, w.Ai, ordering=w.perm, max_super_width=16385)
