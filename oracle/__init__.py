"""CPU FP64 oracle for supernodal Cholesky and sparse triangular solve.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the library.  It shares no
code with the GPU library; the arithmetic lives in ``oracle.c`` (plain C,
compiled with gcc) and this module only marshals numpy arrays.

Functions and the passages of the Sympiler paper they follow:

- ``permute``            C = P A P^T, lower triangle (plumbing).
- ``bool_elim``          O1, elimination game on a dense boolean matrix;
                         the fill definition behind Eq. (1) and Section 3.2.
- ``symbolic_eq1``       O2, column patterns by Eq. (1); parent[j] =
                         min{i > j : L_ij != 0} (Section 3.2).
- ``etree_from_pattern`` Section 3.2's definition of the elimination tree.
- ``supernodes``         the fundamental-supernode rule stated after Eq. (1).
- ``chol_column``        O3, left-looking column Cholesky: update phase, then
                         column factorization (Section 3.2).
- ``fwd``, ``bwd``       O4, forward substitution (Section 1.1) and its
                         transpose.
- ``reach``              Reach_L(beta) by DFS on DG_L (Section 1.1, 3.1).
- ``fwd_pruned``         decoupled forward solve over the reach set only
                         (Section 1.1).
- ``llt_residual``, ``symv``, ``lmul``, ``ltmul``, ``eta_inf``: O5
                         invariants (normwise residuals and backward errors).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_bool_elim.restype = ctypes.c_int64
        L.orc_bool_elim.argtypes = [ctypes.c_int32, _i64p, _i32p, _i64p, _i32p, ctypes.c_int64]
        L.orc_symbolic_eq1.restype = ctypes.c_void_p
        L.orc_symbolic_eq1.argtypes = [ctypes.c_int32, _i64p, _i32p]
        L.orc_pattern_nnz.restype = ctypes.c_int64
        L.orc_pattern_nnz.argtypes = [ctypes.c_void_p]
        L.orc_pattern_copy.restype = None
        L.orc_pattern_copy.argtypes = [ctypes.c_void_p, _i64p, _i32p, _i32p]
        L.orc_pattern_free.restype = None
        L.orc_pattern_free.argtypes = [ctypes.c_void_p]
        L.orc_supernodes.restype = ctypes.c_int32
        L.orc_supernodes.argtypes = [ctypes.c_int32, _i32p, _i64p, _i32p]
        L.orc_chol_column.restype = ctypes.c_int64
        L.orc_chol_column.argtypes = [ctypes.c_int32, _i64p, _i32p, _f64p, _i64p, _i32p,
                                      _f64p, ctypes.POINTER(ctypes.c_double)]
        for name in ("orc_fwd", "orc_bwd"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [ctypes.c_int32, _i64p, _i32p, _f64p, _f64p]
        L.orc_reach.restype = ctypes.c_int64
        L.orc_reach.argtypes = [ctypes.c_int32, _i64p, _i32p, _i32p, ctypes.c_int64, _i32p]
        L.orc_fwd_pruned.restype = None
        L.orc_fwd_pruned.argtypes = [ctypes.c_int32, _i64p, _i32p, _f64p, _i32p,
                                     ctypes.c_int64, _f64p]
        L.orc_llt_residual.restype = ctypes.c_double
        L.orc_llt_residual.argtypes = [ctypes.c_int32, _i64p, _i32p, _f64p, _i64p, _i32p, _f64p]
        for name in ("orc_symv_lower", "orc_lmul", "orc_ltmul"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [ctypes.c_int32, _i64p, _i32p, _f64p, _f64p, _f64p]
        _lib = L
    return _lib


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# plumbing
# --------------------------------------------------------------------------

def permute(n, Ap, Ai, Ax, perm):
    """Lower triangle of C = P A P^T, where (P A P^T)[a, b] = A[perm[a], perm[b]].
    Returns (Cp, Ci, Cx) with rows sorted within each column."""
    Ap, Ai = _i64(Ap), _i32(Ai)
    perm = _i64(perm)
    pinv = np.empty(n, dtype=np.int64)
    pinv[perm] = np.arange(n)
    cols = np.repeat(np.arange(n, dtype=np.int64), np.diff(Ap))
    r = pinv[Ai.astype(np.int64)]
    c = pinv[cols]
    hi, lo = np.maximum(r, c), np.minimum(r, c)
    order = np.lexsort((hi, lo))
    Cp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(Cp, lo + 1, 1)
    Cp = np.cumsum(Cp)
    Cx = None if Ax is None else _f64(np.asarray(Ax)[order])
    return Cp, _i32(hi[order]), Cx


# --------------------------------------------------------------------------
# symbolic
# --------------------------------------------------------------------------

def bool_elim(n, Cp, Ci):
    """O1: L pattern by the elimination game.  Returns (Lp, Li)."""
    Cp, Ci = _i64(Cp), _i32(Ci)
    Lp = np.zeros(n + 1, dtype=np.int64)
    dummy = np.zeros(1, dtype=np.int32)
    nnz = lib().orc_bool_elim(n, Cp, Ci, Lp, dummy, 0)
    if nnz < 0:
        raise MemoryError("bool_elim")
    Li = np.zeros(max(nnz, 1), dtype=np.int32)
    lib().orc_bool_elim(n, Cp, Ci, Lp, Li, nnz)
    return Lp, Li[:nnz]


def symbolic_eq1(n, Cp, Ci):
    """O2: column patterns of L by Eq. (1).  Returns (Lp, Li, parent)."""
    Cp, Ci = _i64(Cp), _i32(Ci)
    h = lib().orc_symbolic_eq1(n, Cp, Ci)
    if not h:
        raise MemoryError("symbolic_eq1")
    try:
        nnz = lib().orc_pattern_nnz(h)
        Lp = np.zeros(n + 1, dtype=np.int64)
        Li = np.zeros(max(nnz, 1), dtype=np.int32)
        parent = np.zeros(max(n, 1), dtype=np.int32)
        lib().orc_pattern_copy(h, Lp, Li, parent)
    finally:
        lib().orc_pattern_free(h)
    return Lp, Li[:nnz], parent[:n]


def etree_from_pattern(n, Lp, Li):
    """parent[j] = min{i > j : L_ij != 0}, or -1 (Section 3.2)."""
    parent = np.full(n, -1, dtype=np.int32)
    for j in range(n):
        below = Li[Lp[j]:Lp[j + 1]]
        below = below[below > j]
        if below.size:
            parent[j] = below.min()
    return parent


def colcounts(Lp):
    return np.diff(_i64(Lp))


def supernodes(n, parent, colcount):
    """Fundamental supernodes; returns super_ptr (first column of each
    supernode, then n)."""
    sp = np.zeros(n + 1, dtype=np.int32)
    ns = lib().orc_supernodes(n, _i32(parent), _i64(colcount), sp)
    if ns < 0:
        raise MemoryError("supernodes")
    return sp[:ns + 1]


def reach(n, Lp, Li, beta):
    """Reach_L(beta) in DG_L, returned in increasing column order."""
    out = np.zeros(max(n, 1), dtype=np.int32)
    beta = _i32(beta)
    cnt = lib().orc_reach(n, _i64(Lp), _i32(Li), beta, beta.size, out)
    if cnt < 0:
        raise MemoryError("reach")
    return out[:cnt]


# --------------------------------------------------------------------------
# numeric
# --------------------------------------------------------------------------

def chol_column(n, Cp, Ci, Cx, Lp, Li):
    """O3: returns (Lx, info, flops); info = 0 or 1 + first failing column
    (permuted numbering)."""
    Lp, Li = _i64(Lp), _i32(Li)
    Lx = np.zeros(max(int(Lp[-1]), 1), dtype=np.float64)
    fl = ctypes.c_double(0.0)
    info = lib().orc_chol_column(n, _i64(Cp), _i32(Ci), _f64(Cx), Lp, Li, Lx, ctypes.byref(fl))
    if info < 0:
        raise MemoryError("chol_column")
    return Lx[:int(Lp[-1])], int(info), fl.value


def fwd(n, Lp, Li, Lx, b):
    x = _f64(b).copy()
    lib().orc_fwd(n, _i64(Lp), _i32(Li), _f64(Lx), x)
    return x


def bwd(n, Lp, Li, Lx, b):
    x = _f64(b).copy()
    lib().orc_bwd(n, _i64(Lp), _i32(Li), _f64(Lx), x)
    return x


def fwd_pruned(n, Lp, Li, Lx, cols, b):
    x = _f64(b).copy()
    cols = _i32(cols)
    lib().orc_fwd_pruned(n, _i64(Lp), _i32(Li), _f64(Lx), cols, cols.size, x)
    return x


def solve(n, perm, Lp, Li, Lx, b):
    """Full solve of A x = b with P A P^T = L L^T: x = P^T L^-T L^-1 P b."""
    perm = _i64(perm)
    y = _f64(b)[perm]
    y = bwd(n, Lp, Li, Lx, fwd(n, Lp, Li, Lx, y))
    x = np.empty(n)
    x[perm] = y
    return x


def llt_residual(n, Cp, Ci, Cx, Lp, Li, Lx):
    """||L L^T - C||_F / ||C||_F."""
    r = lib().orc_llt_residual(n, _i64(Cp), _i32(Ci), _f64(Cx), _i64(Lp), _i32(Li), _f64(Lx))
    if r == -1.0:
        raise MemoryError("llt_residual")
    if r == -2.0:
        raise ValueError("C has an entry outside L's pattern")
    return r


def symv(n, Cp, Ci, Cx, x):
    y = np.zeros(n)
    lib().orc_symv_lower(n, _i64(Cp), _i32(Ci), _f64(Cx), _f64(x), y)
    return y


def lmul(n, Lp, Li, Lx, x):
    y = np.zeros(n)
    lib().orc_lmul(n, _i64(Lp), _i32(Li), _f64(Lx), _f64(x), y)
    return y


def ltmul(n, Lp, Li, Lx, x):
    y = np.zeros(n)
    lib().orc_ltmul(n, _i64(Lp), _i32(Li), _f64(Lx), _f64(x), y)
    return y


def eta_inf(n, Ap, Ai, Ax, x, b):
    """Normwise backward error ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)."""
    r = _f64(b) - symv(n, Ap, Ai, Ax, x)
    rowabs = symv(n, Ap, Ai, np.abs(_f64(Ax)), np.ones(n))
    den = rowabs.max(initial=0.0) * np.abs(x).max(initial=0.0) + np.abs(b).max(initial=0.0)
    return float(np.abs(r).max(initial=0.0) / den) if den > 0 else float(np.abs(r).max(initial=0.0))


def factor(n, Ap, Ai, Ax, perm):
    """Convenience: permute, Eq. (1) symbolic, column Cholesky.
    Returns a dict with the permuted matrix, pattern, values and flops."""
    Cp, Ci, Cx = permute(n, Ap, Ai, Ax, perm)
    Lp, Li, parent = symbolic_eq1(n, Cp, Ci)
    Lx, info, flops = chol_column(n, Cp, Ci, Cx, Lp, Li)
    return dict(Cp=Cp, Ci=Ci, Cx=Cx, Lp=Lp, Li=Li, Lx=Lx, parent=parent,
                info=info, flops=flops)
