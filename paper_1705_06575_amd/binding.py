"""ctypes binding for libsym.so (names follow include/sym.h).

Device buffers are torch tensors on the current CUDA (HIP) device; the
stream is torch's current stream.  The library allocates no device memory:
the handle's workspace is a torch uint8 tensor kept alive by the Python
object.  If the library is missing this module raises; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsym.so")

SYM_ORDER_ND, SYM_ORDER_NATURAL, SYM_ORDER_USER = 0, 1, 2
SYM_F64, SYM_F32, SYM_BF16, SYM_F16 = 0, 1, 2, 3
PRECISIONS = {"f64": SYM_F64, "f32": SYM_F32, "bf16": SYM_BF16, "f16": SYM_F16}

_ERRORS = {
    -1: "SYM_EINVAL", -2: "SYM_EPATTERN", -3: "SYM_ENOMEM", -4: "SYM_EHIP",
    -5: "SYM_ESTATE", -6: "SYM_EWORKSPACE", -7: "SYM_ESCHED", -8: "SYM_ENUMERIC",
}

GET = dict(perm=1, parent=2, colcount=3, Lp=4, Li=5, super=6, sparent=7, blocks=8, blevel=9,
           super_feat=10, task_super=11, variant=12)
GET_DTYPE = dict(perm=np.int32, parent=np.int32, colcount=np.int64, Lp=np.int64, Li=np.int32,
                 super=np.int32, sparent=np.int32, blocks=np.int32, blevel=np.int32,
                 super_feat=np.float64, task_super=np.int32, variant=np.uint8)
STAT = dict(n=1, nnzA=2, nnzL=3, flops=4, nsuper=5, nblocks=6, nlevels=7, npairs=8,
            panel_entries=9, analyze_ms=10, sum_rows=11, nphases=12, nincidences=13,
            nslevels=14, ndsuper=15, stored_lower=16, ext_operand_entries=17, walkers=18)


class SymError(RuntimeError):
    def __init__(self, call, code):
        super().__init__(f"{call} failed: {_ERRORS.get(code, code)}")
        self.code = code
        self.name = _ERRORS.get(code, str(code))


class sym_opts(ctypes.Structure):
    _fields_ = [("ordering", ctypes.c_int32),
                ("perm", ctypes.POINTER(ctypes.c_int32)),
                ("block_width", ctypes.c_int32),
                ("precision", ctypes.c_int32),
                ("nd_leaf", ctypes.c_int32),
                ("amalgamate", ctypes.c_int32),
                ("pivot_floor_exp", ctypes.c_int32),
                ("max_super_width", ctypes.c_int32),
                ("split_share", ctypes.c_int32),
                ("chain_launch", ctypes.c_int32),
                ("update_depth", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


EXPORTS = ["sym_opts_default", "sym_analyze", "sym_workspace", "sym_bind", "sym_factor",
           "sym_solve", "sym_solve_static", "sym_solve_lower", "sym_solve_upper", "sym_rhs_analyze",
           "sym_rhs_workspace", "sym_rhs_bind", "sym_solve_lower_sparse", "sym_solve_sparse", "sym_status",
           "sym_export_factor", "sym_pivots_perturbed", "sym_get_size", "sym_get", "sym_rhs_get", "sym_stat",
           "sym_profile", "sym_profile_read", "sym_refine", "sym_refine_pcg", "sym_destroy",
           "sym_rhs_destroy", "sym_batch_create", "sym_batch_workspace", "sym_batch_bind",
           "sym_batch_factor", "sym_batch_solve", "sym_batch_refine", "sym_batch_eta",
           "sym_batch_status", "sym_batch_destroy", "sym_set_variants", "sym_task_times", "sym_mlp_param_count", "sym_mlp_work_size", "sym_mlp_forward",
           "sym_mlp_backward", "sym_mlp_adam"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsym.so; raises OSError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it with paper_1705_06575_amd/build.py")
    # the library runs on PyTorch's HIP runtime: PyTorch is loaded first, so
    # that the library's HIP dependency resolves to the runtime already in
    # the process (loaded the other way round, the process holds a second
    # runtime, which sees no device)
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    L.sym_opts_default.restype = None
    L.sym_opts_default.argtypes = [ctypes.POINTER(sym_opts)]
    L.sym_analyze.argtypes = [i64, vp, vp, ctypes.POINTER(sym_opts), ctypes.POINTER(vp)]
    L.sym_workspace.argtypes = [vp, ctypes.POINTER(sz)]
    L.sym_bind.argtypes = [vp, vp, sz, vp]
    L.sym_factor.argtypes = [vp, vp, vp]
    L.sym_solve.argtypes = [vp, vp, vp]
    L.sym_solve_static.argtypes = [vp, vp, vp]
    L.sym_solve_lower.argtypes = [vp, vp, vp, vp]
    L.sym_solve_upper.argtypes = [vp, vp, vp]
    L.sym_rhs_analyze.argtypes = [vp, i64, vp, ctypes.POINTER(vp)]
    L.sym_rhs_workspace.argtypes = [vp, ctypes.POINTER(sz)]
    L.sym_rhs_bind.argtypes = [vp, vp, sz, vp]
    L.sym_solve_lower_sparse.argtypes = [vp, vp, vp, vp, vp]
    L.sym_solve_sparse.argtypes = [vp, vp, vp, vp, vp]
    L.sym_status.argtypes = [vp, ctypes.POINTER(i64)]
    L.sym_export_factor.argtypes = [vp, vp, vp]
    L.sym_pivots_perturbed.argtypes = [vp, ctypes.POINTER(i64)]
    L.sym_get_size.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i64)]
    L.sym_get.argtypes = [vp, ctypes.c_int, vp]
    L.sym_rhs_get.argtypes = [vp, ctypes.POINTER(i64), vp]
    L.sym_stat.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.sym_refine.argtypes = [vp, vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp,
                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    L.sym_refine_pcg.argtypes = L.sym_refine.argtypes
    L.sym_profile.argtypes = [vp, ctypes.c_int]
    L.sym_profile_read.argtypes = [vp, vp, vp, vp]
    L.sym_destroy.restype = None
    L.sym_destroy.argtypes = [vp]
    L.sym_rhs_destroy.restype = None
    L.sym_rhs_destroy.argtypes = [vp]
    L.sym_batch_create.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(vp)]
    L.sym_batch_workspace.argtypes = [vp, ctypes.POINTER(sz)]
    L.sym_batch_bind.argtypes = [vp, vp, sz, vp]
    L.sym_batch_factor.argtypes = [vp, vp, vp]
    L.sym_batch_solve.argtypes = [vp, vp, vp]
    L.sym_batch_refine.argtypes = [vp, vp, vp, vp, ctypes.c_int32, vp]
    L.sym_batch_eta.argtypes = [vp, vp, vp, vp, vp, vp]
    L.sym_batch_status.argtypes = [vp, vp]
    L.sym_mlp_param_count.argtypes = [ctypes.c_int32, ctypes.POINTER(i64)]
    L.sym_mlp_work_size.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(i64)]
    L.sym_mlp_forward.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, vp, vp]
    L.sym_mlp_backward.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    L.sym_mlp_adam.argtypes = [vp, vp, vp, vp, i64, ctypes.c_int32, ctypes.c_float, vp]
    L.sym_set_variants.argtypes = [vp, vp, ctypes.c_int32]
    L.sym_task_times.argtypes = [vp, vp]
    L.sym_batch_destroy.restype = None
    L.sym_batch_destroy.argtypes = [vp]
    no_ret = ("sym_opts_default", "sym_destroy", "sym_rhs_destroy", "sym_batch_destroy")
    for name in EXPORTS:
        f = getattr(L, name)
        if f.restype is not None and name not in no_ret:
            f.restype = ctypes.c_int
    _lib = L
    return L


def _check(call, rc):
    if rc != 0:
        raise SymError(call, rc)


def mlp_work_size(n: int, d_in: int) -> int:
    """Floats of scratch sym_mlp_backward needs for n samples of d_in inputs."""
    L = load_library()
    out = ctypes.c_int64()
    _check("sym_mlp_work_size", L.sym_mlp_work_size(int(n), int(d_in), ctypes.byref(out)))
    return out.value


def opts_default() -> sym_opts:
    o = sym_opts()
    load_library().sym_opts_default(ctypes.byref(o))
    return o


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype_name: str, numel: int | None = None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if str(t.dtype) != dtype_name:
        raise TypeError(f"expected {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Analysis:
    """Symbolic analysis of one sparsity pattern (host), plus its device
    workspace once bound.

    Ap: int64[n+1], Ai: int32[nnz] -- lower triangle of A in CSC, 0-based.
    ordering: "nd" (the library's graph nested dissection), "natural", or
    an int32 permutation array perm[new] = old.
    """

    def __init__(self, n, Ap, Ai, ordering="nd", block_width=64, precision="f64", nd_leaf=24,
                 amalgamate=True, pivot_floor_exp=0, max_super_width=0, split_share=0,
                 chain_launch=False, update_depth=0):
        L = load_library()
        self._lib = L
        self.n = int(n)
        Ap = np.ascontiguousarray(Ap, dtype=np.int64)
        Ai = np.ascontiguousarray(Ai, dtype=np.int32)
        if Ap.size != self.n + 1:
            raise ValueError("Ap must have n+1 entries")
        o = opts_default()
        self._perm_keep = None
        if isinstance(ordering, str):
            o.ordering = {"nd": SYM_ORDER_ND, "natural": SYM_ORDER_NATURAL}[ordering]
        else:
            p = np.ascontiguousarray(ordering, dtype=np.int32)
            if p.size != self.n:
                raise ValueError("perm must have n entries")
            self._perm_keep = p
            o.ordering = SYM_ORDER_USER
            o.perm = p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        o.block_width = int(block_width)
        o.precision = PRECISIONS[precision]
        o.pivot_floor_exp = int(pivot_floor_exp)
        o.max_super_width = int(max_super_width)
        o.split_share = int(split_share)
        o.chain_launch = int(bool(chain_launch))
        o.update_depth = int(update_depth)
        o.nd_leaf = int(nd_leaf)
        o.amalgamate = int(bool(amalgamate))
        self.precision = precision
        h = ctypes.c_void_p()
        _check("sym_analyze", L.sym_analyze(self.n, _ptr(Ap), _ptr(Ai), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.nnzA = int(Ap[-1])
        self._ws = None
        self._factored = False

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.sym_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- symbolic outputs
    def get(self, what: str) -> np.ndarray:
        cnt = ctypes.c_int64()
        _check("sym_get_size", self._lib.sym_get_size(self._h, GET[what], ctypes.byref(cnt)))
        out = np.zeros(max(cnt.value, 1), dtype=GET_DTYPE[what])
        _check("sym_get", self._lib.sym_get(self._h, GET[what], _ptr(out)))
        return out[:cnt.value]

    def stat(self, what: str) -> float:
        v = ctypes.c_double()
        _check("sym_stat", self._lib.sym_stat(self._h, STAT[what], ctypes.byref(v)))
        return v.value

    def set_variants(self, variant):
        """Per-device-supernode kernel variants (0..3); the analysis is
        unbound afterwards and binds again on its next device call."""
        v = np.ascontiguousarray(variant, dtype=np.uint8)
        _check("sym_set_variants", self._lib.sym_set_variants(self._h, _ptr(v), int(v.size)))
        self._ws = None
        self._factored = False

    def task_times(self) -> np.ndarray:
        """Workgroup duration (us) of every factor task of the last profiled
        factorization (external-update tasks; others 0)."""
        out = np.zeros(max(int(self.get_size("task_super")), 1))
        _check("sym_task_times", self._lib.sym_task_times(self._h, _ptr(out)))
        return out[:int(self.get_size("task_super"))]

    def get_size(self, what: str) -> int:
        cnt = ctypes.c_int64()
        _check("sym_get_size", self._lib.sym_get_size(self._h, GET[what], ctypes.byref(cnt)))
        return cnt.value

    @property
    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check("sym_workspace", self._lib.sym_workspace(self._h, ctypes.byref(b)))
        return b.value

    # -- device
    def bind(self, device=None):
        import torch
        nbytes = max(self.workspace_bytes, 256)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8,
                               device=device if device is not None else "cuda")
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        _check("sym_bind", self._lib.sym_bind(self._h, ctypes.c_void_p(aligned),
                                              ctypes.c_size_t(nbytes + 256 - (aligned - base)),
                                              _stream()))
        return self

    def factor(self, Ax):
        if self._ws is None:
            self.bind(Ax.device)
        _check("sym_factor", self._lib.sym_factor(self._h, _dev_ptr(Ax, "torch.float64", self.nnzA),
                                                  _stream()))
        self._factored = True
        return self

    def status(self) -> int:
        info = ctypes.c_int64()
        _check("sym_status", self._lib.sym_status(self._h, ctypes.byref(info)))
        return info.value

    def pivots_perturbed(self) -> int:
        """Pivots the last factorization replaced by their floor."""
        c = ctypes.c_int64()
        _check("sym_pivots_perturbed", self._lib.sym_pivots_perturbed(self._h, ctypes.byref(c)))
        return c.value

    def solve(self, b):
        """x = A^-1 b (b is not modified; returns a new tensor)."""
        x = b.clone()
        _check("sym_solve", self._lib.sym_solve(self._h, _dev_ptr(x, "torch.float64", self.n), _stream()))
        return x

    def solve_(self, bx):
        _check("sym_solve", self._lib.sym_solve(self._h, _dev_ptr(bx, "torch.float64", self.n), _stream()))
        return bx

    def solve_static_(self, bx):
        """In place, as solve_, through sym_solve_static (the sweeps' scratch in
        the library's static device array; nothing is allocated)."""
        _check("sym_solve_static", self._lib.sym_solve_static(
            self._h, _dev_ptr(bx, "torch.float64", self.n), _stream()))
        return bx

    def refine(self, Ax, b, tol=1e-12, maxit=20, out=None, method="ir"):
        """x solving A x = b by the current factor plus FP64 iterative
        refinement on the device: method "ir" (classical, sym_refine) or
        "pcg" (conjugate-gradient accelerated, sym_refine_pcg).  Returns
        (x, iterations, eta_inf)."""
        import torch
        if method not in ("ir", "pcg"):
            raise ValueError(f"method {method!r}: 'ir' or 'pcg'")
        name = "sym_refine" if method == "ir" else "sym_refine_pcg"
        x = out if out is not None else torch.empty_like(b)
        it = ctypes.c_int32()
        eta = ctypes.c_double()
        _check(name, getattr(self._lib, name)(
            self._h, _dev_ptr(Ax, "torch.float64", self.nnzA), _dev_ptr(b, "torch.float64", self.n),
            _dev_ptr(x, "torch.float64", self.n), float(tol), int(maxit), _stream(),
            ctypes.byref(it), ctypes.byref(eta)))
        return x, it.value, eta.value

    def solve_lower(self, b, out=None):
        """y = L^-1 P b, returned in L's (permuted) ordering."""
        import torch
        y = out if out is not None else torch.empty_like(b)
        _check("sym_solve_lower", self._lib.sym_solve_lower(
            self._h, _dev_ptr(b, "torch.float64", self.n), _dev_ptr(y, "torch.float64", self.n), _stream()))
        return y

    def solve_upper_(self, y):
        """In place: y <- L^-T y (permuted ordering)."""
        _check("sym_solve_upper", self._lib.sym_solve_upper(self._h, _dev_ptr(y, "torch.float64", self.n),
                                                            _stream()))
        return y

    def rhs_analyze(self, bi) -> "RhsPlan":
        return RhsPlan(self, bi)

    def solve_lower_sparse(self, r: "RhsPlan", bv, out=None):
        import torch
        y = out if out is not None else torch.empty(self.n, dtype=torch.float64, device=bv.device)
        if r._ws is None:
            r.bind(bv.device)
        _check("sym_solve_lower_sparse", self._lib.sym_solve_lower_sparse(
            self._h, r._r, _dev_ptr(bv, "torch.float64", r.nb), _dev_ptr(y, "torch.float64", self.n), _stream()))
        return y

    def solve_sparse(self, r: "RhsPlan", bv, out=None):
        """x = A^-1 b for the sparse b (values bv at r's positions), original
        ordering: reach-pruned forward sweep, full backward sweep."""
        import torch
        x = out if out is not None else torch.empty(self.n, dtype=torch.float64, device=bv.device)
        if r._ws is None:
            r.bind(bv.device)
        _check("sym_solve_sparse", self._lib.sym_solve_sparse(
            self._h, r._r, _dev_ptr(bv, "torch.float64", r.nb), _dev_ptr(x, "torch.float64", self.n), _stream()))
        return x

    PROFILE_KINDS = ("scatter", "external", "trsm", "internal")

    def profile(self, enable: bool = True):
        _check("sym_profile", self._lib.sym_profile(self._h, int(enable)))
        return self

    def profile_read(self):
        """Per launch kind of the last factorization: (ms, launches,
        algorithmic flops) dicts keyed by PROFILE_KINDS."""
        k = len(self.PROFILE_KINDS)
        ms = np.zeros(k)
        n = np.zeros(k, np.int64)
        fl = np.zeros(k)
        _check("sym_profile_read", self._lib.sym_profile_read(self._h, _ptr(ms), _ptr(n), _ptr(fl)))
        return ({a: float(ms[i]) for i, a in enumerate(self.PROFILE_KINDS)},
                {a: int(n[i]) for i, a in enumerate(self.PROFILE_KINDS)},
                {a: float(fl[i]) for i, a in enumerate(self.PROFILE_KINDS)})

    def kind_flops(self):
        """Algorithmic flops per launch kind (host-side, no GPU needed)."""
        k = len(self.PROFILE_KINDS)
        ms = np.zeros(k)
        n = np.zeros(k, np.int64)
        fl = np.zeros(k)
        self._lib.sym_profile_read(self._h, _ptr(ms), _ptr(n), _ptr(fl))
        return {a: float(fl[i]) for i, a in enumerate(self.PROFILE_KINDS)}

    def export_factor(self) -> np.ndarray:
        """Host copy of L's values in the CSC pattern of get('Lp'), get('Li')."""
        nnzL = int(self.stat("nnzL"))
        Lx = np.zeros(max(nnzL, 1))
        _check("sym_export_factor", self._lib.sym_export_factor(self._h, _ptr(Lx), _stream()))
        return Lx[:nnzL]


class RhsPlan:
    """Reach set of one right-hand-side pattern (host) and its device copy."""

    def __init__(self, an: Analysis, bi):
        self._an = an
        self._lib = an._lib
        bi = np.ascontiguousarray(bi, dtype=np.int32)
        self.nb = int(bi.size)
        r = ctypes.c_void_p()
        _check("sym_rhs_analyze", self._lib.sym_rhs_analyze(an._h, self.nb, _ptr(bi), ctypes.byref(r)))
        self._r = r
        self._ws = None

    def reach(self) -> np.ndarray:
        cnt = ctypes.c_int64()
        _check("sym_rhs_get", self._lib.sym_rhs_get(self._r, ctypes.byref(cnt), None))
        out = np.zeros(max(cnt.value, 1), dtype=np.int32)
        _check("sym_rhs_get", self._lib.sym_rhs_get(self._r, ctypes.byref(cnt), _ptr(out)))
        return out[:cnt.value]

    def bind(self, device=None):
        import torch
        b = ctypes.c_size_t()
        _check("sym_rhs_workspace", self._lib.sym_rhs_workspace(self._r, ctypes.byref(b)))
        self._ws = torch.empty(b.value + 256, dtype=torch.uint8,
                               device=device if device is not None else "cuda")
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        _check("sym_rhs_bind", self._lib.sym_rhs_bind(self._r, ctypes.c_void_p(aligned),
                                                      ctypes.c_size_t(b.value + 256 - (aligned - base)),
                                                      _stream()))
        return self

    def close(self):
        if getattr(self, "_r", None) is not None and self._r.value:
            self._lib.sym_rhs_destroy(self._r)
            self._r = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """m value sets on the pattern of one bound Analysis, factored and
    solved together (one launch per schedule step for all of them).
    Values: float64 tensors of shape (m, nnz(A)); right-hand sides and
    solutions (m, n).  Every call is asynchronous and allocation-free
    except eta() and status(), so a sequence can be captured in a graph."""

    def __init__(self, an: Analysis, m: int, device=None):
        import torch
        if an._ws is None:
            an.bind(device)
        self._an = an
        self._lib = an._lib
        self.m = int(m)
        b = ctypes.c_void_p()
        _check("sym_batch_create", self._lib.sym_batch_create(an._h, self.m, ctypes.byref(b)))
        self._b = b
        nb = ctypes.c_size_t()
        _check("sym_batch_workspace", self._lib.sym_batch_workspace(b, ctypes.byref(nb)))
        self._ws = torch.empty(nb.value + 256, dtype=torch.uint8,
                               device=device if device is not None else an._ws.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        _check("sym_batch_bind", self._lib.sym_batch_bind(
            b, ctypes.c_void_p(aligned), ctypes.c_size_t(nb.value + 256 - (aligned - base)),
            _stream()))

    def factor(self, Ax):
        _check("sym_batch_factor", self._lib.sym_batch_factor(
            self._b, _dev_ptr(Ax, "torch.float64", self.m * self._an.nnzA), _stream()))
        return self

    def solve_(self, B):
        """In place: row i of B becomes A_i^-1 B_i."""
        _check("sym_batch_solve", self._lib.sym_batch_solve(
            self._b, _dev_ptr(B, "torch.float64", self.m * self._an.n), _stream()))
        return B

    def refine(self, Ax, B, X, steps: int):
        """X_i = solve(B_i) plus `steps` FP64 refinement steps (no host sync)."""
        n = self.m * self._an.n
        _check("sym_batch_refine", self._lib.sym_batch_refine(
            self._b, _dev_ptr(Ax, "torch.float64", self.m * self._an.nnzA),
            _dev_ptr(B, "torch.float64", n), _dev_ptr(X, "torch.float64", n), int(steps),
            _stream()))
        return X

    def eta(self, Ax, B, X) -> np.ndarray:
        """Normwise backward error of every instance (synchronizes)."""
        n = self.m * self._an.n
        out = np.zeros(self.m)
        _check("sym_batch_eta", self._lib.sym_batch_eta(
            self._b, _dev_ptr(Ax, "torch.float64", self.m * self._an.nnzA),
            _dev_ptr(B, "torch.float64", n), _dev_ptr(X, "torch.float64", n), _ptr(out),
            _stream()))
        return out

    def status(self) -> np.ndarray:
        out = np.zeros(self.m, dtype=np.int64)
        _check("sym_batch_status", self._lib.sym_batch_status(self._b, _ptr(out)))
        return out

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self._lib.sym_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
