"""Seeded synthetic SPD workloads for supernodal Cholesky and triangular solve.

This module only builds inputs: sparsity patterns, values, right-hand sides
and a geometric nested-dissection ordering for each pattern.  It holds none
of the factorization's arithmetic, and both the oracle tests and the GPU
library's tests and benchmark draw their inputs from here.

Every matrix is returned as the lower triangle (i >= j) of a symmetric matrix
in compressed sparse column form with 0-based indices: ``Ap`` int64[n+1],
``Ai`` int32[nnz] (rows sorted within each column) and ``Ax`` float64[nnz].
Orderings follow the convention ``perm[new] = old``.

The paper measures on SuiteSparse SPD matrices (Section 4, the matrix-set
table); those are not available here, and the stencil and k-NN families
below stand in for them with sizes that bracket that table's range.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED_BASE = 20260000        # config i draws from PCG64(SEED_BASE + i)
SEED_INSTANCE = 20261000    # instance k of a batch / k-NN family


def rng_for(config: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + config))


def rng_for_instance(k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_INSTANCE + k))


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    Ap: np.ndarray          # int64[n+1]
    Ai: np.ndarray          # int32[nnz]
    Ax: np.ndarray          # float64[nnz]
    perm: np.ndarray        # int32[n], geometric nested dissection, perm[new] = old
    shape: tuple = ()       # grid shape, when the pattern is a grid

    @property
    def nnz(self) -> int:
        return int(self.Ap[-1])


# --------------------------------------------------------------------------
# assembly helpers (pattern plumbing only)
# --------------------------------------------------------------------------

def _lower_csc(n: int, ei: np.ndarray, ej: np.ndarray, ev: np.ndarray,
               diag: np.ndarray):
    """Lower CSC from off-diagonal edges (ei > ej) plus a diagonal."""
    rows = np.concatenate([np.arange(n, dtype=np.int64), ei.astype(np.int64)])
    cols = np.concatenate([np.arange(n, dtype=np.int64), ej.astype(np.int64)])
    vals = np.concatenate([diag, ev])
    order = np.lexsort((rows, cols))
    rows, cols, vals = rows[order], cols[order], vals[order]
    Ap = np.zeros(n + 1, dtype=np.int64)
    np.add.at(Ap, cols + 1, 1)
    Ap = np.cumsum(Ap)
    return Ap, rows.astype(np.int32), np.ascontiguousarray(vals, dtype=np.float64)


def _stencil_edges(shape, offsets):
    """All undirected grid edges (hi, lo) for the given half-stencil offsets."""
    shape = tuple(shape)
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    E_hi, E_lo = [], []
    for off in offsets:
        src = [slice(None)] * len(shape)
        dst = [slice(None)] * len(shape)
        for d, o in enumerate(off):
            if o > 0:
                src[d] = slice(0, shape[d] - o)
                dst[d] = slice(o, shape[d])
            elif o < 0:
                src[d] = slice(-o, shape[d])
                dst[d] = slice(0, shape[d] + o)
        a = idx[tuple(src)].ravel()
        b = idx[tuple(dst)].ravel()
        E_hi.append(np.maximum(a, b))
        E_lo.append(np.minimum(a, b))
    hi = np.concatenate(E_hi)
    lo = np.concatenate(E_lo)
    order = np.lexsort((hi, lo))
    return hi[order], lo[order]


def _half_offsets(dim: int, full: bool):
    """Half of a 2*dim+1 (full=False) or 3^dim (full=True) stencil."""
    offs = []
    rng = [-1, 0, 1]
    for o in np.array(np.meshgrid(*([rng] * dim), indexing="ij")).reshape(dim, -1).T:
        o = tuple(int(v) for v in o)
        if all(v == 0 for v in o):
            continue
        if not full and sum(abs(v) for v in o) != 1:
            continue
        # keep the lexicographically positive half
        first = next(v for v in o if v != 0)
        if first > 0:
            offs.append(o)
    return offs


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def _laplacian_from_edges(n, hi, lo, w, diag_extra):
    """A_ij = -w_ij off the diagonal; A_ii = sum_j w_ij then ``diag_extra``."""
    rowsum = np.zeros(n)
    np.add.at(rowsum, hi, w)
    np.add.at(rowsum, lo, w)
    return _lower_csc(n, hi, lo, -w, diag_extra(rowsum))


# --------------------------------------------------------------------------
# geometric nested dissection (an ordering choice, not part of the method)
# --------------------------------------------------------------------------

def grid_nd_order(shape, leaf: int = 32) -> np.ndarray:
    """Recursive bisection of a box on its longest axis; the middle slab is
    the separator (one slab separates any stencil that reaches only +-1 in
    each coordinate).  Leaves of <= ``leaf`` points keep natural order.
    Returns perm[new] = old."""
    shape = tuple(int(s) for s in shape)
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    out = []

    def rec(box):
        ext = [b1 - b0 for b0, b1 in box]
        size = int(np.prod(ext))
        if size == 0:
            return
        if size <= leaf or max(ext) < 3:
            out.append(idx[tuple(slice(b0, b1) for b0, b1 in box)].ravel())
            return
        d = int(np.argmax(ext))
        b0, b1 = box[d]
        mid = (b0 + b1) // 2
        left = list(box); left[d] = (b0, mid)
        right = list(box); right[d] = (mid + 1, b1)
        sep = list(box); sep[d] = (mid, mid + 1)
        rec(left)
        rec(right)
        out.append(idx[tuple(slice(a, b) for a, b in sep)].ravel())

    rec([(0, s) for s in shape])
    perm = np.concatenate(out).astype(np.int32)
    assert perm.size == idx.size and np.unique(perm).size == perm.size
    return perm


def points_nd_order(pts: np.ndarray, adj_ptr: np.ndarray, adj_idx: np.ndarray,
                    leaf: int = 64) -> np.ndarray:
    """Nested dissection of a geometric graph: split the points at the median
    of the widest coordinate; the separator is the set of left-side points
    with a neighbour on the right side.  Returns perm[new] = old over the
    points (graph vertices)."""
    nv = pts.shape[0]
    side = np.zeros(nv, dtype=np.int8)
    touch = np.zeros(nv, dtype=bool)
    out = []

    def neighbours(verts):
        starts = adj_ptr[verts]
        lens = adj_ptr[verts + 1] - starts
        total = int(lens.sum())
        base = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
        return np.repeat(verts, lens), adj_idx[base + np.arange(total)]

    # emit order per region: left part, right part, separator
    def rec(verts):
        if verts.size <= leaf:
            out.append(verts)
            return
        ext = pts[verts].max(0) - pts[verts].min(0)
        d = int(np.argmax(ext))
        order = verts[np.argsort(pts[verts, d], kind="stable")]
        half = order.size // 2
        left, right = order[:half], order[half:]
        side[right] = 2
        owner, nbr = neighbours(left)
        touch[owner[side[nbr] == 2]] = True
        side[right] = 0
        in_sep = touch[left]
        touch[left] = False
        sep = left[in_sep]
        left = left[~in_sep]
        rec(left)
        rec(right)
        out.append(sep)

    import sys
    lim = sys.getrecursionlimit()
    sys.setrecursionlimit(max(lim, 10000))
    try:
        rec(np.arange(nv))
    finally:
        sys.setrecursionlimit(lim)
    perm = np.concatenate(out).astype(np.int64)
    assert perm.size == nv and np.unique(perm).size == nv
    return perm


# --------------------------------------------------------------------------
# the five workload families
# --------------------------------------------------------------------------

def laplace2d_5pt(nx: int = 64, ny: int = 64) -> Workload:
    """Dirichlet 5-point Laplacian: 4 on the diagonal, -1 off it."""
    n = nx * ny
    hi, lo = _stencil_edges((nx, ny), _half_offsets(2, full=False))
    Ap, Ai, Ax = _lower_csc(n, hi, lo, -np.ones(hi.size), np.full(n, 4.0))
    return Workload(f"laplace2d_5pt_{nx}x{ny}", n, Ap, Ai, Ax,
                    grid_nd_order((nx, ny)), (nx, ny))


def weighted_grid(shape, full_stencil: bool, wlo: float, whi: float,
                  diag: str, seed_rng: np.random.Generator, name: str) -> Workload:
    """Weighted graph Laplacian on a grid with log-uniform edge weights.

    diag = "shift1e-6": A_ii = sum_j w_ij + 1e-6
    diag = "scale1e-6": A_ii = sum_j w_ij * (1 + 1e-6)
    diag = "shift1e-3": A_ii = sum_j w_ij + 1e-3
    """
    n = int(np.prod(shape))
    hi, lo = _stencil_edges(shape, _half_offsets(len(shape), full=full_stencil))
    w = _log_uniform(seed_rng, wlo, whi, hi.size)
    if diag == "shift1e-6":
        f = lambda s: s + 1e-6
    elif diag == "scale1e-6":
        f = lambda s: s * (1.0 + 1e-6)
    elif diag == "shift1e-3":
        f = lambda s: s + 1e-3
    else:
        raise ValueError(diag)
    Ap, Ai, Ax = _laplacian_from_edges(n, hi, lo, w, f)
    return Workload(name, n, Ap, Ai, Ax, grid_nd_order(shape), tuple(shape))


def config1() -> Workload:
    """2-D 5-point Laplacian, 64 x 64 (n = 4096)."""
    return laplace2d_5pt(64, 64)


def config2(m: int = 64) -> Workload:
    """3-D 7-point weighted Laplacian on an m^3 grid, w ~ logU[0.1, 10],
    A_ii = row sum + 1e-6 (m = 64 gives n = 262144)."""
    return weighted_grid((m, m, m), False, 0.1, 10.0, "shift1e-6", rng_for(2),
                         f"grid3d_7pt_{m}^3")


def config3(m: int = 80) -> Workload:
    """3-D 27-point weighted Laplacian on an m^3 grid, w ~ logU[1e-3, 1e3],
    A_ii = row sum * (1 + 1e-6) (m = 80 gives n = 512000)."""
    return weighted_grid((m, m, m), True, 1e-3, 1e3, "scale1e-6", rng_for(3),
                         f"grid3d_27pt_{m}^3")


def config4_instance(kind: str, k: int) -> Workload:
    """Batched family: ``kind`` in {"9pt128", "7pt24", "7pt40"}; instance k
    draws its weights w ~ logU[1e-2, 1e2]; A = L_G(w) + 1e-3 I."""
    rng = rng_for_instance(k)
    if kind == "9pt128":
        return weighted_grid((128, 128), True, 1e-2, 1e2, "shift1e-3", rng,
                             f"grid2d_9pt_128^2#{k}")
    if kind == "7pt24":
        return weighted_grid((24, 24, 24), False, 1e-2, 1e2, "shift1e-3", rng,
                             f"grid3d_7pt_24^3#{k}")
    if kind == "7pt40":
        return weighted_grid((40, 40, 40), False, 1e-2, 1e2, "shift1e-3", rng,
                             f"grid3d_7pt_40^3#{k}")
    raise ValueError(kind)


_CONFIG4_SHAPES = {"9pt128": ((128, 128), True), "7pt24": ((24, 24, 24), False),
                   "7pt40": ((40, 40, 40), False)}


def config4_batch(kind: str, m: int, k0: int = 0):
    """Instances k0 .. k0+m-1 of config4_instance(kind, k) at once: the
    shared pattern (n, Ap, Ai), the grid's ordering, and the m value sets
    as an (m, nnz) array (each row equal to that instance's Ax)."""
    shape, full = _CONFIG4_SHAPES[kind]
    n = int(np.prod(shape))
    hi, lo = _stencil_edges(shape, _half_offsets(len(shape), full=full))
    rows = np.concatenate([np.arange(n, dtype=np.int64), hi.astype(np.int64)])
    cols = np.concatenate([np.arange(n, dtype=np.int64), lo.astype(np.int64)])
    order = np.lexsort((rows, cols))
    Ap = np.zeros(n + 1, dtype=np.int64)
    np.add.at(Ap, cols + 1, 1)
    Ap = np.cumsum(Ap)
    Ai = rows[order].astype(np.int32)
    X = np.empty((m, order.size))
    for j in range(m):
        w = _log_uniform(rng_for_instance(k0 + j), 1e-2, 1e2, hi.size)
        rowsum = np.bincount(hi, w, minlength=n) + np.bincount(lo, w, minlength=n)
        X[j] = np.concatenate([rowsum + 1e-3, -w])[order]
    return n, Ap, Ai, X, grid_nd_order(shape)


def block_diagonal(parts):
    """The block-diagonal union of patterns: parts = [(n_i, Ap_i, Ai_i,
    X_i, perm_i), ...] with X_i an (m, nnz_i) value array (the same m for
    every part).  Returns (n, Ap, Ai, X, perm, offsets): the union's lower
    CSC, its (m, nnz) values (each row the parts' rows side by side), the
    parts' orderings placed one after another, and each part's first
    unknown (offsets[-1] = n)."""
    m = parts[0][3].shape[0]
    offsets = np.cumsum([0] + [p[0] for p in parts])
    Ap = [np.zeros(1, np.int64)]
    Ai, X, perm = [], [], []
    nnz = 0
    for (n_i, Ap_i, Ai_i, X_i, perm_i), off in zip(parts, offsets[:-1]):
        assert X_i.shape[0] == m
        Ap.append(Ap_i[1:] + nnz)
        Ai.append(Ai_i.astype(np.int64) + off)
        X.append(X_i)
        perm.append(np.asarray(perm_i, np.int64) + off)
        nnz += int(Ap_i[-1])
    return (int(offsets[-1]), np.concatenate(Ap), np.concatenate(Ai).astype(np.int32),
            np.concatenate(X, axis=1), np.concatenate(perm).astype(np.int32), offsets)


def config4_union(m: int = 64, copies_9pt: int = 8):
    """The batched workload as one pattern with m value sets: the
    block-diagonal union of copies_9pt 2-D 9-point 128^2 grids, one 3-D
    7-point 24^3 and one 40^3 grid.  Value set i holds instances
    copies_9pt * i .. copies_9pt * i + copies_9pt - 1 of the 9-point family
    and instance i of each 3-D family (the same values as config4_batch),
    so m = 64 value sets carry 512 + 64 + 64 instances.  Returns
    block_diagonal's tuple."""
    n9, Ap9, Ai9, X9, p9 = config4_batch("9pt128", copies_9pt * m)
    parts = [(n9, Ap9, Ai9, X9[c::copies_9pt], p9) for c in range(copies_9pt)]
    for kind in ("7pt24", "7pt40"):
        parts.append(config4_batch(kind, m))
    return block_diagonal(parts)


def random_spd_3x3(rng, count):
    """count random SPD 3x3 blocks Q diag(lambda) Q^T, Q Haar, lambda ~ U[0.1, 10]."""
    g = rng.standard_normal((count, 3, 3))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diagonal(r, axis1=1, axis2=2))[:, None, :]
    lam = rng.uniform(0.1, 10.0, (count, 3))
    return np.einsum("cij,cj,ckj->cik", q, lam, q)


def knn_instance(k: int, nv: int | None = None, knn: int = 13) -> Workload:
    """k-NN geometric graph (union-symmetrised) on uniform points in the unit
    cube, 3 dofs per vertex; each edge (u, v) carries B_uv SPD 3x3,
    A_uv = -B_uv and A_uu = sum_v B_uv + 0.1 I."""
    from scipy.spatial import cKDTree
    rng = rng_for_instance(1000 + k)
    if nv is None:
        nv = int(np.exp(rng.uniform(np.log(20000), np.log(200000))))
    pts = rng.uniform(0.0, 1.0, (nv, 3))
    _, nb = cKDTree(pts).query(pts, knn + 1)
    u = np.repeat(np.arange(nv), knn)
    v = nb[:, 1:].ravel()
    a, b = np.maximum(u, v), np.minimum(u, v)
    key = np.unique(a.astype(np.int64) * nv + b)
    ea, eb = key // nv, key % nv                      # ea > eb, unique edges
    B = random_spd_3x3(rng, ea.size)
    D = np.zeros((nv, 3, 3))
    np.add.at(D, ea, B)
    np.add.at(D, eb, B)
    D += 0.1 * np.eye(3)
    n = 3 * nv
    # off-diagonal blocks (ea > eb): all 9 entries go to the lower triangle
    oi = (3 * ea[:, None, None] + np.arange(3)[None, :, None]).repeat(3, 2)
    oj = (3 * eb[:, None, None] + np.arange(3)[None, None, :]).repeat(3, 1)
    ov = -B
    # diagonal blocks: lower triangle incl. the diagonal
    tri_r, tri_c = np.tril_indices(3)
    di = (3 * np.arange(nv)[:, None] + tri_r[None, :])
    dj = (3 * np.arange(nv)[:, None] + tri_c[None, :])
    dv = D[:, tri_r, tri_c]
    rows = np.concatenate([oi.ravel(), di.ravel()]).astype(np.int64)
    cols = np.concatenate([oj.ravel(), dj.ravel()]).astype(np.int64)
    vals = np.concatenate([ov.ravel(), dv.ravel()])
    order = np.lexsort((rows, cols))
    rows, cols, vals = rows[order], cols[order], vals[order]
    Ap = np.zeros(n + 1, dtype=np.int64)
    np.add.at(Ap, cols + 1, 1)
    Ap = np.cumsum(Ap)
    # vertex adjacency for the ordering
    adj_u = np.concatenate([ea, eb])
    adj_v = np.concatenate([eb, ea])
    o = np.argsort(adj_u, kind="stable")
    adj_u, adj_v = adj_u[o], adj_v[o]
    adj_ptr = np.zeros(nv + 1, dtype=np.int64)
    np.add.at(adj_ptr, adj_u + 1, 1)
    adj_ptr = np.cumsum(adj_ptr)
    vperm = points_nd_order(pts, adj_ptr, adj_v)
    perm = (3 * vperm[:, None] + np.arange(3)[None, :]).ravel().astype(np.int32)
    return Workload(f"knn13_{nv}v#{k}", n, Ap, rows.astype(np.int32),
                    np.ascontiguousarray(vals), perm, ())



KNN_FAMILY = 50             # instances 0..49 of the k-NN family


def knn_size(k: int) -> int:
    """Vertex count of k-NN instance k (the first draw of its stream, as in
    knn_instance with nv=None): log-uniform in [20000, 200000]."""
    rng = rng_for_instance(1000 + k)
    return int(np.exp(rng.uniform(np.log(20000), np.log(200000))))


def knn_split():
    """The seeded subset of the 50-instance k-NN family used for the
    learned cost model.  Instances are ranked by vertex count; ranks
    0, 5, ..., 45 and the largest (rank 49) train the model (21.9k to
    200k vertices), rank 17 (46k vertices) is the held-out test instance
    and rank 28 (83k vertices) the held-out benchmark instance.  Returns
    {"train": [k, ...], "test": k, "bench": k}."""
    order = sorted(range(KNN_FAMILY), key=knn_size)
    return {"train": [order[r] for r in list(range(0, 50, 5)) + [49]],
            "test": order[17], "bench": order[28]}

# --------------------------------------------------------------------------
# right-hand sides
# --------------------------------------------------------------------------

def dense_rhs(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, n)


def sparse_rhs(n: int, nnz: int, rng: np.random.Generator):
    """``nnz`` distinct positions uniform over [0, n) (original ordering),
    values U(-1, 1).  Returns (sorted int32 positions, float64 values)."""
    pos = np.sort(rng.choice(n, size=nnz, replace=False)).astype(np.int32)
    return pos, rng.uniform(-1.0, 1.0, nnz)


# --------------------------------------------------------------------------
# small random patterns for exhaustive tests
# --------------------------------------------------------------------------

def random_spd(n: int, density: float, rng: np.random.Generator,
               dominance: float = 1.0) -> Workload:
    """Random symmetric pattern with a strictly diagonally dominant SPD
    matrix on it (values and pattern from ``rng``)."""
    if n == 0:
        z = np.zeros(0)
        return Workload("empty", 0, np.zeros(1, np.int64), np.zeros(0, np.int32),
                        z, np.zeros(0, np.int32))
    m = rng.random((n, n)) < density
    m = np.tril(m, -1)
    hi, lo = np.nonzero(m)
    w = rng.uniform(-1.0, 1.0, hi.size)
    rowsum = np.zeros(n)
    np.add.at(rowsum, hi, np.abs(w))
    np.add.at(rowsum, lo, np.abs(w))
    diag = rowsum + dominance * rng.uniform(0.5, 1.5, n)
    Ap, Ai, Ax = _lower_csc(n, hi, lo, w, diag)
    return Workload(f"random_{n}_{density}", n, Ap, Ai, Ax,
                    rng.permutation(n).astype(np.int32))


def to_dense(w: Workload) -> np.ndarray:
    """Full symmetric dense matrix (original ordering); small n only."""
    A = np.zeros((w.n, w.n))
    for j in range(w.n):
        for p in range(w.Ap[j], w.Ap[j + 1]):
            i = w.Ai[p]
            A[i, j] = w.Ax[p]
            A[j, i] = w.Ax[p]
    return A
