"""Seeded synthetic LP generators.

This module builds inputs only; it holds none of the solver's arithmetic and is
shared by the CPU oracle, the tests and the benchmark.  Every LP has the form

    min c^T x   s.t.   lc <= A x <= uc,   lv <= x <= uv          (paper, Sec. 2.1)

with IEEE +-inf for absent bounds.  The recipe (draw order is part of the
definition, so a seed fixes every byte):

  1. row lengths: fixed ``rowlen`` or Zipf(alpha) clipped at ``cap`` (and at n);
  2. column indices: per row, drawn uniformly without replacement from [0, n)
     (rejection of rows with repeats), sorted;
  3. values: N(0,1), or sign * 10^U[-3,3] ("logu");
  4. a feasible point xhat ~ U[0,1]^n, and b = A xhat;
  5. rows: the first floor(eq_frac*m) are equalities lc = uc = b, the rest
     lc = b - U[0,1], uc = +inf;
  6. columns: lv = 0, uv = 1, except the last floor(free_frac*n) columns which
     get uv = +inf; c ~ N(0,1) with c_j = |N(0,1)| on those free columns.

xhat satisfies every constraint, so the LP is feasible; the box plus the
nonnegative costs on the columns without an upper bound keep it bounded.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

INF = np.inf


@dataclass
class LP:
    """An LP in the paper's primal form, with CSR storage (int32 columns)."""

    A: sp.csr_matrix
    c: np.ndarray
    lc: np.ndarray
    uc: np.ndarray
    lv: np.ndarray
    uv: np.ndarray
    xhat: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]

    @property
    def nnz(self) -> int:
        return int(self.A.nnz)


def _columns_fixed(rng, m, n, L):
    """m rows of L distinct sorted columns in [0, n)."""
    if L == 0 or m == 0:
        return np.zeros((m, 0), dtype=np.int64)
    cols = rng.integers(0, n, size=(m, L))
    cols.sort(axis=1)
    bad = (np.diff(cols, axis=1) == 0).any(axis=1) if L > 1 else np.zeros(m, bool)
    while bad.any():
        idx = np.nonzero(bad)[0]
        new = rng.integers(0, n, size=(idx.size, L))
        new.sort(axis=1)
        cols[idx] = new
        bad[idx] = (np.diff(new, axis=1) == 0).any(axis=1)
    return cols


def _columns_var(rng, n, lengths):
    """Rows of the given lengths, distinct sorted columns each, as flat arrays."""
    m = lengths.size
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=indptr[1:])
    indices = np.empty(int(indptr[-1]), dtype=np.int64)
    # Group rows by length so each group is drawn as a dense block; group order
    # is ascending length, rows inside a group in ascending row order.
    for L in np.unique(lengths):
        rows = np.nonzero(lengths == L)[0]
        if L == 0:
            continue
        if L * L > n:  # repeats likely: draw each row directly without replacement
            block = np.empty((rows.size, L), dtype=np.int64)
            for i in range(rows.size):
                block[i] = np.sort(rng.choice(n, size=L, replace=False))
        else:
            block = _columns_fixed(rng, rows.size, n, int(L))
        starts = indptr[rows]
        pos = starts[:, None] + np.arange(L)[None, :]
        indices[pos.ravel()] = block.ravel()
    return indptr, indices


def _draw_values(rng, nnz, values):
    if values == "normal":
        return rng.standard_normal(nnz)
    if values == "logu":
        sign = np.where(rng.random(nnz) < 0.5, -1.0, 1.0)
        return sign * 10.0 ** rng.uniform(-3.0, 3.0, size=nnz)
    raise ValueError(values)


def _zipf_rows(rng, m, n, zipf_alpha, cap):
    lengths = rng.zipf(zipf_alpha, size=m).astype(np.int64)
    lengths = np.minimum(lengths, min(cap if cap is not None else n, n))
    return _columns_var(rng, n, lengths)


def _zipf_chunk(args):
    """Rows of one chunk (its own seed): lengths, columns, values."""
    seed_seq, m, n, zipf_alpha, cap, values = args
    rng = np.random.default_rng(seed_seq)
    indptr, indices = _zipf_rows(rng, m, n, zipf_alpha, cap)
    return np.diff(indptr), indices.astype(np.int32), _draw_values(rng, indices.size, values)


def _zipf_rows_chunked(seed, m, n, zipf_alpha, cap, values, chunks, progress=None):
    """The Zipf-row matrix drawn in `chunks` row chunks, chunk k from the k-th
    child of SeedSequence(seed) (so chunks are independent of each other);
    progress(k, chunks) is called after each chunk."""
    bounds = np.linspace(0, m, chunks + 1).astype(np.int64)
    kids = np.random.SeedSequence(seed).spawn(chunks)
    parts = []
    for k in range(chunks):
        parts.append(_zipf_chunk((kids[k], int(bounds[k + 1] - bounds[k]), n, zipf_alpha, cap, values)))
        if progress:
            progress(k + 1, chunks)
    lengths = np.concatenate([p[0] for p in parts])
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=indptr[1:])
    indices = np.concatenate([p[1] for p in parts])
    del lengths
    vals = np.concatenate([p[2] for p in parts])
    return indptr, indices, vals


def gen(m, n, rowlen=8, eq_frac=0.3, free_frac=0.0, seed=1, values="normal",
        zipf_alpha=None, cap=None, eq_rows=None, row_chunks=0, progress=None) -> LP:
    """The synthetic LP family described in the module docstring.  With
    row_chunks > 0 (Zipf rows only) the matrix is drawn chunk by chunk from
    child seeds; the rest of the recipe then continues from the generator of
    `seed` itself."""
    rng = np.random.default_rng(seed)
    if zipf_alpha is not None and row_chunks > 0:
        indptr, indices, vals = _zipf_rows_chunked(seed, m, n, zipf_alpha, cap, values, row_chunks, progress)
    else:
        if zipf_alpha is not None:
            indptr, indices = _zipf_rows(rng, m, n, zipf_alpha, cap)
        else:
            L = min(int(rowlen), n)
            cols = _columns_fixed(rng, m, n, L)
            indptr = np.arange(m + 1, dtype=np.int64) * L
            indices = cols.ravel()
        vals = _draw_values(rng, indices.size, values)
    nnz = indices.size
    A = sp.csr_matrix((vals, indices.astype(np.int32, copy=False), indptr), shape=(m, n))
    xhat = rng.random(n)
    b = A @ xhat
    neq = int(eq_frac * m) if eq_rows is None else int(eq_rows)
    slack = rng.random(m - neq)
    lc = b.copy()
    uc = b.copy()
    lc[neq:] = b[neq:] - slack
    uc[neq:] = INF
    nfree = int(free_frac * n)
    lv = np.zeros(n)
    uv = np.ones(n)
    c = rng.standard_normal(n)
    if nfree:
        uv[n - nfree:] = INF
        c[n - nfree:] = np.abs(c[n - nfree:])
    lens = np.diff(indptr)
    meta = dict(m=m, n=n, nnz=int(nnz), seed=seed, max_row=int(lens.max()) if m else 0,
                rows_at_cap=int((lens == cap).sum()) if cap else 0)
    return LP(A, c, lc, uc, lv, uv, xhat, meta)


def gen_mixed(m, n, rowlen=3, seed=1, box_only=False) -> LP:
    """Small LPs that exercise every bound pattern of the paper's sets Y and R.

    Rows cycle through: equality, lower-only, upper-only, ranged, free.
    Columns cycle through: boxed, lower-only (c >= 0), upper-only (c <= 0),
    free (c = 0) -- unless ``box_only``, where every column is boxed (the
    polytope is then bounded, as vertex enumeration needs).
    """
    rng = np.random.default_rng(seed)
    L = min(rowlen, n)
    cols = _columns_fixed(rng, m, n, L)
    indptr = np.arange(m + 1, dtype=np.int64) * L
    vals = rng.standard_normal(m * L)
    A = sp.csr_matrix((vals, cols.ravel().astype(np.int32), indptr), shape=(m, n))
    xhat = rng.uniform(-1.0, 1.0, size=n)
    b = A @ xhat
    s1 = rng.uniform(0.1, 1.0, size=m)
    s2 = rng.uniform(0.1, 1.0, size=m)
    lc = np.empty(m)
    uc = np.empty(m)
    for i in range(m):
        kind = i % 5
        if kind == 0:
            lc[i] = uc[i] = b[i]
        elif kind == 1:
            lc[i], uc[i] = b[i] - s1[i], INF
        elif kind == 2:
            lc[i], uc[i] = -INF, b[i] + s2[i]
        elif kind == 3:
            lc[i], uc[i] = b[i] - s1[i], b[i] + s2[i]
        else:
            lc[i], uc[i] = -INF, INF
    t1 = rng.uniform(0.1, 1.0, size=n)
    t2 = rng.uniform(0.1, 1.0, size=n)
    c = rng.standard_normal(n)
    lv = xhat - t1
    uv = xhat + t2
    if not box_only:
        for j in range(n):
            kind = j % 4
            if kind == 1:
                uv[j] = INF
                c[j] = abs(c[j])
            elif kind == 2:
                lv[j] = -INF
                c[j] = -abs(c[j])
            elif kind == 3:
                lv[j], uv[j] = -INF, INF
                c[j] = 0.0
    return LP(A, c, lc, uc, lv, uv, xhat, dict(m=m, n=n, nnz=int(A.nnz), seed=seed))


# The workload configurations.  C3a takes the literal Zipf(1.5) law; C3b the
# exponent that gives the stated ~3e7 nonzeros.
CONFIGS = {
    "c1": dict(m=1000, n=2000, rowlen=5, eq_rows=500, free_frac=0.0, tol=1e-4),
    "c2": dict(m=100_000, n=200_000, rowlen=8, eq_frac=0.3, free_frac=0.2, tol=1e-8),
    "c3a": dict(m=2_000_000, n=5_000_000, zipf_alpha=1.5, cap=50_000, eq_frac=0.3,
                free_frac=0.2, values="logu", row_chunks=64, tol=1e-8),
    "c3b": dict(m=2_000_000, n=5_000_000, zipf_alpha=1.882, cap=50_000, eq_frac=0.3,
                free_frac=0.2, values="logu", tol=1e-8),
    "c5": dict(m=50_000, n=100_000, rowlen=8, eq_frac=0.3, free_frac=0.2, tol=1e-8),
}


def config(name: str, seed: int = 1, scale: float = 1.0, progress=None) -> LP:
    """One of the named configurations; ``scale`` shrinks m and n together."""
    cfg = dict(CONFIGS[name])
    if "row_chunks" in cfg:
        cfg["progress"] = progress
    cfg.pop("tol")
    cfg["m"] = max(1, int(cfg["m"] * scale))
    cfg["n"] = max(1, int(cfg["n"] * scale))
    if "eq_rows" in cfg:
        cfg["eq_rows"] = int(cfg["eq_rows"] * scale)
    return gen(seed=seed, **cfg)


def tolerance(name: str) -> float:
    return CONFIGS[name]["tol"]


def x_target(n: int, seed: int = 1) -> np.ndarray:
    """Target vector for the differentiation workload, U[0,1]^n."""
    return np.random.default_rng(10_000 + seed).random(n)


def directions(lp: LP, seed: int = 1):
    """Random unit-scale perturbation directions for c and the finite bounds."""
    rng = np.random.default_rng(20_000 + seed)
    def fin(v):
        d = rng.standard_normal(v.size)
        d[~np.isfinite(v)] = 0.0
        return d
    d = dict(c=rng.standard_normal(lp.n), lc=fin(lp.lc), uc=fin(lp.uc),
             lv=fin(lp.lv), uv=fin(lp.uv))
    eq = lp.lc == lp.uc          # an equality row moves as one right-hand side b
    d["uc"][eq] = d["lc"][eq]
    eqv = lp.lv == lp.uv
    d["uv"][eqv] = d["lv"][eqv]
    return d
