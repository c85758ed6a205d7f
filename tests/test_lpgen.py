"""The seeded input generators: reproducible, well-formed CSR, and the stated
recipe (feasible point, bound pattern, row-length law)."""
import numpy as np

import lpgen


def _well_formed(lp):
    A = lp.A
    assert A.indptr[0] == 0 and A.indptr[-1] == A.nnz
    assert (np.diff(A.indptr) >= 0).all()
    for i in range(0, A.shape[0], max(1, A.shape[0] // 200)):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        assert (np.diff(cols) > 0).all() and (cols.size == 0 or (cols[0] >= 0 and cols[-1] < A.shape[1]))
    ax = A @ lp.xhat
    assert (ax >= lp.lc - 1e-9).all() and (ax <= lp.uc + 1e-9).all()
    assert ((lp.xhat >= lp.lv) & (lp.xhat <= lp.uv)).all()


def test_fixed_rows_reproducible_and_feasible():
    a = lpgen.config("c2", seed=3, scale=0.05)
    b = lpgen.config("c2", seed=3, scale=0.05)
    assert (a.A != b.A).nnz == 0 and np.array_equal(a.c, b.c) and np.array_equal(a.lc, b.lc)
    assert (np.diff(a.A.indptr) == 8).all()
    _well_formed(a)
    free = ~np.isfinite(a.uv)
    assert free.sum() == int(0.2 * a.n) and (a.c[free] >= 0).all()
    assert (a.lc == a.uc).sum() == int(0.3 * a.m)


def test_zipf_rows_chunked_reproducible():
    """The chunked Zipf recipe (used for c3a): same seed, same LP; chunks from
    independent child seeds; rows capped; columns distinct and sorted."""
    kw = dict(m=3000, n=20000, zipf_alpha=1.5, cap=5000, eq_frac=0.3, free_frac=0.2, values="logu", seed=9)
    a = lpgen.gen(row_chunks=6, **kw)
    b = lpgen.gen(row_chunks=6, **kw)
    assert (a.A != b.A).nnz == 0 and np.array_equal(a.lc, b.lc) and np.array_equal(a.c, b.c)
    lens = np.diff(a.A.indptr)
    assert lens.max() <= 5000 and lens.min() >= 1
    assert a.meta["rows_at_cap"] == int((lens == 5000).sum())
    v = np.abs(a.A.data)
    assert v.min() >= 1e-3 * (1 - 1e-12) and v.max() <= 1e3 * (1 + 1e-12)
    _well_formed(a)
    c = lpgen.gen(row_chunks=0, **kw)          # the unchunked recipe draws another matrix
    assert c.nnz != a.nnz or (c.A != a.A).nnz > 0


def test_c3_configs_scaled():
    b = lpgen.config("c3b", seed=1, scale=0.01)
    assert b.m == 20000 and b.n == 50000
    _well_formed(b)
    a = lpgen.config("c3a", seed=1, scale=0.002)
    assert a.m == 4000 and a.n == 10000
    _well_formed(a)
    # Zipf(1.5) is much heavier than Zipf(1.882): mean row length far larger
    assert a.nnz / a.m > 3 * (b.nnz / b.m)
