"""GPU parity of the column-panel dual half-step (long rows split by column
panels, partial row sums added in panel order) against the FP64 oracle and
against the unsplit GPU path.

The panel kernels run in the plain iterations of a run; the first and last
iteration of each run of eval_freq iterations (and traced ones) take the
check kernels.  So the end point after K iterations is compared, for K inside
one run (63: 61 panel iterations) and across several runs and restarts.  Bars:
1e-10 relative to the oracle (only the summation order differs), 1e-12 to the
unsplit GPU path, bitwise repeatable, graphs bitwise equal to direct launches.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
import oracle
from oracle.pdhg import Params
from tests._gpu import announce, np_out, oracle_eta, problem, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _lp_from_matrix(A, seed, eq_frac=0.3):
    """Bounds and costs around a given matrix, as in the generator's recipe."""
    rng = np.random.default_rng(seed)
    A = sp.csr_matrix(A)
    A.sort_indices()
    m, n = A.shape
    xhat = rng.random(n)
    b = A @ xhat
    neq = int(eq_frac * m)
    lc = b.copy()
    uc = b.copy()
    lc[neq:] = b[neq:] - rng.random(m - neq)
    uc[neq:] = np.inf
    return lpgen.LP(A=A, c=rng.standard_normal(n), lc=lc, uc=uc, lv=np.zeros(n), uv=np.ones(n), xhat=xhat)


def _random_rows(rng, m, n, lengths):
    rows, cols = [], []
    for i, L in enumerate(lengths):
        L = int(min(L, n))
        if L == 0:
            continue
        cols.append(rng.choice(n, size=L, replace=False))
        rows.append(np.full(L, i))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    return sp.csr_matrix((rng.standard_normal(r.size), (r, c)), shape=(m, n))


def _end_point_case(lp, K, panels, row_min, dense_min=4096):
    eta = oracle_eta(lp)
    prob = problem(lp, eta=eta, column_panels=panels, panel_row_min=row_min, dense_row_min=dense_min)
    P, nl = prob.panels()
    PD, nd = prob.dense()
    lens = np.diff(lp.A.indptr)
    dense = (lens >= dense_min) if dense_min else np.zeros(lens.size, bool)
    assert P == 8 * ((panels + 7) // 8)
    assert nl == int(((lens > row_min) & ~dense).sum()) and nd == int(dense.sum()) and nl + nd > 0
    assert PD == (-(-lp.n // 2048) if nd else 0)
    out = np_out(prob.solve(tol=0.0, max_iter=K))
    prob.close()
    plain = problem(lp, eta=eta, column_panels=0)
    assert plain.panels() == (0, 0)
    ref_gpu = np_out(plain.solve(tol=0.0, max_iter=K))
    plain.close()
    ref = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, Params(tol=0.0, max_iter=K, eta_override=eta))
    ex, ey = rel(out["x"], ref.x), rel(out["y"], ref.y)
    gx, gy = rel(out["x"], ref_gpu["x"]), rel(out["y"], ref_gpu["y"])
    print(f"K={K} P={P} long rows={nl} dense rows={nd}: vs oracle {ex:.1e} {ey:.1e}; vs unsplit {gx:.1e} {gy:.1e}")
    assert ex <= TOL and ey <= TOL
    assert gx <= 1e-12 and gy <= 1e-12
    assert out["info"]["restarts"] == ref.restarts
    assert out["info"]["omega"] == pytest.approx(ref.omega, rel=1e-9)
    return out, ref


@pytest.mark.parametrize("K", [63, 200])
def test_panels_skewed_rows_match_oracle(K):
    """Zipf rows up to 9,000 nonzeros: segments longer than the LDS stage take
    the block-wide reduction, short segments share blocks."""
    lp = lpgen.gen(3000, 20000, zipf_alpha=1.3, cap=9000, eq_frac=0.3, free_frac=0.2, values="normal", seed=7)
    announce(f"panels skewed K={K} nnz={lp.nnz}")
    _end_point_case(lp, K, panels=16, row_min=8)


@pytest.mark.parametrize("panels", [1, 1024])
def test_panels_count_extremes(panels):
    """The fewest (8) and the most (1024) wide panels: with 1024 panels of 20
    columns most (panel, long row) segments are empty and each XCD holds 128
    panels, so the slots of k_dual_ps are mostly panel blocks; with 8 panels
    one per XCD."""
    lp = lpgen.gen(3000, 20000, zipf_alpha=1.3, cap=9000, eq_frac=0.3, free_frac=0.2, values="normal", seed=9)
    announce(f"panels count {panels} nnz={lp.nnz}")
    _end_point_case(lp, 130, panels=panels, row_min=8, dense_min=1024)


@pytest.mark.parametrize("dense_min", [0, 512])
def test_panels_long_and_dense_rows(dense_min):
    """Rows above 512 nonzeros in the narrow LDS-staged panels, the rest of the
    long rows in the wide panels; and the same LP with no dense class."""
    lp = lpgen.gen(3000, 20000, zipf_alpha=1.3, cap=9000, eq_frac=0.3, free_frac=0.2, values="normal", seed=7)
    announce(f"panels long + dense ({dense_min}) nnz={lp.nnz}")
    _end_point_case(lp, 200, panels=16, row_min=8, dense_min=dense_min)


def test_panels_only_dense_rows():
    """Every row above panel_row_min is dense: the wide panels are empty."""
    lp = lpgen.config("c1", seed=2)
    announce("panels only dense rows (c1)")
    _end_point_case(lp, 200, panels=8, row_min=2, dense_min=3)


def test_panels_dense_rows_wider_than_one_narrow_panel():
    """n = 9,000 (five narrow panels, the last one partial); dense rows of
    2,000-8,000 nonzeros next to short ones."""
    rng = np.random.default_rng(12)
    m, n = 400, 9000
    lens = rng.integers(0, 8, size=m)
    lens[::50] = rng.integers(2000, 8000, size=lens[::50].size)
    lp = _lp_from_matrix(_random_rows(rng, m, n, lens), seed=12)
    announce(f"panels dense partial narrow panel nnz={lp.nnz}")
    _end_point_case(lp, 130, panels=8, row_min=16, dense_min=1000)


def test_panels_primal_split_several_slices():
    """9,000 dense rows of 40-90 nonzeros (n = 20,000): the primal split takes
    five slices of the compact y copy, the last one partial, next to a few
    short rows."""
    rng = np.random.default_rng(21)
    m, n = 9500, 20000
    lens = rng.integers(40, 91, size=m)
    lens[9000:] = rng.integers(1, 10, size=500)
    lp = _lp_from_matrix(_random_rows(rng, m, n, lens), seed=21)
    announce(f"panels primal split, several slices nnz={lp.nnz}")
    _end_point_case(lp, 130, panels=8, row_min=16, dense_min=32)


def test_panels_all_rows_long():
    """panel_row_min below every row length: the short part is empty."""
    lp = lpgen.config("c1", seed=2)
    announce("panels all rows long (c1)")
    _end_point_case(lp, 200, panels=8, row_min=2)


def test_panels_single_long_row_and_empty_rows():
    rng = np.random.default_rng(11)
    m, n = 700, 6000
    lens = rng.integers(0, 6, size=m)
    lens[::37] = 0
    lens[5] = 5000                      # the one long row; its segments exceed the LDS stage
    lp = _lp_from_matrix(_random_rows(rng, m, n, lens), seed=11)
    announce(f"panels single long row nnz={lp.nnz}")
    _end_point_case(lp, 63, panels=8, row_min=16)


def test_panels_more_panels_than_columns():
    """n = 10 < 16 panels: panels of width 1, six of them empty."""
    rng = np.random.default_rng(5)
    m, n = 60, 10
    lens = rng.integers(1, 11, size=m)
    lp = _lp_from_matrix(_random_rows(rng, m, n, lens), seed=5)
    announce("panels P > n")
    _end_point_case(lp, 200, panels=16, row_min=4)


def test_panels_fp64_solve_to_tolerance_and_repeatable():
    lp = lpgen.config("c1", seed=3)
    announce("panels c1 solve 1e-8")
    eta = oracle_eta(lp)
    prob = problem(lp, eta=eta, column_panels=8, panel_row_min=3, dense_row_min=5)
    assert prob.panels()[0] == 8 and prob.dense()[1] > 0
    a = np_out(prob.solve(tol=1e-8))
    b = np_out(prob.solve(tol=1e-8))
    c = np_out(prob.solve(tol=1e-8, graphs=0))
    prob.close()
    for k in ("x", "y"):
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k])
    ref = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, Params(tol=1e-8, eta_override=eta))
    assert a["info"]["status"] == oracle.pdhg.OPTIMAL == ref.status
    assert a["info"]["iters"] == ref.iters and a["info"]["restarts"] == ref.restarts
    k = oracle.kkt(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, a["x"], a["y"])
    assert k["rel_kkt"] <= 1e-8 * (1 + 1e-6)
    assert rel(a["x"], ref.x) <= 1e-8 and rel(a["y"], ref.y) <= 1e-8


def test_panels_mixed_precision():
    """FP32 panel path (wide and narrow panels): same tolerance by the oracle's
    KKT; graphs bitwise equal to direct launches; close to the unsplit FP32 path."""
    from paper_2507_14051_amd import MIXED
    lp = lpgen.gen(3000, 20000, zipf_alpha=1.3, cap=9000, eq_frac=0.3, free_frac=0.2, values="normal", seed=7)
    announce("panels mixed")
    prob = problem(lp, precision=MIXED, column_panels=16, panel_row_min=8, dense_row_min=512)
    assert prob.panels()[0] == 16 and prob.dense()[1] > 0
    a = np_out(prob.solve(tol=0.0, max_iter=300))
    b = np_out(prob.solve(tol=0.0, max_iter=300, graphs=0))
    prob.close()
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["y"], b["y"])
    _, _, eta, _ = problem(lp, precision=MIXED, column_panels=16, panel_row_min=8, dense_row_min=512).scaling()
    plain = problem(lp, eta=eta, precision=MIXED, column_panels=0)
    c = np_out(plain.solve(tol=0.0, max_iter=300))
    plain.close()
    print(f"mixed panels vs unsplit after 300: x {rel(a['x'], c['x']):.1e} y {rel(a['y'], c['y']):.1e}")
    assert rel(a["x"], c["x"]) <= 1e-4 and rel(a["y"], c["y"]) <= 1e-4
    lp1 = lpgen.config("c1", seed=1)
    p1 = problem(lp1, precision=MIXED, column_panels=8, panel_row_min=3, dense_row_min=5)
    o = np_out(p1.solve(tol=1e-8))
    p1.close()
    k = oracle.kkt(lp1.A, lp1.c, lp1.lc, lp1.uc, lp1.lv, lp1.uv, o["x"], o["y"])
    assert o["info"]["status"] == oracle.pdhg.OPTIMAL and k["rel_kkt"] <= 1e-8 * (1 + 1e-6)


def test_panels_automatic_on_large_skewed_lp():
    """The large skewed LP (m=2e6, n=5e6, ~30M nonzeros): the automatic rule
    takes 40 panels; 200 iterations agree with the unsplit path."""
    lp = lpgen.config("c3b", seed=1)
    announce(f"panels c3b nnz={lp.nnz}")
    a = problem(lp)
    P, nl = a.panels()
    PD, nd = a.dense()
    lens = np.diff(lp.A.indptr)
    assert P == 40 and nl == int(((lens > 16) & (lens < 2048)).sum())
    assert PD == 2442 and nd == int((lens >= 2048).sum()) > 0
    _, _, eta, _ = a.scaling()
    oa = np_out(a.solve(tol=0.0, max_iter=200))
    a.close()
    b = problem(lp, eta=eta, column_panels=0)
    ob = np_out(b.solve(tol=0.0, max_iter=200))
    b.close()
    print(f"c3b panels vs unsplit: x {rel(oa['x'], ob['x']):.1e} y {rel(oa['y'], ob['y']):.1e}")
    assert rel(oa["x"], ob["x"]) <= 1e-10 and rel(oa["y"], ob["y"]) <= 1e-10
    assert oa["info"]["restarts"] == ob["info"]["restarts"]


def test_panels_off_by_default_on_small_lp():
    lp = lpgen.config("c1", seed=1)
    prob = problem(lp)
    assert prob.panels() == (0, 0)
    prob.close()


def test_panels_leave_adjoint_and_later_solves_unchanged():
    """The unrolled forward/reverse pass runs with the unsplit dual step (the
    panel layout is switched off inside it), so its outputs and gradients are
    bitwise those of a handle without panels; a solve after it still keeps
    the compact copy of the long rows' y entries (same end point as before)."""
    from tests.test_gpu_adjoint import KEYS, _grads
    lp = lpgen.gen(800, 3000, zipf_alpha=1.4, cap=2500, eq_frac=0.3, free_frac=0.2, values="normal", seed=4)
    announce(f"panels adjoint nnz={lp.nnz}")
    rng = np.random.default_rng(4)
    gx = rng.standard_normal(lp.n); gy = rng.standard_normal(lp.m)
    pa = problem(lp, column_panels=8, panel_row_min=8, dense_row_min=400)
    assert pa.panels()[0] == 8 and pa.dense()[1] > 0
    _, _, eta, _ = pa.scaling()
    before = np_out(pa.solve(tol=0.0, max_iter=150))
    xa, ya, ga = _grads(pa, lp, 120, 25, gx, gy, eval_freq=16)
    after = np_out(pa.solve(tol=0.0, max_iter=150))
    pa.close()
    pb = problem(lp, eta=eta, column_panels=0)
    xb, yb, gb = _grads(pb, lp, 120, 25, gx, gy, eval_freq=16)
    pb.close()
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    for k in KEYS:
        assert np.array_equal(ga[k], gb[k]), k
    assert np.array_equal(before["x"], after["x"]) and np.array_equal(before["y"], after["y"])


def test_panels_and_dense_rows_on_c3a_full_size():
    """The largest LP (m=2e6, n=5e6, 692M nonzeros, 7,007 rows at the
    50,000 cap): wide panels, narrow LDS-staged panels on both half-steps and
    int32 offsets near 7e8; 130 iterations (two runs, a check) agree with the
    unsplit path."""
    lp = lpgen.config("c3a", seed=1)
    announce(f"panels c3a nnz={lp.nnz}")
    lens = np.diff(lp.A.indptr)
    a = problem(lp)
    P, nl = a.panels()
    PD, nd = a.dense()
    assert P == 40 and nd == int((lens >= 2048).sum()) and nl == int(((lens > 16) & (lens < 2048)).sum())
    _, _, eta, _ = a.scaling()
    oa = np_out(a.solve(tol=0.0, max_iter=130))
    a.close()
    b = problem(lp, eta=eta, column_panels=0)
    ob = np_out(b.solve(tol=0.0, max_iter=130))
    b.close()
    print(f"c3a panels vs unsplit: x {rel(oa['x'], ob['x']):.1e} y {rel(oa['y'], ob['y']):.1e}")
    assert rel(oa["x"], ob["x"]) <= 1e-10 and rel(oa["y"], ob["y"]) <= 1e-10


def test_power_iteration_with_panels_matches_oracle():
    """The setup's power iteration through the panel kernels (wide and narrow
    panels, the split transpose) gives the oracle's norm estimate."""
    from oracle.pdhg import power_norm, rescale
    lp = lpgen.gen(3000, 20000, zipf_alpha=1.3, cap=9000, eq_frac=0.3, free_frac=0.2, values="normal", seed=7)
    announce("power iteration with panels")
    prob = problem(lp, column_panels=16, panel_row_min=8, dense_row_min=512)
    assert prob.dense()[1] > 0
    _, _, eta, pit = prob.scaling()
    prob.close()
    At, _, _ = rescale(lp.A, 10, 1)
    nrm, it = power_norm(At, 5000, 1e-8)
    assert eta == pytest.approx(0.998 / nrm, rel=1e-9)
    assert abs(pit - it) <= 1


def test_more_dense_rows_than_reserved_raise_the_threshold():
    """With dense_row_min = 20 the c3b LP has about 100,000 rows above it, more
    than the 65,536 dense rows the workspace holds: the threshold doubles until
    they fit, and the end point is that of the unsplit layout."""
    lp = lpgen.config("c3b", seed=1)
    lens = np.diff(lp.A.indptr)
    assert (lens >= 20).sum() > 65536
    Ld = 20
    while (lens >= Ld).sum() > 65536:
        Ld *= 2
    announce(f"panels dense overflow (c3b): threshold 20 -> {Ld}")
    a = problem(lp, dense_row_min=20)
    assert a.dense() == (2442, int((lens >= Ld).sum()))
    assert a.panels() == (40, int(((lens > 16) & (lens < Ld)).sum()))
    _, _, eta, _ = a.scaling()
    oa = np_out(a.solve(tol=0.0, max_iter=70))
    a.close()
    b = problem(lp, eta=eta, column_panels=0)
    ob = np_out(b.solve(tol=0.0, max_iter=70))
    b.close()
    assert rel(oa["x"], ob["x"]) <= 1e-10 and rel(oa["y"], ob["y"]) <= 1e-10


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("layout", ["plain", "panels"])
def test_streamed_matrix_loads_change_nothing(layout, precision):
    """stream_matrix = 1 turns on the non-temporal matrix loads in every
    half-step kernel (the default only does so above 128 MB of matrix): the
    iterates are the same bit for bit as with cached loads, with and without
    the panel and dense-row layouts, in FP64 and in FP32 + refinement."""
    lp = lpgen.gen(3000, 20000, zipf_alpha=1.3, cap=9000, eq_frac=0.3, free_frac=0.2, values="normal", seed=7)
    announce(f"streamed matrix loads {layout} precision={precision} nnz={lp.nnz}")
    eta = oracle_eta(lp)
    lay = dict(column_panels=16, panel_row_min=8, dense_row_min=512) if layout == "panels" else dict(column_panels=0)
    outs = []
    for nt in (0, 1):
        prob = problem(lp, eta=eta, precision=precision, stream_matrix=nt, **lay)
        if layout == "panels":
            assert prob.panels()[1] > 0 and prob.dense()[1] > 0
        outs.append(np_out(prob.solve(tol=0.0, max_iter=200)))
        prob.close()
    assert np.array_equal(outs[0]["x"], outs[1]["x"]) and np.array_equal(outs[0]["y"], outs[1]["y"])
    assert outs[0]["info"]["restarts"] == outs[1]["info"]["restarts"]
    if precision == 0:
        ref = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, Params(tol=0.0, max_iter=200, eta_override=eta))
        assert rel(outs[1]["x"], ref.x) <= TOL and rel(outs[1]["y"], ref.y) <= TOL


@pytest.mark.parametrize("precision", [0, 1])
def test_workspace_sized_for_the_rows_gives_the_same_bits(precision):
    """A handle laid out in the workspace sized for the matrix's rows
    (hlp_workspace_bytes_csr, Problem's layout="rows") and one laid out for the
    worst rows (hlp_workspace_bytes) build the same panel layout and give the
    same bits; the row-sized workspace is the smaller one."""
    import torch
    from paper_2507_14051_amd import hlp
    lp = lpgen.gen(3000, 20000, zipf_alpha=1.3, cap=9000, eq_frac=0.3, free_frac=0.2, values="normal", seed=7)
    announce(f"row-sized vs worst-case workspace precision={precision}")
    kw = dict(column_panels=16, panel_row_min=8, dense_row_min=512, precision=precision)
    a = problem(lp, layout="rows", **kw)
    assert a.panels()[0] == 16 and a.dense()[1] > 0
    oa = np_out(a.solve(tol=0.0, max_iter=300))
    params = a.params_for()
    worst = hlp.hlp_workspace_bytes(lp.m, lp.n, lp.nnz, params)
    assert a.workspace.numel() < worst
    base = torch.empty(worst + 256, dtype=torch.uint8, device="cuda:0")
    off = (-base.data_ptr()) % 256
    ws = base[off:off + worst]
    h = hlp.hlp_lp_create(lp.m, lp.n, lp.nnz, a.row_ptr, a.col_idx, a.val, *a.vectors, params, ws)
    assert hlp.hlp_lp_panels(h) == (*a.panels(), *a.dense())
    f64 = dict(dtype=torch.float64, device="cuda:0")
    x, y = torch.empty(lp.n, **f64), torch.empty(lp.m, **f64)
    info = hlp.hlp_solve(h, hlp.hlp_params_default(**{**kw, "tol": 0.0, "max_iter": 300}), None, None, x, y)
    hlp.hlp_lp_destroy(h)
    a.close()
    assert np.array_equal(oa["x"], x.cpu().numpy()) and np.array_equal(oa["y"], y.cpu().numpy())
    assert info.iters == oa["info"]["iters"] == 300
