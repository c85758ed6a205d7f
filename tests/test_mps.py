"""The MPS reader (paper_2507_14051_amd/mps.py): a hand-written file covering
every section, row type, range sign and bound type against hand-derived
arrays; write/read round trips of LPs with every bound pattern; malformed
files rejected.  CPU only."""
import math

import numpy as np
import pytest

import lpgen
from paper_2507_14051_amd.mps import read_mps, write_mps

INF = math.inf

HAND = """* a maximisation with every section; hand-derived form in test_hand_file
NAME          HAND
OBJSENSE
    MAX
ROWS
 N  cost
 L  lim1
 G  lim2
 E  myeqn
 N  free2
 E  rng_e
COLUMNS
    MARKER                 'MARKER'                 'INTORG'
    x1        cost         1.0   lim1         1.0
    MARKER                 'MARKER'                 'INTEND'
    x1        lim2         1.0   rng_e   2.0
    x2        cost         2.0   lim1         1.0
    x2        myeqn       -1.0   free2 5.0
    x3        cost        -1.0   myeqn        1.0
    x4        lim2         3.0
RHS
    RHS       cost         -3.5
    RHS       lim1         4.0   lim2         1.0
    RHS       myeqn        7.0   rng_e 1.0
RANGES
    RNG       lim1         2.5   rng_e -0.5
BOUNDS
 UP BND       x1           4.0
 MI BND       x2
 UP BND       x2           1.0
 FX BND       x3           2.5
 UP BND       x4          -2.0
ENDATA
"""


def test_hand_file():
    lp = read_mps(HAND)
    assert lp.name == "HAND" and lp.sense == -1
    assert lp.row_names == ["lim1", "lim2", "myeqn", "rng_e"] and lp.col_names == ["x1", "x2", "x3", "x4"]
    # maximise x1 + 2 x2 - x3 + 3.5  ->  minimise -x1 - 2 x2 + x3 - 3.5
    np.testing.assert_array_equal(lp.c, [-1.0, -2.0, 1.0, 0.0])
    assert lp.offset == -3.5
    np.testing.assert_array_equal(lp.A.toarray(), [[1, 1, 0, 0], [1, 0, 0, 3], [0, -1, 1, 0], [2, 0, 0, 0]])
    # L 4 range 2.5 -> [1.5, 4]; G 1 -> [1, inf); E 7; E 1 range -0.5 -> [0.5, 1]
    np.testing.assert_array_equal(lp.lc, [1.5, 1.0, 7.0, 0.5])
    np.testing.assert_array_equal(lp.uc, [4.0, INF, 7.0, 1.0])
    # x1 [0, 4]; x2 MI then UP 1; x3 FX 2.5; x4 UP -2 with the default lower -> (-inf, -2]
    np.testing.assert_array_equal(lp.lv, [0.0, -INF, 2.5, -INF])
    np.testing.assert_array_equal(lp.uv, [4.0, 1.0, 2.5, -2.0])
    x = np.array([0.5, 1.0, 2.5, -3.0])
    assert lp.objective(x) == pytest.approx(0.5 + 2.0 - 2.5 + 3.5)


def test_objsense_on_the_keyword_line_and_ranges_on_g_rows():
    txt = "NAME t\nOBJSENSE MAX\nROWS\n N obj\n G g1\nCOLUMNS\n x obj 2 g1 1\nRHS\n rhs g1 3\nRANGES\n r g1 -2\nENDATA\n"
    lp = read_mps(txt)
    assert lp.sense == -1 and lp.c[0] == -2.0
    assert (lp.lc[0], lp.uc[0]) == (3.0, 5.0)        # G row: [rhs, rhs + |R|]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_round_trip_every_bound_pattern(seed):
    lp = lpgen.gen_mixed(40, 50, rowlen=3, seed=seed)
    keep = np.isfinite(lp.lc) | np.isfinite(lp.uc)      # a row without finite bounds has no MPS form
    lp = lpgen.LP(A=lp.A[keep], c=lp.c, lc=lp.lc[keep], uc=lp.uc[keep], lv=lp.lv, uv=lp.uv)
    back = read_mps(write_mps(lp, name="rt", offset=-0.75))
    np.testing.assert_array_equal(back.A.toarray(), lp.A.toarray())
    for k in ("c", "uc", "lv", "uv"):
        np.testing.assert_array_equal(getattr(back, k), getattr(lp, k))
    # a two-sided row is stored as rhs = uc and range R = uc - lc: lc comes back as uc - R, exact up to an ulp
    np.testing.assert_allclose(back.lc, lp.lc, rtol=4e-16, atol=4e-16)
    assert np.array_equal(np.isinf(back.lc), np.isinf(lp.lc))
    assert back.offset == -0.75 and back.sense == 1
    assert back.A.indices.dtype == np.int32 and back.A.has_sorted_indices


def test_read_then_oracle_solve_matches_highs():
    import oracle
    from tests._highs import highs
    lp = lpgen.gen_mixed(30, 40, rowlen=3, seed=5)
    keep = np.isfinite(lp.lc) | np.isfinite(lp.uc)
    lp = lpgen.LP(A=lp.A[keep], c=lp.c, lc=lp.lc[keep], uc=lp.uc[keep], lv=lp.lv, uv=lp.uv)
    m = read_mps(write_mps(lp))
    fun, _, _ = highs(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv)
    res = oracle.solve(m.A, m.c, m.lc, m.uc, m.lv, m.uv, oracle.Params(tol=1e-9))
    assert res.status == oracle.pdhg.OPTIMAL
    assert m.objective(res.x) == pytest.approx(fun, rel=1e-7, abs=1e-7)


@pytest.mark.parametrize("bad, msg", [
    ("NAME t\nROWS\n N obj\n L r\nCOLUMNS\n x obj 1 q 2\nENDATA\n", "unknown row"),
    ("NAME t\nROWS\n N obj\n L r\nCOLUMNS\n x r 1\n x r 2\nENDATA\n", "given twice"),
    ("NAME t\nROWS\n N obj\n L r\nCOLUMNS\n x r one\nENDATA\n", "not a number"),
    ("NAME t\nROWS\n N obj\n Q r\nENDATA\n", "unknown row type"),
    ("NAME t\nROWS\n N obj\n L r\nCOLUMNS\n x r 1\nBOUNDS\n UP b y 1\nENDATA\n", "unknown column"),
])
def test_malformed_files_are_rejected(bad, msg):
    with pytest.raises(ValueError, match=msg):
        read_mps(bad)
