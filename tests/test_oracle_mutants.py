"""The oracle's pins must be able to fail: each plausible mistake below is
planted in a scratch copy of the oracle package (on the CPU, never in the
product), and at least one pin of tests/_pins.py must reject the copy.  The
unmodified copy must pass every pin.

The mistakes are those a reader checking the oracle against the paper by eye
could miss: a sign, a factor or a swapped pair in r(z) (Sec. 2.2), the
Halpern weight one step off (Sec. 3), the restart bookkeeping (Sec. 3,
"Adaptive restart"), the Pock-Chambolle pass without its root or with maxima,
and the duality-gap denominator (Sec. 4); the PID update's sign, error and
integral, the new anchor at a restart and the sign of the reflection (Sec.
3); the power iteration's square root (Sec. 3, stepsize); the primal bound
norm and the projected dual residual of the KKT error (Sec. 4).
"""
import importlib
import itertools
import os
import shutil
import sys

import pytest

from tests import _pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

# (name, file, original text, planted text)
MUTANTS = [
    ("residual_cross_sign", "pdhg.py", "+ 2.0 * float(dy @ (At @ dx))", "- 2.0 * float(dy @ (At @ dx))"),
    ("residual_cross_factor", "pdhg.py", "+ 2.0 * float(dy @ (At @ dx))", "+ 1.0 * float(dy @ (At @ dx))"),
    ("residual_weights_swapped", "pdhg.py",
     "q = (omega / eta) * float(dx @ dx) + 2.0 * float(dy @ (At @ dx)) + float(dy @ dy) / (eta * omega)",
     "q = float(dx @ dx) / (eta * omega) + 2.0 * float(dy @ (At @ dx)) + (omega / eta) * float(dy @ dy)"),
    ("halpern_weight_one_ahead", "pdhg.py", "a = k / (k + 1)", "a = (k + 1) / (k + 2)"),
    ("artificial_total_offset", "pdhg.py", "restart_decision(r, r0, r_prev, k, t, p)",
     "restart_decision(r, r0, r_prev, k, t + 64, p)"),
    ("r0_reset_every_check", "pdhg.py", "            if k == 0:\n                r0 = r",
     "            if True:\n                r0 = r"),
    ("pock_chambolle_no_root", "pdhg.py",
     "rho = np.where(rsum > 0, np.sqrt(rsum), 1.0)\n        kap = np.where(csum > 0, np.sqrt(csum), 1.0)",
     "rho = np.where(rsum > 0, rsum, 1.0)\n        kap = np.where(csum > 0, csum, 1.0)"),
    ("pock_chambolle_max", "pdhg.py",
     "rsum = np.asarray(absA.sum(axis=1)).ravel()\n        csum = np.asarray(absA.sum(axis=0)).ravel()",
     "rsum = np.asarray(absA.max(axis=1).todense()).ravel()\n"
     "        csum = np.asarray(absA.max(axis=0).todense()).ravel()"),
    ("gap_denominator", "kkt.py", "(1.0 + abs(pobj) + abs(dobj))", "(1.0 + abs(pobj - dobj))"),
    ("pid_sign", "pdhg.py", "math.exp(math.log(omega) - (p.kp * e", "math.exp(math.log(omega) + (p.kp * e"),
    ("pid_error_inverted", "pdhg.py", "e = math.log(omega * dxn / dyn)", "e = math.log(omega * dyn / dxn)"),
    ("pid_integral_lags", "pdhg.py", 'state["sum"] = state.get("sum", 0.0) + e',
     'state["sum"] = state.get("sum", 0.0) + (state.get("prev") or 0.0)'),
    ("anchor_is_halpern_iterate", "pdhg.py", "            if p.restart_to_current:\n",
     "            if not p.restart_to_current:\n"),
    ("reflection_sign", "pdhg.py", "x = a * ((1.0 + gam) * xh - gam * x) + (1.0 - a) * xa",
     "x = a * ((1.0 - gam) * xh + gam * x) + (1.0 - a) * xa"),
    ("power_norm_squared", "pdhg.py", "    return math.sqrt(s), it", "    return s, it"),
    ("primal_bound_norm_lower_only", "kkt.py",
     "bnd = np.concatenate([lc[np.isfinite(lc)], uc[np.isfinite(uc)]])", "bnd = lc[np.isfinite(lc)]"),
    ("dual_residual_unprojected", "kkt.py", "rho_d = float(np.linalg.norm(g - r))",
     "rho_d = float(np.linalg.norm(g))"),
]


_counter = itertools.count()


def _load_copy(tmp_path, edit=None):
    """Copy oracle/ under a fresh package name, apply one textual edit, import it."""
    name = f"oracle_copy_{next(_counter)}"
    dst = tmp_path / name
    shutil.copytree(ORACLE, dst, ignore=shutil.ignore_patterns("__pycache__"))
    if edit is not None:
        fname, old, new = edit
        path = dst / fname
        src = path.read_text()
        assert src.count(old) == 1, f"planting site not unique in {fname}: {old!r}"
        path.write_text(src.replace(old, new))
    sys.path.insert(0, str(tmp_path))
    try:
        return importlib.import_module(name)
    finally:
        sys.path.remove(str(tmp_path))


def _failing_pins(orc):
    failed = []
    for pin in _pins.ALL_PINS:
        try:
            pin(orc)
        except (AssertionError, ArithmeticError, ValueError) as e:   # noqa: PERF203
            failed.append((pin.__name__, type(e).__name__))
    return failed


def test_unmodified_copy_passes_every_pin(tmp_path):
    assert _failing_pins(_load_copy(tmp_path)) == []


@pytest.mark.parametrize("name,fname,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, fname, old, new):
    failed = _failing_pins(_load_copy(tmp_path, (fname, old, new)))
    assert failed, f"no pin rejects the planted mistake {name}"
