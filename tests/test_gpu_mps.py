"""An LP read from an MPS file and solved on the GPU: the objective in the
file's sense against the oracle's solve of the same LP, and the command-line
entry point on a file."""
import numpy as np
import pytest

import lpgen
import oracle
from paper_2507_14051_amd.mps import main, read_mps, write_mps
from tests._gpu import announce, np_out, problem

pytestmark = pytest.mark.gpu


def test_mps_file_solved_on_gpu_matches_oracle(tmp_path, capsys):
    lp = lpgen.gen_mixed(200, 300, rowlen=4, seed=11)
    keep = np.isfinite(lp.lc) | np.isfinite(lp.uc)
    lp = lpgen.LP(A=lp.A[keep], c=lp.c, lc=lp.lc[keep], uc=lp.uc[keep], lv=lp.lv, uv=lp.uv)
    path = tmp_path / "mixed.mps"
    path.write_text(write_mps(lp, name="MIXED", offset=2.5))
    announce(f"mps: m={lp.m} n={lp.n} nnz={lp.nnz}")
    m = read_mps(str(path))
    prob = problem(m)
    out = np_out(prob.solve(tol=1e-9))
    prob.close()
    ref = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, oracle.Params(tol=1e-9))
    assert out["info"]["status"] == oracle.pdhg.OPTIMAL == ref.status
    k = oracle.kkt(m.A, m.c, m.lc, m.uc, m.lv, m.uv, out["x"], out["y"])
    assert k["rel_kkt"] <= 1e-9 * (1 + 1e-6)
    assert m.objective(out["x"]) == pytest.approx(ref.info["pobj"] + 2.5, rel=1e-7, abs=1e-7)
    assert main([str(path), "--tol", "1e-8"]) == 0
    printed = capsys.readouterr().out
    assert "status OPTIMAL" in printed and "MIXED" in printed
