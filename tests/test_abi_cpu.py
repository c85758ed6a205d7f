"""CPU-only checks of the C ABI: the library loads, exports every function the
header declares, and the ctypes mirrors of the structs match the C layout
(checked with a tiny C program compiled by gcc against include/hlp.h)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hlp.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hlp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2507_14051_amd import hlp
    L = hlp.lib()
    names = _declared_functions()
    assert set(names) == set(hlp.SYMBOLS)
    for name in names:
        assert hasattr(L, name), name
    nm = subprocess.run(["nm", "-D", "--defined-only", hlp.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (hlp_\w+)", nm))
    assert set(names) <= exported


def _c_layout(tmp_path, struct, fields):
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){",
             f'printf("size %zu\\n", sizeof({struct}));']
    for f in fields:
        lines.append(f'printf("{f} %zu\\n", offsetof({struct}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return {k: int(v) for k, v in (ln.split() for ln in out.strip().splitlines())}


@pytest.mark.parametrize("name", ["HlpParams", "HlpInfo", "HlpCheck"])
def test_struct_layout_matches_header(tmp_path, name):
    from paper_2507_14051_amd import hlp
    cls = getattr(hlp, name)
    cname = {"HlpParams": "hlp_params", "HlpInfo": "hlp_info", "HlpCheck": "hlp_check"}[name]
    fields = [f for f, _ in cls._fields_]
    lay = _c_layout(tmp_path, cname, fields)
    assert lay["size"] == C.sizeof(cls)
    for f in fields:
        assert lay[f] == getattr(cls, f).offset, f


def test_defaults_match_oracle_readings():
    import oracle
    from paper_2507_14051_amd import hlp_params_default
    p = hlp_params_default()
    o = oracle.Params()
    for f in ("tol", "max_iter", "eval_freq", "gamma", "beta_sufficient", "beta_necessary", "beta_artificial",
              "kp", "ki", "kd", "omega0", "eta_override", "ruiz_iters", "pock_chambolle", "power_max_iter",
              "power_tol", "restart_to_current", "pid_min_norm", "trace_iters"):
        assert getattr(p, f) == getattr(o, f), f


def test_workspace_bytes_and_argument_errors():
    from paper_2507_14051_amd import HlpError, hlp_params_default, hlp_workspace_bytes
    p = hlp_params_default()
    a = hlp_workspace_bytes(1000, 2000, 5000, p)
    b = hlp_workspace_bytes(1000, 2000, 50000, p)
    assert 0 < a < b
    pm = hlp_params_default(precision=1)
    assert hlp_workspace_bytes(1000, 2000, 5000, pm) > a       # FP32 mirrors
    with pytest.raises(HlpError) as e:
        hlp_workspace_bytes(-1, 2, 3, p)
    assert e.value.code == -1
    with pytest.raises(HlpError) as e:
        hlp_workspace_bytes(10, 10, 2 ** 31, p)
    assert e.value.code == -4


def test_graft_build_compiles(tmp_path):
    """build() always recompiles every source and the result loads."""
    import importlib
    import __graft_entry__ as g
    g.build()
    from paper_2507_14051_amd import hlp
    assert os.path.getsize(hlp.LIB_PATH) > 0


def test_panel_parameters_and_workspace():
    """Column panels are reserved only for large n (or when asked), dense rows
    only with them; bad panel parameters are rejected before any device work."""
    import ctypes as C
    from paper_2507_14051_amd import HlpError, hlp_params_default, hlp_workspace_bytes
    from paper_2507_14051_amd import hlp as H
    m, n, nnz = 2_000_000, 5_000_000, 30_000_000
    base = hlp_workspace_bytes(m, n, nnz, hlp_params_default(column_panels=0))
    auto = hlp_workspace_bytes(m, n, nnz, hlp_params_default())
    nodense = hlp_workspace_bytes(m, n, nnz, hlp_params_default(dense_row_min=0))
    assert base < nodense < auto
    small = dict(m=1000, n=2000, nnz=5000)
    assert (hlp_workspace_bytes(*small.values(), hlp_params_default())
            == hlp_workspace_bytes(*small.values(), hlp_params_default(column_panels=0)))
    assert (hlp_workspace_bytes(*small.values(), hlp_params_default(column_panels=8))
            > hlp_workspace_bytes(*small.values(), hlp_params_default(column_panels=0)))
    # invalid parameters: hlp_lp_create returns HLP_EINVAL before touching the pointers
    L = H.lib()
    fake = C.c_void_p(1 << 20)        # never dereferenced: validation fails first
    out = C.c_void_p()
    for bad in (dict(column_panels=-2), dict(panel_row_min=0), dict(panel_row_min=16, dense_row_min=16)):
        p = hlp_params_default(**bad)
        rc = L.hlp_lp_create(10, 10, 10, fake, fake, fake, fake, fake, fake, fake, fake, C.byref(p), fake,
                             C.c_size_t(1 << 30), None, C.byref(out))
        assert rc == -1, bad
        assert b"panel" in L.hlp_last_error()


def test_workspace_sized_for_the_rows():
    """hlp_workspace_bytes_csr sizes the column-panel layout for the matrix's
    own rows: never above the worst case for (m, n, nnz), equal to it when no
    panel layout is used, well below it for skewed rows; bad row pointers are
    rejected."""
    import lpgen
    from paper_2507_14051_amd import HlpError, hlp_params_default, hlp_workspace_bytes, hlp_workspace_bytes_csr
    lp = lpgen.config("c1", seed=1)
    p = hlp_params_default()
    assert hlp_workspace_bytes_csr(lp.m, lp.n, lp.nnz, lp.A.indptr, p) == hlp_workspace_bytes(lp.m, lp.n, lp.nnz, p)
    sk = lpgen.gen(3000, 20000, zipf_alpha=1.3, cap=9000, eq_frac=0.3, free_frac=0.2, values="normal", seed=7)
    for kw in (dict(column_panels=16, panel_row_min=8, dense_row_min=512), dict(column_panels=16, panel_row_min=8),
               dict(column_panels=8, panel_row_min=8, dense_row_min=0), dict(column_panels=8, precision=1)):
        q = hlp_params_default(**kw)
        w = hlp_workspace_bytes(sk.m, sk.n, sk.nnz, q)
        e = hlp_workspace_bytes_csr(sk.m, sk.n, sk.nnz, sk.A.indptr, q)
        assert e < w, kw
    bad = sk.A.indptr.copy()
    bad[5], bad[6] = bad[6], bad[5]
    with pytest.raises(HlpError) as err:
        hlp_workspace_bytes_csr(sk.m, sk.n, sk.nnz, bad, p)
    assert err.value.code == -1
