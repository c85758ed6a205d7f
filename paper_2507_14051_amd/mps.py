"""LPs in MPS format, in the form the solver takes:

    min  c^T x + offset   s.t.   lc <= A x <= uc,   lv <= x <= uv

(the paper's eq. (lp), Sec. 2.1; its experiments, Sec. 4, read the MIPLIB 2017
and Mittelmann instances from MPS files).  Free-format MPS: whitespace
separated fields, names without blanks.

Sections: NAME, OBJSENSE (MIN/MAX, on its own line or after the keyword),
ROWS (N, E, L, G; the first N row is the objective, further N rows are free
rows and are dropped), COLUMNS (integrality MARKER lines are skipped: the LP
relaxation is read, and integer columns keep the default bounds [0, +inf)),
RHS (a right-hand side on the objective row is minus the objective's constant),
RANGES, BOUNDS (UP, LO, FX, FR, MI, PL, BV, LI, UI), ENDATA.

Row bounds: E rows lc = uc = rhs, widened by a range R to [rhs, rhs + R] for
R > 0 and [rhs + R, rhs] for R < 0; L rows (-inf, rhs], with a range
[rhs - |R|, rhs]; G rows [rhs, +inf), with a range [rhs, rhs + |R|].  Column
bounds default to [0, +inf); an UP bound below zero on a column whose lower
bound is still the default 0 sets that lower bound to -inf (the usual MPS
convention).  A maximisation is returned as the minimisation of -c, with
``sense = -1`` recorded so that objective values can be reported in the
file's sense.

    python -m paper_2507_14051_amd.mps model.mps [--tol 1e-8] [--time-limit 3600] [--mixed]

reads a file and solves it on the GPU with the library.
"""
from __future__ import annotations

import argparse
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

INF = math.inf


@dataclass
class MpsLP:
    name: str
    A: sp.csr_matrix
    c: np.ndarray
    lc: np.ndarray
    uc: np.ndarray
    lv: np.ndarray
    uv: np.ndarray
    offset: float = 0.0          # constant of the minimised objective
    sense: int = 1               # 1: the file minimises, -1: it maximises (c above is already negated)
    row_names: list = field(default_factory=list)
    col_names: list = field(default_factory=list)

    @property
    def m(self):
        return self.A.shape[0]

    @property
    def n(self):
        return self.A.shape[1]

    def objective(self, x):
        """The file's objective at x (its sense and constant included)."""
        return self.sense * (float(self.c @ x) + self.offset)


def _num(tok, where):
    try:
        return float(tok)
    except ValueError:
        raise ValueError(f"MPS: not a number {tok!r} in {where}") from None


def read_mps(source) -> MpsLP:
    """Parse MPS text (a str holding the file's contents, or a path)."""
    if "\n" not in source:
        with open(source) as f:
            source = f.read()
    name = ""
    sense = 1
    section = None
    obj_row = None
    row_type = {}          # name -> 'E'/'L'/'G'
    row_order = []
    free_rows = set()
    col_index = {}
    col_names = []
    entries = {}           # (row, col) -> value
    cost = {}
    rhs = {}
    ranges = {}
    lower = {}
    upper = {}
    offset = 0.0
    for lineno, raw in enumerate(source.splitlines(), 1):
        line = raw.rstrip()
        if not line or line.lstrip().startswith("*"):
            continue
        tok = line.split()
        where = f"line {lineno}"
        if not raw[0].isspace():
            key = tok[0].upper()
            if key == "NAME":
                name = tok[1] if len(tok) > 1 else ""
                section = None
            elif key == "OBJSENSE":
                section = "OBJSENSE"
                if len(tok) > 1:
                    sense = -1 if tok[1].upper() in ("MAX", "MAXIMIZE") else 1
            elif key in ("ROWS", "COLUMNS", "RHS", "RANGES", "BOUNDS"):
                section = key
            elif key == "ENDATA":
                break
            elif section == "OBJSENSE" and key in ("MAX", "MAXIMIZE", "MIN", "MINIMIZE"):
                sense = -1 if key.startswith("MAX") else 1
            else:
                raise ValueError(f"MPS: unknown section {tok[0]!r} at {where}")
            continue
        if section == "OBJSENSE":
            sense = -1 if tok[0].upper() in ("MAX", "MAXIMIZE") else 1
        elif section == "ROWS":
            kind, rname = tok[0].upper(), tok[1]
            if kind == "N":
                if obj_row is None:
                    obj_row = rname
                else:
                    free_rows.add(rname)
            elif kind in ("E", "L", "G"):
                if rname in row_type:
                    raise ValueError(f"MPS: row {rname!r} defined twice ({where})")
                row_type[rname] = kind
                row_order.append(rname)
            else:
                raise ValueError(f"MPS: unknown row type {kind!r} ({where})")
        elif section == "COLUMNS":
            if len(tok) >= 3 and tok[1].upper() == "'MARKER'":
                continue
            cname = tok[0]
            if cname not in col_index:
                col_index[cname] = len(col_names)
                col_names.append(cname)
            j = col_index[cname]
            if len(tok) not in (3, 5):
                raise ValueError(f"MPS: COLUMNS line needs 1 or 2 (row, value) pairs ({where})")
            for rname, val in zip(tok[1::2], tok[2::2]):
                v = _num(val, where)
                if rname == obj_row:
                    cost[j] = cost.get(j, 0.0) + v
                elif rname in free_rows:
                    continue
                elif rname in row_type:
                    if (rname, j) in entries:
                        raise ValueError(f"MPS: entry ({rname}, {cname}) given twice ({where})")
                    entries[(rname, j)] = v
                else:
                    raise ValueError(f"MPS: unknown row {rname!r} ({where})")
        elif section in ("RHS", "RANGES"):
            pairs = tok[1:] if len(tok) % 2 == 1 else tok
            for rname, val in zip(pairs[0::2], pairs[1::2]):
                v = _num(val, where)
                if section == "RHS" and rname == obj_row:
                    offset = -v
                elif rname in free_rows:
                    continue
                elif rname not in row_type:
                    raise ValueError(f"MPS: unknown row {rname!r} ({where})")
                elif section == "RHS":
                    rhs[rname] = v
                else:
                    ranges[rname] = v
        elif section == "BOUNDS":
            # type [bound-set name] column [value]
            kind = tok[0].upper()
            if kind in ("UP", "LO", "FX", "LI", "UI"):
                if len(tok) == 4:
                    cname, val = tok[2], _num(tok[3], where)
                elif len(tok) == 3:
                    cname, val = tok[1], _num(tok[2], where)
                else:
                    raise ValueError(f"MPS: malformed BOUNDS line ({where})")
            elif len(tok) in (3, 4):
                cname, val = tok[2], None
            elif len(tok) == 2:
                cname, val = tok[1], None
            else:
                raise ValueError(f"MPS: malformed BOUNDS line ({where})")
            if cname not in col_index:
                raise ValueError(f"MPS: bound on unknown column {cname!r} ({where})")
            j = col_index[cname]
            if kind in ("UP", "UI"):
                upper[j] = val
                if val < 0 and j not in lower:
                    lower[j] = -INF
            elif kind in ("LO", "LI"):
                lower[j] = val
            elif kind == "FX":
                lower[j] = upper[j] = val
            elif kind == "FR":
                lower[j], upper[j] = -INF, INF
            elif kind == "MI":
                lower[j] = -INF
            elif kind == "PL":
                upper[j] = INF
            elif kind == "BV":
                lower[j], upper[j] = 0.0, 1.0
            else:
                raise ValueError(f"MPS: unknown bound type {kind!r} ({where})")
        else:
            raise ValueError(f"MPS: data outside a section at {where}")
    if obj_row is None and not row_order and not col_names:
        raise ValueError("MPS: no ROWS/COLUMNS found")
    m, n = len(row_order), len(col_names)
    rix = {r: i for i, r in enumerate(row_order)}
    if entries:
        ri = np.fromiter((rix[r] for r, _ in entries), dtype=np.int64, count=len(entries))
        ci = np.fromiter((j for _, j in entries), dtype=np.int64, count=len(entries))
        vv = np.fromiter(entries.values(), dtype=np.float64, count=len(entries))
    else:
        ri = ci = np.zeros(0, dtype=np.int64)
        vv = np.zeros(0)
    A = sp.csr_matrix((vv, (ri, ci)), shape=(m, n))
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    c = np.zeros(n)
    for j, v in cost.items():
        c[j] = v
    lc = np.empty(m)
    uc = np.empty(m)
    for i, r in enumerate(row_order):
        b = rhs.get(r, 0.0)
        k = row_type[r]
        R = ranges.get(r)
        if k == "E":
            lc[i] = uc[i] = b
            if R is not None:
                if R > 0:
                    uc[i] = b + R
                elif R < 0:
                    lc[i] = b + R
        elif k == "L":
            lc[i], uc[i] = (-INF if R is None else b - abs(R)), b
        else:
            lc[i], uc[i] = b, (INF if R is None else b + abs(R))
    lv = np.zeros(n)
    uv = np.full(n, INF)
    for j, v in lower.items():
        lv[j] = v
    for j, v in upper.items():
        uv[j] = v
    if sense == -1:
        c = -c
        offset = -offset
    return MpsLP(name, A, c, lc, uc, lv, uv, offset, sense, row_order, col_names)


def _fmt(v):
    return repr(float(v))


def write_mps(lp, name="LP", offset=0.0) -> str:
    """MPS text of min c^T x + offset s.t. lc <= A x <= uc, lv <= x <= uv:
    one E, L or G row per constraint (a two-sided row as an L row with a
    range); a row with no finite bound cannot be written and is rejected."""
    A = sp.csr_matrix(lp.A)
    m, n = A.shape
    out = [f"NAME {name}", "ROWS", " N obj"]
    kinds = []
    for i in range(m):
        lo, hi = lp.lc[i], lp.uc[i]
        if lo == hi:
            k = "E"
        elif math.isfinite(hi):
            k = "L"
        elif math.isfinite(lo):
            k = "G"
        else:
            raise ValueError(f"row {i} has no finite bound: not representable in MPS")
        kinds.append(k)
        out.append(f" {k} r{i}")
    out.append("COLUMNS")
    At = A.tocsc()
    for j in range(n):
        if lp.c[j] != 0.0:
            out.append(f" x{j} obj {_fmt(lp.c[j])}")
        for p in range(At.indptr[j], At.indptr[j + 1]):
            out.append(f" x{j} r{At.indices[p]} {_fmt(At.data[p])}")
        if lp.c[j] == 0.0 and At.indptr[j] == At.indptr[j + 1]:
            out.append(f" x{j} obj 0.0")
    out.append("RHS")
    if offset != 0.0:
        out.append(f" rhs obj {_fmt(-offset)}")
    for i, k in enumerate(kinds):
        b = lp.uc[i] if k in ("E", "L") else lp.lc[i]
        if b != 0.0:
            out.append(f" rhs r{i} {_fmt(b)}")
    rng = [(i, lp.uc[i] - lp.lc[i]) for i, k in enumerate(kinds)
           if k == "L" and math.isfinite(lp.lc[i])]
    if rng:
        out.append("RANGES")
        out += [f" rng r{i} {_fmt(R)}" for i, R in rng]
    out.append("BOUNDS")
    for j in range(n):
        lo, hi = lp.lv[j], lp.uv[j]
        if lo == hi:
            out.append(f" FX bnd x{j} {_fmt(lo)}")
            continue
        if lo == -INF and hi == INF:
            out.append(f" FR bnd x{j}")
            continue
        if lo == -INF:
            out.append(f" MI bnd x{j}")
        elif lo != 0.0:
            out.append(f" LO bnd x{j} {_fmt(lo)}")
        if hi != INF:
            out.append(f" UP bnd x{j} {_fmt(hi)}")
    out.append("ENDATA")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description="Solve an LP in MPS format with restarted Halpern PDHG on the GPU")
    ap.add_argument("path")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--time-limit", type=float, default=3600.0)
    ap.add_argument("--mixed", action="store_true", help="FP32 iteration with FP64 refinement")
    args = ap.parse_args(argv)
    from . import MIXED, STATUS_NAMES, Problem
    t0 = time.perf_counter()
    lp = read_mps(args.path)
    t1 = time.perf_counter()
    setup = {"precision": MIXED} if args.mixed else {}
    prob = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device="cuda", **setup)
    out = prob.solve(tol=args.tol, time_limit_s=args.time_limit, want_r=False)
    info = out["info"]
    x = out["x"].cpu().numpy()
    prob.close()
    print(f"{lp.name}: m={lp.m} n={lp.n} nnz={lp.A.nnz}; read {t1 - t0:.2f} s, setup {info['setup_s']:.2f} s, "
          f"solve {info['solve_s']:.2f} s")
    print(f"status {STATUS_NAMES[info['status']]}, {info['iters']} iterations, {info['restarts']} restarts, "
          f"relative KKT {info['rel_kkt']:.3e}, objective {lp.objective(x):.12g}")
    return 0 if info["status"] == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
