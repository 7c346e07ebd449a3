"""MPS reader and writer for the LP form the solver takes.

The solver's LP (Section 2.2) is  min c'x  s.t.  Gx >= h,  Ax = b,
l <= x <= u.  An MPS model maps onto it row by row:

    N row (the first one)   objective c; its RHS entry r adds the constant -r
    G row  a'x >= r         ">=" row  a, r
    L row  a'x <= r         ">=" row -a, -r
    E row  a'x  = r         "=" row   a, r
    RANGES R on a row       the row becomes two ">=" rows, lo <= a'x <= hi with
                            G: [r, r + |R|], L: [r - |R|, r],
                            E: [r, r + R] for R > 0, [r + R, r] for R < 0

and bounds default to [0, +inf): UP u (u < 0 with the default lower bound
also sets l = -inf), LO, FX (l = u), FR (-inf, inf), MI (l = -inf), PL
(u = +inf), BV ([0, 1]), LI / UI (as LO / UP).  Integrality markers and
integer bound types are read as their LP relaxation.  OBJSENSE MAX (or
MAXIMIZE) negates c, so the solver always minimises; ``objective(x)``
reports the value in the model's own sense.

Fields are split on whitespace (free MPS; fixed-format files whose names
hold no blanks read the same way).  Lines starting with ``*`` are comments.
"""
from __future__ import annotations

import dataclasses
import gzip
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

GE, EQ = 0, 1  # PDHG_ROW_GE, PDHG_ROW_EQ


@dataclasses.dataclass
class MPSModel:
    """An LP in the solver's form plus what maps results back to the file."""

    n: int
    m: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    row_type: np.ndarray
    rhs: np.ndarray
    c: np.ndarray
    l: np.ndarray
    u: np.ndarray
    name: str = ""
    col_names: List[str] = dataclasses.field(default_factory=list)
    # per solver row: (index of the MPS row, +1 or -1 = sign applied to it)
    row_origin: List[Tuple[int, int]] = dataclasses.field(default_factory=list)
    row_names: List[str] = dataclasses.field(default_factory=list)  # constraint rows of the file
    obj_name: str = ""
    obj_offset: float = 0.0  # added to c'x (minimisation form)
    maximize: bool = False

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def objective(self, x) -> float:
        """Objective of x in the model's own sense (with the constant)."""
        v = float(np.dot(self.c, x)) + self.obj_offset
        return -v if self.maximize else v

    def row_duals(self, y) -> np.ndarray:
        """Multipliers of the file's constraint rows from the solver's y
        (ranged rows: the sum over their two halves), in the sign convention
        d(objective in the model's sense) / d(rhs)."""
        out = np.zeros(len(self.row_names))
        for k, (i, sgn) in enumerate(self.row_origin):
            out[i] += sgn * y[k]
        return -out if self.maximize else out


def _open(path):
    if str(path).endswith(".gz"):
        return gzip.open(path, "rt")
    return open(path, "r")


def _num(tok: str, where: str) -> float:
    try:
        return float(tok)
    except ValueError:
        raise ValueError(f"MPS: bad number {tok!r} in {where}") from None


def read_mps(path) -> MPSModel:
    """Reads a (free or blank-free fixed) MPS file, optionally gzip-compressed."""
    with _open(path) as f:
        return parse_mps(f.read())


def parse_mps(text: str) -> MPSModel:
    name = ""
    section = None
    maximize = False
    row_kind: Dict[str, str] = {}
    row_order: List[str] = []
    obj: Optional[str] = None
    col_index: Dict[str, int] = {}
    col_names: List[str] = []
    entries: List[Tuple[int, int, float]] = []  # (row, col, value) over constraint rows
    cost: Dict[int, float] = {}
    rhs: Dict[str, float] = {}
    rng: Dict[str, float] = {}
    lo: Dict[int, float] = {}
    up: Dict[int, float] = {}
    obj_const = 0.0
    row_id: Dict[str, int] = {}
    for lineno, raw in enumerate(text.splitlines(), 1):
        line = raw.rstrip()
        if not line or line.startswith("*"):
            continue
        tok = line.split()
        head = tok[0].upper()
        if not raw[0].isspace():
            # section header
            if head == "NAME":
                name = " ".join(tok[1:])
                section = None
                continue
            if head == "OBJSENSE":
                section = "OBJSENSE"
                if len(tok) > 1:
                    maximize = tok[1].upper() in ("MAX", "MAXIMIZE")
                continue
            if head in ("ROWS", "COLUMNS", "RHS", "RANGES", "BOUNDS"):
                section = head
                continue
            if head == "ENDATA":
                break
            raise ValueError(f"MPS line {lineno}: unknown section {tok[0]!r}")
        where = f"line {lineno}"
        if section == "OBJSENSE":
            maximize = head in ("MAX", "MAXIMIZE")
        elif section == "ROWS":
            if len(tok) != 2:
                raise ValueError(f"MPS {where}: ROWS entry needs a type and a name")
            kind, rname = head, tok[1]
            if kind not in ("N", "G", "L", "E"):
                raise ValueError(f"MPS {where}: bad row type {tok[0]!r}")
            if rname in row_kind:
                raise ValueError(f"MPS {where}: duplicate row {rname!r}")
            row_kind[rname] = kind
            if kind == "N":
                if obj is None:
                    obj = rname
            else:
                row_id[rname] = len(row_order)
                row_order.append(rname)
        elif section == "COLUMNS":
            if len(tok) >= 3 and tok[1].upper() == "'MARKER'":
                continue  # integrality markers: the LP relaxation is read
            if len(tok) not in (3, 5):
                raise ValueError(f"MPS {where}: COLUMNS entry needs 3 or 5 fields")
            cname = tok[0]
            j = col_index.get(cname)
            if j is None:
                j = col_index[cname] = len(col_names)
                col_names.append(cname)
            for rname, sval in zip(tok[1::2], tok[2::2]):
                v = _num(sval, where)
                kind = row_kind.get(rname)
                if kind is None:
                    raise ValueError(f"MPS {where}: unknown row {rname!r}")
                if kind == "N":
                    if rname == obj:
                        cost[j] = cost.get(j, 0.0) + v
                else:
                    entries.append((row_id[rname], j, v))
        elif section in ("RHS", "RANGES"):
            # an optional set name precedes (row, value) pairs
            pairs = tok[1:] if len(tok) % 2 == 1 else tok
            for rname, sval in zip(pairs[0::2], pairs[1::2]):
                v = _num(sval, where)
                kind = row_kind.get(rname)
                if kind is None:
                    raise ValueError(f"MPS {where}: unknown row {rname!r}")
                if section == "RHS":
                    if kind == "N":
                        if rname == obj:
                            obj_const = -v
                    else:
                        rhs[rname] = v
                else:
                    if kind == "N":
                        raise ValueError(f"MPS {where}: RANGES on the objective row")
                    rng[rname] = v
        elif section == "BOUNDS":
            btype = head
            if btype in ("FR", "MI", "PL", "BV"):
                # [type, set, column] or [type, column]; a value after BV is ignored
                if len(tok) not in (2, 3, 4):
                    raise ValueError(f"MPS {where}: bad BOUNDS entry")
                cname = tok[2] if len(tok) >= 3 else tok[1]
                sval = None
            else:
                # [type, set, column, value] or [type, column, value]
                if len(tok) == 4:
                    cname, sval = tok[2], tok[3]
                elif len(tok) == 3:
                    cname, sval = tok[1], tok[2]
                else:
                    raise ValueError(f"MPS {where}: bad BOUNDS entry")
            j = col_index.get(cname)
            if j is None:
                raise ValueError(f"MPS {where}: unknown column {cname!r}")
            if btype in ("UP", "UI"):
                v = _num(sval, where)
                up[j] = v
                if v < 0.0 and j not in lo:
                    lo[j] = -math.inf
            elif btype in ("LO", "LI"):
                lo[j] = _num(sval, where)
            elif btype == "FX":
                v = _num(sval, where)
                lo[j] = up[j] = v
            elif btype == "FR":
                lo[j], up[j] = -math.inf, math.inf
            elif btype == "MI":
                lo[j] = -math.inf
            elif btype == "PL":
                up[j] = math.inf
            elif btype == "BV":
                lo[j], up[j] = 0.0, 1.0
            else:
                raise ValueError(f"MPS {where}: unsupported bound type {tok[0]!r}")
        else:
            raise ValueError(f"MPS {where}: data outside a section")
    n = len(col_names)
    if n == 0:
        raise ValueError("MPS: no columns")
    # constraint rows of the file -> solver rows
    nr = len(row_order)
    per_row: List[List[Tuple[int, float]]] = [[] for _ in range(nr)]
    for i, j, v in entries:
        per_row[i].append((j, v))
    rows_out: List[Tuple[List[Tuple[int, float]], int, float, int, int]] = []  # (entries, type, rhs, origin, sign)
    for i, rname in enumerate(row_order):
        kind = row_kind[rname]
        r = rhs.get(rname, 0.0)
        ent = per_row[i]
        neg = [(j, -v) for j, v in ent]
        if rname in rng:
            R = rng[rname]
            if kind == "G":
                lo_r, hi_r = r, r + abs(R)
            elif kind == "L":
                lo_r, hi_r = r - abs(R), r
            else:
                lo_r, hi_r = (r, r + R) if R >= 0 else (r + R, r)
            if lo_r == hi_r:
                rows_out.append((ent, EQ, lo_r, i, 1))
            else:
                rows_out.append((ent, GE, lo_r, i, 1))
                rows_out.append((neg, GE, -hi_r, i, -1))
        elif kind == "G":
            rows_out.append((ent, GE, r, i, 1))
        elif kind == "L":
            rows_out.append((neg, GE, -r, i, -1))
        else:
            rows_out.append((ent, EQ, r, i, 1))
    m = len(rows_out)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    for k, row in enumerate(rows_out):
        rowptr[k + 1] = rowptr[k] + len(row[0])
    col = np.empty(int(rowptr[-1]), dtype=np.int32)
    val = np.empty(int(rowptr[-1]), dtype=np.float64)
    for k, row in enumerate(rows_out):
        a, b = int(rowptr[k]), int(rowptr[k + 1])
        if b > a:
            col[a:b] = [j for j, _ in row[0]]
            val[a:b] = [v for _, v in row[0]]
    c = np.zeros(n)
    for j, v in cost.items():
        c[j] = v
    l = np.zeros(n)
    u = np.full(n, math.inf)
    for j, v in lo.items():
        l[j] = v
    for j, v in up.items():
        u[j] = v
    offset = obj_const
    if maximize:
        c = -c
        offset = -offset
    return MPSModel(n=n, m=m, rowptr=rowptr, col=col, val=val,
                    row_type=np.array([row[1] for row in rows_out], dtype=np.uint8),
                    rhs=np.array([row[2] for row in rows_out], dtype=np.float64), c=c, l=l, u=u, name=name,
                    col_names=col_names, row_origin=[(row[3], row[4]) for row in rows_out],
                    row_names=list(row_order), obj_name=obj or "", obj_offset=offset, maximize=maximize)


def _fmt(v: float) -> str:
    return repr(float(v))


def write_mps(lp, path, name: str = "LP") -> None:
    """Writes an LP in the solver's form (rows G / E as given, bounds as
    given) as free MPS; reading it back gives the same arrays."""
    n, m = int(lp.n), int(lp.m)
    rowptr = np.asarray(lp.rowptr)
    col = np.asarray(lp.col)
    val = np.asarray(lp.val)
    rt = np.asarray(lp.row_type)
    by_col: List[List[Tuple[int, float]]] = [[] for _ in range(n)]
    for i in range(m):
        for k in range(int(rowptr[i]), int(rowptr[i + 1])):
            by_col[int(col[k])].append((i, float(val[k])))
    opener = gzip.open if str(path).endswith(".gz") else open
    with opener(path, "wt") as f:
        f.write(f"NAME {name}\nROWS\n N OBJ\n")
        for i in range(m):
            f.write(f" {'G' if rt[i] == GE else 'E'} R{i}\n")
        f.write("COLUMNS\n")
        for j in range(n):
            if lp.c[j] != 0.0:
                f.write(f" C{j} OBJ {_fmt(lp.c[j])}\n")
            for i, v in by_col[j]:
                f.write(f" C{j} R{i} {_fmt(v)}\n")
            if lp.c[j] == 0.0 and not by_col[j]:
                f.write(f" C{j} OBJ 0.0\n")
        f.write("RHS\n")
        for i in range(m):
            if lp.rhs[i] != 0.0:
                f.write(f" RHS R{i} {_fmt(lp.rhs[i])}\n")
        f.write("BOUNDS\n")
        for j in range(n):
            lj, uj = float(lp.l[j]), float(lp.u[j])
            if lj == -math.inf and uj == math.inf:
                f.write(f" FR BND C{j}\n")
                continue
            if lj == uj:
                f.write(f" FX BND C{j} {_fmt(lj)}\n")
                continue
            if lj == -math.inf:
                f.write(f" MI BND C{j}\n")
            elif lj != 0.0:
                f.write(f" LO BND C{j} {_fmt(lj)}\n")
            if uj != math.inf:
                f.write(f" UP BND C{j} {_fmt(uj)}\n")
        f.write("ENDATA\n")
