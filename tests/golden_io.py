"""Readers for the transcribed paper fixtures under tests/golden/."""
import os
import re

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def table_a1():
    """Velocity vectors of Table A-1 expanded to a [19, 3] integer array."""
    e = np.full((19, 3), 99, dtype=np.int64)
    for line in _rows("table_a1_d3q19.txt"):
        idx, vec = [s.strip() for s in line.split("|")]
        ids = [int(s) for s in idx.split(",")]
        comps = [c.strip() for c in vec.strip("()").split(",")]
        for k, a in enumerate(ids):
            v = []
            for c in comps:
                if c.startswith("+-"):
                    v.append(int(c[2:]) * (1 if k == 0 else -1))
                elif c.startswith("-+"):
                    v.append(int(c[2:]) * (-1 if k == 0 else 1))
                else:
                    v.append(int(c))
            e[a] = v
    return e


def moment_sums():
    """List of (equation, moment, coefficient vector[19], revised-set)."""
    out = []
    for line in _rows("eq10_eq11_moment_sums.txt"):
        eq, mom, expr = [s.strip() for s in line.split("|")]
        coef = np.zeros(19, dtype=np.int64)
        revised = set()
        for sign, tilde, idx in re.findall(r"([+-]?)\s*(~?)f(\d+)", expr.replace(" ", "")):
            a = int(idx)
            coef[a] += -1 if sign == "-" else 1
            if tilde:
                revised.add(a)
        out.append((eq, mom, coef, revised))
    return out


def eq14():
    """(shifted, reversed): shifted = [(a, b, sign, comp)], reversed = [(a, b)]."""
    shifted, reversed_ = [], []
    for line in _rows("eq14_wfb_collision.txt"):
        parts = line.split()
        if parts[0] == "R":
            reversed_.append((int(parts[1]), int(parts[2])))
        elif parts[0] == "C":
            continue
        else:
            shifted.append((int(parts[0]), int(parts[1]), 1 if parts[2] == "+" else -1, parts[3]))
    return shifted, reversed_


def eq14_copies():
    """Eq. 14c's out-pointing diagonals: [(a, b)] meaning f_a* = ~f_b*."""
    return [(int(p[1]), int(p[2])) for p in (line.split() for line in _rows("eq14_wfb_collision.txt"))
            if p[0] == "C"]


def table1():
    out = []
    for line in _rows("table1_cases.txt"):
        case, re_tau, res, mesh, yp, ma = [s.strip() for s in line.split("|")]
        nx, ny, nz = (int(s) for s in mesh.split("x"))
        out.append(dict(case=case, re_tau=float(re_tau), res=int(res), nx=nx, ny=ny, nz=nz,
                        yplus=float(yp), ma=float(ma)))
    return out


def table_b1():
    out = []
    for line in _rows("table_b1_mass.txt"):
        case, rate, order = [s.strip() for s in line.split("|")]
        out.append(dict(case=case, rate=float(rate), order=float(order)))
    return out
