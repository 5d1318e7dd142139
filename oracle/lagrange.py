"""Lagrange P_p basis on a tetrahedron with exact integration (oracle).

The paper discretises with hierarchic basis functions of arbitrary order (Sec.
1 and Sec. 7, p = 1, 2, 3).  Any basis of the complete P_p space on each tet
spans the same conforming space, so the discrete solution, and everything
homogenised from it, does not depend on the basis.  The oracle therefore uses
the textbook equispaced Lagrange basis, written in barycentric coordinates:

    phi_alpha(lam) = prod_i prod_{k < alpha_i} (p lam_i - k) / (k + 1),   |alpha| = p.

Integrals use the exact barycentric monomial formulas
    (1/|T|) int_T lam^b dV = 3! b0! b1! b2! b3! / (|b| + 3)!
    (1/|F|) int_F lam^b dA = 2! b0! b1! b2!    / (|b| + 2)!
evaluated in rational arithmetic, so no quadrature rule is involved.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from functools import lru_cache
from math import factorial

import numpy as np


def multi_indices(p: int):
    """All (a0, a1, a2, a3) with a0+a1+a2+a3 = p, lexicographic order."""
    return [a for a in itertools.product(range(p + 1), repeat=4) if sum(a) == p]


def _pmul(a, b):
    out = {}
    for ea, ca in a.items():
        for eb, cb in b.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0) + ca * cb
    return {e: c for e, c in out.items() if c != 0}


def _pdiff(a, i):
    out = {}
    for e, c in a.items():
        if e[i] > 0:
            e2 = list(e)
            e2[i] -= 1
            e2 = tuple(e2)
            out[e2] = out.get(e2, 0) + c * e[i]
    return out


def _vol_int(poly):
    s = Fraction(0)
    for e, c in poly.items():
        s += c * Fraction(6 * factorial(e[0]) * factorial(e[1]) * factorial(e[2]) * factorial(e[3]),
                          factorial(sum(e) + 3))
    return s


def _face_int(poly, opposite):
    s = Fraction(0)
    for e, c in poly.items():
        if e[opposite] != 0:
            continue
        r = [e[i] for i in range(4) if i != opposite]
        s += c * Fraction(2 * factorial(r[0]) * factorial(r[1]) * factorial(r[2]), factorial(sum(r) + 2))
    return s


def basis_polys(p: int):
    polys = []
    for alpha in multi_indices(p):
        poly = {(0, 0, 0, 0): Fraction(1)}
        for i in range(4):
            for k in range(alpha[i]):
                e = [0, 0, 0, 0]
                e[i] = 1
                factor = {tuple(e): Fraction(p, k + 1)}
                if k:
                    factor[(0, 0, 0, 0)] = Fraction(-k, k + 1)
                poly = _pmul(poly, factor)
        polys.append(poly)
    return polys


@lru_cache(maxsize=None)
def reference_tables(p: int):
    """Geometry-free tables of the P_p Lagrange basis (float64).

    Returns dict with
      nodes : [nn, 4] multi-indices alpha
      S     : [4, 4, nn, nn]  (1/|T|) int d(phi_a)/d(lam_i) d(phi_b)/d(lam_j) dV
      W     : [nn]            (1/|T|) int phi_a dV
      Wd    : [4, nn]         (1/|T|) int d(phi_a)/d(lam_i) dV
      F     : [4, nn]         (1/|F_o|) int_{F_o} phi_a dA, F_o the face opposite vertex o
    """
    polys = basis_polys(p)
    nn = len(polys)
    d = [[_pdiff(ph, i) for i in range(4)] for ph in polys]
    S = np.zeros((4, 4, nn, nn))
    for i in range(4):
        for j in range(4):
            for a in range(nn):
                for b in range(a, nn):
                    v = float(_vol_int(_pmul(d[a][i], d[b][j])))
                    S[i, j, a, b] = v
                    S[j, i, b, a] = v
    W = np.array([float(_vol_int(ph)) for ph in polys])
    Wd = np.array([[float(_vol_int(d[a][i])) for a in range(nn)] for i in range(4)])
    F = np.array([[float(_face_int(ph, o)) for ph in polys] for o in range(4)])
    return dict(nodes=np.array(multi_indices(p)), S=S, W=W, Wd=Wd, F=F)


def eval_basis(p: int, lam):
    """Values of all basis functions at barycentric points lam [m, 4] -> [m, nn]."""
    polys = basis_polys(p)
    lam = np.asarray(lam, float)
    out = np.zeros((lam.shape[0], len(polys)))
    for a, poly in enumerate(polys):
        for e, c in poly.items():
            out[:, a] += float(c) * np.prod(lam ** np.array(e), axis=1)
    return out
