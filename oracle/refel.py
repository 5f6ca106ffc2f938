"""Reference-element matrices by exact rational integration.

Sec. 3.1 builds the spatial DG space from a nodal Lagrange basis mapped
affinely from a reference simplex, with quadratures exact to degree 2k so
that every element matrix is an exact polynomial integral (the quadrature
assumption of Sec. 3.1).  Here every basis function is a polynomial in the
barycentric coordinates lambda_0..lambda_d with Fraction coefficients and is
integrated with the simplex monomial formula

    int_K prod_i lambda_i^a_i dx = |K| * d! * prod_i a_i! / (|a| + d)!

so the matrices below are exact rationals, rounded once to float64.

Node sets (the ordering the whole oracle uses):
  P1: the d+1 vertices.
  P2 (triangles): vertices 0,1,2, then edge midpoints (0,1), (1,2), (2,0).
Face k is the facet opposite vertex k; its nodes are the nodes with
lambda_k = 0, in ascending local index.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import factorial

import numpy as np

Poly = dict  # exponent tuple over (lambda_0..lambda_d) -> Fraction


def _mul(p: Poly, q: Poly) -> Poly:
    out: Poly = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, Fraction(0)) + ca * cb
    return {e: c for e, c in out.items() if c != 0}


def _add(p: Poly, q: Poly, s=Fraction(1)) -> Poly:
    out = dict(p)
    for e, c in q.items():
        out[e] = out.get(e, Fraction(0)) + s * c
    return {e: c for e, c in out.items() if c != 0}


def _lam(i: int, d: int) -> Poly:
    e = [0] * (d + 1)
    e[i] = 1
    return {tuple(e): Fraction(1)}


def _const(c, d: int) -> Poly:
    return {tuple([0] * (d + 1)): Fraction(c)}


def _dlam(p: Poly, i: int) -> Poly:
    """Partial derivative with respect to lambda_i (treating all lambdas as independent)."""
    out: Poly = {}
    for e, c in p.items():
        if e[i] > 0:
            e2 = list(e)
            e2[i] -= 1
            out[tuple(e2)] = out.get(tuple(e2), Fraction(0)) + c * e[i]
    return out


def _dxi(p: Poly, beta: int) -> Poly:
    """d/dxi_beta with lambda_0 = 1 - sum xi, lambda_beta = xi_beta (beta = 1..d)."""
    return _add(_dlam(p, beta), _dlam(p, 0), Fraction(-1))


def _int_simplex(p: Poly, dim: int, drop: int | None = None) -> Fraction:
    """Integral over a simplex of unit measure of p, with lambda_drop set to 0
    when integrating over a facet (dim is then the facet dimension)."""
    tot = Fraction(0)
    for e, c in p.items():
        if drop is not None:
            if e[drop] != 0:
                continue
            e = tuple(x for i, x in enumerate(e) if i != drop)
        num = 1
        for a in e:
            num *= factorial(a)
        tot += c * Fraction(factorial(dim) * num, factorial(sum(e) + dim))
    return tot


def node_barycentric(dim: int, order: int) -> list[tuple]:
    """Barycentric coordinates of the nodes, as Fractions, in the oracle's order."""
    verts = []
    for k in range(dim + 1):
        b = [Fraction(0)] * (dim + 1)
        b[k] = Fraction(1)
        verts.append(tuple(b))
    if order == 1:
        return verts
    if order == 2 and dim == 2:
        mids = []
        for (i, j) in ((0, 1), (1, 2), (2, 0)):
            b = [Fraction(0)] * 3
            b[i] = b[j] = Fraction(1, 2)
            mids.append(tuple(b))
        return verts + mids
    raise ValueError("supported elements: P1 (d=2,3) and P2 (d=2)")


def basis(dim: int, order: int) -> list[Poly]:
    if order == 1:
        return [_lam(k, dim) for k in range(dim + 1)]
    if order == 2 and dim == 2:
        out = [_mul(_lam(k, 2), _add(_mul(_const(2, 2), _lam(k, 2)), _const(-1, 2)))
               for k in range(3)]
        for (i, j) in ((0, 1), (1, 2), (2, 0)):
            out.append(_mul(_const(4, 2), _mul(_lam(i, 2), _lam(j, 2))))
        return out
    raise ValueError("supported elements: P1 (d=2,3) and P2 (d=2)")


def _eval(p: Poly, lam) -> Fraction:
    tot = Fraction(0)
    for e, c in p.items():
        t = c
        for x, a in zip(lam, e):
            t *= x ** a
        tot += t
    return tot


@lru_cache(maxsize=None)
def reference(dim: int, order: int):
    """Return a dict with exact-then-rounded reference matrices.

    mass[a][b]      = (1/|K|) int_K phi_a phi_b      (measure-normalised)
    stiff[beta][a][b] = int_ref phi_b d(phi_a)/d(xi_beta)  over the reference
                      simplex of measure 1/d!
    face_mass[k][a][b] = (1/|F_k|) int_{F_k} phi_a phi_b  (facet-normalised)
    face_nodes[k]   = local nodes on facet k (ascending)
    """
    phis = basis(dim, order)
    nodes = node_barycentric(dim, order)
    npn = len(phis)
    # nodal property check: phi_a(x_b) = delta_ab
    for a, p in enumerate(phis):
        for b, lam in enumerate(nodes):
            if _eval(p, lam) != (1 if a == b else 0):
                raise AssertionError("basis is not nodal")
    mass = np.zeros((npn, npn))
    for a in range(npn):
        for b in range(npn):
            mass[a, b] = float(_int_simplex(_mul(phis[a], phis[b]), dim))
    vol_ref = Fraction(1, factorial(dim))
    stiff = np.zeros((dim, npn, npn))
    for beta in range(dim):
        for a in range(npn):
            da = _dxi(phis[a], beta + 1)
            for b in range(npn):
                stiff[beta, a, b] = float(vol_ref * _int_simplex(_mul(phis[b], da), dim))
    face_nodes = []
    face_mass = np.zeros((dim + 1, npn, npn))
    for k in range(dim + 1):
        fn = [a for a, lam in enumerate(nodes) if lam[k] == 0]
        face_nodes.append(fn)
        for a in fn:
            for b in fn:
                face_mass[k, a, b] = float(_int_simplex(_mul(phis[a], phis[b]), dim - 1, drop=k))
    return {
        "dim": dim, "order": order, "n_p": npn, "n_fp": len(face_nodes[0]),
        "mass": mass, "stiff": stiff, "face_mass": face_mass,
        "face_nodes": face_nodes,
        "node_bary": np.array([[float(x) for x in lam] for lam in nodes]),
    }
