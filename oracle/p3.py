"""Reference P3 Lagrange tetrahedron, built with exact rational arithmetic.

TEST INFRASTRUCTURE ONLY: the oracle package is imported by tests/, the graft smoke
check and the CPU baseline leg of bench.py, never by the product path.

The paper discretises the Helmholtz equation with continuous Lagrange elements of order
3 on tetrahedra (section "Tetrahedral finite element method", text after eq. (1)).
Everything here is a plain definition: basis polynomials in barycentric coordinates and
exact integrals of monomials over the simplex,
    int_T  l^a  = 6|T| a0! a1! a2! a3! / (|a| + 3)!
    int_f  l^a  = 2|f| a0! a1! a2!     / (|a| + 2)!

Local node numbering (20 nodes, shared convention with the solver library):
  0..3    vertices
  4..15   two nodes per edge, edges in order (0,1),(0,2),(0,3),(1,2),(1,3),(2,3);
          for edge (a,b) the first node sits at 2/3 a + 1/3 b, the second at 1/3 a + 2/3 b
  16..19  face nodes; face f is opposite local vertex f
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import factorial

import numpy as np

EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
FACES = tuple(tuple(v for v in range(4) if v != f) for f in range(4))


def node_barycentrics():
    """Barycentric coordinates (Fractions) of the 20 local nodes."""
    pts = []
    for v in range(4):
        pts.append(tuple(Fraction(1 if w == v else 0) for w in range(4)))
    for a, b in EDGES:
        for wa, wb in ((Fraction(2, 3), Fraction(1, 3)), (Fraction(1, 3), Fraction(2, 3))):
            p = [Fraction(0)] * 4
            p[a], p[b] = wa, wb
            pts.append(tuple(p))
    for f in range(4):
        pts.append(tuple(Fraction(0) if w == f else Fraction(1, 3) for w in range(4)))
    return pts


def _mono(*exps):
    return tuple(exps)


def _pmul(p, q):
    out = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0) + ca * cb
    return {e: c for e, c in out.items() if c != 0}


def _lam(a, scale=Fraction(1), shift=Fraction(0)):
    """Polynomial scale*lambda_a + shift."""
    e = [0, 0, 0, 0]
    e[a] = 1
    p = {tuple(e): Fraction(scale)}
    if shift != 0:
        p[(0, 0, 0, 0)] = Fraction(shift)
    return p


@lru_cache(maxsize=None)
def basis():
    """The 20 basis polynomials as dicts {exponent tuple: Fraction}.

    vertex a:                  1/2 l_a (3 l_a - 1)(3 l_a - 2)
    edge (a,b), node near a:   9/2 l_a l_b (3 l_a - 1)
    face (a,b,c):              27 l_a l_b l_c
    """
    out = []
    for a in range(4):
        p = _pmul(_pmul(_lam(a, Fraction(1, 2)), _lam(a, 3, -1)), _lam(a, 3, -2))
        out.append(p)
    for a, b in EDGES:
        out.append(_pmul(_pmul(_lam(a, Fraction(9, 2)), _lam(b)), _lam(a, 3, -1)))
        out.append(_pmul(_pmul(_lam(b, Fraction(9, 2)), _lam(a)), _lam(b, 3, -1)))
    for f in range(4):
        a, b, c = FACES[f]
        out.append(_pmul(_pmul(_lam(a, 27), _lam(b)), _lam(c)))
    return tuple(out)


def evaluate(p, lam):
    """Evaluate a polynomial dict at barycentric point lam (Fractions or floats)."""
    s = 0
    for e, c in p.items():
        t = c
        for k in range(4):
            if e[k]:
                t = t * lam[k] ** e[k]
        s = s + t
    return s


def derivative(p, a):
    out = {}
    for e, c in p.items():
        if e[a] > 0:
            ne = list(e)
            ne[a] -= 1
            out[tuple(ne)] = out.get(tuple(ne), 0) + c * e[a]
    return out


def _int_tet(p):
    """(1/|T|) int_T p  for a polynomial in the 4 barycentrics."""
    s = Fraction(0)
    for e, c in p.items():
        num = 1
        for x in e:
            num *= factorial(x)
        s += c * Fraction(6 * num, factorial(sum(e) + 3))
    return s


def _int_face(p, f):
    """(1/|f|) int_f p over the face opposite vertex f (monomials with l_f drop out)."""
    s = Fraction(0)
    for e, c in p.items():
        if e[f] != 0:
            continue
        num = 1
        for x in e:
            num *= factorial(x)
        s += c * Fraction(2 * num, factorial(sum(e) + 2))
    return s


@lru_cache(maxsize=None)
def mass_exact():
    """Mhat[i][j] = (1/|T|) int_T phi_i phi_j (Fractions, 20 x 20)."""
    B = basis()
    return tuple(tuple(_int_tet(_pmul(B[i], B[j])) for j in range(20)) for i in range(20))


@lru_cache(maxsize=None)
def stiff_exact():
    """Shat[a][b][i][j] = (1/|T|) int_T d phi_i/d l_a * d phi_j / d l_b (Fractions)."""
    B = basis()
    D = [[derivative(B[i], a) for a in range(4)] for i in range(20)]
    return tuple(
        tuple(
            tuple(tuple(_int_tet(_pmul(D[i][a], D[j][b])) for j in range(20)) for i in range(20))
            for b in range(4)
        )
        for a in range(4)
    )


@lru_cache(maxsize=None)
def face_mass_exact(f):
    """Fhat_f[i][j] = (1/|f|) int_f phi_i phi_j on face f (20 x 20, zero off the face)."""
    B = basis()
    return tuple(tuple(_int_face(_pmul(B[i], B[j]), f) for j in range(20)) for i in range(20))


def face_nodes(f):
    """The 10 local nodes lying on face f (opposite vertex f)."""
    lam = node_barycentrics()
    return [i for i in range(20) if lam[i][f] == 0]


def to_float(m):
    return np.array([[float(x) for x in row] for row in m], dtype=np.float64)


@lru_cache(maxsize=None)
def reference_matrices():
    """FP64 copies: Mhat (20,20), Shat (4,4,20,20), Fhat (4,20,20)."""
    M = to_float(mass_exact())
    S = np.array([[to_float(stiff_exact()[a][b]) for b in range(4)] for a in range(4)])
    F = np.array([to_float(face_mass_exact(f)) for f in range(4)])
    return M, S, F


def eval_basis_float(lam):
    """Basis values at barycentric points lam (N, 4) -> (N, 20), FP64."""
    lam = np.asarray(lam, np.float64)
    out = np.empty((lam.shape[0], 20))
    for i, p in enumerate(basis()):
        v = np.zeros(lam.shape[0])
        for e, c in p.items():
            t = np.full(lam.shape[0], float(c))
            for k in range(4):
                if e[k]:
                    t = t * lam[:, k] ** e[k]
            v += t
        out[:, i] = v
    return out
