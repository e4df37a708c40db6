"""Quadrature rules used by the oracle (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Gauss-Legendre on [0, 1] from numpy's Legendre module.
* Radon's seven-point rule of degree 5 on a triangle: the "7-point Gauss
  quadrature" used for regular (non-touching) near-field pairs.
* Collapsed (Duffy) Gauss rules on a triangle, exact for a stated total degree;
  used for the leaf matrices of eq. (leafV), whose integrands are tensor
  polynomials of degree m-1 per coordinate, i.e. total degree 3(m-1).
* Sauter-Schwab rules for identical triangles, triangles with a common edge and
  triangles with a common vertex (the paper's experiments use Sauter-Schwab
  quadrature for the singular Galerkin integrals).  Each rule maps the 4D unit
  cube onto T x T, T = {0 <= x2 <= x1 <= 1}, by relative coordinates followed by
  Duffy transformations, so that the 1/|x-y| singularity is cancelled by the
  Jacobian.  The triangles are parametrised as chi(x) = P0 + x1 (P1-P0) + x2 (P2-P1);
  a common edge is P0P1 in both triangles, a common vertex is P0 in both.
"""
from __future__ import annotations

import math

import numpy as np


def gauss_legendre01(q: int):
    """q-point Gauss-Legendre nodes and weights on [0, 1] (exact to degree 2q-1)."""
    t, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (t + 1.0), 0.5 * w


def radon7():
    """Radon's degree-5 rule: barycentric coordinates (7,3) and weights summing to 1."""
    s15 = math.sqrt(15.0)
    a1, b1 = (6.0 - s15) / 21.0, (9.0 + 2.0 * s15) / 21.0
    a2, b2 = (6.0 + s15) / 21.0, (9.0 - 2.0 * s15) / 21.0
    w0, w1, w2 = 9.0 / 40.0, (155.0 - s15) / 1200.0, (155.0 + s15) / 1200.0
    lam = np.array([
        [1 / 3, 1 / 3, 1 / 3],
        [b1, a1, a1], [a1, b1, a1], [a1, a1, b1],
        [b2, a2, a2], [a2, b2, a2], [a2, a2, b2],
    ])
    w = np.array([w0, w1, w1, w1, w2, w2, w2])
    return lam, w


def collapsed_triangle(q: int):
    """Collapsed Gauss rule on a triangle, exact to total degree 2q-2.

    Returns barycentric coordinates (q*q, 3) and weights summing to 1.  The
    standard simplex {u, v >= 0, u + v <= 1} is reached from the unit square by
    u = s, v = t (1 - s) with Jacobian (1 - s).
    """
    s, ws = gauss_legendre01(q)
    t, wt = gauss_legendre01(q)
    S, Tt = np.meshgrid(s, t, indexing="ij")
    W = np.outer(ws, wt) * (1.0 - S) * 2.0  # reference area 1/2 -> weights sum to 1
    u = S.ravel()
    v = (Tt * (1.0 - S)).ravel()
    lam = np.stack([1.0 - u - v, u, v], axis=1)
    return lam, W.ravel()


def exact_rule_for_degree(deg: int):
    """Smallest collapsed Gauss rule exact to total degree `deg`."""
    q = max(1, math.ceil((deg + 2) / 2))
    return collapsed_triangle(q)


# ---------------------------------------------------------------- Sauter-Schwab
def _cube4(q: int):
    t, w = gauss_legendre01(q)
    xi, e1, e2, e3 = (a.ravel() for a in np.meshgrid(t, t, t, t, indexing="ij"))
    W = np.einsum("a,b,c,d->abcd", w, w, w, w).ravel()
    return xi, e1, e2, e3, W


def sauter_schwab(case: str, q: int):
    """Sauter-Schwab rule on T x T for case in {'identical', 'edge', 'vertex'}.

    Returns (xhat, yhat, weight): xhat, yhat of shape (M, 2) in reference
    coordinates of T = {0 <= x2 <= x1 <= 1} and weights (M,) whose sum is
    |T|^2 = 1/4.  Gauss-Legendre of order q in each of the four variables.
    """
    xi, e1, e2, e3, W = _cube4(q)
    pairs = []
    if case == "identical":
        J = xi ** 3 * e1 ** 2 * e2
        pairs = [
            ((xi, xi * (1 - e1 + e1 * e2)), (xi * (1 - e1 * e2 * e3), xi * (1 - e1)), J),
            ((xi * (1 - e1 * e2 * e3), xi * (1 - e1)), (xi, xi * (1 - e1 + e1 * e2)), J),
            ((xi, xi * e1 * (1 - e2 + e2 * e3)), (xi * (1 - e1 * e2), xi * e1 * (1 - e2)), J),
            ((xi * (1 - e1 * e2), xi * e1 * (1 - e2)), (xi, xi * e1 * (1 - e2 + e2 * e3)), J),
            ((xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3)), (xi, xi * e1 * (1 - e2)), J),
            ((xi, xi * e1 * (1 - e2)), (xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3)), J),
        ]
    elif case == "edge":
        J1 = xi ** 3 * e1 ** 2
        J = xi ** 3 * e1 ** 2 * e2
        pairs = [
            ((xi, xi * e1 * e3), (xi * (1 - e1 * e2), xi * e1 * (1 - e2)), J1),
            ((xi, xi * e1), (xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3)), J),
            ((xi * (1 - e1 * e2), xi * e1 * (1 - e2)), (xi, xi * e1 * e2 * e3), J),
            ((xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3)), (xi, xi * e1), J),
            ((xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3)), (xi, xi * e1 * e2), J),
        ]
    elif case == "vertex":
        J = xi ** 3 * e2
        pairs = [
            ((xi, xi * e1), (xi * e2, xi * e2 * e3), J),
            ((xi * e2, xi * e2 * e3), (xi, xi * e1), J),
        ]
    else:
        raise ValueError(case)
    X = np.concatenate([np.stack(p[0], 1) for p in pairs], 0)
    Y = np.concatenate([np.stack(p[1], 1) for p in pairs], 0)
    Wt = np.concatenate([W * p[2] for p in pairs], 0)
    return X, Y, Wt


def chi(P: np.ndarray, xhat: np.ndarray) -> np.ndarray:
    """Affine map of T = {0<=x2<=x1<=1} onto triangle P = (P0, P1, P2): P0 + x1 (P1-P0) + x2 (P2-P1)."""
    return P[0] + xhat[:, :1] * (P[1] - P[0]) + xhat[:, 1:2] * (P[2] - P[1])
