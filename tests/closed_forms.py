"""Closed forms that pin the oracle from outside (potential theory and calculus).

Nothing here imports the oracle.  Values:
* self-energy of a flat triangle, int_T int_T 1/|x-y|, for side lengths a, b, c
  and area A: (4 A^2 / 3) * sum over the three sides of
  (1/a) ln(((a+b)^2 - c^2) / (b^2 - (c-a)^2)) (cyclic), which gives (3/4) a^3 ln 3
  for the equilateral triangle of side a;
* self-energy of an a x b rectangle: (2/3)(a^3 + b^3 - d^3)
  + 2ab (a ln((b+d)/a) + b ln((a+d)/b)), d = sqrt(a^2 + b^2), which gives
  4 ln(1 + sqrt 2) - (4/3)(sqrt 2 - 1) for the unit square;
* exact monomial moments on the reference triangle: int x^a y^b over
  {x, y >= 0, x + y <= 1} = a! b! / (a + b + 2)!;
* Galerkin products for polynomial kernels (g = 1, x.y, (x.y)^2) with
  piecewise-constant functions, through triangle areas, first and second moments.
"""
import math

import numpy as np


def tri_self_energy(P):
    P0, P1, P2 = (np.asarray(p, float) for p in P)
    l1 = np.linalg.norm(P1 - P0)
    l2 = np.linalg.norm(P2 - P1)
    l3 = np.linalg.norm(P0 - P2)
    A = 0.5 * np.linalg.norm(np.cross(P1 - P0, P2 - P0))

    def term(a, b, c):
        return (1.0 / a) * math.log(((a + b) ** 2 - c ** 2) / (b ** 2 - (c - a) ** 2))

    return 4.0 * A * A / 3.0 * (term(l1, l2, l3) + term(l2, l3, l1) + term(l3, l1, l2))


def rect_self_energy(a, b):
    d = math.hypot(a, b)
    return (2.0 / 3.0) * (a ** 3 + b ** 3 - d ** 3) + 2.0 * a * b * (
        a * math.log((b + d) / a) + b * math.log((a + d) / b))


def simplex_moment(a, b):
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


def tri_geometry(V, T):
    P = V[T]                                     # (n, 3, 3)
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    first = area[:, None] * P.mean(axis=1)       # int_T x
    S = np.einsum("nai,naj->nij", P, P) + np.einsum("ni,nj->nij", P.sum(1), P.sum(1))
    second = area[:, None, None] / 12.0 * S      # int_T x x^T
    return area, first, second


def poly_kernel_product(V, T, kind, x):
    """(G x)_i for g = 1 ('one'), x.y ('bilinear'), (x.y)^2 ('quadratic')."""
    area, first, second = tri_geometry(V, T)
    if kind == "one":
        return area * (area @ x)
    if kind == "bilinear":
        return first @ (first.T @ x)
    if kind == "quadratic":
        M = np.einsum("nij,n->ij", second, x)
        return np.einsum("nij,ij->n", second, M)
    raise ValueError(kind)
