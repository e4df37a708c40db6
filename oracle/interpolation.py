"""Tensor Chebyshev interpolation: points, Lagrange polynomials, V, E, S.  FP64.

TEST INFRASTRUCTURE ONLY.

* Interpolation points in a box (eq. interpolation leaves them open): Chebyshev
  points of the first kind, c + (w/2) cos(pi (2j+1) / (2m)), j = 0..m-1, per
  axis, with multi-index nu = nu_x + m nu_y + m^2 nu_z.  An axis of zero (or
  tiny) width, e.g. a cluster on one face of a cube, is widened to
  w = max(h, 1e-3 diam(tau)) about its centre; only the points use the widened
  box, never the admissibility test.
* Lagrange polynomials l_{tau,nu}: products of 1D Lagrange polynomials.
* Leaf matrices (eq. leafV): v_{tau,i nu} = int_{T_i} l_{tau,nu}, evaluated with
  a triangle rule exact for total degree 3(m-1), the degree of l_{tau,nu}.
* Transfer matrices (eq. transfer): e_{tau', nu' nu} = l_{tau,nu}(xi_{tau',nu'}).
* Coupling matrices (eq. coupling): s_{tau sigma, nu mu} = g(xi_{tau,nu}, xi_{sigma,mu}).
"""
from __future__ import annotations

import math

import numpy as np

from . import quadrature as Q


def axis_points(c, m: int):
    """Per-axis Chebyshev points (3, m) for cluster box c."""
    diam = c.diam()
    j = np.arange(m)
    cosv = np.cos(math.pi * (2.0 * j + 1.0) / (2.0 * m))
    out = np.empty((3, m))
    for d in range(3):
        w = max(float(c.hi[d] - c.lo[d]), 1e-3 * diam)
        ctr = 0.5 * (float(c.lo[d]) + float(c.hi[d]))
        out[d] = ctr + 0.5 * w * cosv
    return out


def tensor_points(c, m: int) -> np.ndarray:
    """Interpolation points xi_{tau,nu}, shape (m^3, 3), x fastest."""
    t = axis_points(c, m)
    iz, iy, ix = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    return np.stack([t[0][ix.ravel()], t[1][iy.ravel()], t[2][iz.ravel()]], 1)


def lagrange_1d(t: np.ndarray, x: np.ndarray) -> np.ndarray:
    """L_j(x) = prod_{i != j} (x - t_i)/(t_j - t_i); returns (len(x), m)."""
    m = t.size
    out = np.ones((x.size, m))
    for j in range(m):
        for i in range(m):
            if i != j:
                out[:, j] *= (x - t[i]) / (t[j] - t[i])
    return out


def lagrange(c, m: int, x: np.ndarray) -> np.ndarray:
    """l_{tau,nu}(x) for points x (N, 3); returns (N, m^3)."""
    t = axis_points(c, m)
    Lx, Ly, Lz = (lagrange_1d(t[d], x[:, d]) for d in range(3))
    return np.einsum("nc,nb,na->ncba", Lz, Ly, Lx).reshape(x.shape[0], m ** 3)


def basis_matrix(c, m: int, mesh, rows: np.ndarray) -> np.ndarray:
    """v_{tau, i nu} = int_{T_i} l_{tau,nu} for i in rows (eq. leafV); shape (len(rows), m^3)."""
    lam, w = Q.exact_rule_for_degree(3 * (m - 1))
    X = np.einsum("qk,nkd->nqd", lam, mesh.P[rows])            # (r, nq, 3)
    L = lagrange(c, m, X.reshape(-1, 3)).reshape(rows.size, lam.shape[0], m ** 3)
    return mesh.area[rows][:, None] * np.einsum("q,rqk->rk", w, L)


def transfer(child, parent, m: int) -> np.ndarray:
    """E_{tau'} with rows nu' (child points) and columns nu (parent polynomials)."""
    return lagrange(parent, m, tensor_points(child, m))


def coupling(t, s, m: int, kernel) -> np.ndarray:
    """S_{tau sigma}[nu, mu] = g(xi_{tau,nu}, xi_{sigma,mu})."""
    X = tensor_points(t, m)
    Y = tensor_points(s, m)
    return kernel(X[:, None, :], Y[None, :, :])
