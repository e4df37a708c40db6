"""Pins for interpolation, leaf matrices (eq. leafV) and transfer matrices (eq. transfer)."""
import numpy as np
import pytest

from oracle import interpolation as IP
from oracle import quadrature as Q
from tests.oracle_cache import cube, sphere


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_chebyshev_points_are_roots(m):
    H = sphere(3, 3, 32)
    c = H.tree.clusters[3]
    t = IP.axis_points(c, m)
    for d in range(3):
        lo, hi = c.lo[d], c.hi[d]
        ref = np.sort(0.5 * (lo + hi) + 0.5 * (hi - lo) * np.polynomial.chebyshev.chebroots([0] * m + [1]))
        assert np.allclose(np.sort(t[d]), ref, atol=1e-15)


@pytest.mark.parametrize("m", [1, 2, 4])
def test_lagrange_partition_of_unity_and_delta(m):
    H = sphere(3, 3, 32)
    c = H.tree.clusters[5]
    xi = IP.tensor_points(c, m)
    L = IP.lagrange(c, m, xi)
    assert np.allclose(L, np.eye(m ** 3), atol=1e-13)
    x = np.random.default_rng(1).uniform(c.lo, c.hi, (50, 3))
    assert np.allclose(IP.lagrange(c, m, x).sum(1), 1.0, atol=1e-13)


def test_leaf_matrix_row_sums_and_exactness():
    H = sphere(3, 4, 32)
    for c in H.tree.leaves[:5]:
        V = H.V(c)
        assert np.allclose(V.sum(1), H.mesh.area[c.idx], rtol=1e-13)
        # an exact rule of higher order gives the same matrix
        lam, w = Q.collapsed_triangle(12)
        X = np.einsum("qk,nkd->nqd", lam, H.mesh.P[c.idx])
        L = IP.lagrange(c, 4, X.reshape(-1, 3)).reshape(c.idx.size, lam.shape[0], 64)
        Vh = H.mesh.area[c.idx][:, None] * np.einsum("q,rqk->rk", w, L)
        assert np.abs(V - Vh).max() < 1e-14 * np.abs(V).max()


@pytest.mark.parametrize("H", [lambda: sphere(3, 4, 32), lambda: cube(16, 3, 32)])
def test_nested_bases(H):
    """eq. (V_nested): V_tau restricted to tau' equals V_tau' E_tau' (to rounding)."""
    H = H()
    for c in H.tree.clusters:
        if c.children:
            Vd = H.V_direct(c)
            Vn = H.Vbar(c)
            assert np.abs(Vd - Vn).max() < 1e-12 * np.abs(Vd).max(), c.id


def test_transfer_reproduces_polynomials():
    H = sphere(3, 4, 32)
    rng = np.random.default_rng(3)
    coef = rng.standard_normal((4, 4, 4))
    p = lambda X: np.polynomial.polynomial.polyval3d(X[:, 0], X[:, 1], X[:, 2], coef)
    for c in H.tree.clusters[1:20]:
        E = H.E(c)
        assert np.allclose(E @ p(IP.tensor_points(c.parent, 4)), p(IP.tensor_points(c, 4)), rtol=1e-10, atol=1e-10)


def test_degenerate_box_padding():
    H = cube(16, 3, 32)
    flat = [c for c in H.tree.clusters if (c.hi - c.lo).min() == 0]
    assert flat, "cube mesh must produce clusters of zero thickness"
    for c in flat[:10]:
        t = IP.axis_points(c, 3)
        assert np.isfinite(t).all() and all(np.unique(t[d]).size == 3 for d in range(3))


@pytest.mark.parametrize("H,m", [(lambda: sphere(3, 4, 32), 4), (lambda: cube(16, 3, 32), 3)])
def test_transfer_is_kronecker_product(H, m):
    """eq. (transfer) with tensor Lagrange polynomials factors per axis:
    E_c = E_z (x) E_y (x) E_x (x fastest), E_d[i][j] = l_j(xi_i) on axis d.  The
    one-dimensional factors are built here from the monomial (Vandermonde) form
    of the Lagrange polynomials, not from the oracle's product formula."""
    H = H()
    for c in H.tree.clusters[1:40]:
        tp, tc = IP.axis_points(c.parent, m), IP.axis_points(c, m)
        F = []
        for d in range(3):
            ctr, half = 0.5 * (tp[d].max() + tp[d].min()), 0.5 * (tp[d].max() - tp[d].min())
            Vp = np.vander((tp[d] - ctr) / half, m, increasing=True)       # Vp[j][k] = t_j^k
            Vc = np.vander((tc[d] - ctr) / half, m, increasing=True)
            F.append(Vc @ np.linalg.inv(Vp))                               # l_j(s_i)
        K = np.kron(F[2], np.kron(F[1], F[0]))
        E = H.E(c)
        assert np.abs(E - K).max() <= 1e-12 * max(1.0, np.abs(E).max()), c.id
