"""Pins for the oracle's H^2 product (Algorithms 1-3) against definitions and closed forms."""
import functools
import math

import numpy as np
import pytest

import h2_inputs as I
from oracle.galerkin import dense_G
from oracle.h2 import H2Oracle
from oracle.kernels import HELMHOLTZ, LAPLACE, TEST_BILINEAR, TEST_ONE, TEST_QUADRATIC, Kernel
from tests.closed_forms import poly_kernel_product
from tests.oracle_cache import cube, sphere


@functools.lru_cache(maxsize=None)
def denseG_sphere(r, kind=LAPLACE, kappa=0.0):
    V, T = I.icosphere(r)
    H = H2Oracle(V, T, Kernel(kind, kappa), m=1, leaf=10 ** 9, build_blocks=False)
    return dense_G(H.mesh, H.g)


@pytest.mark.parametrize("H", [lambda: sphere(3, 3, 32), lambda: cube(8, 3, 32), lambda: sphere(2, 4, 16)])
def test_algorithms_equal_dense_gtilde(H):
    H = H()
    x = I.random_vector(H.mesh.n, 1, "uniform")
    y = H.matvec(x)
    yd = H.dense_Gtilde() @ x
    assert np.linalg.norm(y - yd) <= 1e-14 * np.linalg.norm(yd)
    # accumulate semantics y <- y + G x
    y0 = I.random_vector(H.mesh.n, 7, "normal")
    assert np.linalg.norm(H.matvec(x, y0.copy()) - (y0 + yd)) <= 1e-14 * np.linalg.norm(y0 + yd)


def test_no_admissible_blocks_gives_G():
    """With eta so small that no block is admissible, G-tilde is G itself."""
    V, T = I.icosphere(2)
    H = H2Oracle(V, T, Kernel(), m=2, leaf=16, eta=1e-9)
    assert len(H.adm) == 0
    assert np.array_equal(H.dense_Gtilde(), denseG_sphere(2))


@pytest.mark.parametrize("kind,m,name", [(TEST_ONE, 1, "one"), (TEST_BILINEAR, 2, "bilinear"),
                                         (TEST_QUADRATIC, 3, "quadratic")])
@pytest.mark.parametrize("mesh", ["sphere", "cube"])
def test_polynomial_kernels_closed_form(kind, m, name, mesh):
    V, T = I.icosphere(3) if mesh == "sphere" else I.cube_surface(12)
    H = H2Oracle(V, T, Kernel(kind), m=m, leaf=24, eta=0.5)
    assert len(H.adm) > 0
    x = I.random_vector(H.mesh.n, 5, "normal")
    ref = poly_kernel_product(V, T, name, x)
    assert np.linalg.norm(H.matvec(x) - ref) <= 1e-13 * np.linalg.norm(ref)


def test_symmetry():
    H = sphere(3, 3, 32)
    x = I.random_vector(H.mesh.n, 11, "normal")
    z = I.random_vector(H.mesh.n, 12, "normal")
    Gz, Gx = H.matvec(z), H.matvec(x)
    assert abs(x @ Gz - z @ Gx) <= 1e-14 * np.linalg.norm(x) * np.linalg.norm(Gz)
    A = {(t.id, s.id) for t, s in H.adm}
    for t, s in H.adm[:50]:
        assert np.array_equal(H.S(t, s), H.S(s, t).T)


def test_error_falls_with_order():
    G = denseG_sphere(3)
    x = I.random_vector(1280, 1, "uniform")
    ref = G @ x
    errs = []
    for m in (1, 2, 3, 4):
        H = sphere(3, m, 32)
        errs.append(np.linalg.norm(H.matvec(x) - ref) / np.linalg.norm(ref))
    assert all(errs[i + 1] < errs[i] / 2 for i in range(3)), errs
    assert errs[2] < 1e-3


def test_unit_sphere_identities():
    """Single layer on the unit sphere: V 1 = 1 and V Y_1 = Y_1 / 3; Galerkin: (G 1)_i ~ |T_i|."""
    d1, dz = [], []
    for r in (1, 2, 3):
        V, T = I.icosphere(r)
        G = denseG_sphere(r)
        P = V[T]
        area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
        z = P.mean(1)[:, 2]
        d1.append(np.abs(G @ np.ones(len(T)) - area).max() / area.max())
        dz.append(np.abs(G @ z - area * z / 3).max() / (area * np.abs(z)).max())
    assert d1[0] > d1[1] > d1[2] and d1[2] < 5e-3, d1
    assert dz[0] > dz[1] > dz[2] and dz[2] < 5e-2, dz


def test_helmholtz_sphere_identity():
    kappa = 2.0
    exact = np.exp(1j * kappa) * np.sin(kappa) / kappa
    d = []
    for r in (1, 2, 3):
        V, T = I.icosphere(r)
        G = denseG_sphere(r, HELMHOLTZ, kappa)
        P = V[T]
        area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
        d.append(np.abs(G @ np.ones(len(T)) - exact * area).max() / area.max())
    assert d[0] > d[1] > d[2] and d[2] < 1e-2, d


def test_helmholtz_h2_close_to_dense():
    H = sphere(3, 4, 32, 0.5, HELMHOLTZ, 4.0)
    x = I.random_vector(1280, 1, "uniform")
    ref = denseG_sphere(3, HELMHOLTZ, 4.0) @ x
    y = H.matvec(x)
    assert np.iscomplexobj(y)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-3
    assert np.linalg.norm(y - H.dense_Gtilde() @ x) <= 1e-14 * np.linalg.norm(y)


def test_sampled_rows_match_full_product():
    H = sphere(3, 3, 32)
    x = I.random_vector(H.mesh.n, 1, "uniform")
    y = H.matvec(x)
    ids = [c.id for c in H.tree.leaves[::7]]
    for lid, (rows, val) in H.sampled_rows(x, ids).items():
        assert np.abs(val - y[rows]).max() <= 1e-14 * np.abs(y).max()


def test_sparse_support_rows_match_full_product():
    """Rows computed with the sparse-support forward transformation equal the
    rows of the full product for an x supported on a few leaves."""
    H = sphere(3, 3, 32)
    sup = [c.id for c in H.tree.leaves[3::11]]
    x = np.zeros(H.mesh.n)
    rng = np.random.default_rng(5)
    for lid in sup:
        x[H.tree.clusters[lid].idx] = rng.standard_normal(H.tree.clusters[lid].idx.size)
    y = H.matvec(x)
    ids = [c.id for c in H.tree.leaves[::5]] + sup[:2]
    for lid, (rows, val) in H.sampled_rows(x, ids, support=sup).items():
        assert np.abs(val - y[rows]).max() <= 1e-14 * np.abs(y).max()
