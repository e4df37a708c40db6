"""Pins for the oracle's Krylov solvers: library solves and the unit-sphere solution."""
import numpy as np

import h2_inputs as I
from oracle.krylov import cg, gmres
from tests.oracle_cache import sphere


def test_cg_and_gmres_against_direct_solve():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((80, 80))
    S = A @ A.T + 80 * np.eye(80)
    N = A + 25 * np.eye(80)
    C = N + 1j * rng.standard_normal((80, 80))
    C = C + C.T
    b = rng.standard_normal(80)
    bc = b + 1j * rng.standard_normal(80)
    z, _, _ = cg(lambda v: S @ v, b, 1e-13)
    assert np.linalg.norm(z - np.linalg.solve(S, b)) < 1e-11 * np.linalg.norm(z)
    z, _, _ = gmres(lambda v: N @ v, b, 10, 1e-13, 2000)
    assert np.linalg.norm(z - np.linalg.solve(N, b)) < 1e-11 * np.linalg.norm(z)
    z, _, _ = gmres(lambda v: C @ v, bc, 20, 1e-13, 4000)
    assert np.linalg.norm(z - np.linalg.solve(C, bc)) < 1e-10 * np.linalg.norm(z)


def test_sphere_solution_is_one():
    """G z = b with b_i = |T_i| on the unit sphere: z ~ 1 (V 1 = 1)."""
    H = sphere(3, 3, 32)
    b = H.mesh.area.copy()
    for solver in ("cg", "gmres"):
        if solver == "cg":
            z, it, hist = cg(H.matvec, b, 1e-8, 500)
        else:
            z, it, hist = gmres(H.matvec, b, 50, 1e-8, 500)
        r = b - H.matvec(z)
        assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(b)
        assert np.abs(z - 1).max() < 2e-2
