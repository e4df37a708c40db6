"""Pins for the oracle's algebraic recompression of G-tilde (orthogonalised,
truncated nested bases) against what the construction must satisfy:
exactness without truncation, orthonormal nested bases, symmetry, and the
Frobenius error bound by the discarded weights."""
import numpy as np
import pytest

import h2_inputs as I
from oracle.recompress import Recompressed
from tests.oracle_cache import cube, sphere

CASES = [lambda: sphere(3, 4, 32), lambda: cube(8, 3, 32)]


@pytest.mark.parametrize("H", CASES)
def test_orthogonalisation_is_exact(H):
    """eps = 0 only changes the bases: the represented matrix is G-tilde."""
    H = H()
    C = Recompressed(H, 0.0)
    G0 = H.dense_Gtilde()
    assert np.abs(C.dense() - G0).max() <= 1e-13 * np.abs(G0).max()
    assert C.discarded == 0.0


@pytest.mark.parametrize("H", CASES)
@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_bases_orthonormal_and_nested(H, eps):
    H = H()
    C = Recompressed(H, eps)
    for c in H.tree.clusters[:: max(1, len(H.tree.clusters) // 25)]:
        B = C.Vbar(c)
        r = C.rank[c.id]
        assert B.shape == (len(c.idx), r)
        if r:
            assert np.abs(B.T @ B - np.eye(r)).max() <= 1e-12


@pytest.mark.parametrize("H", CASES)
def test_truncation_error_bound(H):
    """||G~ - G~'||_F^2 <= 2 * discarded, the error falls with eps, ranks do not grow."""
    H = H()
    G0 = H.dense_Gtilde()
    errs, ranks = [], []
    for eps in (1e-1, 1e-2, 1e-3, 1e-4, 1e-6):
        C = Recompressed(H, eps)
        D = C.dense()
        err = np.linalg.norm(D - G0)
        assert err ** 2 <= 2.0 * C.discarded * (1 + 1e-9) + (1e-13 * np.linalg.norm(G0)) ** 2, eps
        assert np.abs(D - D.T).max() <= 1e-13 * np.abs(D).max()
        errs.append(err)
        ranks.append(C.max_rank)
    assert all(a >= b for a, b in zip(errs, errs[1:]))
    assert all(a <= b for a, b in zip(ranks, ranks[1:]))
    assert errs[-1] <= 1e-5 * np.linalg.norm(G0)
    assert ranks[0] < H.k


@pytest.mark.parametrize("H", CASES)
def test_three_phase_product_matches_dense(H):
    H = H()
    C = Recompressed(H, 1e-3)
    x = I.random_vector(H.mesh.n, 3, "normal")
    yd = C.dense() @ x
    assert np.linalg.norm(C.matvec(x) - yd) <= 1e-13 * np.linalg.norm(yd)


def test_rank_cap():
    H = sphere(3, 4, 32)
    C = Recompressed(H, 0.0, max_rank=12)
    assert C.max_rank == 12
    G0 = H.dense_Gtilde()
    assert np.linalg.norm(C.dense() - G0) ** 2 <= 2.0 * C.discarded * (1 + 1e-9) + (1e-13 * np.linalg.norm(G0)) ** 2
