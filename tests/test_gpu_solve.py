"""h2_solve on the GPU: FP64 Krylov solves, mixed precision with FP64
iterative refinement, the unit-sphere solution z = 1 and error reporting.
The final residual is recomputed by the oracle's own product."""
import functools

import numpy as np
import pytest

import h2_inputs as I
from oracle.h2 import H2Oracle
from oracle.kernels import Kernel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05665_amd import h2  # noqa: E402


@functools.lru_cache(maxsize=None)
def oracle(level=3, m=3, leaf=32):
    V, T = I.icosphere(level)
    return H2Oracle(V, T, Kernel(), m=m, leaf=leaf, eta=0.5)


def solve(A, b, **kw):
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    z, info = A.solve(bd, **kw)
    torch.cuda.synchronize()
    return z.cpu().numpy(), info


@pytest.mark.parametrize("method", ["cg", "gmres"])
def test_fp64_solve_unit_sphere(method):
    H = oracle()
    b = H.mesh.area.copy()
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=3, leaf=32, eta=0.5, storage="f64")
    try:
        z, info = solve(A, b, method=method, rtol=1e-8, maxit=500, restart=50)
    finally:
        A.close()
    assert info["converged"] and info["rel_residual"] <= 1e-8
    r = b - H.matvec(z)
    assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(b)
    assert np.abs(z - 1).max() < 2e-2


@pytest.mark.parametrize("storage,tol", [("f32", 1e-6), ("f32_sbf16", 5e-3)])
def test_mixed_precision_refinement(storage, tol):
    """FP32 (or BF16 coupling) inner solves, FP64 outer residuals: the result
    solves the stored operator to 1e-8 and is within the storage rounding of the
    FP64 solution (measured with the oracle's FP64 product)."""
    H = oracle()
    b = H.mesh.area.copy()
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=3, leaf=32, eta=0.5, storage="f64")
    B = h2.H2Matrix(H.mesh.V, H.mesh.T, order=3, leaf=32, eta=0.5, storage=storage)
    try:
        z64, i64 = solve(A, b, method="cg", rtol=1e-8, maxit=500)
        zm, im = solve(B, b, method="cg", rtol=1e-8, maxit=500, refine=True, inner_rtol=1e-4)
    finally:
        A.close()
        B.close()
    assert im["converged"] and im["rel_residual"] <= 1e-8 and im["outer"] >= 2
    assert np.linalg.norm(zm - z64) / np.linalg.norm(z64) <= tol
    r = b - H.matvec(zm)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= tol


def test_not_converged_is_reported():
    H = oracle()
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=3, leaf=32, eta=0.5, storage="f64")
    try:
        bd = torch.tensor(H.mesh.area, dtype=torch.float64, device="cuda")
        z = torch.zeros_like(bd)
        info = h2.h2_solve(A.h, bd, z, method="cg", rtol=1e-12, maxit=2, check=False)
        assert not info["converged"] and info["iterations"] == 2 and info["rel_residual"] > 1e-12
        with pytest.raises(h2.H2Error) as e:
            h2.h2_solve(A.h, bd, z.zero_(), method="cg", rtol=1e-12, maxit=2)
        assert e.value.code == h2.H2_ENOTCONV
    finally:
        A.close()


def test_gmres_327k_sphere():
    """GMRES(50) to 1e-8 on the 327,680-triangle sphere with b_i = |T_i|: z ~ 1
    (RMS deviation at the level of the discretisation error), and the residual
    recomputed by the oracle on sampled rows is bounded by 1e-8 ||b||."""
    V, T = I.icosphere(7)
    H = H2Oracle(V, T, Kernel(), m=4, leaf=64, eta=0.5, build_blocks=False)
    area = H.mesh.area
    A = h2.H2Matrix(V, T, order=4, leaf=64, eta=0.5, storage="f64")
    try:
        z, info = solve(A, area, method="gmres", restart=50, rtol=1e-8, maxit=400)
    finally:
        A.close()
    print("gmres 327k", info)
    assert info["converged"] and info["rel_residual"] <= 1e-8
    assert np.sqrt(np.mean((z - 1) ** 2)) < 2e-3 and np.abs(z - 1).max() < 3e-2
    rng = np.random.default_rng(7)
    sample = [H.tree.leaves[i].id for i in rng.choice(len(H.tree.leaves), 3, replace=False)]
    for rows, val in H.sampled_rows(z, sample).values():
        assert np.abs(area[rows] - val).max() <= 1.01e-8 * np.linalg.norm(area)
