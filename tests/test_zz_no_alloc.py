"""The allocation-free solve entry point h2_solve_noalloc (through the C ABI)
against h2_solve on the same inputs: two calls in a row, the second with a
smaller input, so nothing the first call left in the shared scratch array may
leak into the second."""
import ctypes as C

import numpy as np
import pytest

import h2_inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05665_amd import h2  # noqa: E402


def fblock(B, dtype=torch.float64):
    return torch.tensor(np.asarray(B).T.copy(), dtype=dtype, device="cuda").t()


def both(A, B, **kw):
    """(solution, info) from h2_solve_noalloc and from h2_solve, same inputs."""
    out = []
    for noalloc in (True, False):
        bd = fblock(B, torch.complex128 if np.iscomplexobj(B) else torch.float64)
        zd = torch.zeros_like(bd)
        info = h2.h2_solve(A.h, bd, zd, noalloc=noalloc, **kw)
        torch.cuda.synchronize()
        out.append((zd.cpu().numpy(), info))
    return out


def test_noalloc_equals_h2_solve_fp64_two_calls():
    """FP64 storage: the same kernels in the same order, so bitwise equal; the
    second call (a smaller mesh, one column) after a larger one (three columns)."""
    rng = np.random.default_rng(51)
    V, T = I.icosphere(3)
    A = h2.H2Matrix(V, T, order=3, leaf=32, eta=0.5, storage="f64")
    V2, T2 = I.icosphere(2)
    A2 = h2.H2Matrix(V2, T2, order=3, leaf=32, eta=0.5, storage="f64")
    try:
        n = T.shape[0]
        B = rng.standard_normal((n, 3))
        (z0, i0), (z1, i1) = both(A, B, method="gmres", restart=20, rtol=1e-9, maxit=500)
        assert i0["converged"] and i1["converged"]
        assert np.array_equal(z0, z1) and i0["iterations"] == i1["iterations"]
        B2 = rng.standard_normal(T2.shape[0])
        (y0, j0), (y1, j1) = both(A2, B2, method="cg", rtol=1e-9, maxit=500)
        assert j0["converged"] and np.array_equal(y0, y1) and j0["iterations"] == j1["iterations"]
    finally:
        A.close()
        A2.close()


def test_noalloc_refined_fp32_and_complex():
    """FP32 storage with refinement (k = 64: the many-RHS path when its
    workspaces exist, else one column at a time) and complex Helmholtz GMRES: the
    allocation-free solve meets the tolerance and agrees with h2_solve within
    the conditioning of the FP32-stored operator (both solve it to 1e-8)."""
    rng = np.random.default_rng(52)
    V, T = I.icosphere(3)
    n = T.shape[0]
    A = h2.H2Matrix(V, T, order=4, leaf=64, eta=0.5, storage="f32")
    C2 = h2.H2Matrix(V, T, kernel="helmholtz", kappa=2.0, order=3, leaf=32, eta=0.5, storage="f32")
    try:
        B = rng.standard_normal((n, 4))
        (z0, i0), (z1, i1) = both(A, B, method="cg", rtol=1e-8, maxit=800, refine=True)
        assert i0["converged"] and i1["converged"] and i0["rel_residual"] <= 1e-8
        assert np.linalg.norm(z0 - z1) <= 1e-5 * np.linalg.norm(z1)
        # now the many-RHS workspaces exist: the same path as h2_solve, bitwise
        (z2, i2), (z3, _) = both(A, B, method="cg", rtol=1e-8, maxit=800, refine=True)
        assert np.array_equal(z2, z3)
        Bc = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
        (w0, k0), (w1, k1) = both(C2, Bc, method="gmres", restart=20, rtol=1e-8, maxit=800, refine=True)
        assert k0["converged"] and k1["converged"]
        assert np.linalg.norm(w0 - w1) <= 1e-5 * np.linalg.norm(w1)
    finally:
        A.close()
        C2.close()


def test_noalloc_rejects_what_does_not_fit():
    V, T = I.icosphere(7)
    A = h2.H2Matrix(V, T, order=4, leaf=64, eta=0.5, storage="f32")
    try:
        n = T.shape[0]
        p = h2.solve_params("gmres", 1e-8, 10, 50, False, 1e-4)
        info = h2.h2_solve_info()
        b = torch.ones((4, n), dtype=torch.float64, device="cuda").t()
        z = torch.zeros_like(b)
        rc = h2.lib().h2_solve_noalloc(A.h, 4, h2.H2_R64, b.data_ptr(), n, z.data_ptr(), n, C.byref(p),
                                       C.byref(info), None)
        assert rc == h2.H2_EINVAL and "scratch" in h2.h2_last_error()
        rc = h2.lib().h2_solve_noalloc(A.h, 65, h2.H2_R64, b.data_ptr(), n, z.data_ptr(), n, C.byref(p),
                                       C.byref(info), None)
        assert rc == h2.H2_EINVAL and "at most" in h2.h2_last_error()
        # a solve that fits still works after the refusals
        z1 = torch.zeros(n, dtype=torch.float64, device="cuda")
        out = h2.h2_solve(A.h, b[:, 0].contiguous(), z1, method="cg", rtol=1e-6, maxit=300, refine=True,
                          noalloc=True)
        assert out["converged"]
    finally:
        A.close()
