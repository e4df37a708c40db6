"""Helmholtz kernel exp(i kappa r)/(4 pi r) on the GPU: complex coupling and
near-field storage, real V and E, against the complex128 oracle.

Tolerances: FP64 storage ||y - y_ref|| <= 1e-12 ||G~ x||; FP32 storage
<= 1e-6 ||G~_L |x| || where G~_L is the Laplace matrix (|g_Helmholtz| = g_Laplace,
so G~_L |x| is the scale of the absolute terms of every sum).
"""
import functools

import numpy as np
import pytest

import h2_inputs as I
from oracle.h2 import H2Oracle
from oracle.kernels import HELMHOLTZ, LAPLACE, Kernel
from tests import bounds

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05665_amd import h2  # noqa: E402


@functools.lru_cache(maxsize=None)
def oracle(kind, level, m, leaf, kernel, kappa):
    V, T = I.mesh_for(kind, level)
    return H2Oracle(V, T, Kernel(kernel, kappa), m=m, leaf=leaf, eta=0.5)


def cvec(n, seed):
    return I.random_vector(n, seed, "uniform") + 1j * I.random_vector(n, seed + 100, "uniform")


@pytest.mark.parametrize("storage", ["f64", "f32", "f32_otf"])
@pytest.mark.parametrize("case", [("sphere", 3, 3, 32, 2.0), ("sphere", 3, 4, 16, 4.0), ("cube", 16, 4, 32, 4.0)])
def test_helmholtz_matvec_matches_oracle(case, storage):
    """f32_otf: FP32 storage with the coupling evaluated during the product (m = 4 only)."""
    kind, level, m, leaf, kappa = case
    otf = storage == "f32_otf"
    storage = "f32" if otf else storage
    H = oracle(kind, level, m, leaf, HELMHOLTZ, kappa)
    if otf and m != 4:
        with pytest.raises(h2.H2Error):
            h2.H2Matrix(H.mesh.V, H.mesh.T, kernel="helmholtz", kappa=kappa, order=m, leaf=leaf, storage="f32",
                        coupling_otf=True)
        return
    L = oracle(kind, level, m, leaf, LAPLACE, 0.0)
    x = cvec(H.mesh.n, 3)
    ref = H.matvec(x)
    scale = L.matvec(np.abs(x))
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, kernel="helmholtz", kappa=kappa, order=m, leaf=leaf, eta=0.5,
                    storage=storage, coupling_otf=otf)
    if otf:
        assert A.info["s_blocks_stored"] == 0 and A.info["bytes_S"] < 1024
    try:
        for dt in (torch.complex128, torch.complex64):
            xd = torch.tensor(x, dtype=dt, device="cuda")
            yd = torch.zeros_like(xd)
            A.matvec(xd, yd, alpha=1.0)
            torch.cuda.synchronize()
            y = yd.cpu().numpy().astype(np.complex128)
            if storage == "f64" and dt == torch.complex128:
                assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
            else:
                assert np.linalg.norm(y - ref) <= 1e-6 * np.linalg.norm(scale)
                bounds.check(y, ref, scale, "f32", "Helmholtz %s %s %s" % (case, storage + ("_otf" if otf else ""),
                                                                           dt))
        if storage == "f32":
            xd = torch.tensor(x, dtype=torch.complex128, device="cuda")
            yd = torch.zeros_like(xd)
            A.matvec(xd, yd, acc64=True)
            y64 = yd.cpu().numpy()
            assert np.linalg.norm(y64 - ref) <= 1e-6 * np.linalg.norm(scale)
            bounds.check(y64, ref, scale, "f32", "Helmholtz acc64 %s otf=%d" % (case, otf))
        # real vectors are rejected for a complex matrix
        with pytest.raises(h2.H2Error):
            A.matvec(torch.zeros(H.mesh.n, dtype=torch.float64, device="cuda"))
    finally:
        A.close()


def test_helmholtz_assembled_data():
    H = oracle("sphere", 3, 4, 16, HELMHOLTZ, 4.0)
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, kernel="helmholtz", kappa=4.0, order=4, leaf=16, eta=0.5, storage="f64")
    try:
        dfs = A.export(h2.H2_X_DFS)
        adm = A.export(h2.H2_X_ADM).reshape(-1, 2)
        near = A.export(h2.H2_X_NEAR).reshape(-1, 2)
        for b in range(0, adm.shape[0], 101):
            t, s = H.tree.clusters[dfs[adm[b, 0]]], H.tree.clusters[dfs[adm[b, 1]]]
            S = A.export(h2.H2_X_S, b).reshape(64, 64, 2)
            S = S[..., 0] + 1j * S[..., 1]
            assert np.abs(S - H.S(t, s)).max() <= 1e-14 * np.abs(S).max()
        for b in range(0, near.shape[0], 17):
            t, s = H.tree.clusters[dfs[near[b, 0]]], H.tree.clusters[dfs[near[b, 1]]]
            N = A.export(h2.H2_X_N, b, count=2 * t.idx.size * s.idx.size).reshape(t.idx.size, s.idx.size, 2)
            N = N[..., 0] + 1j * N[..., 1]
            ref = H.N(t, s)
            assert np.abs(N - ref).max() <= 1e-14 * np.abs(ref).max()
    finally:
        A.close()


@pytest.mark.parametrize("storage,refine,tol", [("f64", False, 1e-8), ("f32", True, 1e-5)])
def test_helmholtz_gmres_unit_sphere(storage, refine, tol):
    """Single layer on the unit sphere: V_kappa 1 = exp(i kappa) sin(kappa)/kappa, so
    G z = b with b_i = |T_i| has z close to kappa / (exp(i kappa) sin kappa)."""
    kappa = 2.0
    H = oracle("sphere", 3, 3, 32, HELMHOLTZ, kappa)
    b = H.mesh.area.astype(np.complex128)
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, kernel="helmholtz", kappa=kappa, order=3, leaf=32, eta=0.5,
                    storage=storage)
    try:
        bd = torch.tensor(b, device="cuda")
        z, info = A.solve(bd, method="gmres", restart=40, rtol=1e-8, maxit=400, refine=refine, inner_rtol=1e-4)
        z = z.cpu().numpy()
    finally:
        A.close()
    assert info["converged"] and info["rel_residual"] <= 1e-8
    r = b - H.matvec(z)
    assert np.linalg.norm(r) <= tol * np.linalg.norm(b)
    # discretisation-level agreement with the constant solution of the continuous
    # problem (1,280 triangles: about 1-5 % pointwise)
    zc = kappa / (np.exp(1j * kappa) * np.sin(kappa))
    assert np.mean(np.abs(z - zc)) / abs(zc) < 2e-2 and np.abs(z - zc).max() / abs(zc) < 1e-1


def test_helmholtz_cg_is_rejected():
    H = oracle("sphere", 3, 3, 32, HELMHOLTZ, 2.0)
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, kernel="helmholtz", kappa=2.0, order=3, leaf=32, eta=0.5)
    try:
        bd = torch.ones(H.mesh.n, dtype=torch.complex128, device="cuda")
        with pytest.raises(h2.H2Error):
            A.solve(bd, method="cg")
    finally:
        A.close()


@pytest.mark.parametrize("otf", [False, True])
@pytest.mark.parametrize("case", [("sphere", 3, 4, 16, 4.0), ("cube", 16, 4, 64, 2.0), ("cube", 10, 4, 32, 4.0)])
@pytest.mark.parametrize("nrhs", [2, 5, 16, 17, 33])
def test_helmholtz_multi_rhs(case, nrhs, otf):
    """Complex many-RHS product on the matrix cores: every column against the oracle."""
    kind, level, m, leaf, kappa = case
    H = oracle(kind, level, m, leaf, HELMHOLTZ, kappa)
    L = oracle(kind, level, m, leaf, LAPLACE, 0.0)
    rng = np.random.default_rng(nrhs)
    X = rng.standard_normal((H.mesh.n, nrhs)) + 1j * rng.standard_normal((H.mesh.n, nrhs))
    Y0 = rng.standard_normal((H.mesh.n, nrhs)) + 1j * rng.standard_normal((H.mesh.n, nrhs))
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, kernel="helmholtz", kappa=kappa, order=m, leaf=leaf, eta=0.5, storage="f32",
                    coupling_otf=otf)
    try:
        xd = torch.tensor(X, device="cuda").t().contiguous().t()
        yd = torch.tensor(Y0, device="cuda").t().contiguous().t()
        A.matvec(xd, yd, alpha=-0.5)
        Y = yd.cpu().numpy()
    finally:
        A.close()
    for j in range(nrhs):
        gx = H.matvec(X[:, j])
        ref = Y0[:, j] - 0.5 * gx
        scale = 0.5 * L.matvec(np.abs(X[:, j]))
        assert np.linalg.norm(Y[:, j] - ref) <= 1e-6 * np.linalg.norm(scale), j
        bounds.check(Y[:, j] - Y0[:, j], -0.5 * gx, scale, "f32", "Helmholtz multi %s R=%d otf=%d col %d"
                     % (case, nrhs, otf, j), extra=4.5e-16 * np.abs(Y0[:, j]))


def test_helmholtz_otf_full_size_sphere327k():
    """327,680 triangles, kappa = 4, FP32: the product with the coupling evaluated
    during the product agrees with the stored one within twice the FP32 bound
    (both are G~ in FP32), for one column and for 16 columns."""
    V, T = I.mesh_for("sphere", 7)
    n = T.shape[0]
    rng = np.random.default_rng(11)
    X = rng.standard_normal((n, 16)) + 1j * rng.standard_normal((n, 16))
    xd = torch.tensor(X.T.copy(), device="cuda").t()
    out = {}
    for otf in (False, True):
        A = h2.H2Matrix(V, T, kernel="helmholtz", kappa=4.0, order=4, leaf=64, eta=0.5, storage="f32",
                        coupling_otf=otf)
        try:
            Y = torch.zeros_like(xd)
            A.matvec(xd, Y)
            y1 = torch.zeros_like(xd[:, 0])
            A.matvec(xd[:, 0].contiguous(), y1)
            torch.cuda.synchronize()
            out[otf] = (Y.cpu().numpy(), y1.cpu().numpy())
        finally:
            A.close()
    # scale of the absolute terms: the Laplace matrix applied to |x_j| (|g_Helmholtz| = g_Laplace)
    Lp = h2.H2Matrix(V, T, kernel="laplace", order=4, leaf=64, eta=0.5, storage="f32")
    try:
        ad = torch.tensor(np.abs(X).T.copy(), device="cuda").t()
        sc = torch.zeros_like(ad)
        Lp.matvec(ad, sc)
        SC = sc.cpu().numpy()
        scale = np.linalg.norm(SC, axis=0)
    finally:
        Lp.close()
    (Ys, y1s), (Yo, y1o) = out[False], out[True]
    assert np.linalg.norm(y1o - y1s) <= 2e-6 * scale[0]
    # both products carry FP32 errors: twice the bounds of one
    bounds.check(y1o, y1s, 2 * SC[:, 0], "f32", "Helmholtz 327k otf vs stored, one column", t_rel=1e-5)
    for j in range(16):
        assert np.linalg.norm(Yo[:, j] - Ys[:, j]) <= 2e-6 * scale[j], j
        bounds.check(Yo[:, j], Ys[:, j], 2 * SC[:, j], "f32", "Helmholtz 327k otf vs stored col %d" % j,
                     t_rel=1e-5)


def test_helmholtz_multi_rhs_fallback_near():
    """A row with 68 near blocks (1,280 triangles, leaf size 6) takes the
    per-block complex near field (mnear_backward16c) for several columns, the
    structures of the other tests (at most 44 near blocks per row) the streamed
    one (mnear_stream16c)."""
    kind, level, m, leaf, kappa = "sphere", 3, 4, 6, 4.0
    H = oracle(kind, level, m, leaf, HELMHOLTZ, kappa)
    L = oracle(kind, level, m, leaf, LAPLACE, 0.0)
    rng = np.random.default_rng(11)
    n, nrhs = H.mesh.n, 2
    X = rng.standard_normal((n, nrhs)) + 1j * rng.standard_normal((n, nrhs))
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, kernel="helmholtz", kappa=kappa, order=m, leaf=leaf, eta=0.5,
                    storage="f32")
    try:
        xd = torch.tensor(X, device="cuda").t().contiguous().t()
        yd = torch.zeros_like(xd)
        A.matvec(xd, yd)
        Y = yd.cpu().numpy()
    finally:
        A.close()
    for j in range(nrhs):
        gx = H.matvec(X[:, j])
        scale = L.matvec(np.abs(X[:, j]))
        assert np.linalg.norm(Y[:, j] - gx) <= 1e-6 * np.linalg.norm(scale), j
        bounds.check(Y[:, j], gx, scale, "f32", "Helmholtz multi fallback near col %d" % j)
