"""GPU parity: the HIP H^2 product against the FP64 oracle (through the C ABI).

Tolerances (2-norm over the compared entries):
  FP64 storage    ||y - y_ref|| <= 1e-12 ||G~ x||      (rounding only: quadrature
                  rules and conventions are the same on both sides)
  FP32 storage    ||y - y_ref|| <= 1e-6  ||G~ |x| ||   (FP32 unit roundoff 6e-8 of
                  stored entries and partial sums; a floating-point sum is accurate
                  relative to the sum of the absolute terms, and with x ~ N(0,1)
                  the sums over all n columns cancel by a factor of order sqrt(n),
                  so the scale is G~ applied to |x|, not G~ x)
  BF16 coupling   ||y - y_ref|| <= 2e-3  ||G~ |x| ||   (BF16 unit roundoff 2e-3)
The same bounds hold with FP64 accumulation over FP32/BF16 storage.  Every
FP32/BF16 comparison also holds the product to a bound relative to ||G~ x|| and
entry by entry to a multiple of u (G~ |x|)_i (tests/bounds.py).
"""
import functools

import numpy as np
import pytest

import h2_inputs as I
from oracle.h2 import H2Oracle
from oracle.kernels import Kernel
from tests import bounds
from tests.closed_forms import poly_kernel_product

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05665_amd import h2  # noqa: E402

TOL = {"f64": 1e-12, "f32": 1e-6, "f32_sbf16": 2e-3}


def rel(a, b, scale=None):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b if scale is None else scale))


def err(storage, y, ref, ref_abs):
    """Error in the norm the tolerance of `storage` is stated in."""
    return rel(y, ref) if storage == "f64" else rel(y, ref, ref_abs)


@functools.lru_cache(maxsize=None)
def oracle(kind, level, m, leaf, eta=0.5, kernel=0, kappa=0.0):
    V, T = I.mesh_for(kind, level)
    return H2Oracle(V, T, Kernel(kernel, kappa), m=m, leaf=leaf, eta=eta)


def gpu_matvec(A, x, y0=None, alpha=1.0, acc64=False, dtype=torch.float64):
    xd = torch.tensor(x, dtype=dtype, device="cuda")
    yd = torch.zeros_like(xd) if y0 is None else torch.tensor(y0, dtype=dtype, device="cuda")
    A.matvec(xd, yd, alpha=alpha, acc64=acc64)
    torch.cuda.synchronize()
    return yd.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("storage", ["f64", "f32", "f32_sbf16"])
@pytest.mark.parametrize("case", [("sphere", 3, 3, 32), ("sphere", 3, 4, 16), ("cube", 16, 3, 32),
                                  ("sphere", 2, 4, 24)])
def test_matvec_matches_oracle(case, storage):
    kind, level, m, leaf = case
    H = oracle(kind, level, m, leaf)
    V, T = H.mesh.V, H.mesh.T
    print("case", case, storage, flush=True)
    x = I.random_vector(H.mesh.n, 1, "uniform")
    ref = H.matvec(x)
    ref_abs = H.matvec(np.abs(x))
    A = h2.H2Matrix(V, T, order=m, leaf=leaf, eta=0.5, storage=storage)
    try:
        y = gpu_matvec(A, x)
        assert err(storage, y, ref, ref_abs) <= TOL[storage]
        if storage != "f64":
            bounds.check(y, ref, ref_abs, storage, "matvec %s" % (case,))
            y64 = gpu_matvec(A, x, acc64=True)
            assert err(storage, y64, ref, ref_abs) <= TOL[storage]
            bounds.check(y64, ref, ref_abs, storage, "matvec acc64 %s" % (case,))
    finally:
        A.close()


def test_assembled_data_matches_oracle():
    H = oracle("sphere", 3, 4, 16)
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=4, leaf=16, eta=0.5, storage="f64")
    try:
        dfs = A.export(h2.H2_X_DFS)
        cl = A.export(h2.H2_X_CLUSTERS).reshape(-1, 6)
        adm = A.export(h2.H2_X_ADM).reshape(-1, 2)
        near = A.export(h2.H2_X_NEAR).reshape(-1, 2)
        for c in range(cl.shape[0]):
            o = H.tree.clusters[dfs[c]]
            if o.is_leaf:
                Vl = A.export(h2.H2_X_V, c, count=o.idx.size * 64).reshape(-1, 64)
                assert np.abs(Vl - H.V(o)).max() <= 1e-14 * np.abs(H.V(o)).max()
            if c > 0:
                E = A.export(h2.H2_X_E, c).reshape(64, 64)
                assert np.abs(E - H.E(o)).max() <= 1e-13
        for b in range(0, adm.shape[0], 97):
            t, s = H.tree.clusters[dfs[adm[b, 0]]], H.tree.clusters[dfs[adm[b, 1]]]
            S = A.export(h2.H2_X_S, b).reshape(64, 64)
            assert np.abs(S - H.S(t, s)).max() <= 1e-14 * np.abs(S).max()
        for b in range(0, near.shape[0], 13):
            t, s = H.tree.clusters[dfs[near[b, 0]]], H.tree.clusters[dfs[near[b, 1]]]
            N = A.export(h2.H2_X_N, b, count=t.idx.size * s.idx.size).reshape(t.idx.size, s.idx.size)
            ref = H.N(t, s)
            assert np.abs(N - ref).max() <= 1e-14 * np.abs(ref).max()
    finally:
        A.close()


def test_accumulate_alpha_and_float32_vectors():
    H = oracle("sphere", 3, 3, 32)
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=3, leaf=32, eta=0.5, storage="f64")
    try:
        x = I.random_vector(H.mesh.n, 3, "normal")
        y0 = I.random_vector(H.mesh.n, 4, "normal")
        y = gpu_matvec(A, x, y0, alpha=-0.75)
        ref = y0 - 0.75 * H.matvec(x)
        assert rel(y, ref) <= 1e-12
        y32 = gpu_matvec(A, x, dtype=torch.float32)
        assert rel(y32, H.matvec(x), H.matvec(np.abs(x))) <= 1e-6
        bounds.check(y32, H.matvec(x), H.matvec(np.abs(x)), "f32", "float32 vectors")
    finally:
        A.close()


def test_multiple_rhs_and_determinism():
    H = oracle("sphere", 3, 3, 32)
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=3, leaf=32, eta=0.5, storage="f32")
    try:
        X = I.random_vector(H.mesh.n, 9, "normal", nrhs=3)
        xd = torch.tensor(X, dtype=torch.float64, device="cuda").t().contiguous().t()
        yd = torch.zeros_like(xd)
        A.matvec(xd, yd)
        y1 = yd.cpu().numpy()
        yd.zero_()
        A.matvec(xd, yd)
        y2 = yd.cpu().numpy()
        assert np.array_equal(y1, y2)
        for j in range(3):
            single = gpu_matvec(A, X[:, j].copy())
            assert np.array_equal(single, y1[:, j])
    finally:
        A.close()


@pytest.mark.parametrize("case", [("sphere", 0, 2, 32), ("sphere", 1, 1, 8), ("sphere", 1, 2, 3),
                                  ("cube", 2, 2, 4), ("sphere", 2, 5, 40)])
def test_edge_cases(case):
    """Single leaf (no admissible block), m = 1 (k = 1), tiny leaves, k = 125 > 64."""
    kind, level, m, leaf = case
    H = oracle(kind, level, m, leaf)
    x = I.random_vector(H.mesh.n, 2, "uniform")
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=m, leaf=leaf, eta=0.5, storage="f64")
    try:
        assert rel(gpu_matvec(A, x), H.matvec(x)) <= 1e-12
    finally:
        A.close()


def test_empty_nrhs_and_bad_arguments():
    V, T = I.icosphere(1)
    A = h2.H2Matrix(V, T, order=2, leaf=8)
    try:
        x = torch.zeros(T.shape[0], 0, dtype=torch.float64, device="cuda")
        assert h2.lib().h2_matvec(A.h, 0, 0, x.data_ptr(), T.shape[0], x.data_ptr(), T.shape[0], 1.0, 0,
                                  None) == 0
        with pytest.raises(ValueError):             # the binding checks the length
            h2.h2_matvec(A.h, torch.zeros(5, dtype=torch.float64, device="cuda"),
                         torch.zeros(5, dtype=torch.float64, device="cuda"))
        v5 = torch.zeros(5, dtype=torch.float64, device="cuda")
        assert h2.lib().h2_matvec(A.h, 1, 0, v5.data_ptr(), 5, v5.data_ptr(), 5, 1.0, 0,
                                  None) == h2.H2_EINVAL     # the C ABI rejects ld < n
        assert h2.lib().h2_matvec(A.h, 1, 7, x.data_ptr(), T.shape[0], x.data_ptr(), T.shape[0], 1.0, 0,
                                  None) == h2.H2_EINVAL
    finally:
        A.close()


@pytest.mark.parametrize("kernel,m,name", [("one", 1, "one"), ("bilinear", 2, "bilinear"),
                                           ("quadratic", 4, "quadratic")])
@pytest.mark.parametrize("mesh", [("sphere", 6), ("cube", 64)])
def test_closed_forms_medium(kernel, m, name, mesh):
    V, T = I.mesh_for(*mesh)
    x = I.random_vector(T.shape[0], 5, "normal")
    ref = poly_kernel_product(V, T, name, x)
    A = h2.H2Matrix(V, T, kernel=kernel, order=m, leaf=64, eta=0.5, storage="f64")
    try:
        assert A.info["n_adm"] > 0
        assert rel(gpu_matvec(A, x), ref) <= 1e-12
    finally:
        A.close()


@pytest.mark.parametrize("case", [("sphere", 3, 4, 16), ("sphere", 3, 4, 64), ("cube", 16, 4, 32),
                                  ("sphere", 2, 4, 100)])
@pytest.mark.parametrize("nrhs", [2, 17, 32, 33, 64, 70])
@pytest.mark.parametrize("otf", [False, True])
def test_multi_rhs_matches_oracle(case, nrhs, otf):
    """Many right-hand sides (matrix-core path, FP32 storage, k = 64; S stored or
    evaluated on the fly): every column against the oracle, in the FP32 norm of
    each column."""
    kind, level, m, leaf = case
    H = oracle(kind, level, m, leaf)
    X = I.random_vector(H.mesh.n, 11, "normal", nrhs=nrhs)
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=m, leaf=leaf, eta=0.5, storage="f32", coupling_otf=otf)
    try:
        xd = torch.tensor(X, dtype=torch.float64, device="cuda").t().contiguous().t()
        Y0 = I.random_vector(H.mesh.n, 12, "normal", nrhs=nrhs)
        yd = torch.tensor(Y0, dtype=torch.float64, device="cuda").t().contiguous().t()
        A.matvec(xd, yd, alpha=0.5)
        torch.cuda.synchronize()
        Y = yd.cpu().numpy()
        yd2 = torch.tensor(Y0, dtype=torch.float64, device="cuda").t().contiguous().t()
        A.matvec(xd, yd2, alpha=0.5)
        assert np.array_equal(yd2.cpu().numpy(), Y)                # reproducible
    finally:
        A.close()
    for j in range(nrhs):
        gx = H.matvec(X[:, j])
        ref = Y0[:, j] + 0.5 * gx
        scale = 0.5 * H.matvec(np.abs(X[:, j]))
        assert np.linalg.norm(Y[:, j] - ref) <= 1e-6 * np.linalg.norm(scale), j
        # Y0 ~ N(0,1) is larger than G~x: the FP64 rounding of the sum enters
        d = Y[:, j] - Y0[:, j]
        bounds.check(d, 0.5 * gx, scale, "f32", "multi-RHS %s R=%d otf=%d col %d" % (case, nrhs, otf, j),
                     extra=4.5e-16 * np.abs(Y0[:, j]))


@pytest.mark.parametrize("case", [("cube", 10, 4, 32), ("cube", 5, 4, 16), ("sphere", 1, 4, 8), ("cube", 2, 4, 16)])
@pytest.mark.parametrize("nrhs", [3, 64])
def test_multi_rhs_ragged_sizes(case, nrhs):
    """Many right-hand sides on meshes whose triangle count is not a multiple of
    the 64 user indices one permutation workgroup moves (1,200, 300, 80 and 48
    triangles: the last tile is partial, and on the smallest meshes it is the only
    one), with the leaves' rows and the coupling's groups as ragged as they come."""
    kind, level, m, leaf = case
    H = oracle(kind, level, m, leaf)
    n = H.mesh.n
    assert n % 64 != 0
    X = I.random_vector(n, 31, "normal", nrhs=nrhs)
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=m, leaf=leaf, eta=0.5, storage="f32")
    try:
        xd = torch.tensor(X, dtype=torch.float64, device="cuda").t().contiguous().t()
        yd = torch.zeros_like(xd)
        A.matvec(xd, yd)
        torch.cuda.synchronize()
        Y = yd.cpu().numpy()
    finally:
        A.close()
    for j in (0, nrhs - 1):
        bounds.check(Y[:, j], H.matvec(X[:, j]), H.matvec(np.abs(X[:, j])), "f32",
                     "ragged multi %s%d R=%d col %d" % (kind, level, nrhs, j))


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", [("sphere", 3, 3, 32), ("sphere", 3, 4, 16), ("cube", 16, 4, 32),
                                  ("sphere", 2, 5, 40)])
def test_on_the_fly_coupling_matches_oracle(case, storage):
    """Coupling matrices evaluated during the product (not stored) give the
    same product as the oracle, to the tolerance of the storage precision."""
    kind, level, m, leaf = case
    H = oracle(kind, level, m, leaf)
    x = I.random_vector(H.mesh.n, 1, "uniform")
    ref = H.matvec(x)
    ref_abs = H.matvec(np.abs(x))
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=m, leaf=leaf, eta=0.5, storage=storage, coupling_otf=True)
    try:
        assert A.info["bytes_S"] <= 16
        y = gpu_matvec(A, x)
        assert err(storage, y, ref, ref_abs) <= TOL[storage]
        if storage == "f32":
            bounds.check(y, ref, ref_abs, storage, "on-the-fly S %s" % (case,))
            y64 = gpu_matvec(A, x, acc64=True)
            assert err(storage, y64, ref, ref_abs) <= TOL[storage]
            bounds.check(y64, ref, ref_abs, storage, "on-the-fly S acc64 %s" % (case,))
        with pytest.raises(h2.H2Error):
            A.export(h2.H2_X_S, 0)
    finally:
        A.close()


@pytest.mark.parametrize("kernel,m,name", [("one", 1, "one"), ("bilinear", 2, "bilinear"),
                                           ("quadratic", 4, "quadratic")])
def test_on_the_fly_closed_forms(kernel, m, name):
    V, T = I.mesh_for("sphere", 6)
    x = I.random_vector(T.shape[0], 5, "normal")
    ref = poly_kernel_product(V, T, name, x)
    A = h2.H2Matrix(V, T, kernel=kernel, order=m, leaf=64, eta=0.5, storage="f64", coupling_otf=True)
    try:
        assert rel(gpu_matvec(A, x), ref) <= 1e-12
    finally:
        A.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("otf", [False, True])
@pytest.mark.parametrize("case", [("sphere", 3, 4, 16), ("sphere", 3, 4, 64), ("cube", 16, 4, 32),
                                  ("sphere", 4, 4, 48)])
def test_symmetric_storage_matches_oracle(case, storage, otf):
    """One block per symmetric pair, applied as itself and as its transpose
    (stored or on-the-fly S): the same product as the oracle, to the storage
    precision's tolerance, with y accumulated (alpha) and with FP64 accumulation
    over FP32 entries; bitwise reproducible; several columns apply one by one."""
    kind, level, m, leaf = case
    H = oracle(kind, level, m, leaf)
    x = I.random_vector(H.mesh.n, 21, "normal")
    y0 = I.random_vector(H.mesh.n, 22, "normal")
    ref, ref_abs = H.matvec(x), H.matvec(np.abs(x))
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=m, leaf=leaf, eta=0.5, storage=storage, coupling_otf=otf,
                    symmetric=True)
    try:
        assert A.info["s_blocks_stored"] == (0 if otf else A.info["n_adm"] // 2)
        y = gpu_matvec(A, x)
        assert err(storage, y, ref, ref_abs) <= TOL[storage]
        assert np.array_equal(gpu_matvec(A, x), y)
        ya = gpu_matvec(A, x, y0=y0, alpha=-0.5)
        # y0 ~ N(0,1) is much larger than G~x: its own FP64 rounding enters the bound
        scale = np.linalg.norm(ref if storage == "f64" else ref_abs)
        assert np.linalg.norm(ya - (y0 - 0.5 * ref)) <= 0.5 * TOL[storage] * scale + 4e-16 * np.linalg.norm(y0)
        if storage == "f32":
            bounds.check(y, ref, ref_abs, storage, "symmetric %s otf=%d" % (case, otf))
            y64 = gpu_matvec(A, x, acc64=True)
            assert err(storage, y64, ref, ref_abs) <= TOL[storage]
            bounds.check(y64, ref, ref_abs, storage, "symmetric acc64 %s otf=%d" % (case, otf))
        X = np.asfortranarray(np.stack([x, y0], axis=1))
        xd = torch.tensor(X, device="cuda").t().contiguous().t()
        yd = torch.zeros_like(xd)
        A.matvec(xd, yd)
        Y = yd.cpu().numpy()
        assert np.array_equal(Y[:, 0], y)
        assert err(storage, Y[:, 1], H.matvec(y0), H.matvec(np.abs(y0))) <= TOL[storage]
    finally:
        A.close()


def test_symmetric_storage_solve():
    """CG through h2_solve on symmetric storage reaches the same solution as on
    full storage (unit sphere, b_i = |T_i|, z ~ 1)."""
    V, T = I.icosphere(4)
    P = V[T]
    b = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    bd = torch.tensor(b, device="cuda")
    out = {}
    for sym in (False, True):
        A = h2.H2Matrix(V, T, order=4, leaf=64, eta=0.5, storage="f64", symmetric=sym)
        try:
            z, info = A.solve(bd, method="cg", rtol=1e-10, maxit=500)
            assert info["converged"]
            out[sym] = z.cpu().numpy()
        finally:
            A.close()
    assert np.linalg.norm(out[True] - out[False]) <= 1e-8 * np.linalg.norm(out[False])


@pytest.mark.parametrize("case", [("sphere", 0, 4, 32), ("sphere", 1, 4, 64), ("sphere", 1, 4, 4), ("cube", 2, 4, 8)])
@pytest.mark.parametrize("otf", [False, True])
def test_symmetric_storage_edge_cases(case, otf):
    """Symmetric storage on a single leaf (only a diagonal near block, no scratch),
    on meshes without admissible blocks, and with one-to-four-triangle leaves."""
    kind, level, m, leaf = case
    H = oracle(kind, level, m, leaf)
    x = I.random_vector(H.mesh.n, 23, "uniform")
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=m, leaf=leaf, eta=0.5, storage="f64", coupling_otf=otf,
                    symmetric=True)
    try:
        assert rel(gpu_matvec(A, x), H.matvec(x)) <= 1e-12
    finally:
        A.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_near_field_fallback_kernels(storage):
    """The kernels kept for structures outside the fast paths' limits.  Leaves of
    up to 87 triangles (leaf size 100, m = 3) take the per-block near field
    (near_backward) for one vector; a row with 67 near blocks (5,120 triangles,
    leaf size 8, m = 4) takes the per-block many-column near field
    (mnear_backward16) for 40 columns, while the single vector still runs
    near_backward64 (at most 256 blocks per row)."""
    for kind, level, m, leaf in (("sphere", 3, 3, 100), ("sphere", 4, 4, 8)):
        H = oracle(kind, level, m, leaf)
        n = H.mesh.n
        x = I.random_vector(n, 5, "normal")
        ref, ref_abs = H.matvec(x), H.matvec(np.abs(x))
        A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=m, leaf=leaf, eta=0.5, storage=storage)
        try:
            y = gpu_matvec(A, x)
            assert err(storage, y, ref, ref_abs) <= TOL[storage], (kind, level, leaf)
            if storage == "f32":
                bounds.check(y, ref, ref_abs, storage, "fallback %s%d leaf %d" % (kind, level, leaf))
            if m == 4 and storage == "f32":
                X = np.random.default_rng(9).standard_normal((n, 40))
                xd = torch.tensor(np.ascontiguousarray(X.T), device="cuda").t()
                yd = torch.zeros_like(xd)
                A.matvec(xd, yd)
                torch.cuda.synchronize()
                Y = yd.cpu().numpy()
                for j in (0, 39):
                    bounds.check(Y[:, j], H.matvec(X[:, j]), H.matvec(np.abs(X[:, j])), storage,
                                 "fallback multi %s%d leaf %d col %d" % (kind, level, leaf, j))
        finally:
            A.close()
