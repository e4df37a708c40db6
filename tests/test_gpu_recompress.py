"""GPU: algebraic recompression (h2_recompress) through the C ABI.

Pins: with eps = 0 the recompressed product equals G~ x from the oracle to FP64
parity (1e-12); with eps > 0 it equals the oracle's own recompression (same
rank k', same discarded weight, same product to 1e-10) and respects the
Frobenius bound ||(G~ - G~')x|| <= sqrt(2 * discarded) ||x|| (the bound the
construction guarantees; the oracle's tests pin it on dense matrices)."""
import functools

import numpy as np
import pytest

import h2_inputs as I
from tests import bounds
from oracle.h2 import H2Oracle
from oracle.kernels import Kernel
from oracle.recompress import Recompressed

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05665_amd import h2  # noqa: E402

CASES = [("sphere", 3, 4, 32), ("cube", 8, 3, 32), ("sphere", 4, 4, 64)]


@functools.lru_cache(maxsize=None)
def oracle(kind, level, m, leaf):
    V, T = I.mesh_for(kind, level)
    return H2Oracle(V, T, Kernel(), m=m, leaf=leaf, eta=0.5)


@functools.lru_cache(maxsize=None)
def oracle_rc(kind, level, m, leaf, eps):
    return Recompressed(oracle(kind, level, m, leaf), eps)


def padded(r, k):
    """The library pads every cluster to one rank: the largest rank rounded up to a
    multiple of 4, but never above k."""
    return min(k, (max(1, r) + 3) // 4 * 4)


def product(A, X, dtype=torch.float64):
    xd = torch.tensor(np.ascontiguousarray(X.T), dtype=dtype, device="cuda").t() if X.ndim == 2 else \
        torch.tensor(X, dtype=dtype, device="cuda")
    yd = torch.zeros_like(xd)
    A.matvec(xd, yd)
    torch.cuda.synchronize()
    return yd.cpu().numpy().astype(np.float64)


def build(case, storage="f64"):
    kind, level, m, leaf = case
    V, T = I.mesh_for(kind, level)
    return h2.H2Matrix(V, T, order=m, leaf=leaf, eta=0.5, storage=storage)


@pytest.mark.parametrize("case", CASES)
def test_orthogonalisation_keeps_gtilde(case):
    H = oracle(*case)
    x = I.random_vector(H.mesh.n, 1, "normal")
    ref = H.matvec(x)
    A = build(case)
    try:
        info = A.recompress(0.0)
        assert info["rank"] <= H.k and info["discarded"] == 0.0 and info["rank_before"] == H.k
        assert A.info["k"] == info["rank"]
        y = product(A, x)
    finally:
        A.close()
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("eps", [1e-3, 1e-5])
def test_truncation_matches_oracle_and_bound(case, eps):
    H = oracle(*case)
    O = oracle_rc(*case, eps)
    x = I.random_vector(H.mesh.n, 2, "normal")
    ref, ref_c = H.matvec(x), O.matvec(x)
    A = build(case)
    try:
        info = A.recompress(eps)
        y = product(A, x)
    finally:
        A.close()
    assert info["rank"] == padded(O.max_rank, H.k)
    # the discarded eigenvalues are tiny next to the largest ones, so two eigensolvers
    # agree on them to about machine precision times the largest, not relatively
    assert abs(info["discarded"] - O.discarded) <= 1e-3 * O.discarded + 1e-30
    assert np.linalg.norm(y - ref_c) <= 1e-10 * np.linalg.norm(ref_c)
    assert np.linalg.norm(y - ref) <= np.sqrt(2.0 * info["discarded"]) * np.linalg.norm(x) + 1e-12 * np.linalg.norm(ref)
    assert info["bytes_after"] < info["bytes_before"]


def test_fp32_storage_and_many_columns():
    case = ("sphere", 4, 4, 64)
    H = oracle(*case)
    X = np.stack([I.random_vector(H.mesh.n, s, "normal") for s in (3, 4, 5)], 1)
    ref = np.stack([H.matvec(X[:, j]) for j in range(3)], 1)
    L = np.stack([H.matvec(np.abs(X[:, j])) for j in range(3)], 1)
    A = build(case, "f32")
    try:
        info = A.recompress(1e-4)
        Y = product(A, X)
        y0 = product(A, X[:, 0])
    finally:
        A.close()
    assert np.array_equal(Y[:, 0], y0)                      # several columns: the single-column path
    for j in range(3):
        bound = np.sqrt(2.0 * info["discarded"]) * np.linalg.norm(X[:, j]) + 1e-6 * np.linalg.norm(L[:, j])
        assert np.linalg.norm(Y[:, j] - ref[:, j]) <= bound


def test_solve_after_recompression():
    case = ("sphere", 4, 4, 64)
    V, T = I.mesh_for(case[0], case[1])
    A = build(case)
    try:
        A.recompress(1e-6)
        P = V[T]
        area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
        b = torch.tensor(area, device="cuda")
        z, info = A.solve(b, method="cg", rtol=1e-8)
        zh = z.cpu().numpy()
        y = product(A, zh)
    finally:
        A.close()
    assert info["rel_residual"] <= 1e-8
    assert np.linalg.norm(y - area) <= 2e-8 * np.linalg.norm(area)
    # unit sphere: V 1 = 1, so z is close to 1 (to the discretisation error)
    assert abs(zh.mean() - 1.0) < 0.05


def test_unsupported_handles_are_rejected():
    V, T = I.mesh_for("sphere", 3)
    for kw in (dict(coupling_otf=True), dict(symmetric=True), dict(kernel="helmholtz", kappa=2.0),
               dict(storage="f32_sbf16")):
        args = dict(order=4, leaf=32, eta=0.5, storage="f32")
        args.update(kw)
        A = h2.H2Matrix(V, T, **args)
        try:
            with pytest.raises(h2.H2Error):
                A.recompress(1e-4)
        finally:
            A.close()
    A = h2.H2Matrix(V, T, order=4, leaf=32, eta=0.5)
    try:
        for bad in (dict(eps=-1.0), dict(eps=float("nan")), dict(eps=1e-3, max_rank=-1)):
            with pytest.raises(h2.H2Error):
                A.recompress(**bad)
        x = I.random_vector(A.n, 1, "normal")
        y = product(A, x)                                   # the handle is still valid
        assert np.isfinite(y).all()
    finally:
        A.close()


def test_sphere327k_fp32_change_within_bound():
    """Full-size C2 mesh: the change of the product by recompression stays inside
    the Frobenius bound, and the rank and the stored bytes drop."""
    V, T = I.mesh_for("sphere", 7)
    n = T.shape[0]
    x = I.random_vector(n, 2, "normal")
    A = h2.H2Matrix(V, T, order=4, leaf=64, eta=0.5, storage="f32")
    try:
        y0 = product(A, x)
        ya = product(A, np.abs(x))
        info = A.recompress(1e-5)
        y1 = product(A, x)
    finally:
        A.close()
    print("recompression at 327,680 triangles:", info)
    assert info["rank"] < 64 and info["bytes_after"] < 0.7 * info["bytes_before"]
    assert np.linalg.norm(y1 - y0) <= np.sqrt(2.0 * info["discarded"]) * np.linalg.norm(x) + 2e-6 * np.linalg.norm(ya)


@pytest.mark.parametrize("case", [("sphere", 3, 4, 32), ("cube", 8, 3, 32)])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_symmetric_near_field_alone_and_recompressed(case, storage):
    """H2_SYMMETRIC_NEAR: the near field stored once per pair (any k) gives G~ x;
    recompressed on top it gives the oracle's recompressed product."""
    H = oracle(*case)
    O = oracle_rc(*case, 1e-4)
    x = I.random_vector(H.mesh.n, 5, "normal")
    ref, ref_c, ref_abs = H.matvec(x), O.matvec(x), H.matvec(np.abs(x))
    kind, level, m, leaf = case
    V, T = I.mesh_for(kind, level)
    A = h2.H2Matrix(V, T, order=m, leaf=leaf, eta=0.5, storage=storage, symmetric_near=True)
    try:
        y = product(A, x)
        info = A.recompress(1e-4)
        yc = product(A, x)
    finally:
        A.close()
    tol = 1e-12 if storage == "f64" else 1e-6
    scale = np.linalg.norm(ref) if storage == "f64" else np.linalg.norm(ref_abs)
    assert np.linalg.norm(y - ref) <= tol * scale
    if storage == "f32":
        bounds.check(y, ref, ref_abs, "f32", "symmetric near field %s" % (case,))
    if storage == "f64":
        assert info["rank"] == padded(O.max_rank, H.k)
        assert np.linalg.norm(yc - ref_c) <= 1e-10 * np.linalg.norm(ref_c)
    else:
        # FP32 S moves the weights' small eigenvalues: the rank may differ from the
        # FP64 oracle's, the bound still holds
        bound = np.sqrt(2.0 * info["discarded"]) * np.linalg.norm(x) + 1e-6 * np.linalg.norm(ref_abs)
        assert np.linalg.norm(yc - ref) <= bound


def test_many_columns_on_dense_transfers_after_orthogonalisation():
    """eps = 0 keeps k' = 64 but replaces the Kronecker-structured transfers by
    orthonormal dense ones: many columns then run the dense (matrix-core)
    transfer kernels, and the product is still G~ x."""
    case = ("sphere", 4, 4, 64)
    H = oracle(*case)
    X = np.stack([I.random_vector(H.mesh.n, s, "normal") for s in range(30, 64)], 1)   # 34 columns
    A = build(case, "f32")
    try:
        info = A.recompress(0.0)
        assert info["rank"] == 64
        Y = product(A, X)
    finally:
        A.close()
    for j in range(X.shape[1]):
        ref, scale = H.matvec(X[:, j]), H.matvec(np.abs(X[:, j]))
        assert np.linalg.norm(Y[:, j] - ref) <= 1e-6 * np.linalg.norm(scale), j
        bounds.check(Y[:, j], ref, scale, "f32", "dense transfers after orthogonalisation col %d" % j)
