"""GPU: tile-shape autotuning (h2_tune, h2_set_tuning) through the C ABI.

Every value of a knob computes the same product with other tiles, so each is
held to the parity bar of its storage: FP32 storage 1e-6 in the norm of G~|x|
against the oracle's G~x; recompressed FP64 bases 1e-10 against the oracle's own
recompression (as for h2_recompress); recompressed FP32 bases within the
Frobenius bound of the discarded weights plus the FP32 term.  The tuner must time
every value the path admits and keep one of them, and the handle must then run
exactly that value."""
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


@functools.lru_cache(maxsize=None)
def oracle(kind, level, m, leaf):
    V, T = I.mesh_for(kind, level)
    return H2Oracle(V, T, Kernel(), m=m, leaf=leaf, eta=0.5)


def product(A, X):
    xd = torch.tensor(np.ascontiguousarray(X.T), dtype=torch.float64, device="cuda").t() if X.ndim == 2 else \
        torch.tensor(X, dtype=torch.float64, device="cuda")
    yd = torch.zeros_like(xd)
    A.matvec(xd, yd)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


@pytest.mark.parametrize("nrhs", [2, 40, 64])
def test_pass_columns_every_value_matches_oracle(nrhs):
    """Many right-hand sides, FP32 storage: 32 or 64 columns per pass (40 runs as
    32 + 8 or as one padded pass of 64)."""
    H = oracle("sphere", 3, 4, 64)
    X = I.random_vector(H.mesh.n, 21, "normal", nrhs=nrhs)
    ref = np.stack([H.matvec(X[:, j]) for j in range(nrhs)], 1)
    scale = np.stack([H.matvec(np.abs(X[:, j])) for j in range(nrhs)], 1)
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=4, leaf=64, eta=0.5, storage="f32")
    try:
        out = {}
        for v in (0, 32, 64):
            A.set_tuning("pass_columns", v)
            out[v] = product(A, X)
        info = A.tune(nrhs, "f64", reps=3)
        yt = product(A, X)
    finally:
        A.close()
    print("tuning, %d columns:" % nrhs, info)
    for v, Y in list(out.items()) + [("tuned", yt)]:
        for j in range(nrhs):
            assert np.linalg.norm(Y[:, j] - ref[:, j]) <= 1e-6 * np.linalg.norm(scale[:, j]), (v, j)
            bounds.check(Y[:, j], ref[:, j], scale[:, j], "f32", "pass columns %s, R=%d col %d" % (v, nrhs, j))
    assert np.array_equal(out[0], out[32 if nrhs <= 32 else 64])      # the built-in rule
    assert info["knob"] == "pass_columns" and info["values"] == [32, 64]
    assert all(t > 0 for t in info["ms"]) and info["chosen"] in (32, 64)
    assert np.array_equal(yt, out[info["chosen"]])


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", [("sphere", 3, 4, 32), ("cube", 8, 3, 32)])
def test_small_slot_every_value_matches_oracle(case, storage):
    """Recompressed bases (k' <= 16): slots of 16 or 32 lanes in the coupling."""
    H = oracle(*case)
    O = Recompressed(H, 1e-4)
    x = I.random_vector(H.mesh.n, 22, "normal")
    X2 = np.stack([x, I.random_vector(H.mesh.n, 23, "normal")], 1)
    ref, ref_c, ref_abs = H.matvec(x), O.matvec(x), H.matvec(np.abs(x))
    kind, level, m, leaf = case
    V, T = I.mesh_for(kind, level)
    A = h2.H2Matrix(V, T, order=m, leaf=leaf, eta=0.5, storage=storage)
    try:
        rc = A.recompress(1e-4)
        assert rc["rank"] <= 16
        out = {}
        for v in (0, 16, 32):
            A.set_tuning("small_slot", v)
            out[v] = product(A, x)
        info = A.tune(1, "f64", reps=3)
        yt = product(A, x)
        Y2 = product(A, X2)                                  # columns one at a time, same kernels
    finally:
        A.close()
    print("tuning, %s %s k'=%d:" % (case, storage, rc["rank"]), info)
    for v, y in list(out.items()) + [("tuned", yt)]:
        if storage == "f64":
            assert np.linalg.norm(y - ref_c) <= 1e-10 * np.linalg.norm(ref_c), v
        else:
            bound = np.sqrt(2.0 * rc["discarded"]) * np.linalg.norm(x) + 1e-6 * np.linalg.norm(ref_abs)
            assert np.linalg.norm(y - ref) <= bound, v
    assert np.array_equal(out[0], out[16])                   # the built-in rule for k' <= 16
    assert info["knob"] == "small_slot" and info["values"] == [16, 32] and info["chosen"] in (16, 32)
    assert np.array_equal(yt, out[info["chosen"]])
    assert np.array_equal(Y2[:, 0], yt)


def test_paths_without_alternatives():
    """k = 64 single vectors and FP64 many right-hand sides have one tile shape:
    h2_tune reports no knob and the product is unchanged."""
    H = oracle("sphere", 3, 4, 32)
    x = I.random_vector(H.mesh.n, 24, "normal")
    ref = H.matvec(x)
    A = h2.H2Matrix(H.mesh.V, H.mesh.T, order=4, leaf=32, eta=0.5, storage="f64")
    try:
        for nrhs in (1, 3):
            assert A.tune(nrhs, "f64", reps=2) == {"knob": None, "values": [], "ms": [], "chosen": None}
        y = product(A, x)
    finally:
        A.close()
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("kernel", ["laplace", "helmholtz"])
def test_row_order_every_value_matches_oracle(kernel):
    """Many right-hand sides: both row orders of the coupling kernels (XCD chunks,
    interleaved) give the oracle's product, and h2_tune_knob times both and keeps
    one."""
    from oracle.kernels import HELMHOLTZ, LAPLACE
    kind, level, m, leaf = "sphere", 3, 4, 64
    V, T = I.mesh_for(kind, level)
    cx = kernel == "helmholtz"
    H = H2Oracle(V, T, Kernel(HELMHOLTZ if cx else LAPLACE, 2.0 if cx else 0.0), m=m, leaf=leaf, eta=0.5)
    L = oracle(kind, level, m, leaf)
    n, nrhs = H.mesh.n, 20
    rng = np.random.default_rng(61)
    X = rng.standard_normal((n, nrhs)) + (1j * rng.standard_normal((n, nrhs)) if cx else 0)
    A = h2.H2Matrix(V, T, kernel=kernel, kappa=2.0 if cx else 0.0, order=m, leaf=leaf, eta=0.5, storage="f32")
    try:
        out = {}
        for v in (1, 2):
            A.set_tuning("row_order", v)
            xd = torch.tensor(np.ascontiguousarray(X.T), device="cuda").t()
            yd = torch.zeros_like(xd)
            A.matvec(xd, yd)
            torch.cuda.synchronize()
            out[v] = yd.cpu().numpy()
        info = A.tune(nrhs, "c128" if cx else "f64", reps=3, knob="row_order")
    finally:
        A.close()
    print("row order tuning (%s):" % kernel, info)
    assert info["knob"] == "row_order" and info["chosen"] in info["values"]
    assert info["values"] == ([1, 2] if cx else [1, 2, 3])
    for v, Y in out.items():
        for j in range(nrhs):
            ref = H.matvec(X[:, j])
            scale = L.matvec(np.abs(X[:, j]))
            bounds.check(Y[:, j], ref, scale, "f32", "row order %d %s col %d" % (v, kernel, j))


@pytest.mark.parametrize("kind,level,nrhs", [("sphere", 4, 40), ("cube", 32, 64)])
def test_grouped_coupling_schedule(kind, level, nrhs):
    """Schedule 3 of the many-column coupling (four row clusters per workgroup,
    x^ shared through LDS; 64-column passes) sums every tile's products in the
    order of schedule 1, so the two agree bit for bit; both hold the FP32 bounds
    against the oracle on sampled columns.  Two products in a row on the same
    handle repeat exactly (the staging buffers leave nothing behind)."""
    m, leaf = 4, 64
    V, T = I.mesh_for(kind, level)
    H = oracle(kind, level, m, leaf)
    n = H.mesh.n
    X = np.random.default_rng(71).standard_normal((n, nrhs))
    A = h2.H2Matrix(V, T, order=m, leaf=leaf, eta=0.5, storage="f32")
    try:
        A.set_tuning("pass_columns", 64)
        out = {}
        for v in (1, 3, 3):
            A.set_tuning("row_order", v)
            out.setdefault(v, []).append(product(A, X))
    finally:
        A.close()
    assert np.array_equal(out[1][0], out[3][0]), np.abs(out[1][0] - out[3][0]).max()
    assert np.array_equal(out[3][0], out[3][1])
    Y = out[3][0]
    for j in (0, nrhs // 2, nrhs - 1):
        ref = H.matvec(X[:, j])
        scale = H.matvec(np.abs(X[:, j]))  # G~|x|: the Laplace kernel is positive
        bounds.check(Y[:, j], ref, scale, "f32", "grouped %s%d col %d" % (kind, level, j))
