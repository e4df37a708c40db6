"""The solve service on the GPU: a mixed stream (Laplace and Helmholtz, several
meshes, 1-3 right-hand sides, staggered arrivals) served with continuous
batching; every result equals the same request served alone.

Tolerance of "the same": both runs solve the same FP32-stored operator A (the
outer residuals of the FP64 refinement use the per-column product with FP64
accumulation) to ||b - A z|| <= 1e-8 ||b||, so ||z_alone - z_mix|| <=
cond(A) * 2e-8 ||z||; the single-layer matrices here have cond(A) < 500, hence
1e-5.  Each result's residual is also recomputed with the library's FP64-
accumulated product, and against the oracle's FP64 matrix on the smallest mesh.
"""
import numpy as np
import pytest

import h2_inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05665_amd import h2  # noqa: E402
from paper_2203_05665_amd.serve import GPUBackend, H2Server  # noqa: E402

MESHES = {"s3": I.icosphere(3), "s4": I.icosphere(4), "c16": I.cube_surface(16)}


def server(storage="f32", otf=False):
    S = H2Server(GPUBackend(order=4, leaf=64, eta=0.5, storage=storage, coupling_otf=otf), mem_budget=60e9,
                 max_active=16, vec_budget=4e9)
    for k, (V, T) in MESHES.items():
        S.register_mesh(k, V, T)
    return S


def workload():
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(10):
        mesh = ["s3", "s4", "c16"][i % 3]
        n = MESHES[mesh][1].shape[0]
        kernel = "helmholtz" if i % 4 == 3 else "laplace"
        kappa = [2.0, 4.0][i % 2] if kernel == "helmholtz" else 0.0
        r = 1 + i % 3
        b = rng.standard_normal((n, r))
        if kernel == "helmholtz":
            b = b + 1j * rng.standard_normal((n, r))
        reqs.append(dict(mesh=mesh, kernel=kernel, kappa=kappa, b=b, arrival=0.01 * i))
    return reqs


@pytest.mark.parametrize("otf", [False, True])
def test_mix_equals_alone_and_converges(otf):
    """Laplace structures with stored or on-the-fly coupling matrices."""
    W = workload()
    S = server(otf=otf)
    t0 = S.clock()
    mixed = [S.submit(w["mesh"], w["b"], kernel=w["kernel"], kappa=w["kappa"], rtol=1e-8, arrival=t0 + w["arrival"])
             for w in W]
    S.run()
    st = S.stats()
    print("serve stats", st)
    assert st["done"] == len(W)
    assert st["batched_products"] < sum(q.products for q in mixed)   # products were shared
    for w, qm in zip(W, mixed):
        A = server(otf=otf)
        qa = A.submit(w["mesh"], w["b"], kernel=w["kernel"], kappa=w["kappa"], rtol=1e-8)
        A.run()
        assert qa.status == "done"
        za, zm = qa.result.cpu().numpy(), qm.result.cpu().numpy()
        assert np.linalg.norm(za - zm) <= 1e-5 * np.linalg.norm(za), (w["mesh"], w["kernel"])
        # residual with the library's FP64-accumulated product of the stored operator
        B = S.resident[qm.key].obj.A
        R = torch.tensor(w["b"], device="cuda").t().contiguous().t()
        R = R.to(torch.complex128 if w["kernel"] == "helmholtz" else torch.float64)
        B.matvec(qm.result, R, alpha=-1.0, acc64=True)
        torch.cuda.synchronize()
        Rh, bh = R.cpu().numpy(), qm.b.cpu().numpy()
        rel = float((np.linalg.norm(Rh, axis=0) / np.linalg.norm(bh, axis=0)).max())
        assert rel <= 1.01e-8
        for res in A.resident.values():
            A.be.free(res.obj)
    for res in S.resident.values():
        S.be.free(res.obj)


def test_against_oracle_smallest_mesh():
    from oracle.h2 import H2Oracle
    from oracle.kernels import Kernel
    V, T = MESHES["s3"]
    H = H2Oracle(V, T, Kernel(), m=4, leaf=64, eta=0.5)
    b = H.mesh.area.copy()
    S = server()
    q = S.submit("s3", b, rtol=1e-8)
    S.run()
    z = q.result.cpu().numpy()[:, 0]
    # FP32 storage: the stored operator differs from the FP64 one by ~1e-7 relative
    assert np.linalg.norm(b - H.matvec(z)) <= 1e-6 * np.linalg.norm(b)
    for res in S.resident.values():
        S.be.free(res.obj)
