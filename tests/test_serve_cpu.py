"""The continuous-batching solve service, driven by a dense CPU backend (no GPU).

Covers admission (arrivals, slots, memory budget, eviction of idle structures),
grouping of products across requests, the Krylov state machines (CG, complex
GMRES, FP64 refinement over a rounded operator) and every failure path
(unknown mesh, bad sizes, non-finite data, non-convergence, a backend that
returns NaN, a structure larger than the budget)."""
import numpy as np
import pytest
import torch

import h2_inputs as I
from paper_2203_05665_amd.serve import H2Server
from tests import cpu_krylov

torch.set_default_dtype(torch.float64)


class _Dense:
    def __init__(self, A, width):
        n = A.shape[0]
        self.A = A
        self.X = torch.zeros((width, n), dtype=A.dtype).t()
        self.Y = torch.zeros((width, n), dtype=A.dtype).t()


class DenseBackend:
    """Products with a dense matrix on the CPU; optional FP32 rounding of the
    operator to exercise the refinement path (FP64 accumulation uses the same
    rounded entries with FP64 accumulation); Krylov steps by the CPU model of the
    library's step-wise solver."""

    device = torch.device("cpu")
    torch = torch

    def __init__(self, refine=False, poison=False, nbytes_per_entry=8, product_width=64):
        self._refine = refine
        self.poison = poison
        self.built, self.freed, self.products = 0, 0, 0
        self.nb = nbytes_per_entry
        self.product_width = product_width
        self.widths = []

    def estimate(self, V, T, kernel, kappa):
        return int(T.shape[0] ** 2 * self.nb)

    def build(self, V, T, kernel, kappa):
        n = T.shape[0]
        P = V[T]
        c = P.mean(1)
        d = np.linalg.norm(c[:, None] - c[None], axis=-1)
        if kernel == "helmholtz":
            A = np.exp(1j * kappa * d) / (4 * np.pi * (d + 0.3)) + 0.5 * np.eye(n)
        else:
            A = 1.0 / (4 * np.pi * (d + 0.3)) + 0.5 * np.eye(n)
        if self._refine:
            A = A.astype(np.complex64 if kernel == "helmholtz" else np.float32).astype(A.dtype)
        self.built += 1
        return _Dense(torch.tensor(A), self.product_width), int(n * n * self.nb)

    def buffers(self, S):
        return S.X, S.Y

    def matvec(self, S, ncols, flags, stream):
        self.products += 1
        self.widths.append(ncols)
        X, Y, A = S.X[:, :ncols], S.Y[:, :ncols], S.A
        if self.poison:
            Y.fill_(float("nan"))
            return
        if self._refine and not flags & cpu_krylov.ACC_F64:
            lo = torch.complex64 if A.is_complex() else torch.float32
            Y.copy_((A.to(lo) @ X.to(lo)).to(Y.dtype))
        else:
            Y.copy_(A @ X)

    def free(self, S):
        self.freed += 1

    def new_stream(self):
        return None

    def refine(self):
        return self._refine

    def request_arena(self, nbytes):
        return None

    def status_pool(self, slots, per_slot):
        return None

    def solver_params(self, method, rtol, maxit, restart, refine, inner_rtol):
        return cpu_krylov.params(method, rtol, maxit, restart, refine, inner_rtol)

    def workspace_bytes(self, n, r, cx, p):
        return cpu_krylov.workspace_bytes(n, r, cx, p)

    def new_solver(self, n, r, cx, p, ws_ptr, ws_bytes, status_ptr):
        return cpu_krylov.CPUKrylov(n, r, cx, p)

    def to_device(self, b, cx):
        b = torch.as_tensor(np.asarray(b))
        if b.dim() == 1:
            b = b[:, None]
        return b.to(torch.complex128 if cx else torch.float64).t().contiguous().t()

    def empty_like(self, b):
        return torch.zeros((b.shape[1], b.shape[0]), dtype=b.dtype).t()

    def all_finite(self, b):
        return bool(torch.isfinite(b).all())


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t


def make_server(backend, budget=1e12, slots=8, vec_budget=None):
    S = H2Server(backend, mem_budget=budget, max_active=slots, clock=Clock(), vec_budget=vec_budget)
    for r in (1, 2):
        S.register_mesh("sphere%d" % r, *I.icosphere(r))
    S.register_mesh("cube2", *I.cube_surface(2))
    return S


def dense(backend, S, mesh, kernel="laplace", kappa=0.0):
    A, _ = backend.build(*S.meshes[mesh], kernel, kappa)
    return A.A.numpy()


def test_cg_and_gmres_requests_solve():
    be = DenseBackend()
    S = make_server(be)
    n1 = S.meshes["sphere1"][1].shape[0]
    b = np.random.default_rng(0).standard_normal((n1, 3))
    q1 = S.submit("sphere1", b, rtol=1e-10)
    bc = b[:, 0] + 1j * b[:, 1]
    q2 = S.submit("sphere1", bc, kernel="helmholtz", kappa=2.0, rtol=1e-10, restart=8)
    S.run()
    assert q1.status == "done" and q2.status == "done"
    A = dense(be, S, "sphere1")
    Z = q1.result.numpy()
    assert np.linalg.norm(A @ Z - b) <= 1e-9 * np.linalg.norm(b)
    Ac = dense(be, S, "sphere1", "helmholtz", 2.0)
    z = q2.result.numpy()[:, 0]
    assert np.linalg.norm(Ac @ z - bc) <= 1e-9 * np.linalg.norm(bc)
    assert q2.iterations > 8          # needed more than one restart cycle


def test_refinement_reaches_tolerance_of_rounded_operator():
    be = DenseBackend(refine=True)
    S = make_server(be)
    n = S.meshes["sphere2"][1].shape[0]
    b = np.random.default_rng(1).standard_normal(n)
    q = S.submit("sphere2", b, rtol=1e-10, inner_rtol=1e-3)
    qc = S.submit("sphere2", b + 1j * b[::-1], kernel="helmholtz", kappa=4.0, rtol=1e-10, inner_rtol=1e-3)
    S.run()
    for req, A in ((q, dense(be, S, "sphere2")), (qc, dense(be, S, "sphere2", "helmholtz", 4.0))):
        assert req.status == "done"
        z = req.result.numpy()[:, 0]
        rhs = req.b.numpy()[:, 0]
        assert np.linalg.norm(A @ z - rhs) <= 1.01e-10 * np.linalg.norm(rhs)


def test_products_are_batched_across_requests():
    be = DenseBackend()
    S = make_server(be)
    n = S.meshes["sphere2"][1].shape[0]
    rng = np.random.default_rng(2)
    reqs = [S.submit("sphere2", rng.standard_normal((n, 1 + i % 3)), rtol=1e-8, arrival=0.0) for i in range(6)]
    S.run()
    assert all(q.status == "done" for q in reqs)
    total = sum(q.products for q in reqs)
    assert be.products < total / 3      # one product per tick served all six requests
    st = S.stats()
    assert st["done"] == 6 and st["p50_s"] is not None and st["p99_s"] >= st["p50_s"]


def test_alone_equals_mix():
    rng = np.random.default_rng(3)
    n2 = I.icosphere(2)[1].shape[0]
    b = rng.standard_normal(n2)
    alone = make_server(DenseBackend())
    qa = alone.submit("sphere2", b, rtol=1e-10)
    alone.run()
    mix = make_server(DenseBackend())
    others = [mix.submit("sphere1", rng.standard_normal(80), rtol=1e-10),
              mix.submit("cube2", rng.standard_normal(48) * 1j, kernel="helmholtz", kappa=2.0, rtol=1e-10)]
    qm = mix.submit("sphere2", b, rtol=1e-10)
    others.append(mix.submit("sphere2", rng.standard_normal((n2, 2)), rtol=1e-10))
    mix.run()
    assert qa.status == qm.status == "done" and all(o.status == "done" for o in others)
    za, zm = qa.result.numpy(), qm.result.numpy()
    assert np.linalg.norm(za - zm) <= 1e-9 * np.linalg.norm(za)


def test_arrivals_and_slots():
    be = DenseBackend()
    S = make_server(be, slots=2)
    n = S.meshes["sphere1"][1].shape[0]
    rng = np.random.default_rng(4)
    reqs = [S.submit("sphere1", rng.standard_normal(n), rtol=1e-8, arrival=0.002 * i) for i in range(5)]
    seen_active = []
    while S.queue or S.active:
        S.tick()
        seen_active.append(len(S.active))
        assert len(S.active) <= 2
    assert all(q.status == "done" for q in reqs)
    assert all(q.start >= q.arrival for q in reqs)
    assert max(seen_active) == 2


def _ws(n, r=1, method="cg"):
    return cpu_krylov.workspace_bytes(n, r, False, cpu_krylov.params(method))


def test_memory_budget_admission_and_eviction():
    be = DenseBackend()
    n1 = I.icosphere(1)[1].shape[0]
    n2 = I.icosphere(2)[1].shape[0]
    vec = 4 * _ws(n2)
    # room for the request arena and the larger structure, not for both structures
    budget = vec + n2 * n2 * 8 + n1 * n1 * 8 // 2
    S = make_server(be, budget=budget, vec_budget=vec)
    rng = np.random.default_rng(5)
    a = S.submit("sphere2", rng.standard_normal(n2), rtol=1e-8, arrival=0.0)
    b = S.submit("sphere1", rng.standard_normal(n1), rtol=1e-8, arrival=0.0)
    S.run()
    assert a.status == b.status == "done"
    assert b.start >= a.finish            # waited until the first structure became idle
    assert be.freed >= 1                   # the idle structure was evicted
    assert S.used_bytes() <= budget


def test_requests_wait_for_room_in_the_vector_arena():
    """The request arena holds one request's vectors: a second request on the
    same (resident) structure starts when the first one has released them."""
    be = DenseBackend()
    n2 = I.icosphere(2)[1].shape[0]
    S = make_server(be, vec_budget=_ws(n2) + 255)
    rng = np.random.default_rng(7)
    a = S.submit("sphere2", rng.standard_normal(n2), rtol=1e-8, arrival=0.0)
    c = S.submit("sphere2", rng.standard_normal(n2), rtol=1e-8, arrival=0.0)
    S.run()
    assert a.status == c.status == "done", S.stats()["errors"]
    assert c.start >= a.finish and be.built == 1
    assert S.arena.used() == 0 and sorted(S.free_slots) == list(range(S.max_active))


def test_request_vectors_larger_than_the_arena_fail_cleanly():
    be = DenseBackend()
    n2 = I.icosphere(2)[1].shape[0]
    S = make_server(be, vec_budget=_ws(n2) // 2)
    q = S.submit("sphere2", np.ones(n2), rtol=1e-8)
    S.run()
    assert q.status == "failed" and "vectors do not fit" in q.error
    w = S.submit("sphere2", np.ones((n2, 65)), rtol=1e-8)
    assert w.status == "failed" and "right-hand sides" in w.error


def test_structure_larger_than_budget_fails_cleanly():
    be = DenseBackend()
    S = make_server(be, budget=1000.0)
    q = S.submit("sphere1", np.ones(80), rtol=1e-8)
    S.run()
    assert q.status == "failed" and "memory" in q.error
    assert not S.active and not S.queue


def test_bad_requests_fail_without_stopping_the_server():
    be = DenseBackend()
    S = make_server(be)
    n = S.meshes["sphere1"][1].shape[0]
    bad = [S.submit("nope", np.ones(10)), S.submit("sphere1", np.ones(n + 1)),
           S.submit("sphere1", np.full(n, np.nan))]
    good = S.submit("sphere1", np.ones(n), rtol=1e-8)
    S.run()
    assert [q.status for q in bad] == ["failed"] * 3
    assert "unknown mesh" in bad[0].error and "rows" in bad[1].error and "finite" in bad[2].error
    assert good.status == "done"


def test_non_convergence_and_poisoned_products():
    S = make_server(DenseBackend())
    n = S.meshes["sphere2"][1].shape[0]
    q = S.submit("sphere2", np.random.default_rng(6).standard_normal(n), rtol=1e-14, maxit=3)
    qg = S.submit("sphere2", np.ones(n) + 0j, kernel="helmholtz", kappa=4.0, rtol=1e-14, maxit=3, restart=2)
    S.run()
    assert q.status == "not_converged" and q.iterations == 3 and q.result is not None
    assert qg.status == "not_converged" and qg.result is not None
    P = make_server(DenseBackend(poison=True))
    p = P.submit("sphere1", np.ones(80), rtol=1e-8)
    P.run()
    assert p.status == "failed" and "non-finite" in p.error
    assert "a product returned a non-finite entry" in p.error       # blamed on the product, not the solver


def test_failures_are_reported():
    S = make_server(DenseBackend())
    S.submit("nope", np.ones(10))
    S.run()
    assert S.stats()["errors"] == {"unknown mesh 'nope'": 1}
    (f,) = S.failures()
    assert f["mesh"] == "nope" and f["error"].startswith("unknown mesh")


def test_mixed_stream_of_wide_requests_has_no_failures():
    """60 staggered requests (Laplace and Helmholtz kappa 2 / 4, 1..16 columns,
    three meshes) through FP64 refinement over an FP32-rounded operator: every
    request converges and nothing turns non-finite."""
    be = DenseBackend(refine=True)
    S = H2Server(be, mem_budget=1e12, max_active=32, clock=Clock())
    for r in (2, 3):
        S.register_mesh("sphere%d" % r, *I.icosphere(r))
    S.register_mesh("cube8", *I.cube_surface(8))
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(60):
        mesh = ["sphere2", "sphere3", "cube8"][rng.integers(3)]
        n = S.meshes[mesh][1].shape[0]
        kern = ["laplace", "helmholtz", "helmholtz"][rng.integers(3)]
        kap = 4.0 if rng.random() < 0.5 else 2.0
        r = int(rng.integers(1, 17))
        B = rng.standard_normal((n, r))
        if kern == "helmholtz":
            B = B + 1j * rng.standard_normal((n, r))
        reqs.append(S.submit(mesh, B, kernel=kern, kappa=kap if kern == "helmholtz" else 0.0, rtol=1e-8,
                             arrival=0.002 * i * rng.random()))
    S.run()
    st = S.stats()
    assert st["done"] == 60 and st["errors"] == {} and S.failures() == []
    for q in reqs:
        A = dense(be, S, q.mesh, q.kernel, q.kappa)
        Z = q.result.numpy()
        Bq = q.b.numpy()
        assert np.linalg.norm(A @ Z - Bq) <= 1.01e-8 * np.linalg.norm(Bq) * np.sqrt(Bq.shape[1])


def test_products_are_chunked_to_the_buffer_width():
    """With room for 4 columns per product, six requests of 1-3 columns are served
    by several products per tick, none wider than 4 columns, and each result is
    the same as with one wide product."""
    rng = np.random.default_rng(9)
    n = I.icosphere(2)[1].shape[0]
    Bs = [rng.standard_normal((n, 1 + i % 3)) for i in range(6)]
    out = {}
    for width in (4, 64):
        be = DenseBackend(product_width=width)
        S = make_server(be)
        reqs = [S.submit("sphere2", B, rtol=1e-10, arrival=0.0) for B in Bs]
        S.run()
        assert all(q.status == "done" for q in reqs)
        assert max(be.widths) <= width
        out[width] = [q.result.numpy() for q in reqs]
    assert max(be.widths) > 4
    for a, b in zip(out[4], out[64]):
        assert np.array_equal(a, b)
