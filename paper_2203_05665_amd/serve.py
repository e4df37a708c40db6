"""Continuous-batching solve service over HBM-resident H^2 matrices.

Requests ask for G~ z = b on a registered mesh (Laplace, or Helmholtz with a
wave number) with 1..R right-hand sides.  The engine

* keeps the H^2 structures resident on the device and admits a structure by its
  footprint against a memory budget, evicting idle structures (least recently
  used first) when a new one does not fit;
* admits requests into a bounded number of slots as slots and memory free up;
* runs every admitted request as a step-wise Krylov iteration (CG for the
  symmetric positive definite Laplace matrix, restarted GMRES for Helmholtz),
  optionally wrapped in FP64 iterative refinement for FP32 storage;
* on every scheduler tick gathers the pending matrix products of all active
  requests, groups them by structure, and issues ONE many-right-hand-side
  product per group (h2_matvec with all the groups' columns) on that
  structure's stream, so requests on different meshes overlap on the device and
  requests on the same mesh share one pass over its matrix data;
* reports per-request latency (arrival to result), p50/p99 and throughput.

The product y <- y + G~ X is the library's (libh2mi355x.so through the ctypes
binding); the Krylov vector algebra of each request runs in FP64 on the
request's stream.  Every reduction the scheduler or a solver takes a decision
from (inner products, norms, the finiteness checks) goes through the backend's
`dots` / `norms`: on the GPU these are the library's dot kernel, which reduces
each output inside one workgroup in a fixed order, so the values are
reproducible and need no communication between workgroups; elementwise updates
are tensor operations.  A backend object supplies the products and these
reductions, so the scheduler can also be driven by a CPU backend in tests.
"""
from __future__ import annotations

import math
from collections import Counter
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

# ---------------------------------------------------------------------------- backends


class GPUBackend:
    """Builds H^2 matrices with the HIP library; vectors are CUDA tensors."""

    def __init__(self, order=4, leaf=64, eta=0.5, storage="f32", device="cuda", coupling_otf=False):
        import torch
        from . import h2
        self.torch, self.h2 = torch, h2
        self.order, self.leaf, self.eta, self.storage = order, leaf, eta, storage
        self.device = torch.device(device)
        # real kernels may evaluate the coupling matrices during each product instead of storing them
        self.coupling_otf = coupling_otf

    def _otf(self, kernel):
        if not self.coupling_otf:
            return False
        if kernel == "helmholtz":          # FP32 evaluation of e^{i kappa r}/(4 pi r), m = 4
            return self.storage == "f32" and self.order == 4
        return self.storage in ("f32", "f64")

    def estimate(self, V, T, kernel, kappa):
        """Device bytes of the structure, from a host-only build of its trees."""
        h2 = self.h2
        h = h2.build_h2(V, T, kernel=kernel, kappa=kappa, order=self.order, leaf=self.leaf, eta=self.eta,
                        storage=self.storage, host_only=True)
        try:
            i = h2.h2_info(h)
        finally:
            h2.h2_free(h)
        cw = 2 if kernel == "helmholtz" else 1
        vb = 8 if self.storage == "f64" else 4
        sb = {"f64": 8, "f32": 4, "f32_sbf16": 2}[self.storage]
        k, n, nc = i["k"], i["n"], i["nclusters"]
        s_bytes = 0 if self._otf(kernel) else sb * k * k * i["n_adm"]
        data = cw * (s_bytes + vb * i["near_entries"]) + vb * (4 * n * k + 2 * k * k * nc + 48 * nc) + 8 * 15 * nc
        work = 2 * 8 * cw * (n + nc * k) + 4 * 64 * (2 * n + 2 * nc * k)   # one- and many-RHS workspaces
        return int(data + work)

    def build(self, V, T, kernel, kappa):
        A = self.h2.H2Matrix(V, T, kernel=kernel, kappa=kappa, order=self.order, leaf=self.leaf, eta=self.eta,
                             storage=self.storage, coupling_otf=self._otf(kernel))
        return A, self.estimate(V, T, kernel, kappa)

    def matvec(self, A, X, Y, acc64, stream):
        """Y <- Y + G~ X (X, Y: n x R Fortran-ordered device tensors)."""
        A.matvec(X, Y, alpha=1.0, acc64=acc64, stream=stream.cuda_stream if stream is not None else None)

    def free(self, A):
        A.close()

    def new_stream(self):
        return self.torch.cuda.Stream(device=self.device)

    def refine(self):
        return self.storage != "f64"

    # reductions and batched Gram-Schmidt steps on the library's kernels (current stream)
    def krylov_dots(self, Q, W, nvec):
        return self.h2.h2_krylov_dots(Q, W, nvec)

    def krylov_update(self, Q, h, W, sign):
        self.h2.h2_krylov_update(Q, h.contiguous(), W, sign)

    def dots(self, A, B):
        """<a_c, b_c> for every row c of the (r, n) blocks A, B (conjugating A)."""
        return self.h2.h2_krylov_dots(A[:, None, :], B, 1)[:, 0]

    def norms(self, Z):
        """Euclidean norm of every row of the (r, n) block Z (FP64)."""
        d = self.h2.h2_krylov_dots(Z[:, None, :], Z, 1)[:, 0]
        return self.torch.sqrt(d.real if d.is_complex() else d)


class _TensorOps:
    """Plain tensor versions of the reductions and Gram-Schmidt steps (for
    backends without native kernels, e.g. the CPU test backend)."""

    @staticmethod
    def krylov_dots(Q, W, nvec):
        Qj = Q[:, :nvec]
        return ((Qj.conj() if Qj.is_complex() else Qj) * W[:, None, :]).sum(-1)

    @staticmethod
    def krylov_update(Q, h, W, sign):
        W += sign * (h[:, :, None] * Q[:, : h.shape[1]]).sum(1)

    @staticmethod
    def dots(A, B):
        return ((A.conj() if A.is_complex() else A) * B).sum(1)

    @staticmethod
    def norms(Z):
        import torch
        return torch.linalg.vector_norm(Z, dim=1)


# ---------------------------------------------------------------------------- Krylov state machines


# All Krylov vectors are held right-hand-side-major, shape (r, n): row c is
# column c of the n x r block, so X.t() is the Fortran-ordered n x r block the
# product takes, with no copy.


class _CG:
    """Conjugate gradients for all right-hand sides at once (independent columns)."""

    def __init__(self, torch, B, tol, maxit, ops):
        self.t = torch
        self.ops = ops
        self.B = B
        self.X = torch.zeros_like(B)
        self.R = B.clone()
        self.P = B.clone()
        self.rr = ops.dots(B, B)
        self.nb = torch.sqrt(self.rr)
        self.tol, self.maxit, self.it = tol, maxit, 0

    def operand(self):
        return self.P

    def advance(self, Q):
        t = self.t
        pq = self.ops.dots(self.P, Q)
        ok = pq > 0
        alpha = t.where(ok, self.rr / t.where(ok, pq, t.ones_like(pq)), t.zeros_like(pq))[:, None]
        self.X += alpha * self.P
        self.R -= alpha * Q
        rr2 = self.ops.dots(self.R, self.R)
        okr = self.rr > 0
        beta = t.where(okr, rr2 / t.where(okr, self.rr, t.ones_like(self.rr)), t.zeros_like(rr2))[:, None]
        self.P = self.R + beta * self.P
        self.rr = rr2
        self.it += 1

    def relres(self):
        t = self.t
        return t.sqrt(self.rr) / t.where(self.nb > 0, self.nb, t.ones_like(self.nb))

    def solution(self):
        return self.X


class _GMRES:
    """Restarted GMRES for all right-hand sides at once (independent Arnoldi
    processes advanced in lockstep; classical Gram-Schmidt twice as batched
    matrix-vector products; complex Givens rotations), FP64 / complex128.  The
    basis vectors and products stay on the device; the Hessenberg columns, the
    rotations and the residual estimates (a few numbers per right-hand side) are
    kept on the host, so a step issues the Gram-Schmidt kernels, one
    normalisation and one small device-to-host copy.

    phase "arnoldi": the next product is A q_j;  phase "residual": the next
    product is A X (true residual at the end of a restart cycle)."""

    def __init__(self, torch, B, tol, maxit, restart, ops):
        self.t = torch
        self.ops = ops
        self.B = B
        self.m = restart
        self.tol, self.maxit, self.it = tol, maxit, 0
        self.X = torch.zeros_like(B)
        r, n = B.shape
        self.nb = ops.norms(B).cpu().numpy()
        self.Q = torch.zeros((r, self.m + 1, n), dtype=B.dtype, device=B.device)
        self.H = np.zeros((r, self.m + 1, self.m), dtype=np.complex128)
        self.cs = np.zeros((self.m, r), dtype=np.complex128)
        self.sn = np.zeros((self.m, r), dtype=np.complex128)
        self.g = np.zeros((self.m + 1, r), dtype=np.complex128)
        self.j = 0
        self._start(B)                       # X = 0: the residual is B itself

    def _scale(self, v):
        return v / np.where(self.nb > 0, self.nb, 1.0)

    def _start(self, R):
        t = self.t
        beta_d = self.ops.norms(R)
        self.Q[:, 0, :] = R / t.where(beta_d > 0, beta_d, t.ones_like(beta_d)).to(R.dtype)[:, None]
        beta = beta_d.cpu().numpy()
        self._rel = self._scale(beta)
        self.H[:] = 0
        self.g[:] = 0
        self.g[0] = beta
        self.j = 0
        self.phase = "arnoldi"

    def operand(self):
        return self.X if self.phase == "residual" else self.Q[:, self.j, :]

    def advance(self, Y):
        t = self.t
        if self.phase == "residual":
            self._start(self.B - Y)
            return
        j = self.j
        W = Y.clone()
        hsum = None
        for _ in range(2):                                           # classical Gram-Schmidt, twice
            h = self.ops.krylov_dots(self.Q, W, j + 1)               # (r, j+1) = <q_i, w>
            self.ops.krylov_update(self.Q, h, W, -1.0)
            hsum = h if hsum is None else hsum + h
        hn = self.ops.norms(W)
        self.Q[:, j + 1, :] = W / t.where(hn > 0, hn, t.ones_like(hn)).to(W.dtype)[:, None]
        cdt = t.complex128
        hcol = t.cat([hsum.to(cdt), hn[:, None].to(cdt)], dim=1).cpu().numpy().T.copy()   # (j+2, r)
        for i in range(j):                                           # previous rotations
            tmp = self.cs[i] * hcol[i] + self.sn[i] * hcol[i + 1]
            hcol[i + 1] = -np.conj(self.sn[i]) * hcol[i] + self.cs[i] * hcol[i + 1]
            hcol[i] = tmp
        a, c = hcol[j].copy(), hcol[j + 1].copy()
        absa = np.abs(a)
        den = np.sqrt(absa ** 2 + np.abs(c) ** 2)
        safe = absa > 0
        dsafe = np.where(den > 0, den, 1.0)
        cs = np.where(safe, absa / dsafe, 0.0).astype(np.complex128)
        unit = np.where(safe, a / np.where(safe, absa, 1.0), 1.0)
        sn = np.where(safe, unit * np.conj(c) / dsafe, 1.0).astype(np.complex128)
        self.cs[j], self.sn[j] = cs, sn
        hcol[j] = cs * a + sn * c
        hcol[j + 1] = 0
        self.g[j + 1] = -np.conj(sn) * self.g[j]
        self.g[j] = cs * self.g[j]
        self.H[:, : j + 2, j] = hcol.T
        self.it += 1
        self.j += 1
        self._rel = self._scale(np.abs(self.g[self.j]))

    def close_cycle(self):
        """Solve the small triangular systems (host), update X (device), and ask for
        the true residual."""
        t = self.t
        k = self.j
        if k > 0:
            Hk = self.H[:, :k, :k]
            r = Hk.shape[0]
            y = np.zeros((r, k), dtype=np.complex128)
            for i in range(k - 1, -1, -1):                           # back substitution, all columns at once
                d = Hk[:, i, i]
                acc = self.g[i] - np.einsum("rl,rl->r", Hk[:, i, i + 1:k], y[:, i + 1:k])
                y[:, i] = acc / np.where(d == 0, 1.0, d)
            yq = y if self.X.is_complex() else y.real
            yd = t.as_tensor(np.ascontiguousarray(yq), device=self.X.device).to(self.X.dtype)
            self.ops.krylov_update(self.Q, yd, self.X, 1.0)
        self.phase = "residual"
        self.j = 0

    def fresh(self):
        """True right after a (re)start: _rel is the true relative residual."""
        return self.phase == "arnoldi" and self.j == 0

    def step_done(self):
        """After an Arnoldi step: close the cycle when it is full, when the residual
        estimate meets the tolerance, or when the iteration budget is spent (the
        next product then yields the true residual)."""
        if self.phase == "arnoldi" and self.j > 0:
            if self.j >= self.m or float(self._rel.max()) <= self.tol or self.it >= self.maxit:
                self.close_cycle()

    def relres(self):
        return self.t.as_tensor(self._rel)

    def solution(self):
        return self.X


# ---------------------------------------------------------------------------- requests


@dataclass
class Request:
    rid: int
    mesh: str
    kernel: str
    kappa: float
    b: object                      # n x r tensor (float64 or complex128) on the backend device
    rtol: float = 1e-8
    arrival: float = 0.0
    maxit: int = 1000
    restart: int = 30
    inner_rtol: float = 1e-4
    # runtime
    status: str = "queued"         # queued, active, done, not_converged, failed
    error: str = ""
    start: float = 0.0
    finish: float = 0.0
    iterations: int = 0
    products: int = 0
    result: object = None
    rel_residual: float = float("nan")
    _solver: object = None
    _phase: str = "outer"          # outer (FP64 residual) or inner (Krylov)
    _z: object = None
    _resid: object = None
    _outer_R: object = None
    _bad_product: object = None    # device flag: some product returned a non-finite entry

    @property
    def key(self):
        return (self.mesh, self.kernel, float(self.kappa))

    @property
    def latency(self):
        return self.finish - self.arrival


@dataclass
class _Resident:
    obj: object
    nbytes: int
    stream: object
    active: int = 0
    last_used: float = 0.0


class H2Server:
    """Continuous-batching scheduler (see module docstring)."""

    def __init__(self, backend, mem_budget: float, max_active: int = 32, clock: Callable[[], float] = time.perf_counter):
        self.be = backend
        self.t = __import__("torch")
        # reductions and Gram-Schmidt steps: the backend's own, else plain tensor operations
        self.ops = backend if hasattr(backend, "norms") else _TensorOps
        self.budget = float(mem_budget)
        self.max_active = int(max_active)
        self.clock = clock
        self.meshes: Dict[str, Tuple[np.ndarray, np.ndarray]] = {}
        self.resident: Dict[tuple, _Resident] = {}
        self.queue: List[Request] = []
        self.active: List[Request] = []
        self.finished: List[Request] = []
        self._next = 0
        self._est: Dict[tuple, int] = {}
        self.ticks = 0
        self.batched_products = 0
        self.busy_s = 0.0          # wall time of ticks that issued products (device work and host steps)

    # -- registry ---------------------------------------------------------------------
    def register_mesh(self, name: str, vertices, triangles):
        self.meshes[name] = (np.asarray(vertices, np.float64), np.asarray(triangles, np.int32))

    def submit(self, mesh: str, b, kernel="laplace", kappa=0.0, rtol=1e-8, arrival=None, **kw) -> Request:
        t = self.t
        b = t.as_tensor(b)
        if b.dim() == 1:
            b = b[:, None]
        cx = kernel == "helmholtz"
        # held right-hand-side-major (r, n); results are returned as n x r views
        b = b.to(device=self.be.device, dtype=t.complex128 if cx else t.float64).t().contiguous()
        req = Request(self._next, mesh, kernel, float(kappa), b, rtol=rtol,
                      arrival=self.clock() if arrival is None else arrival, **kw)
        self._next += 1
        if mesh not in self.meshes:
            req.status, req.error = "failed", "unknown mesh %r" % mesh
            self.finished.append(req)
        elif b.shape[1] != self.meshes[mesh][1].shape[0]:
            req.status, req.error = "failed", "right-hand side has %d rows, mesh has %d triangles" % (
                b.shape[1], self.meshes[mesh][1].shape[0])
            self.finished.append(req)
        elif not np.isfinite(self.ops.norms(b).cpu().numpy()).all():
            req.status, req.error = "failed", "right-hand side is not finite"
            self.finished.append(req)
        else:
            self.queue.append(req)
        return req

    # -- memory -----------------------------------------------------------------------
    def used_bytes(self) -> int:
        return sum(r.nbytes for r in self.resident.values()) + sum(self._req_bytes(q) for q in self.active)

    def _req_bytes(self, q: Request) -> int:
        r, n = q.b.shape
        es = q.b.element_size()
        nvec = (q.restart + 6) if q.kernel == "helmholtz" else 8
        return int(n * r * es * nvec)

    def _footprint(self, key) -> int:
        if key not in self._est:
            mesh, kernel, kappa = key
            V, T = self.meshes[mesh]
            self._est[key] = int(self.be.estimate(V, T, kernel, kappa))
        return self._est[key]

    def _make_resident(self, key, extra) -> Optional[_Resident]:
        """The resident structure for `key`, building it if the budget allows after
        evicting idle structures (least recently used first) until the structure
        and `extra` bytes of request vectors fit; None = wait."""
        have = self.resident.get(key)
        nbytes = 0 if have is not None else self._footprint(key)
        while self.used_bytes() + nbytes + extra > self.budget:
            idle = [(r.last_used, k) for k, r in self.resident.items() if r.active == 0 and k != key]
            if not idle:
                return None
            _, victim = min(idle)
            self.be.free(self.resident.pop(victim).obj)
        if have is not None:
            return have
        mesh, kernel, kappa = key
        V, T = self.meshes[mesh]
        obj, real = self.be.build(V, T, kernel, kappa)
        res = _Resident(obj, int(real), self.be.new_stream(), 0, self.clock())
        self.resident[key] = res
        return res

    # -- scheduling ---------------------------------------------------------------------
    def _admit(self, now):
        keep = []
        for q in self.queue:
            if q.arrival > now or len(self.active) >= self.max_active:
                keep.append(q)
                continue
            try:
                need = self._req_bytes(q)
                if self._footprint(q.key) + need > self.budget:
                    q.status, q.error, q.finish = "failed", "does not fit the memory budget", now
                    self.finished.append(q)
                    continue
                res = self._make_resident(q.key, need)
            except Exception as e:  # a failed build fails the request, not the server
                q.status, q.error, q.finish = "failed", "build failed: %s" % e, self.clock()
                self.finished.append(q)
                continue
            if res is None or self.used_bytes() + need > self.budget:
                keep.append(q)
                continue
            res.active += 1
            q.status, q.start = "active", now
            q._z = self.t.zeros_like(q.b)
            q._phase = "outer" if self._refine(q) else "inner"
            if q._phase == "inner":
                q._solver = self._new_solver(q, q.b, q.rtol)
            self.active.append(q)
        self.queue = keep

    def _refine(self, q):
        return self.be.refine()

    def _new_solver(self, q, rhs, tol):
        left = max(1, q.maxit - q.iterations)
        if q.kernel == "helmholtz":
            return _GMRES(self.t, rhs, tol, left, q.restart, self.ops)
        return _CG(self.t, rhs, tol, left, self.ops)

    def _operand(self, q) -> Tuple[object, bool]:
        """The vector block whose product this request needs next, and whether the
        product accumulates in FP64 (outer residual of the refinement)."""
        if q._phase == "outer":
            return q._z, True
        return q._solver.operand(), False

    def tick(self) -> int:
        """Admit arrivals, run one batched product per (structure, accumulation)
        group, advance every active request.  Returns the number of products."""
        t = self.t
        now = self.clock()
        self._admit(now)
        if not self.active:
            return 0
        t_start = time.perf_counter()
        groups: Dict[tuple, List[Request]] = {}
        for q in self.active:
            X, acc64 = self._operand(q)
            groups.setdefault((q.key, acc64), []).append(q)
        outs = {}
        for (key, acc64), reqs in groups.items():
            res = self.resident[key]
            res.last_used = now
            stream = res.stream
            ctx = t.cuda.stream(stream) if stream is not None else _nullcontext()
            with ctx:
                if stream is not None:       # right-hand sides were made on the submitting stream
                    stream.wait_stream(t.cuda.default_stream(stream.device))
                ops = [self._operand(q)[0] for q in reqs]           # (r_i, n) each
                Xr = t.cat(ops, dim=0) if len(ops) > 1 else ops[0].contiguous()
                Yr = t.zeros_like(Xr)
                self.be.matvec(res.obj, Xr.t(), Yr.t(), acc64, stream)  # n x R Fortran views
                outs[(key, acc64)] = (reqs, Yr, [o.shape[0] for o in ops])
            self.batched_products += 1
        # advance (same stream as the group's product)
        for gk, (reqs, Y, widths) in outs.items():
            stream = self.resident[gk[0]].stream
            ctx = t.cuda.stream(stream) if stream is not None else _nullcontext()
            with ctx:
                c0 = 0
                for q, w in zip(reqs, widths):
                    self._advance(q, Y[c0:c0 + w])
                    c0 += w
        if self.be.device.type == "cuda":
            t.cuda.synchronize()
        self._retire()
        self.ticks += 1
        self.busy_s += time.perf_counter() - t_start
        return len(outs)

    def _advance(self, q, Y):
        q.products += 1
        # per column: did the product return a non-finite entry (a non-finite norm)?
        bad = ~self.t.isfinite(self.ops.norms(Y))
        q._bad_product = bad if q._bad_product is None else (q._bad_product | bad)
        if q._phase == "outer":
            R = q.b - Y
            nb = self.ops.norms(q.b)
            q._resid = self.ops.norms(R) / self.t.where(nb > 0, nb, self.t.ones_like(nb))
            q._outer_R = R
            return
        s = q._solver
        s.advance(Y)
        q.iterations += 1

    def _retire(self):
        t = self.t
        now = None
        keep = []
        for q in self.active:
            finished = False
            if q._phase == "outer":
                rel = _host_max(q._resid)
                if not math.isfinite(rel):
                    q.status, q.error, finished = "failed", self._nonfinite(q, "outer residual"), True
                elif rel <= q.rtol:
                    q.status, finished = "done", True
                    q.rel_residual = rel
                elif q.iterations >= q.maxit:
                    q.status, finished = "not_converged", True
                    q.rel_residual = rel
                else:
                    q._phase = "inner"
                    tol = max(q.inner_rtol, 0.5 * q.rtol / rel)
                    q._solver = self._new_solver(q, q._outer_R, tol)
            else:
                s = q._solver
                if isinstance(s, _GMRES):
                    if s.fresh():                   # true residual of the current iterate
                        converged = _host_max(s.relres()) <= s.tol
                        exhausted = s.it >= s.maxit
                    else:
                        s.step_done()
                        converged = exhausted = False
                else:
                    converged = _host_max(s.relres()) <= s.tol
                    exhausted = s.it >= s.maxit
                relmax = _host_max(s.relres())
                if not math.isfinite(relmax):
                    q.status, q.error, finished = "failed", self._nonfinite(q, "inner residual"), True
                elif converged:
                    if self._refine(q):
                        q._z = q._z + s.solution()
                        q._phase = "outer"
                    else:
                        q._z = s.solution()
                        q.status, finished = "done", True
                        q.rel_residual = relmax
                elif exhausted or q.iterations >= q.maxit:
                    if isinstance(s, _GMRES) and s.phase == "arnoldi":
                        s.close_cycle()
                    q._z = (q._z + s.solution()) if self._refine(q) else s.solution()
                    q.status, finished = "not_converged", True
                    q.rel_residual = relmax
            if finished:
                now = self.clock() if now is None else now
                q.finish = now
                q.result = q._z.t()                 # n x r
                q._solver = None
                self.resident[q.key].active -= 1
                self.finished.append(q)
            else:
                keep.append(q)
        self.active = keep

    def _nonfinite(self, q, where):
        """Failure message: which residual, and whether a product itself returned a
        non-finite entry (the library) or only the solver's arithmetic did."""
        from_product = q._bad_product is not None and bool(q._bad_product.cpu().numpy().any())
        detail = "a product returned a non-finite entry" if from_product else "all products were finite"
        s = q._solver
        if isinstance(s, _GMRES):
            detail += "; GMRES step %d of cycle, phase %s" % (s.j, s.phase)
        return "non-finite residual (%s after %d iterations; %s)" % (where, q.iterations, detail)

    def run(self, until_idle=True, max_ticks=10 ** 9, progress: Optional[Callable[[dict], None]] = None,
            progress_every: float = 5.0, deadline: Optional[float] = None):
        """Serve until the queue and the slots are empty.  `progress` is called with
        stats() at most every `progress_every` seconds; past `deadline` (clock
        value) unfinished requests are cancelled (status "cancelled")."""
        last = self.clock()
        while (self.queue or self.active) and self.ticks < max_ticks:
            if deadline is not None and self.clock() > deadline:
                for q in self.queue + self.active:
                    q.status, q.error, q.finish = "cancelled", "deadline", self.clock()
                    if q in self.active:
                        self.resident[q.key].active -= 1
                    self.finished.append(q)
                self.queue, self.active = [], []
                break
            if progress is not None and self.clock() - last >= progress_every:
                last = self.clock()
                progress(dict(self.stats(), active=len(self.active), queued=len(self.queue),
                              active_iterations=[q.iterations for q in self.active][:8]))
            if not self.active and self.queue and min(q.arrival for q in self.queue) > self.clock():
                time.sleep(min(1e-3, max(0.0, min(q.arrival for q in self.queue) - self.clock())))
                continue
            n = self.tick()
            if n == 0 and not self.active and not self.queue:
                break
            if n == 0 and self.queue and not self.active:
                # nothing admissible right now (memory or arrivals): do not spin on a stuck queue
                if all(q.arrival <= self.clock() for q in self.queue):
                    for q in self.queue:
                        q.status, q.error, q.finish = "failed", "does not fit the memory budget", self.clock()
                        self.finished.append(q)
                    self.queue = []

    def stats(self) -> dict:
        done = [q for q in self.finished if q.status == "done"]
        lat = np.array([q.latency for q in done]) if done else np.zeros(0)
        span = (max(q.finish for q in self.finished) - min(q.arrival for q in self.finished)) if self.finished else 0.0
        return {
            "requests": len(self.finished), "done": len(done),
            "failed": sum(q.status == "failed" for q in self.finished),
            "cancelled": sum(q.status == "cancelled" for q in self.finished),
            "not_converged": sum(q.status == "not_converged" for q in self.finished),
            "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_s": float(lat.mean()) if lat.size else None,
            "throughput_req_s": len(done) / span if span > 0 else None,
            "rhs_solved": int(sum(q.b.shape[0] for q in done)),
            "ticks": self.ticks, "batched_products": self.batched_products,
            "busy_s": self.busy_s, "busy_frac": self.busy_s / span if span > 0 else None,
            "errors": dict(Counter(q.error for q in self.finished if q.status in ("failed", "cancelled"))),
        }

    def failures(self) -> List[dict]:
        """What each failed or unconverged request was and why (mesh, kernel, width,
        iterations, last relative residual)."""
        return [{"rid": q.rid, "status": q.status, "mesh": q.mesh, "kernel": q.kernel, "kappa": q.kappa,
                 "rhs": int(q.b.shape[0]), "iterations": q.iterations, "products": q.products,
                 "rel_residual": q.rel_residual, "error": q.error}
                for q in self.finished if q.status in ("failed", "not_converged")]


def _host_max(v) -> float:
    """Largest entry of a small vector (tensor on any device, or array), taken on
    the host (NaN if any entry is NaN)."""
    a = v.cpu().numpy() if hasattr(v, "cpu") else np.asarray(v)
    return float(np.max(a)) if a.size else float("nan")


class _nullcontext:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False
