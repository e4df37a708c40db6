"""Continuous-batching solve service over HBM-resident H^2 matrices.

Requests ask for G~ Z = B on a registered mesh (Laplace, or Helmholtz with a
wave number) with 1..R right-hand sides.  The engine

* keeps the H^2 structures resident on the device and admits a structure by its
  footprint against a memory budget, evicting idle structures (least recently
  used first) when a new one does not fit;
* holds every request's Krylov vectors in one device arena allocated when the
  server starts (a request waits while its vectors do not fit), and its residual
  status in a pinned host pool, so serving allocates no device memory per tick;
* admits requests into a bounded number of slots as slots and memory free up;
* runs every admitted request on the library's step-wise Krylov solver
  (h2_krylov_* in include/h2.h: CG for the symmetric positive definite Laplace
  matrix, restarted GMRES for Helmholtz, FP64 iterative refinement for FP32
  storage), whose vector algebra, inner products and small solves all run in
  the library's kernels;
* steps every resident structure on its own stream and at its own pace: when
  the structure's previous step has completed on the device (an event, polled
  without blocking), it retires its finished requests, asks each remaining one
  which product it needs, groups them by product flags (outer residuals of a
  refinement accumulate in FP64), lets each solver write its operand into the
  structure's product buffer, and issues ONE many-right-hand-side product per
  group (in chunks of at most `product_width` columns), then the solvers' update
  steps, and records a new event.  Requests on different meshes overlap on the
  device without waiting for each other's steps (a small mesh iterates while a
  large one computes), and requests on the same mesh share one pass over its
  matrix data;
* reports per-request latency (arrival to result), p50/p99 and throughput.

A backend object supplies the structures, the products and the solvers, so the
scheduler can also be driven by a CPU backend in tests.
"""
from __future__ import annotations

import math
import time
from collections import Counter
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

ACC_F64 = 1                     # h2_matvec flag: FP64 accumulation (outer residual of a refinement)

# ---------------------------------------------------------------------------- GPU backend


class _Structure:
    """A resident H^2 matrix with its product buffers X, Y (n x width, Fortran order)."""

    def __init__(self, A, X, Y):
        self.A, self.X, self.Y = A, X, Y


class GPUBackend:
    """H^2 matrices, products and Krylov solvers of the HIP library; vectors are
    CUDA tensors.  Device memory is allocated only when a structure is built and
    once for the request arena."""

    def __init__(self, order=4, leaf=64, eta=0.5, storage="f32", device="cuda", coupling_otf=False,
                 product_width=64):
        import torch
        from . import h2
        self.torch, self.h2 = torch, h2
        self.order, self.leaf, self.eta, self.storage = order, leaf, eta, storage
        self.device = torch.device(device)
        # real kernels may evaluate the coupling matrices during each product instead of storing them
        self.coupling_otf = coupling_otf
        self.product_width = int(product_width)

    def _otf(self, kernel):
        if not self.coupling_otf:
            return False
        if kernel == "helmholtz":          # FP32 evaluation of e^{i kappa r}/(4 pi r), m = 4
            return self.storage == "f32" and self.order == 4
        return self.storage in ("f32", "f64")

    def estimate(self, V, T, kernel, kappa):
        """Device bytes of the structure and its product buffers, from a host-only
        build of its trees."""
        h2 = self.h2
        h = h2.build_h2(V, T, kernel=kernel, kappa=kappa, order=self.order, leaf=self.leaf, eta=self.eta,
                        storage=self.storage, host_only=True)
        try:
            i = h2.h2_info(h)
        finally:
            h2.h2_free(h)
        cw = 2 if kernel == "helmholtz" else 1
        vb = 8 if self.storage == "f64" else 4
        sb = {"f64": 8, "f32": 4, "f32_sbf16": 6}[self.storage]     # BF16 S keeps an FP32 copy
        k, n, nc = i["k"], i["n"], i["nclusters"]
        s_bytes = 0 if self._otf(kernel) else sb * k * k * i["n_adm"]
        data = cw * (s_bytes + vb * i["near_entries"]) + vb * (4 * n * k + 2 * k * k * nc + 48 * nc) + 8 * 15 * nc
        work = 2 * 8 * cw * (n + nc * k) + 4 * 64 * (2 * n + 2 * nc * k)   # one- and many-RHS workspaces
        return int(data + work + self._buffers_bytes(n, kernel))

    def _buffers_bytes(self, n, kernel):
        return 2 * n * self.product_width * (16 if kernel == "helmholtz" else 8)

    def build(self, V, T, kernel, kappa):
        t = self.torch
        A = self.h2.H2Matrix(V, T, kernel=kernel, kappa=kappa, order=self.order, leaf=self.leaf, eta=self.eta,
                             storage=self.storage, coupling_otf=self._otf(kernel))
        dt = t.complex128 if kernel == "helmholtz" else t.float64
        n, w = A.n, self.product_width
        X = t.zeros((w, n), dtype=dt, device=self.device).t()
        Y = t.zeros((w, n), dtype=dt, device=self.device).t()
        return _Structure(A, X, Y), self.estimate(V, T, kernel, kappa)

    def buffers(self, S):
        return S.X, S.Y

    def matvec(self, S, ncols, flags, stream):
        """Y[:, :ncols] <- G~ X[:, :ncols] (flags: ACC_F64 or 0)."""
        S.A.matvec(S.X[:, :ncols], S.Y[:, :ncols], alpha=1.0, acc64=bool(flags & ACC_F64),
                   stream=stream.cuda_stream if stream is not None else None, overwrite=True)

    def free(self, S):
        S.A.close()
        S.X = S.Y = None

    def new_stream(self):
        return self.torch.cuda.Stream(device=self.device)

    def mark(self, stream):
        """An event recorded on `stream` now (the end of the work issued so far)."""
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return ev

    def refine(self):
        return self.storage != "f64"

    # request memory: one arena of device bytes and a pinned status pool, made once
    def request_arena(self, nbytes):
        self._arena = self.torch.empty(int(nbytes) + 256, dtype=self.torch.uint8, device=self.device)
        return (self._arena.data_ptr() + 255) // 256 * 256

    def status_pool(self, slots, per_slot):
        self._status = self.torch.zeros((slots, per_slot), dtype=self.torch.float64, pin_memory=True)
        return self._status.data_ptr()

    def solver_params(self, method, rtol, maxit, restart, refine, inner_rtol):
        return self.h2.solve_params(method, rtol, maxit, restart, refine, inner_rtol)

    def workspace_bytes(self, n, r, complex_, params):
        return self.h2.KrylovSolve.workspace_bytes(n, r, complex_, params)

    def new_solver(self, n, r, complex_, params, ws_ptr, ws_bytes, status_ptr):
        return self.h2.KrylovSolve(n, r, complex_, params, ws_ptr, ws_bytes, status_ptr)

    def to_device(self, b, complex_):
        """The right-hand sides as a Fortran-ordered n x r device block (allocated at submit)."""
        t = self.torch
        b = t.as_tensor(b)
        if b.dim() == 1:
            b = b[:, None]
        dt = t.complex128 if complex_ else t.float64
        return b.to(dtype=dt).t().contiguous().to(self.device).t()

    def empty_like(self, b):
        return self.torch.zeros((b.shape[1], b.shape[0]), dtype=b.dtype, device=b.device).t()

    def all_finite(self, b):
        """Whether every entry of a device block is finite, from the library's own
        reduction (FP64 norms; a non-finite entry gives a non-finite norm)."""
        B = b.t()                                                  # (r, n), rows contiguous
        d = self.h2.h2_krylov_dots(B[:, None, :], B, 1)[:, 0]
        return bool(np.isfinite(d.cpu().numpy()).all())


# ---------------------------------------------------------------------------- requests


@dataclass
class Request:
    rid: int
    mesh: str
    kernel: str
    kappa: float
    b: object                      # n x r block (Fortran order) on the backend device
    rtol: float = 1e-8
    arrival: float = 0.0
    maxit: int = 1000
    restart: int = 30
    inner_rtol: float = 1e-4
    # runtime
    status: str = "queued"         # queued, active, done, not_converged, failed, cancelled
    error: str = ""
    start: float = 0.0
    finish: float = 0.0
    iterations: int = 0
    products: int = 0
    result: object = None          # n x r block, written when the request ends
    rel_residual: float = float("nan")
    _solver: object = None
    _ws: Optional[Tuple[int, int]] = None    # (offset, bytes) in the request arena
    _slot: int = -1                # pinned status slot

    @property
    def key(self):
        return (self.mesh, self.kernel, float(self.kappa))

    @property
    def nrhs(self):
        return int(self.b.shape[1])

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
    pending: object = None         # event at the end of the structure's last issued step


class _Arena:
    """First-fit sub-allocation of [0, size) in 256-byte units (offsets only)."""

    def __init__(self, size):
        self.size = int(size)
        self.free_list = [(0, self.size)]            # sorted (offset, length)

    def alloc(self, nbytes):
        need = (int(nbytes) + 255) // 256 * 256
        for i, (o, ln) in enumerate(self.free_list):
            if ln >= need:
                if ln == need:
                    del self.free_list[i]
                else:
                    self.free_list[i] = (o + need, ln - need)
                return o, need
        return None

    def free(self, block):
        o, ln = block
        fl = self.free_list
        fl.append((o, ln))
        fl.sort()
        merged = [fl[0]]
        for a, b in fl[1:]:
            po, pl = merged[-1]
            if po + pl == a:
                merged[-1] = (po, pl + b)
            else:
                merged.append((a, b))
        self.free_list = merged

    def used(self):
        return self.size - sum(ln for _, ln in self.free_list)


class H2Server:
    """Continuous-batching scheduler (see module docstring)."""

    def __init__(self, backend, mem_budget: float, max_active: int = 32, clock: Callable[[], float] = time.perf_counter,
                 vec_budget: Optional[float] = None, max_rhs: int = 64):
        self.be = backend
        self.budget = float(mem_budget)
        self.max_active = int(max_active)
        self.max_rhs = int(max_rhs)
        self.clock = clock
        # request vectors: a fixed share of the budget, allocated now
        self.vec_budget = int(0.25 * self.budget if vec_budget is None else vec_budget)
        self.arena = _Arena(self.vec_budget)
        self.arena_base = backend.request_arena(self.vec_budget)
        self._per_slot = 3 * self.max_rhs
        self.status_base = backend.status_pool(self.max_active, self._per_slot)
        self.free_slots = list(range(self.max_active))
        self.meshes: Dict[str, Tuple[np.ndarray, np.ndarray]] = {}
        self.resident: Dict[tuple, _Resident] = {}
        self.queue: List[Request] = []
        self.active: List[Request] = []
        self.finished: List[Request] = []
        self._next = 0
        self._est: Dict[tuple, int] = {}
        self.ticks = 0
        self.batched_products = 0
        self.busy_s = 0.0          # wall time with at least one request active (solving or waiting on the device)
        self.host_s = 0.0          # wall time of ticks that issued steps (host side of the scheduler)
        self._t_last = None        # clock of the previous tick, while requests were active

    # -- registry ---------------------------------------------------------------------
    def register_mesh(self, name: str, vertices, triangles):
        self.meshes[name] = (np.asarray(vertices, np.float64), np.asarray(triangles, np.int32))

    def submit(self, mesh: str, b, kernel="laplace", kappa=0.0, rtol=1e-8, arrival=None, **kw) -> Request:
        cx = kernel == "helmholtz"
        on_device = getattr(b, "is_cuda", False)
        bh = None if on_device else (b.numpy() if hasattr(b, "numpy") else np.asarray(b))
        bd = self.be.to_device(b, cx)                   # n x r (Fortran) on the backend device
        req = Request(self._next, mesh, kernel, float(kappa), bd, rtol=rtol,
                      arrival=self.clock() if arrival is None else arrival, **kw)
        self._next += 1
        if mesh not in self.meshes:
            req.status, req.error = "failed", "unknown mesh %r" % mesh
        elif bd.shape[0] != self.meshes[mesh][1].shape[0]:
            req.status, req.error = "failed", "right-hand side has %d rows, mesh has %d triangles" % (
                bd.shape[0], self.meshes[mesh][1].shape[0])
        elif not 1 <= bd.shape[1] <= self.max_rhs:
            req.status, req.error = "failed", "between 1 and %d right-hand sides per request" % self.max_rhs
        elif not (np.isfinite(bh).all() if bh is not None else self.be.all_finite(bd)):
            req.status, req.error = "failed", "right-hand side is not finite"
        else:
            req.result = self.be.empty_like(bd)
            self.queue.append(req)
            return req
        self.finished.append(req)
        return req

    # -- memory -----------------------------------------------------------------------
    def used_bytes(self) -> int:
        """Structures plus the request arena (its whole size: it is allocated at start)."""
        return sum(r.nbytes for r in self.resident.values()) + self.vec_budget

    def _params(self, q):
        method = "gmres" if q.kernel == "helmholtz" else "cg"
        return self.be.solver_params(method, q.rtol, q.maxit, q.restart, self.be.refine(), q.inner_rtol)

    def _ws_bytes(self, q) -> int:
        return self.be.workspace_bytes(q.b.shape[0], q.nrhs, q.kernel == "helmholtz", self._params(q))

    def _footprint(self, key) -> int:
        if key not in self._est:
            mesh, kernel, kappa = key
            V, T = self.meshes[mesh]
            self._est[key] = int(self.be.estimate(V, T, kernel, kappa))
        return self._est[key]

    def _make_resident(self, key) -> Optional[_Resident]:
        """The resident structure for `key`, building it if the budget allows after
        evicting idle structures (least recently used first); None = wait."""
        have = self.resident.get(key)
        if have is not None:
            return have
        nbytes = self._footprint(key)
        while self.used_bytes() + nbytes > self.budget:
            idle = [(r.last_used, k) for k, r in self.resident.items() if r.active == 0]
            if not idle:
                return None
            _, victim = min(idle)
            self.be.free(self.resident.pop(victim).obj)
        mesh, kernel, kappa = key
        V, T = self.meshes[mesh]
        obj, real = self.be.build(V, T, kernel, kappa)
        res = _Resident(obj, int(real), self.be.new_stream(), 0, self.clock())
        self.resident[key] = res
        return res

    # -- scheduling ---------------------------------------------------------------------
    def _fail(self, q, msg, when=None):
        q.status, q.error, q.finish = "failed", msg, self.clock() if when is None else when
        self.finished.append(q)

    def _admit(self, now):
        keep = []
        for q in self.queue:
            if q.arrival > now or len(self.active) >= self.max_active:
                keep.append(q)
                continue
            try:
                need = self._ws_bytes(q)
                if need > self.vec_budget:
                    self._fail(q, "request vectors do not fit the memory budget", now)
                    continue
                if self._footprint(q.key) + self.vec_budget > self.budget:
                    self._fail(q, "structure does not fit the memory budget", now)
                    continue
                ws = self.arena.alloc(need)
                if ws is None:                               # wait for other requests' vectors
                    keep.append(q)
                    continue
                res = self._make_resident(q.key)
            except Exception as e:  # a failed build fails the request, not the server
                self._fail(q, "build failed: %s" % e)
                continue
            if res is None:
                self.arena.free(ws)
                keep.append(q)
                continue
            slot = self.free_slots.pop()
            try:
                base = None if self.arena_base is None else self.arena_base + ws[0]
                status = None if self.status_base is None else self.status_base + 8 * self._per_slot * slot
                q._solver = self.be.new_solver(q.b.shape[0], q.nrhs, q.kernel == "helmholtz", self._params(q),
                                               base, ws[1], status)
                with self._on(res.stream):
                    if res.stream is not None:                # the right-hand sides came from the default stream
                        res.stream.wait_stream(self.be.torch.cuda.default_stream(res.stream.device))
                    q._solver.begin(q.b, None, self._sid(res.stream))
                self._mark(res)                               # its status is read after this completes
            except Exception as e:
                self.arena.free(ws)
                self.free_slots.append(slot)
                self._fail(q, "solver failed to start: %s" % e)
                continue
            q._ws, q._slot = ws, slot
            res.active += 1
            q.status, q.start = "active", now
            self.active.append(q)
        self.queue = keep

    @staticmethod
    def _sid(stream):
        return stream.cuda_stream if stream is not None else None

    def _on(self, stream):
        if stream is None:
            return _nullcontext()
        return self.be.torch.cuda.stream(stream)

    def _mark(self, res):
        if res.stream is not None:
            res.pending = self.be.mark(res.stream)

    @staticmethod
    def _ready(res):
        """Whether the structure's last issued step has completed on the device."""
        return res.pending is None or res.pending.query()

    def tick(self) -> int:
        """Admit arrivals; for every structure whose last step has completed,
        retire its finished requests and issue its next step (one product per
        flags group and chunk, then every request's update).  Returns the number
        of products issued; waits briefly when no structure is ready."""
        now = self.clock()
        t_start = time.perf_counter()
        if self._t_last is not None:
            self.busy_s += t_start - self._t_last
        self._admit(now)
        self._t_last = t_start if self.active else None
        if not self.active:
            return 0
        by_key: Dict[tuple, List[Request]] = {}
        for q in self.active:
            by_key.setdefault(q.key, []).append(q)
        width = getattr(self.be, "product_width", self.max_rhs)
        nprod = 0
        stepped = False
        n_before = len(self.active)
        for key, reqs in by_key.items():
            res = self.resident[key]
            if not self._ready(res):
                continue
            stepped = True
            res.last_used = now
            reqs = self._retire(res, reqs)
            if not reqs:
                continue
            sid = self._sid(res.stream)
            X, Y = self.be.buffers(res.obj)
            classes: Dict[int, List[Request]] = {}
            for q in reqs:
                state, flags = q._solver.next(None)
                if state == 1:                                # another product is needed
                    classes.setdefault(flags, []).append(q)
            with self._on(res.stream):
                for flags, qs in classes.items():
                    for chunk in _chunks(qs, width):
                        off = 0
                        for q in chunk:
                            q._solver.next(X[:, off:off + q.nrhs], sid)
                            off += q.nrhs
                        self.be.matvec(res.obj, off, flags, res.stream)
                        off = 0
                        for q in chunk:
                            q._solver.advance(Y[:, off:off + q.nrhs], sid)
                            off += q.nrhs
                        nprod += 1
            self._mark(res)
        if not stepped:                                       # every structure is busy on the device
            time.sleep(1e-4)
            return nprod
        if len(self.active) < n_before:                       # requests finished: their room is free now
            self._admit(self.clock())
        self.batched_products += nprod
        self.ticks += 1
        self.host_s += time.perf_counter() - t_start
        return nprod

    def _sync(self):
        if self.be.device.type == "cuda":
            self.be.torch.cuda.synchronize()

    def _retire(self, res, reqs):
        """Finish the requests of `res` whose solver has stopped (the structure's
        last step has completed, so their status is current); returns the others."""
        keep, done = [], []
        for q in reqs:
            st = q._solver.poll()
            q.iterations, q.products = st["iterations"], st["products"]
            if st["state"] == "product":
                keep.append(q)
                continue
            q.rel_residual = st["rel_residual"]
            q.status = st["state"]
            if q.status == "failed":
                q.error = "%s (%d right-hand sides)" % (st["message"], q.nrhs)
            with self._on(res.stream):
                q._solver.solution(q.result, self._sid(res.stream))
            done.append(q)
        if done:
            if res.stream is not None:
                res.stream.synchronize()                      # the solutions are copied before release
            now = self.clock()
            for q in done:
                q.finish = now
                self._release(q)
                self.finished.append(q)
            gone = set(id(q) for q in done)
            self.active = [q for q in self.active if id(q) not in gone]
        return keep

    def _release(self, q):
        q._solver.close()
        q._solver = None
        self.arena.free(q._ws)
        self.free_slots.append(q._slot)
        q._ws, q._slot = None, -1
        self.resident[q.key].active -= 1

    def run(self, until_idle=True, max_ticks=10 ** 9, progress: Optional[Callable[[dict], None]] = None,
            progress_every: float = 5.0, deadline: Optional[float] = None):
        """Serve until the queue and the slots are empty.  `progress` is called with
        stats() at most every `progress_every` seconds; past `deadline` (clock
        value) unfinished requests are cancelled (status "cancelled")."""
        last = self.clock()
        while (self.queue or self.active) and self.ticks < max_ticks:
            if deadline is not None and self.clock() > deadline:
                self._sync()
                for q in self.queue + self.active:
                    q.status, q.error, q.finish = "cancelled", "deadline", self.clock()
                    if q._solver is not None:
                        self._release(q)
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
                        self._fail(q, "does not fit the memory budget")
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
            "rhs_solved": int(sum(q.nrhs for q in done)),
            "ticks": self.ticks, "batched_products": self.batched_products,
            "busy_s": self.busy_s, "busy_frac": self.busy_s / span if span > 0 else None,
            "host_s": self.host_s,
            "errors": dict(Counter(q.error for q in self.finished if q.status in ("failed", "cancelled"))),
        }

    def failures(self) -> List[dict]:
        """What each failed or unconverged request was and why (mesh, kernel, width,
        iterations, last relative residual)."""
        return [{"rid": q.rid, "status": q.status, "mesh": q.mesh, "kernel": q.kernel, "kappa": q.kappa,
                 "rhs": q.nrhs, "iterations": q.iterations, "products": q.products,
                 "rel_residual": q.rel_residual, "error": q.error}
                for q in self.finished if q.status in ("failed", "not_converged")]


def _chunks(qs, width):
    """Consecutive groups of requests of at most `width` columns in all."""
    out, cur, w = [], [], 0
    for q in qs:
        if cur and w + q.nrhs > width:
            out.append(cur)
            cur, w = [], 0
        cur.append(q)
        w += q.nrhs
    if cur:
        out.append(cur)
    return out


class _nullcontext:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False
