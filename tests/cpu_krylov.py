"""A CPU model of the library's step-wise Krylov solver (h2_krylov_* in
include/h2.h), for driving the solve service without a GPU.  TEST
INFRASTRUCTURE ONLY.

It keeps the same protocol and control decisions as the native solver -- `next`
writes the block whose product is needed (or, with x = None, only reports the
flags), `advance` consumes the product, `poll` decides; outer residuals of a
refinement ask for FP64 accumulation; CG or restarted GMRES(m) with classical
Gram-Schmidt twice and complex Givens rotations run all columns in lockstep --
in plain torch CPU arithmetic.
"""
import math
from types import SimpleNamespace

import torch

ACC_F64 = 1
PRODUCT, DONE, NOTCONV, FAILED = 1, 2, 3, 4
NAMES = {PRODUCT: "product", DONE: "done", NOTCONV: "not_converged", FAILED: "failed"}


def params(method="cg", rtol=1e-8, maxit=1000, restart=30, refine=False, inner_rtol=1e-4):
    return SimpleNamespace(method=method, rtol=rtol, maxit=maxit, restart=restart, refine=refine,
                           inner_rtol=inner_rtol)


def workspace_bytes(n, r, cx, p):
    """Bytes the native solver would need (vectors only; same order of size)."""
    nvec = 5 if p.method == "cg" else 4 + p.restart
    return 8 * (2 if cx else 1) * n * r * nvec


def _dots(A, B):
    """<a_c, b_c> per column of n x r blocks (conjugating A)."""
    return ((A.conj() if A.is_complex() else A) * B).sum(0)


class CPUKrylov:
    def __init__(self, n, r, cx, p):
        self.n, self.r, self.cx, self.P = n, r, cx, p
        self.cg = p.method == "cg"
        self.m = 0 if self.cg else p.restart
        self.state, self.iterations, self.outer, self.products = PRODUCT, 0, 0, 0
        self.last_rel, self.message = 1.0, ""
        self.max_outer = 30 if p.refine else 5
        self.bad = 0

    # ------------------------------------------------------------------ protocol
    def begin(self, b, z0=None, stream=None):
        self.B = b
        self.nb = torch.sqrt(_dots(b, b).real)
        self.Z = torch.zeros_like(b)
        self.rel_out = (self.nb > 0).to(torch.float64)
        self.rel_in = torch.zeros(self.r, dtype=torch.float64)
        self.pend_inner = self.pend_close = self.pend_zupd = False
        if z0 is not None:
            self.Z = torch.where(self.nb[None, :] > 0, z0, torch.zeros_like(z0))
            self.phase = "outer"
        else:
            self.rhs = self.B
            self.outer += 1
            self._start_inner(1.0)

    def _start_inner(self, rel):
        p = self.P
        tol = max(p.inner_rtol, 0.5 * p.rtol / rel) if p.refine else p.rtol / rel
        self.inner_tol = min(tol, 1.0)
        self.pend_inner = True
        self.pend_close = self.pend_zupd = False
        self.phase = "cg" if self.cg else "arnoldi"
        self.j = 0

    def _flags(self):
        outer_next = self.pend_zupd or (self.phase == "outer" and not self.pend_inner and not self.pend_close)
        return ACC_F64 if outer_next and self.P.refine else 0

    def next(self, x=None, stream=None):
        if self.state != PRODUCT:
            return self.state, 0
        if x is None:
            return self.state, self._flags()
        fl = self._flags()
        if self.pend_inner:
            self.pend_inner = False
            F = self.rhs
            if self.cg:
                self.X = torch.zeros_like(F)
                self.R = F.clone()
                self.Pd = F.clone()
                self.rr = _dots(F, F).real
                self.nb_in = torch.sqrt(self.rr)
                self.rel_in = (self.rr > 0).to(torch.float64)
            else:
                self.X = torch.zeros_like(F)
                beta = torch.sqrt(_dots(F, F).real)
                self.nb_in = beta
                self._restart(F, beta)
        if self.pend_close:
            self.pend_close = False
            k = self.j
            y = torch.zeros((k, self.r), dtype=torch.complex128)
            for i in range(k - 1, -1, -1):
                acc = self.g[i].clone()
                for l in range(i + 1, k):
                    acc -= self.H[i, l] * y[l]
                d = self.H[i, i]
                y[i] = torch.where(d.abs() > 0, acc / torch.where(d.abs() > 0, d, torch.ones_like(d)),
                                   torch.zeros_like(acc))
            yq = y if self.cx else y.real
            for i in range(k):
                self.X += yq[i][None, :] * self.Q[i]
            self.phase = "resid"
        if self.pend_zupd:
            self.pend_zupd = False
            self.Z += self.X
            self.phase = "outer"
        src = {"outer": lambda: self.Z, "cg": lambda: self.Pd, "arnoldi": lambda: self.Q[self.j],
               "resid": lambda: self.X}[self.phase]()
        x.copy_(src)
        return self.state, fl

    def _restart(self, R, beta):
        m = max(self.m, 1)
        self.Q = [R / torch.where(beta > 0, beta, torch.ones_like(beta))[None, :].to(R.dtype)] + \
                 [None] * m
        self.H = torch.zeros((m + 1, m, self.r), dtype=torch.complex128)
        self.cs = torch.zeros((m, self.r), dtype=torch.complex128)
        self.sn = torch.zeros((m, self.r), dtype=torch.complex128)
        self.g = torch.zeros((m + 1, self.r), dtype=torch.complex128)
        self.g[0] = beta.to(torch.complex128)
        self.rel_in = torch.where(self.nb_in > 0, beta / torch.where(self.nb_in > 0, self.nb_in,
                                                                     torch.ones_like(beta)), torch.zeros_like(beta))
        self.j = 0

    def _mark(self, v, from_product):
        if self.bad == 0 and not bool(torch.isfinite(torch.as_tensor(v)).all()):
            self.bad = 1 if from_product else 2

    def advance(self, y, stream=None):
        self.products += 1
        Y = y.clone()
        if self.phase == "outer":
            self.Ro = self.B - Y
            nr = torch.sqrt(_dots(self.Ro, self.Ro).real)
            self._mark(nr, True)
            self.rel_out = torch.where(self.nb > 0, nr / torch.where(self.nb > 0, self.nb, torch.ones_like(nr)),
                                       torch.zeros_like(nr))
        elif self.phase == "cg":
            pq = _dots(self.Pd, Y).real
            self._mark(pq, True)
            ok = (pq > 0) & torch.isfinite(pq)
            alpha = torch.where(ok, self.rr / torch.where(ok, pq, torch.ones_like(pq)), torch.zeros_like(pq))
            self.X += alpha[None, :] * self.Pd
            self.R -= alpha[None, :] * Y
            rr2 = _dots(self.R, self.R).real
            self._mark(rr2, False)
            beta = torch.where(self.rr > 0, rr2 / torch.where(self.rr > 0, self.rr, torch.ones_like(rr2)),
                               torch.zeros_like(rr2))
            self.Pd = self.R + beta[None, :] * self.Pd
            self.rr = rr2
            self.rel_in = torch.where(self.nb_in > 0, torch.sqrt(rr2) / torch.where(self.nb_in > 0, self.nb_in,
                                                                                    torch.ones_like(rr2)),
                                      torch.zeros_like(rr2))
            self.iterations += 1
        elif self.phase == "arnoldi":
            j = self.j
            hsum = torch.zeros((j + 2, self.r), dtype=torch.complex128)
            W = Y
            for npass in range(2):                                    # classical Gram-Schmidt, twice
                h = torch.stack([_dots(self.Q[i], W) for i in range(j + 1)]).to(torch.complex128)
                self._mark(h, npass == 0)
                hq = h if self.cx else h.real
                W = W - sum(hq[i][None, :] * self.Q[i] for i in range(j + 1))
                hsum[: j + 1] += h
            hn = torch.sqrt(_dots(W, W).real)
            self._mark(hn, False)
            self.Q[j + 1] = W * torch.where(hn > 0, 1.0 / torch.where(hn > 0, hn, torch.ones_like(hn)),
                                            torch.zeros_like(hn))[None, :].to(W.dtype)
            hsum[j + 1] = hn
            for i in range(j):                                        # the earlier rotations
                a, b = hsum[i].clone(), hsum[i + 1].clone()
                hsum[i + 1] = self.cs[i] * b - self.sn[i].conj() * a
                hsum[i] = self.cs[i] * a + self.sn[i] * b
            a, b = hsum[j].clone(), hsum[j + 1].clone()
            aa = a.abs()
            den = torch.sqrt(aa ** 2 + b.abs() ** 2)
            safe = aa > 0
            cj = torch.where(safe, aa / torch.where(safe, den, torch.ones_like(den)), torch.zeros_like(aa))
            unit = torch.where(safe, a / torch.where(safe, aa, torch.ones_like(aa)), torch.ones_like(a))
            sj = torch.where(safe, unit * b.conj() / torch.where(safe, den, torch.ones_like(den)),
                             torch.ones_like(a))
            cj = cj.to(torch.complex128)
            self.cs[j], self.sn[j] = cj, sj
            hsum[j] = cj * a + sj * b
            gj = self.g[j].clone()
            self.g[j + 1] = -sj.conj() * gj
            self.g[j] = cj * gj
            self.H[: j + 1, j] = hsum[: j + 1]
            gn = self.g[j + 1].abs()
            self.rel_in = torch.where(self.nb_in > 0, gn / torch.where(self.nb_in > 0, self.nb_in,
                                                                       torch.ones_like(gn)), torch.zeros_like(gn))
            self.j += 1
            self.iterations += 1
        else:                                                         # end of a cycle: true inner residual
            R = self.rhs - Y
            beta = torch.sqrt(_dots(R, R).real)
            self._mark(beta, True)
            self._restart(R, beta)

    def poll(self):
        if self.state == PRODUCT:
            self._decide()
        return dict(state=NAMES[self.state], iterations=self.iterations, outer=self.outer, products=self.products,
                    rel_residual=self.last_rel, message=self.message)

    def _decide(self):
        rel_out = float(self.rel_out.max())
        rel_in = float(self.rel_in.max())
        if self.bad or math.isnan(rel_out) or math.isnan(rel_in):
            self.state = FAILED
            self.message = ("non-finite outer residual" if self.phase == "outer" else "non-finite inner residual") + \
                " after %d iterations; " % self.iterations + \
                ("a product returned a non-finite entry" if self.bad == 1 else "all products were finite")
            return
        self.last_rel = rel_out if self.phase == "outer" else rel_in
        p = self.P
        if self.phase == "outer":
            if rel_out <= p.rtol:
                self.state = DONE
            elif self.iterations >= p.maxit or self.outer >= self.max_outer:
                self.state = NOTCONV
            else:
                self.rhs = self.Ro
                self.outer += 1
                self._start_inner(rel_out)
        elif self.phase == "cg":
            if rel_in <= self.inner_tol or self.iterations >= p.maxit:
                self.pend_zupd = True
        elif self.phase == "arnoldi":
            if self.j >= self.m or rel_in <= self.inner_tol or self.iterations >= p.maxit:
                self.pend_close = True
        else:
            if rel_in <= self.inner_tol or self.iterations >= p.maxit:
                self.pend_zupd = True
            else:
                self.phase = "arnoldi"

    def residuals(self):
        return self.rel_out.numpy().copy()

    def solution(self, z, stream=None):
        z.copy_(self.Z)

    def close(self):
        pass
