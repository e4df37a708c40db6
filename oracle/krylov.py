"""Krylov solvers for G z = b in FP64 (the paper's introduction names Krylov methods).

TEST INFRASTRUCTURE ONLY.  Textbook conjugate gradients (for the symmetric
positive definite Laplace single-layer matrix) and restarted GMRES with
modified Gram-Schmidt and Givens rotations (for any nonsingular matrix,
including the complex symmetric Helmholtz matrix).  The stopping test is the
relative residual ||b - G z|| / ||b|| <= rtol of the recursively updated
residual; callers recompute the true residual themselves.
"""
from __future__ import annotations

import numpy as np


def cg(matvec, b, rtol=1e-8, maxit=1000, z0=None):
    b = np.asarray(b)
    z = np.zeros_like(b) if z0 is None else np.array(z0, dtype=b.dtype)
    r = b - matvec(z)
    p = r.copy()
    rr = np.vdot(r, r).real
    nb = np.linalg.norm(b)
    hist = [np.sqrt(rr) / nb]
    it = 0
    while hist[-1] > rtol and it < maxit:
        q = matvec(p)
        alpha = rr / np.vdot(p, q).real
        z = z + alpha * p
        r = r - alpha * q
        rr_new = np.vdot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        hist.append(np.sqrt(rr) / nb)
    return z, it, hist


def gmres(matvec, b, restart=50, rtol=1e-8, maxit=1000, z0=None):
    b = np.asarray(b)
    dt = np.result_type(b, np.float64)
    z = np.zeros(b.shape, dtype=dt) if z0 is None else np.array(z0, dtype=dt)
    nb = np.linalg.norm(b)
    hist, it = [], 0
    while it < maxit:
        r = b - matvec(z)
        beta = np.linalg.norm(r)
        hist.append(beta / nb)
        if beta / nb <= rtol:
            break
        m = restart
        Q = np.zeros((b.size, m + 1), dtype=dt)
        H = np.zeros((m + 1, m), dtype=dt)
        cs = np.zeros(m, dtype=dt)
        sn = np.zeros(m, dtype=dt)
        g = np.zeros(m + 1, dtype=dt)
        g[0] = beta
        Q[:, 0] = r / beta
        j_done = 0
        for j in range(m):
            w = matvec(Q[:, j])
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = np.vdot(Q[:, i], w)
                w = w - H[i, j] * Q[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                Q[:, j + 1] = w / H[j + 1, j]
            for i in range(j):                           # apply earlier rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, c = H[j, j], H[j + 1, j]                  # new rotation zeroing H[j+1, j]
            den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
            if abs(a) == 0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(c) / den
            H[j, j] = cs[j] * a + sn[j] * c
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) / nb <= rtol or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        z = z + Q[:, :j_done] @ y
        if hist[-1] <= rtol:
            r = b - matvec(z)
            hist.append(np.linalg.norm(r) / nb)
            if hist[-1] <= rtol:
                break
    return z, it, hist
