"""Galerkin entries g_ij for piecewise-constant test and trial functions (FP64).

TEST INFRASTRUCTURE ONLY.

phi_i = psi_i is the characteristic function of triangle T_i (test space =
trial space), so g_ij = int_{T_i} int_{T_j} g(x, y) dy dx (Introduction,
definition of g_ij).  The paper evaluates the singular integrals with
Sauter-Schwab quadrature; the quadrature rules fixed here are:

* identical triangles, common edge, common vertex ("touching" = sharing at
  least one vertex index): Sauter-Schwab with Gauss-Legendre of order q_ss in
  each of the four parameters;
* all other pairs: Radon's 7-point rule on each triangle (49 kernel
  evaluations per pair).

For a pair (i, j) the triangle with the smaller index is the x-triangle, so
g_ij and g_ji are the same floating-point number for a symmetric kernel.
Vertex order inside the Sauter-Schwab parametrisations:
  identical: the stored order;
  common edge {u, w}: (min(u,w), max(u,w), third vertex) for both triangles;
  common vertex v: the stored cyclic order rotated to start at v.
Smooth (polynomial) test kernels use the 7-point rule for every pair.
"""
from __future__ import annotations

import numpy as np

from . import quadrature as Q


class Mesh:
    """Vertex/triangle arrays with the derived per-triangle geometry."""

    def __init__(self, vertices: np.ndarray, triangles: np.ndarray):
        self.V = np.asarray(vertices, dtype=np.float64)
        self.T = np.asarray(triangles, dtype=np.int64)
        p0, p1, p2 = self.V[self.T[:, 0]], self.V[self.T[:, 1]], self.V[self.T[:, 2]]
        self.P = np.stack([p0, p1, p2], 1)                      # (n, 3, 3)
        self.area = 0.5 * np.sqrt((np.cross(p1 - p0, p2 - p0) ** 2).sum(1))
        self.centroid = (p0 + p1 + p2) / 3.0                    # characteristic points
        self.n = self.T.shape[0]
        self._vt = None

    def vertex_triangles(self):
        """List, per vertex, of the triangles that contain it."""
        if self._vt is None:
            vt = [[] for _ in range(self.V.shape[0])]
            for t, tri in enumerate(self.T):
                for v in tri:
                    vt[v].append(t)
            self._vt = [np.array(sorted(x), dtype=np.int64) for x in vt]
        return self._vt

    def touching(self, i: int) -> np.ndarray:
        """Triangles sharing at least one vertex with triangle i (including i)."""
        vt = self.vertex_triangles()
        return np.unique(np.concatenate([vt[v] for v in self.T[i]]))


class NearField:
    """Evaluator of Galerkin entries g_ij with the quadrature fixed above."""

    def __init__(self, mesh: Mesh, kernel, q_ss: int = 4):
        self.mesh = mesh
        self.g = kernel
        lam, w = Q.radon7()
        self.reg_w = w
        # quadrature points of every triangle: (n, 7, 3)
        self.reg_x = np.einsum("qk,nkd->nqd", lam, mesh.P)
        self.ss = {c: Q.sauter_schwab(c, q_ss) for c in ("identical", "edge", "vertex")}
        self._cache = {}

    # -- regular pairs --------------------------------------------------------
    def regular(self, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        """7-point x 7-point rule for all (rows x cols) pairs (no singularity check)."""
        m = self.mesh
        out = np.empty((rows.size, cols.size), dtype=self.g.dtype)
        step = max(1, 200000 // max(1, cols.size))
        for r0 in range(0, rows.size, step):
            r = rows[r0:r0 + step]
            a = np.minimum(r[:, None], cols[None, :])          # x-triangle = smaller index
            b = np.maximum(r[:, None], cols[None, :])
            X = self.reg_x[a][:, :, :, None, :]
            Y = self.reg_x[b][:, :, None, :, :]
            with np.errstate(divide="ignore", invalid="ignore"):
                G = self.g(X, Y)
            s = np.einsum("a,b,ijab->ij", self.reg_w, self.reg_w, G)
            out[r0:r0 + step] = m.area[r][:, None] * m.area[cols][None, :] * s
        return out

    # -- touching pairs -------------------------------------------------------
    def _orient(self, a: int, b: int):
        """Case and vertex order (Pa, Pb) of a touching pair with a <= b."""
        m = self.mesh
        ta, tb = [int(v) for v in m.T[a]], [int(v) for v in m.T[b]]
        shared = set(ta) & set(tb)
        if a == b:
            return "identical", ta, tb
        if len(shared) == 2:
            u, w = min(shared), max(shared)
            return ("edge", [u, w] + [v for v in ta if v not in shared],
                    [u, w] + [v for v in tb if v not in shared])
        if len(shared) == 1:
            v = next(iter(shared))
            ka, kb = ta.index(v), tb.index(v)
            return "vertex", ta[ka:] + ta[:ka], tb[kb:] + tb[:kb]
        raise ValueError("pair (%d, %d) does not touch" % (a, b))

    def singular(self, pairs) -> np.ndarray:
        """Sauter-Schwab values for a list of touching pairs (i, j)."""
        m = self.mesh
        out = np.empty(len(pairs), dtype=self.g.dtype)
        groups = {"identical": [], "edge": [], "vertex": []}
        for n, (i, j) in enumerate(pairs):
            a, b = (i, j) if i <= j else (j, i)
            key = (a, b)
            if key in self._cache:
                out[n] = self._cache[key]
                continue
            case, Pa, Pb = self._orient(a, b)
            groups[case].append((n, a, b, Pa, Pb))
        for case, lst in groups.items():
            if not lst:
                continue
            xh, yh, w = self.ss[case]
            for c0 in range(0, len(lst), 256):
                chunk = lst[c0:c0 + 256]
                PA = m.V[np.array([c[3] for c in chunk])]          # (B, 3, 3)
                PB = m.V[np.array([c[4] for c in chunk])]
                X = PA[:, None, 0] + xh[None, :, :1] * (PA[:, None, 1] - PA[:, None, 0]) \
                    + xh[None, :, 1:2] * (PA[:, None, 2] - PA[:, None, 1])
                Y = PB[:, None, 0] + yh[None, :, :1] * (PB[:, None, 1] - PB[:, None, 0]) \
                    + yh[None, :, 1:2] * (PB[:, None, 2] - PB[:, None, 1])
                vals = np.einsum("q,bq->b", w, self.g(X, Y))
                for (n, a, b, _, _), v in zip(chunk, vals):
                    val = 4.0 * m.area[a] * m.area[b] * v
                    self._cache[(a, b)] = val
                    out[n] = val
        return out

    def block(self, rows, cols) -> np.ndarray:
        """Entries g_ij for i in rows, j in cols."""
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        out = self.regular(rows, cols)
        if not self.g.smooth:
            where = {int(j): c for c, j in enumerate(cols)}
            hits, pairs = [], []
            for r, i in enumerate(rows):
                for j in self.mesh.touching(int(i)):
                    c = where.get(int(j))
                    if c is not None:
                        hits.append((r, c))
                        pairs.append((int(i), int(j)))
            if pairs:
                vals = self.singular(pairs)
                for (r, c), v in zip(hits, vals):
                    out[r, c] = v
        return out

    def row(self, i: int, js) -> np.ndarray:
        return self.block(np.array([i]), js)[0]


def dense_G(mesh: Mesh, kernel, q_ss: int = 4) -> np.ndarray:
    """The full Galerkin matrix G (tier 1 of the oracle): every entry by the rules above."""
    nf = NearField(mesh, kernel, q_ss)
    allj = np.arange(mesh.n)
    return nf.block(allj, allj)
