"""The H^2 matrix G-tilde and its matrix-vector product.  FP64.  TEST INFRASTRUCTURE ONLY.

G-tilde is fixed by the leaf partition of the block tree: admissible leaves
(tau, sigma) carry V_tau S_{tau sigma} W_sigma^T (eq. vsw), inadmissible leaves
carry the Galerkin block G|_{tau x sigma}.  Test and trial spaces coincide, so
W = V and F = E.

Three ways to apply it, each written from a different passage:
* dense_Gtilde: the block-by-block definition, with V_tau of a non-leaf
  cluster expanded through eq. (V_nested);
* H2Oracle.matvec: Algorithms 1-3 as recursions (forward transformation,
  interaction phase, backward transformation), y <- y + G-tilde x, with
  y-hat := 0 before the interaction phase;
* H2Oracle.sampled_rows: rows of G-tilde x for a few leaf clusters at sizes
  where the full product is out of reach in Python; the block tree is only
  descended along the path of the requested row cluster, S and V_tau are
  evaluated from their definitions on the fly, and x-hat comes from Alg. 1.
"""
from __future__ import annotations

import sys

import numpy as np

from . import interpolation as IP
from .blocks import admissible, build_block_tree, leaves, pair_children
from .cluster import ClusterTree
from .galerkin import Mesh, NearField
from .kernels import Kernel


class H2Oracle:
    def __init__(self, vertices, triangles, kernel: Kernel | None = None, m: int = 3,
                 leaf: int = 32, eta: float = 0.5, q_ss: int = 4, build_blocks: bool = True):
        self.mesh = Mesh(vertices, triangles)
        self.g = kernel or Kernel()
        self.m, self.k = int(m), int(m) ** 3
        self.eta = float(eta)
        self.tree = ClusterTree(self.mesh, leaf)
        self.nf = NearField(self.mesh, self.g, q_ss)
        self._V, self._E, self._S, self._N = {}, {}, {}, {}
        self.btree = None
        if build_blocks:
            old = sys.getrecursionlimit()
            sys.setrecursionlimit(max(old, 20000))
            try:
                self.btree = build_block_tree(self.tree.root, self.tree.root, self.eta)
            finally:
                sys.setrecursionlimit(old)
            self.adm, self.inadm = [], []
            leaves(self.btree, self.adm, self.inadm)

    # ------------------------------------------------------------ stored data
    def V(self, c):
        """Leaf matrix V_tau (eq. leafV), rows in the order of c.idx."""
        if c.id not in self._V:
            self._V[c.id] = IP.basis_matrix(c, self.m, self.mesh, c.idx)
        return self._V[c.id]

    def E(self, c):
        """Transfer matrix E_tau of a non-root cluster (eq. transfer)."""
        if c.id not in self._E:
            self._E[c.id] = IP.transfer(c, c.parent, self.m)
        return self._E[c.id]

    def S(self, t, s, store: bool = True):
        key = (t.id, s.id)
        if key in self._S:
            return self._S[key]
        S = IP.coupling(t, s, self.m, self.g)
        if store:
            self._S[key] = S
        return S

    def N(self, t, s, store: bool = True):
        """Near-field block G|_{tau x sigma} (Galerkin entries, rows t.idx, cols s.idx)."""
        key = (t.id, s.id)
        if key in self._N:
            return self._N[key]
        B = self.nf.block(t.idx, s.idx)
        if store:
            self._N[key] = B
        return B

    # ------------------------------------------------------------ Algorithms 1-3
    def forward(self, sig, x, xhat):
        """Algorithm 1: x-hat_sigma = W_sigma^T x|sigma, via the children and F^T."""
        if sig.is_leaf:
            xhat[sig.id] = self.V(sig).T @ x[sig.idx]
        else:
            acc = np.zeros(self.k, dtype=np.result_type(x, self.g.dtype))
            for ch in sig.children:
                self.forward(ch, x, xhat)
                acc = acc + self.E(ch).T @ xhat[ch.id]
            xhat[sig.id] = acc

    def backward(self, tau, yhat, y):
        """Algorithm 2: add V_tau y-hat_tau to y|tau, via E_{tau'} y-hat_tau for the children."""
        if tau.is_leaf:
            y[tau.idx] += self.V(tau) @ yhat[tau.id]
        else:
            for ch in tau.children:
                yhat[ch.id] = yhat[ch.id] + self.E(ch) @ yhat[tau.id]
                self.backward(ch, yhat, y)

    def interaction(self, b, xhat, x, yhat, y):
        """Algorithm 3 over the block tree."""
        if b.children:
            for c in b.children:
                self.interaction(c, xhat, x, yhat, y)
        elif b.adm:
            yhat[b.t.id] = yhat[b.t.id] + self.S(b.t, b.s) @ xhat[b.s.id]
        else:
            y[b.t.idx] += self.N(b.t, b.s) @ x[b.s.idx]

    def matvec(self, x, y=None):
        """y <- y + G-tilde x (x, y in the original triangle order)."""
        x = np.asarray(x)
        dt = np.result_type(x, self.g.dtype)
        y = np.zeros(self.mesh.n, dtype=dt) if y is None else y.astype(dt)
        nc = len(self.tree.clusters)
        xhat = [None] * nc
        old = sys.getrecursionlimit()
        sys.setrecursionlimit(max(old, 20000))
        try:
            self.forward(self.tree.root, x, xhat)
            yhat = [np.zeros(self.k, dtype=dt) for _ in range(nc)]     # y-hat := 0
            self.interaction(self.btree, xhat, x, yhat, y)
            self.backward(self.tree.root, yhat, y)
        finally:
            sys.setrecursionlimit(old)
        return y

    # ------------------------------------------------------------ dense forms
    def Vbar(self, c):
        """V_tau of any cluster via eq. (V_nested): rows of child tau' are V_tau' E_tau'."""
        if c.is_leaf:
            return self.V(c)
        return np.concatenate([self.Vbar(ch) @ self.E(ch) for ch in c.children], 0)

    def V_direct(self, c):
        """V_tau of any cluster directly from eq. (leafV) on tau's own box."""
        return IP.basis_matrix(c, self.m, self.mesh, c.idx)

    def dense_Gtilde(self):
        n = self.mesh.n
        G = np.zeros((n, n), dtype=self.g.dtype)
        for t, s in self.adm:
            G[np.ix_(t.idx, s.idx)] = self.Vbar(t) @ self.S(t, s) @ self.Vbar(s).T
        for t, s in self.inadm:
            G[np.ix_(t.idx, s.idx)] = self.N(t, s)
        return G

    # ------------------------------------------------------------ sampled rows
    def all_xhat(self, x):
        xhat = [None] * len(self.tree.clusters)
        old = sys.getrecursionlimit()
        sys.setrecursionlimit(max(old, 20000))
        try:
            self.forward(self.tree.root, x, xhat)
        finally:
            sys.setrecursionlimit(old)
        return xhat

    def row_blocks(self, leaf):
        """Leaves (tau, sigma) of the block tree with leaf's indices inside tau.

        Follows the block-tree recursion from (root, root), keeping only pairs
        whose row cluster contains the given leaf cluster.
        """
        path = set()
        c = leaf
        while c is not None:
            path.add(c.id)
            c = c.parent
        adm, inadm, stack = [], [], [(self.tree.root, self.tree.root)]
        while stack:
            t, s = stack.pop()
            if admissible(t, s, self.eta):
                adm.append((t, s))
                continue
            ch = pair_children(t, s)
            if not ch:
                inadm.append((t, s))
                continue
            stack.extend((a, b) for a, b in ch if a.id in path)
        return adm, inadm

    def forward_sparse(self, x, support):
        """Algorithm 1 for an x that vanishes outside the given leaf clusters.

        A cluster containing none of the support leaves has x|sigma = 0 and hence
        x-hat_sigma = 0, so the recursion only descends into clusters that contain
        support; all other entries of the returned list are exact zeros.
        """
        x = np.asarray(x)
        dt = np.result_type(x, self.g.dtype)
        keep = set()
        for lid in support:
            c = self.tree.clusters[lid]
            while c is not None:
                keep.add(c.id)
                c = c.parent
        xhat = [None] * len(self.tree.clusters)

        def fwd(sig):
            if sig.is_leaf:
                xhat[sig.id] = self.V(sig).T @ x[sig.idx]
                return
            acc = np.zeros(self.k, dtype=dt)
            for ch in sig.children:
                if ch.id in keep:
                    fwd(ch)
                    acc = acc + self.E(ch).T @ xhat[ch.id]
            xhat[sig.id] = acc

        fwd(self.tree.root)
        zero = np.zeros(self.k, dtype=dt)
        return [zero if v is None else v for v in xhat], keep

    def sampled_rows(self, x, leaf_ids, xhat=None, support=None):
        """(G-tilde x)|leaf for each requested leaf cluster id -> dict id -> (rows idx, values)."""
        x = np.asarray(x)
        keep = None
        if xhat is None:
            if support is None:
                xhat = self.all_xhat(x)
            else:
                xhat, keep = self.forward_sparse(x, support)
        out = {}
        for lid in leaf_ids:
            leaf = self.tree.clusters[lid]
            assert leaf.is_leaf
            adm, inadm = self.row_blocks(leaf)
            y = np.zeros(leaf.idx.size, dtype=np.result_type(x, self.g.dtype))
            pos = {int(i): r for r, i in enumerate(leaf.idx)}
            for t, s in adm:
                if keep is not None and s.id not in keep:
                    continue                        # x-hat_sigma = 0
                rows = np.array([pos[int(i)] for i in leaf.idx])
                # rows of V_t that belong to the leaf, evaluated from eq. (leafV) on t's box
                Vt = IP.basis_matrix(t, self.m, self.mesh, leaf.idx)
                y[rows] += Vt @ (self.S(t, s, store=False) @ xhat[s.id])
            for t, s in inadm:
                if keep is not None and s.id not in keep:
                    continue                        # x|sigma = 0
                y += self.nf.block(leaf.idx, s.idx) @ x[s.idx]
            out[lid] = (leaf.idx.copy(), y)
        return out
