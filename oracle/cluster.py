"""Cluster tree (Definition 1) by bisection of characteristic points.  FP64.

TEST INFRASTRUCTURE ONLY.

Construction (the paper's description of cluster trees, with the choices it
leaves open fixed as follows):
* characteristic point of phi_i: the centroid ((p0 + p1) + p2) / 3 of T_i;
* a cluster with more than `leaf` indices is split; the split axis is the
  longest extent of the bounding box of its characteristic points (ties: the
  lowest axis), the plane is that box's midpoint 0.5*(lo + hi); indices whose
  centroid coordinate is < the midpoint form child 0, the others child 1, each
  keeping the parent's relative order.  A cluster whose points cannot be split
  (zero extent, or an empty side) stays a leaf;
* the geometric cluster tau is the minimal axis-parallel box containing the
  supports (all vertices of all triangles) of its indices, which gives
  supp phi_i subset tau as Definition 1 requires;
* clusters are numbered in depth-first pre-order (child 0 before child 1), and
  every cluster's index list is the concatenation of its children's lists, so
  the leaves in DFS order give a permutation of the index set in which every
  cluster is a contiguous range.
"""
from __future__ import annotations

import sys

import numpy as np


class Cluster:
    __slots__ = ("id", "idx", "lo", "hi", "children", "level", "parent", "begin", "end")

    def __init__(self):
        self.children = []
        self.parent = None

    @property
    def is_leaf(self) -> bool:
        return not self.children

    def diam(self) -> float:
        d0 = self.hi[0] - self.lo[0]
        d1 = self.hi[1] - self.lo[1]
        d2 = self.hi[2] - self.lo[2]
        return float(np.sqrt(d0 * d0 + d1 * d1 + d2 * d2))


class ClusterTree:
    def __init__(self, mesh, leaf: int):
        self.mesh = mesh
        self.leaf = int(leaf)
        self.clusters: list[Cluster] = []
        old = sys.getrecursionlimit()
        sys.setrecursionlimit(max(old, 10000))
        try:
            self.root = self._build(np.arange(mesh.n, dtype=np.int64), 0, None)
        finally:
            sys.setrecursionlimit(old)
        self.perm = self.root.idx.copy()
        self._ranges(self.root, 0)
        self.leaves = [c for c in self.clusters if c.is_leaf]
        self.depth = max(c.level for c in self.clusters)

    def _build(self, cand: np.ndarray, level: int, parent):
        c = Cluster()
        c.id = len(self.clusters)
        c.level = level
        c.parent = parent
        self.clusters.append(c)
        verts = self.mesh.P[cand].reshape(-1, 3)
        c.lo = verts.min(axis=0)
        c.hi = verts.max(axis=0)
        if cand.size > self.leaf:
            pts = self.mesh.centroid[cand]
            plo, phi = pts.min(axis=0), pts.max(axis=0)
            ext = phi - plo
            axis = 0
            for d in (1, 2):
                if ext[d] > ext[axis]:
                    axis = d
            mid = 0.5 * (plo[axis] + phi[axis])
            low = pts[:, axis] < mid
            if ext[axis] > 0.0 and low.any() and (~low).any():
                c.children = [self._build(cand[low], level + 1, c),
                              self._build(cand[~low], level + 1, c)]
        c.idx = cand if not c.children else np.concatenate([ch.idx for ch in c.children])
        return c

    def _ranges(self, c: Cluster, begin: int):
        c.begin, c.end = begin, begin + c.idx.size
        b = begin
        for ch in c.children:
            self._ranges(ch, b)
            b = ch.end
