"""Block tree and admissibility (eq. admissibility).  FP64.  TEST INFRASTRUCTURE ONLY.

A pair (tau, sigma) is admissible if max(diam tau, diam sigma) <= 2 eta dist(tau, sigma)
with diam the Euclidean length of a box's diagonal and dist the Euclidean
distance of the two boxes (zero if they intersect).  The block tree starts at
(root, root); an admissible pair is an admissible leaf, a pair of two leaf
clusters that is not admissible is an inadmissible leaf, and otherwise the
pair is split into chil(tau) x chil(sigma), {tau} x chil(sigma) or
chil(tau) x {sigma}, whichever of the two clusters have children.
"""
from __future__ import annotations

import math


def box_dist(t, s) -> float:
    g = []
    for d in range(3):
        a = float(s.lo[d]) - float(t.hi[d])
        b = float(t.lo[d]) - float(s.hi[d])
        g.append(max(0.0, a, b))
    return math.sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2])


def admissible(t, s, eta: float) -> bool:
    return max(t.diam(), s.diam()) <= 2.0 * eta * box_dist(t, s)


class Block:
    __slots__ = ("t", "s", "children", "adm")

    def __init__(self, t, s):
        self.t, self.s, self.children, self.adm = t, s, [], False

    @property
    def is_leaf(self):
        return not self.children


def pair_children(t, s):
    """chil(tau, sigma) for a pair that is not an admissible leaf."""
    if t.children and s.children:
        return [(a, b) for a in t.children for b in s.children]
    if s.children:
        return [(t, b) for b in s.children]
    if t.children:
        return [(a, s) for a in t.children]
    return []


def build_block_tree(t, s, eta: float) -> Block:
    b = Block(t, s)
    if admissible(t, s, eta):
        b.adm = True
        return b
    b.children = [build_block_tree(a, c, eta) for a, c in pair_children(t, s)]
    return b


def leaves(b: Block, adm_out: list, inadm_out: list):
    """Collect admissible and inadmissible leaves (tau, sigma) in recursion order."""
    stack = [b]
    while stack:
        x = stack.pop()
        if x.children:
            stack.extend(reversed(x.children))
        elif x.adm:
            adm_out.append((x.t, x.s))
        else:
            inadm_out.append((x.t, x.s))
