"""Pins for the oracle's cluster tree (Definition 1) and block tree (eq. admissibility)."""
import numpy as np
import pytest
from scipy.optimize import minimize

import h2_inputs as I
from oracle.blocks import admissible, box_dist
from tests.oracle_cache import cube, sphere


def test_meshes():
    for r in range(4):
        V, T = I.icosphere(r)
        assert T.shape[0] == 20 * 4 ** r and V.shape[0] == 10 * 4 ** r + 2
        edges = {tuple(sorted(e)) for t in T for e in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
        assert V.shape[0] - len(edges) + T.shape[0] == 2          # Euler characteristic
        assert np.allclose(np.linalg.norm(V, axis=1), 1.0)
    for N in (1, 3, 8):
        V, T = I.cube_surface(N)
        assert T.shape[0] == 12 * N * N and V.shape[0] == 6 * N * N + 2
        P = V[T]
        area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
        assert abs(area.sum() - 6.0) < 1e-12
        nrm = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        assert (np.einsum("ij,ij->i", nrm, P.mean(1)) > 0).all()   # outward
    # sphere area converges to 4 pi
    errs = []
    for r in (2, 3, 4):
        V, T = I.icosphere(r)
        P = V[T]
        errs.append(abs(0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1).sum() - 4 * np.pi))
    assert errs[0] > errs[1] > errs[2]


@pytest.mark.parametrize("H", [lambda: sphere(3, 3, 32), lambda: cube(8, 3, 32), lambda: sphere(4, 4, 64)])
def test_definition1(H):
    H = H()
    tr, mesh = H.tree, H.mesh
    assert np.array_equal(np.sort(tr.root.idx), np.arange(mesh.n))
    for c in tr.clusters:
        verts = mesh.P[c.idx].reshape(-1, 3)
        assert (verts >= c.lo).all() and (verts <= c.hi).all()       # supp phi_i in tau
        assert np.array_equal(tr.perm[c.begin:c.end], c.idx)       # contiguous range
        if c.children:
            a, b = c.children
            assert np.intersect1d(a.idx, b.idx).size == 0
            assert np.array_equal(np.sort(np.concatenate([a.idx, b.idx])), np.sort(c.idx))
            assert (c.lo <= a.lo).all() and (c.hi >= a.hi).all()
        else:
            assert c.idx.size <= tr.leaf
    # bisection rule: child 0 centroids strictly below the midpoint of the parent's centroid box
    for c in tr.clusters:
        if c.children:
            pts = mesh.centroid[c.idx]
            ext = pts.max(0) - pts.min(0)
            ax = int(np.argmax(ext))
            mid = 0.5 * (pts.min(0)[ax] + pts.max(0)[ax])
            assert (mesh.centroid[c.children[0].idx][:, ax] < mid).all()
            assert (mesh.centroid[c.children[1].idx][:, ax] >= mid).all()


@pytest.mark.parametrize("H", [lambda: sphere(3, 3, 32), lambda: cube(8, 3, 32)])
def test_leaf_partition(H):
    """{tau x sigma : leaves} is a partition of I x J (brute force)."""
    H = H()
    n = H.mesh.n
    cover = np.zeros((n, n), dtype=np.int32)
    for t, s in H.adm + H.inadm:
        cover[np.ix_(t.idx, s.idx)] += 1
    assert (cover == 1).all()
    for t, s in H.adm:
        assert admissible(t, s, H.eta)
    for t, s in H.inadm:
        assert t.is_leaf and s.is_leaf and not admissible(t, s, H.eta)
    A = {(t.id, s.id) for t, s in H.adm}
    N = {(t.id, s.id) for t, s in H.inadm}
    assert A == {(b, a) for a, b in A} and N == {(b, a) for a, b in N}


def test_box_distance_by_optimisation():
    """dist(tau, sigma) equals the minimum distance of two points in the boxes."""
    H = sphere(3, 3, 32)
    rng = np.random.default_rng(0)
    cl = H.tree.clusters
    for _ in range(20):
        t, s = cl[rng.integers(len(cl))], cl[rng.integers(len(cl))]
        bounds = list(zip(t.lo, t.hi)) + list(zip(s.lo, s.hi))
        x0 = np.concatenate([0.5 * (t.lo + t.hi), 0.5 * (s.lo + s.hi)])
        res = minimize(lambda z: np.sum((z[:3] - z[3:]) ** 2), x0, bounds=bounds,
                       method="L-BFGS-B", options=dict(ftol=1e-15, gtol=1e-12))
        assert abs(np.sqrt(max(res.fun, 0)) - box_dist(t, s)) < 1e-6


def test_eta_controls_block_count():
    a = sphere(3, 3, 32, 0.5)
    b = sphere(3, 3, 32, 1.0)
    assert len(b.adm) + len(b.inadm) < len(a.adm) + len(a.inadm)


def _box(lo, hi):
    from oracle.cluster import Cluster
    c = Cluster()
    c.lo, c.hi = np.array(lo, dtype=np.float64), np.array(hi, dtype=np.float64)
    return c


def test_diam_is_box_diagonal():
    """diam tau is the Euclidean length of the box diagonal, not its longest side:
    the box [0,1]x[0,2]x[0,2] has diagonal sqrt(1+4+4) = 3 and longest side 2."""
    assert _box([0, 0, 0], [1, 2, 2]).diam() == 3.0
    assert _box([-1, 5, 2], [1, 8, 8]).diam() == 7.0            # sqrt(4 + 9 + 36)
    assert _box([0.25, 0.25, 0.25], [0.25, 0.25, 0.25]).diam() == 0.0


def test_admissibility_boundary_hand_built_boxes():
    """eq. (admissibility) with eta = 1/2 reads max(diam) <= dist.  Two boxes of
    diagonal 3 separated along x by a gap g have dist = g: admissible at g = 3
    (the boundary, equality allowed), not at g = 3 - 2^-40 just across it, and
    not at g = 2.5 (a longest-side diameter, 2, would wrongly accept it); with
    eta = 1 the condition is max(diam) <= 2 dist, so g = 1.5 is the boundary.
    Writing eta for 2 eta, or the longest side for the diagonal, fails a case."""
    A = _box([0, 0, 0], [1, 2, 2])
    for gap, eta, want in ((3.0, 0.5, True), (3.0 - 2.0 ** -40, 0.5, False), (2.5, 0.5, False),
                           (4.0, 0.5, True), (1.5, 1.0, True), (1.5 - 2.0 ** -40, 1.0, False),
                           (3.0, 0.25, False), (6.0, 0.25, True)):
        B = _box([1 + gap, 0, 0], [2 + gap, 2, 2])
        assert box_dist(A, B) == gap and box_dist(B, A) == gap
        assert admissible(A, B, eta) is want, (gap, eta)
        assert admissible(B, A, eta) is want, (gap, eta)
    # gaps in two axes: dist = sqrt(3^2 + 4^2) = 5
    B = _box([4, 6, 0], [5, 8, 2])
    assert box_dist(A, B) == 5.0
    assert admissible(A, B, 0.5) and not admissible(A, B, 0.25)   # 3 <= 5, 3 > 2.5
    # intersecting or touching boxes have dist 0 and are never admissible
    for lo in ([0.5, 1, 1], [1, 0, 0], [1, 2, 2]):
        B = _box(lo, np.add(lo, [1, 2, 2]))
        assert box_dist(A, B) == 0.0 and not admissible(A, B, 1e6)
    # the larger of the two diameters decides
    small = _box([10, 0, 0], [10.5, 0.5, 0.5])                   # diam sqrt(0.75) < 3
    assert box_dist(A, small) == 9.0
    assert admissible(A, small, 0.5)
    big = _box([4, 0, 0], [14, 0, 0])                              # diam 10 > dist 3
    assert not admissible(A, big, 0.5) and admissible(A, big, 10.0 / 6.0)
