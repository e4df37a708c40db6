"""Pins for the oracle's quadrature rules: exactness and closed-form singular integrals."""
import itertools
import math

import numpy as np
import pytest

from oracle import quadrature as Q
from oracle.galerkin import Mesh, NearField
from oracle.kernels import Kernel
from tests.closed_forms import rect_self_energy, simplex_moment, tri_self_energy


def _simplex_integral(lam, w, a, b):
    # standard simplex coordinates u = lam1, v = lam2, area 1/2
    return 0.5 * np.sum(w * lam[:, 1] ** a * lam[:, 2] ** b)


def test_gauss_legendre_exact():
    for q in (1, 3, 4, 6):
        t, w = Q.gauss_legendre01(q)
        for p in range(2 * q):
            assert abs(np.sum(w * t ** p) - 1.0 / (p + 1)) < 1e-15


def test_radon7_degree5():
    lam, w = Q.radon7()
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(lam.sum(1), 1)
    for a, b in itertools.product(range(6), repeat=2):
        if a + b <= 5:
            assert abs(_simplex_integral(lam, w, a, b) - simplex_moment(a, b)) < 1e-15
    # and it is not exact at degree 6 (it is the degree-5 rule, not a richer one)
    errs = [abs(_simplex_integral(lam, w, a, 6 - a) - simplex_moment(a, 6 - a)) for a in range(7)]
    assert max(errs) > 1e-6


@pytest.mark.parametrize("q", [2, 4, 6])
def test_collapsed_rule_exact(q):
    lam, w = Q.collapsed_triangle(q)
    assert abs(w.sum() - 1) < 1e-14
    for a, b in itertools.product(range(2 * q - 1), repeat=2):
        if a + b <= 2 * q - 2:
            assert abs(_simplex_integral(lam, w, a, b) - simplex_moment(a, b)) < 1e-15


def test_exact_rule_for_degree():
    for m in (1, 2, 3, 4, 5):
        deg = 3 * (m - 1)
        lam, w = Q.exact_rule_for_degree(deg)
        for a in range(deg + 1):
            b = deg - a
            assert abs(_simplex_integral(lam, w, a, b) - simplex_moment(a, b)) < 1e-15


@pytest.mark.parametrize("case", ["identical", "edge", "vertex"])
def test_sauter_schwab_is_change_of_variables(case):
    """Every rule maps the 4D cube onto T x T: polynomial moments of T x T are exact."""
    X, Y, W = Q.sauter_schwab(case, 6)
    assert abs(W.sum() - 0.25) < 1e-15
    # moments over T = {0 <= x2 <= x1 <= 1}: int x1^a x2^b = 1 / ((b + 1)(a + b + 2))
    mom = lambda a, b: 1.0 / ((b + 1) * (a + b + 2))
    for a, b, c, d in itertools.product(range(3), repeat=4):
        val = np.sum(W * X[:, 0] ** a * X[:, 1] ** b * Y[:, 0] ** c * Y[:, 1] ** d)
        assert abs(val - mom(a, b) * mom(c, d)) < 1e-15


def _ss_integral(case, P, Qtri, q):
    X, Y, W = Q.sauter_schwab(case, q)
    x = Q.chi(np.asarray(P, float), X)
    y = Q.chi(np.asarray(Qtri, float), Y)
    r = np.sqrt(((x - y) ** 2).sum(1))
    A = np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[1]))
    B = np.linalg.norm(np.cross(Qtri[1] - Qtri[0], Qtri[2] - Qtri[1]))
    return A * B * np.sum(W / r)


TRIS = [
    np.array([[0, 0, 0], [1, 0, 0], [0.5, math.sqrt(3) / 2, 0]]),
    np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.0]]),
    np.array([[0.1, 0.2, 0.3], [1.3, -0.2, 0.5], [0.4, 0.9, -0.7]]),
]


@pytest.mark.parametrize("P", TRIS)
def test_identical_closed_form(P):
    exact = tri_self_energy(P)
    assert abs(_ss_integral("identical", P, P, 22) - exact) < 1e-12 * exact
    e4 = abs(_ss_integral("identical", P, P, 4) - exact) / exact
    e8 = abs(_ss_integral("identical", P, P, 8) - exact) / exact
    assert e4 < 5e-4 and e8 < e4 / 50


def test_equilateral_value():
    # (3/4) a^3 ln 3 for side a = 1
    assert abs(tri_self_energy(TRIS[0]) - 0.75 * math.log(3.0)) < 1e-14


def test_unit_square_value():
    assert abs(rect_self_energy(1, 1) - (4 * math.log(1 + math.sqrt(2)) - 4 * (math.sqrt(2) - 1) / 3)) < 1e-14


def test_common_edge_closed_form():
    a, b = 1.0, 0.6
    p00, p10, p11, p01 = (np.array(v, float) for v in ([0, 0, 0], [a, 0, 0], [a, b, 0], [0, b, 0]))
    T1, T2 = np.array([p00, p11, p10]), np.array([p00, p11, p01])
    exact = (rect_self_energy(a, b) - tri_self_energy(T1) - tri_self_energy(T2)) / 2
    assert abs(_ss_integral("edge", T1, T2, 14) - exact) < 1e-12 * exact
    assert abs(_ss_integral("edge", T1, T2, 4) - exact) < 1e-3 * exact


def test_common_vertex_closed_form():
    c = np.array([0.5, 0.5, 0])
    c00, c10, c11, c01 = (np.array(v, float) for v in ([0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]))
    A, Ap = np.array([c, c00, c10]), np.array([c, c11, c01])
    i_self = tri_self_energy(A)
    i_edge = (tri_self_energy(np.array([c00, c10, c11])) - 2 * i_self) / 2
    exact = (rect_self_energy(1, 1) - 4 * i_self - 8 * i_edge) / 4
    assert abs(_ss_integral("vertex", A, Ap, 14) - exact) < 1e-12 * exact


def test_nearfield_orientation_on_planar_mesh():
    """The oracle's entry selection and vertex ordering on a real mesh: a unit
    square cut into four triangles around its centre.  The sum of all 16
    entries is the square's self-energy / (4 pi); each class of entry matches
    its closed form."""
    V = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0.5, 0.5, 0]], float)
    T = np.array([[4, 0, 1], [4, 1, 2], [4, 2, 3], [4, 3, 0]])
    mesh = Mesh(V, T)
    nf = NearField(mesh, Kernel(), q_ss=14)
    G = nf.block(np.arange(4), np.arange(4)) * 4 * math.pi
    i_self = tri_self_energy(V[T[0]])
    i_edge = (tri_self_energy(V[[0, 1, 2]]) - 2 * i_self) / 2
    i_vert = (rect_self_energy(1, 1) - 4 * i_self - 8 * i_edge) / 4
    for i in range(4):
        assert abs(G[i, i] - i_self) < 1e-12
        assert abs(G[i, (i + 1) % 4] - i_edge) < 1e-12
        assert abs(G[i, (i + 2) % 4] - i_vert) < 1e-12
    assert abs(G.sum() - rect_self_energy(1, 1)) < 1e-11
    assert np.array_equal(G, G.T)


def test_regular_rule_far_pair_converges():
    """7-point rule on well-separated triangles: error of a smooth integrand is small."""
    V = np.array([[0, 0, 0], [0.1, 0, 0], [0, 0.1, 0], [2, 0, 0], [2.1, 0, 0], [2, 0.1, 0.05]], float)
    T = np.array([[0, 1, 2], [3, 4, 5]])
    mesh = Mesh(V, T)
    val = NearField(mesh, Kernel()).block(np.array([0]), np.array([1]))[0, 0]
    # reference: collapsed rule of high order on both triangles
    lam, w = Q.collapsed_triangle(12)
    x = lam @ V[T[0]]
    y = lam @ V[T[1]]
    r = np.sqrt(((x[:, None] - y[None]) ** 2).sum(-1))
    ref = mesh.area[0] * mesh.area[1] * np.einsum("a,b,ab->", w, w, 1 / (4 * math.pi * r))
    assert abs(val - ref) < 1e-9 * abs(ref)


def _subdivide(P, levels):
    """Midpoint subdivision of one triangle into 4**levels congruent pieces."""
    tris = [np.asarray(P, float)]
    for _ in range(levels):
        out = []
        for a, b, c in tris:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            out += [np.array([a, ab, ca]), np.array([ab, b, bc]), np.array([ca, bc, c]), np.array([ab, bc, ca])]
        tris = out
    return np.array(tris)


def _composite(PA, PB, levels, q=8):
    """Mean of 1/(4 pi |x - y|) over T_a x T_b: both triangles subdivided, the
    collapsed Gauss rule of order q (exact to degree 2q - 1) on every sub-pair."""
    lam, w = Q.collapsed_triangle(q)
    A, B = _subdivide(PA, levels), _subdivide(PB, levels)
    X = np.einsum("qk,nkd->nqd", lam, A).reshape(-1, 3)
    Y = np.einsum("qk,nkd->nqd", lam, B).reshape(-1, 3)
    wa, wb = np.tile(w, len(A)) / len(A), np.tile(w, len(B)) / len(B)
    r = np.sqrt(((X[:, None] - Y[None]) ** 2).sum(-1))
    return wa @ (1.0 / (4.0 * math.pi * r)) @ wb


@pytest.mark.parametrize("kind,level", [("sphere", 3), ("cube", 8)])
def test_regular_rule_on_closest_non_touching_pairs(kind, level):
    """Accuracy of the regular 7 x 7-point rule where it is weakest: the nearest
    triangles that share no vertex (the paper fixes the rule, not its error).
    Reference: the composite high-order rule, converged in the subdivision level
    (one level vs two agree to 1e-12).  Measured worst relative error: 1.3e-5 on
    the sphere, 9.4e-5 on the cube (right triangles, closer relative to size)."""
    import h2_inputs as I
    V, T = I.mesh_for(kind, level)
    mesh = Mesh(V, T)
    nf = NearField(mesh, Kernel())
    c = mesh.P.mean(1)
    worst = 0.0
    for i in (0, 100):
        touch = set(int(j) for j in mesh.touching(i)) | {i}
        order = [int(j) for j in np.argsort(np.linalg.norm(c - c[i], axis=1)) if int(j) not in touch]
        for j in order[:4]:
            val = nf.regular(np.array([i]), np.array([j]))[0, 0]
            r1 = mesh.area[i] * mesh.area[j] * _composite(mesh.P[i], mesh.P[j], 1)
            r2 = mesh.area[i] * mesh.area[j] * _composite(mesh.P[i], mesh.P[j], 2)
            assert abs(r1 / r2 - 1.0) <= 1e-12, (i, j)
            worst = max(worst, abs(val / r2 - 1.0))
    assert worst <= 2e-4
    assert worst >= 1e-7  # the rule is not exact here: the reference is independent of it
