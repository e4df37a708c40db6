"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the H^2 method itself: it only produces
the polyhedral surfaces on which the Galerkin discretisation is set up
(the paper's experiments use polyhedral approximations of the unit sphere,
Section "Distributed H^2-matrices", experiments paragraph) and seeded
random right-hand sides.  Both the CPU oracle and the GPU library read the
same vertex/triangle arrays, so the two sides never have to agree on how a
mesh is generated.

Meshes
  icosphere(r): icosahedron refined r times; every refinement splits each
      triangle into four at its edge midpoints and projects the new vertices
      onto the unit sphere.  20*4^r triangles, 10*4^r + 2 vertices.
  cube_surface(N): surface of [-1/2, 1/2]^3, each face split into N x N
      squares and each square into two triangles along a fixed diagonal.
      12*N^2 triangles, 6*N^2 + 2 vertices.
Triangles are int32 vertex-index triples with outward orientation; vertices
are shared between neighbouring triangles, so "touching" triangles can be
recognised from vertex indices.
"""
from __future__ import annotations

import numpy as np

__all__ = ["icosphere", "cube_surface", "random_vector", "WORKLOADS", "mesh_for"]

_PHI = (1.0 + 5.0 ** 0.5) / 2.0

_ICO_V = np.array([
    [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
    [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
    [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
], dtype=np.float64)

_ICO_T = np.array([
    [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
    [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
    [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
    [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
], dtype=np.int64)


def _normalise(v: np.ndarray) -> np.ndarray:
    return v / np.sqrt((v * v).sum(axis=1))[:, None]


def icosphere(r: int):
    """Unit-sphere icosahedral mesh after r refinements -> (vertices, triangles)."""
    if r < 0:
        raise ValueError("refinement level must be >= 0")
    V = _normalise(_ICO_V.copy())
    T = _ICO_T.copy()
    for _ in range(r):
        nv = V.shape[0]
        a, b, c = T[:, 0], T[:, 1], T[:, 2]
        e = np.stack([np.stack([a, b], 1), np.stack([b, c], 1), np.stack([c, a], 1)], 1)  # (nt,3,2)
        ek = np.sort(e.reshape(-1, 2), axis=1)
        uniq, inv = np.unique(ek, axis=0, return_inverse=True)
        inv = inv.reshape(-1, 3)
        mid = _normalise(V[uniq[:, 0]] + V[uniq[:, 1]])
        V = np.concatenate([V, mid], 0)
        ab, bc, ca = inv[:, 0] + nv, inv[:, 1] + nv, inv[:, 2] + nv
        T = np.stack([
            np.stack([a, ab, ca], 1), np.stack([ab, b, bc], 1),
            np.stack([ca, bc, c], 1), np.stack([ab, bc, ca], 1)], 1).reshape(-1, 3)
    return np.ascontiguousarray(V), np.ascontiguousarray(T.astype(np.int32))


def cube_surface(N: int):
    """Surface of the cube [-1/2,1/2]^3 with N x N squares per face -> (vertices, triangles)."""
    if N < 1:
        raise ValueError("N must be >= 1")
    keys, tris = [], []
    g = np.arange(N + 1)
    U, W = np.meshgrid(g, g, indexing="ij")
    for axis in range(3):
        for side in (0, N):
            o1, o2 = [d for d in range(3) if d != axis]
            P = np.zeros((N + 1, N + 1, 3), dtype=np.int64)
            P[..., axis] = side
            P[..., o1] = U
            P[..., o2] = W
            k = P.reshape(-1, 3)
            base = sum(len(x) for x in keys)
            keys.append(k)
            idx = (np.arange((N + 1) * (N + 1)).reshape(N + 1, N + 1) + base)
            p00, p10 = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel()
            p11, p01 = idx[1:, 1:].ravel(), idx[:-1, 1:].ravel()
            tris.append(np.stack([p00, p10, p11], 1))
            tris.append(np.stack([p00, p11, p01], 1))
    K = np.concatenate(keys, 0)
    T = np.concatenate(tris, 0)
    uk, inv = np.unique(K, axis=0, return_inverse=True)
    T = inv.reshape(-1)[T]
    V = -0.5 + uk.astype(np.float64) / N
    # orient outward: normal must point away from the cube centre
    p0, p1, p2 = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    flip = (nrm * (p0 + p1 + p2)).sum(1) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return np.ascontiguousarray(V), np.ascontiguousarray(T.astype(np.int32))


def random_vector(n: int, seed: int, dist: str = "normal", nrhs: int = 1) -> np.ndarray:
    """Seeded float64 vector(s): dist 'normal' -> N(0,1), 'uniform' -> U(-1,1).

    Shape (n,) for nrhs == 1, else (n, nrhs) column-major-compatible (Fortran order).
    """
    rng = np.random.default_rng(seed)
    shape = (nrhs, n)
    if dist == "normal":
        x = rng.standard_normal(shape)
    elif dist == "uniform":
        x = rng.uniform(-1.0, 1.0, shape)
    else:
        raise ValueError(dist)
    return x[0].copy() if nrhs == 1 else np.asfortranarray(x.T)


# Named workloads: the meshes and parameters of the measured configurations.
WORKLOADS = {
    "sphere1280_m3": dict(mesh=("sphere", 3), order=3, leaf=32, eta=0.5, seed=1, dist="uniform"),
    "sphere327k_m4": dict(mesh=("sphere", 7), order=4, leaf=64, eta=0.5, seed=2, dist="normal"),
    "sphere1310k_m4": dict(mesh=("sphere", 8), order=4, leaf=64, eta=0.5, seed=3, dist="normal"),
    "cube786k_m4_r64": dict(mesh=("cube", 256), order=4, leaf=64, eta=0.5, seed=4, dist="normal", nrhs=64),
}


def mesh_for(kind: str, level: int):
    if kind == "sphere":
        return icosphere(level)
    if kind == "cube":
        return cube_surface(level)
    raise ValueError(kind)
