"""Cached oracle instances shared by several test modules (built once per process)."""
import functools

import h2_inputs as I
from oracle.h2 import H2Oracle
from oracle.kernels import Kernel


@functools.lru_cache(maxsize=None)
def sphere(r=3, m=3, leaf=32, eta=0.5, kind=0, kappa=0.0):
    V, T = I.icosphere(r)
    return H2Oracle(V, T, Kernel(kind, kappa), m=m, leaf=leaf, eta=eta)


@functools.lru_cache(maxsize=None)
def cube(N=8, m=3, leaf=32, eta=0.5, kind=0, kappa=0.0):
    V, T = I.cube_surface(N)
    return H2Oracle(V, T, Kernel(kind, kappa), m=m, leaf=leaf, eta=eta)
