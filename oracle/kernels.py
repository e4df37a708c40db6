"""Kernel functions g(x, y) (FP64).  TEST INFRASTRUCTURE ONLY.

Laplace g = 1/(4 pi |x-y|) and Helmholtz g = exp(i kappa |x-y|)/(4 pi |x-y|)
are the two kernels named in the paper's introduction.  The polynomial test
kernels (1, x.y, (x.y)^2) are not in the paper; they are interpolated exactly by
tensor Chebyshev interpolation of order m >= 1, 2, 3 respectively and their
Galerkin products have closed forms, which pins the whole H^2 product at any
mesh size.
"""
from __future__ import annotations

import math

import numpy as np

LAPLACE, HELMHOLTZ, TEST_ONE, TEST_BILINEAR, TEST_QUADRATIC = 0, 1, 2, 3, 4


class Kernel:
    def __init__(self, kind: int = LAPLACE, kappa: float = 0.0):
        self.kind = int(kind)
        self.kappa = float(kappa)
        self.complex = self.kind == HELMHOLTZ
        self.dtype = np.complex128 if self.complex else np.float64
        self.smooth = self.kind in (TEST_ONE, TEST_BILINEAR, TEST_QUADRATIC)

    def __call__(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        """g(x, y) for broadcastable arrays of points (..., 3)."""
        if self.kind == TEST_ONE:
            return np.ones(np.broadcast_shapes(x.shape, y.shape)[:-1])
        if self.kind == TEST_BILINEAR:
            return x[..., 0] * y[..., 0] + x[..., 1] * y[..., 1] + x[..., 2] * y[..., 2]
        if self.kind == TEST_QUADRATIC:
            return (x[..., 0] * y[..., 0] + x[..., 1] * y[..., 1] + x[..., 2] * y[..., 2]) ** 2
        d0 = x[..., 0] - y[..., 0]
        d1 = x[..., 1] - y[..., 1]
        d2 = x[..., 2] - y[..., 2]
        r = np.sqrt(d0 * d0 + d1 * d1 + d2 * d2)
        if self.kind == LAPLACE:
            return 1.0 / (4.0 * math.pi * r)
        if self.kind == HELMHOLTZ:
            return np.exp(1j * self.kappa * r) / (4.0 * math.pi * r)
        raise ValueError(self.kind)
