"""Parity bounds of the reduced-precision products (FP32 storage, BF16 coupling).

The oracle gives y_ref = G~ x in FP64 and a = G~ |x|, the sum of the absolute
terms of every row for the positive kernels (for Helmholtz the Laplace matrix
applied to |x|, since |g_Helmholtz| = g_Laplace).  A product computed with
storage precision p (unit roundoff u_p: 2^-24 for FP32, 2^-8 for the BF16
coupling matrices) is held to three bounds at once:

  1. norm, sum scale     ||y - y_ref||    <= T_ABS[p] ||a||
     (a floating-point sum is accurate relative to the sum of its absolute terms)
  2. norm, result scale  ||y - y_ref||    <= T_REL[p] ||y_ref||
     (the accuracy of the product itself; with x ~ N(0,1) the rows of G~ x cancel,
     so ||a|| / ||y_ref|| grows like sqrt(n) and bound 1 alone loosens with n)
  3. entry by entry      |y_i - y_ref_i| <= C_ELEM[p] u_p a_i   for every i
     (no row may carry a local error that a 2-norm over many rows would hide;
     C_ELEM covers the Lebesgue constant of the interpolation, which enters
     because V and E hold Lagrange values of both signs, and the length of the
     partial sums)
Every check prints the three measured ratios, so the margins can be read off a
run with `pytest -s`.  Over the 2,702 FP32 comparisons of the GPU suite (1,280 to
1,310,720 triangles, one to 70 columns) the largest measured values were
|d|/|a| = 8.3e-8, |d|/|ref| = 2.8e-6 (a column of the 786,432-triangle cube) and
an entry ratio of 0.49 against C = 16; over the BF16 cases 2.1e-5, 6.7e-4 and
0.08 against C = 1/4.
"""
import numpy as np

U = {"f32": 2.0 ** -24, "f32_sbf16": 2.0 ** -8}
T_ABS = {"f32": 1e-6, "f32_sbf16": 2e-3}
T_REL = {"f32": 5e-6, "f32_sbf16": 2e-3}
C_ELEM = {"f32": 16.0, "f32_sbf16": 0.25}


def ratios(y, ref, a, storage, extra=0.0):
    """(||y-ref||/||a||, ||y-ref||/||ref||, max_i |y_i-ref_i| / (C u a_i + extra_i)) ."""
    y, ref, a = (np.asarray(v) for v in (y, ref, a))
    d = np.abs(y - ref)
    nd = float(np.linalg.norm(y - ref))
    r_abs = nd / float(np.linalg.norm(a))
    nr = float(np.linalg.norm(ref))
    r_rel = nd / nr if nr > 0 else (0.0 if nd == 0 else np.inf)
    lim = C_ELEM[storage] * U[storage] * np.abs(a) + extra
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(lim > 0, d / np.where(lim > 0, lim, 1.0), np.where(d > 0, np.inf, 0.0))
    return r_abs, r_rel, float(q.max()) if q.size else 0.0


def check(y, ref, a, storage, label="", extra=0.0, t_rel=None, t_abs=None):
    """Assert bounds 1-3 for `storage` ("f32" or "f32_sbf16").  `extra` (scalar or
    per entry) is added to the entry-wise limit, e.g. the FP64 rounding of a large
    y0 accumulated into; t_rel / t_abs override the norm bounds where a case
    states its own (the bound 1 factor for a scaled product, for instance)."""
    r_abs, r_rel, r_elem = ratios(y, ref, a, storage, extra)
    ta = T_ABS[storage] if t_abs is None else t_abs
    tr = T_REL[storage] if t_rel is None else t_rel
    print("bounds %s [%s]: |d|/|a| = %.3e (<= %.0e)  |d|/|ref| = %.3e (<= %.0e)  max entry ratio = %.3f"
          % (label, storage, r_abs, ta, r_rel, tr, r_elem), flush=True)
    assert r_abs <= ta, (label, "sum-scale bound", r_abs)
    assert r_rel <= tr, (label, "result-scale bound", r_rel)
    assert r_elem <= 1.0, (label, "entry-wise bound", r_elem)
