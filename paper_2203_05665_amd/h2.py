"""ctypes binding of the C ABI in include/h2.h (argument marshalling only).

Every computation happens in libh2mi355x.so; this module converts arrays to
pointers and checks return codes.  Device vectors are torch CUDA tensors
(float64 or float32, contiguous, length n or n x nrhs in Fortran order); the
stream is torch's current stream unless given.  Loading fails loudly if the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libh2mi355x.so")

# constants of include/h2.h
H2_OK, H2_EINVAL, H2_ENOMEM, H2_EHIP, H2_ENOTCONV, H2_EINTERNAL = 0, -1, -2, -3, -4, -5
H2_LAPLACE, H2_HELMHOLTZ, H2_TEST_ONE, H2_TEST_BILINEAR, H2_TEST_QUADRATIC = 0, 1, 2, 3, 4
H2_F64, H2_F32, H2_F32_SBF16 = 0, 1, 2
H2_R64, H2_R32, H2_C128, H2_C64 = 0, 1, 2, 3
H2_ACC_F64, H2_OVERWRITE = 1, 2
H2_KS_PRODUCT, H2_KS_DONE, H2_KS_NOTCONV, H2_KS_FAILED = 1, 2, 3, 4
KS_STATES = {H2_KS_PRODUCT: "product", H2_KS_DONE: "done", H2_KS_NOTCONV: "not_converged", H2_KS_FAILED: "failed"}
H2_HOST_ONLY, H2_COUPLING_OTF, H2_SYMMETRIC, H2_SYMMETRIC_NEAR = 1, 2, 4, 8
H2_CG, H2_GMRES = 0, 1
(H2_X_PERM, H2_X_CLUSTERS, H2_X_BOXES, H2_X_ADM, H2_X_NEAR, H2_X_DFS, H2_X_V, H2_X_E, H2_X_S,
 H2_X_N) = range(10)
H2_PH_FORWARD, H2_PH_COUPLING, H2_PH_DOWN, H2_PH_NEAR, H2_PH_TOTAL, H2_NPHASE = 0, 1, 2, 3, 4, 5
H2_TUNE_NONE, H2_TUNE_PASS_COLUMNS, H2_TUNE_SMALL_SLOT, H2_TUNE_ROW_ORDER = -1, 0, 1, 2
TUNE_KNOBS = {"pass_columns": H2_TUNE_PASS_COLUMNS, "small_slot": H2_TUNE_SMALL_SLOT, "row_order": H2_TUNE_ROW_ORDER}

KERNELS = {"laplace": H2_LAPLACE, "helmholtz": H2_HELMHOLTZ, "one": H2_TEST_ONE,
           "bilinear": H2_TEST_BILINEAR, "quadratic": H2_TEST_QUADRATIC}
STORAGE = {"f64": H2_F64, "f32": H2_F32, "f32_sbf16": H2_F32_SBF16}


class h2_mesh(C.Structure):
    _fields_ = [("nv", C.c_int64), ("nt", C.c_int64), ("vertices", C.POINTER(C.c_double)),
                ("triangles", C.POINTER(C.c_int32))]


class h2_params(C.Structure):
    _fields_ = [("kernel", C.c_int), ("kappa", C.c_double), ("order_m", C.c_int), ("leaf_size", C.c_int),
                ("eta", C.c_double), ("q_ss", C.c_int), ("storage", C.c_int), ("flags", C.c_int)]


class h2_stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in ("n", "nclusters", "nleaves", "depth", "n_adm", "n_near",
                                         "near_entries", "m", "k", "storage", "kernel", "bytes_S",
                                         "bytes_N", "bytes_V", "bytes_E", "bytes_total")] + \
               [("matvec_bytes", C.c_double), ("matvec_flops", C.c_double),
                ("s_blocks_stored", C.c_int64), ("near_entries_stored", C.c_int64)]


class h2_solve_params(C.Structure):
    _fields_ = [("method", C.c_int), ("restart", C.c_int), ("maxit", C.c_int), ("rtol", C.c_double),
                ("refine", C.c_int), ("inner_rtol", C.c_double)]


class h2_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outer", C.c_int), ("rel_residual", C.c_double),
                ("seconds", C.c_double)]


class h2_krylov_status(C.Structure):
    _fields_ = [("state", C.c_int), ("iterations", C.c_int), ("outer", C.c_int), ("products", C.c_int),
                ("rel_residual", C.c_double), ("message", C.c_char * 128)]


class h2_recompress_info(C.Structure):
    _fields_ = [("rank", C.c_int64), ("rank_before", C.c_int64), ("discarded", C.c_double),
                ("seconds", C.c_double), ("bytes_before", C.c_int64), ("bytes_after", C.c_int64)]


class h2_tune_info(C.Structure):
    _fields_ = [("knob", C.c_int), ("ncand", C.c_int), ("value", C.c_int * 4), ("ms", C.c_double * 4),
                ("chosen", C.c_int)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError("HIP library %s is missing: build it first "
                               "(python paper_2203_05665_amd/build_lib.py)" % LIBPATH)
        L = C.CDLL(LIBPATH)
        L.build_h2.argtypes = [C.POINTER(h2_mesh), C.POINTER(h2_params), C.POINTER(C.c_void_p)]
        L.h2_matvec.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                C.c_double, C.c_int, C.c_void_p]
        L.h2_solve.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                               C.POINTER(h2_solve_params), C.POINTER(h2_solve_info), C.c_void_p]
        L.h2_solve_noalloc.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                       C.POINTER(h2_solve_params), C.POINTER(h2_solve_info), C.c_void_p]
        L.h2_krylov_workspace.argtypes = [C.c_int, C.c_int64, C.c_int, C.POINTER(h2_solve_params)]
        L.h2_krylov_workspace.restype = C.c_int64
        L.h2_krylov_create.argtypes = [C.c_int, C.c_int64, C.c_int, C.POINTER(h2_solve_params), C.c_void_p,
                                       C.c_int64, C.c_void_p, C.POINTER(C.c_void_p)]
        L.h2_krylov_begin.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]
        L.h2_krylov_next.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int), C.c_void_p]
        L.h2_krylov_advance.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.h2_krylov_poll.argtypes = [C.c_void_p, C.POINTER(h2_krylov_status)]
        L.h2_krylov_residuals.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
        L.h2_krylov_solution.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.h2_krylov_destroy.argtypes = [C.c_void_p]
        L.h2_krylov_destroy.restype = None
        L.h2_stream_read.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_int64, C.c_void_p]
        L.h2_info.argtypes = [C.c_void_p, C.POINTER(h2_stats)]
        L.h2_free.argtypes = [C.c_void_p]
        L.h2_free.restype = None
        L.h2_last_error.restype = C.c_char_p
        L.h2_export.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_int64]
        L.h2_profile.argtypes = [C.c_void_p, C.c_int]
        L.h2_profile_read.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.h2_krylov_dots.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_int64, C.c_int64,
                                     C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.h2_krylov_update.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_int64, C.c_int64,
                                       C.c_void_p, C.c_double, C.c_void_p, C.c_int64, C.c_void_p]
        L.h2_recompress.argtypes = [C.c_void_p, C.c_double, C.c_int, C.POINTER(h2_recompress_info), C.c_void_p]
        L.h2_tune.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(h2_tune_info), C.c_void_p]
        L.h2_set_tuning.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.h2_tune_knob.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(h2_tune_info),
                                   C.c_void_p]
        for f in ("build_h2", "h2_matvec", "h2_solve", "h2_solve_noalloc", "h2_info", "h2_export", "h2_profile", "h2_profile_read",
                  "h2_krylov_dots", "h2_krylov_update", "h2_recompress", "h2_tune", "h2_set_tuning",
                  "h2_krylov_create", "h2_krylov_begin", "h2_krylov_next", "h2_krylov_advance", "h2_krylov_poll",
                  "h2_krylov_residuals", "h2_krylov_solution", "h2_stream_read", "h2_tune_knob"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


class H2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("h2 error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc != H2_OK:
        raise H2Error(rc, h2_last_error())
    return rc


def h2_last_error() -> str:
    m = lib().h2_last_error()
    return m.decode() if m else ""


def build_h2(vertices, triangles, kernel="laplace", kappa=0.0, order=4, leaf=64, eta=0.5, q_ss=4,
             storage="f64", host_only=False, coupling_otf=False, symmetric=False, symmetric_near=False):
    """Calls build_h2; returns the raw handle (int)."""
    V = np.ascontiguousarray(vertices, dtype=np.float64)
    T = np.ascontiguousarray(triangles, dtype=np.int32)
    mesh = h2_mesh(V.shape[0], T.shape[0], V.ctypes.data_as(C.POINTER(C.c_double)),
                   T.ctypes.data_as(C.POINTER(C.c_int32)))
    prm = h2_params(KERNELS[kernel] if isinstance(kernel, str) else int(kernel), float(kappa), int(order),
                    int(leaf), float(eta), int(q_ss), STORAGE[storage] if isinstance(storage, str) else int(storage),
                    (H2_HOST_ONLY if host_only else 0) | (H2_COUPLING_OTF if coupling_otf else 0) |
                    (H2_SYMMETRIC if symmetric else 0) | (H2_SYMMETRIC_NEAR if symmetric_near else 0))
    h = C.c_void_p()
    _check(lib().build_h2(C.byref(mesh), C.byref(prm), C.byref(h)))
    return h.value


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def h2_matvec(h, x, y, alpha=1.0, acc64=False, stream=None, overwrite=False):
    """y <- y + alpha G~ x (or y <- alpha G~ x with overwrite) for torch CUDA tensors
    x, y (n or n x nrhs, Fortran order)."""
    import torch
    dtypes = {torch.float64: H2_R64, torch.float32: H2_R32, torch.complex128: H2_C128, torch.complex64: H2_C64}
    if x.dtype != y.dtype or x.dtype not in dtypes:
        raise TypeError("x and y must have the same dtype: float64, float32, complex128 or complex64")
    if x.dim() not in (1, 2) or x.shape != y.shape:
        raise ValueError("x and y must have the same shape, n or n x nrhs")
    nrhs = 1 if x.dim() == 1 else x.shape[1]
    n = x.shape[0]
    if n != h2_info(h)["n"]:
        raise ValueError("x has %d rows, the matrix has %d" % (n, h2_info(h)["n"]))
    if not (x.is_cuda and y.is_cuda):
        raise TypeError("x and y must be device tensors")
    # a single column may carry any stride in its second dimension
    ldx = x.stride(1) if x.dim() == 2 and nrhs > 1 else n
    ldy = y.stride(1) if y.dim() == 2 and nrhs > 1 else n
    if n > 1 and (x.stride(0) != 1 or y.stride(0) != 1):
        raise ValueError("columns must be contiguous")
    dt = dtypes[x.dtype]
    _check(lib().h2_matvec(h, nrhs, dt, x.data_ptr(), ldx, y.data_ptr(), ldy, float(alpha),
                           (H2_ACC_F64 if acc64 else 0) | (H2_OVERWRITE if overwrite else 0), _stream(stream)))
    return y


def _block(v, n, name):
    """(pointer, nrhs, ld) of a device vector or Fortran-ordered n x nrhs block."""
    if v.dim() == 1:
        v2 = v[:, None]
    elif v.dim() == 2:
        v2 = v
    else:
        raise ValueError("%s must have shape (n,) or (n, nrhs)" % name)
    if v2.shape[0] != n:
        raise ValueError("%s has %d rows, the matrix has %d" % (name, v2.shape[0], n))
    r = v2.shape[1]
    if r > 0 and n > 1 and v2.stride(0) != 1:
        raise ValueError("%s: columns must be contiguous" % name)
    ld = v2.stride(1) if r > 1 else n
    if r > 1 and ld < n:
        raise ValueError("%s: columns overlap" % name)
    return v2.data_ptr(), r, ld


def solve_params(method="cg", rtol=1e-8, maxit=1000, restart=50, refine=False, inner_rtol=1e-4):
    return h2_solve_params(H2_CG if method == "cg" else H2_GMRES, int(restart), int(maxit), float(rtol),
                           1 if refine else 0, float(inner_rtol))


def h2_solve(h, b, z, method="cg", rtol=1e-8, maxit=1000, restart=50, refine=False, inner_rtol=1e-4,
             stream=None, check=True, noalloc=False):
    """Solves G~ Z = B for float64 (complex128 for Helmholtz) device blocks b, z of
    shape (n,) or (n, nrhs) with contiguous columns; z holds the initial guess
    and the result.  noalloc: the allocation-free entry point h2_solve_noalloc."""
    import torch
    want = torch.complex128 if b.is_complex() else torch.float64
    if b.dtype != want or z.dtype != want:
        raise TypeError("b and z must be float64 (complex128 for Helmholtz) tensors")
    n = h2_info(h)["n"]
    pb, rb, ldb = _block(b, n, "b")
    pz, rz, ldz = _block(z, n, "z")
    if rb != rz:
        raise ValueError("b and z must have the same number of columns")
    if not (b.is_cuda and z.is_cuda):
        raise TypeError("b and z must be device tensors")
    p = solve_params(method, rtol, maxit, restart, refine, inner_rtol)
    info = h2_solve_info()
    dt = H2_C128 if b.is_complex() else H2_R64
    fn = lib().h2_solve_noalloc if noalloc else lib().h2_solve
    rc = fn(h, rb, dt, pb, ldb, pz, ldz, C.byref(p), C.byref(info), _stream(stream))
    if rc != H2_ENOTCONV or check:
        _check(rc)
    return dict(iterations=info.iterations, outer=info.outer, rel_residual=info.rel_residual,
                seconds=info.seconds, converged=rc == H2_OK)


class KrylovSolve:
    """The step-wise solver of include/h2.h (h2_krylov_*) on caller-owned device
    workspace: `next` writes the block whose product the solve needs, `advance`
    takes the product, `poll` (after the stream completed) decides."""

    def __init__(self, n, nrhs, complex_, params, workspace_ptr, workspace_bytes, status_ptr=None):
        self.n, self.nrhs = int(n), int(nrhs)
        self.dtype = H2_C128 if complex_ else H2_R64
        self.params = params
        k = C.c_void_p()
        _check(lib().h2_krylov_create(self.dtype, self.n, self.nrhs, C.byref(params), workspace_ptr,
                                      int(workspace_bytes), status_ptr, C.byref(k)))
        self.k = k.value
        self._res = (C.c_double * self.nrhs)()

    @staticmethod
    def workspace_bytes(n, nrhs, complex_, params):
        b = lib().h2_krylov_workspace(H2_C128 if complex_ else H2_R64, int(n), int(nrhs), C.byref(params))
        if b < 0:
            raise ValueError("invalid solver parameters")
        return int(b)

    def begin(self, b, z0=None, stream=None):
        pb, _, ldb = _block(b, self.n, "b")
        pz, ldz = (None, self.n) if z0 is None else _block(z0, self.n, "z0")[::2]
        _check(lib().h2_krylov_begin(self.k, pb, ldb, pz, ldz, _stream(stream)))

    def next(self, x=None, stream=None):
        """(state, flags); with x = None only reports what the next product needs."""
        fl = C.c_int(0)
        if x is None:
            rc = lib().h2_krylov_next(self.k, None, 0, C.byref(fl), _stream(stream))
        else:
            px, _, ldx = _block(x, self.n, "x")
            rc = lib().h2_krylov_next(self.k, px, ldx, C.byref(fl), _stream(stream))
        if rc < 0:
            _check(rc)
        return rc, fl.value

    def advance(self, y, stream=None):
        py, _, ldy = _block(y, self.n, "y")
        _check(lib().h2_krylov_advance(self.k, py, ldy, _stream(stream)))

    def poll(self):
        st = h2_krylov_status()
        rc = lib().h2_krylov_poll(self.k, C.byref(st))
        if rc < 0:
            _check(rc)
        return dict(state=KS_STATES[st.state], iterations=st.iterations, outer=st.outer, products=st.products,
                    rel_residual=st.rel_residual, message=st.message.decode())

    def residuals(self):
        _check(lib().h2_krylov_residuals(self.k, self._res))
        return np.array(self._res[:], dtype=np.float64)

    def solution(self, z, stream=None):
        pz, _, ldz = _block(z, self.n, "z")
        _check(lib().h2_krylov_solution(self.k, pz, ldz, _stream(stream)))

    def close(self):
        if self.k:
            lib().h2_krylov_destroy(self.k)
            self.k = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _kdtype(t):
    import torch
    if t.dtype == torch.complex128:
        return H2_C128
    if t.dtype == torch.float64:
        return H2_R64
    raise TypeError("Krylov kernels take float64 or complex128 tensors")


def h2_krylov_dots(Q, W, nvec, stream=None):
    """h[r, i] = sum_k conj(Q[r, i, k]) W[r, k] for i < nvec; Q (r, m, n), W (r, n), unit last stride."""
    import torch
    r, _, n = Q.shape
    if Q.stride(2) != 1 or W.stride(1) != 1 or W.dtype != Q.dtype or W.shape != (r, n):
        raise ValueError("bad Krylov operands")
    h = torch.empty((r, nvec), dtype=Q.dtype, device=Q.device)
    _check(lib().h2_krylov_dots(_kdtype(Q), r, nvec, n, Q.data_ptr(), Q.stride(0), Q.stride(1), W.data_ptr(),
                                W.stride(0), h.data_ptr(), _stream(stream)))
    return h


def h2_krylov_update(Q, h, W, sign=1.0, stream=None):
    """W[r, k] += sign * sum_i h[r, i] Q[r, i, k] for i < h.shape[1]."""
    r, nvec = h.shape
    n = W.shape[1]
    if Q.stride(2) != 1 or W.stride(1) != 1 or not h.is_contiguous() or h.dtype != Q.dtype or W.dtype != Q.dtype:
        raise ValueError("bad Krylov operands")
    _check(lib().h2_krylov_update(_kdtype(Q), r, nvec, n, Q.data_ptr(), Q.stride(0), Q.stride(1), h.data_ptr(),
                                  float(sign), W.data_ptr(), W.stride(0), _stream(stream)))
    return W


def h2_stream_read(buf, sink, loads=8, stream=None):
    """Launch the read-only streaming kernel over the bytes of device tensor `buf`
    with `loads` (4, 8, 16) loads in flight per thread (sink: a device tensor of
    at least 16 KiB)."""
    _check(lib().h2_stream_read(buf.data_ptr(), buf.numel() * buf.element_size(), int(loads), sink.data_ptr(),
                                sink.numel() * sink.element_size(), _stream(stream)))


def h2_recompress(h, eps, max_rank=0, stream=None) -> dict:
    """Algebraic recompression in place (orthonormal nested bases truncated at the
    relative tolerance eps per cluster, uniform rank k'); returns the info fields."""
    info = h2_recompress_info()
    _check(lib().h2_recompress(h, float(eps), int(max_rank), C.byref(info), _stream(stream)))
    return {f: getattr(info, f) for f, _ in h2_recompress_info._fields_}


def h2_tune(h, nrhs=1, dtype="f64", reps=10, stream=None, knob=None) -> dict:
    """Time every tile choice of the product path for nrhs columns of the given
    vector type ("f64", "f32", "c128", "c64") on the handle and keep the fastest
    (see h2_tune in include/h2.h; `knob` names one knob, h2_tune_knob); returns
    the knob, the values tried, their median ms and the value kept."""
    dt = {"f64": H2_R64, "f32": H2_R32, "c128": H2_C128, "c64": H2_C64}[dtype]
    info = h2_tune_info()
    if knob is None:
        _check(lib().h2_tune(h, int(nrhs), dt, int(reps), C.byref(info), _stream(stream)))
    else:
        _check(lib().h2_tune_knob(h, TUNE_KNOBS[knob] if isinstance(knob, str) else int(knob), int(nrhs), dt,
                                  int(reps), C.byref(info), _stream(stream)))
    names = {v: k for k, v in TUNE_KNOBS.items()}
    vals = [info.value[i] for i in range(info.ncand)]
    return {"knob": names.get(info.knob), "values": vals, "ms": [info.ms[i] for i in range(info.ncand)],
            "chosen": vals[info.chosen] if vals else None}


def h2_set_tuning(h, knob, value):
    """Set a tile knob ("pass_columns", "small_slot" or "row_order") directly; 0 restores the rule."""
    _check(lib().h2_set_tuning(h, TUNE_KNOBS[knob] if isinstance(knob, str) else int(knob), int(value)))


def h2_info(h) -> dict:
    s = h2_stats()
    _check(lib().h2_info(h, C.byref(s)))
    return {f: getattr(s, f) for f, _ in h2_stats._fields_}


def h2_free(h):
    if h:
        lib().h2_free(h)


def h2_export(h, what, index=0, count=None, dtype=None):
    """Host copy of structure or matrix data (see H2_X_* in include/h2.h)."""
    info = h2_info(h)
    nc, k = info["nclusters"], info["k"]
    cplx = info["kernel"] == H2_HELMHOLTZ
    sizes = {H2_X_PERM: (info["n"], np.int32), H2_X_CLUSTERS: (6 * nc, np.int32),
             H2_X_BOXES: (6 * nc, np.float64), H2_X_ADM: (2 * info["n_adm"], np.int32),
             H2_X_NEAR: (2 * info["n_near"], np.int32), H2_X_DFS: (nc, np.int32),
             H2_X_E: (k * k, np.float64), H2_X_S: (k * k * (2 if cplx else 1), np.float64)}
    if what in sizes:
        cnt, dt = sizes[what]
    else:
        cnt, dt = count, np.float64
    out = np.zeros(max(int(cnt), 1), dtype=dt)
    _check(lib().h2_export(h, what, int(index), out.ctypes.data, int(cnt)))
    return out[:cnt]


def h2_profile(h, enable: bool):
    _check(lib().h2_profile(h, 1 if enable else 0))


def h2_profile_read(h):
    ms = (C.c_double * H2_NPHASE)()
    calls = (C.c_int64 * H2_NPHASE)()
    _check(lib().h2_profile_read(h, ms, calls))
    names = ["forward", "coupling", "down", "near", "total"]
    return {nm: (ms[i], calls[i]) for i, nm in enumerate(names)}


class H2Matrix:
    """Owning wrapper: H2Matrix(vertices, triangles, ...) builds; .matvec / .solve apply."""

    def __init__(self, vertices, triangles, **kw):
        self.h = build_h2(vertices, triangles, **kw)
        self.info = h2_info(self.h)
        self.n = self.info["n"]

    def matvec(self, x, y=None, alpha=1.0, acc64=False, stream=None, overwrite=False):
        import torch
        if y is None:
            y = torch.zeros_like(x)
        return h2_matvec(self.h, x, y, alpha, acc64, stream, overwrite)

    def recompress(self, eps, max_rank=0, stream=None):
        """Replace V, E and S by a recompressed representation of rank k' (see h2_recompress)."""
        out = h2_recompress(self.h, eps, max_rank, stream)
        self.info = h2_info(self.h)
        return out

    def tune(self, nrhs=1, dtype="f64", reps=10, stream=None, knob=None):
        """Pick the fastest tile shapes for products with nrhs columns (see h2_tune)."""
        return h2_tune(self.h, nrhs, dtype, reps, stream, knob)

    def set_tuning(self, knob, value):
        h2_set_tuning(self.h, knob, value)

    def solve(self, b, z=None, **kw):
        import torch
        if z is None:
            z = torch.zeros_like(b)
        return z, h2_solve(self.h, b, z, **kw)

    def export(self, what, index=0, count=None):
        return h2_export(self.h, what, index, count)

    def close(self):
        h2_free(self.h)
        self.h = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.close()
        except Exception:
            pass
