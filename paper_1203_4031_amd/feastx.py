"""Thin ctypes binding of libfeastx.so (declared in include/feastx.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Host arrays are numpy arrays (converted to column-major);
device arrays are torch CUDA tensors in column-major layout (strides
(1, ld)), see :func:`fortran_tensor`.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfeastx.so")

_lib = None


class feast_z(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class feast_opts(C.Structure):
    _fields_ = [("ne", C.c_int), ("maxloop", C.c_int), ("conv", C.c_int), ("x0", C.c_int),
                ("keep_factors", C.c_int), ("precision", C.c_int), ("refine", C.c_int),
                ("mode", C.c_int), ("verbose", C.c_int), ("tol", C.c_double),
                ("seed", C.c_ulonglong)]


class feast_stats(C.Structure):
    _fields_ = [("t_total", C.c_double), ("t_shift", C.c_double), ("t_factor", C.c_double),
                ("t_solve", C.c_double), ("t_accum", C.c_double), ("t_rr", C.c_double),
                ("t_reduced", C.c_double), ("t_resid", C.c_double), ("t_lu_gemm", C.c_double),
                ("lu_gemm_flops", C.c_double), ("lu_gemm_launches", C.c_longlong),
                ("factor_flops", C.c_double), ("solve_flops", C.c_double), ("loops", C.c_int),
                ("m0_final", C.c_int), ("eig_calls", C.c_int), ("eig_sweeps", C.c_int)]


def lib():
    """Load libfeastx.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1203_4031_amd.build`")
        L = C.CDLL(LIB_PATH)
        dp, ip, vp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_void_p
        op = C.POINTER(feast_opts)
        L.feast_default_opts.argtypes = [op]
        L.feast_default_opts.restype = None
        for name in ("feast_solve_d", "feast_solve_z"):
            f = getattr(L, name)
            f.argtypes = [C.c_int, vp, vp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double,
                          dp, vp, ip, dp]
        for name in ("feast_solve_d_ex", "feast_solve_z_ex"):
            f = getattr(L, name)
            f.argtypes = [C.c_int, vp, C.c_int, vp, C.c_int, C.c_double, C.c_double, ip, op, dp, vp,
                          C.c_int, ip, dp, ip, dp]
        for name in ("feast_solve_d_dev", "feast_solve_z_dev"):
            f = getattr(L, name)
            f.argtypes = [C.c_int, vp, C.c_int, vp, C.c_int, C.c_double, C.c_double, ip, op, dp, vp,
                          C.c_int, ip, dp, ip, dp, vp]
        L.feast_contour.argtypes = [C.c_double, C.c_double, C.c_int, vp, vp]
        L.feast_rational.argtypes = [C.c_double, C.c_double, C.c_int, dp, C.c_int, dp]
        L.feast_last_stats.argtypes = [C.POINTER(feast_stats)]
        L.feast_set_timing.argtypes = [C.c_int]
        L.feast_set_timing.restype = None
        L.feast_release.argtypes = []
        L.feast_release.restype = None
        L.feast_version.restype = C.c_char_p
        _lib = L
    return _lib


def default_opts() -> feast_opts:
    o = feast_opts()
    lib().feast_default_opts(C.byref(o))
    return o


def make_opts(ne=8, tol=1e-12, maxloop=20, conv=1, x0=None, keep_factors=1, precision="fp64",
              refine=0, mode=0, verbose=0, seed=None) -> feast_opts:
    o = default_opts()
    o.ne, o.tol, o.maxloop, o.conv = ne, tol, maxloop, conv
    o.keep_factors, o.refine, o.mode, o.verbose = keep_factors, refine, mode, verbose
    o.precision = {"fp64": 0, "mixed": 1}[precision] if isinstance(precision, str) else precision
    if x0 is not None:
        o.x0 = int(bool(x0))
    if seed is not None:
        o.seed = seed
    return o


@dataclass
class Result:
    info: int
    E: np.ndarray
    X: object
    res: np.ndarray
    M: int
    m0: int
    loop: int
    epsout: float


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def solve(A, B, emin, emax, m0, X0=None, **kw) -> Result:
    """Host-array solve (numpy).  A, B: (N, N) float64 or complex128 (B may be
    None); X0: optional (N, M0) start subspace.  Options as in make_opts."""
    cplx = np.iscomplexobj(A) or (B is not None and np.iscomplexobj(B))
    dt = np.complex128 if cplx else np.float64
    A = np.asfortranarray(A, dtype=dt)
    n = A.shape[0]
    Bf = None if B is None else np.asfortranarray(B, dtype=dt)
    o = make_opts(x0=X0 is not None, **kw)
    X = np.zeros((n, m0), dtype=dt, order="F")
    if X0 is not None:
        X[:, :] = X0
    E = np.zeros(m0)
    res = np.zeros(m0)
    M = C.c_int(0)
    loop = C.c_int(0)
    eps = C.c_double(0)
    m0c = C.c_int(m0)
    f = lib().feast_solve_z_ex if cplx else lib().feast_solve_d_ex
    info = f(n, A.ctypes.data, n, None if Bf is None else Bf.ctypes.data, n, float(emin), float(emax),
             C.byref(m0c), C.byref(o), _dp(E), X.ctypes.data, n, C.byref(M), _dp(res),
             C.byref(loop), C.byref(eps))
    k = m0c.value if info != 4 else m0
    return Result(info, E[:k].copy(), X[:, :k].copy(order="F"), res[:k].copy(), M.value, k,
                  loop.value, eps.value)


def fortran_tensor(arr, device="cuda"):
    """A torch tensor on `device` holding `arr` column-major (strides (1, N))."""
    import torch

    a = np.asarray(arr)
    t = torch.from_numpy(np.ascontiguousarray(a.T)).to(device)
    return t.t()


def solve_device(A, B, emin, emax, m0, X, stream=None, **kw) -> Result:
    """Device solve: A, B, X are column-major torch CUDA tensors (see
    fortran_tensor); X holds the start subspace if x0=True and receives the
    eigenvectors.  Runs on `stream` (default: torch's current stream)."""
    import torch

    cplx = A.is_complex()
    n = A.shape[0]
    for t in (A, B, X):
        if t is not None and (t.stride(0) != 1 or not t.is_cuda):
            raise ValueError("device arrays must be column-major CUDA tensors")
    if stream is None:
        stream = torch.cuda.current_stream()
    o = make_opts(**kw)
    E = np.zeros(m0)
    res = np.zeros(m0)
    M = C.c_int(0)
    loop = C.c_int(0)
    eps = C.c_double(0)
    m0c = C.c_int(m0)
    f = lib().feast_solve_z_dev if cplx else lib().feast_solve_d_dev
    info = f(n, A.data_ptr(), A.stride(1), None if B is None else B.data_ptr(),
             n if B is None else B.stride(1), float(emin), float(emax), C.byref(m0c), C.byref(o),
             _dp(E), X.data_ptr(), X.stride(1), C.byref(M), _dp(res), C.byref(loop),
             C.byref(eps), C.c_void_p(stream.cuda_stream))
    k = m0c.value if info != 4 else m0
    return Result(info, E[:k].copy(), X[:, :k], res[:k].copy(), M.value, k, loop.value, eps.value)


def contour(emin, emax, ne):
    z = (feast_z * ne)()
    w = (feast_z * ne)()
    info = lib().feast_contour(emin, emax, ne, z, w)
    if info:
        raise ValueError(f"feast_contour info {info}")
    return (np.array([v.re + 1j * v.im for v in z]), np.array([v.re + 1j * v.im for v in w]))


def rational(emin, emax, ne, lam):
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    f = np.zeros(lam.size)
    info = lib().feast_rational(emin, emax, ne, _dp(lam), lam.size, _dp(f))
    if info:
        raise ValueError(f"feast_rational info {info}")
    return f


def stats() -> feast_stats:
    s = feast_stats()
    lib().feast_last_stats(C.byref(s))
    return s


def set_timing(on: bool):
    lib().feast_set_timing(int(bool(on)))


def release():
    lib().feast_release()
