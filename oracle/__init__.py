"""ctypes wrapper around the FP64 CPU oracle (``feast_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this; the GPU library never does.  The shared object is
built by :func:`build` (``gcc -O2 -fopenmp``), which ``__graft_entry__.build``
calls.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "feast_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so``."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-fcx-fortran-rules", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        vp = C.c_void_p
        lib.orc_gauss_legendre.argtypes = [C.c_int, dp, dp]
        lib.orc_contour.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, vp, vp]
        lib.orc_rational.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, dp, C.c_int, dp]
        lib.orc_rationalx.argtypes = [C.c_int, vp, vp, dp, C.c_int, dp]
        lib.orc_rationalx.restype = None
        lib.orc_zgetrf.argtypes = [C.c_int, vp, C.c_int, ip]
        lib.orc_zgetrs.argtypes = [C.c_char, C.c_int, C.c_int, vp, C.c_int, ip, vp, C.c_int]
        lib.orc_zgemm.argtypes = [C.c_char, C.c_int, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int,
                                  vp, C.c_int]
        lib.orc_zgemm.restype = None
        lib.orc_zheev_jacobi.argtypes = [C.c_int, vp, C.c_int, dp, vp, C.c_int]
        lib.orc_feast.argtypes = [C.c_int, C.c_int, vp, vp, C.c_double, C.c_double, ip, C.c_int,
                                  C.c_double, C.c_int, C.c_int, C.c_int, vp, dp, vp, dp, ip, ip,
                                  dp, C.c_int, C.c_int, vp, vp]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _z(a):
    return np.asfortranarray(a, dtype=np.complex128)


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    if _load().orc_gauss_legendre(n, _dp(x), _dp(w)):
        raise ValueError("n must be >= 1")
    return x, w


def contour(emin: float, emax: float, ne: int, integration: int = 0, ellipse: int = 100):
    """Half-contour nodes and weights: integration = fpm(16) (0 Gauss-Legendre,
    1 trapezoidal), ellipse = fpm(18) (vertical / horizontal semi-axis, %)."""
    z = np.zeros(ne, np.complex128)
    w = np.zeros(ne, np.complex128)
    if _load().orc_contour(emin, emax, ne, integration, ellipse, z.ctypes.data, w.ctypes.data):
        raise ValueError("bad contour arguments")
    return z, w


def rational(emin: float, emax: float, ne: int, lam, integration: int = 0, ellipse: int = 100):
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    f = np.zeros(lam.size)
    if _load().orc_rational(emin, emax, ne, integration, ellipse, _dp(lam), lam.size, _dp(f)):
        raise ValueError("bad contour arguments")
    return f


def rationalx(z, w, lam):
    """The filter Re sum_j w_j / (z_j - lambda) of given nodes and weights."""
    z = np.ascontiguousarray(z, dtype=np.complex128)
    w = np.ascontiguousarray(w, dtype=np.complex128)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    f = np.zeros(lam.size)
    _load().orc_rationalx(z.size, z.ctypes.data, w.ctypes.data, _dp(lam), lam.size, _dp(f))
    return f


def zgetrf(a):
    """LU with partial pivoting; returns (lu, ipiv, info)."""
    lu = _z(a).copy(order="F")
    n = lu.shape[0]
    ipiv = np.zeros(n, np.int32)
    info = _load().orc_zgetrf(n, lu.ctypes.data, n, _ip(ipiv))
    return lu, ipiv, info


def zgetrs(lu, ipiv, b, trans: str = "N"):
    lu = _z(lu)
    b2 = _z(b).copy(order="F")
    if b2.ndim == 1:
        b2 = b2.reshape(-1, 1, order="F")
    n = lu.shape[0]
    _load().orc_zgetrs(trans.encode(), n, b2.shape[1], lu.ctypes.data, n,
                       _ip(np.ascontiguousarray(ipiv, np.int32)), b2.ctypes.data, n)
    return b2


def zgemm(a, b, opa: str = "N"):
    a = _z(a)
    b = _z(b)
    m = a.shape[0] if opa == "N" else a.shape[1]
    k = a.shape[1] if opa == "N" else a.shape[0]
    n = b.shape[1]
    c = np.zeros((m, n), np.complex128, order="F")
    _load().orc_zgemm(opa.encode(), m, n, k, a.ctypes.data, a.shape[0], b.ctypes.data,
                      b.shape[0], c.ctypes.data, m)
    return c


def jacobi_eigh(a):
    """Hermitian eigendecomposition by cyclic Jacobi: (w ascending, V, info)."""
    a2 = _z(a).copy(order="F")
    n = a2.shape[0]
    w = np.zeros(n)
    v = np.zeros((n, n), np.complex128, order="F")
    info = _load().orc_zheev_jacobi(n, a2.ctypes.data, n, _dp(w), v.ctypes.data, n)
    return w, v, info


@dataclass
class OracleResult:
    info: int
    E: np.ndarray
    X: np.ndarray
    res: np.ndarray
    M: int
    m0: int
    loop: int
    epsout: float


def feast(A, B, emin, emax, m0, ne, tol, X0, *, hermitian=False, maxloop=20, conv=1,
          mode=0, integration=0, ellipse=100, zne=None, wne=None) -> OracleResult:
    """Run the oracle's FEAST iteration.  Real symmetric input returns real X."""
    A = _z(A)
    n = A.shape[0]
    Bz = None if B is None else _z(B)
    X0z = _z(X0)
    if X0z.shape != (n, m0):
        raise ValueError("X0 must be (N, M0)")
    E = np.zeros(m0)
    X = np.zeros((n, m0), np.complex128, order="F")
    res = np.zeros(m0)
    M = np.zeros(1, np.int32)
    loop = np.zeros(1, np.int32)
    eps = np.zeros(1)
    m0a = np.array([m0], np.int32)
    if (zne is None) != (wne is None):
        raise ValueError("zne and wne go together")
    if zne is not None:
        zc = np.ascontiguousarray(zne, dtype=np.complex128)
        wc = np.ascontiguousarray(wne, dtype=np.complex128)
        if zc.size != ne or wc.size != ne:
            raise ValueError("zne and wne need ne entries")
    info = _load().orc_feast(int(bool(hermitian)), n, A.ctypes.data,
                             None if Bz is None else Bz.ctypes.data, float(emin), float(emax),
                             _ip(m0a), int(ne), float(tol), int(maxloop), int(conv), int(mode),
                             X0z.ctypes.data, _dp(E), X.ctypes.data, _dp(res), _ip(M),
                             _ip(loop), _dp(eps), int(integration), int(ellipse),
                             None if zne is None else zc.ctypes.data,
                             None if wne is None else wc.ctypes.data)
    m0o = int(m0a[0])
    if not hermitian:
        X = np.asfortranarray(X.real)
    return OracleResult(info, E[:m0o].copy(), X[:, :m0o].copy(order="F"), res[:m0o].copy(),
                        int(M[0]), m0o, int(loop[0]), float(eps[0]))
