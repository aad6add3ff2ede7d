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
                ("seed", C.c_ulonglong), ("integration", C.c_int), ("ellipse", C.c_int),
                ("Zne", C.c_void_p), ("Wne", C.c_void_p), ("ne_full", C.c_int),
                ("integration_full", C.c_int), ("angle", C.c_int)]


class feast_stats(C.Structure):
    _fields_ = [("t_total", C.c_double), ("t_shift", C.c_double), ("t_factor", C.c_double),
                ("t_solve", C.c_double), ("t_accum", C.c_double), ("t_rr", C.c_double),
                ("t_reduced", C.c_double), ("t_resid", C.c_double), ("t_lu_gemm", C.c_double),
                ("lu_gemm_flops", C.c_double), ("lu_gemm_launches", C.c_longlong),
                ("factor_flops", C.c_double), ("solve_flops", C.c_double), ("loops", C.c_int),
                ("m0_final", C.c_int), ("eig_calls", C.c_int), ("eig_sweeps", C.c_int),
                ("t_lu_update", C.c_double), ("lu_update_flops", C.c_double), ("lu_update_launches", C.c_longlong),
                ("fp64_nodes", C.c_int)]


class feast_job(C.Structure):
    _fields_ = [("n", C.c_int), ("A", C.c_void_p), ("lda", C.c_int), ("B", C.c_void_p), ("ldb", C.c_int),
                ("emin", C.c_double), ("emax", C.c_double), ("m0", C.c_int), ("X", C.c_void_p),
                ("ldx", C.c_int), ("E", C.c_void_p), ("res", C.c_void_p), ("info", C.c_int),
                ("M", C.c_int), ("m0_out", C.c_int), ("loop", C.c_int), ("epsout", C.c_double),
                ("ms", C.c_double)]


class feast_server_cfg(C.Structure):
    _fields_ = [("slots", C.c_int), ("hbm_budget_gb", C.c_double)]


class feast_request(C.Structure):
    _fields_ = [("hermitian", C.c_int), ("n", C.c_int), ("A", C.c_void_p), ("lda", C.c_int),
                ("B", C.c_void_p), ("ldb", C.c_int), ("emin", C.c_double), ("emax", C.c_double),
                ("m0", C.c_int), ("X0", C.c_void_p), ("ldx", C.c_int), ("opts", feast_opts)]


class feast_result(C.Structure):
    _fields_ = [("info", C.c_int), ("M", C.c_int), ("m0", C.c_int), ("loop", C.c_int),
                ("epsout", C.c_double), ("E", C.c_void_p), ("res", C.c_void_p), ("X", C.c_void_p),
                ("ldx", C.c_int), ("queue_ms", C.c_double), ("run_ms", C.c_double),
                ("latency_ms", C.c_double)]


TILE_VARIANTS = 3


class feast_tiles(C.Structure):
    _fields_ = [("choice", (C.c_int * 2) * 2), ("tflops", ((C.c_double * TILE_VARIANTS) * 2) * 2)]


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
        for name in ("feast_solve_d_dev", "feast_solve_z_dev", "feast_solve_d_dev_noalloc"):
            f = getattr(L, name)
            f.argtypes = [C.c_int, vp, C.c_int, vp, C.c_int, C.c_double, C.c_double, ip, op, dp, vp,
                          C.c_int, ip, dp, ip, dp, vp]
        L.feast_contour.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, vp, vp]
        L.feast_rational.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, dp, C.c_int, dp]
        L.feast_rationalx.argtypes = [vp, vp, C.c_int, dp, C.c_int, dp]
        L.feast_last_stats.argtypes = [C.POINTER(feast_stats)]
        L.feast_set_timing.argtypes = [C.c_int]
        L.feast_set_timing.restype = None
        L.feast_release.argtypes = []
        L.feast_release.restype = None
        L.feast_autotune.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(feast_tiles)]
        L.feast_get_tiles.argtypes = [C.POINTER(feast_tiles)]
        L.feast_get_tiles.restype = None
        L.feast_set_tiles.argtypes = [C.POINTER(feast_tiles)]
        L.feast_lu_schedule.argtypes = [C.c_int, C.c_int, C.c_int, ip, C.c_int]
        L.feast_set_lu_form.argtypes = [C.c_int]
        L.feast_get_lu_form.argtypes = []
        L.feast_version.restype = C.c_char_p
        for name in ("feast_solve_batched_d", "feast_solve_batched_z"):
            f = getattr(L, name)
            f.argtypes = [C.c_int, C.POINTER(feast_job), op, C.c_int, C.c_int]
        for f in (L.feast_gsolve_d, L.feast_gsolve_z):
            f.argtypes = [C.c_int, vp, C.c_int, vp, C.c_int, feast_z, C.c_double, ip, op, vp, vp, C.c_int, ip,
                          dp, ip, dp]
        L.feast_gsolve_z_dev.argtypes = [C.c_int, vp, C.c_int, vp, C.c_int, feast_z, C.c_double, ip, op, vp, vp,
                                         C.c_int, ip, dp, ip, dp, vp]
        for f in (L.feast_solve_slices_d, L.feast_solve_slices_z):
            f.argtypes = [C.c_int, vp, C.c_int, vp, C.c_int, C.c_int, dp, C.POINTER(feast_job), op, C.c_int,
                          C.c_int, C.c_int]
        L.feast_server_create.argtypes = [C.POINTER(feast_server_cfg)]
        L.feast_server_create.restype = C.c_void_p
        L.feast_server_submit.argtypes = [C.c_void_p, C.POINTER(feast_request),
                                          C.POINTER(C.c_ulonglong)]
        L.feast_server_poll.argtypes = [C.c_void_p, C.c_ulonglong, C.POINTER(feast_result)]
        L.feast_server_wait.argtypes = [C.c_void_p, C.c_ulonglong, C.POINTER(feast_result)]
        L.feast_server_destroy.argtypes = [C.c_void_p]
        L.feast_server_destroy.restype = None
        _lib = L
    return _lib


def default_opts() -> feast_opts:
    o = feast_opts()
    lib().feast_default_opts(C.byref(o))
    return o


def _zarray(v):
    v = np.asarray(v, dtype=np.complex128).ravel()
    a = (feast_z * v.size)()
    for i, x in enumerate(v):
        a[i].re, a[i].im = float(x.real), float(x.imag)
    return a


def make_opts(ne=8, tol=1e-12, maxloop=20, conv=1, x0=None, keep_factors=1, precision="fp64",
              refine=0, mode=0, verbose=0, seed=None, integration=0, ellipse=100, zne=None,
              wne=None) -> feast_opts:
    """Options (Table "tab_fpm"): integration = fpm(16) (0 Gauss-Legendre, 1
    trapezoidal), ellipse = fpm(18) (percent), zne/wne = custom half-contour
    nodes and weights (expert mode; ne is then their length)."""
    o = default_opts()
    o.ne, o.tol, o.maxloop, o.conv = ne, tol, maxloop, conv
    o.keep_factors, o.refine, o.mode, o.verbose = keep_factors, refine, mode, verbose
    o.precision = {"fp64": 0, "mixed": 1}[precision] if isinstance(precision, str) else precision
    o.integration, o.ellipse = integration, ellipse
    if x0 is not None:
        o.x0 = int(bool(x0))
    if seed is not None:
        o.seed = seed
    if (zne is None) != (wne is None):
        raise ValueError("zne and wne go together")
    if zne is not None:
        za, wa = _zarray(zne), _zarray(wne)
        if len(za) != len(wa):
            raise ValueError("zne and wne differ in length")
        o.ne = len(za)
        o._keep = (za, wa)   # the arrays must outlive the call
        o.Zne, o.Wne = C.addressof(za), C.addressof(wa)
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
    k = m0c.value if info not in (4, 5) else m0
    return Result(info, E[:k].copy(), X[:, :k].copy(order="F"), res[:k].copy(), M.value, k,
                  loop.value, eps.value)


def fortran_tensor(arr, device="cuda"):
    """A torch tensor on `device` holding `arr` column-major (strides (1, N))."""
    import torch

    a = np.asarray(arr)
    t = torch.from_numpy(np.ascontiguousarray(a.T)).to(device)
    return t.t()


def _check_device_operands(A, B, X, xcols, dtypes):
    """Validate torch operands before their raw pointers reach a *_dev entry
    point, which cannot check them: A square, B (or None) the same shape, X
    with N rows and at least `xcols` columns, one dtype from `dtypes` shared
    by all, column-major with leading dimension >= N, all on one CUDA device.
    Raises ValueError; the shape and dtype checks come first, so they fire on
    CPU tensors as well."""
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError(f"A must be square (N, N), got {tuple(A.shape)}")
    n = A.shape[0]
    if A.dtype not in dtypes:
        raise ValueError(f"A has dtype {A.dtype}; expected one of {sorted(str(d) for d in dtypes)}")
    if B is not None:
        if tuple(B.shape) != (n, n):
            raise ValueError(f"B must be ({n}, {n}) like A, got {tuple(B.shape)}")
        if B.dtype != A.dtype:
            raise ValueError(f"B has dtype {B.dtype}, A has {A.dtype}")
    if X is not None:
        if X.dim() != 2 or X.shape[0] != n or X.shape[1] < xcols:
            raise ValueError(f"X must be ({n}, >= {xcols}), got {tuple(X.shape)}")
        if X.dtype != A.dtype:
            raise ValueError(f"X has dtype {X.dtype}, A has {A.dtype}")
    for name, t in (("A", A), ("B", B), ("X", X)):
        if t is None:
            continue
        if t.stride(0) != 1 or t.stride(1) < n:
            raise ValueError(f"{name} must be column-major with leading dimension >= {n} "
                             f"(strides {tuple(t.stride())})")
        if not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA tensor")
        if t.device != A.device:
            raise ValueError(f"{name} is on {t.device}, A on {A.device}")


def solve_device(A, B, emin, emax, m0, X, stream=None, noalloc=False, **kw) -> Result:
    """Device solve: A, B, X are column-major torch CUDA tensors (see
    fortran_tensor); X holds the start subspace if x0=True and receives the
    eigenvectors.  Runs on `stream` (default: torch's current stream).
    noalloc=True calls feast_solve_d_dev_noalloc (real pencils only), whose
    device workspace is the library's fixed scratch array."""
    import torch

    _check_device_operands(A, B, X, m0, (torch.float64,) if noalloc else (torch.float64, torch.complex128))
    cplx = A.is_complex()
    n = A.shape[0]
    if stream is None:
        stream = torch.cuda.current_stream()
    o = make_opts(**kw)
    E = np.zeros(m0)
    res = np.zeros(m0)
    M = C.c_int(0)
    loop = C.c_int(0)
    eps = C.c_double(0)
    m0c = C.c_int(m0)
    if noalloc:
        f = lib().feast_solve_d_dev_noalloc
    else:
        f = lib().feast_solve_z_dev if cplx else lib().feast_solve_d_dev
    info = f(n, A.data_ptr(), A.stride(1), None if B is None else B.data_ptr(),
             n if B is None else B.stride(1), float(emin), float(emax), C.byref(m0c), C.byref(o),
             _dp(E), X.data_ptr(), X.stride(1), C.byref(M), _dp(res), C.byref(loop),
             C.byref(eps), C.c_void_p(stream.cuda_stream))
    k = m0c.value if info not in (4, 5) else m0
    return Result(info, E[:k].copy(), X[:, :k], res[:k].copy(), M.value, k, loop.value, eps.value)


def contour(emin, emax, ne, integration=0, ellipse=100):
    """Tool "[cz]feast_contour": half-contour nodes and weights."""
    z = (feast_z * ne)()
    w = (feast_z * ne)()
    info = lib().feast_contour(emin, emax, ne, integration, ellipse, z, w)
    if info:
        raise ValueError(f"feast_contour info {info}")
    return (np.array([v.re + 1j * v.im for v in z]), np.array([v.re + 1j * v.im for v in w]))


def rational(emin, emax, ne, lam, integration=0, ellipse=100):
    """Tool "[sd]feast_rational": the filter at the points lam."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    f = np.zeros(lam.size)
    info = lib().feast_rational(emin, emax, ne, integration, ellipse, _dp(lam), lam.size, _dp(f))
    if info:
        raise ValueError(f"feast_rational info {info}")
    return f


def rationalx(zne, wne, lam):
    """Tool "[sd]feast_rationalx": the filter of custom nodes and weights."""
    za, wa = _zarray(zne), _zarray(wne)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    f = np.zeros(lam.size)
    info = lib().feast_rationalx(za, wa, len(za), _dp(lam), lam.size, _dp(f))
    if info:
        raise ValueError(f"feast_rationalx info {info}")
    return f


def stats() -> feast_stats:
    s = feast_stats()
    lib().feast_last_stats(C.byref(s))
    return s


def set_timing(on: bool):
    lib().feast_set_timing(int(bool(on)))


def release():
    lib().feast_release()


_PRECISIONS = ("complex64", "complex128")
_CLASSES = ("depth<=64", "deeper")


def _tiles_dict(t: feast_tiles) -> dict:
    return {"choice": {p: {c: t.choice[i][j] for j, c in enumerate(_CLASSES)} for i, p in enumerate(_PRECISIONS)},
            "tflops": {p: {c: [round(t.tflops[i][j][v], 2) for v in range(TILE_VARIANTS)]
                           for j, c in enumerate(_CLASSES)} for i, p in enumerate(_PRECISIONS)}}


def autotune(n: int, m0: int, ne: int) -> dict:
    """feast_autotune: time the product kernel's tile variants on this
    device for a solve of order n, m0 columns, ne nodes, install the fastest
    and return {"choice": {precision: {class: variant}}, "tflops": ...}."""
    t = feast_tiles()
    info = lib().feast_autotune(int(n), int(m0), int(ne), C.byref(t))
    if info != 0:
        raise RuntimeError(f"feast_autotune: {info}")
    return _tiles_dict(t)


def tiles() -> dict:
    """The installed tile table (choices)."""
    t = feast_tiles()
    lib().feast_get_tiles(C.byref(t))
    return _tiles_dict(t)["choice"]


LU_OP_INTS = 12
LU_OP_FIELDS = ("kind", "side", "k", "nbw", "c0", "c1", "c2", "c3", "kc0", "kc1", "mode", "list")


LU_FORMS = {"auto": -1, "pairs": 0, "blocks": 1}


def lu_schedule(n: int, side: bool, form: str = "auto") -> np.ndarray:
    """feast_lu_schedule: the factorisation's launch steps for order n, one
    row of LU_OP_FIELDS per step (host logic only, no device call).  form:
    "auto" (what the library runs), "pairs" or "blocks"."""
    f = LU_FORMS[form]
    cnt = lib().feast_lu_schedule(int(n), int(bool(side)), f, None, 0)
    if cnt < 0:
        raise ValueError(f"feast_lu_schedule: {cnt}")
    ops = np.zeros((cnt, LU_OP_INTS), dtype=np.int32)
    got = lib().feast_lu_schedule(int(n), int(bool(side)), f, ops.ctypes.data_as(C.POINTER(C.c_int)), cnt)
    assert got == cnt
    return ops


def set_lu_form(form: str) -> None:
    """feast_set_lu_form: the factorisation schedule of later solves
    ("auto", "pairs" or "blocks")."""
    if lib().feast_set_lu_form(LU_FORMS[form]) != 0:
        raise ValueError(f"feast_set_lu_form: {form}")


def lu_form() -> str:
    """The current factorisation schedule setting."""
    v = lib().feast_get_lu_form()
    return next(k for k, f in LU_FORMS.items() if f == v)


def set_tiles(choice: dict) -> None:
    """Install a table {precision: {class: variant}} as returned by tiles()."""
    t = feast_tiles()
    for i, p in enumerate(_PRECISIONS):
        for j, c in enumerate(_CLASSES):
            t.choice[i][j] = int(choice[p][c])
    info = lib().feast_set_tiles(C.byref(t))
    if info != 0:
        raise ValueError(f"feast_set_tiles: {info}")


def solve_batched(problems, concurrency=4, **kw) -> list[Result]:
    """Solve many independent problems in one call (host arrays).  `problems`
    is a list of (A, B, emin, emax, m0, X0) tuples of one kind (all real or
    all complex); X0 may be None only if every X0 is None."""
    if not problems:
        return []
    cplx = any(np.iscomplexobj(p[0]) or (p[1] is not None and np.iscomplexobj(p[1])) for p in problems)
    dt = np.complex128 if cplx else np.float64
    x0 = problems[0][5] is not None
    o = make_opts(x0=x0, **kw)
    keep, jobs = [], (feast_job * len(problems))()
    for i, (A, B, emin, emax, m0, X0) in enumerate(problems):
        A = np.asfortranarray(A, dtype=dt)
        n = A.shape[0]
        Bf = None if B is None else np.asfortranarray(B, dtype=dt)
        X = np.zeros((n, m0), dtype=dt, order="F")
        if X0 is not None:
            X[:, :] = X0
        E = np.zeros(m0)
        res = np.zeros(m0)
        keep.append((A, Bf, X, E, res))
        j = jobs[i]
        j.n, j.A, j.lda = n, A.ctypes.data, n
        j.B, j.ldb = (None if Bf is None else Bf.ctypes.data), n
        j.emin, j.emax, j.m0 = float(emin), float(emax), m0
        j.X, j.ldx, j.E, j.res = X.ctypes.data, n, E.ctypes.data, res.ctypes.data
    f = lib().feast_solve_batched_z if cplx else lib().feast_solve_batched_d
    rc = f(len(problems), jobs, C.byref(o), 0, concurrency)
    if rc:
        raise ValueError(f"feast_solve_batched: {rc}")
    out = []
    for (A, Bf, X, E, res), j in zip(keep, jobs):
        k = j.m0_out if j.info not in (4, 5) else j.m0
        r = Result(j.info, E[:k].copy(), X[:, :k].copy(order="F"), res[:k].copy(), j.M, k, j.loop,
                   j.epsout)
        r.ms = j.ms
        out.append(r)
    return out


def gsolve(A, B, emid, r, m0, X0=None, **kw) -> Result:
    """Non-Hermitian FEAST (host arrays): A, B general real or complex (B may
    be None); the search region is the ellipse centred at emid (complex) with
    horizontal semi-axis r.  X0: optional (N, 2 M0) start subspaces (right,
    then left).  Options as in make_opts plus ne_full (fpm(8)),
    integration_full (fpm(17)) and angle (fpm(19)).  Returns E complex (M0),
    X (N, 2 M0) with right then left eigenvectors, res (2 M0)."""
    ne_full = kw.pop("ne_full", 16)
    integration_full = kw.pop("integration_full", 1)
    angle = kw.pop("angle", 0)
    real = not (np.iscomplexobj(A) or (B is not None and np.iscomplexobj(B)))
    dt = np.float64 if real else np.complex128
    A = np.asfortranarray(A, dtype=dt)
    n = A.shape[0]
    Bf = None if B is None else np.asfortranarray(B, dtype=dt)
    o = make_opts(x0=X0 is not None, **kw)
    o.ne_full, o.integration_full, o.angle = ne_full, integration_full, angle
    X = np.zeros((n, 2 * m0), dtype=np.complex128, order="F")
    if X0 is not None:
        X[:, :] = X0
    E = np.zeros(m0, dtype=np.complex128)
    res = np.zeros(2 * m0)
    M, loop, eps, m0c = C.c_int(0), C.c_int(0), C.c_double(0), C.c_int(m0)
    z = feast_z(float(np.real(emid)), float(np.imag(emid)))
    f = lib().feast_gsolve_d if real else lib().feast_gsolve_z
    info = f(n, A.ctypes.data, n, None if Bf is None else Bf.ctypes.data, n, z, float(r), C.byref(m0c),
             C.byref(o), E.ctypes.data, X.ctypes.data, n, C.byref(M), _dp(res), C.byref(loop), C.byref(eps))
    return Result(info, E, X, res, M.value, m0, loop.value, eps.value)


def gsolve_device(A, B, emid, r, m0, X, stream=None, **kw) -> Result:
    """Non-Hermitian FEAST on device arrays: A, B (or None), X complex128
    column-major torch CUDA tensors (see fortran_tensor), X of shape (N, 2 M0)
    holding the start subspaces if x0=True and receiving right then left
    eigenvectors.  Options as in gsolve."""
    import torch

    ne_full = kw.pop("ne_full", 16)
    integration_full = kw.pop("integration_full", 1)
    angle = kw.pop("angle", 0)
    _check_device_operands(A, B, X, 2 * m0, (torch.complex128,))
    n = A.shape[0]
    if stream is None:
        stream = torch.cuda.current_stream()
    o = make_opts(**kw)
    o.ne_full, o.integration_full, o.angle = ne_full, integration_full, angle
    E = np.zeros(m0, dtype=np.complex128)
    res = np.zeros(2 * m0)
    M, loop, eps, m0c = C.c_int(0), C.c_int(0), C.c_double(0), C.c_int(m0)
    z = feast_z(float(np.real(emid)), float(np.imag(emid)))
    info = lib().feast_gsolve_z_dev(n, A.data_ptr(), A.stride(1), None if B is None else B.data_ptr(),
                                    n if B is None else B.stride(1), z, float(r), C.byref(m0c), C.byref(o),
                                    E.ctypes.data, X.data_ptr(), X.stride(1), C.byref(M), _dp(res), C.byref(loop),
                                    C.byref(eps), C.c_void_p(stream.cuda_stream))
    return Result(info, E, X, res, M.value, m0, loop.value, eps.value)


def solve_slices(A, B, bounds, m0, X0=None, concurrency=4, auto_m0=False, **kw) -> list[Result]:
    """Spectrum slicing: the neighbouring intervals [bounds[s], bounds[s+1]] of
    one pencil as one batched job sharing A and B on the device.  A, B: numpy
    arrays (staged by the library), or column-major torch CUDA tensors (see
    fortran_tensor; each slice's X is then a device tensor too).  m0: one
    subspace size for every slice or a list (with auto_m0, the most each slice
    may use); X0: None or a list of start subspaces, one per slice."""
    device = hasattr(A, "is_cuda")
    if device:
        import torch

        _check_device_operands(A, B, None, 0, (torch.float64, torch.complex128))
        cplx = A.is_complex()
        n = A.shape[0]
        pa = A.data_ptr()
        pb = None if B is None else B.data_ptr()
        lda, ldb = A.stride(1), (n if B is None else B.stride(1))
        torch.cuda.synchronize()
    else:
        cplx = np.iscomplexobj(A) or (B is not None and np.iscomplexobj(B))
        dt = np.complex128 if cplx else np.float64
        A = np.asfortranarray(A, dtype=dt)
        n = A.shape[0]
        B = None if B is None else np.asfortranarray(B, dtype=dt)
        pa, pb, lda, ldb = A.ctypes.data, (None if B is None else B.ctypes.data), n, n
    b = np.ascontiguousarray(bounds, dtype=np.float64)
    ns = b.size - 1
    m0s = [int(m0)] * ns if np.isscalar(m0) else [int(x) for x in m0]
    if len(m0s) != ns:
        raise ValueError("one m0 per slice")
    if X0 is not None:
        if len(X0) != ns:
            raise ValueError("one start subspace per slice")
        for s_, (x, mm) in enumerate(zip(X0, m0s)):
            if tuple(x.shape) != (n, mm):
                raise ValueError(f"X0[{s_}] has shape {tuple(x.shape)}, expected ({n}, {mm})")
    o = make_opts(x0=X0 is not None and not auto_m0, **kw)
    keep, jobs = [], (feast_job * ns)()
    for s_, mm in enumerate(m0s):
        if device:
            X = torch.zeros((mm, n), dtype=A.dtype, device=A.device).t()
            if X0 is not None:
                X.copy_(X0[s_])
            px = X.data_ptr()
        else:
            X = np.zeros((n, mm), dtype=dt, order="F")
            if X0 is not None:
                X[:, :] = X0[s_]
            px = X.ctypes.data
        E, res = np.zeros(mm), np.zeros(mm)
        keep.append((X, E, res))
        j = jobs[s_]
        j.m0, j.X, j.ldx, j.E, j.res = mm, px, n, E.ctypes.data, res.ctypes.data
    if device:
        torch.cuda.synchronize()
    f = lib().feast_solve_slices_z if cplx else lib().feast_solve_slices_d
    rc = f(n, pa, lda, pb, ldb, ns, _dp(b), jobs, C.byref(o), int(device), concurrency, int(bool(auto_m0)))
    if rc:
        raise ValueError(f"feast_solve_slices: {rc}")
    out = []
    for (X, E, res), j in zip(keep, jobs):
        k = j.m0_out if j.info in (0, 1, 2, 3) else 0
        Xk = X[:, :k] if device else X[:, :k].copy(order="F")
        r = Result(j.info, E[:k].copy(), Xk, res[:k].copy(), j.M, k, j.loop, j.epsout)
        r.ms = j.ms
        r.emin, r.emax = j.emin, j.emax
        out.append(r)
    return out


class Server:
    """The library's request loop: submit() returns an id, wait()/poll()
    return a Result with queue/run/latency times in milliseconds."""

    def __init__(self, slots=4, hbm_budget_gb=64.0):
        cfg = feast_server_cfg(slots, hbm_budget_gb)
        self._h = lib().feast_server_create(C.byref(cfg))
        if not self._h:
            raise RuntimeError("feast_server_create failed")
        self._keep = {}

    def submit(self, A, B, emin, emax, m0, X0=None, **kw):
        cplx = np.iscomplexobj(A) or (B is not None and np.iscomplexobj(B))
        dt = np.complex128 if cplx else np.float64
        A = np.asfortranarray(A, dtype=dt)
        n = A.shape[0]
        Bf = None if B is None else np.asfortranarray(B, dtype=dt)
        X0f = None if X0 is None else np.asfortranarray(X0, dtype=dt)
        req = feast_request()
        req.hermitian, req.n, req.A, req.lda = int(cplx), n, A.ctypes.data, n
        req.B, req.ldb = (None if Bf is None else Bf.ctypes.data), n
        req.emin, req.emax, req.m0 = float(emin), float(emax), m0
        req.X0, req.ldx = (None if X0f is None else X0f.ctypes.data), n
        req.opts = make_opts(**kw)
        rid = C.c_ulonglong(0)
        rc = lib().feast_server_submit(self._h, C.byref(req), C.byref(rid))
        if rc:
            raise ValueError(f"feast_server_submit: {rc}")
        self._keep[rid.value] = (A, Bf, X0f, n, m0, dt)
        return rid.value

    def _take(self, rid, block):
        A, Bf, X0f, n, m0, dt = self._keep[rid]
        E = np.zeros(m0)
        res = np.zeros(m0)
        X = np.zeros((n, m0), dtype=dt, order="F")
        out = feast_result()
        out.E, out.res, out.X, out.ldx = E.ctypes.data, res.ctypes.data, X.ctypes.data, n
        f = lib().feast_server_wait if block else lib().feast_server_poll
        rc = f(self._h, rid, C.byref(out))
        if rc == 1:
            return None
        if rc:
            raise ValueError(f"feast_server: {rc}")
        del self._keep[rid]
        k = out.m0
        r = Result(out.info, E[:k].copy(), X[:, :k].copy(order="F"), res[:k].copy(), out.M, k,
                   out.loop, out.epsout)
        r.queue_ms, r.run_ms, r.latency_ms = out.queue_ms, out.run_ms, out.latency_ms
        return r

    def wait(self, rid):
        return self._take(rid, True)

    def poll(self, rid):
        return self._take(rid, False)

    def close(self):
        if self._h:
            lib().feast_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
