"""FP64 CPU oracle for non-Hermitian FEAST (dense, real non-symmetric or
complex general pencils).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this; the GPU library never does.

The guide gives the non-Hermitian variant in outline (section "FEAST v3.0",
the list of changes: dual subspaces Q and Q-hat for right and left
eigenvectors, a two-dimensional search region; Table "tab_fpm" fpm(8),
fpm(17), fpm(18), fpm(19); Table "tab_common" for E, X, res and alpha) and
defers the mathematics to Kestyn, Polizzi and Tang (2015).  This module
follows those steps in order, with numpy and scipy routines as the
primitives (LU factorisation and solves, the matrix product, the QZ
eigensolver of the small reduced pencil):

  right:  Q  = sum_j  w_j       (z_j B - A)^{-1}   B   X
  left:   Qh = sum_j  conj(w_j) (z_j B - A)^{-H}   B^H Xh
  reduced pencil  Aq = Qh^H A Q,  Bq = Qh^H B Q
  Aq W = Bq W Lambda,  Wh^H Aq = Lambda Wh^H Bq
  X = Q W,  Xh = Qh Wh  (columns scaled to unit 2-norm)

The readings taken where the guide is silent are stated beside each
function.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sl

SPURIOUS_RES = 0.1


def contour(emid: complex, r: float, ne: int, integration: int = 1, ellipse: int = 100,
            angle: float = 0.0):
    """Nodes z_j and weights w_j of the full contour (fpm(8) nodes).

    The contour is z(t) = c + e^{i phi} (r cos t + i a r sin t), t in
    [0, 2 pi), with c = Emid, a = fpm(18)/100 and phi = fpm(19) degrees
    (reading: the angle turns the ellipse counter-clockwise about its centre;
    at 0 its second axis is the vertical one).  With step dt_j, the weight of
    dz / (2 pi i) at t_j is w_j = (dt_j / 2 pi) e^{i phi} (a r cos t_j +
    i r sin t_j).
    Trapezoidal (fpm(17) = 1, the default): t_j = 2 pi (j + 1/2) / ne, equal
    steps.  Gauss (fpm(17) = 0): one ne-point Gauss-Legendre rule over
    [0, 2 pi] (reading: the guide does not say how the nodes are split).
    Returns complex arrays (z, w) of length ne, in increasing t."""
    if ne < 1:
        raise ValueError("ne >= 1")
    if integration == 1:
        t = 2.0 * math.pi * (np.arange(ne) + 0.5) / ne
        dt = np.full(ne, 2.0 * math.pi / ne)
    elif integration == 0:
        x, om = np.polynomial.legendre.leggauss(ne)
        t = math.pi * (1.0 + x)
        dt = math.pi * om
    else:
        raise ValueError("integration is 0 or 1")
    a = ellipse / 100.0
    rot = np.exp(1j * math.radians(angle))
    z = emid + rot * (r * np.cos(t) + 1j * a * r * np.sin(t))
    w = (dt / (2.0 * math.pi)) * rot * (a * r * np.cos(t) + 1j * r * np.sin(t))
    return z, w


def rational(emid, r, ne, lam, integration=1, ellipse=100, angle=0.0):
    """The filter rho(lambda) = sum_j w_j / (z_j - lambda) of the full
    contour: about 1 inside, about 0 outside (complex in general)."""
    z, w = contour(emid, r, ne, integration, ellipse, angle)
    lam = np.asarray(lam, dtype=np.complex128)
    return (w[None, :] / (z[None, :] - lam.reshape(-1, 1))).sum(axis=1).reshape(lam.shape)


def inside(emid, r, lam, ellipse=100, angle=0.0):
    """Whether lambda lies in the closed search region bounded by the
    contour."""
    a = ellipse / 100.0
    u = (np.asarray(lam, dtype=np.complex128) - emid) * np.exp(-1j * math.radians(angle))
    return (u.real / r) ** 2 + (u.imag / (a * r)) ** 2 <= 1.0


@dataclass
class Result:
    info: int
    E: np.ndarray      # complex, m0
    X: np.ndarray      # complex, n x 2 m0: right vectors, then left vectors
    res: np.ndarray    # 2 m0: right residuals, then left residuals
    M: int
    loop: int
    epsout: float


def _order(lam):
    """Reading: eigenvalues are listed by increasing real part, then
    increasing imaginary part."""
    return np.lexsort((lam.imag, lam.real))


def feast(A, B, emid, r, m0, ne, tol, X0, maxloop=20, conv=1, integration=1, ellipse=100,
          angle=0.0) -> Result:
    """Non-Hermitian FEAST on the dense pencil (A, B) (B = None: identity).

    X0 (n x 2 m0) holds the right start subspace, then the left one.
    alpha = |Emid| + r (Table "tab_common").  Right residual
    ||A x - lambda B x||_1 / (alpha ||B x||_1), left residual
    ||A^H xh - conj(lambda) B^H xh||_1 / (alpha ||B^H xh||_1).  A Ritz pair
    inside the region counts when both residuals are below 0.1 from loop 1 on
    (the Hermitian spurious rule, applied to both sides); convergence
    (fpm(6) = 1) needs both residuals of every counted pair below tol; with
    fpm(6) = 0 the relative change of the trace sum of counted lambda,
    divided by alpha, is below tol.  info: 0, 1 (nothing inside at loop 0),
    2 (maxloop reached), 3 (M0 too small: M >= M0 before convergence),
    202 / 201 / 108 / 103 / 104 / 106 / 117 / 118 / 119 / 200 argument errors, -2 a
    shifted matrix is singular, -3 the reduced pencil is singular."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    if n < 1:
        return Result(202, None, None, None, 0, 0, 1.0)
    if m0 < 1 or m0 > n:
        return Result(201, None, None, None, 0, 0, 1.0)
    if ne < 1:
        return Result(108, None, None, None, 0, 0, 1.0)
    if not tol > 0:
        return Result(103, None, None, None, 0, 0, 1.0)
    if maxloop < 0:
        return Result(104, None, None, None, 0, 0, 1.0)
    if conv not in (0, 1):
        return Result(106, None, None, None, 0, 0, 1.0)
    if integration not in (0, 1):
        return Result(117, None, None, None, 0, 0, 1.0)
    if ellipse < 1:
        return Result(118, None, None, None, 0, 0, 1.0)
    if not -180 <= angle <= 180:
        return Result(119, None, None, None, 0, 0, 1.0)
    if not r > 0:
        return Result(200, None, None, None, 0, 0, 1.0)
    Bm = np.eye(n, dtype=np.complex128) if B is None else np.asarray(B, dtype=np.complex128)
    alpha = abs(emid) + r
    z, w = contour(emid, r, ne, integration, ellipse, angle)
    facs = []
    for zj in z:
        lu, piv = sl.lu_factor(zj * Bm - A, check_finite=False)
        if not np.all(np.isfinite(lu)) or np.any(np.abs(np.diag(lu)) == 0.0):
            return Result(-2, None, None, None, 0, 0, 1.0)
        facs.append((lu, piv))
    X = np.array(X0[:, :m0], dtype=np.complex128)
    Xh = np.array(X0[:, m0:2 * m0], dtype=np.complex128)
    trace_prev, epsout, M = 0.0, 1.0, 0
    for k in range(maxloop + 1):
        # contour step, right and left
        R, Rh = Bm @ X, Bm.conj().T @ Xh
        Q = np.zeros((n, m0), np.complex128)
        Qh = np.zeros((n, m0), np.complex128)
        for (lu, piv), wj in zip(facs, w):
            Q += wj * sl.lu_solve((lu, piv), R, trans=0, check_finite=False)
            Qh += np.conj(wj) * sl.lu_solve((lu, piv), Rh, trans=2, check_finite=False)
        # reduced pencil and its right and left eigenvectors
        Aq = Qh.conj().T @ A @ Q
        Bq = Qh.conj().T @ Bm @ Q
        try:
            lam, Wl, Wr = sl.eig(Aq, Bq, left=True, right=True)
        except sl.LinAlgError:
            return Result(-3, None, None, None, 0, k, 1.0)
        if not np.all(np.isfinite(lam)):
            return Result(-3, None, None, None, 0, k, 1.0)
        X = Q @ Wr
        Xh = Qh @ Wl
        X /= np.linalg.norm(X, axis=0)
        Xh /= np.linalg.norm(Xh, axis=0)
        BX, BhXh = Bm @ X, Bm.conj().T @ Xh
        rr = np.abs(A @ X - BX * lam).sum(0) / (alpha * np.abs(BX).sum(0))
        rl = np.abs(A.conj().T @ Xh - BhXh * np.conj(lam)).sum(0) / (alpha * np.abs(BhXh).sum(0))
        ins = inside(emid, r, lam, ellipse, angle)
        spur = ins & (k >= 1) & (np.maximum(rr, rl) > SPURIOUS_RES)
        cnt = ins & ~spur
        M = int(cnt.sum())
        if k == 0 and M == 0:
            info = 1
            break
        trace = lam[cnt].sum()
        epsout = 1.0 if k == 0 else abs(trace - trace_prev) / alpha
        trace_prev = trace
        if conv == 1:
            done = M > 0 and max(rr[cnt].max(), rl[cnt].max()) < tol
        else:
            done = k > 0 and epsout < tol
        if done:
            info = 0
            break
        if M >= m0:
            info = 3
            break
        if k == maxloop:
            info = 2
            break
    # output order: counted pairs, then the others outside, then spurious
    o_in = [i for i in _order(lam) if cnt[i]]
    o_out = [i for i in _order(lam) if not ins[i]]
    o_sp = [i for i in _order(lam) if spur[i]]
    order = np.array(o_in + o_out + o_sp, dtype=int)
    res = np.concatenate([rr[order], rl[order]])
    nsp = len(o_sp)
    if nsp:
        res[m0 - nsp:m0] = -1.0
        res[2 * m0 - nsp:] = -1.0
    Xout = np.concatenate([X[:, order], Xh[:, order]], axis=1)
    return Result(info, lam[order], Xout, res, M, k, float(epsout))
