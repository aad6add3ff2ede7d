"""Pins for the FP64 CPU oracle: each test checks the oracle against something
other than itself -- closed forms, exact identities of the quadrature, values
printed in the FEAST guide, textbook/library routines, brute force and
inertia counts -- so that a dropped term, a wrong sign or index, or a
transposed operand anywhere in it fails at least one of them."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl

from paper_1203_4031_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
U = np.finfo(np.float64).eps


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n,xs,ws", [
    (1, [0.0], [2.0]),
    (2, [-1 / math.sqrt(3), 1 / math.sqrt(3)], [1.0, 1.0]),
    (3, [-math.sqrt(0.6), 0.0, math.sqrt(0.6)], [5 / 9, 8 / 9, 5 / 9]),
])
def test_gauss_legendre_closed_forms(orc, n, xs, ws):
    x, w = orc.gauss_legendre(n)
    assert np.allclose(x, xs, atol=4 * U, rtol=0)
    assert np.allclose(w, ws, atol=4 * U, rtol=0)


@pytest.mark.parametrize("n", [1, 2, 4, 5, 8, 16, 20, 24, 32, 56])
def test_gauss_legendre_exact_on_polynomials(orc, n):
    x, w = orc.gauss_legendre(n)
    assert abs(w.sum() - 2.0) < 8 * U
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 50 * U, k
    # third-party cross-check
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.abs(x - xr).max() < 8 * U
    assert np.abs(w - wr).max() < 50 * U


@pytest.mark.parametrize("ne", [1, 2, 3, 8, 16])
def test_contour_geometry(orc, ne):
    emin, emax = -0.3, 1.7
    z, w = orc.contour(emin, emax, ne)
    c, r = 0.5 * (emin + emax), 0.5 * (emax - emin)
    assert np.allclose(np.abs(z - c), r, rtol=0, atol=8 * U)
    assert (z.imag > 0).all()                       # upper half only
    x, om = orc.gauss_legendre(ne)
    # |w_j| = omega_j r / 2 and w_j is parallel to z_j - c
    assert np.allclose(np.abs(w), 0.5 * om * r, rtol=0, atol=8 * U)
    assert np.allclose(w / np.abs(w), (z - c) / r, atol=8 * U)


@pytest.mark.parametrize("ne", [1, 2, 3, 8, 16])
def test_filter_identities(orc, ne):
    """rho(c) = 1, rho(Emin) = rho(Emax) = 1/2, rho(c + t r) = rho(c - t r):
    exact for the half-contour Gauss rule with the 1/2 weight factor."""
    emin, emax = 2.0, 5.0
    c, r = 3.5, 1.5
    f = orc.rational(emin, emax, ne, [c, emin, emax])
    assert abs(f[0] - 1) < 16 * U
    # near theta = 0 or pi the denominator e^{i theta} + 1 cancels: allow 32 u
    assert abs(f[1] - 0.5) < 32 * U and abs(f[2] - 0.5) < 32 * U
    t = np.array([0.1, 0.5, 0.9, 1.1, 1.5, 3.0, 10.0])
    assert np.allclose(orc.rational(emin, emax, ne, c + t * r),
                       orc.rational(emin, emax, ne, c - t * r), rtol=0, atol=16 * U)


def test_filter_tends_to_indicator(orc):
    """With many nodes the filter approaches the interval's indicator function."""
    f = orc.rational(-1.0, 1.0, 56, [-0.5, 0.0, 0.7, -1.5, 2.0, 4.0])
    assert np.allclose(f[:3], 1.0, atol=1e-12)
    assert np.allclose(f[3:], 0.0, atol=1e-12)


def test_filter_is_the_contour_integral(orc):
    """rho(lambda) equals (1/2 pi i) times the closed contour integral of
    1/(z - lambda), evaluated independently with a fine trapezoid rule on
    the full circle (1 inside, 0 outside) -- in the limit of many nodes."""
    emin, emax = 0.0, 2.0
    lam = np.array([0.3, 1.2, 2.6, -0.9])
    th = np.linspace(0, 2 * np.pi, 20001)[:-1]
    zz = 1.0 + np.exp(1j * th)
    # dz = i e^{i theta} d theta, so (1/2 pi i) dz/(z - l) = e^{i theta}/(z - l) d theta / 2 pi
    ref = [((zz - 1.0) / (zz - l)).mean().real for l in lam]
    assert np.allclose(orc.rational(emin, emax, 48, lam), ref, atol=1e-10)


# ------------------------------------------ other rules and contours (fpm(16), fpm(18))
@pytest.mark.parametrize("ne", [1, 2, 3, 5, 8, 16])
def test_trapezoidal_circle_closed_form(orc, ne):
    """Equally spaced midpoint nodes on the circle give the rational filter
    1 / (1 + t^(2 ne)), t = (lambda - c)/r, in closed form (sum of the
    partial fractions of 1/(1 + s^(2 ne)) over its 2 ne roots)."""
    emin, emax = -0.4, 2.6
    c, r = 1.1, 1.5
    t = np.array([0.0, 0.3, -0.3, 0.9, -0.9, 1.0, -1.0, 1.2, -1.7, 3.0])
    ref = 1.0 / (1.0 + t ** (2 * ne))
    assert np.allclose(orc.rational(emin, emax, ne, c + t * r, integration=1), ref, rtol=0, atol=64 * U)


@pytest.mark.parametrize("integration", [0, 1])
@pytest.mark.parametrize("ratio", [50, 200])
def test_ellipse_geometry(orc, integration, ratio):
    """Nodes on the upper half of the ellipse through Emin and Emax with
    vertical semi-axis a r, and each weight along the contour's outward
    normal i.e. -i times the tangent direction (the orientation dz/(2 pi i))."""
    emin, emax, ne = -0.3, 1.7, 9
    z, w = orc.contour(emin, emax, ne, integration, ratio)
    c, r, a = 0.5 * (emin + emax), 0.5 * (emax - emin), ratio / 100.0
    assert np.allclose(((z.real - c) / r) ** 2 + (z.imag / (a * r)) ** 2, 1.0, atol=16 * U)
    assert (z.imag > 0).all() and (np.diff(z.real) > 0).all()
    th = np.arctan2(z.imag / a, z.real - c)                 # the parameter of each node
    tangent = -r * np.sin(th) + 1j * a * r * np.cos(th)
    cosang = (w * np.conj(-1j * tangent)).real / (np.abs(w) * np.abs(tangent))
    assert np.allclose(cosang, 1.0, atol=1e-12)


@pytest.mark.parametrize("integration,ne", [(0, 56), (1, 400)])
@pytest.mark.parametrize("ratio", [50, 100, 200])
def test_ellipse_filter_is_the_contour_integral(orc, integration, ne, ratio):
    """With many nodes the filter tends to (1 / 2 pi i) times the closed
    contour integral of 1/(z - lambda) around the ellipse, i.e. 1 inside and
    0 outside, computed here on the full ellipse with a fine independent rule."""
    emin, emax = 0.0, 2.0
    c, r, a = 1.0, 1.0, ratio / 100.0
    lam = np.array([0.4, 1.0, 1.5, -1.0, 3.2, 5.0])
    th = np.linspace(0, 2 * np.pi, 40001)[:-1]
    zz = c + r * np.cos(th) + 1j * a * r * np.sin(th)
    dz = -r * np.sin(th) + 1j * a * r * np.cos(th)
    # (1 / 2 pi i) int dz/(z - l) = mean over theta of dz/dtheta / (i (z - l))
    ref = np.array([(dz / (1j * (zz - l))).mean().real for l in lam])
    assert np.allclose(ref, [1, 1, 1, 0, 0, 0], atol=1e-9)
    f = orc.rational(emin, emax, ne, lam, integration=integration, ellipse=ratio)
    assert np.allclose(f, ref, atol=1e-8)


@pytest.mark.parametrize("integration,ratio", [(1, 100), (0, 50), (1, 200)])
def test_other_contours_find_the_same_eigenpairs(orc, integration, ratio):
    """The contour only changes the filter, not the answer: FEAST with the
    trapezoidal rule or an ellipse finds the brute-force eigenvalues of a
    small pencil, with residuals below tol."""
    p = W.dense_real_generalized(40, count=7, seed=151, tol=1e-12)
    r = orc.feast(p.A, p.B, p.emin, p.emax, p.m0, 12, p.tol, p.X0, integration=integration,
                  ellipse=ratio)
    assert r.info == 0
    allev = sl.eigh(p.A, p.B, eigvals_only=True)
    inside = allev[(allev >= p.emin) & (allev <= p.emax)]
    alpha = max(abs(p.emin), abs(p.emax))
    assert r.M == inside.size
    assert np.abs(r.E[:r.M] - inside).max() < 1e-12 * alpha
    assert (r.res[:r.M] < p.tol).all()


def test_custom_nodes_are_used_as_given(orc):
    """Expert mode: passing the trapezoidal nodes as custom nodes gives the
    trapezoidal run exactly; passing a rule the solver would not pick (an
    ellipse) changes the iterates but not the eigenvalues."""
    p = W.dense_real_generalized(40, count=7, seed=152, tol=1e-12)
    z, w = orc.contour(p.emin, p.emax, 10, 1, 100)
    a = orc.feast(p.A, p.B, p.emin, p.emax, p.m0, 10, p.tol, p.X0, integration=1)
    b = orc.feast(p.A, p.B, p.emin, p.emax, p.m0, 10, p.tol, p.X0, zne=z, wne=w)
    assert a.info == b.info == 0 and a.M == b.M and a.loop == b.loop
    assert np.array_equal(a.E, b.E) and np.array_equal(a.res, b.res)
    z2, w2 = orc.contour(p.emin, p.emax, 10, 0, 60)
    c = orc.feast(p.A, p.B, p.emin, p.emax, p.m0, 10, p.tol, p.X0, zne=z2, wne=w2)
    assert c.info == 0 and c.M == a.M
    assert np.abs(c.E[:c.M] - a.E[:a.M]).max() < 1e-12
    assert np.allclose(orc.rationalx(z, w, [0.1, 7.0]), orc.rational(p.emin, p.emax, 10, [0.1, 7.0], 1), atol=0)


# --------------------------------------------------------- dense linear algebra
def _rand(n, m, seed, cplx=True):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, m))
    if cplx:
        a = a + 1j * rng.standard_normal((n, m))
    return np.asfortranarray(a)


# ------------------------------------------------ stochastic count estimate
def _filter_matrix(A, B, rho):
    """rho(B^{-1} A) = V diag(rho(lambda)) V^H B from the B-orthonormal
    eigenvectors V of the whole pencil (LAPACK through scipy)."""
    lam, V = sl.eigh(A, B)
    return lam, (V * rho(lam)) @ V.conj().T @ B


@pytest.mark.parametrize("herm", [False, True])
@pytest.mark.parametrize("integration,ne", [(1, 4), (0, 8)])
def test_count_estimate_with_identity_probes_is_the_trace(orc, herm, integration, ne):
    """Probes e_1..e_n (M0 = n) make sample c equal to n P_cc, with P the
    filter matrix rho(B^{-1} A), so res[c] is the running mean of n P_cc and
    res[n-1] the trace sum_i rho(lambda_i) (section "Stochastic estimate").
    rho is the trapezoidal circle's closed form 1/(1 + t^(2 ne)), or the
    Gauss-Legendre filter through the (separately pinned) rational tool."""
    n = 24
    if herm:
        p = W.dense_complex_hermitian(n, count=5, seed=171, ne=ne, nclusters=2)
    else:
        p = W.dense_real_generalized(n, count=5, seed=172)
    c, r = 0.5 * (p.emin + p.emax), 0.5 * (p.emax - p.emin)
    if integration == 1:
        rho = lambda x: 1.0 / (1.0 + ((x - c) / r) ** (2 * ne))
    else:
        rho = lambda x: orc.rational(p.emin, p.emax, ne, np.asarray(x, float))
    lam, P = _filter_matrix(p.A, p.B, rho)
    X0 = np.eye(n, dtype=np.complex128 if herm else np.float64)
    out = orc.feast(p.A, p.B, p.emin, p.emax, n, ne, 1e-10, X0, hermitian=herm, mode=2,
                    integration=integration)
    assert out.info == 5 and out.loop == 0 and out.m0 == n
    ref = np.cumsum(n * np.diag(P).real) / np.arange(1, n + 1)
    assert np.allclose(out.res, ref, rtol=0, atol=1e-11 * n)
    assert abs(out.res[-1] - rho(lam).sum()) < 1e-11 * n
    assert out.M == max(0, int(np.floor(out.res[-1] + 0.5)))
    # the filtered probes come back in X: column c is P e_c
    assert np.allclose(out.X, P, rtol=0, atol=1e-11)


@pytest.mark.parametrize("ne", [2, 3, 8])
def test_count_estimate_exact_for_sign_probes_on_a_diagonal_pencil(orc, ne):
    """For diagonal A and B the filter matrix is diagonal, so a +-1 probe gives
    x^T P x = sum_i rho(a_i / b_i) exactly: every sample, and so every running
    average, equals the trace."""
    rng = np.random.default_rng(173)
    n, m0 = 40, 7
    a = rng.uniform(-2.0, 2.0, n)
    b = rng.uniform(0.5, 2.0, n)
    emin, emax = -0.7, 0.9
    lam = a / b
    t = (lam - 0.5 * (emin + emax)) / (0.5 * (emax - emin))
    trace = (1.0 / (1.0 + t ** (2 * ne))).sum()
    X0 = W.sign_probes(n, m0, seed=174)
    out = orc.feast(np.diag(a), np.diag(b), emin, emax, m0, ne, 1e-10, X0, mode=2, integration=1)
    assert out.info == 5
    assert np.allclose(out.res, trace, rtol=0, atol=1e-12 * n)
    assert out.M == int(np.floor(trace + 0.5))


def test_count_estimate_is_within_its_sampling_error(orc):
    """A dense pencil with +-1 probes: the estimate lies within 5 standard
    deviations of the trace.  For a +-1 probe, x^T P x has mean trace(P) and
    variance 2 (||S||_F^2 - sum_i S_ii^2), S = (P + P^T)/2 (Hutchinson);
    the mean of m0 probes divides it by m0."""
    n, m0, ne = 160, 48, 8
    p = W.dense_real_generalized(n, count=16, seed=175)
    rho = lambda x: orc.rational(p.emin, p.emax, ne, np.asarray(x, float))
    lam, P = _filter_matrix(p.A, p.B, rho)
    S = 0.5 * (P + P.T)
    sigma = math.sqrt(2.0 * (np.sum(S * S) - np.sum(np.diag(S) ** 2)) / m0)
    X0 = W.sign_probes(n, m0, seed=176)
    out = orc.feast(p.A, p.B, p.emin, p.emax, m0, ne, 1e-10, X0, mode=2)
    assert out.info == 5
    # the samples are the quadratic forms themselves, recomputed from P
    samples = np.einsum("ic,ij,jc->c", X0, P, X0)
    assert np.allclose(out.res, np.cumsum(samples) / np.arange(1, m0 + 1), rtol=0, atol=1e-10)
    assert abs(out.res[-1] - rho(lam).sum()) < 5.0 * sigma
    assert abs(rho(lam).sum() - p.count_in_interval()) < 0.5


@pytest.mark.parametrize("n", [1, 2, 7, 33, 96])
def test_lu_backward_error_and_solve(orc, n):
    A = _rand(n, n, n)
    lu, ipiv, info = orc.zgetrf(A)
    assert info == 0
    L = np.tril(lu, -1) + np.eye(n)
    Uu = np.triu(lu)
    PA = A.copy()
    for k, p in enumerate(ipiv):
        PA[[k, p]] = PA[[p, k]]
    assert np.linalg.norm(PA - L @ Uu) / np.linalg.norm(A) < 10 * n * U
    # pivot = largest |re|+|im|, so |l_ik| <= sqrt(2)
    assert (np.abs(L) <= math.sqrt(2) + 1e-15).all()
    b = _rand(n, 5, n + 1)
    x = orc.zgetrs(lu, ipiv, b, "N")
    xr = sl.lu_solve(sl.lu_factor(A), b)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) < 1e-12
    xh = orc.zgetrs(lu, ipiv, b, "C")
    xhr = sl.lu_solve(sl.lu_factor(A), b, trans=2)
    assert np.linalg.norm(xh - xhr) / np.linalg.norm(xhr) < 1e-12


def test_lu_triangular_and_diagonal_exact(orc):
    n = 12
    D = np.diag(np.arange(1, n + 1) * (1 + 1j))
    b = _rand(n, 3, 5)
    lu, ipiv, info = orc.zgetrf(D)
    assert info == 0 and (ipiv == np.arange(n)).all()
    x = orc.zgetrs(lu, ipiv, b)
    # one complex division per entry: equal up to that division's rounding
    assert np.allclose(x, b / np.diag(D)[:, None], rtol=4 * U, atol=0)
    Uu = np.triu(_rand(n, n, 6)) + 8 * np.eye(n)
    lu, ipiv, info = orc.zgetrf(Uu)
    assert info == 0 and np.array_equal(lu, Uu) and (ipiv == np.arange(n)).all()


def test_lu_reports_singular_and_nan(orc):
    A = np.zeros((4, 4), complex)
    A[0, 0] = 1
    assert orc.zgetrf(A)[2] == 2
    B = _rand(5, 5, 1)
    B[2, 3] = np.nan
    assert orc.zgetrf(B)[2] > 0


@pytest.mark.parametrize("opa", ["N", "C"])
def test_gemm_against_numpy(orc, opa):
    a = _rand(9, 7, 1)
    b = _rand(9 if opa == "C" else 7, 4, 2)
    ref = (a.conj().T if opa == "C" else a) @ b
    assert np.allclose(orc.zgemm(a, b, opa), ref, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("n,cplx", [(1, True), (2, False), (10, True), (40, True), (40, False)])
def test_jacobi_against_eigh(orc, n, cplx):
    a = _rand(n, n, 10 + n, cplx)
    a = 0.5 * (a + a.conj().T)
    w, V, info = orc.jacobi_eigh(a)
    assert info == 0
    wr = np.linalg.eigh(a)[0]
    nrm = np.linalg.norm(a)
    assert np.abs(w - wr).max() < 1e-13 * nrm
    assert np.linalg.norm(V.conj().T @ V - np.eye(n)) < 1e-13 * n
    assert np.linalg.norm(a @ V - V * w) < 1e-13 * nrm * n
    if not cplx:
        assert np.abs(V.imag).max() == 0.0


def test_jacobi_degenerate_cluster(orc):
    rng = np.random.default_rng(3)
    Q = np.linalg.qr(rng.standard_normal((20, 20)) + 1j * rng.standard_normal((20, 20)))[0]
    lam = np.r_[np.full(6, 0.5), 0.5 + 1e-12 * np.arange(4), np.linspace(-1, 2, 10)]
    a = (Q * lam) @ Q.conj().T
    a = 0.5 * (a + a.conj().T)
    w, V, info = orc.jacobi_eigh(a)
    assert info == 0
    assert np.abs(w - np.sort(lam)).max() < 1e-14 * 20
    assert np.linalg.norm(a @ V - V * w) < 1e-13


# ------------------------------------------- the contour step in closed form
def _filter_only(orc, A, B, emin, emax, ne, X0, herm):
    r = orc.feast(A, B, emin, emax, X0.shape[1], ne, 1e-12, X0, hermitian=herm, mode=1,
                  maxloop=0)
    assert r.info == 4
    return r.X


def test_contour_step_diagonal(orc):
    """A = diag(lambda), B = I: Q = diag(rho(lambda)) X exactly (up to rounding)."""
    n, m0, ne = 40, 6, 8
    lam = np.linspace(-2.0, 3.0, n)
    A = np.asfortranarray(np.diag(lam))
    X0 = W.start_subspace(n, m0, 7)
    Q = _filter_only(orc, A, None, -0.4, 1.1, ne, X0, False)
    ref = orc.rational(-0.4, 1.1, ne, lam)[:, None] * X0
    assert np.abs(Q - ref).max() < 1e-13


def test_contour_step_laplacian(orc):
    """1D Laplacian with its sine eigenvectors: Q = V diag(rho) V^T X."""
    n = 200
    p = W.laplacian_1d(n)
    k = np.arange(1, n + 1)
    V = math.sqrt(2.0 / (n + 1)) * np.sin(np.outer(k, k) * math.pi / (n + 1))
    lam = 2 - 2 * np.cos(k * math.pi / (n + 1))
    rho = orc.rational(p.emin, p.emax, p.ne, lam)
    # the guide's own expectations for this filter shape: strong pass-band,
    # strong decay outside
    assert rho[45] > 0.5 and abs(rho[46]) < 1e-2 and abs(rho[69]) < 1e-6
    ref = V @ (rho[:, None] * (V.T @ p.X0))
    Q = _filter_only(orc, p.A, None, p.emin, p.emax, p.ne, p.X0, False)
    assert np.abs(Q - ref).max() / np.abs(ref).max() < 1e-12


def test_contour_step_generalized_shared_vectors(orc):
    """A = Q diag(l) Q^T, B = Q diag(mu) Q^T: filter of (A, B) is
    Q diag(rho(l/mu)) Q^T X."""
    n, m0 = 48, 5
    rng = np.random.default_rng(11)
    Qo = np.linalg.qr(rng.standard_normal((n, n)))[0]
    l = rng.uniform(-1, 1, n)
    mu = rng.uniform(0.5, 2.0, n)
    A = np.asfortranarray((Qo * l) @ Qo.T)
    B = np.asfortranarray((Qo * mu) @ Qo.T)
    X0 = W.start_subspace(n, m0, 12)
    Q = _filter_only(orc, A, B, -0.2, 0.3, 8, X0, False)
    ref = Qo @ (orc.rational(-0.2, 0.3, 8, l / mu)[:, None] * (Qo.T @ X0))
    assert np.abs(Q - ref).max() / np.abs(ref).max() < 1e-11


def test_contour_step_hermitian_adjoint_half(orc):
    """Complex Hermitian A = U diag(l) U^H (B = I): the upper-half solves plus
    the adjoint solves for the mirrored lower half give U diag(rho) U^H X."""
    n, m0 = 36, 4
    rng = np.random.default_rng(13)
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Uu = np.linalg.qr(Z)[0]
    l = rng.uniform(-1, 1, n)
    A = np.asfortranarray((Uu * l) @ Uu.conj().T)
    A = np.asfortranarray(0.5 * (A + A.conj().T))
    X0 = W.start_subspace(n, m0, 14)
    Q = _filter_only(orc, A, None, -0.3, 0.4, 8, X0, True)
    ref = Uu @ (orc.rational(-0.3, 0.4, 8, l)[:, None] * (Uu.conj().T @ X0))
    assert np.abs(Q - ref).max() / np.abs(ref).max() < 1e-12
    # the real-symmetric formula Re(sum w_j Y_j) would be wrong here
    assert np.abs(Q.imag).max() > 1e-3


# ----------------------------------------------------------------- end to end
def _golden(name):
    vals = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            vals[k] = [float(t) for t in v]
    return vals


def test_helloworld_matches_guide(orc):
    g = _golden("helloworld.txt")
    A = np.asfortranarray(np.array(g["A"]).reshape(2, 2))
    p = W.helloworld()
    assert np.array_equal(A, p.A)
    r = orc.feast(A, None, g["emin"][0], g["emax"][0], int(g["m0"][0]), int(g["ne"][0]), 1e-12,
                  p.X0)
    assert r.info == int(g["info"][0])
    assert r.M == int(g["M"][0])
    assert r.loop == int(g["loop"][0])
    assert np.allclose(r.E, g["eigenvalues"], rtol=0, atol=2e-14)
    assert abs(r.E.sum() - g["trace"][0]) < 1e-13
    assert r.epsout == g["epsout"][0]
    assert (r.res[:2] < 1e-14).all()
    for i, key in enumerate(["vector1", "vector2"]):
        v = r.X[:, i] * np.sign(r.X[0, i])
        assert np.allclose(v, g[key], atol=1e-14)


def test_laplacian_closed_form(orc):
    p = W.laplacian_1d()
    r = orc.feast(p.A, p.B, p.emin, p.emax, p.m0, p.ne, p.tol, p.X0)
    k = np.arange(1, 47)
    exact = 2 - 2 * np.cos(k * math.pi / 201)
    assert r.info == 0 and r.M == 46
    assert np.abs(r.E[:46] - exact).max() < 1e-12 * exact.max()
    assert (r.res[:46] < p.tol).all()
    X = r.X[:, :46]
    assert np.abs(X.T @ X - np.eye(46)).max() < 1e-12
    # eigenvectors: each is +-(the sine vector)
    Vk = math.sqrt(2 / 201) * np.sin(np.outer(np.arange(1, 201), k) * math.pi / 201)
    assert np.abs(np.abs(np.sum(X * Vk, 0)) - 1).max() < 1e-10


def _brute_force(orc, A, B):
    """All eigenvalues of the pencil with the oracle's Jacobi alone:
    B = W diag(b) W^H, C = b^{-1/2} W^H A W b^{-1/2}, eig(C)."""
    b, Wb, info = orc.jacobi_eigh(B)
    assert info == 0 and b.min() > 0
    T = Wb / np.sqrt(b)
    C = T.conj().T @ A @ T
    return orc.jacobi_eigh(0.5 * (C + C.conj().T))[0]


def _inertia_count(A, B, emin, emax):
    """Sylvester: #eig in [emin, emax] = nu(A - emax B) - nu(A - emin B)."""
    def nu(s):
        _, D, _ = sl.ldl(A - s * B, hermitian=True)
        return int(np.sum(np.linalg.eigvalsh(D) < 0))
    return nu(emax) - nu(emin)


@pytest.mark.parametrize("n,herm,seed", [(24, False, 1), (40, False, 2), (32, True, 3),
                                         (48, True, 4)])
def test_small_pencils_brute_force_and_inertia(orc, n, herm, seed):
    if herm:
        p = W.dense_complex_hermitian(n, count=max(2, n // 6), seed=100 + seed, ne=8,
                                      tol=1e-12, nclusters=2)
    else:
        p = W.dense_real_generalized(n, count=max(2, n // 6), seed=100 + seed, tol=1e-12)
    r = orc.feast(p.A, p.B, p.emin, p.emax, p.m0, p.ne, p.tol, p.X0, hermitian=herm)
    assert r.info == 0
    allev = _brute_force(orc, p.A, p.B)
    inside = allev[(allev >= p.emin) & (allev <= p.emax)]
    assert r.M == inside.size == _inertia_count(p.A, p.B, p.emin, p.emax)
    alpha = max(abs(p.emin), abs(p.emax))
    assert np.abs(r.E[:r.M] - inside).max() < 1e-12 * alpha
    assert np.allclose(r.E[:r.M], sl.eigh(p.A, p.B, eigvals_only=True)[
        (allev >= p.emin) & (allev <= p.emax)], rtol=0, atol=1e-12 * alpha)
    X = r.X[:, :r.M]
    G = X.conj().T @ p.B @ X
    assert np.abs(G - np.eye(r.M)).max() < 1e-12
    # residuals as the guide defines them, recomputed here
    R = p.A @ X - (p.B @ X) * r.E[:r.M]
    res = np.abs(R).sum(0) / (alpha * np.abs(p.B @ X).sum(0))
    # AX = (AQ) Phi in the oracle vs A (Q Phi) here: equal up to rounding
    assert np.allclose(res, r.res[:r.M], rtol=1e-6, atol=1e-15)
    assert (res < p.tol).all()


# ------------------------------------------------------------------ info codes
def _hw():
    p = W.helloworld()
    return p.A, p.X0


@pytest.mark.parametrize("kw,code", [
    (dict(emin=1.0, emax=1.0), 200),
    (dict(emin=2.0, emax=-1.0), 200),
    (dict(ne=0), 102),
    (dict(tol=0.0), 103),
    (dict(maxloop=-1), 104),
    (dict(conv=2), 106),
])
def test_info_argument_errors(orc, kw, code):
    A, X0 = _hw()
    args = dict(emin=-5.0, emax=5.0, ne=8, tol=1e-12, maxloop=20, conv=1)
    args.update(kw)
    r = orc.feast(A, None, args["emin"], args["emax"], 2, args["ne"], args["tol"], X0,
                  maxloop=args["maxloop"], conv=args["conv"])
    assert r.info == code


def test_info_sizes(orc):
    lib = orc._load()
    import ctypes as C
    z = np.zeros(4, complex)
    m = np.array([1], np.int32)
    out = [np.zeros(4), np.zeros(4, complex), np.zeros(4), np.zeros(1, np.int32),
           np.zeros(1, np.int32), np.zeros(1)]
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))

    def call(n, m0):
        m[0] = m0
        return lib.orc_feast(0, n, z.ctypes.data, None, -1.0, 1.0, ip(m), 8, 1e-12, 5, 1, 0,
                             z.ctypes.data, dp(out[0]), out[1].ctypes.data, dp(out[2]),
                             ip(out[3]), ip(out[4]), dp(out[5]), 0, 100, None, None)
    assert call(0, 1) == 202
    assert call(2, 0) == 201
    assert call(2, 3) == 201


def test_info_nan_is_inner_solver_error(orc):
    A, X0 = _hw()
    A = A.copy()
    A[0, 1] = np.nan
    assert orc.feast(A, None, -5, 5, 2, 8, 1e-12, X0).info == -2


def test_info_indefinite_B(orc):
    p = W.laplacian_1d(30, emin=0.0, emax=1.0, m0=12)
    B = -np.eye(30)
    assert orc.feast(p.A, B, p.emin, p.emax, p.m0, p.ne, p.tol, p.X0).info == -3


def test_info_empty_interval(orc):
    p = W.laplacian_1d(30, m0=6)
    r = orc.feast(p.A, None, 10.0, 11.0, 6, 8, 1e-12, p.X0)
    assert r.info == 1 and r.M == 0


def test_info_no_convergence(orc):
    p = W.laplacian_1d(60, emin=0.0, emax=1.0, m0=32)   # 20 eigenvalues inside
    r = orc.feast(p.A, None, p.emin, p.emax, p.m0, p.ne, 1e-30, p.X0, maxloop=1)
    assert r.info == 2 and r.loop == 1


def test_info_subspace_too_small(orc):
    p = W.laplacian_1d(60, emin=0.0, emax=1.0, m0=8)   # 20 eigenvalues inside
    r = orc.feast(p.A, None, p.emin, p.emax, p.m0, p.ne, 1e-12, p.X0)
    assert r.info == 3 and r.M >= r.m0


def test_trace_convergence_criterion(orc):
    p = W.laplacian_1d()
    r = orc.feast(p.A, None, p.emin, p.emax, p.m0, p.ne, 1e-12, p.X0, conv=0)
    assert r.info == 0 and r.loop >= 1 and r.epsout < 1e-12 and r.M == 46


def test_output_order(orc):
    p = W.laplacian_1d()
    r = orc.feast(p.A, None, p.emin, p.emax, p.m0, p.ne, p.tol, p.X0)
    inside = r.E[:r.M]
    outside = r.E[r.M:]
    assert (np.diff(inside) > 0).all() and (np.diff(outside) >= 0).all()
    assert ((inside >= p.emin) & (inside <= p.emax)).all()
    assert ((outside < p.emin) | (outside > p.emax)).all()


def _gap_problem():
    """Real symmetric A (B = I) whose spectrum avoids [-0.5, 0.5]: the
    search interval [-0.2, 0.2] holds no eigenvalue and every point of it is
    at least 0.3 from the spectrum."""
    rng = np.random.default_rng(21)
    n, m0 = 40, 12
    lam = np.concatenate([rng.uniform(-1, -0.5, n // 2), rng.uniform(0.5, 1, n - n // 2)])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T), rng.uniform(-1, 1, (n, m0)), m0


def test_spurious_pairs_in_a_spectral_gap(orc):
    """The spurious flag (section "The FEAST Algorithm" reading R11) pinned
    by a bound: for a Ritz pair (theta, x) with theta in the interval,
    ||A x - theta x||_2 >= 0.3 ||x||_2 (the distance to the spectrum), so
    its residual ||A x - theta x||_1 / (alpha ||x||_1) >= 0.3 / (alpha sqrt(n))
    = 0.24 > 0.1: every such pair is spurious from the second loop on, and
    none counts towards M.  At the first loop nothing is flagged."""
    A, X0, m0 = _gap_problem()
    n = A.shape[0]
    emin, emax = -0.2, 0.2
    alpha = max(abs(emin), abs(emax))
    assert 0.3 / (alpha * math.sqrt(n)) > 0.1
    out0 = orc.feast(A, None, emin, emax, m0, 8, 1e-10, X0, maxloop=0)
    in0 = (out0.E >= emin) & (out0.E <= emax)
    assert in0.any(), "the random start should leave Ritz values in the gap at the first loop"
    assert out0.M == in0.sum() and (out0.res[in0] > 0.1).all()   # counted, not flagged
    out1 = orc.feast(A, None, emin, emax, m0, 8, 1e-10, X0, maxloop=1)
    in1 = (out1.E >= emin) & (out1.E <= emax)
    assert out1.M == 0 and out1.info == 2
    assert (out1.res[in1] == -1.0).all()
    # spurious pairs come last
    k = int(in1.sum())
    if k:
        assert in1[m0 - k:].all()
        X = out1.X[:, m0 - k:]
        th = out1.E[m0 - k:]
        r = np.abs(A @ X - X * th).sum(0) / (alpha * np.abs(X).sum(0))
        assert (r > 0.1).all()


def test_oracle_is_not_used_by_the_product():
    """The oracle is test infrastructure: the package and headers never name it."""
    root = os.path.dirname(HERE)
    for sub in ("paper_1203_4031_amd", "include"):
        for dp, _, files in os.walk(os.path.join(root, sub)):
            for fn in files:
                if fn.endswith((".py", ".hip", ".h", ".hpp", ".cpp", ".c")):
                    with open(os.path.join(dp, fn), errors="ignore") as f:
                        txt = f.read()
                    assert "import oracle" not in txt and "from oracle" not in txt, fn
                    assert "feast_oracle" not in txt and "liboracle" not in txt, fn
