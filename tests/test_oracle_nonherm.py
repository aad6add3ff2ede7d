"""Pins for the non-Hermitian oracle (oracle/nonherm.py): closed forms of the
full-contour filter, the residue theorem, spectra known by construction
(rotation blocks, triangular matrices), brute force with LAPACK on the whole
pencil, the left-eigenvector equation, and the info codes."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import nonherm as NH
from paper_1203_4031_amd import workloads as W

U = np.finfo(np.float64).eps


@pytest.mark.parametrize("ne", [1, 2, 3, 8, 16])
def test_trapezoidal_circle_filter_closed_form(ne):
    """Nodes at the ne-th roots of -1 on the circle give
    rho(lambda) = 1 / (1 + s^ne), s = (lambda - c) / r, for complex lambda
    (partial fractions of 1/(1 + s^ne) over its ne roots)."""
    c, r = 0.3 - 0.2j, 1.7
    s = np.array([0.0, 0.4 + 0.2j, -0.5j, 0.9 - 0.3j, 1.3 + 0.7j, -2.0 + 0.5j, 3.0j])
    ref = 1.0 / (1.0 + s ** ne)
    got = NH.rational(c, r, ne, c + r * s, integration=1)
    assert np.allclose(got, ref, rtol=0, atol=64 * U)


@pytest.mark.parametrize("integration,ne,bar", [(0, 128, 1e-4), (1, 200, 1e-8)])
@pytest.mark.parametrize("ellipse,angle", [(100, 0), (40, 0), (250, 30), (60, -75)])
def test_filter_tends_to_the_indicator(integration, ne, bar, ellipse, angle):
    """With many nodes the quadrature of dz / (2 pi i (z - lambda)) reaches
    its exact value (residue theorem): 1 inside the region, 0 outside, for
    every rule, ellipse ratio and rotation -- which pins the orientation and
    the weights of the rotated ellipse.  (The trapezoidal rule converges
    geometrically on this periodic integrand, Gauss-Legendre over one period
    more slowly.)"""
    c, r = 0.1 + 0.4j, 2.0
    a, phi = ellipse / 100.0, math.radians(angle)
    rng = np.random.default_rng(5)
    u = rng.uniform(-2, 2, 400) + 1j * rng.uniform(-2, 2, 400)
    u = u[(np.abs(u) < 0.6) | (np.abs(u) > 1.5)]   # well inside or well outside the unit circle
    lam = c + np.exp(1j * phi) * (r * u.real + 1j * a * r * u.imag)
    ins = NH.inside(c, r, lam, ellipse, angle)
    assert ins.any() and (~ins).any()
    rho = NH.rational(c, r, ne, lam, integration, ellipse, angle)
    assert np.abs(rho[ins] - 1.0).max() < bar
    assert np.abs(rho[~ins]).max() < bar


def test_contour_geometry():
    """Nodes on the rotated ellipse, listed by increasing parameter, and each
    weight along -i times the contour's tangent (dz / (2 pi i))."""
    c, r, a, ang = -0.4 + 0.3j, 1.2, 0.5, 20.0
    z, w = NH.contour(c, r, 12, 1, 50, ang)
    u = (z - c) * np.exp(-1j * math.radians(ang))
    assert np.allclose((u.real / r) ** 2 + (u.imag / (a * r)) ** 2, 1.0, atol=16 * U)
    t = np.mod(np.arctan2(u.imag / a, u.real), 2 * math.pi)
    assert (np.diff(t) > 0).all()
    tangent = np.exp(1j * math.radians(ang)) * (-r * np.sin(t) + 1j * a * r * np.cos(t))
    cosang = (w * np.conj(-1j * tangent)).real / (np.abs(w) * np.abs(tangent))
    assert np.allclose(cosang, 1.0, atol=1e-12)
    # trapezoidal weights sum to the integral of dz / (2 pi i) = 0
    assert abs(w.sum()) < 32 * U


def _check(out, A, B, lam_ref, emid, r, tol, ellipse=100, angle=0.0):
    n = A.shape[0]
    B = np.eye(n) if B is None else B
    alpha = abs(emid) + r
    ins = NH.inside(emid, r, lam_ref, ellipse, angle)
    ref = lam_ref[ins]
    assert out.info == 0, out.info
    assert out.M == ref.size
    got = out.E[:out.M]
    # every reference eigenvalue found once, within 1e-10 of its value
    for l in ref:
        d = np.abs(got - l)
        assert d.min() <= 1e-10 * max(abs(l), alpha), (l, d.min())
    m0 = out.E.size
    X, Xh = out.X[:, :out.M], out.X[:, m0:m0 + out.M]
    rr = np.abs(A @ X - (B @ X) * got).sum(0) / (alpha * np.abs(B @ X).sum(0))
    rl = np.abs(A.conj().T @ Xh - (B.conj().T @ Xh) * np.conj(got)).sum(0) / (alpha * np.abs(B.conj().T @ Xh).sum(0))
    assert (rr < tol).all() and (rl < tol).all(), (rr.max(), rl.max())
    assert np.allclose(out.res[:out.M], rr, rtol=1e-6, atol=1e-15)
    assert np.allclose(out.res[m0:m0 + out.M], rl, rtol=1e-6, atol=1e-15)
    assert np.allclose(np.linalg.norm(X, axis=0), 1.0) and np.allclose(np.linalg.norm(Xh, axis=0), 1.0)


def test_rotation_blocks_known_spectrum():
    """A real matrix similar to 2 x 2 blocks [[a, b], [-b, a]] (eigenvalues
    a +- i b) and real 1 x 1 blocks: the eigenvalues are known exactly."""
    rng = np.random.default_rng(11)
    n = 40
    D = np.zeros((n, n))
    lam = []
    for k in range(0, 30, 2):
        a, b = rng.uniform(-1, 1), rng.uniform(0.1, 1)
        D[k, k] = D[k + 1, k + 1] = a
        D[k, k + 1], D[k + 1, k] = b, -b
        lam += [a + 1j * b, a - 1j * b]
    for k in range(30, n):
        D[k, k] = rng.uniform(-1, 1)
        lam.append(D[k, k] + 0j)
    lam = np.array(lam)
    S = np.eye(n) + rng.standard_normal((n, n)) / (2 * math.sqrt(n))
    A = S @ D @ np.linalg.inv(S)
    emid, r = 0.1 + 0.0j, 0.62
    m0 = int(NH.inside(emid, r, lam).sum()) * 2 + 4
    X0 = rng.uniform(-1, 1, (n, 2 * m0))
    out = NH.feast(A, None, emid, r, m0, 16, 1e-11, X0)
    _check(out, A, None, lam, emid, r, 1e-11)
    # a real pencil's eigenvalues inside a real-symmetric region come in conjugate pairs
    got = out.E[:out.M]
    assert max(np.abs(got - np.conj(l)).min() for l in got) < 1e-10


def test_triangular_nonnormal():
    """Upper triangular A: the eigenvalues are its diagonal, however far from
    normal the matrix is."""
    rng = np.random.default_rng(12)
    n = 32
    d = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    A = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), 1) * 0.3 + np.diag(d)
    emid, r = 0.0 + 0.0j, 0.55
    m0 = int(NH.inside(emid, r, d).sum()) + 6
    X0 = rng.uniform(-1, 1, (n, 2 * m0))
    out = NH.feast(A, None, emid, r, m0, 24, 1e-10, X0, integration=0)
    _check(out, A, None, d, emid, r, 1e-10)


@pytest.mark.parametrize("real,generalized", [(False, True), (True, False), (True, True)])
def test_random_pencils_against_lapack(real, generalized):
    """Random non-normal pencils: the eigenvalues inside the region are those
    LAPACK finds for the whole pencil; left eigenvectors satisfy
    y^H A = lambda y^H B."""
    p = W.dense_general(80, count=8, seed=601 + 2 * real + generalized, real=real, generalized=generalized)
    full = sl.eig(p.A, p.B, right=False)
    assert max(np.abs(full - l).min() for l in p.spectrum) < 1e-9   # the generator's spectrum
    out = NH.feast(p.A, p.B, p.emin, p.emax, p.m0, p.ne, p.tol, p.X0)
    _check(out, p.A, p.B, full, p.emin, p.emax, p.tol)
    assert out.M == p.meta["count"] >= 8


def test_ellipse_and_rotation_region():
    p = W.dense_general(60, count=6, seed=611)
    out = NH.feast(p.A, p.B, p.emin, p.emax, p.m0, 16, 1e-10, p.X0, ellipse=60, angle=35)
    full = sl.eig(p.A, p.B, right=False)
    _check(out, p.A, p.B, full, p.emin, p.emax, 1e-10, ellipse=60, angle=35)


@pytest.mark.parametrize("kw,code", [
    (dict(m0=0), 201), (dict(m0=99), 201), (dict(ne=0), 108), (dict(tol=0.0), 103), (dict(maxloop=-1), 104),
    (dict(conv=2), 106), (dict(integration=2), 117), (dict(ellipse=0), 118), (dict(angle=181), 119),
    (dict(r=0.0), 200),
])
def test_info_argument_errors(kw, code):
    n = 10
    args = dict(m0=3, ne=8, tol=1e-10, maxloop=20, conv=1, integration=1, ellipse=100, angle=0, r=1.0)
    args.update(kw)
    A = np.eye(n)
    X0 = np.ones((n, 2 * max(args["m0"], 1)))
    out = NH.feast(A, None, 0.0, args["r"], args["m0"], args["ne"], args["tol"], X0, maxloop=args["maxloop"],
                   conv=args["conv"], integration=args["integration"], ellipse=args["ellipse"], angle=args["angle"])
    assert out.info == code


def test_info_empty_region_and_no_convergence():
    p = W.dense_general(60, count=6, seed=612)
    out = NH.feast(p.A, p.B, 5.0 + 5.0j, 0.5, p.m0, 16, 1e-10, p.X0)
    assert out.info == 1 and out.M == 0
    out = NH.feast(p.A, p.B, p.emin, p.emax, p.m0, 4, 1e-14, p.X0, maxloop=1)
    assert out.info == 2


def _normal_annulus(seed, n=48):
    """A normal complex matrix U diag(lambda) U^H (U Haar unitary) with every
    eigenvalue in the annulus 0.8 <= |lambda| <= 1.2."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Qm, R = np.linalg.qr(G)
    Qm = Qm * (np.diag(R) / np.abs(np.diag(R)))
    lam = rng.uniform(0.8, 1.2, n) * np.exp(1j * rng.uniform(0.0, 2.0 * math.pi, n))
    return (Qm * lam) @ Qm.conj().T, lam, rng


def test_spurious_pairs_in_a_spectral_hole():
    """The spurious flag of the non-Hermitian oracle (reading: a pair inside
    the region with either residual above 0.1 from the second loop on),
    pinned by a bound.  A is normal with its spectrum in 0.8 <= |lambda| <= 1.2
    and the region is the disk |z| <= 0.3, so any theta in the region is at
    least 0.5 from the spectrum and ||A x - theta x||_2 >= 0.5 ||x||_2 (the
    same for A^H and conj(theta)).  With ||v||_1 >= ||v||_2 and
    ||x||_1 <= sqrt(n) ||x||_2 both residuals are >= 0.5 / (alpha sqrt(n)) =
    0.24 > 0.1 (alpha = |Emid| + r = 0.3): every Ritz pair in the region is
    spurious from the second loop on and none counts.  At the first loop
    nothing is flagged."""
    A, lam, rng = _normal_annulus(2)
    n, m0, r = A.shape[0], 12, 0.3
    alpha = r
    assert 0.5 / (alpha * math.sqrt(n)) > 0.1
    X0 = rng.uniform(-1, 1, (n, 2 * m0))
    out0 = NH.feast(A, None, 0.0, r, m0, 16, 1e-10, X0, maxloop=0)
    in0 = NH.inside(0.0, r, out0.E)
    assert in0.any(), "the random start leaves Ritz values in the region at the first loop"
    assert out0.info == 2 and out0.M == in0.sum()
    assert (out0.res[:m0][in0] > 0.1).all() and (out0.res[m0:][in0] > 0.1).all()   # counted, not flagged
    out1 = NH.feast(A, None, 0.0, r, m0, 16, 1e-10, X0, maxloop=1)
    in1 = NH.inside(0.0, r, out1.E)
    k = int(in1.sum())
    assert k >= 1, "a Ritz value stays in the region at the second loop"
    assert out1.M == 0 and out1.info == 2
    # flagged pairs come last on both sides, with res = -1
    assert in1[m0 - k:].all() and (out1.res[m0 - k:m0] == -1.0).all() and (out1.res[2 * m0 - k:] == -1.0).all()
    th = out1.E[m0 - k:]
    X, Xh = out1.X[:, m0 - k:m0], out1.X[:, 2 * m0 - k:]
    rr = np.abs(A @ X - X * th).sum(0) / (alpha * np.abs(X).sum(0))
    rl = np.abs(A.conj().T @ Xh - Xh * np.conj(th)).sum(0) / (alpha * np.abs(Xh).sum(0))
    assert (rr > 0.1).all() and (rl > 0.1).all()


def test_trace_convergence_test_conv0():
    """fpm(6) = 0: stop at the first loop k >= 1 whose relative trace change
    |sum_M lambda (loop k) - sum_M lambda (loop k - 1)| / alpha is below tol,
    alpha = |Emid| + r.  Pinned by the known spectrum of a rotation-block
    matrix (the counted eigenvalues at the stop are the exact ones), by the
    previous loop's trace (a run of the same start stopped one loop
    earlier), and by the first loop never stopping under this test."""
    rng = np.random.default_rng(21)
    n = 40
    D = np.zeros((n, n))
    lam = []
    for k in range(0, 24, 2):
        a, b = rng.uniform(-1, 1), rng.uniform(0.1, 1)
        D[k, k] = D[k + 1, k + 1] = a
        D[k, k + 1], D[k + 1, k] = b, -b
        lam += [a + 1j * b, a - 1j * b]
    for k in range(24, n):
        D[k, k] = rng.uniform(-1, 1)
        lam.append(D[k, k] + 0j)
    lam = np.array(lam)
    S = np.eye(n) + rng.standard_normal((n, n)) / (2 * math.sqrt(n))
    A = S @ D @ np.linalg.inv(S)
    emid, r, tol = 0.05 + 0.0j, 0.6, 1e-12
    alpha = abs(emid) + r
    count = int(NH.inside(emid, r, lam).sum())
    m0 = 2 * count + 4
    X0 = rng.uniform(-1, 1, (n, 2 * m0))
    out = NH.feast(A, None, emid, r, m0, 16, tol, X0, conv=0)
    assert out.info == 0 and out.M == count and out.loop >= 1
    assert out.epsout < tol
    exact = lam[NH.inside(emid, r, lam)]
    got = out.E[:out.M]
    assert max(np.abs(exact - g).min() for g in got) < 1e-9
    prev = NH.feast(A, None, emid, r, m0, 16, tol, X0, conv=0, maxloop=out.loop - 1)
    assert prev.info == 2 and prev.loop == out.loop - 1
    expected = abs(got.sum() - prev.E[:prev.M].sum()) / alpha
    assert abs(out.epsout - expected) <= 1e-13 * max(1.0, expected)
    if prev.loop >= 1:
        assert prev.epsout >= tol
    # the first loop never stops under the trace test, even on a converged start
    once = NH.feast(A, None, emid, r, m0, 16, tol, out.X, conv=0, maxloop=0)
    assert once.info == 2 and once.loop == 0 and once.epsout == 1.0
