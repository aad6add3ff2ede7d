"""GPU parity of non-Hermitian FEAST (dual subspaces, full contour) against
the FP64 oracle in oracle/nonherm.py, through feast_gsolve_{z,d}.

Bar: the same count M; every eigenvalue the oracle finds inside the region
matched by one of the library's within 1e-10 max(|lambda|, alpha), alpha =
|Emid| + r; right and left residuals below tol on both sides, recomputed here
in FP64; the matched right and left eigenvectors (unit 2-norm on both sides)
equal up to a unimodular factor, |x^H x_ref| >= 1 - 1e-8.  The order of
eigenvalues with equal real parts may differ by rounding, so pairs are
matched by value."""
import numpy as np
import pytest
import scipy.linalg as sl

torch = pytest.importorskip("torch")

from oracle import nonherm as NH  # noqa: E402
from paper_1203_4031_amd import feastx  # noqa: E402
from paper_1203_4031_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _resid(A, B, X, lam, alpha):
    B = np.eye(A.shape[0]) if B is None else B
    return np.abs(A @ X - (B @ X) * lam).sum(0) / (alpha * np.abs(B @ X).sum(0))


def _check(p, r, ref, ellipse=100, angle=0):
    emid, rad = p.emin, p.emax
    alpha = abs(emid) + rad
    assert r.info == 0 and ref.info == 0, (r.info, ref.info)
    assert r.M == ref.M == p.meta["count"]
    m0, M = r.m0, r.M
    got, exp = r.E[:M], ref.E[:M]
    for k in range(M):
        d = np.abs(got - exp[k])
        j = int(np.argmin(d))
        assert d[j] <= 1e-10 * max(abs(exp[k]), alpha), (exp[k], d[j])
        for off in (0, m0):   # right, then left vectors
            c = abs(np.vdot(r.X[:, off + j], ref.X[:, off + k]))
            assert c >= 1 - 1e-8, (off, k, c)
    B = p.B
    Bh = None if B is None else B.conj().T
    X, Xh = r.X[:, :M], r.X[:, m0:m0 + M]
    assert (_resid(p.A, B, X, got, alpha) < p.tol).all()
    assert (_resid(p.A.conj().T, Bh, Xh, np.conj(got), alpha) < p.tol).all()
    assert (r.res[:M] < p.tol).all() and (r.res[m0:m0 + M] < p.tol).all()
    # the reported residuals are those of the returned pairs (to the rounding
    # of a cancelling sum: N u relative to alpha ||B x||)
    assert np.allclose(r.res[:M], _resid(p.A, B, X, got, alpha), rtol=1e-6, atol=1e-13)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("real,generalized", [(False, True), (True, False), (True, True), (False, False)])
def test_gsolve_matches_oracle(real, generalized, precision):
    """Both precisions reach the FP64 oracle's eigenpairs: in mixed
    precision the complex64 solves act on the FP64 Ritz residuals after the
    first loop."""
    p = W.dense_general(200, count=12, seed=6101 + 2 * real + generalized, real=real, generalized=generalized)
    print(f"gsolve real {real} generalized {generalized} {precision} n {p.n} m0 {p.m0}", flush=True)
    ref = NH.feast(p.A, p.B, p.emin, p.emax, p.m0, p.ne, p.tol, p.X0)
    r = feastx.gsolve(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, tol=p.tol, ne_full=p.ne, precision=precision)
    _check(p, r, ref)


def test_gsolve_gauss_rotated_ellipse():
    p = W.dense_general(160, count=8, seed=6111, real=True)
    ref = NH.feast(p.A, p.B, p.emin, p.emax, p.m0, 24, p.tol, p.X0, integration=0, ellipse=60, angle=35)
    r = feastx.gsolve(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, tol=p.tol, ne_full=24, integration_full=0,
                      ellipse=60, angle=35)
    inside = NH.inside(p.emin, p.emax, sl.eig(p.A, p.B, right=False), 60, 35)
    assert r.M == ref.M == int(inside.sum())
    p.meta["count"] = r.M
    _check(p, r, ref, 60, 35)


def test_gsolve_library_start_finds_the_spectrum():
    """x0 = 0 (the library's seeded start): the eigenvalues inside the region
    are LAPACK's for the whole pencil."""
    p = W.dense_general(150, count=10, seed=6121)
    r = feastx.gsolve(p.A, p.B, p.emin, p.emax, p.m0, tol=p.tol, ne_full=16)
    assert r.info == 0 and r.M == p.meta["count"]
    full = sl.eig(p.A, p.B, right=False)
    ref = full[NH.inside(p.emin, p.emax, full)]
    alpha = abs(p.emin) + p.emax
    for l in ref:
        assert np.abs(r.E[:r.M] - l).min() <= 1e-10 * max(abs(l), alpha)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gsolve_matches_oracle_beyond_lds_size(precision):
    """M0 = 76 > 64: the reduced eigensolver and inverses work in memory
    instead of LDS."""
    p = W.dense_general(300, count=48, seed=6131)
    assert p.m0 > 64
    ref = NH.feast(p.A, p.B, p.emin, p.emax, p.m0, p.ne, p.tol, p.X0)
    r = feastx.gsolve(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, tol=p.tol, ne_full=p.ne, precision=precision)
    _check(p, r, ref)


def test_gsolve_device_arrays_match_host_arrays():
    """feast_gsolve_z_dev (A, B, X in HBM, caller's stream) returns what the
    host-array entry point returns."""
    p = W.dense_general(200, count=12, seed=6141)
    host = feastx.gsolve(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, tol=p.tol, ne_full=16)
    A = feastx.fortran_tensor(p.A.astype(np.complex128))
    B = feastx.fortran_tensor(p.B.astype(np.complex128))
    X = feastx.fortran_tensor(p.X0.astype(np.complex128))
    dev = feastx.gsolve_device(A, B, p.emin, p.emax, p.m0, X, x0=True, tol=p.tol, ne_full=16)
    torch.cuda.synchronize()
    assert dev.info == host.info == 0 and dev.M == host.M and dev.loop == host.loop
    assert np.array_equal(dev.E, host.E)
    assert np.array_equal(dev.res, host.res)
    assert np.array_equal(X.cpu().numpy(), host.X)
