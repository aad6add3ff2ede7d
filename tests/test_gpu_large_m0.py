"""A subspace wider than the Cholesky path takes (M0 > 1024): the
B-orthonormal basis of the reduced problem then comes from the
eigendecomposition of Bq with truncation (the route the oracle always takes,
and the fallback of the Cholesky path when it meets a negative pivot), and
the reduced eigensolve runs on a 1080-column problem.

The oracle at this size takes minutes on the host, so the checks are the
properties of tests/test_gpu_fullsize.py against the spectrum LAPACK gives
for the generator: the count, every eigenvalue within the 1e-10 relative
bar, the reported residuals, host-recomputed FP64 residuals and
B-orthonormality on a seeded sample of eigenpairs (parity with the oracle
itself unpinned at this size)."""
import numpy as np
import pytest

from paper_1203_4031_amd import feastx
from paper_1203_4031_amd import workloads as W

pytestmark = pytest.mark.gpu

N, COUNT = 1536, 720


@pytest.fixture(scope="module")
def problem():
    p = W.dense_real_generalized(N, COUNT, ne=8, tol=1e-10, seed=2501)
    assert p.m0 > 1024
    return p


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_wide_subspace(problem, precision):
    p = problem
    print(f"wide subspace n {p.n} m0 {p.m0} {precision}", flush=True)
    r = feastx.solve(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, ne=p.ne, tol=p.tol, precision=precision)
    assert r.info == 0, r.info
    inside = p.spectrum[(p.spectrum >= p.emin) & (p.spectrum <= p.emax)]
    assert r.M == len(inside) == COUNT
    a = max(abs(p.emin), abs(p.emax))
    E = np.sort(r.E[:r.M])
    assert (np.abs(E - inside) / np.maximum(np.abs(inside), a)).max() <= 1e-10
    assert (r.res[:r.M] < p.tol).all()
    rng = np.random.default_rng(7)
    idx = rng.choice(r.M, 40, replace=False)
    X = r.X[:, idx]
    BX = p.B @ X
    res = np.abs(p.A @ X - BX * r.E[idx]).sum(0) / (a * np.abs(BX).sum(0))
    assert (res < p.tol).all(), res.max()
    G = X.T @ BX
    assert np.abs(G - np.eye(len(idx))).max() < 1e-10
