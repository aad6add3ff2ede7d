"""GPU check of feast_solve_d_dev_noalloc, the entry point that allocates
nothing (its device workspace is the library's static scratch array): on the
same seeded inputs it must give what feast_solve_d_dev gives, to the parity
bar of every other GPU test (eigenvalues within 1e-10 relative, the same
count, residuals below tol, the same eigenspace), on two calls in a row, the
second with a smaller problem, in both precisions.  A problem too large for
the scratch is refused with info -1 before any GPU work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _solve(p, prec, noalloc):
    from paper_1203_4031_amd import feastx

    A = feastx.fortran_tensor(p.A)
    B = feastx.fortran_tensor(p.B)
    X = feastx.fortran_tensor(p.X0)
    print(f"noalloc={noalloc} {p.name} N={p.n} M0={p.m0} {prec}", flush=True)
    r = feastx.solve_device(A, B, p.emin, p.emax, p.m0, X, x0=True, ne=p.ne, tol=p.tol, precision=prec,
                            noalloc=noalloc)
    torch.cuda.synchronize()
    return r, X.cpu().numpy()


def _same(p, ra, Xa, rb, Xb):
    assert ra.info == 0 and rb.info == 0, (ra.info, rb.info)
    assert ra.M == rb.M == p.count_in_interval()
    alpha = max(abs(p.emin), abs(p.emax))
    a, b = ra.E[:ra.M], rb.E[:rb.M]
    assert np.all(np.abs(a - b) <= 1e-10 * np.maximum(np.abs(b), alpha))
    assert np.all(ra.res[:ra.M] < p.tol) and np.all(rb.res[:rb.M] < p.tol)
    # same eigenspace: the B-inner products of the two bases have singular values 1
    G = Xa[:, :ra.M].T @ (p.B @ Xb[:, :rb.M])
    sv = np.linalg.svd(G, compute_uv=False)
    assert sv.min() >= 1 - 1e-8, sv.min()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_matches_dev_two_calls(prec):
    from paper_1203_4031_amd import workloads as W

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    big = W.dense_real_generalized(448, count=40, seed=2401, tol=1e-10)
    small = W.dense_real_generalized(200, count=16, seed=2402, tol=1e-10)
    for p in (big, small):
        rn, Xn = _solve(p, prec, True)
        rd, Xd = _solve(p, prec, False)
        _same(p, rn, Xn, rd, Xd)


def test_noalloc_refuses_too_large():
    from paper_1203_4031_amd import feastx
    from paper_1203_4031_amd import workloads as W

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n, m0 = 1536, 64
    A = feastx.fortran_tensor(np.eye(n))
    X = feastx.fortran_tensor(W.start_subspace(n, m0, seed=1))
    r = feastx.solve_device(A, None, 0.5, 1.5, m0, X, x0=True, ne=8, tol=1e-10, precision="fp64", noalloc=True)
    assert r.info == -1
