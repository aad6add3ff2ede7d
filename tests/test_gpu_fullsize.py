"""Full-size GPU checks on the workload the bench times (dense real symmetric
generalized pencil, N = 4096, M0 = 300, Ne = 8, tol 1e-10, inputs resident in
HBM, the same `feast_solve_d_dev` call and options as bench.py).

The FP64 oracle's own runs on this workload and on the N = 8192 complex
Hermitian one are stored in tests/golden/oracle_{realgen_n4096,
hermgen_n8192}.json (written by tests/golden/make_oracle_fixtures.py, which
calls only the oracle): both precisions are compared with them element by
element (eigenvalues) and through a sketch of the interval's eigenprojector.  The other checks are properties
that hold at any size (guide: Table "tab_common" for E, X, res and M; Table
"tab_info"):

* M equals the number of generalized eigenvalues in [Emin, Emax], counted from
  the spectrum LAPACK computes for the generator;
* every eigenvalue found matches that spectrum within the 1e-10 relative bar;
* every reported residual is below tol;
* for a seeded sample of eigenpairs, the residual recomputed on the host in
  FP64 from A, B, lambda and x is below tol, and the sampled X is B-orthonormal;
* the mixed-precision and FP64 solves give the same eigenvalues.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

N, COUNT, M0, NE, TOL, SEED = 4096, 200, 300, 8, 1e-10, 2001


@pytest.fixture(scope="module")
def bench_problem():
    from paper_1203_4031_amd import workloads as W

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return W.dense_real_generalized(N, COUNT, m0=M0, ne=NE, tol=TOL, seed=SEED)


@pytest.fixture(scope="module")
def solved(bench_problem):
    from paper_1203_4031_amd import feastx

    p = bench_problem
    A = feastx.fortran_tensor(p.A)
    B = feastx.fortran_tensor(p.B)
    X0 = feastx.fortran_tensor(p.X0)
    out = {}
    for prec in ("mixed", "fp64"):
        X = X0.clone().t().contiguous().t()
        r = feastx.solve_device(A, B, p.emin, p.emax, p.m0, X, x0=True, ne=p.ne, tol=p.tol, precision=prec)
        torch.cuda.synchronize()
        out[prec] = (r, X.cpu().numpy())
    return out


def _inside(p):
    s = p.spectrum
    return s[(s >= p.emin) & (s <= p.emax)]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_count_eigenvalues_and_residuals(bench_problem, solved, prec):
    p = bench_problem
    r, _ = solved[prec]
    ref = _inside(p)
    assert r.info == 0
    assert r.M == len(ref) == p.count_in_interval()
    alpha = max(abs(p.emin), abs(p.emax))
    lam = np.sort(r.E[:r.M])
    bar = 1e-10 * np.maximum(np.abs(ref), alpha)
    assert np.all(np.abs(lam - ref) <= bar), np.max(np.abs(lam - ref) / np.maximum(np.abs(ref), alpha))
    assert np.all(r.res[:r.M] < p.tol)
    assert np.all((r.E[:r.M] >= p.emin) & (r.E[:r.M] <= p.emax))


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_sampled_residuals_and_b_orthonormality(bench_problem, solved, prec):
    p = bench_problem
    r, X = solved[prec]
    alpha = max(abs(p.emin), abs(p.emax))
    rng = np.random.default_rng(77)
    idx = np.unique(np.concatenate([[0, r.M - 1], rng.choice(r.M, 6, replace=False)]))
    Xs = X[:, idx]
    lam = r.E[idx]
    AX = p.A @ Xs
    BX = p.B @ Xs
    R = AX - BX * lam
    res = np.abs(R).sum(axis=0) / (alpha * np.abs(BX).sum(axis=0))
    assert np.all(res < p.tol), res
    G = Xs.T @ BX
    assert np.max(np.abs(G - np.eye(len(idx)))) < 1e-10


def _fixture(name):
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"oracle_{name}.json")
    with open(path) as f:
        return json.load(f)


def _compare_with_oracle_run(p, name, r, X):
    """Parity with the oracle's stored run on the same workload (reading
    R14).  Eigenvalues: the 1e-10 relative bar, element by element.
    Eigenvectors: the sketch K = S2^T X_M X_M^H B S of the interval's
    B-orthogonal eigenprojector, with S, S2 seeded N x 16 blocks, does not
    depend on phases or rotations inside clusters.  Its relative difference
    is bounded by the projectors' distance, which the Davis-Kahan bound
    ||R|| / gap puts near 1e-7 at residuals below 1e-10 and end gaps of about
    2e-4; 1e-6 is the bar."""
    import sys
    import os

    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_oracle_fixtures as F

    ref = _fixture(name)
    assert F.inputs_match(p, ref), "generator output differs from the oracle's inputs beyond rounding"
    assert abs(p.emin - ref["emin"]) <= 1e-12 and abs(p.emax - ref["emax"]) <= 1e-12
    assert ref["info"] == 0
    assert r.info == 0 and r.M == ref["M"]
    alpha = max(abs(p.emin), abs(p.emax))
    e_ref = np.array(ref["E"][:ref["M"]])
    err = np.abs(r.E[:r.M] - e_ref) / np.maximum(np.abs(e_ref), alpha)
    assert err.max() <= 1e-10, err.max()
    assert np.all(r.res[:r.M] < p.tol) and np.all(np.array(ref["res"][:ref["M"]]) < p.tol)
    S, S2 = F.sketch_blocks(p.n)
    K = F.projector_sketch(X[:, :r.M], p.B, S, S2)
    K_ref = np.array(ref["sketch_re"]) + 1j * np.array(ref["sketch_im"])
    rel = np.linalg.norm(K - K_ref) / np.linalg.norm(K_ref)
    assert rel <= 1e-6, rel


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_matches_stored_oracle_run(bench_problem, solved, prec):
    r, X = solved[prec]
    _compare_with_oracle_run(bench_problem, "realgen_n4096", r, X)


def test_mixed_matches_fp64(bench_problem, solved):
    p = bench_problem
    rm, _ = solved["mixed"]
    rf, _ = solved["fp64"]
    assert rm.M == rf.M
    alpha = max(abs(p.emin), abs(p.emax))
    a, b = np.sort(rm.E[:rm.M]), np.sort(rf.E[:rf.M])
    assert np.all(np.abs(a - b) <= 1e-10 * np.maximum(np.abs(b), alpha))


# ---------------------------------------------------------------------------
# Complex Hermitian pencils with clustered spectra (the N = 8192, M0 = 600,
# Ne = 16 configuration), which exercise the adjoint solves; N = 2048 with the
# same recipe and node count as well.

def _check_hermitian(p, r, X):
    ref = _inside(p)
    assert r.info == 0
    assert r.M == len(ref)
    alpha = max(abs(p.emin), abs(p.emax))
    lam = r.E[:r.M]
    assert np.all(np.abs(lam - ref) <= 1e-10 * np.maximum(np.abs(ref), alpha))
    assert np.all(r.res[:r.M] < p.tol)
    rng = np.random.default_rng(78)
    idx = np.unique(np.concatenate([[0, r.M - 1], rng.choice(r.M, 6, replace=False)]))
    Xs = X[:, idx]
    BX = p.B @ Xs
    R = p.A @ Xs - BX * lam[idx]
    res = np.abs(R).sum(axis=0) / (alpha * np.abs(BX).sum(axis=0))
    assert np.all(res < p.tol), res
    G = Xs.conj().T @ BX
    assert np.max(np.abs(G - np.eye(len(idx)))) < 1e-10


def _solve_hermitian(p, prec):
    from paper_1203_4031_amd import feastx

    A = feastx.fortran_tensor(p.A)
    B = feastx.fortran_tensor(p.B)
    X = feastx.fortran_tensor(p.X0.astype(np.complex128))
    r = feastx.solve_device(A, B, p.emin, p.emax, p.m0, X, x0=True, ne=p.ne, tol=p.tol, precision=prec)
    torch.cuda.synchronize()
    return r, X.cpu().numpy()


@pytest.fixture(scope="module")
def herm2048():
    from paper_1203_4031_amd import workloads as W

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return W.dense_complex_hermitian(2048, 150, ne=16, tol=1e-10, seed=3002)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_complex_hermitian_clustered_n2048(herm2048, prec):
    r, X = _solve_hermitian(herm2048, prec)
    _check_hermitian(herm2048, r, X)


def test_complex_hermitian_config_n8192():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_4031_amd import workloads as W

    p = W.dense_complex_hermitian(8192, 400, m0=600, ne=16, tol=1e-10)
    for prec in ("mixed", "fp64"):
        print(f"N=8192 complex Hermitian, {prec}", flush=True)
        r, X = _solve_hermitian(p, prec)
        _check_hermitian(p, r, X)
        _compare_with_oracle_run(p, "hermgen_n8192", r, X)


# ---------------------------------------------------------------------------
# Batched problems of uneven N (the batched configuration's recipe: N
# log-uniform on [256, 2048], 5-15 % of each spectrum in the interval,
# M0 = 1.5 count, Ne = 8), 24 of them in one call.

def test_batched_uneven_sizes():
    from paper_1203_4031_amd import feastx, workloads as W

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    probs = W.batched_real_generalized(nprob=24, seed=4001)
    results = feastx.solve_batched([(p.A, p.B, p.emin, p.emax, p.m0, p.X0) for p in probs], precision="mixed",
                                   concurrency=4, ne=8, tol=1e-10)
    for p, r in zip(probs, results):
        ref = _inside(p)
        alpha = max(abs(p.emin), abs(p.emax))
        assert r.info == 0, (p.name, r.info)
        assert r.M == len(ref), p.name
        assert np.all(np.abs(r.E[:r.M] - ref) <= 1e-10 * np.maximum(np.abs(ref), alpha)), p.name
        assert np.all(r.res[:r.M] < p.tol), p.name
