"""Spectrum slicing on the GPU (section "Multiple search intervals and
FEAST-MPI": neighbouring intervals without overlap, each an independent
FEAST run), through feast_solve_slices_{d,z}.

* Each slice is compared with the FP64 oracle run on that interval alone,
  with the same start subspace, to the single-interval bar (eigenvalues within
  1e-10 max(|lambda|, alpha), the same M, residuals below tol, the same
  invariant subspace).
* Together the slices find every eigenvalue LAPACK finds in the union of the
  intervals, and eigenvectors of different slices are B-orthogonal (the
  guide expects overall orthogonality to be preserved).
* With auto_m0 the subspace sizes come from the stochastic count estimate;
  every slice still finds its exact count."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1203_4031_amd import feastx  # noqa: E402
from paper_1203_4031_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _check_slice(p, emin, emax, r, ref):
    alpha = max(abs(emin), abs(emax))
    assert r.info == 0 and ref.info == 0, (r.info, ref.info)
    assert r.M == ref.M
    M = r.M
    err = np.abs(r.E[:M] - ref.E[:M]) / np.maximum(np.abs(ref.E[:M]), alpha)
    assert err.max() <= 1e-10, err.max()
    assert (r.res[:M] < p.tol).all()
    B = np.eye(p.n) if p.B is None else p.B
    s = np.linalg.svd(ref.X[:, :M].conj().T @ B @ r.X[:, :M], compute_uv=False)
    assert s.min() > 1 - 1e-8, s.min()


def _check_union(p, bounds, rs):
    s = np.sort(p.spectrum)
    inside = s[(s >= bounds[0]) & (s <= bounds[-1])]
    lam = np.sort(np.concatenate([r.E[:r.M] for r in rs]))
    assert lam.size == inside.size
    alpha = max(abs(bounds[0]), abs(bounds[-1]))
    assert (np.abs(lam - inside) <= 1e-10 * np.maximum(np.abs(inside), alpha)).all()
    B = np.eye(p.n) if p.B is None else p.B
    X = np.concatenate([r.X[:, :r.M] for r in rs], axis=1)
    G = X.conj().T @ B @ X
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_slices_match_oracle_per_interval(orc, precision):
    p = W.dense_real_generalized(300, count=30, seed=2107, tol=1e-10)
    counts = [9, 14, 11]
    start = int(np.searchsorted(np.sort(p.spectrum), p.emin))
    bounds = W.slice_bounds(p.spectrum, start, counts)
    m0s = [int(np.ceil(1.5 * c)) + 2 for c in counts]
    X0 = [W.start_subspace(p.n, m, seed=2108 + k) for k, m in enumerate(m0s)]
    print(f"slices {precision} bounds {bounds}", flush=True)
    rs = feastx.solve_slices(p.A, p.B, bounds, m0s, X0=X0, concurrency=3, ne=8, tol=p.tol,
                             precision=precision)
    for k, r in enumerate(rs):
        assert (r.emin, r.emax) == (bounds[k], bounds[k + 1])
        ref = orc.feast(p.A, p.B, bounds[k], bounds[k + 1], m0s[k], 8, p.tol, X0[k])
        _check_slice(p, bounds[k], bounds[k + 1], r, ref)
        assert r.M == counts[k]
    _check_union(p, bounds, rs)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_slices_auto_m0_complex(precision):
    p = W.dense_complex_hermitian(256, count=40, seed=3107, ne=8, tol=1e-10, nclusters=3)
    counts = [8, 12, 6, 14]
    start = int(np.searchsorted(np.sort(p.spectrum), p.emin))
    bounds = W.slice_bounds(p.spectrum, start, counts)
    print(f"auto-m0 slices {precision} bounds {bounds}", flush=True)
    rs = feastx.solve_slices(p.A, p.B, bounds, 64, concurrency=4, auto_m0=True, ne=8, tol=p.tol,
                             precision=precision)
    for k, r in enumerate(rs):
        assert r.info == 0, (k, r.info)
        assert r.M == counts[k]
        assert r.m0 <= 64
        assert (r.res[:r.M] < p.tol).all()
    _check_union(p, bounds, rs)


def test_slices_on_device_arrays_match_host_arrays():
    """device = 1 (A, B and every X in HBM) gives the same results as host
    arrays staged by the library."""
    p = W.dense_real_generalized(300, count=30, seed=2107, tol=1e-10)
    counts = [9, 14, 11]
    start = int(np.searchsorted(np.sort(p.spectrum), p.emin))
    bounds = W.slice_bounds(p.spectrum, start, counts)
    m0s = [int(np.ceil(1.5 * c)) + 2 for c in counts]
    X0 = [W.start_subspace(p.n, m, seed=2108 + k) for k, m in enumerate(m0s)]
    host = feastx.solve_slices(p.A, p.B, bounds, m0s, X0=X0, concurrency=3, ne=8, tol=p.tol, precision="mixed")
    A, B = feastx.fortran_tensor(p.A), feastx.fortran_tensor(p.B)
    dev = feastx.solve_slices(A, B, bounds, m0s, X0=[feastx.fortran_tensor(x) for x in X0], concurrency=3, ne=8,
                              tol=p.tol, precision="mixed")
    torch.cuda.synchronize()
    for h, d in zip(host, dev):
        assert d.info == h.info == 0 and d.M == h.M and d.loop == h.loop
        assert np.array_equal(d.E, h.E)
        assert np.array_equal(d.X.cpu().numpy(), h.X)
