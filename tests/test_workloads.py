"""Properties of the seeded input generators (no method arithmetic): the
spectra they promise, the interval and region rules, and determinism."""
import numpy as np
import scipy.linalg as sl

from paper_1203_4031_amd import workloads as W


def test_sign_probes_are_signs_and_seeded():
    a = W.sign_probes(50, 7, seed=3)
    assert a.shape == (50, 7) and a.flags.f_contiguous
    assert set(np.unique(a)) == {-1.0, 1.0}
    assert np.array_equal(a, W.sign_probes(50, 7, seed=3))
    assert not np.array_equal(a, W.sign_probes(50, 7, seed=4))


def test_slice_bounds_hold_the_requested_counts():
    rng = np.random.default_rng(5)
    spec = np.sort(rng.uniform(-1, 1, 200))
    counts = [7, 13, 4, 20]
    b = W.slice_bounds(spec, 30, counts)
    assert (np.diff(b) > 0).all()
    for k, c in enumerate(counts):
        assert np.count_nonzero((spec >= b[k]) & (spec <= b[k + 1])) == c
    # every bound sits at the midpoint of its gap
    idx = 30 + np.concatenate([[0], np.cumsum(counts)])
    assert np.allclose(b, 0.5 * (spec[idx - 1] + spec[idx]))


def test_dense_general_spectrum_and_region():
    for real, gen in [(False, True), (True, False), (True, True)]:
        p = W.dense_general(60, count=6, seed=77, real=real, generalized=gen)
        full = sl.eig(p.A, p.B, right=False)
        assert max(np.abs(full - l).min() for l in p.spectrum) < 1e-9
        inside = np.abs(p.spectrum - p.emin) < p.emax
        assert inside.sum() == p.meta["count"] >= 6
        if real:
            assert np.isrealobj(p.A) and p.emin.imag == 0.0
            got = p.spectrum[inside]
            assert max(np.abs(got - np.conj(l)).min() for l in got) < 1e-12   # conjugate-closed
        assert p.X0.shape == (60, 2 * p.m0)
