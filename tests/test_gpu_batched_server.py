"""Batched solves and the request loop: every result equals the same problem
solved alone (same kernels, same inputs), and agrees with the FP64 oracle."""
import time

import numpy as np
import pytest

from paper_1203_4031_amd import feastx
from paper_1203_4031_amd import workloads as W

pytestmark = pytest.mark.gpu


def _same(r, alone, tol=1e-12):
    assert r.info == alone.info == 0
    assert r.M == alone.M and r.m0 == alone.m0
    scale = np.maximum(np.abs(alone.E[:r.M]), 1e-3)
    assert np.max(np.abs(r.E[:r.M] - alone.E[:r.M]) / scale) <= tol
    assert np.abs(r.res[:r.M] - alone.res[:r.M]).max() <= 1e-12


@pytest.fixture(scope="module")
def real_batch():
    # uneven sizes, as in the batched workload (N log-uniform, 5-15 % of the spectrum)
    return [W.dense_real_generalized(n, count=c, seed=4100 + i, tol=1e-10)
            for i, (n, c) in enumerate([(256, 20), (389, 40), (300, 18), (512, 60), (333, 30),
                                        (270, 25)])]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batched_equals_alone(real_batch, precision):
    print(f"batched {precision}", flush=True)
    probs = [(p.A, p.B, p.emin, p.emax, p.m0, p.X0) for p in real_batch]
    out = feastx.solve_batched(probs, concurrency=3, ne=8, tol=1e-10, precision=precision)
    for p, r in zip(real_batch, out):
        alone = feastx.solve(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, ne=8, tol=1e-10,
                             precision=precision)
        _same(r, alone)
        assert r.M == p.count_in_interval()
        assert (r.res[:r.M] < 1e-10).all()


def test_batched_matches_oracle(orc, real_batch):
    p = real_batch[1]
    ref = orc.feast(p.A, p.B, p.emin, p.emax, p.m0, p.ne, p.tol, p.X0)
    r = feastx.solve_batched([(p.A, p.B, p.emin, p.emax, p.m0, p.X0)], ne=8, tol=1e-10,
                             precision="mixed")[0]
    assert r.M == ref.M
    alpha = max(abs(p.emin), abs(p.emax))
    assert np.max(np.abs(r.E[:r.M] - ref.E[:r.M]) / np.maximum(np.abs(ref.E[:r.M]), alpha)) < 1e-10


def test_server_mix_equals_alone():
    """Requests of mixed size arrive while others run; each result is the
    same as that request solved alone."""
    probs = [W.dense_complex_hermitian(n, count=c, seed=5100 + i, ne=8, tol=1e-10, nclusters=3)
             for i, (n, c) in enumerate([(256, 20), (384, 30), (200, 12), (320, 24), (256, 16)])]
    srv = feastx.Server(slots=3, hbm_budget_gb=8.0)
    try:
        ids = []
        for i, p in enumerate(probs):
            ids.append(srv.submit(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, ne=8, tol=1e-10,
                                  precision="mixed"))
            time.sleep(0.002 * i)
        # poll until the first finishes, then wait for the rest
        got = None
        for _ in range(20000):
            got = srv.poll(ids[0])
            if got is not None:
                break
            time.sleep(0.001)
        results = [got if got is not None else srv.wait(ids[0])] + [srv.wait(i) for i in ids[1:]]
    finally:
        srv.close()
    for p, r in zip(probs, results):
        alone = feastx.solve(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, ne=8, tol=1e-10,
                             precision="mixed")
        _same(r, alone)
        assert r.latency_ms >= r.run_ms >= 0 and r.queue_ms >= 0


def test_server_admission_budget_serialises():
    """With a budget below two requests' footprint, requests still all
    complete (admitted one at a time)."""
    p = W.dense_real_generalized(300, count=20, seed=5200, tol=1e-10)
    srv = feastx.Server(slots=4, hbm_budget_gb=0.01)
    try:
        ids = [srv.submit(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, ne=8, tol=1e-10) for _ in range(3)]
        rs = [srv.wait(i) for i in ids]
    finally:
        srv.close()
    for r in rs:
        assert r.info == 0 and r.M == p.count_in_interval()
    # admitted one at a time: each waits for the previous
    assert rs[2].queue_ms >= rs[0].run_ms * 0.5


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batched_one_round_jacobi(precision):
    """Reduced problems of m <= 32 give the block Jacobi a single round per
    sweep, where every workgroup rewrites its off-norm partial before the
    next grid barrier; the partials alternate by sweep parity so that no
    workgroup can read a partial of the next sweep.  Sixteen such problems
    at the executor's full 8 slots, each checked against its spectrum."""
    probs = [W.dense_real_generalized(n, count=c, seed=4300 + i, tol=1e-10)
             for i, (n, c) in enumerate([(256, 12), (300, 16), (270, 14), (320, 18)] * 4)]
    assert all(p.m0 <= 32 for p in probs)
    print(f"batched one-round Jacobi {precision}", flush=True)
    out = feastx.solve_batched([(p.A, p.B, p.emin, p.emax, p.m0, p.X0) for p in probs], concurrency=8, ne=8,
                               tol=1e-10, precision=precision)
    for p, r in zip(probs, out):
        s = p.spectrum
        ref = s[(s >= p.emin) & (s <= p.emax)]
        alpha = max(abs(p.emin), abs(p.emax))
        assert r.info == 0, (p.name, r.info)
        assert r.M == len(ref), p.name
        assert np.all(np.abs(r.E[:r.M] - ref) <= 1e-10 * np.maximum(np.abs(ref), alpha)), p.name
        assert np.all(r.res[:r.M] < 1e-10), p.name
