"""The serving workload (complex Hermitian requests, N in {512, ..., 8192} with
p(N) ~ N^-2) against the FP64 oracle's stored runs:
tests/golden/oracle_serving_sample.json holds the oracle's info, eigenvalue
count and loops for every fifth request of the bench's 2000-request stream with
N <= 2048, and the in-interval eigenvalues of every fiftieth (written by
tests/golden/make_oracle_fixtures.py from the oracle alone).  Those requests go
through the request loop (8 slots) in each precision: the info must be the
oracle's, and for converged requests the count equal, the eigenvalues within
1e-10 relative (to max(|lambda|, max(|Emin|, |Emax|))) and every in-interval
residual within tol."""
import json
import os
import sys

import numpy as np
import pytest

from paper_1203_4031_amd import feastx
from paper_1203_4031_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "oracle_serving_sample.json")


@pytest.fixture(scope="module")
def stored():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_oracle_fixtures as F

    with open(FIXTURE) as f:
        ref = json.load(f)
    entries = [e for e in ref["entries"] if "E" in e]
    pool = {}
    for e in entries:
        key = (e["n"], e["k"])
        if key not in pool:
            print(f"generating pool matrix n {key[0]} k {key[1]}", flush=True)
            A, B, _ = W.serving_pool_matrix(*key)
            pool[key] = (A, B)
        assert F.serving_sample_matches(*pool[key], e), f"request {e['i']}: pool matrix differs beyond rounding"
    return ref, entries, pool


def test_sample_ran_in_the_oracle(stored):
    ref, entries, _ = stored
    assert ref["requests_in_stream"] == 2000 and ref["sampled"] == len(ref["entries"])
    assert all(e["n"] <= 2048 and e["i"] % 5 == 0 for e in ref["entries"])
    assert len(entries) >= 30


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_request_loop_matches_stored_oracle_runs(stored, precision):
    _, entries, pool = stored
    print(f"request loop {precision}: {len(entries)} requests", flush=True)
    srv = feastx.Server(slots=8, hbm_budget_gb=64.0)
    try:
        ids = [srv.submit(*pool[(e["n"], e["k"])], e["emin"], e["emax"], e["m0"],
                          X0=W.start_subspace(e["n"], e["m0"], e["x0_seed"]), ne=8, tol=1e-10,
                          precision=precision)
               for e in entries]
        rs = [srv.wait(i) for i in ids]
    finally:
        srv.close()
    for e, r in zip(entries, rs):
        assert r.info == e["info"], (e["i"], r.info, e["info"])
        assert r.M == e["M"], (e["i"], r.M, e["M"])
        if e["info"] != 0:
            continue
        E_ref = np.array(e["E"])
        alpha = max(abs(e["emin"]), abs(e["emax"]))
        err = np.abs(r.E[:r.M] - E_ref) / np.maximum(np.abs(E_ref), alpha)
        assert err.max() <= 1e-10, (e["i"], err.max())
        assert (r.res[:r.M] <= 1e-10).all(), (e["i"], r.res[:r.M].max())
