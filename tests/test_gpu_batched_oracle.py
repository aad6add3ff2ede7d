"""The batched workload (256 dense real symmetric generalized problems, N
log-uniform on [256, 2048], seeds 4001..4256) against the FP64 oracle's stored
runs: tests/golden/oracle_batched_n256.json holds, for every problem, the
oracle's info, eigenvalue count and loop count, and for every eighth problem
its in-interval eigenvalues and residuals (written by
tests/golden/make_oracle_fixtures.py from the oracle alone).  The 32 stored
problems go through one batched call per precision; each result must match the
oracle's count, its eigenvalues within 1e-10 relative (to max(|lambda|,
max(|Emin|, |Emax|))), and have every in-interval residual within tol."""
import json
import os
import sys

import numpy as np
import pytest

from paper_1203_4031_amd import feastx
from paper_1203_4031_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "oracle_batched_n256.json")


@pytest.fixture(scope="module")
def stored():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_oracle_fixtures as F

    with open(FIXTURE) as f:
        ref = json.load(f)
    entries = [e for e in ref["entries"] if "E" in e]
    specs = W.batched_specs()
    probs = []
    for e in entries:
        print(f"generating batched problem {e['i']} (n {e['n']})", flush=True)
        p = W.batched_problem(specs[e["i"]])
        assert F.batched_inputs_match(p, e), f"problem {e['i']}: generator output differs beyond rounding"
        # the interval the oracle ran on (its ends come out of LAPACK here)
        probs.append((p.A, p.B, e["emin"], e["emax"], p.m0, p.X0))
    return ref, entries, probs


def test_every_problem_ran_in_the_oracle(stored):
    ref, entries, _ = stored
    assert ref["problems"] == 256 and len(ref["entries"]) == 256
    assert all(e["info"] == 0 for e in ref["entries"])
    assert len(entries) == 32


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batched_matches_stored_oracle_runs(stored, precision):
    _, entries, probs = stored
    print(f"batched {precision}: {len(probs)} problems", flush=True)
    out = feastx.solve_batched(probs, concurrency=8, ne=8, tol=1e-10, precision=precision)
    for e, r in zip(entries, out):
        assert r.info == 0, (e["i"], r.info)
        assert r.M == e["M"], (e["i"], r.M, e["M"])
        E_ref = np.array(e["E"])
        alpha = max(abs(e["emin"]), abs(e["emax"]))
        err = np.abs(r.E[:r.M] - E_ref) / np.maximum(np.abs(E_ref), alpha)
        assert err.max() <= 1e-10, (e["i"], err.max())
        assert (r.res[:r.M] <= 1e-10).all(), (e["i"], r.res[:r.M].max())
