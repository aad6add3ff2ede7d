"""GPU parity for the contour options (fpm(16) trapezoidal rule, fpm(18)
ellipses, caller-supplied nodes) against the FP64 oracle: the library, given
the same rule, finds the same eigenpairs (the single-solve bar of
tests/test_gpu_parity.py).  Sizes and node counts differ from the skipped
cases in tests/test_gpu_parity.py."""
import numpy as np
import pytest

from paper_1203_4031_amd import feastx
from paper_1203_4031_amd import workloads as W

pytestmark = pytest.mark.gpu

# The trapezoidal cases vary the one that stalled a GPU run silently
# (test_gpu_parity.py::test_other_contours_match_oracle, trapezoidal, FP64,
# N=300, Ne=10).  Its cause is not established, so no trapezoidal case runs
# on the GPU until it is; the rule's nodes, weights and filter are checked
# against the oracle on the CPU (tests/test_abi.py).
TRAPEZOID_STALL = ("variant of the trapezoidal case that stalled a GPU run with no cause found; "
                   "kept off the GPU until the cause is shown and fixed")

CASES = [
    # (integration, ellipse, custom, precision, n, ne)
    (0, 50, False, "fp64", 256, 12),
    (0, 200, True, "mixed", 256, 12),
    pytest.param(1, 100, False, "mixed", 256, 12, marks=pytest.mark.skip(reason=TRAPEZOID_STALL)),
    pytest.param(1, 60, True, "fp64", 240, 9, marks=pytest.mark.skip(reason=TRAPEZOID_STALL)),
]


@pytest.mark.parametrize("integration,ellipse,custom,precision,n,ne", CASES)
def test_contour_options_match_oracle(orc, integration, ellipse, custom, precision, n, ne):
    from test_gpu_parity import _check_pairs

    p = W.dense_real_generalized(n, count=24, seed=2400 + n + ne, tol=1e-10)
    zne = wne = None
    if custom:
        zne, wne = orc.contour(p.emin, p.emax, ne, integration, ellipse)
    print(f"contour case rule {integration} ellipse {ellipse} custom {custom} {precision} n {n} ne {ne}",
          flush=True)
    ref = orc.feast(p.A, p.B, p.emin, p.emax, p.m0, ne, p.tol, p.X0, integration=integration, ellipse=ellipse,
                    zne=zne, wne=wne)
    assert ref.info == 0
    r = feastx.solve(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, ne=ne, tol=p.tol, precision=precision,
                     integration=0 if custom else integration, ellipse=100 if custom else ellipse, zne=zne,
                     wne=wne)
    _check_pairs(p, r, ref)
