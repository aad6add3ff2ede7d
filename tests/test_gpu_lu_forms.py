"""GPU parity of both factorisation schedules against the FP64 oracle.

The library factors the shifted matrices with panels in pairs below order
6144 and in blocks of four from there (feast_set_lu_form).  Here each
schedule is forced on small orders that end in a partial block (300 = 2*128
+ 44, 389 = 3*128 + 5, 520 = 4*128 + 8), so that the blocked schedule's
look-ahead corrections, its depth-128 products and its ragged tail run on
the GPU, and the solves are held to the single-solve bar of
tests/test_gpu_parity.py."""
import pytest

from paper_1203_4031_amd import feastx
from paper_1203_4031_amd import workloads as W

pytestmark = pytest.mark.gpu


def _problems():
    yield W.dense_real_generalized(300, count=30, seed=2111, tol=1e-10)
    yield W.dense_complex_hermitian(389, count=32, seed=3111, ne=16, tol=1e-10, nclusters=3)
    yield W.dense_real_generalized(520, count=40, seed=2112, tol=1e-10)


@pytest.fixture(scope="module")
def cases(orc):
    out = []
    for p in _problems():
        ref = orc.feast(p.A, p.B, p.emin, p.emax, p.m0, p.ne, p.tol, p.X0, hermitian=p.hermitian)
        assert ref.info == 0
        out.append((p, ref))
    return out


@pytest.mark.parametrize("form", ["blocks", "pairs"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("idx", [0, 1, 2])
def test_lu_form_matches_oracle(cases, form, precision, idx):
    from test_gpu_parity import _check_pairs

    p, ref = cases[idx]
    print(f"lu form {form} {precision} n {p.n}", flush=True)
    feastx.set_lu_form(form)
    try:
        r = feastx.solve(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, ne=p.ne, tol=p.tol, precision=precision)
    finally:
        feastx.set_lu_form("auto")
    _check_pairs(p, r, ref)
