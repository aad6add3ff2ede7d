"""The product kernel's tile autotuner: it measures every variant, installs a
valid table, and a solve gives the same bits whichever variants the table
selects (every variant accumulates over the depth in the same order)."""
import numpy as np
import pytest

from paper_1203_4031_amd import feastx
from paper_1203_4031_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture
def restore_tiles():
    before = feastx.tiles()
    yield
    feastx.set_tiles(before)


def test_autotune_measures_every_variant(restore_tiles):
    print("autotune n=512 m0=64 ne=8", flush=True)
    t = feastx.autotune(512, 64, 8)
    for prec in ("complex64", "complex128"):
        for cls in ("depth<=64", "deeper"):
            rates = t["tflops"][prec][cls]
            assert len(rates) == feastx.TILE_VARIANTS and all(r > 0 for r in rates), (prec, cls, rates)
            v = t["choice"][prec][cls]
            assert 0 <= v < feastx.TILE_VARIANTS
            # the default stays unless another variant is at least 5 % faster
            assert v == 0 or rates[v] >= 1.05 * rates[0]
    assert feastx.tiles() == t["choice"]


@pytest.mark.parametrize("case", ["real_mixed", "complex_fp64"])
def test_every_variant_gives_the_same_bits(restore_tiles, case):
    if case == "real_mixed":
        p, precision = W.dense_real_generalized(300, count=24, seed=4301, tol=1e-10), "mixed"
    else:
        p, precision = W.dense_complex_hermitian(300, count=24, seed=4302, tol=1e-10), "fp64"
    out = []
    for v in range(feastx.TILE_VARIANTS):
        print(f"{case}: all products on tile variant {v}", flush=True)
        feastx.set_tiles({q: {c: v for c in ("depth<=64", "deeper")} for q in ("complex64", "complex128")})
        r = feastx.solve(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, ne=8, tol=1e-10, precision=precision)
        assert r.info == 0 and r.M == p.count_in_interval()
        out.append(r)
    for r in out[1:]:
        assert r.loop == out[0].loop and r.M == out[0].M
        assert np.array_equal(r.E, out[0].E)
        assert np.array_equal(r.X, out[0].X)
        assert np.array_equal(r.res, out[0].res)
