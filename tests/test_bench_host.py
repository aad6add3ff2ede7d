"""Host-side checks of bench.py (no GPU): the one-GPU rule, argument
validation, and that the HBM traffic figures it reports belong to the kernel
sources in the tree (bench.py reports them only while the sources hash to the
value they were measured with, so a kernel change without new counters
shows up here first)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bad_precision_list():
    r = _bench("--precisions", "fp32")
    assert r.returncode != 0 and "--precisions" in r.stderr


def test_traffic_table_matches_the_sources():
    import bench

    sha = bench.kernel_sources_sha256()
    assert len(sha) == 64 and sha == bench.kernel_sources_sha256()
    assert "hermgen_n8192_mixed" in bench.TRAFFIC   # the headline workload's faster precision
    for key, (nbytes, key_sha, tiles) in bench.TRAFFIC.items():
        assert 1e7 < nbytes < 1e11, key
        assert key_sha == sha, f"{key}: traffic measured on other kernel sources; take the counters again"
        assert set(tiles) == {"depth<=64", "deeper"}


def test_roofline_kernel_names_and_peaks():
    import bench

    class Tiles:   # the default table, without the library
        @staticmethod
        def tiles():
            return {p: {"depth<=64": 0, "deeper": 0} for p in ("complex64", "complex128")}

    n32, p32 = bench.roofline_kernel(Tiles, "mixed", False)
    n64, p64 = bench.roofline_kernel(Tiles, "fp64", True)
    nmx, pmx = bench.roofline_kernel(Tiles, "mixed", True)
    assert (p32, p64, pmx) == (157.3, 78.6, 78.6)
    assert n32.startswith("gemm_kernel<float") and n64.startswith("gemm_kernel<double")
    assert nmx.startswith("gemm_kernel<double") and "node group" in nmx
