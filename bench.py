"""FEAST solves/s on one MI355X.

Headline: the largest single-GPU workload, a dense complex Hermitian
generalized problem A x = lambda B x with N = 8192 (A = U diag(lambda) U^H,
Haar U, clustered spectrum; B = I + 0.1 H), M0 = 600, Ne = 16 Gauss-Legendre
half-contour nodes, about 400 eigenvalues in the interval, tol 1e-10.  Both
precisions are timed the same way, K solves each: mixed (complex64 factors
and solves on the FP32 matrix cores, FP64 residual correction, complex128 for
the contour nodes where complex64 error would limit the iteration) and FP64
(complex128 throughout).  `value` is the faster one's solves/s, `precision`
names it and `dtype` is its arithmetic; both are reported in full.

One step = one complete feast_solve call (all contour nodes: shift, LU,
solves, quadrature, Rayleigh-Ritz, reduced eigensolve, residuals, every FEAST
loop until convergence) on inputs already resident in HBM.

Also measured, each in its own object of the JSON line:
  dense_real_n4096   the N = 4096 real symmetric generalized workload
                     (M0 = 300, Ne = 8, 200 eigenvalues), mixed and FP64,
                     with its own roofline and shifted-LU rates; spectrum
                     slicing, non-Hermitian FEAST and the count estimate on it
  batched            256 independent real generalized problems of uneven N
                     (log-uniform on [256, 2048]) through the batched entry
                     point, mixed and FP64
  serving            Poisson request stream (200 requests/s) of complex
                     Hermitian problems of N in {512, ..., 8192}, p(N) ~ N^-2,
                     through the request loop: throughput, p50/p99 latency,
                     queue depth, mixed and FP64
  cpu_baseline       the FP64 oracle on a bounded sample of the headline workload

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3      # TFLOP/s, dense
PEAK_FP64_MFMA = 78.6

# HBM bytes per launch of the roofline kernel (FETCH_SIZE + WRITE_SIZE, each
# scaled by a 256 MiB copy's reading, averaged over the launches of one
# solve), from the rocprofv3 counter passes summarised in profiles/, per
# workload and precision, with the tile table they ran under.  Each holds only
# for the sources it was measured on -- the kernel itself and every file that
# launches it in a solve (the FP64 reduced-problem kernels in jacobi.hpp and
# bortho.hpp and the tuner in tune.hpp do not) -- and for that table:
# `traffic` is null otherwise.
TRAFFIC = {   # profiles/hbm_traffic_hermgen_n8192_m0600_mixed.md, profiles/hbm_traffic_realgen_n4096_m0300.md
    "hermgen_n8192_mixed": (7.8826e+08, "8eb62fb1a654bb3796540844ed72d84486c0840249cd6c619d3dbdfdff99672e",
                            {"depth<=64": 0, "deeper": 0}),
    "realgen_n4096_mixed": (1.1890e+08, "8eb62fb1a654bb3796540844ed72d84486c0840249cd6c619d3dbdfdff99672e",
                            {"depth<=64": 0, "deeper": 0}),
}


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1203_4031_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".hpp", ".h")) and name not in ("jacobi.hpp", "bortho.hpp", "tune.hpp"):
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- input generation
# All inputs are generated before any GPU measurement, so that no timed
# region shares the host with generation: the large pencils in this process
# (all BLAS threads), then the many small ones in single-threaded worker
# processes.

def _limit_threads(n):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(n)
    except Exception:
        pass


def generate_small(batched_specs, pool_keys, workers=16):
    """Batched problems and serving pool matrices in single-threaded worker
    processes; a progress line every 20 s."""
    import concurrent.futures as cf
    import multiprocessing as mp

    t0 = time.perf_counter()
    # one BLAS/OpenMP thread per worker: the variables are read when each
    # spawned process loads its libraries (numpy's and scipy's own BLAS);
    # this process's libraries are loaded already
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"),
                                    initializer=_limit_threads, initargs=(1,)) as ex:
            fp = [ex.submit(_gen_pool, n, k) for n, k in pool_keys]
            fb = [ex.submit(_gen_batched, sp) for sp in batched_specs]
            pending = set(fp + fb)
            while pending:
                done, pending = cf.wait(pending, timeout=20)
                log(f"generating: {len(fp) + len(fb) - len(pending)} of {len(fp) + len(fb)} small inputs "
                    f"({time.perf_counter() - t0:.0f} s)")
            return [f.result() for f in fb], [f.result() for f in fp]
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _gen_batched(spec):
    from paper_1203_4031_amd import workloads as W
    p = W.batched_problem(spec)
    return (p.A, p.B, p.emin, p.emax, p.m0, p.X0, p.count_in_interval())


def _gen_pool(n, k):
    from paper_1203_4031_amd import workloads as W
    return (n, k) + W.serving_pool_matrix(n, k)


# ---------------------------------------------------------------- single solves

def run_steps(feastx, torch, A, B, X0, X, p, precision, steps, timing):
    feastx.set_timing(timing)
    # product launches: all of them (time, flops, count), then the shifted
    # LU's own (time, flops, count), then the factor stage (time, flops)
    times, results, lu = [], [], [0.0, 0.0, 0, 0.0, 0.0, 0, 0.0, 0.0]
    stream = torch.cuda.current_stream()
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X.copy_(X0)
        r = feastx.solve_device(A, B, p.emin, p.emax, p.m0, X, stream=stream, x0=True, ne=p.ne,
                                tol=p.tol, precision=precision)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        results.append(r)
        if timing:
            s = feastx.stats()
            lu[0] += s.t_lu_gemm
            lu[1] += s.lu_gemm_flops
            lu[2] += s.lu_gemm_launches
            lu[3] += s.t_lu_update
            lu[4] += s.lu_update_flops
            lu[5] += s.lu_update_launches
            lu[6] += s.t_factor
            lu[7] += s.factor_flops
    feastx.set_timing(False)
    return times, results, lu


def check(results, p, expected_m):
    for r in results:
        if r.info != 0:
            raise SystemExit(f"{p.name}: solve failed: info {r.info}")
        if r.M != expected_m:
            raise SystemExit(f"{p.name}: eigenvalue count {r.M} != {expected_m}")
        if not (r.res[:r.M] <= p.tol).all():
            raise SystemExit(f"{p.name}: residual above tol")


def stage_ms(feastx):
    st = feastx.stats()
    d = {k: round(getattr(st, k), 3) for k in ("t_total", "t_shift", "t_factor", "t_solve", "t_accum",
                                                "t_rr", "t_reduced", "t_resid")}
    d["eig_calls"], d["eig_sweeps"], d["fp64_nodes"] = st.eig_calls, st.eig_sweeps, st.fp64_nodes
    return d


PRECISION_TEXT = {
    "mixed": "mixed (complex64 factors and solves, complex128 for the nodes where complex64 error would limit "
             "the iteration, FP64 residual correction)",
    "fp64": "FP64 (complex128 factors and solves, FP64 Rayleigh-Ritz)",
}

# tile variants of the complex product kernel (the autotuner's table picks one
# per precision and depth class)
TILE_KERNELS = {
    "complex64": ["gemm_kernel<float, true, false, 64, 64, 8, 32, 32, 4, true, true>",
                  "gemm_kernel<float, true, false, 128, 64, 8, 32, 32, 2, true, true>",
                  "gemm_kernel<float, true, false, 64, 64, 16, 32, 32, 4, true, true>"],
    "complex128": ["gemm_kernel<double, true, false, 64, 64, 8, 32, 32, 3, true, true>",
                   "gemm_kernel<double, true, false, 64, 64, 8, 64, 16, 3, true, true>",
                   "gemm_kernel<double, true, false, 64, 64, 16, 32, 32, 2, true, true>"],
}


def roofline_kernel(feastx, best, c128):
    """Name, description and peak of the roofline kernel of precision `best`
    under the installed tile table: the complex128 product when `c128` (FP64,
    and mixed solves with at least half of their nodes in complex128, whose
    products take most of the time), else the complex64 product."""
    prec = "complex128" if c128 else "complex64"
    ch = feastx.tiles()[prec]
    names = {cls: TILE_KERNELS[prec][v] for cls, v in ch.items()}
    if not c128:
        what = ("complex64 matrix product on the FP32 matrix cores (LU trailing updates and triangular-solve "
                "updates), every launch of the timed solves; products of at most 32 columns use the 64x32 "
                "instance gemm_kernel<float, true, false, 64, 32, 16, 32, 16, 4, true, true> and the adjoint "
                "solves of Hermitian pencils the A^H instances gemm_kernel<float, true, true, ...>, all counted")
        peak = PEAK_FP32_MFMA
    else:
        what = ("complex128 matrix product on the FP64 matrix cores (LU trailing updates, triangular-solve "
                "updates and, for complex pencils, the Rayleigh-Ritz and Ritz-vector products), every launch of "
                "the timed solves; the adjoint solves of Hermitian pencils use the A^H instances "
                "gemm_kernel<double, true, true, ...>, counted too")
        if best == "mixed":
            what += ("; in this mixed solve the complex128 node group (at least half of the nodes) takes most "
                     "of the product time, so its launches are the ones timed")
        peak = PEAK_FP64_MFMA
    if names["depth<=64"] == names["deeper"]:
        name = names["deeper"]
    else:
        name = f"{names['depth<=64']} (depth <= 64) and {names['deeper']} (deeper)"
    return f"{name}: {what}", peak


def time_precision(feastx, torch, A, B, X0, X, p, precision, steps, expected):
    """`steps` solves back to back, bracketed by device synchronisations."""
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    times, res, _ = run_steps(feastx, torch, A, B, X0, X, p, precision, steps, False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    stages = stage_ms(feastx)
    check(res, p, expected)
    loops = res[-1].loop + 1
    log(f"{p.name} {precision}: {steps} solves in {wall:.3f}s, {loops} loops")
    lat = np.array(times) * 1e3
    return {"solves_per_s": steps / wall, "ms_per_solve": wall / steps * 1e3,
            "eigenpairs_per_s": steps / wall * expected, "loops": loops,
            "latency_ms_single_solves": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "stage_ms_last_solve": stages}


def measure_single(feastx, torch, p, steps, warmup, roofline_steps, traffic_key, precisions=("mixed", "fp64")):
    """Mixed and FP64 solves of one workload with inputs in HBM: solves/s,
    latency and stage times of each precision; the faster one is the
    workload's figure, with the roofline of its complex product kernel."""
    expected = p.count_in_interval()
    A = feastx.fortran_tensor(p.A)
    B = feastx.fortran_tensor(p.B)
    X0 = feastx.fortran_tensor(p.X0.astype(np.complex128) if p.hermitian else p.X0)
    X = X0.clone(memory_format=torch.contiguous_format).t().contiguous().t()
    for precision in precisions:
        run_steps(feastx, torch, A, B, X0, X, p, precision, warmup, False)
    per = {pr: time_precision(feastx, torch, A, B, X0, X, p, pr, steps, expected) for pr in precisions}
    best = max(per, key=lambda pr: per[pr]["solves_per_s"])
    # the same solves of the faster precision with a HIP event pair around
    # every launch of its complex product kernel (on the library's stream)
    _, res_t, lu = run_steps(feastx, torch, A, B, X0, X, p, best, roofline_steps, True)
    check(res_t, p, expected)
    # the library times the complex128 launches of FP64 solves and of mixed
    # solves with at least half of their nodes in complex128
    c128 = best == "fp64" or 2 * feastx.stats().fp64_nodes >= p.ne
    kname, peak = roofline_kernel(feastx, best, c128)
    achieved = lu[1] / (lu[0] * 1e-3) / 1e12 if lu[0] > 0 else 0.0
    traffic_bytes, traffic_sha, traffic_tiles = TRAFFIC.get(f"{traffic_key}_{best}", (None, "", None))
    prec_name = "complex128" if c128 else "complex64"
    traffic_ok = (traffic_bytes is not None and kernel_sources_sha256() == traffic_sha
                  and feastx.tiles()[prec_name] == traffic_tiles)
    out = {
        "precision": best,
        "solves_per_s": per[best]["solves_per_s"],
        "ms_per_solve": per[best]["ms_per_solve"],
        "eigenpairs_per_s": per[best]["eigenpairs_per_s"],
        "count": expected,
        "loops": per[best]["loops"],
        "mixed": per.get("mixed"),
        "fp64": per.get("fp64"),
        "mixed_over_fp64": (per["mixed"]["solves_per_s"] / per["fp64"]["solves_per_s"]
                            if len(per) == 2 else None),
        "roofline": {"kernel": kname, "bound": "mfma", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic_bytes if traffic_ok else None,
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "flop_count": "algorithmic, 8 per complex multiply-add; the kernel's three-multiplication "
                                   "form issues 6 of them to the matrix cores (executed rate 0.75 x achieved)",
                     "launches": lu[2], "avg_launch_ms": lu[0] / max(lu[2], 1),
                     "flops_per_launch": lu[1] / max(lu[2], 1),
                     "measured_over": f"{roofline_steps} extra {best} solves with per-launch HIP events"},
    }
    upd = lu[4] / (lu[3] * 1e-3) / 1e12 if lu[3] > 0 else 0.0
    fac = lu[7] / (lu[6] * 1e-3) / 1e12 if lu[6] > 0 else 0.0
    blocks = np.array_equal(feastx.lu_schedule(p.n, True), feastx.lu_schedule(p.n, True, "blocks"))
    out["shifted_lu"] = {"precision": best,
                         "schedule": ("blocks of four panels (depth-128 trailing products)" if blocks
                                      else "panels in pairs (depth-64 trailing products)"),
                         "update_achieved": upd, "update_frac": upd / peak,
                         "update_launches": lu[5], "unit": "TFLOP/s", "peak": peak,
                         "factor_ms": lu[6] / max(roofline_steps, 1),
                         "factor_rate": fac, "factor_frac": fac / peak,
                         "note": "update_*: the LU's own launches of the roofline kernel (8 flops per complex "
                                 "multiply-add); factor_*: the whole factor stage (shift, panels, interchanges, "
                                 "products, solve form W) against (8/3) N^3 per node and the peak of the roofline "
                                 "kernel's precision, timed with per-launch events on (so slightly slow); in a "
                                 "mixed solve it covers both node groups"}
    return out, (A, B, X0, X)


# ---------------------------------------------------------------- extras on the N = 4096 pencil

def count_estimate(feastx, torch, W, A, B, p, expected, steps=5):
    """Stochastic count estimate (fpm(14) = 2) on the same pencil with the
    guide's suggested small settings: M0 = 16 +-1 probes, Ne = 3, one contour."""
    m0, ne = 16, 3
    P0 = feastx.fortran_tensor(W.sign_probes(p.n, m0, seed=2106))
    P = P0.clone(memory_format=torch.contiguous_format).t().contiguous().t()
    stream = torch.cuda.current_stream()
    times, r = [], None
    for i in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.copy_(P0)
        r = feastx.solve_device(A, B, p.emin, p.emax, m0, P, stream=stream, x0=True, ne=ne, tol=p.tol,
                                precision="mixed", mode=2)
        torch.cuda.synchronize()
        if i:
            times.append(time.perf_counter() - t0)
        if r.info != 5:
            raise SystemExit(f"count estimate failed: info {r.info}")
    return {"m0": m0, "ne": ne, "precision": "mixed", "ms": float(np.mean(times)) * 1e3, "estimate": r.M,
            "running_average_last": float(r.res[-1]), "count": expected,
            "sampling_sd": float(np.sqrt(2.0 * expected / m0))}


def slicing(feastx, torch, W, A, B, p, expected, single_ms, steps=3):
    """Spectrum slicing on the same pencil: the interval's eigenvalues split
    into 4 neighbouring slices of equal count (bounds at gap midpoints), each
    with M0 = 1.5 x its count, solved as one batched job on device arrays
    (mixed precision, 4 concurrent slices)."""
    nsl = 4
    counts = [expected // nsl] * nsl
    counts[-1] += expected - sum(counts)
    spec = np.sort(p.spectrum)
    start = int(np.searchsorted(spec, p.emin))
    bounds = W.slice_bounds(spec, start, counts)
    m0s = [int(np.ceil(1.5 * c)) for c in counts]
    X0 = [feastx.fortran_tensor(W.start_subspace(p.n, m, seed=2200 + k)) for k, m in enumerate(m0s)]
    times, rs = [], None
    for i in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = feastx.solve_slices(A, B, bounds, m0s, X0=X0, concurrency=nsl, ne=p.ne, tol=p.tol,
                                 precision="mixed")
        torch.cuda.synchronize()
        if i:
            times.append(time.perf_counter() - t0)
    found = sum(r.M for r in rs)
    if any(r.info != 0 for r in rs) or found != expected:
        raise SystemExit(f"slicing failed: infos {[r.info for r in rs]}, found {found} of {expected}")
    ms = float(np.mean(times)) * 1e3
    return {"slices": nsl, "counts": counts, "m0": m0s, "ne": p.ne, "precision": "mixed", "ms": ms,
            "eigenpairs_per_s": found / (ms * 1e-3), "single_interval_ms": single_ms,
            "loops": [r.loop + 1 for r in rs], "slice_ms": [round(r.ms, 2) for r in rs]}


def nonhermitian(feastx, W, steps=3):
    """Non-Hermitian FEAST (dual subspaces, full contour of 16 trapezoidal
    nodes) on a dense complex generalized pencil, N = 2048, 40 eigenvalues in
    the region, M0 = 64.  `ms` (FP64) and `mixed_ms`: the device-array entry
    point with A, B, X resident in HBM; `host_arrays_ms`: one FP64 host-array
    call, including the PCIe upload of A and B."""
    import torch

    p = W.dense_general(2048, count=40, m0=64, seed=6201)
    A, B = feastx.fortran_tensor(p.A), feastx.fortran_tensor(p.B)
    X0 = feastx.fortran_tensor(p.X0.astype(np.complex128))
    X = X0.clone(memory_format=torch.contiguous_format).t().contiguous().t()
    times, r = {}, None
    for prec in ("fp64", "mixed"):
        wall = []
        for i in range(steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X.copy_(X0)
            r = feastx.gsolve_device(A, B, p.emin, p.emax, p.m0, X, x0=True, tol=p.tol, ne_full=16, precision=prec)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if r.info != 0 or r.M != p.meta["count"]:
                raise SystemExit(f"non-Hermitian {prec} solve failed: info {r.info}, M {r.M} of {p.meta['count']}")
            if i:
                wall.append(t1 - t0)
        times[prec] = (float(np.mean(wall)) * 1e3, r.loop + 1, float(max(r.res[:r.M].max(), r.res[p.m0:p.m0 + r.M].max())))
    t0 = time.perf_counter()
    rh = feastx.gsolve(p.A, p.B, p.emin, p.emax, p.m0, X0=p.X0, tol=p.tol, ne_full=16)
    host_ms = (time.perf_counter() - t0) * 1e3
    if rh.info != 0 or rh.M != r.M:
        raise SystemExit("non-Hermitian host-array solve disagrees")
    return {"n": p.n, "count": p.meta["count"], "m0": p.m0, "ne_full": 16,
            "ms": times["fp64"][0], "loops": times["fp64"][1], "max_res": times["fp64"][2],
            "mixed_ms": times["mixed"][0], "mixed_loops": times["mixed"][1], "mixed_max_res": times["mixed"][2],
            "host_arrays_ms": host_ms}


# ---------------------------------------------------------------- batched and serving

def batched(feastx, problems, concurrency):
    """All problems through feast_solve_batched_d (host arrays, one call),
    mixed and FP64: problems/s and eigenpairs/s, every result checked."""
    out = {"problems": len(problems), "ne": 8, "tol": 1e-10, "concurrency": concurrency,
           "n_min": min(q[0].shape[0] for q in problems), "n_max": max(q[0].shape[0] for q in problems)}
    for prec in ("mixed", "fp64"):
        t0 = time.perf_counter()
        rs = feastx.solve_batched([q[:6] for q in problems], precision=prec, concurrency=concurrency, ne=8,
                                  tol=1e-10)
        wall = time.perf_counter() - t0
        bad = [i for i, (q, r) in enumerate(zip(problems, rs))
               if r.info != 0 or r.M != q[6] or not (r.res[:r.M] < 1e-10).all()]
        if bad:
            raise SystemExit(f"batched {prec}: {len(bad)} problems failed, first {bad[0]}")
        pairs = sum(r.M for r in rs)
        key = "" if prec == "mixed" else "fp64_"
        out[key + "s"] = wall
        out[key + "problems_per_s"] = len(problems) / wall
        out[key + "eigenpairs_per_s"] = pairs / wall
        log(f"batched {prec}: {len(problems)} problems in {wall:.2f}s")
    out["mixed_over_fp64"] = out["fp64_s"] / out["s"]
    try:
        with open(os.path.join(ROOT, "tests", "golden", "oracle_batched_n256.json")) as f:
            fx = json.load(f)
        out["oracle_measured"] = {"problems": fx["problems"], "wall_s": fx["wall_s"],
                                  "workers": fx["workers"], "threads_per_worker": fx["threads_per_worker"],
                                  "cpu_s": fx["oracle_cpu_s"], "cpu": fx["cpu"],
                                  "problems_per_s": fx["problems"] / fx["wall_s"],
                                  "note": "the FP64 oracle on all 256 problems, measured once when its fixture "
                                          "was written (another host)"}
    except OSError:
        pass
    return out


def hbm_used_gb():
    """Device memory in use on the current GPU (GB), or None if it cannot be read."""
    try:
        import torch

        free, total = torch.cuda.mem_get_info()
        return (total - free) / 1e9
    except Exception:   # no device, or the query failed: the figure is left out
        return None


def serving(feastx, pool, reqs, per_size, slots, budget_gb):
    """Replays the request stream against the request loop, each request
    submitted at its arrival time (host arrays), mixed and FP64: completed
    requests per second (first arrival to last completion), latency from
    submit to result (p50/p99), largest number in flight."""
    from paper_1203_4031_amd import workloads as W

    out = {"requests": len(reqs), "rate_per_s": 200.0, "slots": slots, "hbm_budget_gb": budget_gb,
           "pool_per_size": {str(n): c for n, c in per_size.items()}, "sizes": list(W.SERVING_SIZES), "ne": 8, "tol": 1e-10,
           "size_mix": {str(n): sum(1 for q in reqs if q["n"] == n) for n in W.SERVING_SIZES}}
    x0 = {}
    for q in reqs:
        x0[q["x0_seed"]] = W.start_subspace(q["n"], q["m0"], q["x0_seed"])
    for prec in ("mixed", "fp64"):
        import queue

        hbm = {"base": hbm_used_gb(), "max": None}
        srv = feastx.Server(slots=slots, hbm_budget_gb=budget_gb)
        pending, results = queue.Queue(), []

        def sample_hbm():
            used = hbm_used_gb()
            if used is not None and (hbm["max"] is None or used > hbm["max"]):
                hbm["max"] = used

        def collect():
            while True:
                item = pending.get()
                if item is None:
                    return
                rid, q, t_sub = item
                results.append((srv.wait(rid), q, t_sub))
                if len(results) % 25 == 0:
                    sample_hbm()

        th = threading.Thread(target=collect, daemon=True)
        th.start()
        t0 = time.perf_counter()
        for i, q in enumerate(reqs):
            if i and i % 250 == 0:
                log(f"serving {prec}: {i} requests submitted, {len(results)} done")
            now = time.perf_counter() - t0
            if q["t"] > now:
                time.sleep(q["t"] - now)
            A, B, _ = pool[(q["n"], q["k"])]
            t_sub = time.perf_counter() - t0
            rid = srv.submit(A, B, q["emin"], q["emax"], q["m0"], X0=x0[q["x0_seed"]], ne=8, tol=1e-10,
                             precision=prec)
            pending.put((rid, q, t_sub))
            if i % 25 == 0:
                sample_hbm()
        pending.put(None)
        th.join()
        wall = time.perf_counter() - t0
        srv.close()
        lat, bad, events = [], [], []
        for r, q, t_sub in results:
            events += [(t_sub, 1), (t_sub + r.latency_ms * 1e-3, -1)]
            if r.info != 0 or r.M != q["count"] or not (r.res[:r.M] < 1e-10).all():
                bad.append({"n": q["n"], "count": q["count"], "m0": q["m0"], "info": r.info, "M": r.M,
                            "loops": r.loop + 1})
            else:
                lat.append(r.latency_ms)
        if bad:
            log(f"serving {prec}: {len(bad)} requests not converged to tol with the right count: {bad[:5]}")
        inflight, inflight_max = 0, 0
        for _, d in sorted(events):
            inflight += d
            inflight_max = max(inflight_max, inflight)
        lat = np.array(lat)
        key = "" if prec == "mixed" else "fp64_"
        out[key + "requests_per_s"] = len(lat) / wall
        out[key + "failed"] = bad
        out[key + "latency_ms"] = {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                                   "max": float(lat.max())}
        out[key + "in_flight_max"] = inflight_max
        # device memory in use (all of it, as the driver reports it), sampled every 25 submissions and
        # completions: the request loop's workspaces on top of what was in use before it started
        out[key + "hbm_gb"] = {"before": hbm["base"], "max_during": hbm["max"],
                               "max_added": (hbm["max"] - hbm["base"]
                                             if hbm["max"] is not None and hbm["base"] is not None else None)}
        out[key + "wall_s"] = wall
        log(f"serving {prec}: {len(reqs)} requests in {wall:.2f}s, p50 {out[key + 'latency_ms']['p50']:.1f} ms, "
            f"p99 {out[key + 'latency_ms']['p99']:.1f} ms")
    try:
        with open(os.path.join(ROOT, "tests", "golden", "oracle_serving_sample.json")) as f:
            fx = json.load(f)
        out["oracle_measured"] = {"requests": fx["sampled"], "sample": f"every {fx['every']}th request of "
                                  f"the stream with N <= {fx['max_n']}", "wall_s": fx["wall_s"],
                                  "workers": fx["workers"], "threads_per_worker": fx["threads_per_worker"],
                                  "cpu_s": fx["oracle_cpu_s"], "cpu": fx["cpu"],
                                  "requests_per_s": fx["sampled"] / fx["wall_s"],
                                  "note": "the FP64 oracle on a sample of the stream, each request alone, "
                                          "measured once when its fixture was written (another host)"}
    except OSError:
        pass
    return out


# ---------------------------------------------------------------- CPU baseline

def cpu_baseline(p, loops, fp64_ms):
    """The FP64 oracle on a bounded sample of the headline workload: the LU of
    one shifted matrix and one solve pair (A_z and its adjoint) of all M0
    columns at full size, scaled to a full solve of Ne LUs and loops x Ne
    solve pairs (Rayleigh-Ritz and the reduced problem not counted, which
    favours the CPU).  The oracle's measured full solve of the N = 4096
    workload, stored with its fixture, is given beside it."""
    import oracle

    oracle._load()
    z, _ = oracle.contour(p.emin, p.emax, p.ne)
    Az = z[0] * p.B - p.A
    t0 = time.perf_counter()
    lu, ipiv, info = oracle.zgetrf(Az)
    t_lu = time.perf_counter() - t0
    R = p.B @ p.X0
    t0 = time.perf_counter()
    oracle.zgetrs(lu, ipiv, R)
    oracle.zgetrs(lu, ipiv, R, trans="C")
    t_solve = time.perf_counter() - t0
    total = p.ne * t_lu + loops * p.ne * t_solve
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    out = {"value": 1.0 / total, "unit": "solves/s", "cores": cores, "kind": "oracle",
           "sample": f"oracle LU of 1 of {p.ne} shifted matrices ({t_lu:.1f} s) + one forward and one adjoint "
                     f"{p.m0}-column solve ({t_solve:.1f} s) at N={p.n}, scaled to {p.ne} LUs + {loops} loops of "
                     f"{p.ne} solve pairs; Rayleigh-Ritz excluded",
           "gpu_fp64_over_cpu": total / (fp64_ms * 1e-3)}
    try:
        with open(os.path.join(ROOT, "tests", "golden", "oracle_realgen_n4096.json")) as f:
            fx = json.load(f)
        out["full_solve_measured"] = {"workload": "dense real generalized N=4096, M0=300, Ne=8",
                                      "seconds": fx["oracle_wall_s"], "threads": fx["threads"],
                                      "cpu": fx["cpu"], "loops": fx["loop"] + 1,
                                      "note": "measured once when the fixture was written (another host)"}
    except OSError:
        pass
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--roofline-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tiles", default=None,
                    help="install this tile table instead of autotuning: c64 depth<=64, c64 deeper, c128 "
                         "depth<=64, c128 deeper (e.g. 1,1,0,0)")
    ap.add_argument("--precisions", default="mixed,fp64",
                    help="precisions to time (profiler passes of one precision's kernels)")
    ap.add_argument("--only", choices=["nonhermitian", "hermgen", "realgen"], default=None,
                    help="run only this measurement and print its JSON object (profiler passes)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the N=4096 extras (slicing, non-Hermitian, count estimate), batched and serving")
    ap.add_argument("--batched-problems", type=int, default=256)
    ap.add_argument("--batched-concurrency", type=int, default=8)
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-pool", type=int, default=2,
                    help="pool matrices per N up to 2048, half as many at 4096, the headline pencil at 8192 "
                         "(the recipe's full pool is 8 per N)")
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device-to-device 5 times (reference for HBM byte counters)")
    args = ap.parse_args()
    precisions = tuple(x for x in args.precisions.split(",") if x)
    if not precisions or any(x not in ("mixed", "fp64") for x in precisions):
        ap.error("--precisions takes mixed, fp64 or both")
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU path "
              "(multi-GPU sharding across contour nodes is a design note, not built).",
              file=sys.stderr)
        sys.exit(2)

    from paper_1203_4031_amd import workloads as W

    # ---- inputs, before anything touches the GPU
    want_extras = not args.no_extras and args.only is None
    p2 = p3 = None
    probs, pool = [], {}
    pool_sizes = {512: args.serving_pool, 1024: args.serving_pool, 2048: args.serving_pool,
                  4096: max(1, args.serving_pool // 2), 8192: 1}
    if not args.copy_calibration and args.only != "nonhermitian":
        t0 = time.perf_counter()
        if args.only in (None, "realgen"):
            p2 = W.dense_real_generalized(4096, 200, m0=300, ne=8, tol=1e-10, seed=2001)
            log(f"generated the N=4096 pencil ({time.perf_counter() - t0:.0f} s)")
        if args.only in (None, "hermgen"):
            p3 = W.dense_complex_hermitian(8192, 400, m0=600, ne=16, tol=1e-10, seed=3001)
            log(f"generated the N=8192 pencil ({time.perf_counter() - t0:.0f} s)")
        if want_extras:
            # the serving pool's N = 8192 matrix is the headline pencil; N = 4096 here
            for k in range(pool_sizes[4096]):
                pool[(4096, k)] = W.serving_pool_matrix(4096, k)
            log(f"generated the N=4096 pool matrices ({time.perf_counter() - t0:.0f} s)")
            pool[(8192, 0)] = (p3.A, p3.B, p3.spectrum)
            keys = [(n, k) for n in (512, 1024, 2048) for k in range(pool_sizes[n])]
            probs, pl = generate_small(W.batched_specs(args.batched_problems), keys)
            for n, k, A, B, spec in pl:
                pool[(n, k)] = (A, B, spec)
            log(f"inputs ready ({time.perf_counter() - t0:.0f} s)")

    import torch

    if args.copy_calibration:
        torch.cuda.set_device(0)
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 8, "launches": 5}), flush=True)
        return

    from paper_1203_4031_amd import feastx

    feastx.lib()
    torch.cuda.set_device(0)
    # tile shapes of the complex product kernel, timed on this device at the
    # headline workload's shapes (capped by the tuner) before any solve, or
    # installed as given (profiler passes repeat a measured table)
    if args.tiles:
        v = [int(x) for x in args.tiles.split(",")]
        if len(v) != 4:
            raise SystemExit("--tiles takes four variants: c64 depth<=64, c64 deeper, c128 depth<=64, c128 deeper")
        feastx.set_tiles({"complex64": {"depth<=64": v[0], "deeper": v[1]},
                          "complex128": {"depth<=64": v[2], "deeper": v[3]}})
        tune = {"choice": feastx.tiles(), "installed": "--tiles"}
    else:
        try:
            tune = feastx.autotune(8192, 600, 16)
        except RuntimeError as e:   # the defaults stay installed
            tune = {"choice": feastx.tiles(), "error": str(e)}
    log(f"tiles: {tune['choice']}")
    if args.only == "nonhermitian":
        print(json.dumps(nonhermitian(feastx, W, steps=max(args.steps, 1))), flush=True)
        feastx.release()
        return

    result = {}
    # ---- the N = 4096 real generalized workload
    if args.only in (None, "realgen"):
        r2, (A2, B2, _, _) = measure_single(feastx, torch, p2, max(args.steps, 5), args.warmup,
                                            max(args.roofline_steps, 2), "realgen_n4096", precisions)
        r2["config"] = {"workload": "dense real symmetric generalized A x = lambda B x, N=4096, M0=300, Ne=8, "
                                    "200 eigenvalues in the interval, tol 1e-10", "seed": 2001}
        if want_extras:
            r2["slicing"] = slicing(feastx, torch, W, A2, B2, p2, r2["count"], r2["ms_per_solve"])
            r2["nonhermitian"] = nonhermitian(feastx, W)
            r2["count_estimate"] = count_estimate(feastx, torch, W, A2, B2, p2, r2["count"])
        result["dense_real_n4096"] = r2
        del A2, B2
        feastx.release()
        torch.cuda.empty_cache()
        if args.only == "realgen":
            r2["autotune"] = tune
            print(json.dumps(r2), flush=True)
            return

    # ---- headline: the N = 8192 complex Hermitian generalized workload
    r3, _ = measure_single(feastx, torch, p3, args.steps, args.warmup, args.roofline_steps, "hermgen_n8192",
                           precisions)
    feastx.release()
    torch.cuda.empty_cache()
    if args.only == "hermgen":
        r3["autotune"] = tune
        print(json.dumps(r3), flush=True)
        return

    out = {
        "metric": "FEAST solves/sec & eigenpairs/sec at resid<=1e-10, mixed vs FP64; p50/p99 latency",
        "value": r3["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r3["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128+f64" if r3["precision"] == "fp64" else "c64+c128+f64",
        "data": "synthetic",
        "config": {"workload": "dense complex Hermitian generalized A x = lambda B x, N=8192 (Haar U, "
                               "clustered spectrum, B = I + 0.1 H), M0=600, Ne=16 Gauss-Legendre, ~400 "
                               "eigenvalues in the interval, tol 1e-10",
                   "n": 8192, "m0": 600, "ne": 16, "count": r3["count"], "tol": 1e-10, "seed": 3001,
                   "precision": PRECISION_TEXT[r3["precision"]],
                   "parallelism": "single GPU"},
    }
    for k in ("precision", "eigenpairs_per_s", "loops", "mixed", "fp64", "mixed_over_fp64", "roofline",
              "shifted_lu"):
        out[k] = r3[k]
    out["autotune"] = tune
    out.update(result)

    if want_extras:
        out["batched"] = batched(feastx, probs, args.batched_concurrency)
        out["batched"]["workload"] = ("256 dense real symmetric generalized problems, N log-uniform on "
                                      "[256, 2048], 5-15 % of each spectrum in its interval, M0 = 1.5 count, "
                                      "Ne=8, seeds 4001..4256")
        del probs
        feastx.release()
        reqs = W.serving_requests({key: v[2] for key, v in pool.items()}, args.serving_requests, pool_sizes)
        out["serving"] = serving(feastx, pool, reqs, pool_sizes, args.serving_slots, 64.0)
        out["serving"]["workload"] = ("dense complex Hermitian generalized requests built as the N=8192 "
                                      "workload, N in {512, 1024, 2048, 4096, 8192} with p(N) ~ N^-2, "
                                      "count ~ U{50..300} (at most N/4) per request, M0 = 1.5 count, Ne=8, "
                                      "Poisson arrivals at 200/s, host arrays; pool matrices per N as in "
                                      "pool_per_size, the N=8192 one being the headline pencil")
        del pool
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle LU and solves of one shifted N=8192 matrix")
        ref = r3["fp64"] or r3["mixed"]
        out["cpu_baseline"] = cpu_baseline(p3, ref["loops"], ref["ms_per_solve"])
    print(json.dumps(out), flush=True)
    feastx.release()


if __name__ == "__main__":
    main()
