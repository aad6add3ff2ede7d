"""FEAST solves/s on one MI355X: dense real symmetric generalized problem,
N = 4096, M0 = 300, Ne = 8 Gauss-Legendre half-contour nodes, ~200
eigenvalues in the interval, tol 1e-10.  Mixed precision (complex64 LU and
solves on the FP32 matrix cores, FP64 residual correction) is the headline;
plain FP64 on the same GPU is reported beside it.

One step = one complete feast_solve call (all contour nodes: shift, LU,
solves, quadrature, Rayleigh-Ritz, reduced eigensolve, residuals, every FEAST
loop until convergence) on inputs already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3      # TFLOP/s, dense
PEAK_FP64_MFMA = 78.6
N, COUNT, M0, NE, TOL, SEED = 4096, 200, 300, 8, 1e-10, 2001

# HBM bytes per launch of the roofline kernel (FETCH_SIZE + WRITE_SIZE, each
# scaled by a 256 MiB copy's reading, averaged over the launches of one
# solve), from the rocprofv3 counter passes summarised in
# profiles/hbm_traffic_realgen_n4096_m0300.md.  It holds only for the
# sources it was measured on -- the kernel itself and every file that
# launches it (the FP64 reduced-problem kernels in jacobi.hpp and
# bortho.hpp do not): `traffic` is null when they differ.
TRAFFIC_BYTES_PER_LAUNCH = 1.196e+08
TRAFFIC_SOURCES_SHA256 = "ba63631afd37f8bc40d54c07744d3e0306fd1ad9a1bf62cc5284ea6550d0421c"


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1203_4031_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".hpp", ".h")) and name not in ("jacobi.hpp", "bortho.hpp"):
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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


def check(results, p, expected_m):
    for r in results:
        if r.info != 0:
            raise SystemExit(f"solve failed: info {r.info}")
        if r.M != expected_m:
            raise SystemExit(f"eigenvalue count {r.M} != {expected_m}")
        if not (r.res[:r.M] <= p.tol).all():
            raise SystemExit("residual above tol")


def cpu_baseline(p, loops):
    """The FP64 oracle on a bounded sample of the same workload: the LU of one
    shifted matrix and its M0-column solve at full size, extrapolated to a
    full solve (Ne LUs + loops x Ne solves; Rayleigh-Ritz not counted, which
    favours the CPU)."""
    import oracle

    oracle._load()
    z, _ = oracle.contour(p.emin, p.emax, p.ne)
    Az = z[0] * p.B - p.A
    t0 = time.perf_counter()
    lu, ipiv, info = oracle.zgetrf(Az)
    t_lu = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.zgetrs(lu, ipiv, p.B @ p.X0)
    t_solve = time.perf_counter() - t0
    total = p.ne * t_lu + loops * p.ne * t_solve
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    return {"value": 1.0 / total, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle LU of 1 of {p.ne} shifted matrices ({t_lu:.1f} s) + its {p.m0}-column "
                      f"solve ({t_solve:.1f} s) at N={p.n}, extrapolated to {p.ne} LUs + {loops} loops "
                      f"of {p.ne} solves; Rayleigh-Ritz excluded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--roofline-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["nonhermitian"], default=None,
                    help="run only this extra measurement and print its JSON object (profiler passes)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the slicing, non-Hermitian and count-estimate measurements (profiler passes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device-to-device 5 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU path "
              "(multi-GPU sharding across contour nodes is a design note, not built).",
              file=sys.stderr)
        sys.exit(2)

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
    from paper_1203_4031_amd import workloads as W

    feastx.lib()
    torch.cuda.set_device(0)
    if args.only == "nonhermitian":
        print(json.dumps(nonhermitian(feastx, W, steps=max(args.steps, 1))), flush=True)
        feastx.release()
        return
    t0 = time.perf_counter()
    p = W.dense_real_generalized(N, COUNT, m0=M0, ne=NE, tol=TOL, seed=SEED)
    expected = p.count_in_interval()
    log(f"generated N={N} in {time.perf_counter() - t0:.1f}s, interval [{p.emin:.6f}, {p.emax:.6f}] "
        f"holds {expected} eigenvalues")
    A = feastx.fortran_tensor(p.A)
    B = feastx.fortran_tensor(p.B)
    X0 = feastx.fortran_tensor(p.X0)
    X = X0.clone(memory_format=torch.contiguous_format).t().contiguous().t()

    # warmup (also sizes the library's workspace)
    run_steps(feastx, torch, A, B, X0, X, p, "mixed", args.warmup, False)
    if args.warmup > 0 and args.fp64_steps != 0:
        run_steps(feastx, torch, A, B, X0, X, p, "fp64", 1, False)
    log("warmup done")

    # timed region: mixed precision
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    times, res_mixed, _ = run_steps(feastx, torch, A, B, X0, X, p, "mixed", args.steps, False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    st = feastx.stats()
    stage_ms = {k: round(getattr(st, k), 3) for k in ("t_total", "t_shift", "t_factor", "t_solve", "t_accum",
                                                      "t_rr", "t_reduced", "t_resid")}
    stage_ms["eig_calls"], stage_ms["eig_sweeps"] = st.eig_calls, st.eig_sweeps
    check(res_mixed, p, expected)
    loops = res_mixed[-1].loop + 1
    log(f"mixed: {args.steps} solves in {wall:.3f}s, loops {loops}")

    # second timed region for the roofline: the same solves with a HIP event
    # pair around every launch of the complex64 product kernel
    _, res_t, lu = run_steps(feastx, torch, A, B, X0, X, p, "mixed", args.roofline_steps, True)
    check(res_t, p, expected)

    fsteps = args.fp64_steps if args.fp64_steps is not None else max(1, args.steps // 2)
    times64 = [float("nan")]
    if fsteps > 0:
        times64, res64, _ = run_steps(feastx, torch, A, B, X0, X, p, "fp64", fsteps, False)
        check(res64, p, expected)
        log(f"fp64: {fsteps} solves, mean {np.mean(times64) * 1e3:.1f} ms")

    solves_per_s = args.steps / wall
    lat = np.array(times) * 1e3
    achieved = lu[1] / (lu[0] * 1e-3) / 1e12 if lu[0] > 0 else 0.0
    out = {
        "metric": "FEAST solves/sec & eigenpairs/sec at resid<=1e-10, mixed vs FP64; p50/p99 latency",
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {"workload": "dense real symmetric generalized A x = lambda B x, N=4096, "
                               "M0=300, Ne=8, ~200 eigenvalues in the interval, tol 1e-10",
                   "n": N, "m0": M0, "ne": NE, "count": expected, "tol": TOL,
                   "precision": "mixed (c64 LU/solves + FP64 residual correction)",
                   "parallelism": "single GPU"},
        "eigenpairs_per_s": solves_per_s * expected,
        "fp64_solves_per_s": 1.0 / float(np.mean(times64)),
        "mixed_over_fp64": solves_per_s * float(np.mean(times64)),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "feast_loops": loops,
        "stage_ms_last_solve": stage_ms,
        "roofline": {"kernel": "gemm_kernel<float, true, false, 64, 64, 16, 32, 32, 4, true, true>: complex64 "
                               "matrix product on the FP32 matrix cores (LU trailing updates and "
                               "triangular-solve updates), every launch of the timed solves; products of at "
                               "most 32 columns use its 64x32 instance gemm_kernel<float, true, false, 64, 32, "
                               "16, 32, 16, 4, true, true>, counted here too",
                     "bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": (TRAFFIC_BYTES_PER_LAUNCH
                                 if kernel_sources_sha256() == TRAFFIC_SOURCES_SHA256 else None),
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "flop_count": "algorithmic, 8 per complex multiply-add; the kernel's three-multiplication "
                                   "form issues 6 of them to the matrix cores (executed rate 0.75 x achieved)",
                     "launches": lu[2], "avg_launch_ms": lu[0] / max(lu[2], 1),
                     "flops_per_launch": lu[1] / max(lu[2], 1),
                     "measured_over": f"{args.roofline_steps} extra mixed solves with per-launch HIP events"},
    }
    # the shifted LU on its own: its product launches (trailing and panel-column
    # updates), and the whole factor stage (panels, interchanges, products and
    # the solve form W) against the (8/3) N^3 flops of each LU
    upd = lu[4] / (lu[3] * 1e-3) / 1e12 if lu[3] > 0 else 0.0
    fac = lu[7] / (lu[6] * 1e-3) / 1e12 if lu[6] > 0 else 0.0
    out["shifted_lu"] = {"update_achieved": upd, "update_frac": upd / PEAK_FP32_MFMA,
                         "update_launches": lu[5], "unit": "TFLOP/s", "peak": PEAK_FP32_MFMA,
                         "factor_ms": lu[6] / max(args.roofline_steps, 1),
                         "factor_rate": fac, "factor_frac": fac / PEAK_FP32_MFMA,
                         "note": "update_*: the LU's complex64 product launches alone (8 flops per complex "
                                 "multiply-add); factor_*: Ne (8/3) N^3 over the whole factor stage, timed with "
                                 "per-launch events on (so slightly slow)"}
    if not args.no_extras:
        out["slicing"] = slicing(feastx, torch, W, A, B, p, expected, wall / args.steps * 1e3)
        log(f"slicing: {out['slicing']['ms']:.1f} ms for {expected} eigenpairs in {out['slicing']['slices']} slices")
        out["nonhermitian"] = nonhermitian(feastx, W)
        log(f"non-Hermitian N=2048: {out['nonhermitian']['ms']:.1f} ms with inputs in HBM, "
            f"{out['nonhermitian']['loops']} loops")
        out["count_estimate"] = count_estimate(feastx, torch, W, A, B, p, expected)
        log(f"count estimate: {out['count_estimate']['estimate']} (count {expected}) in "
            f"{out['count_estimate']['ms']:.1f} ms")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, loops)
    print(json.dumps(out), flush=True)
    feastx.release()


if __name__ == "__main__":
    main()
