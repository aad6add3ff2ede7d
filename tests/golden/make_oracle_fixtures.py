"""Write the oracle's results on the full-size workloads as text fixtures.

    python tests/golden/make_oracle_fixtures.py realgen_n4096     # about 3 min on 8 cores
    python tests/golden/make_oracle_fixtures.py hermgen_n8192     # about 2.5 h on 6 cores
    python tests/golden/make_oracle_fixtures.py --add-input-samples realgen_n4096
    python tests/golden/make_oracle_fixtures.py batched_n256      # about 35 min on 8 cores
    python tests/golden/make_oracle_fixtures.py serving_sample    # about 25 min on 8 cores

Calls only the FP64 CPU oracle (oracle/) on inputs from the seeded generators
(paper_1203_4031_amd/workloads.py, which hold none of the method's
arithmetic).  Nothing here comes from the GPU library.  Each fixture holds:

* the SHA-256 of the start subspace X0 (seeded random numbers only, so the
  same to the bit on every machine) and A, B at 256 seeded positions: A and B
  come out of LAPACK and BLAS calls whose last bits depend on the CPU, so a
  test checks that its own A and B agree with these to rounding, and takes
  the interval [Emin, Emax] from here;
* info, M, the kept subspace size, loop and epsout;
* E and res of every returned Ritz pair (in-interval ones first, ascending);
* a projector sketch K = S2^T X_M X_M^H B S (16 x 16), with X_M the M
  in-interval eigenvectors and S, S2 seeded uniform(-1, 1) N x 16 blocks.
  X_M X_M^H B is the B-orthogonal projector onto the eigenspace of the
  interval, so K does not depend on how eigenvectors inside a cluster are
  rotated or phased, and two subspaces that differ by an angle theta give
  sketches that differ by about theta |K|;
* the oracle's wall time, thread count and CPU model (the CPU baseline).
"""
from __future__ import annotations

import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1203_4031_amd import workloads as W  # noqa: E402

SKETCH_COLS = 16
SKETCH_SEEDS = (7001, 7002)


def workload(name: str):
    """The full-size workloads: the dense real symmetric generalized pencil
    (N = 4096, 200 eigenvalues, M0 = 300, Ne = 8) and the dense complex
    Hermitian generalized pencil (N = 8192, 400 eigenvalues, M0 = 600,
    Ne = 16), both at tol 1e-10."""
    if name == "realgen_n4096":
        return W.dense_real_generalized(4096, 200, m0=300, ne=8, tol=1e-10, seed=2001)
    if name == "hermgen_n8192":
        return W.dense_complex_hermitian(8192, 400, m0=600, ne=16, tol=1e-10, seed=3001)
    raise SystemExit(f"unknown workload {name}")


def input_sha256(p) -> str:
    h = hashlib.sha256()
    for a in (p.A, p.B, p.X0):
        h.update(np.asfortranarray(a).tobytes(order="F"))
    h.update(np.array([p.emin, p.emax]).tobytes())
    return h.hexdigest()


def x0_sha256(p) -> str:
    return hashlib.sha256(np.asfortranarray(p.X0).tobytes(order="F")).hexdigest()


SAMPLE_SEED, SAMPLES = 7003, 256


def input_samples(p):
    """A and B at 256 seeded (row, column) positions, real and imaginary parts."""
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    i = rng.integers(0, p.n, SAMPLES)
    j = rng.integers(0, p.n, SAMPLES)
    a, b = p.A[i, j], p.B[i, j]
    return {"A_re": np.real(a).tolist(), "A_im": np.imag(a).tolist(),
            "B_re": np.real(b).tolist(), "B_im": np.imag(b).tolist()}


def inputs_match(p, ref, rtol=1e-12) -> bool:
    """The generated A, B agree with the fixture's samples to rounding and X0
    is the same to the bit."""
    if x0_sha256(p) != ref["x0_sha256"]:
        return False
    smp = input_samples(p)
    for key, mat in (("A", p.A), ("B", p.B)):
        got = np.array(smp[key + "_re"]) + 1j * np.array(smp[key + "_im"])
        want = np.array(ref["samples"][key + "_re"]) + 1j * np.array(ref["samples"][key + "_im"])
        if np.max(np.abs(got - want)) > rtol * np.max(np.abs(mat)):
            return False
    return True


def sketch_blocks(n: int):
    return [W.start_subspace(n, SKETCH_COLS, seed=s) for s in SKETCH_SEEDS]


def projector_sketch(X_in, B, S, S2):
    """S2^T X X^H B S for the in-interval eigenvectors X (N x M)."""
    BS = S if B is None else B @ S
    return S2.T @ (X_in @ (X_in.conj().T @ BS))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def add_input_samples(name: str):
    """Add the X0 hash and the A, B samples to an existing fixture, from the
    generator alone (the oracle's results in it are left as they are); the
    input SHA-256 must still match, so the samples describe the inputs the
    oracle saw."""
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path) as f:
        out = json.load(f)
    p = workload(name)
    if out["input_sha256"] != input_sha256(p):
        raise SystemExit("inputs differ from the ones the oracle ran on: rerun the oracle")
    out["x0_sha256"] = x0_sha256(p)
    out["samples"] = input_samples(p)
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print(f"updated {path}", flush=True)


# ---- the batched workload: 256 real generalized problems of uneven N
BATCHED_STORED_EVERY = 8      # E and res are stored for problems 0, 8, 16, ...
BATCHED_SAMPLES = 8           # A, B samples per problem


def batched_samples(p):
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    i = rng.integers(0, p.n, BATCHED_SAMPLES)
    j = rng.integers(0, p.n, BATCHED_SAMPLES)
    return {"A": p.A[i, j].tolist(), "B": p.B[i, j].tolist()}


def batched_inputs_match(p, ref, rtol=1e-12) -> bool:
    """The regenerated problem agrees with the fixture's entry: X0 to the bit,
    A and B to rounding at the sampled positions."""
    if x0_sha256(p) != ref["x0_sha256"] or p.n != ref["n"] or p.m0 != ref["m0"]:
        return False
    smp = batched_samples(p)
    for key, mat in (("A", p.A), ("B", p.B)):
        if np.max(np.abs(np.array(smp[key]) - np.array(ref["samples"][key]))) > rtol * np.max(np.abs(mat)):
            return False
    return True


def _batched_one(idx_spec):
    idx, spec = idx_spec
    t0 = time.perf_counter()
    p = W.batched_problem(spec)
    t_gen = time.perf_counter() - t0
    oracle._load()
    t0 = time.perf_counter()
    r = oracle.feast(p.A, p.B, p.emin, p.emax, p.m0, p.ne, p.tol, p.X0)
    wall = time.perf_counter() - t0
    out = {"i": idx, "n": p.n, "m0": p.m0, "count": spec[1], "seed": spec[2], "x0_seed": spec[3],
           "emin": p.emin, "emax": p.emax, "x0_sha256": x0_sha256(p), "samples": batched_samples(p),
           "info": r.info, "M": r.M, "loop": r.loop, "oracle_wall_s": wall, "generate_s": t_gen,
           "max_res": float(np.max(r.res[:r.M])) if r.M > 0 else None}
    if idx % BATCHED_STORED_EVERY == 0:
        out["E"] = [float(x) for x in r.E[:r.M]]
    else:
        del out["samples"]   # only the stored problems are regenerated by the test
    return out


def batched(workers: int):
    """The oracle on every problem of the batched workload, one problem per
    single-threaded worker process at a time."""
    import concurrent.futures as cf
    import multiprocessing as mp

    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    specs = W.batched_specs()
    t0 = time.perf_counter()
    results = []
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for r in ex.map(_batched_one, list(enumerate(specs)), chunksize=1):
            results.append(r)
            print(f"problem {r['i']}: n {r['n']} M {r['M']} info {r['info']} loops {r['loop'] + 1} "
                  f"{r['oracle_wall_s']:.1f} s", flush=True)
    wall = time.perf_counter() - t0
    out = {"workload": "batched_n256", "problems": len(specs), "ne": 8, "tol": 1e-10,
           "stored_every": BATCHED_STORED_EVERY, "sample_seed": SAMPLE_SEED,
           "oracle_cpu_s": sum(r["oracle_wall_s"] for r in results), "wall_s": wall,
           "workers": workers, "threads_per_worker": 1, "nproc": os.cpu_count(), "cpu": cpu_model(),
           "written": time.strftime("%Y-%m-%d"), "entries": results}
    path = os.path.join(HERE, "oracle_batched_n256.json")
    entries = out.pop("entries")
    with open(path, "w") as f:   # one problem per line
        f.write("{\n")
        for k, v in out.items():
            f.write(json.dumps(k) + ": " + json.dumps(v) + ",\n")
        f.write('"entries": [\n')
        f.write(",\n".join(json.dumps(e, separators=(",", ":")) for e in entries))
        f.write("\n]\n}\n")
    print(f"wrote {path}: {len(results)} problems, {wall:.0f} s wall on {workers} workers", flush=True)


# ---- the serving workload: a systematic sample of its request stream
SERVING_POOL = {512: 2, 1024: 2, 2048: 2, 4096: 1, 8192: 1}   # the bench's pool sizes
SERVING_EVERY, SERVING_STORED_EVERY, SERVING_MAX_N = 5, 50, 2048


def serving_stream():
    """The bench's 2000 requests (Poisson 200/s, p(N) ~ N^-2, seed 5000); the
    N = 8192 pool matrix is the headline pencil."""
    spectra = {}
    for n, cnt in SERVING_POOL.items():
        for k in range(cnt):
            if n == 8192:
                spectra[(n, k)] = W.dense_complex_hermitian(8192, 400, m0=600, ne=16, tol=1e-10,
                                                            seed=3001).spectrum
            else:
                spectra[(n, k)] = W.serving_pool_matrix(n, k)[2]
    return W.serving_requests(spectra, 2000, SERVING_POOL)


_pool_cache = {}


def _serving_one(idx_req):
    idx, q = idx_req
    key = (q["n"], q["k"])
    if key not in _pool_cache:
        _pool_cache[key] = W.serving_pool_matrix(*key)
    A, B, _ = _pool_cache[key]
    X0 = W.start_subspace(q["n"], q["m0"], q["x0_seed"])
    oracle._load()
    t0 = time.perf_counter()
    r = oracle.feast(A, B, q["emin"], q["emax"], q["m0"], q["ne"], q["tol"], X0, hermitian=True)
    wall = time.perf_counter() - t0
    out = {"i": idx, "n": q["n"], "k": q["k"], "count": q["count"], "m0": q["m0"], "emin": q["emin"],
           "emax": q["emax"], "x0_seed": q["x0_seed"], "info": r.info, "M": r.M, "loop": r.loop,
           "oracle_wall_s": wall}
    if idx % SERVING_STORED_EVERY == 0:
        out["E"] = [float(x) for x in r.E[:r.M]]
        rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
        i, j = rng.integers(0, q["n"], BATCHED_SAMPLES), rng.integers(0, q["n"], BATCHED_SAMPLES)
        out["samples"] = {"A_re": np.real(A[i, j]).tolist(), "A_im": np.imag(A[i, j]).tolist(),
                          "B_re": np.real(B[i, j]).tolist(), "B_im": np.imag(B[i, j]).tolist()}
    return out


def serving_sample_matches(A, B, ref, rtol=1e-12) -> bool:
    """A regenerated pool matrix agrees with a stored request's samples to rounding."""
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    n = A.shape[0]
    i, j = rng.integers(0, n, BATCHED_SAMPLES), rng.integers(0, n, BATCHED_SAMPLES)
    for key, mat in (("A", A), ("B", B)):
        want = np.array(ref["samples"][key + "_re"]) + 1j * np.array(ref["samples"][key + "_im"])
        if np.max(np.abs(mat[i, j] - want)) > rtol * np.max(np.abs(mat)):
            return False
    return True


def serving_sample(workers: int):
    """The oracle on every fifth request of the serving stream with N <= 2048
    (single-threaded workers), eigenvalues stored for every fiftieth."""
    import concurrent.futures as cf
    import multiprocessing as mp

    reqs = serving_stream()
    pick = [(i, q) for i, q in enumerate(reqs) if i % SERVING_EVERY == 0 and q["n"] <= SERVING_MAX_N]
    print(f"{len(pick)} sampled requests of {len(reqs)}", flush=True)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    t0 = time.perf_counter()
    results = []
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for r in ex.map(_serving_one, pick, chunksize=1):
            results.append(r)
            print(f"request {r['i']}: n {r['n']} M {r['M']} info {r['info']} loops {r['loop'] + 1} "
                  f"{r['oracle_wall_s']:.1f} s", flush=True)
    wall = time.perf_counter() - t0
    out = {"workload": "serving_sample", "requests_in_stream": len(reqs), "sampled": len(results),
           "every": SERVING_EVERY, "max_n": SERVING_MAX_N, "stored_every": SERVING_STORED_EVERY,
           "pool": {str(n): c for n, c in SERVING_POOL.items()}, "sample_seed": SAMPLE_SEED,
           "oracle_cpu_s": sum(r["oracle_wall_s"] for r in results), "wall_s": wall, "workers": workers,
           "threads_per_worker": 1, "nproc": os.cpu_count(), "cpu": cpu_model(),
           "written": time.strftime("%Y-%m-%d")}
    path = os.path.join(HERE, "oracle_serving_sample.json")
    with open(path, "w") as f:   # one request per line
        f.write("{\n")
        for k, v in out.items():
            f.write(json.dumps(k) + ": " + json.dumps(v) + ",\n")
        f.write('"entries": [\n')
        f.write(",\n".join(json.dumps(e, separators=(",", ":")) for e in results))
        f.write("\n]\n}\n")
    print(f"wrote {path}: {len(results)} requests, {wall:.0f} s wall on {workers} workers", flush=True)


def main():
    if sys.argv[1] == "serving_sample":
        serving_sample(int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1))
        return
    if sys.argv[1] == "--add-input-samples":
        add_input_samples(sys.argv[2])
        return
    if sys.argv[1] == "batched_n256":
        batched(int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1))
        return
    name = sys.argv[1]
    t0 = time.perf_counter()
    p = workload(name)
    t_gen = time.perf_counter() - t0
    print(f"{name}: generated in {t_gen:.1f} s, interval [{p.emin!r}, {p.emax!r}]", flush=True)
    oracle._load()
    t0 = time.perf_counter()
    r = oracle.feast(p.A, p.B, p.emin, p.emax, p.m0, p.ne, p.tol, p.X0, hermitian=p.hermitian)
    wall = time.perf_counter() - t0
    print(f"{name}: oracle info {r.info} M {r.M} loops {r.loop + 1} in {wall:.1f} s", flush=True)
    S, S2 = sketch_blocks(p.n)
    K = projector_sketch(r.X[:, :r.M], p.B, S, S2)
    out = {
        "workload": name,
        "n": p.n, "m0": p.m0, "ne": p.ne, "tol": p.tol, "hermitian": bool(p.hermitian),
        "emin": p.emin, "emax": p.emax, "meta": p.meta,
        "input_sha256": input_sha256(p),
        "x0_sha256": x0_sha256(p), "samples": input_samples(p),
        "info": r.info, "M": r.M, "m0_out": r.m0, "loop": r.loop, "epsout": r.epsout,
        "E": [float(x) for x in r.E], "res": [float(x) for x in r.res],
        "sketch_cols": SKETCH_COLS, "sketch_seeds": list(SKETCH_SEEDS),
        "sketch_re": np.real(K).tolist(), "sketch_im": np.imag(K).tolist(),
        "oracle_wall_s": wall, "generate_s": t_gen,
        "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
        "nproc": os.cpu_count(), "cpu": cpu_model(),
        "written": time.strftime("%Y-%m-%d"),
    }
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
