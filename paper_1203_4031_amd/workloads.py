"""Seeded synthetic eigenproblems for the dense Hermitian FEAST path.

This module only *builds inputs*: matrices A and B, a search interval
[Emin, Emax], the start subspace X0 and the sizes M0 / Ne / tol.  It holds
none of the method's arithmetic (no contour, no factorisation, no
Rayleigh-Ritz); both the GPU library and the CPU oracle receive exactly the
same arrays from here.

The FEAST guide ships example matrices that are not available, so these
generators stand in for them (guide, sections "Examples" and "FEAST utility
sparse drivers").  Every array is column-major (Fortran order), the storage
the guide's dense interfaces use (section "Matrix storage").

Random numbers come from numpy's PCG64 with fixed seeds.  The interval rule
needs the generalized spectrum, which is computed with LAPACK through
scipy: that is input generation (choosing an interval with clear gaps at
both ends), not a result the tests compare against.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem",
    "helloworld",
    "laplacian_1d",
    "dense_real_generalized",
    "dense_complex_hermitian",
    "batched_real_generalized",
    "batched_specs",
    "batched_problem",
    "serving_pool_matrix",
    "serving_requests",
    "start_subspace",
    "pick_interval",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Problem:
    """One eigenproblem A x = lambda B x with everything a solve needs."""

    name: str
    A: np.ndarray                 # (N, N) float64 or complex128, Fortran order
    B: np.ndarray | None          # None means B = I (standard problem)
    emin: float
    emax: float
    m0: int
    ne: int
    tol: float
    X0: np.ndarray                # (N, M0) float64, Fortran order
    hermitian: bool               # True: complex Hermitian, False: real symmetric
    spectrum: np.ndarray | None = None   # sorted generalized eigenvalues, if computed
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]

    def count_in_interval(self) -> int | None:
        if self.spectrum is None:
            return None
        s = self.spectrum
        return int(np.count_nonzero((s >= self.emin) & (s <= self.emax)))


def start_subspace(n: int, m0: int, seed: int) -> np.ndarray:
    """Random start subspace: real uniform(-1, 1) entries, (n, m0), Fortran order."""
    return np.asfortranarray(_rng(seed).uniform(-1.0, 1.0, size=(n, m0)))


def sign_probes(n: int, m0: int, seed: int) -> np.ndarray:
    """Probe vectors for the eigenvalue-count estimate: independent +-1
    entries with equal probability, (n, m0), Fortran order."""
    return np.asfortranarray(np.where(_rng(seed).random((n, m0)) < 0.5, -1.0, 1.0))


def slice_bounds(spectrum: np.ndarray, start: int, counts) -> np.ndarray:
    """Bounds of neighbouring intervals over a sorted spectrum: slice k holds
    counts[k] eigenvalues, the first starting at index ``start``; every bound
    is the midpoint of the gap it sits in."""
    s = np.sort(np.asarray(spectrum, dtype=np.float64))
    idx = start + np.concatenate([[0], np.cumsum(counts)])
    if idx[0] < 1 or idx[-1] >= s.size:
        raise ValueError("slices must leave an eigenvalue outside each end")
    return 0.5 * (s[idx - 1] + s[idx])


def pick_interval(spectrum: np.ndarray, count: int, centre_index: int | None = None):
    """Interval holding ``count`` eigenvalues with the widest end gaps.

    The window of ``count`` consecutive eigenvalues starts near the middle of
    the spectrum (or at ``centre_index``) and may shift by up to 5 % of
    ``count`` either way; the shift that maximises the smaller of the two end
    gaps wins.  Emin and Emax are the midpoints of those gaps, so no cluster
    is cut and no eigenvalue sits close to an endpoint.
    Returns (emin, emax, first_index).
    """
    s = np.sort(np.asarray(spectrum, dtype=np.float64))
    n = s.size
    if not 1 <= count <= n - 2:
        raise ValueError("count must leave at least one eigenvalue on each side")
    if centre_index is None:
        centre_index = n // 2
    base = int(centre_index - count // 2)
    slack = max(1, int(round(0.05 * count)))
    best = None
    for shift in range(-slack, slack + 1):
        lo = base + shift
        if lo < 1 or lo + count > n - 1:
            continue
        g_lo = s[lo] - s[lo - 1]
        g_hi = s[lo + count] - s[lo + count - 1]
        g = min(g_lo, g_hi)
        if best is None or g > best[0]:
            best = (g, lo)
    if best is None:
        raise ValueError("no admissible window")
    lo = best[1]
    emin = 0.5 * (s[lo - 1] + s[lo])
    emax = 0.5 * (s[lo + count - 1] + s[lo + count])
    return float(emin), float(emax), lo


def _generalized_spectrum(A, B):
    import scipy.linalg as sl

    if B is None:
        return np.sort(sl.eigh(A, eigvals_only=True))
    return np.sort(sl.eigh(A, B, eigvals_only=True))


def helloworld() -> Problem:
    """The guide's 2x2 example: A = [[2,-1],[-1,2]], B = I, interval [-5, 5],
    M0 = 2, 8 half-contour nodes (section 'A simple Hello World Example').
    The start subspace is random (the guide's example does not supply one)."""
    A = np.asfortranarray(np.array([[2.0, -1.0], [-1.0, 2.0]]))
    return Problem("helloworld", A, None, -5.0, 5.0, 2, 8, 1e-12,
                   start_subspace(2, 2, 1000), False, np.array([1.0, 3.0]))


def laplacian_1d(n: int = 200, emin: float = 0.0, emax: float = 0.5, m0: int = 70,
                 ne: int = 8, tol: float = 1e-12, seed: int = 1100) -> Problem:
    """1D Laplacian tridiag(-1, 2, -1) stored dense, B = I.  Eigenvalues are
    2 - 2 cos(k pi / (n + 1)), k = 1..n, in closed form."""
    A = np.zeros((n, n), order="F")
    i = np.arange(n)
    A[i, i] = 2.0
    A[i[:-1], i[:-1] + 1] = -1.0
    A[i[:-1] + 1, i[:-1]] = -1.0
    k = np.arange(1, n + 1)
    spec = np.sort(2.0 - 2.0 * np.cos(k * math.pi / (n + 1)))
    return Problem(f"laplacian{n}", A, None, emin, emax, m0, ne, tol,
                   start_subspace(n, m0, seed), False, spec)


def _orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Q from QR of a Gaussian matrix, column signs fixed so diag(R) > 0."""
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))


def _haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed unitary: QR of a complex Ginibre matrix with the phases
    of diag(R) divided out (Mezzadri, 2007)."""
    Z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    return Q * (d / np.abs(d))


def dense_real_generalized(n: int = 4096, count: int = 200, m0: int | None = None,
                           ne: int = 8, tol: float = 1e-10, seed: int = 2001,
                           x0_seed: int | None = None, with_B: bool = True) -> Problem:
    """Dense real symmetric generalized problem.

    A = Q diag(lambda) Q^T with Q orthogonal (QR of a Gaussian matrix) and
    lambda ~ U[-1, 1]; B = P diag(mu) P^T with another orthogonal P and
    mu ~ U[0.5, 2].  Both are symmetrised.  The interval holds ``count``
    generalized eigenvalues; M0 defaults to ceil(1.5 count)."""
    rng = _rng(seed)
    Q = _orthogonal(n, rng)
    lam = rng.uniform(-1.0, 1.0, n)
    A = (Q * lam) @ Q.T
    A = np.asfortranarray(0.5 * (A + A.T))
    B = None
    if with_B:
        P = _orthogonal(n, rng)
        mu = rng.uniform(0.5, 2.0, n)
        B = (P * mu) @ P.T
        B = np.asfortranarray(0.5 * (B + B.T))
    spec = _generalized_spectrum(A, B)
    emin, emax, _ = pick_interval(spec, count)
    if m0 is None:
        m0 = int(math.ceil(1.5 * count))
    if x0_seed is None:
        x0_seed = seed + 99
    return Problem(f"realgen{n}", A, B, emin, emax, m0, ne, tol,
                   start_subspace(n, m0, x0_seed), False, spec,
                   {"seed": seed, "x0_seed": x0_seed, "count": count})


def _clustered_spectrum(n: int, rng: np.random.Generator, nclusters: int = 16,
                        width: float = 1e-3, frac: float = 0.2) -> np.ndarray:
    n_cl = int(round(frac * n))
    n_uni = n - n_cl
    uni = rng.uniform(-1.0, 1.0, n_uni)
    centres = rng.uniform(-0.9, 0.9, nclusters)
    which = rng.integers(0, nclusters, n_cl)
    cl = centres[which] + width * rng.standard_normal(n_cl)
    return np.concatenate([uni, cl])


def dense_complex_hermitian(n: int = 8192, count: int = 400, m0: int | None = None,
                            ne: int = 16, tol: float = 1e-10, seed: int = 3001,
                            x0_seed: int | None = None, with_B: bool = True,
                            nclusters: int = 16) -> Problem:
    """Dense complex Hermitian generalized problem.

    A = U diag(lambda) U^H with U Haar unitary; lambda is 80 % U[-1, 1] and
    20 % in Gaussian clusters of width 1e-3 around centres ~ U[-0.9, 0.9].
    B = I + 0.1 H with H = (G + G^H)/2 scaled by 1/(1.01 * ||H||_2), so the
    spectrum of B lies in about [0.9, 1.1]."""
    rng = _rng(seed)
    U = _haar_unitary(n, rng)
    lam = _clustered_spectrum(n, rng, nclusters=nclusters)
    A = (U * lam) @ U.conj().T
    A = np.asfortranarray(0.5 * (A + A.conj().T))
    B = None
    if with_B:
        G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        H = 0.5 * (G + G.conj().T)
        v = rng.standard_normal(n) + 0j
        nrm = 0.0
        for _ in range(30):                 # power iteration for ||H||_2
            w = H @ v
            nrm = float(np.linalg.norm(w) / np.linalg.norm(v))
            v = w / np.linalg.norm(w)
        B = np.eye(n, dtype=np.complex128) + (0.1 / (1.01 * nrm)) * H
        B = np.asfortranarray(0.5 * (B + B.conj().T))
    spec = _generalized_spectrum(A, B)
    emin, emax, _ = pick_interval(spec, count)
    if m0 is None:
        m0 = int(math.ceil(1.5 * count))
    if x0_seed is None:
        x0_seed = seed + 99
    return Problem(f"hermgen{n}", A, B, emin, emax, m0, ne, tol,
                   start_subspace(n, m0, x0_seed), True, spec,
                   {"seed": seed, "x0_seed": x0_seed, "count": count})


def batched_specs(nprob: int = 256, nmin: int = 256, nmax: int = 2048, seed: int = 4000):
    """Sizes and seeds of the batched problems, in order: (n, count, seed, x0_seed)
    with N log-uniform on [nmin, nmax] and count = round(f N), f ~ U[0.05, 0.15]."""
    meta_rng = _rng(seed)
    out = []
    for i in range(nprob):
        n = int(round(math.exp(meta_rng.uniform(math.log(nmin), math.log(nmax)))))
        f = meta_rng.uniform(0.05, 0.15)
        count = max(1, int(round(f * n)))
        out.append((n, count, seed + 1 + i, seed + 100000 + i))
    return out


def batched_problem(spec, ne: int = 8, tol: float = 1e-10) -> Problem:
    """One problem of batched_specs, built as the dense real generalized case."""
    n, count, s, x0s = spec
    return dense_real_generalized(n, count, ne=ne, tol=tol, seed=s, x0_seed=x0s)


def batched_real_generalized(nprob: int = 256, nmin: int = 256, nmax: int = 2048,
                             ne: int = 8, tol: float = 1e-10, seed: int = 4000) -> list[Problem]:
    """Many independent real symmetric generalized problems of uneven size:
    N log-uniform on [nmin, nmax], each interval holding a fraction
    f ~ U[0.05, 0.15] of its spectrum, M0 = ceil(1.5 count)."""
    return [batched_problem(sp, ne=ne, tol=tol) for sp in batched_specs(nprob, nmin, nmax, seed)]


SERVING_SIZES = (512, 1024, 2048, 4096, 8192)


def serving_pool_matrix(n: int, k: int, seed: int = 5000):
    """Pool matrix k of size n for the request stream: a pencil built as the
    dense complex Hermitian case (seed + 100 * log2(n) + k).  Returns
    (A, B, sorted spectrum)."""
    p = dense_complex_hermitian(n, min(50, n // 8), seed=seed + 100 * int(round(math.log2(n))) + k)
    return p.A, p.B, p.spectrum


def serving_requests(spectra: dict, nreq: int, per_size, seed: int = 5000, rate: float = 200.0,
                     sizes=SERVING_SIZES, ne: int = 8, tol: float = 1e-10):
    """The request stream: Poisson arrivals at `rate` per second; N drawn with
    p(N) proportional to N^-2; a pool matrix k uniform in [0, per_size) (an
    int, or a dict of counts per N); the
    interval holds count ~ U{50..300} eigenvalues (at most N/4) around a
    uniformly drawn position of the spectrum (pick_interval); M0 = ceil(1.5
    count).  `spectra[(n, k)]` holds the pool matrices' sorted spectra.
    Returns dicts with t (arrival, seconds from the first), n, k, emin, emax,
    count, m0, ne, tol and x0_seed."""
    rng = _rng(seed + 7)
    w = np.array([1.0 / (n * n) for n in sizes])
    w /= w.sum()
    t, out = 0.0, []
    for i in range(nreq):
        if i:
            t += rng.exponential(1.0 / rate)
        n = int(sizes[rng.choice(len(sizes), p=w)])
        k = int(rng.integers(0, per_size[n] if isinstance(per_size, dict) else per_size))
        count = min(int(rng.integers(50, 301)), n // 4)
        spec = spectra[(n, k)]
        half = count // 2 + max(1, int(round(0.05 * count))) + 1
        # the interval's end gaps at least a fifth of the median gap (no end
        # inside a cluster), redrawing the position otherwise
        gmed = float(np.median(np.diff(spec)))
        for _ in range(100):
            centre = int(rng.integers(half, n - half))
            emin, emax, lo = pick_interval(spec, count, centre)
            if min(spec[lo] - spec[lo - 1], spec[lo + count] - spec[lo + count - 1]) >= 0.2 * gmed:
                break
        out.append({"t": t, "n": n, "k": k, "emin": emin, "emax": emax, "count": count,
                    "m0": int(math.ceil(1.5 * count)), "ne": ne, "tol": tol, "x0_seed": seed + 10000 + i})
    return out


def dense_general(n: int = 512, count: int = 24, m0: int | None = None, ne: int = 16, tol: float = 1e-10,
                  seed: int = 6001, real: bool = False, generalized: bool = True,
                  centre: complex = 0.2 + 0.1j) -> Problem:
    """Dense non-Hermitian pencil with a known spectrum.

    Eigenvalues: uniform in the square [-1, 1] x [-1, 1] (complex), or, for a
    real pencil, real values uniform in [-1, 1] for a fifth of them and
    conjugate pairs a +- i b for the rest.  A0 = S D S^{-1} with S = I + G /
    (2 sqrt(n)) (G Gaussian; non-normal, well conditioned) and D the
    eigenvalues (2 x 2 blocks [[a, b], [-b, a]] for real pairs).  With B =
    I + H / (4 sqrt(n)) (H Gaussian) the pencil is (B A0, B), whose
    eigenvalues are those of A0; without B it is A0.  The search region is
    the circle about ``centre`` (on the real axis for a real pencil) through
    the midpoint between the count-th and (count+1)-th nearest eigenvalues, so
    ``count`` eigenvalues lie inside (one more when the count-th is half of a
    conjugate pair; meta["count"] holds the number).  emin, emax of the returned Problem hold Emid (complex) and r;
    spectrum holds the eigenvalues; X0 holds right and left start subspaces
    (n x 2 M0, real uniform(-1, 1))."""
    rng = _rng(seed)
    if real:
        centre = complex(centre.real, 0.0)
        nreal = n // 5
        npair = (n - nreal) // 2
        nreal = n - 2 * npair
        lr = rng.uniform(-1.0, 1.0, nreal)
        a = rng.uniform(-1.0, 1.0, npair)
        b = rng.uniform(0.05, 1.0, npair)
        D = np.zeros((n, n))
        D[np.arange(nreal), np.arange(nreal)] = lr
        for k in range(npair):
            i = nreal + 2 * k
            D[i, i] = D[i + 1, i + 1] = a[k]
            D[i, i + 1] = b[k]
            D[i + 1, i] = -b[k]
        lam = np.concatenate([lr + 0j, a + 1j * b, a - 1j * b])
        S = np.eye(n) + rng.standard_normal((n, n)) / (2.0 * math.sqrt(n))
        A0 = S @ D @ np.linalg.inv(S)
        Bm = np.eye(n) + rng.standard_normal((n, n)) / (4.0 * math.sqrt(n)) if generalized else None
    else:
        lam = rng.uniform(-1.0, 1.0, n) + 1j * rng.uniform(-1.0, 1.0, n)
        G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
        S = np.eye(n) + G / (2.0 * math.sqrt(n))
        A0 = (S * lam) @ np.linalg.inv(S)
        H = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
        Bm = np.eye(n) + H / (4.0 * math.sqrt(n)) if generalized else None
    A = A0 if Bm is None else Bm @ A0
    d = np.sort(np.abs(lam - centre))
    while count < n and d[count] - d[count - 1] < 1e-9:   # keep conjugate pairs together
        count += 1
    r = 0.5 * (d[count - 1] + d[count])
    if m0 is None:
        m0 = int(math.ceil(1.5 * count)) + 4
    x0 = _rng(seed + 99).uniform(-1.0, 1.0, size=(n, 2 * m0))
    return Problem(f"general{n}{'r' if real else 'c'}", np.asfortranarray(A),
                   None if Bm is None else np.asfortranarray(Bm), centre, r, m0, ne, tol,
                   np.asfortranarray(x0), not real, lam, {"seed": seed, "count": count})
