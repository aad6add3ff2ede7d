"""Host-side checks of the batched LU's launch schedule (feast_lu_schedule).

The library issues the factorisation of every contour node (the LU of
z_j B - A, "The FEAST Algorithm") as a fixed list of steps that depends only
on the order n and on whether a second stream factors the panels.  These
tests take that list from the library and replay it on the CPU:

* numerically, with numpy standing in for each kernel (panel factorisation
  with partial pivoting, row interchanges with the U-row solve and the
  correction by earlier panels, trailing products), and check that the
  result is an LU factorisation of the row-permuted input;
* as a two-stream program: from stream order and the event records and
  waits, every pair of steps that may run at the same time must touch
  disjoint parts of the matrix, the move lists and the permutation.

No GPU is needed.
"""
import numpy as np
import pytest

from paper_1203_4031_amd import feastx

PANEL, SWAP, GEMM, RECORD, WAIT = range(5)
LU_NB = 32
CORR_MAX = 3 * LU_NB

SIZES = [1, 5, 31, 32, 33, 64, 100, 127, 128, 129, 200, 255, 256, 257, 300, 383, 384, 385, 512, 600, 700, 1100]


FORMS = ["pairs", "blocks"]
BLOCKS_MIN_N = 6144   # the library's switch from the paired to the blocked schedule


def _ops(n, side, form="auto"):
    return [dict(zip(feastx.LU_OP_FIELDS, map(int, row))) for row in feastx.lu_schedule(n, side, form)]


def _replay(A, ops):
    """Run the schedule's steps in list order with numpy kernels."""
    n = A.shape[0]
    F = A.copy()
    perm = np.arange(n)
    lists = {}
    for o in ops:
        k, nbw = o["k"], o["nbw"]
        if o["kind"] == PANEL:
            assert nbw == min(LU_NB, n - k)
            piv = []
            for c in range(k, k + nbw):
                p = c + int(np.argmax(np.abs(F[c:, c].real) + np.abs(F[c:, c].imag)))
                piv.append(p)
                F[[c, p], k:k + nbw] = F[[p, c], k:k + nbw]
                perm[[c, p]] = perm[[p, c]]
                F[c + 1:, c] /= F[c, c]
                F[c + 1:, c + 1:k + nbw] -= np.outer(F[c + 1:, c], F[c, c + 1:k + nbw])
            lists[o["list"]] = (k, nbw, piv)
        elif o["kind"] == SWAP:
            lk, lnbw, piv = lists[o["list"]]
            assert (lk, lnbw) == (k, nbw), "a step reads another panel's move list"
            cols = np.r_[o["c0"]:o["c1"], o["c2"]:o["c3"]].astype(int)
            assert len(cols) > 0
            assert not np.any((cols >= k) & (cols < k + nbw)), "interchange step on its own panel's columns"
            if o["mode"] & 1:
                for i, p in enumerate(piv):
                    rows = F[[k + i, p]][:, cols]
                    F[k + i, cols], F[p, cols] = rows[1], rows[0]
            if o["mode"] & 2:
                right = cols[cols >= k + nbw]
                if o["mode"] & 4:
                    kc0, kc1 = o["kc0"], o["kc1"]
                    assert kc1 == k and 0 <= kc0 < kc1 and kc1 - kc0 <= CORR_MAX
                    F[k:k + nbw, right] -= F[k:k + nbw, kc0:kc1] @ F[kc0:kc1, right]
                L11 = np.tril(F[k:k + nbw, k:k + nbw], -1) + np.eye(nbw)
                F[k:k + nbw, right] = np.linalg.solve(L11, F[k:k + nbw, right])
        elif o["kind"] == GEMM:
            r0, r1, c0, c1, kc0, kc1 = (o[x] for x in ("c0", "c1", "c2", "c3", "kc0", "kc1"))
            assert 0 <= r0 < r1 <= n and 0 <= c0 < c1 <= n and 0 <= kc0 < kc1 <= n
            F[r0:r1, c0:c1] -= F[r0:r1, kc0:kc1] @ F[kc0:kc1, c0:c1]
    return F, perm


def _rects(o, n):
    """(writes, reads) of one step: rectangles (r0, r1, c0, c1) of the
    matrix and named resources ('list3', 'perm')."""
    k, nbw = o["k"], o["nbw"]
    W, R = [], []
    if o["kind"] == PANEL:
        W += [(k, n, k, k + nbw), f"list{o['list']}", "perm"]
    elif o["kind"] == SWAP:
        R.append(f"list{o['list']}")
        for c0, c1 in ((o["c0"], o["c1"]), (o["c2"], o["c3"])):
            if c1 > c0:
                W.append((k, n, c0, c1))
                if o["mode"] & 2 and c1 > k + nbw:
                    R.append((k, k + nbw, k, k + nbw))
                    if o["mode"] & 4:
                        R.append((k, k + nbw, o["kc0"], o["kc1"]))
                        R.append((o["kc0"], o["kc1"], max(c0, k + nbw), c1))
    elif o["kind"] == GEMM:
        r0, r1, c0, c1, kc0, kc1 = (o[x] for x in ("c0", "c1", "c2", "c3", "kc0", "kc1"))
        W.append((r0, r1, c0, c1))
        R += [(r0, r1, kc0, kc1), (kc0, kc1, c0, c1)]
    return W, R


def _overlap(a, b):
    if isinstance(a, str) or isinstance(b, str):
        return a == b
    return a[0] < b[1] and b[0] < a[1] and a[2] < b[3] and b[2] < a[3]


def _races(ops, n, side):
    """Pairs of steps that no stream order or event orders, with a conflict."""
    m = len(ops)
    stream = [1 if (o["side"] and side) else 0 for o in ops]
    preds = [[] for _ in range(m)]
    last_on = {0: None, 1: None}
    last_record = {0: None, 1: None}
    for i, o in enumerate(ops):
        s = stream[i]
        if last_on[s] is not None:
            preds[i].append(last_on[s])
        last_on[s] = i
        if o["kind"] == RECORD:
            last_record[s] = i
        elif o["kind"] == WAIT:
            r = last_record[1 - s]
            assert r is not None, "a wait with no record before it"
            preds[i].append(r)
    anc = [0] * m   # bitsets of ancestors
    for i in range(m):
        a = 0
        for p in preds[i]:
            a |= anc[p] | (1 << p)
        anc[i] = a
    acc = [_rects(o, n) for o in ops]
    bad = []
    for i in range(m):
        for j in range(i):
            if stream[i] == stream[j] or (anc[i] >> j) & 1:
                continue
            Wi, Ri = acc[i]
            Wj, Rj = acc[j]
            if any(_overlap(a, b) for a in Wi for b in Wj + Rj) or any(_overlap(a, b) for a in Wj for b in Ri):
                bad.append((j, i))
    return bad


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("side", [False, True])
def test_schedule_factors(n, side, form):
    rng = np.random.default_rng(1000 + n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    ops = _ops(n, side, form)
    F, perm = _replay(A, ops)
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    # pivots by |re| + |im|, which bounds |l| by sqrt(2)
    assert np.all(np.abs(np.tril(F, -1)) <= np.sqrt(2) * (1 + 1e-12)), "L is not from partial pivoting"
    err = np.linalg.norm(A[perm] - L @ U) / np.linalg.norm(A)
    assert err < 1e-12, err
    assert sorted(perm) == list(range(n))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n", [100, 257, 385, 700, 1100, 4096, 6144, 8192])
def test_schedule_two_streams_race_free(n, form):
    ops = _ops(n, True, form)
    assert any(o["side"] for o in ops)
    assert _races(ops, n, True) == []


def test_schedule_shape():
    """Panels run on the panel stream, in column order, each once; every
    trailing product past a block's next block has depth 128."""
    n = 4096
    ops = _ops(n, True, "blocks")
    ks = [o["k"] for o in ops if o["kind"] == PANEL]
    assert ks == list(range(0, n, LU_NB))
    assert all(o["side"] == 1 for o in ops if o["kind"] == PANEL)
    assert all(o["side"] == 0 for o in ops if o["kind"] in (SWAP, GEMM))
    deep = [o for o in ops if o["kind"] == GEMM and o["kc1"] - o["kc0"] > LU_NB]
    assert deep and all(o["kc1"] - o["kc0"] == 4 * LU_NB for o in deep)
    # the flops in depth-128 products: all but the panels' narrow updates
    # (93 % at this order, 97 % at 8192)
    fl = lambda o: (o["c1"] - o["c0"]) * (o["c3"] - o["c2"]) * (o["kc1"] - o["kc0"])
    total = sum(fl(o) for o in ops if o["kind"] == GEMM)
    assert sum(fl(o) for o in deep) > 0.9 * total
    # without a panel stream: the same steps in the same order, no events
    one = _ops(n, False, "blocks")
    strip = lambda v: [{**o, "side": 0} for o in v if o["kind"] not in (RECORD, WAIT)]
    assert strip(ops) == strip(one)


def test_schedule_choice():
    """The library runs the paired schedule below its switch order and the
    blocked one from there; the paired one keeps every product at depth 64
    or less."""
    for n in (512, 4096, BLOCKS_MIN_N - 1):
        assert _ops(n, True) == _ops(n, True, "pairs")
    for n in (BLOCKS_MIN_N, 8192):
        assert _ops(n, True) == _ops(n, True, "blocks")
    assert max(o["kc1"] - o["kc0"] for o in _ops(4096, True, "pairs") if o["kind"] == GEMM) == 64
    with pytest.raises(ValueError):
        feastx.lu_schedule(0, True)
    # a forced form applies to every order, until set back
    assert feastx.lu_form() == "auto"
    try:
        feastx.set_lu_form("blocks")
        assert _ops(512, True) == _ops(512, True, "blocks")
        feastx.set_lu_form("pairs")
        assert _ops(8192, True) == _ops(8192, True, "pairs")
        assert feastx.lu_form() == "pairs"
    finally:
        feastx.set_lu_form("auto")
    assert _ops(8192, True) == _ops(8192, True, "blocks")
    with pytest.raises(KeyError):
        feastx.set_lu_form("quads")
    assert feastx.lib().feast_set_lu_form(2) == -1 and feastx.lu_form() == "auto"


def test_checks_catch_planted_mistakes():
    """The race check and the replay are not vacuous: each planted mistake in
    a copy of the schedule is caught."""
    n = 300
    ops = _ops(n, True, "blocks")
    waits = [i for i, o in enumerate(ops) if o["kind"] == WAIT and o["side"] == 0]
    assert waits
    for w in (waits[0], waits[len(waits) // 2], waits[-1]):
        assert _races(ops[:w] + ops[w + 1:], n, True), f"dropping wait {w} went unnoticed"
    # a trailing product taken at depth 64 instead of 128
    i = next(i for i, o in enumerate(ops) if o["kind"] == GEMM and o["kc1"] - o["kc0"] == 128)
    bad = [dict(o) for o in ops]
    bad[i]["kc0"] += 64
    rng = np.random.default_rng(5)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    F, perm = _replay(A, bad)
    L = np.tril(F, -1) + np.eye(n)
    assert np.linalg.norm(A[perm] - L @ np.triu(F)) / np.linalg.norm(A) > 1e-3
