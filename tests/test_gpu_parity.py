"""GPU parity: every output of the HIP library equals the CPU oracle's,
bit for bit (integer arithmetic in GF(p): the tolerance is zero).

Inputs are seeded (paper_1112_5717_amd.inputs and the structured generator
of the oracle pins); sizes span several 64-row leaves, 64-column windows
and 128 x 128 ffgemm tiles with ragged tails.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1112_5717_amd import inputs
from test_oracle_pins import structured

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a: np.ndarray, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t) -> np.ndarray:
    return t.cpu().numpy().astype(np.int64)


def run_cup(cup, A: np.ndarray, p: int, i8=False):
    d = dev(A, torch.int8 if i8 else torch.int64)
    r, P, Q = (cup.cup_factor_i8 if i8 else cup.cup_factor)(d, p)
    return host(d), r, host(P), host(Q)


def assert_same_cup(got, ref, label=""):
    packed, r, P, Q = got
    rp, rr, rP, rQ = ref
    assert r == rr, f"{label}: rank {r} != {rr}"
    assert np.array_equal(P, rP), f"{label}: P differs at {np.flatnonzero(P != rP)[:8]}"
    assert np.array_equal(Q, rQ), f"{label}: Q differs at {np.flatnonzero(Q != rQ)[:8]}"
    if not np.array_equal(packed, rp):
        bad = np.argwhere(packed != rp)
        raise AssertionError(f"{label}: packed [C\\U] differs at {len(bad)} entries, first {bad[:5].tolist()}")


# ------------------------------------------------------------------ ffgemm

def exact_gemm(C, A, B, p, alpha):
    """C + alpha A B mod p from the CPU oracle's matrix product (Algorithm 1's
    black box written out from the definition; pinned by a product worked by
    hand in tests/golden/mm_gf7_by_hand.txt)."""
    i64 = lambda X: np.asarray(X, dtype=np.int64)
    return oracle.mm(i64(C), i64(A), i64(B), p, alpha)


@pytest.mark.parametrize("p", [2, 127, 65521, 8388593, 33554393])
@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 5, 3), (130, 129, 17), (257, 131, 200), (64, 300, 513),
                                   (300, 130, 64), (129, 65, 63), (4100, 64, 64), (65, 1000, 33),
                                   (150, 300, 128), (64, 700, 256), (200, 90, 129)])
def test_ffgemm_fp64_random(cup_lib, p, shape):
    M, N, K = shape
    rng = np.random.default_rng(M * 7 + N + K + p % 1000)
    A = rng.integers(0, p, size=(M, K), dtype=np.int64)
    B = rng.integers(0, p, size=(K, N), dtype=np.int64)
    C = rng.integers(0, p, size=(M, N), dtype=np.int64)
    for alpha in (-1, 1):
        dC = dev(C)
        cup_lib.cup_set_form("fp64")
        cup_lib.cup_ffgemm(dC, dev(A), dev(B), p, alpha)
        assert np.array_equal(host(dC), exact_gemm(C, A, B, p, alpha))


@pytest.mark.parametrize("p", [127, 65521, 8388593, 33554393])
@pytest.mark.parametrize("K", [2100, 256, 128])
def test_ffgemm_fp64_worst_magnitude(cup_lib, p, K):
    """All operands at p-1 and at the centring threshold: the largest
    products, at and beyond the delayed-reduction interval (K = 2100), and
    through the single-stage 128-deep launches (K = 128, 256)."""
    h = p // 2
    for val_a, val_b in [(p - 1, p - 1), (h, h), (h + 1, h + 1), (h, h + 1)]:
        M, N = 96, 80
        A = np.full((M, K), val_a, dtype=np.int64)
        B = np.full((K, N), val_b, dtype=np.int64)
        C = np.full((M, N), p - 1, dtype=np.int64)
        dC = dev(C)
        cup_lib.cup_set_form("fp64")
        cup_lib.cup_ffgemm(dC, dev(A), dev(B), p, -1)
        assert np.array_equal(host(dC), exact_gemm(C, A, B, p, -1))


def test_ffgemm_views(cup_lib):
    """Operands and result as strided sub-views of one matrix (as in CUP)."""
    p = 65521
    rng = np.random.default_rng(5)
    X = rng.integers(0, p, size=(300, 400), dtype=np.int64)
    d = dev(X)
    cup_lib.cup_ffgemm(d[150:, 100:], d[150:, :77], d[:77, 100:], p, -1)
    ref = X.copy()
    ref[150:, 100:] = exact_gemm(X[150:, 100:], X[150:, :77], X[:77, 100:], p, -1)
    assert np.array_equal(host(d), ref)


# ------------------------------------------------------------------ CUP

CUP_CASES = [
    # (m, n, p, rank or None, structured?)
    (1, 1, 7, None, False), (1, 9, 7, None, True), (9, 1, 7, None, True),
    (5, 5, 2, None, True), (64, 64, 65521, None, False), (65, 63, 101, None, True),
    (100, 150, 3, None, True), (150, 100, 65521, 40, True), (200, 300, 65521, None, True),
    (257, 129, 127, None, True), (128, 520, 2, None, True), (333, 333, 8388593, None, False),
    (400, 260, 65521, 130, False), (300, 300, 33554393, 250, True), (129, 700, 101, None, True),
    # full-rank squares: cached diagonal-block inverses and the fused right
    # solve (orders 64..1024), with a prime past the 64-term bound
    (1100, 1100, 65521, None, False), (2100, 2100, 33554393, None, False),
    (1500, 1300, 8388593, None, False), (1088, 1200, 2, None, False),
    # the INT8-limb right solve at other primes and ragged row counts
    (1300, 1100, 32771, None, False), (777, 1500, 257, None, False),
]


@pytest.mark.parametrize("case", CUP_CASES, ids=[f"{c[0]}x{c[1]}p{c[2]}r{c[3]}" for c in CUP_CASES])
def test_cup_vs_oracle(cup_lib, case):
    m, n, p, rank, struct = case
    if struct:
        A = structured(m, n, p, m * 31 + n, rank=rank)
    elif rank is not None:
        A = inputs.low_rank(m, n, rank, p, seed=m + n)
    else:
        A = inputs.uniform((m, n), p, seed=m * n)
    cup_lib.cup_set_form("auto")
    assert_same_cup(run_cup(cup_lib, A, p), oracle.cup(A, p), f"{m}x{n} p={p}")


def test_cup_edge_matrices(cup_lib):
    p = 65521
    cases = [np.zeros((70, 90), np.int64), np.zeros((1, 200), np.int64)]
    Z = np.zeros((130, 140), np.int64)
    Z[129, 139] = 5            # single nonzero, last row and column
    cases.append(Z)
    R1 = np.outer(np.arange(1, 131) % p, np.arange(3, 143) % p) % p   # rank 1
    cases.append(R1.astype(np.int64))
    E = inputs.uniform((200, 150), p, seed=3)
    E[:, :70] = 0              # leading zero columns: pivots beyond every window
    cases.append(E)
    F = inputs.uniform((150, 300), p, seed=4)
    F[:64] = 0                 # top half rank 0 (r1 = 0 at the first split)
    cases.append(F)
    for A in cases:
        assert_same_cup(run_cup(cup_lib, A, p), oracle.cup(A, p), f"edge {A.shape}")


def test_cup_empty(cup_lib):
    for m, n in [(0, 5), (5, 0), (0, 0)]:
        A = torch.zeros((m, n), dtype=torch.int64, device="cuda")
        r, P, Q = cup_lib.cup_factor(A, 7)
        assert r == 0
        assert np.array_equal(host(P), np.arange(n)) and np.array_equal(host(Q), np.arange(m))


def test_cup_config1(cup_lib):
    """512 x 384 over GF(65521), A = X(512x300) Y(300x384), seed 1: rank 300."""
    p = 65521
    A = inputs.low_rank(512, 384, 300, p, seed=1)
    got = run_cup(cup_lib, A, p)
    assert got[1] == 300
    assert_same_cup(got, oracle.cup(A, p), "config 1")


def test_cup_staircase(cup_lib):
    p = 65521
    A, piv = inputs.staircase(700, 300, 90, p, seed=5)
    got = run_cup(cup_lib, A, p)
    assert got[1] == 90 and np.array_equal(got[3][:90], piv)
    assert_same_cup(got, oracle.cup(A, p), "staircase")


@pytest.mark.parametrize("m,n,r,p,seed", [(256, 17000, 40, 65521, 21), (200, 16600, 25, 3, 22)])
def test_cup_staircase_wide(cup_lib, m, n, r, p, seed):
    """Rank-deficient leaves wider than 256 x 64 columns: workgroups of the
    sparse kernel own two column chunks, the second read from memory each
    round (the first stays in registers)."""
    A, piv = inputs.staircase(m, n, r, p, seed=seed)
    got = run_cup(cup_lib, A, p)
    assert got[1] == r and np.array_equal(got[3][:r], piv)
    assert_same_cup(got, oracle.cup(A, p), f"wide staircase {m}x{n} p={p}")


@pytest.mark.parametrize("p", [2, 3, 127])
def test_cup_i8(cup_lib, p):
    for m, n, rank in [(70, 90, None), (300, 200, None), (256, 256, 100)]:
        A = structured(m, n, p, m + n + p, rank=rank)
        got = run_cup(cup_lib, A, p, i8=True)
        assert_same_cup(got, oracle.cup(A, p), f"i8 {m}x{n} p={p}")


def test_rank_profile(cup_lib):
    p = 101
    A = structured(200, 150, p, 77, rank=60)
    d = dev(A)
    r, Q = cup_lib.cup_rank_profile(d, p)
    ref = oracle.cup(A, p)
    assert r == ref[1] and np.array_equal(host(Q), ref[3])


# ------------------------------------------------------------ RREF / inverse

RREF_CASES = [(10, 12, 7, None), (100, 80, 65521, None), (150, 200, 101, 70), (300, 140, 65521, None),
              (90, 300, 3, None), (260, 260, 127, 200)]


@pytest.mark.parametrize("case", RREF_CASES, ids=[f"{c[0]}x{c[1]}p{c[2]}" for c in RREF_CASES])
def test_rref_vs_oracle(cup_lib, case):
    m, n, p, rank = case
    A = structured(m, n, p, m * 3 + n, rank=rank)
    d = dev(A)
    r, P, Q = cup_lib.cup_rref_inplace(d, p)
    O, rr, rP, rQ = oracle.rref_packed(A, p)
    assert r == rr and np.array_equal(host(P), rP) and np.array_equal(host(Q), rQ)
    assert np.array_equal(host(d), O)


@pytest.mark.parametrize("n,p", [(1, 7), (37, 65521), (130, 101), (200, 2), (257, 8388593)])
def test_inverse_vs_oracle(cup_lib, n, p):
    seed = n
    while True:
        A = inputs.uniform((n, n), p, seed=seed)
        X = oracle.inverse(A, p)
        if X is not None:
            break
        seed += 1000
    d = dev(A)
    ok, r = cup_lib.cup_inverse_inplace(d, p)
    assert ok and r == n
    assert np.array_equal(host(d), X)


def test_inverse_singular(cup_lib):
    p = 65521
    A = inputs.low_rank(100, 100, 60, p, seed=8)
    ok, r = cup_lib.cup_inverse_inplace(dev(A), p)
    assert not ok and r == 60


def test_inverse_i8(cup_lib):
    p = 127
    seed = 30
    while True:
        A = inputs.uniform((150, 150), p, seed=seed)
        X = oracle.inverse(A, p)
        if X is not None:
            break
        seed += 1
    d = dev(A, torch.int8)
    ok, r = cup_lib.cup_inverse_inplace_i8(d, p)
    assert ok and np.array_equal(host(d), X)


# ------------------------------------------------------------------ batched

def _check_batched(cup_lib, hosts, ps, mats=None, views=None, want_pq=True):
    mats = mats if mats is not None else [dev(A) for A in hosts]
    views = views if views is not None else mats
    rank, info, Ps, Qs = cup_lib.cup_factor_batched(views, ps, want_pq=want_pq)
    rank, info = host(rank), host(info)
    for i, A in enumerate(hosts):
        ref = oracle.cup(A, ps[i])
        assert info[i] == 0, (i, info[i])
        assert rank[i] == ref[1], (i, A.shape, ps[i], rank[i], ref[1])
        if want_pq:
            assert np.array_equal(host(Ps[i]), ref[2]), (i, "P")
            assert np.array_equal(host(Qs[i]), ref[3]), (i, "Q")
        got = host(views[i])
        if not np.array_equal(got, ref[0]):
            bad = np.argwhere(got != ref[0])
            raise AssertionError(f"matrix {i} {A.shape} p={ps[i]}: {len(bad)} entries differ, "
                                 f"first {bad[:5].tolist()}")
    return mats


def test_batched_small(cup_lib):
    """The multi-modular workload's recipe at small sizes: m, n ~ U[16, 90]."""
    primes = inputs.largest_primes_below(2 ** 23, 32)
    m, n, r = inputs.batch_specs(40, 16, 90, seed=4)
    hosts = [inputs.batch_matrix(i, m[i], n[i], r[i], primes[i % 32], seed=4) for i in range(40)]
    _check_batched(cup_lib, hosts, [primes[i % 32] for i in range(40)])


def test_batched_recipe_full_range(cup_lib):
    """m, n ~ U[16, 512], ranks ~ U[1, min(m, n)]: several 64-row blocks,
    positions in every register block, more than 128 pending updates."""
    primes = inputs.largest_primes_below(2 ** 23, 32)
    m, n, r = inputs.batch_specs(24, 16, 512, seed=41)
    hosts = [inputs.batch_matrix(i, m[i], n[i], r[i], primes[i % 32], seed=41) for i in range(24)]
    _check_batched(cup_lib, hosts, [primes[i % 32] for i in range(24)])


def test_batched_shapes_and_primes(cup_lib):
    """Edge shapes, structured rank profiles, primes from 2 to the largest below 2^26."""
    cases = []
    for (mm, nn, rr, p, seed) in [(1, 1, 1, 2, 0), (1, 512, 1, 3, 1), (512, 1, 1, 65521, 2),
                                  (512, 512, 512, 8388593, 3), (64, 64, 64, 2, 4), (65, 65, 40, 3, 5),
                                  (300, 500, 7, 33554393, 6), (130, 200, 130, 65521, 7),
                                  (200, 130, 129, 8388593, 8), (129, 511, 100, 5, 9),
                                  (260, 300, 200, 67108859, 15), (256, 256, 256, 67108859, 16)]:
        cases.append((inputs.low_rank(mm, nn, rr, p, seed=seed), p))
    cases.append((np.zeros((70, 90), np.int64), 65521))
    cases.append((inputs.staircase(300, 257, 60, 8388593, seed=11)[0], 8388593))
    cases.append((structured(150, 140, 65521, seed=12), 65521))
    cases.append((structured(200, 300, 3, seed=13, rank=90), 3))
    cases.append((structured(512, 512, 8388593, seed=14), 8388593))
    hosts = [c[0] for c in cases]
    ps = [c[1] for c in cases]
    _check_batched(cup_lib, hosts, ps)


def test_batched_strided_and_no_pq(cup_lib):
    """lda > n (the padding is left alone) and P = Q = NULL."""
    p = 8388593
    hosts = [inputs.low_rank(100, 70, 50, p, seed=21), inputs.low_rank(260, 300, 260, p, seed=22)]
    bigs, views = [], []
    for A in hosts:
        big = np.full((A.shape[0], A.shape[1] + 9), 7, dtype=np.int64)
        big[:, :A.shape[1]] = A
        d = dev(big)
        bigs.append(d)
        views.append(d[:, :A.shape[1]])
    _check_batched(cup_lib, hosts, [p, p], mats=bigs, views=views, want_pq=False)
    for d, A in zip(bigs, hosts):
        assert np.all(host(d)[:, A.shape[1]:] == 7)


def test_batched_argument_errors(cup_lib):
    """Per-matrix codes: composite or out-of-range p -> -5; n > 512 is
    routed to the single-matrix path by cup_factor_batched (a zero 3 x 513
    matrix: rank 0) and refused with -2 by the allocation-free variant;
    empty matrices give rank 0 and identity P, Q; the others still run."""
    A_ok = inputs.low_rank(40, 30, 20, 65521, seed=31)
    for name, wide_code in (("cup_factor_batched", 0), ("cup_factor_batched_noalloc", -2)):
        mats = [dev(A_ok), dev(np.zeros((3, 513), np.int64)), dev(A_ok), dev(A_ok),
                dev(np.zeros((0, 5), np.int64)), dev(np.zeros((4, 0), np.int64))]
        ps = [65521, 65521, 65519 * 3, 1 << 26, 65521, 65521]
        rank, info, Ps, Qs = cup_lib.cup_factor_batched(mats, ps, name=name)
        torch.cuda.synchronize()
        info, rank = host(info), host(rank)
        assert info.tolist() == [0, wide_code, -5, -5, 0, 0], name
        assert rank[1] == 0
        if wide_code == 0:
            assert np.array_equal(host(Ps[1]), np.arange(513)) and np.array_equal(host(Qs[1]), np.arange(3))
        ref = oracle.cup(A_ok, 65521)
        assert rank[0] == ref[1] and np.array_equal(host(mats[0]), ref[0])
        assert rank[4] == 0 and rank[5] == 0
        assert np.array_equal(host(Ps[4]), np.arange(5)) and np.array_equal(host(Qs[5]), np.arange(4))
        assert np.array_equal(host(mats[2]), A_ok) and np.array_equal(host(mats[3]), A_ok)


def test_batched_wide_matrices_routed(cup_lib):
    """Matrices wider than the batched kernels (n > 512) among ordinary ones:
    cup_factor_batched factors them by the recursive path; every result
    equals the oracle's."""
    primes = inputs.largest_primes_below(2 ** 23, 32)
    cases = [(700, 600, 500, 65521), (100, 90, 60, primes[0]), (64, 1000, 64, primes[1]),
             (300, 513, 300, 8388593), (40, 30, 20, primes[2]), (513, 900, 400, 101)]
    hosts = [inputs.low_rank(mm, nn, rr, p, seed=mm + nn) for mm, nn, rr, p in cases]
    _check_batched(cup_lib, hosts, [c[3] for c in cases])


def test_batched_graph_replay(cup_lib):
    """The allocation-free batched call captured in a HIP graph (through
    torch's graph capture) and replayed three times, with eager library work
    between the replays: every replay equals the eager result."""
    primes = inputs.largest_primes_below(2 ** 23, 32)
    m, n, r = inputs.batch_specs(60, 16, 512, seed=77)
    ps = [primes[i % 32] for i in range(60)]
    fb = cup_lib.FlatBatch(m, n, ps)
    src = torch.empty(fb.size, dtype=torch.int64, device="cuda")
    for i in range(60):
        A = inputs.batch_matrix(i, m[i], n[i], r[i], ps[i], seed=77)
        o = int(fb.offsets[i])
        src[o:o + A.size].copy_(torch.from_numpy(A.reshape(-1)))
    work = src.clone()
    ptrs = fb.pointers(work)
    fb.factor(ptrs, name="cup_factor_batched_noalloc")  # eager reference (and first-use set-up)
    torch.cuda.synchronize()
    ref = (work.clone(), fb.rank.clone(), fb.P.clone(), fb.Q.clone(), fb.info.clone())
    assert not ref[4].any()
    graph = torch.cuda.CUDAGraph()
    work.copy_(src)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        fb.factor(ptrs, name="cup_factor_batched_noalloc")
    other = torch.from_numpy(inputs.uniform((200, 150), 65521, seed=5)).cuda()
    for rep in range(3):
        work.copy_(src)
        fb.rank.zero_()
        fb.P.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(work, ref[0]), f"replay {rep}: matrices differ"
        assert torch.equal(fb.rank, ref[1]) and torch.equal(fb.P, ref[2]) and torch.equal(fb.Q, ref[3])
        assert not fb.info.any()
        cup_lib.cup_factor(other.clone(), 65521)  # eager work between replays
        torch.cuda.synchronize()


# --------------------------------------------------------------- INT8 forms

def _i8_small_products(monkeypatch):
    """Send every product with M, N >= 128 and K >= 64 to the INT8 kernels."""
    monkeypatch.setenv("CUP_I8_MIN_WORK", "0")


@pytest.mark.parametrize("form,p,dtype", [("i8", 127, "int8"), ("i8", 2, "int8"), ("i8", 3, "int64"),
                                          ("i8limb", 65521, "int64"), ("i8limb", 257, "int64"),
                                          ("i8limb", 2, "int64"), ("i8limb", 32771, "int64")])
@pytest.mark.parametrize("shape", [(128, 128, 64), (300, 200, 513), (640, 384, 1000)])
def test_ffgemm_int8_forms(cup_lib, monkeypatch, form, p, dtype, shape):
    _i8_small_products(monkeypatch)
    M, N, K = shape
    rng = np.random.default_rng(M + N + K + p)
    A = rng.integers(0, p, size=(M, K), dtype=np.int64)
    B = rng.integers(0, p, size=(K, N), dtype=np.int64)
    C = rng.integers(0, p, size=(M, N), dtype=np.int64)
    tdt = torch.int8 if dtype == "int8" else torch.int64
    cup_lib.cup_set_form(form)
    try:
        for alpha in (-1, 1):
            dC = dev(C, tdt)
            cup_lib.cup_ffgemm(dC, dev(A, tdt), dev(B, tdt), p, alpha)
            assert np.array_equal(host(dC), exact_gemm(C, A, B, p, alpha)), (form, p, alpha)
    finally:
        cup_lib.cup_set_form("auto")


@pytest.mark.parametrize("p", [65521, 40009])
def test_ffgemm_limb_window_extremes(cup_lib, monkeypatch, p):
    """Residues at both ends of the signed limb window and at p - 1."""
    _i8_small_products(monkeypatch)
    vals = np.array([0, 1, 127, 128, 255, 256, 32639, 32640, p - 129, p - 128, p - 1], dtype=np.int64) % p
    M, N, K = 256, 192, 4160
    rng = np.random.default_rng(p)
    A = vals[rng.integers(0, len(vals), size=(M, K))]
    B = vals[rng.integers(0, len(vals), size=(K, N))]
    A[:8, :] = p - 1
    B[:, :8] = p - 1
    A[8:16, :] = 32640 % p
    B[:, 8:16] = 32640 % p
    C = np.full((M, N), p - 1, dtype=np.int64)
    cup_lib.cup_set_form("i8limb")
    try:
        dC = dev(C)
        cup_lib.cup_ffgemm(dC, dev(A), dev(B), p, -1)
        assert np.array_equal(host(dC), exact_gemm(C, A, B, p, -1))
    finally:
        cup_lib.cup_set_form("auto")


def _i8_direct_products(monkeypatch):
    """Keep every product below the packed kernel's work threshold, so that
    every product with K > 64 takes the direct INT8-limb kernel."""
    monkeypatch.setenv("CUP_I8_MIN_WORK", "1e30")


@pytest.mark.parametrize("form,p,dtype", [("i8limb", 65521, "int64"), ("i8limb", 257, "int64"),
                                          ("i8limb", 2, "int64"), ("i8limb", 32771, "int64"),
                                          ("i8", 127, "int8"), ("i8", 3, "int64")])
@pytest.mark.parametrize("shape", [(1, 1, 65), (63, 65, 129), (200, 300, 513), (128, 2100, 128),
                                   (70, 40, 1000), (8, 9, 70000)])
def test_ffgemm_direct_i8(cup_lib, monkeypatch, form, p, dtype, shape):
    """The direct INT8-limb product: ragged tiles, K tails, and K beyond one
    launch's exact accumulation (70000 > 65472 terms: two launches)."""
    _i8_direct_products(monkeypatch)
    M, N, K = shape
    rng = np.random.default_rng(M * 3 + N + K + p)
    A = rng.integers(0, p, size=(M, K), dtype=np.int64)
    B = rng.integers(0, p, size=(K, N), dtype=np.int64)
    C = rng.integers(0, p, size=(M, N), dtype=np.int64)
    tdt = torch.int8 if dtype == "int8" else torch.int64
    cup_lib.cup_set_form(form)
    try:
        for alpha in (-1, 1):
            dC = dev(C, tdt)
            cup_lib.cup_ffgemm(dC, dev(A, tdt), dev(B, tdt), p, alpha)
            assert np.array_equal(host(dC), exact_gemm(C, A, B, p, alpha)), (form, p, alpha)
    finally:
        cup_lib.cup_set_form("auto")


@pytest.mark.parametrize("p", [65521, 40009])
def test_ffgemm_direct_limb_extremes(cup_lib, monkeypatch, p):
    """Residues at both ends of the signed limb window and at p - 1, summed
    over a full launch's worth of terms, through the direct kernel."""
    _i8_direct_products(monkeypatch)
    vals = np.array([0, 1, 127, 128, 255, 256, 32639, 32640, p - 129, p - 128, p - 1], dtype=np.int64) % p
    M, N, K = 96, 80, 65472
    rng = np.random.default_rng(p + 1)
    A = vals[rng.integers(0, len(vals), size=(M, K))]
    B = vals[rng.integers(0, len(vals), size=(K, N))]
    A[:8, :] = p - 1
    B[:, :8] = p - 1
    A[8:16, :] = 32640 % p
    B[:, 8:16] = 32640 % p
    C = np.full((M, N), p - 1, dtype=np.int64)
    cup_lib.cup_set_form("i8limb")
    try:
        dC = dev(C)
        cup_lib.cup_ffgemm(dC, dev(A), dev(B), p, -1)
        assert np.array_equal(host(dC), exact_gemm(C, A, B, p, -1))
    finally:
        cup_lib.cup_set_form("auto")


@pytest.mark.parametrize("form,p,i8", [("i8limb", 65521, False), ("i8", 127, True)])
def test_cup_direct_products_vs_oracle(cup_lib, monkeypatch, form, p, i8):
    """CUP, RREF and inverse with every product below the packed kernel's threshold."""
    _i8_direct_products(monkeypatch)
    cup_lib.cup_set_form(form)
    try:
        for m, n, rank in [(700, 520, None), (600, 600, 350), (1100, 260, None)]:
            A = structured(m, n, p, m + n + 1, rank=rank)
            assert_same_cup(run_cup(cup_lib, A, p, i8=i8), oracle.cup(A, p), f"{form} {m}x{n}")
        if not i8:
            A = structured(500, 420, p, 19, rank=300)
            d = dev(A)
            r, P, Q = cup_lib.cup_rref_inplace(d, p)
            O, rr, rP, rQ = oracle.rref_packed(A, p)
            assert r == rr and np.array_equal(host(d), O)
            B = inputs.uniform((384, 384), p, seed=78)
            X = oracle.inverse(B, p)
            d = dev(B)
            ok, r = cup_lib.cup_inverse_inplace(d, p)
            assert ok and np.array_equal(host(d), X)
    finally:
        cup_lib.cup_set_form("auto")


@pytest.mark.parametrize("form,p,i8", [("i8limb", 65521, False), ("i8", 127, True), ("i8", 127, False),
                                       ("fp64", 65521, False)])
def test_cup_forms_vs_oracle(cup_lib, monkeypatch, form, p, i8):
    """Every form of the product gives the same CUP, bit for bit."""
    _i8_small_products(monkeypatch)
    cup_lib.cup_set_form(form)
    try:
        for m, n, rank in [(700, 520, None), (600, 600, 350), (1100, 260, None)]:
            A = structured(m, n, p, m + n, rank=rank)
            assert_same_cup(run_cup(cup_lib, A, p, i8=i8), oracle.cup(A, p), f"{form} {m}x{n}")
    finally:
        cup_lib.cup_set_form("auto")


def test_rref_inverse_i8limb(cup_lib, monkeypatch):
    _i8_small_products(monkeypatch)
    p = 65521
    cup_lib.cup_set_form("i8limb")
    try:
        A = structured(500, 420, p, 17, rank=300)
        d = dev(A)
        r, P, Q = cup_lib.cup_rref_inplace(d, p)
        O, rr, rP, rQ = oracle.rref_packed(A, p)
        assert r == rr and np.array_equal(host(d), O)
        B = inputs.uniform((384, 384), p, seed=77)
        X = oracle.inverse(B, p)
        d = dev(B)
        ok, r = cup_lib.cup_inverse_inplace(d, p)
        assert ok and np.array_equal(host(d), X)
    finally:
        cup_lib.cup_set_form("auto")


def test_profile_classes(cup_lib, monkeypatch):
    """cup_profile with a class mask times only those classes (here the INT8
    product, whose launches record their own events); other values are refused."""
    _i8_small_products(monkeypatch)
    p = 65521
    A = inputs.uniform((700, 700), p, seed=5)
    cup_lib.cup_set_form("i8limb")
    try:
        cup_lib.cup_profile(8)
        run_cup(cup_lib, A, p)
        st = cup_lib.cup_profile_read()
        cup_lib.cup_profile(False)
        assert st["ffgemm_i8"]["launches"] > 0 and st["ffgemm_i8"]["ms"] > 0
        assert st["window"]["launches"] == 0 and st["pack_i8"]["launches"] == 0
        assert st["ffgemm"]["launches"] == 0
        with pytest.raises(cup_lib.CupError):
            cup_lib.cup_profile(32)
    finally:
        cup_lib.cup_profile(False)
        cup_lib.cup_set_form("auto")


def _row_blocks(blocks, n, p, seed):
    """Rows in blocks of (rows, rank): each block a random product X Y of that
    rank over GF(p) (rank 0: zero rows), so the leaves' ranks are known."""
    rng = np.random.default_rng(seed)
    out = []
    for rows, rank in blocks:
        if rank == 0:
            out.append(np.zeros((rows, n), dtype=np.int64))
            continue
        X = rng.integers(0, p, size=(rows, rank), dtype=np.int64)
        Y = rng.integers(0, p, size=(rank, n), dtype=np.int64)
        out.append(inputs.product_mod(X, Y, p))
    return np.concatenate(out, axis=0)


HELD_BACK_CASES = [
    # a full leaf after a deficient one: the parent's U is not a whole number
    # of 64-blocks (the held-back solve goes out before the general solve)
    ("deficient-then-full", [(64, 50), (64, 64), (128, 128)], 400),
    # a deficient top half: the bottom half's rows move up (row move after a
    # full leaf that held its solve back)
    ("row-move", [(64, 64), (64, 20), (64, 64), (64, 64)], 300),
    # full leaves only, ending the matrix: the last held-back solve goes out
    # when the call returns
    ("full-to-the-end", [(64, 64), (64, 64), (64, 64)], 500),
    # zero rows between full leaves
    ("zero-rows", [(64, 64), (64, 0), (64, 64), (64, 64)], 320),
]


@pytest.mark.parametrize("case", HELD_BACK_CASES, ids=[c[0] for c in HELD_BACK_CASES])
@pytest.mark.parametrize("p", [65521, 257])
def test_cup_held_back_solve_paths(cup_lib, case, p):
    """CUP in the INT8-limb form where full leaves hold their solve back, on
    rank patterns that send it out by each of its paths."""
    name, blocks, n = case
    A = _row_blocks(blocks, n, p, seed=len(name) + p)
    cup_lib.cup_set_form("i8limb")
    try:
        assert_same_cup(run_cup(cup_lib, A, p), oracle.cup(A, p), f"{name} p={p}")
    finally:
        cup_lib.cup_set_form("auto")
