"""GPU parity of the routines built on the CUP decomposition, bit for bit
against the CPU oracle (GF(p) arithmetic: the tolerance is zero):

* PLE (Section 5, Algorithm 10) against ``oracle.ple`` (column by column
  elimination, written independently of the CUP oracle);
* determinant, system solution and nullspace basis (Sections 3.4 and 4.4)
  against ``oracle.det`` (classical elimination), ``oracle.solve``
  (Gauss-Jordan on [A | B]) and ``oracle.nullspace``;
* TRLUM (Algorithm 5) and InPlaceMM (Algorithm 9) against the oracle's
  matrix product.

Sizes span several 64-row leaves and 64-column blocks with ragged tails.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1112_5717_amd import inputs
from test_oracle_pins import structured

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BIG = (8388593, 33554393)  # past the 64-term FP64 bound (2^23.5) for the latter


def dev(a, dtype=torch.int64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    return t.cpu().numpy().astype(np.int64)


def nonsingular(n, p, seed):
    while True:
        A = inputs.uniform((n, n), p, seed=seed)
        if oracle.det(A, p) != 0:
            return A
        seed += 1000


# --------------------------------------------------------------------- PLE

PLE_CASES = [
    (1, 1, 7, None), (5, 9, 2, None), (64, 64, 65521, None), (65, 63, 101, None),
    (130, 200, 3, None), (200, 130, 65521, 70), (300, 300, 65521, 180), (257, 129, 127, None),
    (129, 700, 101, None), (700, 129, 8388593, None), (333, 333, 33554393, None),
    (1100, 900, 65521, None), (900, 1100, 65521, 600), (1024, 1024, 32771, None),
]


@pytest.mark.parametrize("case", PLE_CASES, ids=[f"{c[0]}x{c[1]}p{c[2]}r{c[3]}" for c in PLE_CASES])
def test_ple_vs_oracle(cup_lib, case):
    m, n, p, rank = case
    A = structured(m, n, p, m * 11 + n, rank=rank)
    ref, rr, rP, rQ = oracle.ple(A, p)
    cup_lib.cup_set_form("auto")
    d = dev(A)
    r, P, Q = cup_lib.cup_ple(d, p)
    assert r == rr
    assert np.array_equal(host(P), rP), f"P differs at {np.flatnonzero(host(P) != rP)[:8]}"
    assert np.array_equal(host(Q), rQ), f"Q differs at {np.flatnonzero(host(Q) != rQ)[:8]}"
    got = host(d)
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        raise AssertionError(f"packed [L\\E] differs at {len(bad)} entries, first {bad[:5].tolist()}")


@pytest.mark.parametrize("form", ["fp64", "i8limb"])
def test_ple_forms(cup_lib, form):
    p = 65521
    A = structured(600, 500, p, 3, rank=350)
    ref = oracle.ple(A, p)
    cup_lib.cup_set_form(form)
    try:
        d = dev(A)
        r, P, Q = cup_lib.cup_ple(d, p)
    finally:
        cup_lib.cup_set_form("auto")
    assert r == ref[1] and np.array_equal(host(d), ref[0])
    assert np.array_equal(host(P), ref[2]) and np.array_equal(host(Q), ref[3])


@pytest.mark.parametrize("m,n,p", [(300, 200, 127), (200, 300, 3), (256, 256, 2), (70, 90, 127)])
def test_ple_i8(cup_lib, m, n, p):
    A = structured(m, n, p, m + n, rank=min(m, n) * 2 // 3)
    ref = oracle.ple(A, p)
    d = dev(A, torch.int8)
    r, P, Q = cup_lib.cup_ple_i8(d, p)
    assert r == ref[1] and np.array_equal(host(d), ref[0])
    assert np.array_equal(host(P), ref[2]) and np.array_equal(host(Q), ref[3])


def test_ple_empty_and_strided(cup_lib):
    p = 101
    for shape in [(0, 5), (4, 0)]:
        d = torch.zeros(shape, dtype=torch.int64, device="cuda")
        r, P, Q = cup_lib.cup_ple(d, p)
        assert r == 0
        assert np.array_equal(host(P), np.arange(shape[0])) and np.array_equal(host(Q), np.arange(shape[1]))
    # a strided view of a larger buffer (lda > n), rectangular and square
    X = structured(300, 400, p, 9, rank=150)
    for sub in [(slice(10, 260), slice(50, 330)), (slice(20, 220), slice(100, 300))]:
        d = dev(X)
        view = d[sub]
        r, P, Q = cup_lib.cup_ple(view, p)
        ref = oracle.ple(X[sub], p)
        got = host(d)
        assert r == ref[1] and np.array_equal(got[sub], ref[0])
        outside = np.ones(X.shape, bool)
        outside[sub] = False
        assert np.array_equal(got[outside], X[outside]), "PLE wrote outside its view"


# ------------------------------------------------------------ determinant

@pytest.mark.parametrize("n,p", [(1, 7), (2, 2), (37, 65521), (130, 101), (200, 3), (257, 8388593),
                                 (300, 33554393), (700, 65521), (1100, 127)])
def test_det_vs_oracle(cup_lib, n, p):
    A = inputs.uniform((n, n), p, seed=n + p % 97)
    ref = oracle.det(A, p)
    d, r = cup_lib.cup_det(dev(A), p)
    assert d == ref, (d, ref)
    assert (r == n) == (ref != 0)


def test_det_signs_and_singular(cup_lib):
    p = 65521
    # column exchanges: leading zero columns and a permuted identity
    A = structured(150, 150, p, 4, zero_rows=False, zero_cols=False, dup_rows=False)
    A[:, [0, 5]] = A[:, [5, 0]]
    A[:60, 0] = 0
    B = np.eye(130, dtype=np.int64)[np.random.default_rng(2).permutation(130)]
    S = inputs.low_rank(120, 120, 70, p, seed=3)
    for M in (A, B, S):
        d, r = cup_lib.cup_det(dev(M), p)
        assert d == oracle.det(M, p)
    d, r = cup_lib.cup_det(torch.zeros((0, 0), dtype=torch.int64, device="cuda"), p)
    assert d == 1 and r == 0


# ------------------------------------------------------------------ solve

@pytest.mark.parametrize("n,nrhs,p", [(1, 1, 7), (37, 5, 65521), (130, 1, 101), (200, 130, 2),
                                      (257, 64, 8388593), (300, 7, 33554393), (700, 300, 65521)])
def test_solve_vs_oracle(cup_lib, n, nrhs, p):
    A = nonsingular(n, p, seed=n * 3)
    B = inputs.uniform((n, nrhs), p, seed=n * 3 + 1)
    X = oracle.solve(A, B, p)
    dB = dev(B)
    ok, r = cup_lib.cup_solve(dev(A), dB, p)
    assert ok and r == n
    assert np.array_equal(host(dB), X)


def test_solve_singular(cup_lib):
    p = 65521
    A = inputs.low_rank(100, 100, 60, p, seed=8)
    B = inputs.uniform((100, 3), p, seed=9)
    dB = dev(B)
    ok, r = cup_lib.cup_solve(dev(A), dB, p)
    assert not ok and r == 60
    assert np.array_equal(host(dB), B), "B must be untouched for a singular A"


# -------------------------------------------------------------- nullspace

NULL_CASES = [(5, 9, 7, None), (100, 150, 3, None), (150, 100, 65521, 40), (200, 300, 65521, None),
              (257, 129, 127, 60), (129, 700, 101, None), (300, 300, 33554393, 250), (64, 64, 2, 30),
              (700, 1100, 65521, 500)]


@pytest.mark.parametrize("case", NULL_CASES, ids=[f"{c[0]}x{c[1]}p{c[2]}r{c[3]}" for c in NULL_CASES])
def test_nullspace_vs_oracle(cup_lib, case):
    m, n, p, rank = case
    A = structured(m, n, p, m * 7 + n, rank=rank)
    N_ref, rr, P_ref = oracle.nullspace(A, p)
    N, r, P = cup_lib.cup_nullspace(dev(A), p)
    assert r == rr and np.array_equal(host(P), P_ref)
    assert N.shape == N_ref.shape
    assert np.array_equal(host(N), N_ref)


def test_nullspace_full_and_zero(cup_lib):
    p = 101
    A = nonsingular(90, p, seed=1)
    N, r, P = cup_lib.cup_nullspace(dev(A), p)
    assert r == 90 and N.shape == (90, 0)
    Z = np.zeros((40, 70), np.int64)
    N, r, P = cup_lib.cup_nullspace(dev(Z), p)
    assert r == 0 and np.array_equal(host(N), np.eye(70, dtype=np.int64))


# ------------------------------------------------------- TRLUM / InPlaceMM

def packed_lu(n, p, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, p, size=(n, n), dtype=np.int64)


@pytest.mark.parametrize("n,p", [(1, 7), (40, 65521), (64, 101), (65, 2), (200, 65521), (300, 8388593),
                                 (257, 33554393), (520, 32771)])
def test_trlum_vs_oracle(cup_lib, n, p):
    A = packed_lu(n, p, n + p % 89)
    L = np.tril(A)                      # lower, diagonal stored
    U = np.triu(A, 1) + np.eye(n, dtype=np.int64)  # unit upper
    ref = oracle.mm(np.zeros((n, n), np.int64), L, U, p)
    d = dev(A)
    cup_lib.cup_trlum(d, p)
    assert np.array_equal(host(d), ref)


@pytest.mark.parametrize("m,n,p,rank", [(1, 3, 7, None), (40, 70, 65521, None), (130, 64, 101, None),
                                        (200, 300, 65521, 120), (257, 100, 8388593, None),
                                        (300, 129, 33554393, 200), (600, 500, 65521, None)])
def test_inplace_mm_vs_oracle(cup_lib, m, n, p, rank):
    if rank is None:
        A = inputs.uniform((m, m), p, seed=m)
    else:
        A = structured(m, m, p, m, rank=rank)
    B = inputs.uniform((m, n), p, seed=m + n)
    ref = oracle.mm(np.zeros((m, n), np.int64), A, B, p)
    dA, dB = dev(A), dev(B)
    cup_lib.cup_inplace_mm(dA, dB, p)
    assert np.array_equal(host(dB), ref), "B <- A B"
    assert np.array_equal(host(dA), A), "A must be restored"


# --------------------------------------------------- Strassen-Winograd

WINO_SHAPES = [(300, 300, 300), (257, 390, 520), (640, 384, 1000), (129, 129, 129), (1024, 512, 768)]


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("form,p,dtype", [("fp64", 65521, "int64"), ("fp64", 8388593, "int64"),
                                          ("fp64", 33554393, "int64"), ("fp64", 2, "int64"),
                                          ("i8limb", 65521, "int64"), ("i8", 127, "int8")])
def test_ffgemm_winograd_vs_oracle(cup_lib, monkeypatch, levels, form, p, dtype):
    """Seven-product products (one and two levels, with ragged peels) equal
    the oracle's product bit for bit, in every form; products small enough
    for the packed INT8 kernel are forced onto it too."""
    monkeypatch.setenv("CUP_I8_MIN_WORK", "1e6")
    tdt = torch.int64 if dtype == "int64" else torch.int8
    cup_lib.cup_set_form(form)
    cup_lib.cup_set_winograd(levels, 128)
    try:
        for M, N, K in WINO_SHAPES:
            rng = np.random.default_rng(M + 3 * N + 7 * K + p % 1000)
            A = rng.integers(0, p, size=(M, K), dtype=np.int64)
            B = rng.integers(0, p, size=(K, N), dtype=np.int64)
            C = rng.integers(0, p, size=(M, N), dtype=np.int64)
            for alpha in (-1, 1):
                dC = dev(C, tdt)
                cup_lib.cup_ffgemm(dC, dev(A, tdt), dev(B, tdt), p, alpha)
                ref = oracle.mm(C, A, B, p, alpha)
                assert np.array_equal(host(dC), ref), (M, N, K, alpha)
    finally:
        cup_lib.cup_set_winograd(0, 2048)
        cup_lib.cup_set_form("auto")


def test_ffgemm_winograd_worst_magnitude(cup_lib):
    """Operands at p - 1 and at the centring threshold through two levels."""
    cup_lib.cup_set_form("fp64")
    cup_lib.cup_set_winograd(2, 128)
    try:
        for p in (65521, 33554393):
            h = p // 2
            for va, vb in [(p - 1, p - 1), (h, h + 1)]:
                A = np.full((520, 600), va, dtype=np.int64)
                B = np.full((600, 530), vb, dtype=np.int64)
                C = np.full((520, 530), p - 1, dtype=np.int64)
                dC = dev(C)
                cup_lib.cup_ffgemm(dC, dev(A), dev(B), p, -1)
                assert np.array_equal(host(dC), oracle.mm(C, A, B, p, -1))
    finally:
        cup_lib.cup_set_winograd(0, 2048)
        cup_lib.cup_set_form("auto")


@pytest.mark.parametrize("form", ["fp64", "i8limb"])
def test_cup_rref_inverse_winograd(cup_lib, form):
    """CUP, the reduced echelon form and the inverse with every large enough
    product (Schur updates, triangular solves and products) split."""
    p = 65521
    cup_lib.cup_set_form(form)
    cup_lib.cup_set_winograd(2, 128)
    try:
        A = structured(1100, 1000, p, 21, rank=800)
        d = dev(A)
        r, P, Q = cup_lib.cup_factor(d, p)
        ref = oracle.cup(A, p)
        assert r == ref[1] and np.array_equal(host(d), ref[0])
        assert np.array_equal(host(P), ref[2]) and np.array_equal(host(Q), ref[3])
        d = dev(A)
        cup_lib.cup_rref_inplace(d, p)
        assert np.array_equal(host(d), oracle.rref_packed(A, p)[0])
        B = nonsingular(700, p, seed=5)
        d = dev(B)
        ok, r = cup_lib.cup_inverse_inplace(d, p)
        assert ok and np.array_equal(host(d), oracle.inverse(B, p))
    finally:
        cup_lib.cup_set_winograd(0, 2048)
        cup_lib.cup_set_form("auto")
