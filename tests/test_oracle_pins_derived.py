"""Pins of the oracle's matrix product, PLE decomposition, determinant,
system solution and nullspace basis against facts the paper and the
mathematics fix (no GPU).

Each pin would catch a plausible slip: a transposed operand or a dropped
sign in the product; the wrong pivot rule, a missing row exchange of L or
a mis-ordered permutation in the PLE; a lost sign in the determinant; a
wrong free-column order in the nullspace.
"""
from __future__ import annotations

import itertools
import os

import numpy as np
import pytest

import oracle
from test_oracle_pins import brute_profile, brute_rank, leibniz_det, mat_mod, structured

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_blocks(path):
    blocks, cur, p = {}, None, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        if parts[0] == "p":
            p = int(parts[1])
        elif not parts[0].lstrip("-").isdigit():
            cur = parts[0]
            blocks[cur] = []
        else:
            blocks[cur].append([int(x) for x in parts])
    return p, {k: np.array(v, dtype=np.int64) for k, v in blocks.items()}


# ------------------------------------------------------------------ product

def test_mm_worked_example():
    """Algorithm 1 on a product worked by hand (tests/golden/mm_gf7_by_hand.txt)."""
    p, b = _read_blocks(os.path.join(GOLDEN, "mm_gf7_by_hand.txt"))
    Z = np.zeros_like(b["C"])
    assert np.array_equal(oracle.mm(Z, b["A"], b["B"], p, 1), b["AB"])
    assert np.array_equal(oracle.mm(b["C"], b["A"], b["B"], p, -1), b["C-AB"])


@pytest.mark.parametrize("p", [2, 127, 65521, 33554393])
def test_mm_properties(p):
    """(AB)^T = B^T A^T on non-square shapes, identity, and the alpha sign:
    C - AB + AB = C."""
    rng = np.random.default_rng(p)
    for M, N, K in [(3, 5, 7), (8, 2, 1), (1, 9, 4), (6, 6, 6)]:
        A = rng.integers(0, p, size=(M, K), dtype=np.int64)
        B = rng.integers(0, p, size=(K, N), dtype=np.int64)
        C = rng.integers(0, p, size=(M, N), dtype=np.int64)
        AB = oracle.mm(np.zeros((M, N), np.int64), A, B, p)
        BtAt = oracle.mm(np.zeros((N, M), np.int64), B.T, A.T, p)
        assert np.array_equal(AB.T, BtAt)
        assert np.array_equal(oracle.mm(np.zeros((K, N), np.int64), np.eye(K, dtype=np.int64), B, p), B)
        back = oracle.mm(oracle.mm(C, A, B, p, -1), A, B, p, 1)
        assert np.array_equal(back, C)
        # an entry checked against its own sum of products with exact integers
        i, j = M - 1, N - 1
        assert AB[i, j] == sum(int(A[i, k]) * int(B[k, j]) for k in range(K)) % p


# ------------------------------------------------------------------ PLE

def check_ple_definition(A, p, packed, r, P, Q):
    """P^T A = L E with L unit lower, E row echelon revealing the column rank
    profile Q[:r] (Section 5, Algorithm 10 Ensures)."""
    m, n = A.shape
    L, E = oracle.unpack_ple(packed, r)
    PA = A.copy()
    for t in range(r):
        PA[[t, int(P[t])]] = PA[[int(P[t]), t]]
    assert np.array_equal(PA, mat_mod(L, E, p))
    prof = [int(q) for q in Q[:r]]
    assert prof == sorted(prof) and len(set(prof)) == r
    for t in range(r):
        assert P[t] >= t
        assert np.all(E[t, : prof[t]] == 0), "E is not row echelon"
        assert E[t, prof[t]] != 0, "missing pivot"
    assert np.all(E[r:] == 0)
    assert np.all(np.tril(L, -1)[:, r:] == 0) and np.all(np.diag(L) == 1)
    for t in range(r, m):
        assert P[t] == t
    for t in range(r, n):
        assert Q[t] == t
    for i in range(m):
        for j in range(n):
            if not ((i < r and j >= i) or (j < r and j < i)):
                assert packed[i, j] == 0


@pytest.mark.parametrize("p", [2, 3, 7, 101, 65521, 33554393])
def test_ple_definition_random(p):
    for seed, (m, n) in enumerate([(1, 1), (1, 7), (7, 1), (5, 5), (9, 6), (6, 11), (12, 12), (13, 8)]):
        for rank in (None, 2):
            A = structured(m, n, p, seed * 37 + p % 89, rank=rank)
            packed, r, P, Q = oracle.ple(A, p)
            check_ple_definition(A, p, packed, r, P, Q)


@pytest.mark.parametrize("p", [2, 3])
def test_ple_column_profile_brute_force(p):
    """Rank and column rank profile by enumeration of the column space."""
    rng = np.random.default_rng(p + 40)
    for _ in range(60):
        m, n = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        A = rng.integers(0, p, size=(m, n), dtype=np.int64)
        if rng.random() < 0.3:
            A[:, int(rng.integers(0, n))] = 0
        _, r, _, Q = oracle.ple(A, p)
        prof = brute_profile(A.T.copy(), p)
        assert r == len(prof) == brute_rank(A.T.copy(), p)
        assert [int(q) for q in Q[:r]] == prof


@pytest.mark.parametrize("p", [2, 5, 101, 65521])
def test_ple_is_transposed_cup(p):
    """Section 5: (E^T, L^T, P^T) is the CUP decomposition of A^T, so the
    packed [L\\E] is the transpose of the packed [C\\U] of A^T, with the same
    transpositions and profile (two independently written eliminations)."""
    rng = np.random.default_rng(p + 3)
    for trial in range(30):
        m, n = int(rng.integers(1, 16)), int(rng.integers(1, 16))
        rank = None if trial % 3 else int(rng.integers(0, min(m, n) + 1))
        A = structured(m, n, p, 700 + trial, rank=rank) if rank != 0 else np.zeros((m, n), np.int64)
        packed, r, P, Q = oracle.ple(A, p)
        cpacked, cr, cP, cQ = oracle.cup(A.T.copy(), p)
        assert r == cr
        assert np.array_equal(P, cP) and np.array_equal(Q, cQ)
        assert np.array_equal(packed, cpacked.T)


def test_ple_paper_example_pattern():
    """The row echelon pattern printed in Section 5 (column rank profile [0, 3, 4])."""
    rows, prof = [], None
    for line in open(os.path.join(GOLDEN, "example_ple_E_5x7.txt")):
        line = line.strip()
        if line.startswith("# profile:"):
            prof = [int(x) for x in line.split(":")[1].split()]
        elif line and not line.startswith("#"):
            rows.append(line)
    p = 65521
    rng = np.random.default_rng(9)
    for _ in range(10):
        A = np.zeros((5, 7), dtype=np.int64)
        basis = rng.integers(1, p, size=(5, 3), dtype=np.int64)
        A[:, 0], A[:, 3], A[:, 4] = basis.T
        for j in (1, 2):
            A[:, j] = (A[:, 0] * int(rng.integers(1, p))) % p
        for j in (5, 6):
            A[:, j] = (basis @ rng.integers(1, p, size=3)) % p
        packed, r, P, Q = oracle.ple(A, p)
        assert r == 3 and [int(q) for q in Q[:3]] == prof
        _, E = oracle.unpack_ple(packed, r)
        for i, line in enumerate(rows):
            for j, ch in enumerate(line):
                if ch == ".":
                    assert E[i, j] == 0, (i, j)
                elif ch == "N":
                    assert E[i, j] != 0, (i, j)


def test_ple_edge_cases():
    for m, n in [(0, 0), (0, 5), (5, 0)]:
        packed, r, P, Q = oracle.ple(np.zeros((m, n), np.int64), 7)
        assert r == 0 and np.array_equal(P, np.arange(m)) and np.array_equal(Q, np.arange(n))
    A = np.array([[0], [0], [3], [4]], dtype=np.int64)
    packed, r, P, Q = oracle.ple(A, 7)
    assert r == 1 and P[0] == 2 and Q[0] == 0
    assert list(packed[:, 0]) == [3, 0, 0, 4 * pow(3, 5, 7) % 7]


# ------------------------------------------------------------------ det / solve

@pytest.mark.parametrize("p", [2, 3, 101, 65521])
def test_det_leibniz_and_multiplicative(p):
    rng = np.random.default_rng(p + 17)
    for _ in range(40):
        n = int(rng.integers(1, 7))
        A = rng.integers(0, p, size=(n, n), dtype=np.int64)
        if rng.random() < 0.25 and n > 1:
            A[int(rng.integers(0, n))] = 0
        assert oracle.det(A, p) == leibniz_det(A, p)
    for _ in range(10):
        n = int(rng.integers(1, 30))
        A = rng.integers(0, p, size=(n, n), dtype=np.int64)
        B = rng.integers(0, p, size=(n, n), dtype=np.int64)
        assert oracle.det(mat_mod(A, B, p), p) == oracle.det(A, p) * oracle.det(B, p) % p
        T = np.triu(A)
        assert oracle.det(T, p) == int(np.prod([int(x) for x in np.diag(T)], dtype=object) % p)


@pytest.mark.parametrize("p", [2, 101, 65521, 33554393])
def test_solve_pins(p):
    """A X = B, and the solution of a nonsingular system is unique: it is
    A^{-1} B, with the inverse pinned separately (adjugate over determinant)."""
    rng = np.random.default_rng(p + 23)
    for _ in range(12):
        n, k = int(rng.integers(1, 25)), int(rng.integers(1, 6))
        A = rng.integers(0, p, size=(n, n), dtype=np.int64)
        B = rng.integers(0, p, size=(n, k), dtype=np.int64)
        X = oracle.solve(A, B, p)
        if oracle.det(A, p) == 0:
            assert X is None
            continue
        assert np.array_equal(mat_mod(A, X, p), B)
        assert np.array_equal(X, mat_mod(oracle.inverse(A, p), B, p))
    S = np.zeros((4, 4), np.int64)
    S[0, 0] = 1
    assert oracle.solve(S, np.ones((4, 1), np.int64), p) is None


# ------------------------------------------------------------------ nullspace

def _order(P, r, n):
    order = list(range(n))
    for t in range(r):
        j = int(P[t])
        order[t], order[j] = order[j], order[t]
    return order


@pytest.mark.parametrize("p", [2, 3, 101, 65521])
def test_nullspace_pins(p):
    """A N = 0, N has n - r columns, and the free rows (the last n - r
    positions of the CUP column order) of N form the identity, so the
    columns are independent and, with dim ker A = n - r, span it."""
    rng = np.random.default_rng(p + 29)
    for trial in range(30):
        m, n = int(rng.integers(1, 14)), int(rng.integers(1, 14))
        rank = None if trial % 2 else int(rng.integers(0, min(m, n) + 1))
        A = structured(m, n, p, 900 + trial, rank=rank) if rank != 0 else np.zeros((m, n), np.int64)
        N, r, P = oracle.nullspace(A, p)
        assert N.shape == (n, n - r)
        assert np.all(mat_mod(A, N, p) == 0)
        order = _order(P, r, n)
        free = [order[c] for c in range(r, n)]
        assert np.array_equal(N[free, :], np.eye(n - r, dtype=np.int64))


@pytest.mark.parametrize("p", [2, 3])
def test_nullspace_brute_force(p):
    """On tiny inputs: the kernel enumerated vector by vector has p^(n-r)
    elements, and the span of N is exactly that set."""
    rng = np.random.default_rng(p + 31)
    for _ in range(40):
        m, n = int(rng.integers(1, 4)), int(rng.integers(1, 5))
        A = rng.integers(0, p, size=(m, n), dtype=np.int64)
        N, r, _ = oracle.nullspace(A, p)
        kernel = {x for x in itertools.product(range(p), repeat=n)
                  if not np.any((A @ np.array(x, dtype=np.int64)) % p)}
        assert len(kernel) == p ** (n - r)
        span = {tuple(int(v) for v in (N @ np.array(c, dtype=np.int64)) % p)
                for c in itertools.product(range(p), repeat=n - r)}
        assert span == kernel
