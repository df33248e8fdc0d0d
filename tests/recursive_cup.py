"""Test-only: the CUP decomposition computed by row recursion, as an
independent check of the iterative oracle.

Written from the description of Section 3.3 (Algorithm 6): factor the top
rows, permute the columns of the bottom rows, solve the unit upper
triangular system for the bottom-left block, update the Schur complement with
one product, factor it, permute the columns of the top-right block and bring
the new U rows up next to the old ones.  The split point is a parameter: the
outputs must not depend on it.  Plain numpy int64, small sizes only.
"""
from __future__ import annotations

import numpy as np


def _swap_cols(B, a, b):
    if a != b:
        B[:, [a, b]] = B[:, [b, a]]


def cup_rec(A: np.ndarray, p: int, split, counter=None):
    """Factor the view A in place into packed [C\\U].

    Returns (rank, profile list, transposition list), local to the view.
    """
    m, n = A.shape
    if n == 0 or m == 0:
        return 0, [], []
    if m == 1:
        nz = np.flatnonzero(A[0])
        if nz.size == 0:
            return 0, [], []
        j = int(nz[0])
        _swap_cols(A, 0, j)
        inv = pow(int(A[0, 0]), p - 2, p)
        A[0, 1:] = (A[0, 1:] * inv) % p
        return 1, [0], [j]
    k = split(m)
    assert 0 < k < m
    top, bot = A[:k], A[k:]
    r1, prof1, P1 = cup_rec(top, p, split, counter)
    for t, j in enumerate(P1):
        _swap_cols(bot, t, j)
    if r1 > 0:
        # G <- A21 U1^{-1}, U1 unit upper (strict upper part of top[:r1, :r1])
        G = bot[:, :r1]
        for c in range(r1):
            if c:
                G[:, c] = (G[:, c] - G[:, :c] @ top[:c, c]) % p
        if counter is not None:
            counter[0] += (m - k) * r1 * (r1 - 1)
        if r1 == n:
            return r1, prof1, P1
        # H <- A22 - G V1
        bot[:, r1:] = (bot[:, r1:] - G @ top[:r1, r1:]) % p
        if counter is not None:
            counter[0] += 2 * (m - k) * r1 * (n - r1)
    H = bot[:, r1:]
    r2, prof2, P2 = cup_rec(H, p, split, counter)
    V1 = top[:r1, r1:]
    for t, j in enumerate(P2):
        _swap_cols(V1, t, j)
    if k > r1:
        for j in range(r1, r1 + r2):
            src = j + k - r1
            A[j, j + 1:] = A[src, j + 1:]
            A[src, j + 1:] = 0
    return (r1 + r2, prof1 + [k + q for q in prof2], P1 + [r1 + q for q in P2])


def cup(A, p: int, split=lambda m: m // 2):
    """Returns (packed, rank, P, Q) in the same layout as the oracle."""
    B = np.array(A, dtype=np.int64, copy=True)
    m, n = B.shape
    r, prof, P = cup_rec(B, p, split)
    Pfull = np.arange(n, dtype=np.int64)
    Pfull[:r] = P
    Qfull = np.arange(m, dtype=np.int64)
    Qfull[:r] = prof
    return B, r, Pfull, Qfull
