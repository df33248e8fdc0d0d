"""Seeded synthetic inputs for the CUP workloads.

This module serves both the GPU path's tests/benchmark and the CPU oracle.  It
holds none of the decomposition's arithmetic: it draws uniform residues from a
seeded numpy PCG64 generator and forms exact integer products X.Y mod p to
build matrices of a prescribed rank or row rank profile.

Exactness of the products: float64 sums of products of residues are exact
while K (p-1)^2 < 2^53 (any summation order); larger cases are split into
K-chunks that satisfy that bound and reduced between chunks.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "is_prime", "largest_primes_below", "uniform", "product_mod", "low_rank",
    "staircase", "batch_specs", "batch_matrix",
]


def is_prime(p: int) -> bool:
    """Deterministic Miller-Rabin (bases valid for all n < 3.3e24)."""
    p = int(p)
    if p < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)
    for q in small:
        if p % q == 0:
            return p == q
    d, s = p - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, p)
        if x in (1, p - 1):
            continue
        for _ in range(s - 1):
            x = x * x % p
            if x == p - 1:
                break
        else:
            return False
    return True


def largest_primes_below(bound: int, count: int) -> list[int]:
    """The ``count`` largest primes below ``bound``, in descending order."""
    out = []
    q = int(bound) - 1
    while len(out) < count and q >= 2:
        if is_prime(q):
            out.append(q)
        q -= 1
    return out


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform(shape, p: int, seed: int) -> np.ndarray:
    """Uniform residues in [0, p) as int64."""
    return _rng(seed).integers(0, int(p), size=shape, dtype=np.int64)


def product_mod(X: np.ndarray, Y: np.ndarray, p: int, device=None) -> np.ndarray:
    """Exact X.Y mod p for residue matrices (int64 result).

    Uses float64 products in K-chunks with chunk*(p-1)^2 < 2^53, on ``device``
    through torch when one is given (float64 matmul is exact in that range),
    else with numpy.
    """
    p = int(p)
    K = X.shape[1]
    chunk = max(1, min(K, (2 ** 53 - 1) // max(1, (p - 1) ** 2)))
    if device is not None:
        import torch
        Xt = torch.from_numpy(np.ascontiguousarray(X)).to(device=device, dtype=torch.float64)
        Yt = torch.from_numpy(np.ascontiguousarray(Y)).to(device=device, dtype=torch.float64)
        acc = torch.zeros((X.shape[0], Y.shape[1]), dtype=torch.float64, device=device)
        for k0 in range(0, K, chunk):
            acc += Xt[:, k0:k0 + chunk] @ Yt[k0:k0 + chunk, :]
            acc = torch.remainder(acc, p)
        out = acc.to(torch.int64).cpu().numpy()
        return np.ascontiguousarray(out)
    acc = np.zeros((X.shape[0], Y.shape[1]), dtype=np.float64)
    Xf = X.astype(np.float64)
    Yf = Y.astype(np.float64)
    for k0 in range(0, K, chunk):
        acc += Xf[:, k0:k0 + chunk] @ Yf[k0:k0 + chunk, :]
        acc = np.remainder(acc, p)
    return np.ascontiguousarray(acc.astype(np.int64))


def low_rank(m: int, n: int, r: int, p: int, seed: int, device=None) -> np.ndarray:
    """A = X (m x r) . Y (r x n) mod p with X, Y uniform; rank r w.h.p."""
    rng = _rng(seed)
    X = rng.integers(0, int(p), size=(m, r), dtype=np.int64)
    Y = rng.integers(0, int(p), size=(r, n), dtype=np.int64)
    return product_mod(X, Y, p, device=device)


def staircase(m: int, n: int, r: int, p: int, seed: int, device=None):
    """Rank-r matrix whose row rank profile is a seeded random staircase.

    ``r`` distinct pivot rows are drawn uniformly; each holds uniform entries.
    Every other row is a uniform random combination of ALL pivot rows above
    it (the zero row when none is above).  Returns ``(A, pivot_rows)``.
    """
    rng = _rng(seed)
    piv = np.sort(rng.choice(m, size=r, replace=False)).astype(np.int64)
    B = rng.integers(0, int(p), size=(r, n), dtype=np.int64)
    coef = rng.integers(0, int(p), size=(m, r), dtype=np.int64)
    # row i combines pivot rows piv[s] < i; pivot rows reproduce themselves
    above = piv[None, :] < np.arange(m, dtype=np.int64)[:, None]
    coef = np.where(above, coef, 0)
    coef[piv, :] = 0
    coef[piv, np.arange(r)] = 1
    return product_mod(coef, B, p, device=device), piv


def batch_specs(count: int, lo: int, hi: int, seed: int):
    """Shapes and ranks of the batched workload: m, n ~ U[lo, hi], r ~ U[1, min(m, n)]."""
    rng = _rng(seed)
    m = rng.integers(lo, hi + 1, size=count, dtype=np.int64)
    n = rng.integers(lo, hi + 1, size=count, dtype=np.int64)
    r = np.array([rng.integers(1, min(a, b) + 1) for a, b in zip(m, n)], dtype=np.int64)
    return m, n, r


def batch_matrix(i: int, m: int, n: int, r: int, p: int, seed: int, device=None) -> np.ndarray:
    """Matrix i of the batched workload: X.Y mod p with its own sub-seed
    (the product on ``device`` when given; the values do not depend on it)."""
    return low_rank(int(m), int(n), int(r), int(p), seed=int(seed) * 1_000_003 + int(i), device=device)
