"""CPU oracle for the CUP decomposition over GF(p) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it.

Thin ctypes wrapper over ``cup_oracle.c`` (plain C, int64 residues, OpenMP
over the rows of each elimination step).  Every function cites the passage of
Jeannerod, Pernet and Storjohann's paper it follows; the readings of ambiguous
passages are documented in ``cup_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cup_oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP) into oracle/_build."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        os.makedirs(_LIB_DIR, exist_ok=True)
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64 = ctypes.c_int64
        p64 = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_cup.argtypes = [i64, i64, i64, p64, p64, p64, p64]
        lib.oracle_cup.restype = ctypes.c_int
        lib.oracle_rcef.argtypes = [i64, i64, i64, p64, p64, p64, p64]
        lib.oracle_rcef.restype = ctypes.c_int
        lib.oracle_inverse.argtypes = [i64, i64, p64, p64]
        lib.oracle_inverse.restype = ctypes.c_int
        lib.oracle_rref_pack.argtypes = [i64, i64, i64, p64, i64, p64, p64, p64]
        lib.oracle_rref_pack.restype = ctypes.c_int
        lib.oracle_inv_mod.argtypes = [i64, i64]
        lib.oracle_inv_mod.restype = i64
        lib.oracle_mm.argtypes = [i64, i64, i64, i64, p64, p64, p64, i64]
        lib.oracle_mm.restype = ctypes.c_int
        lib.oracle_ple.argtypes = [i64, i64, i64, p64, p64, p64, p64]
        lib.oracle_ple.restype = ctypes.c_int
        lib.oracle_det.argtypes = [i64, i64, p64]
        lib.oracle_det.restype = i64
        lib.oracle_solve.argtypes = [i64, i64, i64, p64, p64, p64]
        lib.oracle_solve.restype = ctypes.c_int
        lib.oracle_nullspace.argtypes = [i64, i64, i64, p64, i64, p64, p64]
        lib.oracle_nullspace.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _mat(A) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(A, dtype=np.int64))


def inv_mod(a: int, p: int) -> int:
    return int(_load().oracle_inv_mod(int(a), int(p)))


def cup(A, p: int):
    """CUP decomposition (Algorithm 6, unrolled row by row).

    Returns ``(packed, rank, P, Q)``: packed [C\\U] (Section 3.1 storage),
    the rank, the transposition list P (length n) and Q (length m) whose first
    ``rank`` entries are the row rank profile.
    """
    A = _mat(A).copy()
    m, n = A.shape
    P = np.zeros(max(n, 1), dtype=np.int64)
    Q = np.zeros(max(m, 1), dtype=np.int64)
    r = ctypes.c_int64(0)
    rc = _load().oracle_cup(m, n, int(p), _ptr(A), ctypes.byref(r), _ptr(P), _ptr(Q))
    if rc != 0:
        raise MemoryError("oracle_cup failed")
    return A, int(r.value), P[:n].copy(), Q[:m].copy()


def rcef(A, p: int):
    """Canonical reduced column echelon form, via Gauss-Jordan on A^T.

    Returns ``(R, rank, profile)``; independent of :func:`cup`.
    """
    A = _mat(A)
    m, n = A.shape
    R = np.zeros((m, n), dtype=np.int64)
    prof = np.zeros(max(min(m, n), 1), dtype=np.int64)
    r = ctypes.c_int64(0)
    rc = _load().oracle_rcef(m, n, int(p), _ptr(A), _ptr(R), ctypes.byref(r), _ptr(prof))
    if rc != 0:
        raise MemoryError("oracle_rcef failed")
    return R, int(r.value), prof[: r.value].copy()


def inverse(A, p: int):
    """Inverse by Gauss-Jordan on [A | I]; returns None when A is singular."""
    A = _mat(A)
    n = A.shape[0]
    assert A.shape == (n, n)
    X = np.zeros((n, n), dtype=np.int64)
    rc = _load().oracle_inverse(n, int(p), _ptr(A), _ptr(X))
    if rc < 0:
        raise MemoryError("oracle_inverse failed")
    return None if rc == 1 else X


def rref_packed(A, p: int):
    """Packed transformation to reduced column echelon form.

    Section 3.1 storage [X1 X2; R2 0] with X = U^{-1} diag(L1^{-1}, I)
    (Section 3.5, Proposition 5), P from :func:`cup`, R2 from the independent
    :func:`rcef`.  Returns ``(packed, rank, P, Q)``.
    """
    A = _mat(A)
    m, n = A.shape
    CU, r, P, Q = cup(A, p)
    R, r2, prof = rcef(A, p)
    assert r == r2 and np.array_equal(Q[:r], prof), "oracle rank profiles disagree"
    O = np.zeros((m, n), dtype=np.int64)
    Qc = np.ascontiguousarray(Q if m > 0 else np.zeros(1, dtype=np.int64))
    rc = _load().oracle_rref_pack(m, n, int(p), _ptr(np.ascontiguousarray(CU)), r,
                                  _ptr(Qc), _ptr(np.ascontiguousarray(R)), _ptr(O))
    if rc != 0:
        raise MemoryError("oracle_rref_pack failed")
    return O, r, P, Q


def mm(C, A, B, p: int, alpha: int = 1) -> np.ndarray:
    """C + alpha A B mod p (Algorithm 1, from the definition of the product)."""
    A, B = _mat(A), _mat(B)
    out = _mat(C).copy()
    M, K = A.shape
    K2, N = B.shape
    assert K == K2 and out.shape == (M, N) and alpha in (1, -1)
    if M and N:
        A1 = A if A.size else np.zeros(1, dtype=np.int64)
        B1 = B if B.size else np.zeros(1, dtype=np.int64)
        _load().oracle_mm(M, N, K, int(p), _ptr(A1), _ptr(B1), _ptr(out), int(alpha))
    return out


def ple(A, p: int):
    """PLE decomposition (Section 5, Algorithm 10, unrolled column by column).

    Returns ``(packed, rank, P, Q)``: packed [L\\E], the rank, the row
    transposition list P (length m) and Q (length n) whose first ``rank``
    entries are the column rank profile.
    """
    A = _mat(A).copy()
    m, n = A.shape
    P = np.zeros(max(m, 1), dtype=np.int64)
    Q = np.zeros(max(n, 1), dtype=np.int64)
    r = ctypes.c_int64(0)
    rc = _load().oracle_ple(m, n, int(p), _ptr(A), ctypes.byref(r), _ptr(P), _ptr(Q))
    if rc != 0:
        raise MemoryError("oracle_ple failed")
    return A, int(r.value), P[:m].copy(), Q[:n].copy()


def det(A, p: int) -> int:
    """Determinant by classical Gaussian elimination (Section 4.4)."""
    A = _mat(A)
    n = A.shape[0]
    assert A.shape == (n, n)
    if n == 0:
        return 1 % int(p)
    d = int(_load().oracle_det(n, int(p), _ptr(A)))
    if d < 0:
        raise MemoryError("oracle_det failed")
    return d


def solve(A, B, p: int):
    """X with A X = B for nonsingular A (Gauss-Jordan on [A | B]); None if singular."""
    A, B = _mat(A), _mat(B)
    n = A.shape[0]
    nrhs = B.shape[1]
    assert A.shape == (n, n) and B.shape[0] == n
    X = np.zeros((n, nrhs), dtype=np.int64)
    if n == 0 or nrhs == 0:
        return X
    rc = _load().oracle_solve(n, nrhs, int(p), _ptr(A), _ptr(B), _ptr(X))
    if rc < 0:
        raise MemoryError("oracle_solve failed")
    return None if rc == 1 else X


def nullspace(A, p: int):
    """Right nullspace basis N (n x (n - r)) in the column order of the CUP
    transposition list (Section 3.4); returns ``(N, rank, P)``."""
    A = _mat(A)
    m, n = A.shape
    _, r, P, _ = cup(A, p)
    N = np.zeros((n, n - r), dtype=np.int64)
    if n - r > 0:
        A1 = A if A.size else np.zeros(1, dtype=np.int64)
        Pc = np.ascontiguousarray(P if n > 0 else np.zeros(1, dtype=np.int64))
        rc = _load().oracle_nullspace(m, n, int(p), _ptr(A1), r, _ptr(Pc), _ptr(N))
        if rc != 0:
            raise RuntimeError("oracle_nullspace failed (%d)" % rc)
    return N, r, P


def unpack_ple(packed: np.ndarray, r: int):
    """Split packed [L\\E] into L (m x m unit lower) and E (m x n, zero below row r)."""
    m, n = packed.shape
    L = np.eye(m, dtype=np.int64)
    E = np.zeros((m, n), dtype=np.int64)
    for i in range(min(r, m)):
        E[i, i:] = packed[i, i:]
    for j in range(min(r, n)):
        L[j + 1:, j] = packed[j + 1:, j]
    return L, E


def unpack_cup(packed: np.ndarray, r: int):
    """Split packed [C\\U] into C (m x n, zero beyond column r) and U (n x n unit upper)."""
    m, n = packed.shape
    C = np.zeros((m, n), dtype=np.int64)
    U = np.eye(n, dtype=np.int64)
    for j in range(min(r, n)):
        C[j:, j] = packed[j:, j]
    for i in range(min(r, m)):
        U[i, i + 1:] = packed[i, i + 1:]
    return C, U


def perm_matrix_T(P: np.ndarray, r: int, n: int) -> np.ndarray:
    """The n x n matrix P^T such that A P^T applies T(0,P[0])...T(r-1,P[r-1]) to columns."""
    M = np.eye(n, dtype=np.int64)
    for t in range(r):
        j = int(P[t])
        if j != t:
            M[:, [t, j]] = M[:, [j, t]]
    return M
