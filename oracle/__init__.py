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
