"""Python binding of libcup (include/cup.h): argument marshalling only.

Every function here has the name of the C entry point it calls, takes torch
tensors that live on the GPU (torch supplies device memory and the current
stream), passes their device pointers through ctypes and raises
:class:`CupError` on a negative status.  All arithmetic happens in the HIP
library; there is no fallback path: if ``libcup.so`` is missing, :func:`load`
raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcup.so")

FORM_AUTO, FORM_FP64, FORM_I8, FORM_I8LIMB = 0, 1, 2, 3
FORMS = {"auto": FORM_AUTO, "fp64": FORM_FP64, "i8": FORM_I8, "i8limb": FORM_I8LIMB}
CUP_OK, CUP_SINGULAR = 0, 1

# (name, restype, argtypes) of every symbol include/cup.h declares
_I64, _PI64, _VP = ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p
SIGNATURES = {
    "cup_set_stream": (ctypes.c_int, [_VP]),
    "cup_set_form": (ctypes.c_int, [ctypes.c_int]),
    "cup_get_form": (ctypes.c_int, []),
    "cup_set_winograd": (ctypes.c_int, [ctypes.c_int, _I64]),
    "cup_factor": (ctypes.c_int, [_I64, _I64, _VP, _I64, _I64, _PI64, _VP, _VP]),
    "cup_factor_i8": (ctypes.c_int, [_I64, _I64, _VP, _I64, _I64, _PI64, _VP, _VP]),
    "cup_rank_profile": (ctypes.c_int, [_I64, _I64, _VP, _I64, _I64, _PI64, _VP]),
    "cup_rref_inplace": (ctypes.c_int, [_I64, _I64, _VP, _I64, _I64, _PI64, _VP, _VP]),
    "cup_rref_inplace_i8": (ctypes.c_int, [_I64, _I64, _VP, _I64, _I64, _PI64, _VP, _VP]),
    "cup_inverse_inplace": (ctypes.c_int, [_I64, _VP, _I64, _I64, _PI64]),
    "cup_inverse_inplace_i8": (ctypes.c_int, [_I64, _VP, _I64, _I64, _PI64]),
    "cup_factor_batched": (ctypes.c_int, [_I64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "cup_factor_batched_noalloc": (ctypes.c_int, [_I64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "cup_ffgemm": (ctypes.c_int, [_I64, _I64, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _I64,
                                  ctypes.c_int]),
    "cup_ffgemm_i8": (ctypes.c_int, [_I64, _I64, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _I64,
                                     ctypes.c_int]),
    "cup_ple": (ctypes.c_int, [_I64, _I64, _VP, _I64, _I64, _PI64, _VP, _VP]),
    "cup_ple_i8": (ctypes.c_int, [_I64, _I64, _VP, _I64, _I64, _PI64, _VP, _VP]),
    "cup_det": (ctypes.c_int, [_I64, _VP, _I64, _I64, _PI64, _PI64]),
    "cup_solve": (ctypes.c_int, [_I64, _I64, _VP, _I64, _VP, _I64, _I64, _PI64]),
    "cup_nullspace": (ctypes.c_int, [_I64, _I64, _VP, _I64, _I64, _PI64, _VP, _VP, _I64]),
    "cup_trlum": (ctypes.c_int, [_I64, _VP, _I64, _I64]),
    "cup_inplace_mm": (ctypes.c_int, [_I64, _I64, _VP, _I64, _VP, _I64, _I64]),
    "cup_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "cup_profile": (ctypes.c_int, [ctypes.c_int]),
    "cup_profile_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double)]),
    "cup_workspace_bytes": (ctypes.c_size_t, []),
    "cup_finalize": (ctypes.c_int, []),
}

_lib = None


class CupError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: status {code} ({strerror(code)})")


def load():
    """Load libcup.so (built by ``paper_1112_5717_amd.build``); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def lib():
    return load()


def strerror(code: int) -> str:
    return load().cup_strerror(int(code)).decode()


def _sync_stream():
    load().cup_set_stream(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _matrix(A: torch.Tensor, dtype):
    if not isinstance(A, torch.Tensor) or A.device.type != "cuda":
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if A.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {A.dtype}")
    if A.dim() != 2 or (A.numel() > 0 and A.stride(1) != 1):
        raise ValueError("expected a row-major 2-D view (unit column stride)")
    m, n = A.shape
    lda = A.stride(0) if m > 1 else max(1, n)
    return int(m), int(n), int(max(lda, n, 1)), ctypes.c_void_p(A.data_ptr() if A.numel() else 0)


def _vec(x: torch.Tensor | None):
    return ctypes.c_void_p(x.data_ptr()) if x is not None and x.numel() else ctypes.c_void_p(0)


def cup_set_form(form) -> None:
    code = FORMS[form] if isinstance(form, str) else int(form)
    rc = load().cup_set_form(code)
    if rc != 0:
        raise CupError(rc, "cup_set_form")


def cup_set_winograd(levels: int, min_dim: int = 2048) -> None:
    """Strassen-Winograd products up to `levels` recursion levels for products
    whose dimensions all reach `min_dim` (0 levels: classical products)."""
    rc = load().cup_set_winograd(int(levels), int(min_dim))
    if rc != 0:
        raise CupError(rc, "cup_set_winograd")


def cup_get_form() -> int:
    return int(load().cup_get_form())


def _factor(name, A, p, dtype, with_p=True, with_q=True):
    m, n, lda, ptr = _matrix(A, dtype)
    P = torch.empty(n, dtype=torch.int64, device=A.device) if with_p else None
    Q = torch.empty(m, dtype=torch.int64, device=A.device) if with_q else None
    r = ctypes.c_int64(0)
    _sync_stream()
    rc = getattr(load(), name)(m, n, ptr, lda, int(p), ctypes.byref(r), _vec(P), _vec(Q))
    if rc < 0:
        raise CupError(rc, name)
    return int(r.value), P, Q


def cup_factor(A: torch.Tensor, p: int):
    """In-place CUP of an int64 device matrix; returns (rank, P, Q) (device int64)."""
    return _factor("cup_factor", A, p, torch.int64)


def cup_factor_i8(A: torch.Tensor, p: int):
    """In-place CUP of an int8 device matrix (p < 128); returns (rank, P, Q)."""
    return _factor("cup_factor_i8", A, p, torch.int8)


def cup_rank_profile(A: torch.Tensor, p: int):
    """Rank and row rank profile (Q[:rank]); A is overwritten with [C\\U]."""
    m, n, lda, ptr = _matrix(A, torch.int64)
    Q = torch.empty(m, dtype=torch.int64, device=A.device)
    r = ctypes.c_int64(0)
    _sync_stream()
    rc = load().cup_rank_profile(m, n, ptr, lda, int(p), ctypes.byref(r), _vec(Q))
    if rc < 0:
        raise CupError(rc, "cup_rank_profile")
    return int(r.value), Q


def cup_rref_inplace(A: torch.Tensor, p: int):
    """A <- [X1 X2; R2 0]; returns (rank, P, Q)."""
    return _factor("cup_rref_inplace", A, p, torch.int64)


def cup_rref_inplace_i8(A: torch.Tensor, p: int):
    return _factor("cup_rref_inplace_i8", A, p, torch.int8)


def _inverse(name, A, p, dtype):
    m, n, lda, ptr = _matrix(A, dtype)
    if m != n:
        raise ValueError("square matrix expected")
    r = ctypes.c_int64(0)
    _sync_stream()
    rc = getattr(load(), name)(n, ptr, lda, int(p), ctypes.byref(r))
    if rc < 0:
        raise CupError(rc, name)
    return rc == CUP_OK, int(r.value)


def cup_inverse_inplace(A: torch.Tensor, p: int):
    """A <- A^{-1}; returns (nonsingular, rank)."""
    return _inverse("cup_inverse_inplace", A, p, torch.int64)


def cup_inverse_inplace_i8(A: torch.Tensor, p: int):
    return _inverse("cup_inverse_inplace_i8", A, p, torch.int8)


def cup_factor_batched(mats: list[torch.Tensor], primes, want_pq: bool = True,
                       name: str = "cup_factor_batched"):
    """Batched CUP of int64 device matrices, one prime each (``name`` selects
    the entry point: cup_factor_batched or cup_factor_batched_noalloc).

    Returns (rank, info, Ps, Qs): rank and info are device tensors.
    """
    dev = mats[0].device if mats else torch.device("cuda")
    B = len(mats)
    dims = [_matrix(A, torch.int64) for A in mats]
    m = torch.tensor([d[0] for d in dims], dtype=torch.int64, device=dev)
    n = torch.tensor([d[1] for d in dims], dtype=torch.int64, device=dev)
    lda = torch.tensor([d[2] for d in dims], dtype=torch.int64, device=dev)
    pp = torch.tensor([int(q) for q in primes], dtype=torch.int64, device=dev)
    ptrs = torch.tensor([d[3].value or 0 for d in dims], dtype=torch.int64, device=dev)
    Ps = [torch.empty(d[1], dtype=torch.int64, device=dev) for d in dims] if want_pq else None
    Qs = [torch.empty(d[0], dtype=torch.int64, device=dev) for d in dims] if want_pq else None
    pP = torch.tensor([x.data_ptr() for x in Ps], dtype=torch.int64, device=dev) if want_pq else None
    pQ = torch.tensor([x.data_ptr() for x in Qs], dtype=torch.int64, device=dev) if want_pq else None
    rank = torch.zeros(B, dtype=torch.int64, device=dev)
    info = torch.zeros(B, dtype=torch.int32, device=dev)
    _sync_stream()
    rc = getattr(load(), name)(B, _vec(m), _vec(n), _vec(ptrs), _vec(lda), _vec(pp), _vec(rank),
                               _vec(pP), _vec(pQ), _vec(info))
    if rc < 0:
        raise CupError(rc, name)
    return rank, info, Ps, Qs


def cup_factor_batched_noalloc(mats: list[torch.Tensor], primes, want_pq: bool = True):
    """cup_factor_batched through the allocation-free entry point."""
    return cup_factor_batched(mats, primes, want_pq, name="cup_factor_batched_noalloc")


class FlatBatch:
    """A batch stored back to back in one int64 device buffer (matrix i is
    m[i] x n[i] with lda = n[i] at element offset ``offsets[i]``), with its
    device descriptors built once, so that a call only passes pointers."""

    def __init__(self, m, n, primes, device="cuda"):
        import numpy as np
        self.m = np.asarray(m, dtype=np.int64)
        self.n = np.asarray(n, dtype=np.int64)
        self.count = len(self.m)
        sizes = self.m * self.n
        self.offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        self.size = int(sizes.sum())
        dev = torch.device(device)
        self.dm = torch.from_numpy(self.m).to(dev)
        self.dn = torch.from_numpy(self.n).to(dev)
        self.dp = torch.tensor([int(q) for q in primes], dtype=torch.int64, device=dev)
        self.dbyte_offs = torch.from_numpy(self.offsets * 8).to(dev)
        self.P = torch.empty(int(self.n.sum()), dtype=torch.int64, device=dev)
        self.Q = torch.empty(int(self.m.sum()), dtype=torch.int64, device=dev)
        self.p_offsets = np.concatenate([[0], np.cumsum(self.n)[:-1]]).astype(np.int64)
        self.q_offsets = np.concatenate([[0], np.cumsum(self.m)[:-1]]).astype(np.int64)
        self.pP = self.P.data_ptr() + torch.from_numpy(self.p_offsets * 8).to(dev)
        self.pQ = self.Q.data_ptr() + torch.from_numpy(self.q_offsets * 8).to(dev)
        self.rank = torch.zeros(self.count, dtype=torch.int64, device=dev)
        self.info = torch.zeros(self.count, dtype=torch.int32, device=dev)

    def pointers(self, flat: torch.Tensor) -> torch.Tensor:
        """Device array of the matrices' addresses inside ``flat``."""
        if flat.dtype != torch.int64 or flat.numel() < self.size or not flat.is_contiguous():
            raise TypeError("flat must be a contiguous int64 device buffer holding the batch")
        return flat.data_ptr() + self.dbyte_offs

    def factor(self, ptrs: torch.Tensor, name: str = "cup_factor_batched") -> None:
        """cup_factor_batched (or ``name``) over the matrices at ``ptrs`` (asynchronous)."""
        _sync_stream()
        rc = getattr(load(), name)(self.count, _vec(self.dm), _vec(self.dn), _vec(ptrs),
                                   _vec(self.dn), _vec(self.dp), _vec(self.rank),
                                   _vec(self.pP), _vec(self.pQ), _vec(self.info))
        if rc < 0:
            raise CupError(rc, name)


def _ple(name, A, p, dtype):
    m, n, lda, ptr = _matrix(A, dtype)
    P = torch.empty(m, dtype=torch.int64, device=A.device)
    Q = torch.empty(n, dtype=torch.int64, device=A.device)
    r = ctypes.c_int64(0)
    _sync_stream()
    rc = getattr(load(), name)(m, n, ptr, lda, int(p), ctypes.byref(r), _vec(P), _vec(Q))
    if rc < 0:
        raise CupError(rc, name)
    return int(r.value), P, Q


def cup_ple(A: torch.Tensor, p: int):
    """In-place PLE of an int64 device matrix (A <- [L\\E]); returns (rank, P, Q)."""
    return _ple("cup_ple", A, p, torch.int64)


def cup_ple_i8(A: torch.Tensor, p: int):
    return _ple("cup_ple_i8", A, p, torch.int8)


def cup_det(A: torch.Tensor, p: int):
    """Determinant of a square int64 device matrix (A <- [C\\U]); returns (det, rank)."""
    m, n, lda, ptr = _matrix(A, torch.int64)
    if m != n:
        raise ValueError("square matrix expected")
    d, r = ctypes.c_int64(0), ctypes.c_int64(0)
    _sync_stream()
    rc = load().cup_det(n, ptr, lda, int(p), ctypes.byref(d), ctypes.byref(r))
    if rc < 0:
        raise CupError(rc, "cup_det")
    return int(d.value), int(r.value)


def cup_solve(A: torch.Tensor, B: torch.Tensor, p: int):
    """B <- A^{-1} B (A <- [C\\U]); returns (nonsingular, rank)."""
    n, n2, lda, pa = _matrix(A, torch.int64)
    nb, nrhs, ldb, pb = _matrix(B, torch.int64)
    if n != n2 or nb != n:
        raise ValueError("A must be n x n and B n x nrhs")
    r = ctypes.c_int64(0)
    _sync_stream()
    rc = load().cup_solve(n, nrhs, pa, lda, pb, max(ldb, 1), int(p), ctypes.byref(r))
    if rc < 0:
        raise CupError(rc, "cup_solve")
    return rc == CUP_OK, int(r.value)


def cup_nullspace(A: torch.Tensor, p: int):
    """Right nullspace basis N (n x (n - rank)) of an int64 device matrix
    (A is overwritten); returns (N, rank, P)."""
    m, n, lda, ptr = _matrix(A, torch.int64)
    N = torch.empty((max(n, 1), max(n, 1)), dtype=torch.int64, device=A.device)
    P = torch.empty(n, dtype=torch.int64, device=A.device)
    r = ctypes.c_int64(0)
    _sync_stream()
    rc = load().cup_nullspace(m, n, ptr, lda, int(p), ctypes.byref(r), _vec(P), _vec(N), max(n, 1))
    if rc < 0:
        raise CupError(rc, "cup_nullspace")
    rank = int(r.value)
    return N[:n, : n - rank], rank, P


def cup_trlum(A: torch.Tensor, p: int) -> None:
    """A = [L\\U] <- L U in place (L lower with diagonal, U unit upper)."""
    m, n, lda, ptr = _matrix(A, torch.int64)
    if m != n:
        raise ValueError("square matrix expected")
    _sync_stream()
    rc = load().cup_trlum(n, ptr, lda, int(p))
    if rc < 0:
        raise CupError(rc, "cup_trlum")


def cup_inplace_mm(A: torch.Tensor, B: torch.Tensor, p: int) -> None:
    """B <- A B in place (A m x m is restored on return)."""
    m, m2, lda, pa = _matrix(A, torch.int64)
    mb, n, ldb, pb = _matrix(B, torch.int64)
    if m != m2 or mb != m:
        raise ValueError("A must be m x m and B m x n")
    _sync_stream()
    rc = load().cup_inplace_mm(m, n, pa, lda, pb, max(ldb, 1), int(p))
    if rc < 0:
        raise CupError(rc, "cup_inplace_mm")


def cup_ffgemm(C: torch.Tensor, A: torch.Tensor, B: torch.Tensor, p: int, alpha: int = -1):
    """C <- C + alpha A B mod p in place (int64 or int8 device matrices)."""
    dtype = C.dtype
    M, N, ldc, pc = _matrix(C, dtype)
    Ma, K, lda, pa = _matrix(A, dtype)
    Kb, Nb, ldb, pb = _matrix(B, dtype)
    if Ma != M or Kb != K or Nb != N:
        raise ValueError("shape mismatch")
    name = "cup_ffgemm" if dtype == torch.int64 else "cup_ffgemm_i8"
    _sync_stream()
    rc = getattr(load(), name)(M, N, K, pa, lda, pb, ldb, pc, ldc, int(p), int(alpha))
    if rc < 0:
        raise CupError(rc, name)


def cup_profile(enable) -> None:
    """True/False: time every kernel class or stop; an int above 1 selects
    classes by bit (k + 1 for class k, as in include/cup.h)."""
    mode = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
    rc = load().cup_profile(mode)
    if rc < 0:
        raise CupError(rc, "cup_profile")


def cup_profile_read() -> dict:
    """Kernel timing collected since cup_profile(True)."""
    buf = (ctypes.c_double * 16)()
    load().cup_profile_read(buf)
    v = list(buf)
    keys = ("launches", "ms", "flops", "bytes")
    return {"ffgemm": dict(zip(keys, v[0:4])), "window": dict(zip(keys, v[4:8])),
            "ffgemm_i8": dict(zip(keys, v[8:12])), "pack_i8": dict(zip(keys, v[12:16]))}


def cup_workspace_bytes() -> int:
    return int(load().cup_workspace_bytes())


def cup_finalize() -> None:
    load().cup_finalize()
