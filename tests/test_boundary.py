"""C-ABI boundary checks that need no GPU: the library loads, exports every
symbol the header declares, and rejects invalid arguments before any device
work (LAPACK-style codes of include/cup.h)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cup.h")
LIB = os.path.join(ROOT, "paper_1112_5717_amd", "libcup.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libcup.so not built")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cup_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = ctypes.CDLL(LIB)
    syms = declared_symbols()
    assert "cup_factor" in syms and "cup_factor_batched" in syms and "cup_inverse_inplace" in syms
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in include/cup.h but not exported"


def test_binding_covers_header():
    from paper_1112_5717_amd import cup
    assert set(declared_symbols()) == set(cup.SIGNATURES)
    cup.load()


def test_argument_validation():
    from paper_1112_5717_amd import cup
    lib = cup.load()
    r = ctypes.c_int64(0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.cup_factor(-1, 4, fake, 4, 7, ctypes.byref(r), None, None) == -1
    assert lib.cup_factor(4, -2, fake, 4, 7, ctypes.byref(r), None, None) == -2
    assert lib.cup_factor(4, 4, None, 4, 7, ctypes.byref(r), None, None) == -3
    assert lib.cup_factor(4, 4, fake, 3, 7, ctypes.byref(r), None, None) == -4
    for bad_p in (0, 1, 4, 65535, 2 ** 26 + 15, 2 ** 27 - 39):
        assert lib.cup_factor(4, 4, fake, 4, bad_p, ctypes.byref(r), None, None) == -5
    assert lib.cup_factor(4, 4, fake, 4, 7, None, None, None) == -6
    assert lib.cup_factor_i8(4, 4, fake, 4, 131, ctypes.byref(r), None, None) == -5
    assert lib.cup_inverse_inplace(-1, fake, 4, 7, ctypes.byref(r)) == -1
    assert lib.cup_inverse_inplace(4, None, 4, 7, ctypes.byref(r)) == -2
    assert lib.cup_inverse_inplace(4, fake, 3, 7, ctypes.byref(r)) == -3
    assert lib.cup_inverse_inplace(4, fake, 4, 9, ctypes.byref(r)) == -4
    assert lib.cup_factor_batched(-1, None, None, None, None, None, None, None, None, None) == -1
    assert lib.cup_factor_batched(0, None, None, None, None, None, None, None, None, None) == 0
    assert lib.cup_ffgemm(4, 4, 4, fake, 4, fake, 4, fake, 4, 7, 2) == -11
    assert lib.cup_ffgemm(4, 4, 4, fake, 2, fake, 4, fake, 4, 7, 1) == -5
    assert lib.cup_set_form(9) == -1
    for code in (0, 1, -1, -5, -1001, -2000, -3000):
        assert cup.strerror(code)


def test_argument_validation_derived():
    from paper_1112_5717_amd import cup
    lib = cup.load()
    r = ctypes.c_int64(0)
    d = ctypes.c_int64(0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.cup_ple(-1, 4, fake, 4, 7, ctypes.byref(r), None, None) == -1
    assert lib.cup_ple(4, 4, fake, 3, 7, ctypes.byref(r), None, None) == -4
    assert lib.cup_ple_i8(4, 4, fake, 4, 131, ctypes.byref(r), None, None) == -5
    assert lib.cup_det(-1, fake, 4, 7, ctypes.byref(d), ctypes.byref(r)) == -1
    assert lib.cup_det(4, None, 4, 7, ctypes.byref(d), ctypes.byref(r)) == -2
    assert lib.cup_det(4, fake, 3, 7, ctypes.byref(d), ctypes.byref(r)) == -3
    assert lib.cup_det(4, fake, 4, 8, ctypes.byref(d), ctypes.byref(r)) == -4
    assert lib.cup_det(4, fake, 4, 7, None, ctypes.byref(r)) == -5
    assert lib.cup_det(4, fake, 4, 7, ctypes.byref(d), None) == -6
    assert lib.cup_solve(-1, 1, fake, 4, fake, 1, 7, ctypes.byref(r)) == -1
    assert lib.cup_solve(4, -1, fake, 4, fake, 1, 7, ctypes.byref(r)) == -2
    assert lib.cup_solve(4, 2, fake, 4, None, 2, 7, ctypes.byref(r)) == -5
    assert lib.cup_solve(4, 2, fake, 4, fake, 1, 7, ctypes.byref(r)) == -6
    assert lib.cup_solve(4, 2, fake, 4, fake, 2, 9, ctypes.byref(r)) == -7
    assert lib.cup_solve(4, 2, fake, 4, fake, 2, 7, None) == -8
    assert lib.cup_nullspace(4, 5, fake, 5, 7, ctypes.byref(r), None, None, 5) == -8
    assert lib.cup_nullspace(4, 5, fake, 5, 7, ctypes.byref(r), None, fake, 4) == -9
    assert lib.cup_trlum(-1, fake, 4, 7) == -1
    assert lib.cup_trlum(4, fake, 4, 6) == -4
    assert lib.cup_inplace_mm(4, 3, fake, 3, fake, 3, 7) == -4
    assert lib.cup_inplace_mm(4, 3, fake, 4, fake, 2, 7) == -6
    assert lib.cup_set_winograd(-1, 2048) == -1
    assert lib.cup_set_winograd(9, 2048) == -1
    assert lib.cup_set_winograd(1, 64) == -2
    assert lib.cup_set_winograd(0, 2048) == 0


def test_form_from_environment():
    """CUP_FORM sets the initial form (names or digits); anything else leaves
    the automatic choice.  Host-only: no GPU call is made."""
    import subprocess
    import sys
    code = ("import ctypes, sys; from paper_1112_5717_amd import cup; "
            "lib = ctypes.CDLL(cup.LIB_PATH); print(lib.cup_get_form())")
    for value, want in (("fp64", 1), ("i8", 2), ("i8limb", 3), ("3", 3), ("auto", 0), ("bogus", 0), (None, 0)):
        env = dict(os.environ)
        env.pop("CUP_FORM", None)
        if value is not None:
            env["CUP_FORM"] = value
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                             cwd=ROOT, timeout=120)
        assert out.returncode == 0, out.stderr[-2000:]
        assert int(out.stdout.strip().splitlines()[-1]) == want, (value, out.stdout)
