"""The allocation-free batched entry point (cup_factor_batched_noalloc),
called through the C-ABI: on two calls in a row, the second with a smaller
batch, its results equal cup_factor_batched's bit for bit (rank, info, the
packed [C\\U] of every matrix, P and Q).  With the library's allocators made
to fail (CUP_FAULT=alloc) it still runs, since it allocates nothing; a batch
beyond its static scratch is refused before any work."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1112_5717_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def make_batch(count, seed, nmax=512):
    rng = np.random.default_rng(seed)
    primes = inputs.largest_primes_below(1 << 23, 32)
    mats, ps = [], []
    for i in range(count):
        m = int(rng.integers(1, nmax + 1))
        n = int(rng.integers(1, nmax + 1))
        r = int(rng.integers(0, min(m, n) + 1))
        p = int(primes[i % 32]) if i % 3 else 65521
        mats.append(inputs.low_rank(m, n, r, p, seed=seed * 1000 + i) if r < min(m, n)
                    else inputs.uniform((m, n), p, seed=seed * 1000 + i))
        ps.append(p)
    return mats, ps


def run(cup, mats, ps, noalloc):
    dev = [torch.from_numpy(A).cuda() for A in mats]
    fn = cup.cup_factor_batched_noalloc if noalloc else cup.cup_factor_batched
    rank, info, Ps, Qs = fn(dev, ps)
    torch.cuda.synchronize()
    return ([d.cpu().numpy() for d in dev], rank.cpu().numpy(), info.cpu().numpy(),
            [x.cpu().numpy() for x in Ps], [x.cpu().numpy() for x in Qs])


def assert_same(a, b):
    mats_a, rank_a, info_a, P_a, Q_a = a
    mats_b, rank_b, info_b, P_b, Q_b = b
    assert np.array_equal(rank_a, rank_b) and np.array_equal(info_a, info_b)
    assert not info_a.any()
    for i in range(len(mats_a)):
        assert np.array_equal(mats_a[i], mats_b[i]), f"matrix {i}"
        assert np.array_equal(P_a[i], P_b[i]) and np.array_equal(Q_a[i], Q_b[i]), f"P/Q {i}"


def test_noalloc_matches_batched_twice(cup_lib, monkeypatch):
    big, ps_big = make_batch(300, seed=41)
    small, ps_small = make_batch(37, seed=42, nmax=200)
    ref_big = run(cup_lib, big, ps_big, noalloc=False)
    ref_small = run(cup_lib, small, ps_small, noalloc=False)
    # every allocation of the library fails from here on: the entry point
    # must not need one
    monkeypatch.setenv("CUP_FAULT", "alloc")
    got_big = run(cup_lib, big, ps_big, noalloc=True)
    got_small = run(cup_lib, small, ps_small, noalloc=True)
    monkeypatch.delenv("CUP_FAULT")
    assert_same(got_big, ref_big)
    assert_same(got_small, ref_small)


def test_noalloc_refuses_oversized_batch(cup_lib):
    import ctypes
    lib = cup_lib.load()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the size check comes first
    rc = lib.cup_factor_batched_noalloc(32769, fake, fake, fake, fake, fake, fake, None, None, fake)
    assert rc == -4000
    assert "scratch" in cup_lib.strerror(rc)
