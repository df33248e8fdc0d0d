"""Write SHA-256 digests of the CPU oracle's outputs at the full workload sizes.

Calls only ``oracle`` and the seeded input generators; the GPU path never
writes or reads anything here except the digests, which the full-size GPU
parity tests and the benchmark compare against.  Run from the repo root:

    python tests/golden/make_full_size_hashes.py [name ...]

Digest of a CUP (or PLE) result: sha256(packed int64 bytes | P int64 |
Q int64 | rank int64); of an inverse: sha256(inverse int64 bytes); of a batch:
sha256 over the concatenated binary digests of its matrices, in order.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1112_5717_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size_hashes.json")


def cup_digest(packed, r, P, Q) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(packed, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(P, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(Q, dtype=np.int64).tobytes())
    h.update(np.int64(r).tobytes())
    return h.hexdigest()


def mat_digest(X) -> str:
    return hashlib.sha256(np.ascontiguousarray(X, dtype=np.int64).tobytes()).hexdigest()


def first_nonsingular(n, p, seed0):
    seed = seed0
    while True:
        A = inputs.uniform((n, n), p, seed=seed)
        X = oracle.inverse(A, p)
        if X is not None:
            return seed, A, X
        seed += 1


def workloads():
    p16 = 65521
    return {
        "cup_8192_uniform_p65521_seed2": lambda: ("cup", inputs.uniform((8192, 8192), p16, seed=2), p16),
        "cup_8192_rank6000_p65521_seed20": lambda: ("cup", inputs.low_rank(8192, 8192, 6000, p16, seed=20), p16),
        "cup_32768x8192_staircase2048_p65521_seed5": lambda: ("cup", inputs.staircase(32768, 8192, 2048, p16, seed=5)[0], p16),
        "rref_32768x8192_staircase2048_p65521_seed5": lambda: ("rref", inputs.staircase(32768, 8192, 2048, p16, seed=5)[0], p16),
        "cup_16384_rank12000_p127_seed3": lambda: ("cup", inputs.low_rank(16384, 16384, 12000, 127, seed=3), 127),
        "inverse_8192_p127_seed30": lambda: ("inverse", None, 127),
        "batched_4096_m16to512_p2e23_seed4": lambda: ("batched", None, None),
        "cup_512x384_rank300_p65521_seed1": lambda: ("cup", inputs.low_rank(512, 384, 300, p16, seed=1), p16),
        "ple_8192_uniform_p65521_seed2": lambda: ("ple", inputs.uniform((8192, 8192), p16, seed=2), p16),
    }


BATCH = {"count": 4096, "lo": 16, "hi": 512, "seed": 4, "primes_below": 2 ** 23, "nprimes": 32}


def batched_workload():
    """The multi-modular batch: m, n ~ U[16, 512], r ~ U[1, min(m, n)], matrix i
    over the (i mod 32)-th largest prime below 2^23."""
    primes = inputs.largest_primes_below(BATCH["primes_below"], BATCH["nprimes"])
    m, n, r = inputs.batch_specs(BATCH["count"], BATCH["lo"], BATCH["hi"], seed=BATCH["seed"])
    ps = [primes[i % BATCH["nprimes"]] for i in range(BATCH["count"])]
    return m, n, r, ps


def main(names):
    table = json.load(open(OUT)) if os.path.exists(OUT) else {}
    wl = workloads()
    for name in names or list(wl):
        if name in table:
            continue
        kind, A, p = wl[name]()
        t0 = time.time()
        if kind == "cup":
            packed, r, P, Q = oracle.cup(A, p)
            entry = {"digest": cup_digest(packed, r, P, Q), "rank": r}
        elif kind == "ple":
            packed, r, P, Q = oracle.ple(A, p)
            entry = {"digest": cup_digest(packed, r, P, Q), "rank": r}
        elif kind == "rref":
            O, r, P, Q = oracle.rref_packed(A, p)
            entry = {"digest": cup_digest(O, r, P, Q), "rank": r}
        elif kind == "batched":
            m, n, rr, ps = batched_workload()
            h = hashlib.sha256()
            rank_sum, F = 0, 0.0
            for i in range(len(m)):
                B = inputs.batch_matrix(i, m[i], n[i], rr[i], ps[i], seed=BATCH["seed"])
                packed, r, P, Q = oracle.cup(B, ps[i])
                h.update(bytes.fromhex(cup_digest(packed, r, P, Q)))
                rank_sum += int(r)
                F += 2.0 * m[i] * n[i] * r - (m[i] + n[i]) * r * r + 2.0 * r ** 3 / 3.0
            entry = {"digest": h.hexdigest(), "rank_sum": rank_sum, "field_ops": F}
        else:
            seed, A, X = first_nonsingular(8192, p, 30)
            entry = {"digest": mat_digest(X), "seed": seed}
        entry["oracle_seconds"] = round(time.time() - t0, 1)
        table[name] = entry
        json.dump(table, open(OUT, "w"), indent=1, sort_keys=True)
        print(name, entry, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
