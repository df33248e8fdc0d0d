#!/usr/bin/env python3
"""Autotuner of the batched CUP kernels.

Measures every launch configuration of the three width-class kernels
(workgroups per CU for n <= 128, n <= 256 and n <= 512, up to what the
occupancy calculator allows, and sequential or concurrent classes) on the
multi-modular workload (4096 matrices, m, n ~ U[16, 512], r ~ U[1, min(m, n)],
one of the 32 largest primes below 2^23 each, seed 4), through the library's
CUP_BATCHED_TUNE override, and writes the fastest into csrc/batched_tune.h
(rebuild the library afterwards) and the table of measurements to the path
given by --report.  Needs a GPU.

Usage: python -m paper_1112_5717_amd.tune_batched [--reps 5] [--report FILE]
"""
from __future__ import annotations

import argparse
import itertools
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
HEADER = os.path.join(HERE, "csrc", "batched_tune.h")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--report", default=None)
    ap.add_argument("--max-per-cu", type=int, nargs=3, default=[4, 3, 2])
    args = ap.parse_args()

    import numpy as np
    import torch

    from paper_1112_5717_amd import cup, inputs

    cup.load()
    count, seed = 4096, 4
    primes = inputs.largest_primes_below(2 ** 23, 32)
    m, n, r = inputs.batch_specs(count, 16, 512, seed=seed)
    ps = [primes[i % 32] for i in range(count)]
    fb = cup.FlatBatch(m, n, ps)
    src = torch.empty(fb.size, dtype=torch.int64, device="cuda")
    for i in range(count):
        A = inputs.batch_matrix(i, m[i], n[i], r[i], ps[i], seed=seed, device="cuda")
        o = int(fb.offsets[i])
        src[o:o + A.size].copy_(torch.from_numpy(A.reshape(-1)))
    work = src.clone()
    ptrs = fb.pointers(work)
    ref = None
    rows = []
    for w0, w1, w2, conc in itertools.product(range(1, args.max_per_cu[0] + 1),
                                              range(1, args.max_per_cu[1] + 1),
                                              range(1, args.max_per_cu[2] + 1), (0, 1)):
        os.environ["CUP_BATCHED_TUNE"] = f"{w0},{w1},{w2},{conc}"
        times = []
        for k in range(args.reps + 1):
            work.copy_(src)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fb.factor(ptrs, name="cup_factor_batched_noalloc")
            e1.record()
            torch.cuda.synchronize()
            if k:
                times.append(e0.elapsed_time(e1))
        out = (work.clone(), fb.rank.clone())
        if ref is None:
            ref = out
        same = torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]) and not fb.info.any()
        ms = float(np.median(times))
        rows.append((ms, w0, w1, w2, conc, same))
        print(f"[tune] per CU {w0},{w1},{w2} concurrent={conc}: {ms:.3f} ms {'ok' if same else 'MISMATCH'}",
              flush=True)
    del os.environ["CUP_BATCHED_TUNE"]
    good = [x for x in rows if x[5]]
    if len(good) != len(rows):
        sys.exit("a configuration changed the results; nothing written")
    best = min(good)
    with open(HEADER, "w") as f:
        f.write("// Tuning table of the batched kernels, written by tune_batched.py from its\n"
                "// measurements on the multi-modular workload (4096 matrices, m, n ~ U[16, 512]):\n"
                "// workgroups per CU of each width class's persistent kernel (n <= 128,\n"
                "// <= 256, <= 512), and whether the three classes run concurrently.\n"
                f"// Fastest: {best[0]:.3f} ms per batch.\n"
                "#pragma once\n"
                "namespace cup {\n"
                f"constexpr int kTuneWgPerCu[3] = {{{best[1]}, {best[2]}, {best[3]}}};\n"
                f"constexpr int kTuneConcurrent = {best[4]};\n"
                "}  // namespace cup\n")
    if args.report:
        os.makedirs(os.path.dirname(os.path.abspath(args.report)), exist_ok=True)
        with open(args.report, "w") as f:
            f.write("# Batched CUP launch tuning (multi-modular workload, 4096 matrices)\n\n")
            f.write("Command: `python -m paper_1112_5717_amd.tune_batched "
                    f"--reps {args.reps} --report {args.report}`\n\n")
            f.write("| WGs/CU n<=128 | n<=256 | n<=512 | concurrent classes | ms per batch (median) |\n")
            f.write("|---|---|---|---|---|\n")
            for ms, w0, w1, w2, conc, _ in sorted(rows):
                f.write(f"| {w0} | {w1} | {w2} | {conc} | {ms:.3f} |\n")
            f.write(f"\nChosen: {best[1]}, {best[2]}, {best[3]}, concurrent={best[4]}\n")
    print(f"[tune] chosen per CU {best[1]},{best[2]},{best[3]} concurrent={best[4]}: {best[0]:.3f} ms")


if __name__ == "__main__":
    main()
