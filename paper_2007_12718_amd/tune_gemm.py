#!/usr/bin/env python3
"""Autotuner of the batched complex GEMM variants (the level merges of
Algorithm 1 are batched products of many uneven shapes).

Runs one build + solve of each workload family on the GPU with shape
recording on, groups the recorded products by their tuning bucket
(precision and the half-octaves of M, N, K and the batch), times every GEMM
variant (tile shape, LDS depth) on the largest shape of each bucket through
lsh_gemm_tune, and writes the fastest per bucket to tune/gemm_table.txt
(loaded by the binding at start-up) with a readable summary beside it.

    python paper_2007_12718_amd/tune_gemm.py [--quick] [--out DIR]
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def half_octave(x):
    return 0 if x <= 1 else int(round(2 * math.log2(x)))


def record_shapes(lsh, quick):
    import numpy as np
    import torch
    import synth
    # (workload, precision, full_levels): the bench's headline keeps level 1 whole
    runs = [(synth.largest(), "fp32", 1), (synth.largest(), "fp64", 1), (synth.largest(), "fp32", 0),
            (synth.largest(), "fp64", 0), (synth.differentiation(), "fp32", 0), (synth.bumps20(), "fp32", 1),
            (synth.bumps20(), "fp64", 1)]
    if quick:
        runs = [(synth.largest(n=256, kappa=50 * np.pi), "fp32", 1), (synth.bumps20(), "fp64", 0)]
    runs += [(w, "fp32", 0) for w in synth.batched(12)]
    shapes = set()
    for w, prec, fl in runs:
        lsh.gemm_record(True)
        b = torch.from_numpy(w.b).cuda()
        P, F = lsh.build(w.n, w.kappa, b, op_order=w.op_order, leaf=w.leaf, tol=w.tol, proxy_width=w.proxy_width,
                         prec=prec, full_levels=fl)
        F.solve(torch.from_numpy(w.u_inc[:1]).cuda(), tol=w.gmres_tol, maxit=100, want_u=False)
        torch.cuda.synchronize()
        got = lsh.gemm_recorded()
        lsh.gemm_record(False)
        F.close()
        P.close()
        shapes.update(got)
        print(f"# {w.name} {prec} full_levels={fl}: {len(got)} product shapes", flush=True)
    return shapes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="smaller workloads (a check of the tuner itself)")
    ap.add_argument("--out", default=os.path.join(HERE, "tune"))
    ap.add_argument("--reps", type=int, default=4)
    a = ap.parse_args()
    import torch
    from paper_2007_12718_amd import lsh
    torch.cuda.set_device(0)
    lsh.gemm_table_clear()  # choose by the model while recording
    shapes = record_shapes(lsh, a.quick)
    buckets = {}
    for (p, M, N, K, batch) in shapes:
        key = (p, half_octave(M), half_octave(N), half_octave(K), half_octave(batch))
        if key not in buckets or M * N * K * batch > math.prod(buckets[key][1:]):
            buckets[key] = (p, M, N, K, batch)
    names = {1: lsh.gemm_variants("fp32"), 0: lsh.gemm_variants("fp64")}
    lsh.gemm_table_clear()
    rows = []
    t0 = time.time()
    for key in sorted(buckets):
        p, M, N, K, batch = buckets[key]
        best, ms = lsh.gemm_tune("fp32" if p == 1 else "fp64", M, N, K, batch, reps=a.reps)
        rows.append((p, M, N, K, batch, best, ms))
        print(f"# tune {'FP32' if p == 1 else 'FP64'} M={M} N={N} K={K} batch={batch}: {names[p][best]}; ms "
              + " ".join(f"{t:.3f}" for t in ms), flush=True)
    os.makedirs(a.out, exist_ok=True)
    lsh.gemm_table_save(os.path.join(a.out, "gemm_table.txt"))
    with open(os.path.join(a.out, "gemm_tuning.md"), "w") as f:
        f.write("# GEMM variant timings (lsh_gemm_tune, one MI355X)\n\n")
        f.write(f"Written by `python paper_2007_12718_amd/tune_gemm.py{' --quick' if a.quick else ''}` "
                f"({len(rows)} buckets, {time.time() - t0:.0f} s of timing).  ms per launch; the fastest is starred; "
                "algorithmic TF/s = 8 M N K batch / time.\n\n")
        for p in (1, 0):
            sel = [r for r in rows if r[0] == p]
            if not sel:
                continue
            f.write(f"## {'FP32' if p == 1 else 'FP64'}\n\n| M | N | K | batch | " + " | ".join(names[p]) +
                    " | best TF/s |\n|" + "---|" * (5 + len(names[p])) + "\n")
            for (_, M, N, K, batch, best, ms) in sel:
                cells = [f"{'*' if v == best else ''}{t:.3f}" for v, t in enumerate(ms)]
                tf = 8.0 * M * N * K * batch / (ms[best] * 1e-3) / 1e12
                f.write(f"| {M} | {N} | {K} | {batch} | " + " | ".join(cells) + f" | {tf:.1f} |\n")
            f.write("\n")
    print(f"wrote {len(rows)} entries to {a.out}", flush=True)


if __name__ == "__main__":
    main()
