#!/usr/bin/env python3
"""Time-to-1e-10 residual (HBS build + GMRES) on one MI355X.

One step = the whole hot path on one input: lsh_plan_create (tree, weights,
kernel table, per-level proxy row IDs, FFT spectrum) + lsh_factor_create
(Algorithm 1) + lsh_solve (flexible GMRES on the 10th-order FFT operator,
right-preconditioned by Algorithm 2) to a relative residual < 1e-10.  Inputs
(b, u_inc) are resident in HBM before the timed region starts.

Default workload: n = 1024 (N = 1,048,576), kappa = 200 pi (100 wavelengths,
~10 points per wavelength), b a seeded random Fourier field (|k| <= 20 cycles
per unit) scaled to [-1, 0.9], plane wave exp(i kappa x1), HBS at tol 1e-4
with 4th-order corrections (leaf 8x8, proxy width 2), GMRES operator with
10th-order corrections.  The headline value is the FP32-HBS form; the FP64-HBS
form is timed beside it.

Prints one JSON line (rank 0).  --gpus N > 1 is refused: this build runs on
one GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# lsh_build keeps four streams of its own busy beside the caller's; with
# fewer hardware queues per process than streams, two of them share a queue
# and run one after the other (set before the HIP runtime starts)
os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")

PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-HBS comparison form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the bumps-256 and batched-64 records that follow the headline")
    ap.add_argument("--cpu-n", type=int, default=0,
                    help="grid side of the oracle's timed run (default: the workload's own n)")
    ap.add_argument("--no-profile", action="store_true", help="no per-kernel hipEvent records")
    ap.add_argument("--separate", action="store_true",
                    help="lsh_plan_create + lsh_factor_create instead of the pipelined lsh_build")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 256 MiB device copy first (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--batched", type=int, default=0,
                    help="instead of the headline run: time the factor of this many uneven instances "
                         "(sides 64..256, 5-20 wavelengths), batched (lsh_batch_factor) against one by one")
    ap.add_argument("--merge", default="auto", choices=["auto", "schur", "lowrank"],
                    help="form of the merge inverses (lsh_desc.merge)")
    ap.add_argument("--full-levels", type=int, default=1,
                    help="levels 1..N keep all their candidates (lsh_desc.full_levels; 0 = every level compressed, "
                         "the paper's form, timed beside the headline as full_levels0)")
    ap.add_argument("--direct", type=int, default=0,
                    help="instead of the headline run: direct-solver mode on this grid side (the largest "
                         "workload family at the same kappa h): 10th-order HBS, FP64, applied once")
    ap.add_argument("--direct-tol", type=float, default=1e-6,
                    help="compression tolerance of the direct-solver mode (below 1e-7 the row IDs use the "
                         "one-workgroup CPQR, which is slow at large ranks)")
    ap.add_argument("--plan-cache", action="store_true",
                    help="instead of the headline run: the same step for a new b each time with the row IDs "
                         "taken from the plan cache (filled by the warmup), as in an inverse problem")
    ap.add_argument("--multi-rhs", type=int, default=0,
                    help="instead of the headline run: time the FP64 FGMRES solve of this many plane waves "
                         "(512 x 512 grid, kappa = 80 pi) in lockstep (one lsh_solve call) against one call "
                         "per right-hand side, with one FP32 HBS factor")
    return ap.parse_args()


def workload(n):
    import numpy as np
    import synth
    return synth.largest(n=n, kappa=200 * np.pi * n / 1024)


_WS = {}


def workspaces(lsh, w, prec, merge, full_levels=0):
    """The device workspaces of one form (plan, factor, solve), allocated once
    and reused by every step: the library itself allocates nothing."""
    key = (w.n, prec, merge, full_levels)
    if key not in _WS:
        pw, fw = lsh.build_workspaces(w.n, w.kappa, op_order=w.op_order, leaf=w.leaf, tol=w.tol,
                                      proxy_width=w.proxy_width, prec=prec, merge=merge, full_levels=full_levels)
        _WS[key] = {"plan": pw, "factor": fw, "solve": None}
    return _WS[key]


def run_step(lsh, w, b_d, u_d, prec, torch, separate=False, merge="auto", full_levels=0):
    ws = workspaces(lsh, w, prec, merge, full_levels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if separate:  # lsh_plan_create then lsh_factor_create
        P = lsh.Plan(w.n, w.kappa, op_order=w.op_order, leaf=w.leaf, tol=w.tol, proxy_width=w.proxy_width,
                     prec=prec, merge=merge, ws=ws["plan"], full_levels=full_levels)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        F = lsh.Factor(P, b_d, ws=ws["factor"])
    else:  # lsh_build: the same plan and factor, pipelined by level
        P, F = lsh.build(w.n, w.kappa, b_d, op_order=w.op_order, leaf=w.leaf, tol=w.tol,
                         proxy_width=w.proxy_width, prec=prec, merge=merge, workspaces=(ws["plan"], ws["factor"]),
                         full_levels=full_levels)
        t1 = None
    if ws["solve"] is None:  # (first, untimed warmup step)
        ws["solve"] = lsh.workspace(F.solve_workspace_bytes(1, 100))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sig, _, info, rc = F.solve(u_d, tol=w.gmres_tol, maxit=100, want_u=False, ws=ws["solve"])
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    out = {"build_s": t2 - t0, "plan_s": (t1 - t0) if t1 else None, "factor_s": (t2 - t1) if t1 else None,
           "solve_s": t3 - t2, "total_s": t3 - t0,
           "solve_ms_precond": info.ms_precond, "solve_ms_operator": info.ms_operator,
           "solve_ms_ortho": info.ms_ortho,
           "iterations": info.iterations, "true_residual": info.true_residual, "rc": rc,
           "ranks": P.ranks()[1], "lowrank_ranks": P.lowrank_ranks()}
    F.close()
    P.close()
    del sig
    return out


def apply_bytes(n, leaf, ranks, lowrank, esize):
    """Algorithmic bytes of one preconditioner apply (Algorithm 2, one right
    hand side): each stored matrix of the factor read as often as the passes
    use it -- the leaf inverses X_tau in the leaf up and down steps, the merge
    factors of level l >= 1 in the up and the down pass (the root's once), the
    children's scattering matrices in the down pass, and the shared per-level
    matrices (U_l, the sibling block G_ab, the low-rank factors) once per
    launch that reads them.  Vectors (O(N) complex) are left out: they are a
    few percent of the total at these sizes."""
    L = len(ranks) - 1
    nleaf, mL = 2 ** L, leaf * leaf
    tot = 2.0 * nleaf * mL * mL + 2.0 * mL * ranks[L]
    for l in range(L):
        nb, c, r, k = 2 ** l, ranks[l + 1], lowrank[l], ranks[l]
        uses = 1 if l == 0 else 2
        if r > 0:  # [S_a L; S_b R] (2 nb blocks c x r), W' (nb of 2r x 2r), the shared [L; R] and its transpose
            tot += uses * (2.0 * nb * c * r + 4.0 * nb * r * r + 2.0 * c * r)
        else:      # P_a, P_b, C^{-1}
            tot += uses * 3.0 * nb * c * c
        tot += 2.0 * c * c                 # G_ab and its transpose
        if l >= 1:
            tot += 2.0 * nb * c * c        # S of the two children of every box (down pass)
            tot += 2 * 2.0 * c * k         # U_l (up and down pass)
    return esize * tot


def roofline(lsh):
    """Dominant instrumented kernel over the timed region, against its peak."""
    best = None
    for name in lsh.lsh_profile_names():
        if name.startswith("op_"):  # composite operations are not single kernels
            continue
        n, ms, work = lsh.lsh_profile_query(name)
        if n and (best is None or ms > best[2]):
            best = (name, n, ms, work)
    if best is None:
        return None
    name, n, ms, work = best
    if name.startswith("cgemm"):
        peak = PEAK_FP32_TFLOPS if "_f32" in name else PEAK_FP64_TFLOPS
        achieved = work / (ms * 1e-3) / 1e12
        return {"kernel": name, "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None, "launches": n, "ms_total": ms,
                "work_per_launch": work / n,
                "algorithmic_bytes_per_launch": lsh.lsh_profile_bytes(name) / n}
    achieved = work / (ms * 1e-3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": None, "launches": n, "ms_total": ms,
            "work_per_launch": work / n}


def committed_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_2007_12718_amd", "csrc", rec["source"])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if sha != rec["source_sha256"]:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def kernel_table(lsh):
    rows = {}
    for name in lsh.lsh_profile_names():
        n, ms, work = lsh.lsh_profile_query(name)
        rows[name] = {"launches": n, "ms": round(ms, 3), "work": work}
        nbytes = lsh.lsh_profile_bytes(name)
        if nbytes > 0:  # (GEMMs: operand and result bytes beside the flops)
            rows[name]["bytes"] = nbytes
    return rows


def host_cpu():
    """CPU model name (from /proc/cpuinfo, as lscpu reports it) and logical CPU count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(n_full, n_sample):
    """The oracle (numpy/scipy, as written) timed on the host: plan + build +
    FGMRES to 1e-10 on the workload at n_sample (by default the headline size
    itself, so the value is measured, not scaled; a smaller n_sample keeps
    kappa*h and is scaled by the method's O(N^{3/2}) = O(n^3) cost)."""
    import numpy as np
    from oracle import dense, fftop, gmres, hbs
    w = workload(n_sample)
    hbs.Compression(16, w.kappa, 8, w.tol, w.proxy_width)  # warm the weight constants
    t0 = time.perf_counter()
    C = hbs.Compression(w.n, w.kappa, w.leaf, w.tol, w.proxy_width)
    t1 = time.perf_counter()
    print(f"# cpu_baseline n={w.n}: plan {t1 - t0:.1f} s", file=sys.stderr, flush=True)
    M = hbs.Inverse(C, w.b)
    t2 = time.perf_counter()
    print(f"# cpu_baseline n={w.n}: build {t2 - t1:.1f} s", file=sys.stderr, flush=True)
    F = fftop.FFTOperator(w.n, w.kappa, w.op_order)
    f = dense.rhs(w.b, w.u_inc, w.kappa)
    x, it, hist = gmres.fgmres(lambda v: F.apply(w.b, v).reshape(-1), M.apply, f, w.gmres_tol, 100)
    dt = time.perf_counter() - t0
    res = float(np.linalg.norm(f - F.apply(w.b, x).reshape(-1)) / np.linalg.norm(f))
    try:
        from threadpoolctl import threadpool_info
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        blas = os.cpu_count()
    model, ncpu = host_cpu()
    scale = (n_full / n_sample) ** 3
    how = "measured" if scale == 1 else f"{dt:.2f} s measured at n={n_sample}, scaled by (n/{n_sample})^3 = {scale:.0f}"
    return {"value": dt * scale, "unit": "s", "cores": blas, "kind": "oracle",
            "sample": f"oracle plan + build + FGMRES to 1e-10 on the full workload at n={n_sample} "
                      f"(N={n_sample ** 2}): {how}; plan {t1 - t0:.1f} s, build {t2 - t1:.1f} s, "
                      f"FGMRES {dt - (t2 - t0):.1f} s, {it} iterations, residual {res:.1e}; LAPACK/BLAS "
                      f"threads {blas} (numpy FFT single-threaded); host '{model}', os.cpu_count()={ncpu}",
            "host_cpu": model, "cpu_count": ncpu}


def batched_record(count, steps, warmup):
    """Factor time of many uneven instances: the levels aligned from the
    leaves, each level step's products and inverses over all instances
    (lsh_batch_factor; the lower levels as one persistent launch per level),
    against lsh_factor_create per instance; plans are built beforehand
    (b-independent), solves are per instance either way."""
    import torch
    import synth
    from paper_2007_12718_amd import lsh
    ws = synth.batched(count)
    plans = [lsh.Plan(w.n, w.kappa, op_order=w.op_order, leaf=w.leaf, tol=w.tol, proxy_width=2, prec="fp32")
             for w in ws]
    bs = [torch.from_numpy(w.b).cuda() for w in ws]
    res = {}
    for mode in ("separate", "batched"):
        times = []
        for k in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "batched":
                fs = lsh.batch_factor(plans, bs)
            else:
                fs = [lsh.Factor(P, b) for P, b in zip(plans, bs)]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if k >= warmup:
                times.append(dt)
            for F in fs:
                F.close()
        res[mode] = sorted(times)[len(times) // 2]
        print(f"# batched-{count} {mode}: {times}", file=sys.stderr, flush=True)
    # one solve per instance with the batched factors (FP64 FGMRES to 1e-10)
    fs = lsh.batch_factor(plans, bs)
    its, worst = [], 0.0
    for w, F in zip(ws, fs):
        _, _, info, rc = F.solve(torch.from_numpy(w.u_inc).cuda(), tol=1e-10, maxit=100, want_u=False)
        its.append(info.iterations)
        worst = max(worst, info.true_residual)
        F.close()
    for P in plans:
        P.close()
    sizes = {}
    for w in ws:
        sizes[w.n] = sizes.get(w.n, 0) + 1
    return {"value": res["batched"], "unit": "s", "separate_s": res["separate"],
            "speedup": res["separate"] / res["batched"],
            "workload": f"batched-{count}: sides {sizes}, kappa = 2 pi U[5,20], 10 bumps clipped at 0.95, "
                        f"6th-order operator, FP32 HBS at tol 1e-4; factor time of all instances",
            "iterations": its, "max_true_residual": worst}


def batched_run(a):
    r = batched_record(a.batched, a.steps, a.warmup)
    out = {"metric": "batched HBS factor time, uneven instances", "value": r["value"], "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "separate_s": r["separate_s"], "speedup": r["speedup"], "dtype": "c64 HBS", "data": "synthetic",
           "config": {"workload": r["workload"], "iterations": r["iterations"],
                      "max_true_residual": r["max_true_residual"]}}
    print(json.dumps(out))
    return 0


def bumps_record(steps, warmup, full_levels):
    """The 256 x 256 ten-bump workload (kappa = 40 pi, 6th-order operator):
    time to a 1e-10 residual with FP32 and FP64 HBS factors."""
    import torch
    import synth
    from paper_2007_12718_amd import lsh
    w = synth.bumps20()
    b_d = torch.from_numpy(w.b).cuda()
    u_d = torch.from_numpy(w.u_inc).cuda()
    out = {"workload": f"bumps-256: n=256 (N=65536), kappa=40 pi, 10 bumps clipped at 0.95, HBS 4th order tol 1e-4, "
                       f"operator order 6, GMRES tol 1e-10"}
    for prec in ("fp32", "fp64"):
        rs = []
        for k in range(warmup + steps):
            r = run_step(lsh, w, b_d, u_d, prec, torch, full_levels=full_levels)
            if k >= warmup:
                rs.append(r)
        med = sorted(rs, key=lambda r: r["total_s"])[len(rs) // 2]
        out[prec] = {"value": med["total_s"], "unit": "s", "build_s": med["build_s"], "solve_s": med["solve_s"],
                     "iterations": med["iterations"], "true_residual": med["true_residual"]}
    out["speedup_fp32_over_fp64"] = out["fp64"]["value"] / out["fp32"]["value"]
    return out


def direct_run(a):
    """Direct-solver mode (the paper's Sec. 6 experiments): the HBS of the
    10th-order matrix at --direct-tol (proxy ring of 3 layers), built and
    applied once, sigma = M f; its residual in the 10th-order operator is
    checked with the FFT matvec, and FGMRES preconditioned by it finishes to
    1e-12."""
    import numpy as np
    import torch
    from paper_2007_12718_amd import lsh
    w = workload(a.direct)
    b_d = torch.from_numpy(w.b).cuda()
    u_d = torch.from_numpy(w.u_inc).cuda()
    k2 = w.kappa ** 2
    f = (-k2 * b_d * u_d[0]).reshape(1, w.n, w.n).contiguous()
    kw = dict(op_order=10, leaf=w.leaf, tol=a.direct_tol, proxy_width=3, prec="fp64", merge=a.merge, hbs_order=10)
    # lsh_build sizes both workspaces by the rank bounds before any rank is
    # known; where the two do not fit in the free device memory, the plan is
    # created first and the factor sized exactly from its ranks
    d = lsh.LshDesc(n=w.n, h=1.0 / w.n, x0=-0.5, y0=-0.5, kappa=w.kappa, op_order=10, leaf=w.leaf,
                    tol=a.direct_tol, proxy_width=3, hbs_prec=lsh.LSH_FP64, merge=lsh.MERGE[a.merge],
                    hbs_order=10, plan_cache=0)
    pb, fb = lsh._size(), lsh._size()
    lsh._check(lsh.lib().lsh_build_workspace(ctypes.byref(d), 0, ctypes.byref(pb), ctypes.byref(fb)))
    free = torch.cuda.mem_get_info()[0]
    pipelined = pb.value + fb.value < 0.9 * free
    times, res = [], []
    for k in range(a.warmup + a.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if pipelined:
            P, F = lsh.build(w.n, w.kappa, b_d, **kw)
        else:
            P = lsh.Plan(w.n, w.kappa, **kw)
            F = lsh.Factor(P, b_d)
        sig = F.apply_precond(f)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r = (f - P.apply_operator(b_d, sig)).norm().item() / f.norm().item()
        if k >= a.warmup:
            times.append(dt)
            res.append(r)
        print(f"# direct step {k}: {dt:.3f} s, residual {r:.2e}, ranks {P.ranks()[1]}", file=sys.stderr, flush=True)
        if k < a.warmup + a.steps - 1:
            F.close()
            P.close()
    s, _, info, rc = F.solve(u_d, tol=1e-12, maxit=20, want_u=False)
    out = {"metric": "direct-solver time (10th-order HBS build + one apply)", "value": sorted(times)[len(times) // 2],
           "unit": "s", "higher_is_better": False, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "dtype": "c128 HBS", "data": "synthetic",
           "config": {"workload": f"fourier-{w.n}: n={w.n} (N={w.n ** 2}), kappa={w.kappa:.4f}, 10th-order "
                                  f"HBS tol {a.direct_tol:g} leaf {w.leaf} proxy width 3, merge {a.merge}",
                      "build": "lsh_build (pipelined)" if pipelined else
                               f"lsh_plan_create + lsh_factor_create (the pipelined build's rank-bound "
                               f"workspaces, {(pb.value + fb.value) / 2 ** 30:.0f} GiB, exceed the free memory)",
                      "relative_residual_10th_order": max(res), "ranks": P.ranks()[1],
                      "lowrank_ranks": P.lowrank_ranks(), "fgmres_iterations_to_1e-12": info.iterations,
                      "fgmres_true_residual": info.true_residual}}
    print(json.dumps(out))
    F.close()
    P.close()
    return 0


def plan_cache_run(a):
    """The headline step (FP32 HBS build + FGMRES to 1e-10) for a new b each
    step, with every row ID of the plan served by the plan cache (the
    universal compression reused: Sec. 3.2), against the cold step."""
    import numpy as np
    import torch
    import synth
    from paper_2007_12718_amd import lsh
    w = workload(a.n)
    u_d = torch.from_numpy(w.u_inc).cuda()
    bs = [torch.from_numpy(synth.fourier_field(w.n, np.random.default_rng(100 + k))).cuda()
          for k in range(a.warmup + a.steps)]
    res = {}
    for mode in ("cold", "cached"):
        lsh.plan_cache_clear()
        times, its = [], []
        for k, b_d in enumerate(bs):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P, F = lsh.build(w.n, w.kappa, b_d, op_order=w.op_order, leaf=w.leaf, tol=w.tol,
                             proxy_width=w.proxy_width, prec="fp32", merge=a.merge, plan_cache=(mode == "cached"))
            _, _, info, rc = F.solve(u_d, tol=w.gmres_tol, maxit=100, want_u=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            assert rc == 0 and info.true_residual < w.gmres_tol
            if k >= a.warmup:
                times.append(dt)
                its.append(info.iterations)
            F.close()
            P.close()
        res[mode] = (sorted(times)[len(times) // 2], its)
        print(f"# {mode}: {times} iterations {its}", file=sys.stderr, flush=True)
    n_e, by = lsh.plan_cache_info()
    lsh.plan_cache_clear()
    out = {"metric": "time-to-1e-10 residual for a new b, row IDs from the plan cache", "value": res["cached"][0],
           "unit": "s", "higher_is_better": False, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "cold_s": res["cold"][0], "speedup": res["cold"][0] / res["cached"][0], "dtype": "c64 HBS + c128 GMRES",
           "data": "synthetic",
           "config": {"workload": f"fourier-{w.n} with a new seeded random Fourier b per step, FP32 HBS tol {w.tol}, "
                                  f"operator order {w.op_order}", "iterations": res["cached"][1],
                      "cache_entries": n_e, "cache_device_bytes": by}}
    print(json.dumps(out))
    return 0


def multi_rhs_run(a):
    """Solve time of several right-hand sides with one factor: the lockstep
    FGMRES (one preconditioner and one operator application per iteration
    for the whole group) against one lsh_solve call per right-hand side."""
    import numpy as np
    import torch
    import synth
    from paper_2007_12718_amd import lsh
    w = synth.differentiation(nwaves=a.multi_rhs)
    b_d = torch.from_numpy(w.b).cuda()
    u_d = torch.from_numpy(w.u_inc).cuda()
    P, F = lsh.build(w.n, w.kappa, b_d, op_order=w.op_order, leaf=w.leaf, tol=w.tol, proxy_width=w.proxy_width,
                     prec="fp32")
    nr = u_d.shape[0]
    res, its = {}, {}
    for mode in ("one_by_one", "lockstep"):
        times = []
        for k in range(a.warmup + a.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "lockstep":
                s, _, info, rc = F.solve(u_d, tol=1e-10, maxit=100, want_u=False)
                it = [info.iterations]
            else:
                it = []
                for r in range(nr):
                    s, _, info, rc = F.solve(u_d[r:r + 1], tol=1e-10, maxit=100, want_u=False)
                    it.append(info.iterations)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            assert rc == 0 and info.true_residual < 1e-10, (mode, rc, info.true_residual)
            if k >= a.warmup:
                times.append(dt)
        res[mode] = sorted(times)[len(times) // 2]
        its[mode] = it
        print(f"# {mode}: {times} iterations {it}", file=sys.stderr, flush=True)
    out = {"metric": "FGMRES solve time to 1e-10, several right-hand sides, one FP32 HBS factor",
           "value": res["lockstep"], "unit": "s", "higher_is_better": False, "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "one_by_one_s": res["one_by_one"],
           "speedup": res["one_by_one"] / res["lockstep"], "dtype": "f64 FGMRES, c64 HBS", "data": "synthetic",
           "config": {"workload": f"{w.name}: {nr} plane waves at equispaced angles, kappa = 80 pi, 30 smooth "
                                  f"bumps, 10th-order operator, FP32 HBS at tol 1e-4",
                      "iterations_one_by_one": its["one_by_one"],
                      "iterations_last_lockstep": its["lockstep"]}}
    print(json.dumps(out))
    F.close()
    P.close()
    return 0


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "described in DESIGN.md but not built)"}))
        return 2
    import numpy as np
    import torch
    from paper_2007_12718_amd import lsh

    torch.cuda.set_device(0)
    if a.batched:
        return batched_run(a)
    if a.multi_rhs:
        return multi_rhs_run(a)
    if a.direct:
        return direct_run(a)
    if a.plan_cache:
        return plan_cache_run(a)
    if a.calib_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = workload(a.n)
    b_d = torch.from_numpy(w.b).cuda()
    u_d = torch.from_numpy(w.u_inc).cuda()
    forms = ["fp32"] + ([] if a.no_fp64 else ["fp64"])
    # The last FP32 warmup step records every instrumented kernel (the kernel
    # table and the dominant kernel); the timed steps record only the
    # dominant kernel, so that event overhead stays out of the step time.
    kernels_warm, dominant = None, None
    for i in range(a.warmup):
        for prec in forms:
            full = prec == "fp32" and not a.no_profile and i == a.warmup - 1
            if full:
                lsh.lsh_profile_only(None)
                lsh.lsh_profile_enable(True)
            r = run_step(lsh, w, b_d, u_d, prec, torch, a.separate, a.merge, a.full_levels)
            if full:
                kernels_warm = kernel_table(lsh)
                rl = roofline(lsh)
                dominant = rl["kernel"] if rl else None
                lsh.lsh_profile_enable(False)
            print(f"# warmup {prec}: {json.dumps(r)}", file=sys.stderr, flush=True)
    results = {}
    prof = None
    for prec in forms:
        steps = []
        if prec == "fp32" and not a.no_profile:
            lsh.lsh_profile_only(dominant)
            lsh.lsh_profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(a.steps):
            r = run_step(lsh, w, b_d, u_d, prec, torch, a.separate, a.merge, a.full_levels)
            steps.append(r)
            print(f"# step {k} {prec}: {json.dumps(r)}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if prec == "fp32" and not a.no_profile:
            prof = {"roofline": roofline(lsh), "kernels": kernels_warm or kernel_table(lsh),
                    "kernels_from": "last warmup step" if kernels_warm else "timed steps"}
            lsh.lsh_profile_enable(False)
            lsh.lsh_profile_only(None)
        med = sorted(steps, key=lambda r: r["total_s"])[len(steps) // 2]
        results[prec] = {"wall_s": wall, "ms_per_step": 1e3 * wall / a.steps, "median": med}
    head = results["fp32"]
    out = {
        "metric": "time-to-1e-10 residual (HBS build+GMRES), FP32-HBS vs FP64-HBS, N~1M",
        "value": head["ms_per_step"] / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 HBS + c128 GMRES",
        "data": "synthetic",
        "config": {"workload": f"fourier-{w.n}: n={w.n} (N={w.n ** 2}), kappa={w.kappa:.4f}, "
                               f"b random Fourier field |k|<=20 cycles in [-1,0.9], plane wave, "
                               f"HBS 4th order tol={w.tol} leaf={w.leaf} proxy_width={w.proxy_width}, "
                               f"operator order {w.op_order}, GMRES tol {w.gmres_tol}",
                   "hbs_prec": "fp32", "merge": a.merge, "full_levels": a.full_levels,
                   "phases_s": {k: head["median"][k] for k in
                                                    ("build_s", "plan_s", "factor_s", "solve_s", "total_s")},
                   "step_median_s": head["median"]["total_s"],
                   "iterations": head["median"]["iterations"],
                   "true_residual": head["median"]["true_residual"],
                   "ranks": head["median"]["ranks"]},
    }
    # the solve's streams (K6 apply, K7 FFT operator, K8 Gram-Schmidt) from the
    # median step's FGMRES phase clocks (hipEvents around each phase)
    med = head["median"]
    its = max(med["iterations"], 1)
    ab = apply_bytes(w.n, w.leaf, med["ranks"], med["lowrank_ranks"], 8)
    Mfft = 1
    while Mfft < 2 * w.n:
        Mfft *= 2
    Hq = Mfft // 2 + 1
    ob = 16.0 * 2 * w.n ** 2 + 8.0 * w.n ** 2 + 16.0 * Hq ** 2   # x, y, b once and the spectrum quarter once
    # what the five passes move (row transform, transpose, column transform with
    # the spectrum, transpose, inverse row transform with the epilogue): the
    # n x M intermediate is written and read four times
    pb = 16.0 * w.n ** 2 + 16.0 * 8 * w.n * Mfft + 16.0 * Hq ** 2 + 40.0 * w.n ** 2
    t_ap, t_op = med["solve_ms_precond"] / its, med["solve_ms_operator"] / its
    out["solve_streams"] = {
        "apply_ms": t_ap, "apply_algorithmic_GB": ab / 1e9, "apply_GBs": ab / (t_ap * 1e-3) / 1e9,
        "fft_operator_ms": t_op, "fft_operator_algorithmic_GB": ob / 1e9, "fft_operator_GBs": ob / (t_op * 1e-3) / 1e9,
        "fft_operator_pass_GB": pb / 1e9, "fft_operator_pass_GBs": pb / (t_op * 1e-3) / 1e9,
        "gram_schmidt_ms_per_iteration": med["solve_ms_ortho"] / its,
        "note": "per FGMRES iteration of the median timed FP32 step; GB/s of algorithmic bytes against 8000"}
    if "fp64" in results:
        r64 = results["fp64"]
        out["fp64_hbs"] = {"value": r64["ms_per_step"] / 1e3, "unit": "s",
                           "phases_s": {k: r64["median"][k] for k in ("build_s", "plan_s", "factor_s", "solve_s", "total_s")},
                           "iterations": r64["median"]["iterations"],
                           "true_residual": r64["median"]["true_residual"],
                           "speedup_fp32_over_fp64": r64["ms_per_step"] / head["ms_per_step"]}
    if prof:
        if prof["roofline"]:
            rl = prof["roofline"]
            rl["traffic"] = committed_traffic(rl["kernel"])
            if rl["traffic"] and rl.get("algorithmic_bytes_per_launch"):
                rl["traffic_over_algorithmic"] = rl["traffic"] / rl["algorithmic_bytes_per_launch"]
        out["roofline"] = prof["roofline"]
        out["kernels"] = prof["kernels"]
        out["kernels_from"] = prof["kernels_from"]
    if not a.no_extra:  # the other workloads' figures, beside the headline
        if a.full_levels:  # the paper's form (every level below the root compressed), same workload
            rs = [run_step(lsh, w, b_d, u_d, "fp32", torch, a.separate, a.merge, 0) for _ in range(4)][1:]
            med = sorted(rs, key=lambda r: r["total_s"])[len(rs) // 2]
            out["full_levels0"] = {"value": med["total_s"], "unit": "s", "build_s": med["build_s"],
                                   "solve_s": med["solve_s"], "iterations": med["iterations"],
                                   "true_residual": med["true_residual"], "ranks": med["ranks"],
                                   "note": "FP32 HBS with every level below the root compressed; median of 3 "
                                           "steps after 1 warmup"}
        out["bumps256"] = bumps_record(3, 1, a.full_levels)
        out["batched64"] = batched_record(64, 3, 1)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w.n, min(a.cpu_n or w.n, w.n))
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
