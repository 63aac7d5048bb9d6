#!/usr/bin/env python3
"""Throughput of the DG p-multigrid MGCG solver on one MI355X.

Workload (default, --workload c2): 3D Poisson on [0,1]^3, 16^3 uniform
elements, SIPG with P = 8 (2,985,984 unknowns), homogeneous Dirichlet,
right-hand side i.i.d. U[-1,1] (seed 2), face-centred additive Schwarz with
level overlap, V(1,1), MGCG to a 1e-10 relative residual, FP64 throughout.
One step = one complete solve from x = 0 (every stage of the path: operator
applies, patch solves, overlap summation, transfers, coarse solve, PCG
updates).  The other precision (FP32 V-cycle inside FP64 PCG) is timed on the
same workload for the mixed-vs-FP64 ratio.

Other workloads: c3 (32^3 LDG, z stretched to aspect ratio 32, mixed), c5
(8^3 at P = 32 with random per-direction sizes, mixed; --learned adds the
shipped face-weight network with its probe fallback), c4 (64 independent
grids of 4^3..16^3 elements at P in {4,6,8,12,16} solved together in one
batched, graph-replayed MGCG, against the same grids solved one by one in
FP64).

Prints one JSON line: DoF/s (unknowns / solve time), the live roofline of the
dominant kernel (top-level patch solve, HIP events on the solver's stream),
its HBM traffic when measured for the current kernel sources, and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DoF/s to 1e-10 rel. residual (PCG+pMG), smoother HBM GB/s; mixed vs FP64"
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
HBM_PEAK_GBPS = 8000.0

# HBM bytes per launch of the dominant kernel from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE), scaled by the same counters on a plain copy of
# known size (bench.py --copy-calibration); the summary with commands is in
# profiles/.  Valid only for the kernel source it was measured on: the hash of
# the patch-solve section of kernels.hpp is compared at run time and the
# figure dropped on any change.
TRAFFIC = {"bytes_per_launch": 133.7e6,
           "kernel_src_sha256": "dcade7b4b14fe7fab6692c5f761499aa8e5873dff0024b26a2380f6288ca0dd7",
           "profile": "profiles/fdm_p8_c2_fp64_pmc_traffic.md"}
KERNEL_SOURCE = "paper_1603_02524_amd/csrc/kernels.hpp"
KERNEL_SECTION = ("// ================================================================ FDM patch solve",
                  "// ================================================================ overlap summation")


def _kernel_src_hash():
    """sha256 of the patch-solve section of the kernel header (the dominant kernel)."""
    import hashlib
    with open(os.path.join(ROOT, KERNEL_SOURCE), encoding="utf-8") as fh:
        text = fh.read()
    a, b = text.index(KERNEL_SECTION[0]), text.index(KERNEL_SECTION[1])
    return hashlib.sha256(text[a:b].encode()).hexdigest()


def _copy_calibration(mb, reps=5):
    """Plain device copies of a known size (the calibration kernel of the PMC runs)."""
    import torch
    n = mb * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_copy": 8 * n, "bytes_written_per_copy": 8 * n,
                                           "copies": reps}}), flush=True)


def _workload(name):
    import synth
    if name == "c2":
        return synth.c2_poisson3d_p8()
    if name == "c2small":
        return synth.c2_poisson3d_p8(n=8)
    if name == "c3":
        return synth.c3_ldg3d_stretched()
    if name == "c5":
        return synth.c5_poisson3d_p32()
    raise SystemExit(f"unknown workload {name}")


FP32_MFMA_PEAK_TFLOPS = 157.3


def _top_kernel(S, m):
    """Name, element type and peak of the top-level patch-solve kernel."""
    L = S.num_levels - 1
    P, n_o, _ = S.level_info(L)
    nl = P + 1 + 2 * n_o
    na = 2 * P if m.smoother == "FA" else nl
    f64 = m.precision == "fp64"
    t = "double" if f64 else "float"
    big = S.grid.dim == 3 and P == 32
    name = (f"fdm_big_{{a,b,c}}<{t},{na},{nl}>" if big else f"fdm_kernel<{t},3,{na},{nl}>") + \
        f" ({'face' if m.smoother == 'FA' else 'element'}-centred patch solve, P={P}, N_O={n_o})"
    return name, (FP64_VALU_PEAK_TFLOPS if f64 else FP32_MFMA_PEAK_TFLOPS)


def _run_batch(args):
    """Many grids (3D, 4^3..16^3 elements, P in {4, 6, 8, 12, 16}) solved together."""
    import numpy as np
    import torch
    import synth
    from paper_1603_02524_amd import dgmg
    ws = synth.c4_batched()
    _log(f"setup {len(ws)} grids")
    B = dgmg.BatchSolver([(w.grid, w.method) for w in ws], max_iter=200)
    n = B.n_dof
    rhs = torch.tensor(np.concatenate([synth.rhs_uniform(w.seed, w.grid.n_dof(w.method.P)) for w in ws]),
                       device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    if not args.no_autotune:
        _log("autotuning")
        B.autotune()
    for _ in range(args.warmup):
        x.zero_()
        B.solve(rhs, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        st = B.solve(rhs, x)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    its = [s["iterations"] for s in st]
    out = {"metric": METRIC, "value": n / sec, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64/f32", "data": "synthetic",
           "config": {"workload": f"batched_{len(ws)}_grids_3d_mixed", "grids": len(ws), "n_dof": n,
                      "iterations_min_max": [min(its), max(its)], "converged": all(s["converged"] for s in st),
                      "graphs": True}}
    if not args.no_mixed:
        # the same grids one after another with the plain FP64 solver (one handle each)
        _log("timing the same grids one by one in FP64")
        tot = 0.0
        for w, (a, b) in zip(ws, zip(B.offsets[:-1], B.offsets[1:])):
            m64 = synth.with_method(w, precision="fp64").method
            S = dgmg.Solver(w.grid, m64, max_iter=200)
            if not args.no_autotune:
                S.autotune()
            xs = torch.zeros(b - a, dtype=torch.float64, device="cuda")
            r = rhs[a:b].contiguous()
            S.solve(r, xs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(max(1, args.steps // 2)):
                xs.zero_()
                S.solve(r, xs)
            torch.cuda.synchronize()
            tot += (time.perf_counter() - t0) / max(1, args.steps // 2)
            S.close()
        out["fp64_one_by_one"] = {"value": n / tot, "unit": "DoF/s", "ms_per_step": tot * 1e3,
                                  "batched_time_per_dof_vs_fp64": sec / tot}
    B.close()
    print(json.dumps(out), flush=True)


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _time_solves(S, rhs, x, tol, warmup, steps, timing):
    import torch
    st = None
    for _ in range(warmup):
        x.zero_()
        st = S.solve(rhs, x, tol)
    torch.cuda.synchronize()
    if timing:
        S.kernel_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        st = S.solve(rhs, x, tol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = S.kernel_time() if timing else None
    if timing:
        S.kernel_timing(False)
    return (t1 - t0) / steps, st, kt


def _cpu_baseline(w, rhs_np, gpu_iters, sample_iters):
    """Oracle (FP64 numpy/scipy) on the same inputs: the first `sample_iters`
    MGCG iterations, timed, scaled to the full iteration count."""
    import numpy as np
    from oracle import multigrid as mg
    from oracle import operator as op
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = 1
    g, m = w.grid, w.method
    H = mg.Hierarchy(g, m, patch_mode="fdm", assemble=False)
    f = op.to_lex(rhs_np, g.n, m.P)
    t0 = time.perf_counter()
    mg.mgcg(H, f, np.zeros_like(f), tol=w.tol, i_max=sample_iters)
    t = time.perf_counter() - t0
    per_cycle = t / (sample_iters + 1)          # one V-cycle + one operator apply each
    t_full = per_cycle * gpu_iters
    return {"value": w.n_dof / t_full, "unit": "DoF/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"first {sample_iters} MGCG iteration(s) ({sample_iters + 1} V-cycles) of the "
                       f"same workload on the host, {t:.1f} s, scaled to the {gpu_iters} iterations "
                       f"of the full solve")}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c2", "c2small", "c3", "c4", "c5"],
                    help="c2 (default): 16^3 P=8 FP64; c3: 32^3 stretched LDG mixed; c4: 64 batched grids; "
                         "c5: 8^3 P=32 mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--learned", action="store_true",
                    help="also time the solver with the shipped learned face weights")
    ap.add_argument("--cpu-sample-iters", type=int, default=1)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run plain device copies of MB MiB (PMC calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the solver "
              "runs on a single MI355X; multi-GPU sharding is a design note only)", file=sys.stderr)
        raise SystemExit(2)

    if args.copy_calibration:
        _copy_calibration(args.copy_calibration)
        return

    if args.workload == "c4":
        _run_batch(args)
        return

    import numpy as np
    import torch

    import synth
    from paper_1603_02524_amd import dgmg

    w = _workload(args.workload)
    g, m = w.grid, w.method
    _log(f"setup {w.name}")
    S = dgmg.Solver(g, m, max_iter=200)
    n = S.n_dof()
    rhs_np = synth.rhs_uniform(w.seed, n)
    rhs = torch.tensor(rhs_np, dtype=torch.float64, device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    if not args.no_autotune:
        # patch-solve block shapes per (level, sweep kind); bitwise-neutral, outside the timed region
        _log("autotuning patch-solve block shapes")
        tuning = S.autotune()
    else:
        tuning = {}
    _log(f"timing {m.precision} solves")
    sec, st, kt = _time_solves(S, rhs, x, w.tol, args.warmup, args.steps, timing=True)
    _log(f"{m.precision}: {sec * 1e3:.2f} ms per solve, {st['iterations']} iterations")
    # true residual of the final iterate (outside the timed region)
    r = S.residual(S.num_levels - 1, rhs, x)
    true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(rhs))
    if not (st["converged"] and true_rel <= 1.01 * w.tol):
        print(json.dumps({"error": "solve did not reach the tolerance", "stats": st,
                          "true_rel": true_rel}), file=sys.stderr)
        raise SystemExit(1)

    # dominant kernel: top-level patch solve
    k_ms = kt["ms"] / max(kt["launches"], 1)
    k_flops = kt["flops"] / max(kt["launches"], 1)
    k_bytes = kt["bytes"] / max(kt["launches"], 1)
    achieved = k_flops / (k_ms * 1e-3) / 1e12
    traffic = None
    if (args.workload == "c2" and TRAFFIC["bytes_per_launch"]
            and TRAFFIC["kernel_src_sha256"] == _kernel_src_hash()):
        traffic = TRAFFIC["bytes_per_launch"]
    kname, peak = _top_kernel(S, m)
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic, "kernel": kname,
            "avg_ms": k_ms, "launches": kt["launches"], "flops_per_launch": k_flops,
            "alg_bytes_per_launch": k_bytes, "alg_GBps": k_bytes / (k_ms * 1e-3) / 1e9}

    out = {"metric": METRIC, "value": n / sec, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if m.precision == "fp64" else "f64/f32",
           "data": "synthetic",
           "config": {"workload": w.name, "elements": list(g.n), "P": m.P, "n_dof": n,
                      "flux": m.flux, "smoother": f"{m.smoother}_l", "vcycle": "V(1,1)",
                      "precision": m.precision, "tol": w.tol, "seed": w.seed,
                      "iterations": st["iterations"], "true_rel_residual": true_rel,
                      "autotuned_waves": {f"l{l}k{k}": v[0] for (l, k), v in sorted(tuning.items())},
                      "autotuned_sweep_us": {f"l{l}k{k}": round(v[1] * 1e3, 2) for (l, k), v in sorted(tuning.items())}},
           "roofline": roof}

    if not args.no_mixed:
        # the other precision on the same workload: mixed vs FP64 time per DoF
        other = "mixed" if m.precision == "fp64" else "fp64"
        _log(f"timing {other} solves")
        wm = synth.with_method(w, precision=other)
        Sm = dgmg.Solver(wm.grid, wm.method, max_iter=200)
        if not args.no_autotune:
            Sm.autotune()
        xm = torch.zeros(n, dtype=torch.float64, device="cuda")
        secm, stm, _ = _time_solves(Sm, rhs, xm, w.tol, args.warmup, args.steps, timing=False)
        rm = Sm.residual(Sm.num_levels - 1, rhs, xm)
        t_mixed, t_fp64 = (secm, sec) if other == "mixed" else (sec, secm)
        out[other] = {"value": n / secm, "unit": "DoF/s", "ms_per_step": secm * 1e3,
                      "iterations": stm["iterations"],
                      "true_rel_residual": float(torch.linalg.norm(rm) / torch.linalg.norm(rhs)),
                      "mixed_time_per_dof_vs_fp64": t_mixed / t_fp64}
        Sm.close()

    if args.learned and m.smoother == "FA":
        # learned face weights (shipped network, probe fallback) on the main solver
        from paper_1603_02524_amd import learn
        if os.path.exists(learn.DEFAULT_PARAMS):
            _log("timing solves with learned face weights")
            params = torch.tensor(learn.load_params(), device="cuda")
            kept, rl, rf = S.apply_mlp(params, probe_iters=4)
            xl = torch.zeros(n, dtype=torch.float64, device="cuda")
            secl, stl, _ = _time_solves(S, rhs, xl, w.tol, args.warmup, args.steps, timing=False)
            rl_true = S.residual(S.num_levels - 1, rhs, xl)
            out["learned"] = {"kept": kept, "probe_ratio_learned": rl, "probe_ratio_fixed": rf,
                              "value": n / secl, "unit": "DoF/s", "ms_per_step": secl * 1e3,
                              "iterations": stl["iterations"],
                              "true_rel_residual": float(torch.linalg.norm(rl_true) / torch.linalg.norm(rhs)),
                              "time_per_dof_vs_fixed": secl / sec}
            S.set_face_params(None)

    if not args.no_cpu_baseline:
        _log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = _cpu_baseline(w, rhs_np, st["iterations"], args.cpu_sample_iters)
    S.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
