#!/usr/bin/env python3
"""Throughput of the DG p-multigrid MGCG solver on one MI355X.

Workload (the value): 3D Poisson on [0,1]^3, 16^3 uniform elements, SIPG with
P = 8 (2,985,984 unknowns), homogeneous Dirichlet, right-hand side i.i.d.
U[-1,1] (seed 2), face-centred additive Schwarz with level overlap, V(1,1),
MGCG to a 1e-10 relative residual (confirmed on the true residual), FP64
throughout.  One step = one complete solve from x = 0 (every stage of the
path: operator applies, patch solves, overlap summation, transfers, coarse
solve, PCG updates), inputs resident in HBM.

Also on the line:
* roofline: the dominant kernel (top-level patch solve), algorithmic flops per
  launch = flops per unknown of one sweep's fast-diagonalisation patch solves x
  the level's unknowns, over the mean launch time from HIP events on the
  solver's stream; HBM bytes per launch from rocprofv3 counters when they were
  taken on the current kernel source;
* smoothing_step: one whole top-level smoothing step against its attainable
  roof max(bytes / HBM peak, flops / compute peak);
* mixed: the FP32 V-cycle inside FP64 PCG on the same input;
* c3, c5, c4, c4_small (unless --quick): 32^3 LDG stretched to aspect ratio
  32, 8^3 at P = 32 (with the learned face weights), 64 batched grids, and 64
  small batched grids, each against the plain FP64 solver (one by one, and one
  by one in mixed precision, for the batches);
* cpu_baseline: the oracle on a bounded sample of the same workload.
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
           "kernel_src_sha256": "21eeba7092ae86177bd0f64650ee51eb25155c3bbcf43ef78c7fe3c4e1f6d4cc",
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


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# every TIMING_STRIDE-th top-level patch-solve launch of the timed solves carries an
# event pair (a stride prime to the sweep count samples every sweep normal alike)
TIMING_STRIDE = 5


def _time_solves(S, rhs, x, tol, warmup, steps, timing):
    import torch
    st = None
    for _ in range(warmup):
        x.zero_()
        st = S.solve(rhs, x, tol)
    torch.cuda.synchronize()
    if timing:
        S.kernel_timing(True, stride=TIMING_STRIDE)
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


# ---------------------------------------------------------------- algorithmic counts
def sweep_flops_per_dof(dim, P, n_o, smoother):
    """Flops per unknown of one Schwarz sweep's patch solves (fast diagonalisation:
    D forward and D backward 1D contractions per patch, two flops per multiply-add),
    one patch per element: FC tile a x n^(D-1) with a = 2P, n = N_P + 2 N_O:
    4 (a^2 n^(D-1) + (D-1) a n^D) / N_P^D; EC tile n^D: 4 D n^(D+1) / N_P^D."""
    NP = P + 1
    n = NP + 2 * n_o
    if smoother == "FA":
        a = 2 * P
        return 4.0 * (a * a * n ** (dim - 1) + (dim - 1) * a * n ** dim) / NP ** dim
    return 4.0 * dim * n ** (dim + 1) / NP ** dim


def apply_flops_per_dof(dim, P):
    """Operator apply: 2 D N_P (the volume contractions) + 12 D (face terms)."""
    return 2.0 * dim * (P + 1) + 12.0 * dim


def _dominant_roofline(S, m, kt, word):
    """Top-level patch solve: algorithmic flops and bytes per launch from the counts per
    unknown times the level's unknowns, over the mean launch time (HIP events)."""
    L = S.num_levels - 1
    P, n_o, n = S.level_info(L)
    dim = S.grid.dim
    k_ms = kt["ms"] / max(kt["launches"], 1)
    flops = sweep_flops_per_dof(dim, P, n_o, m.smoother) * n
    alg_bytes = 3.0 * word * n                        # one sweep: read u and f, write u
    f64 = m.precision == "fp64"
    peak = FP64_VALU_PEAK_TFLOPS if f64 else FP32_MFMA_PEAK_TFLOPS
    ridge = peak * 1e12 / (HBM_PEAK_GBPS * 1e9)
    bound = "mfma" if flops / alg_bytes > ridge else "hbm"
    achieved = flops / (k_ms * 1e-3) / 1e12
    traffic = None
    if (S.grid.n == (16, 16, 16) and P == 8 and f64 and TRAFFIC["bytes_per_launch"]
            and TRAFFIC["kernel_src_sha256"] == _kernel_src_hash()):
        traffic = TRAFFIC["bytes_per_launch"]
    kname, _ = _top_kernel(S, m)
    roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic, "kernel": kname, "avg_ms": k_ms, "launches": kt["launches"],
            "launch_sampling_stride": TIMING_STRIDE,
            "flops_per_launch": flops, "flops_per_dof": flops / n,
            "alg_bytes_per_launch": alg_bytes, "alg_GBps": alg_bytes / (k_ms * 1e-3) / 1e9,
            "hbm_GBps": None if traffic is None else traffic / (k_ms * 1e-3) / 1e9,
            "hbm_frac": None if traffic is None else traffic / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "arithmetic_intensity": flops / alg_bytes, "ridge": ridge,
            "traffic_profile": TRAFFIC["profile"] if traffic is not None else None}
    return roof


def _smoothing_step_roofline(S, m, word, reps=20, level=None):
    """One smoothing step of the top level (or of `level`) (FA: D sweeps, each residual
    apply + patch solves + overlap summation; EA: one) timed with events on the solver's
    stream, against its attainable roof max(bytes / HBM peak, flops / compute peak)."""
    import torch
    L = S.num_levels - 1 if level is None else level
    P, n_o, n = S.level_info(L)
    dim = S.grid.dim
    dt = torch.float64 if m.precision == "fp64" else torch.float32
    g = torch.Generator(device="cuda").manual_seed(7)
    u = torch.rand(n, dtype=dt, device="cuda", generator=g)
    f = torch.rand(n, dtype=dt, device="cuda", generator=g)
    S.smooth(L, u, f, 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        S.smooth(L, u, f, 1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    sweeps = dim if m.smoother == "FA" else 1
    flops = sweeps * (sweep_flops_per_dof(dim, P, n_o, m.smoother) + apply_flops_per_dof(dim, P)) * n
    byts = sweeps * 3.0 * word * n
    peak = FP64_VALU_PEAK_TFLOPS if m.precision == "fp64" else FP32_MFMA_PEAK_TFLOPS
    t_roof = max(byts / (HBM_PEAK_GBPS * 1e9), flops / (peak * 1e12)) * 1e3
    return {"level": L, "P": P, "n_dof": n, "ms": ms, "roof_ms": t_roof, "frac": t_roof / ms, "flops": flops,
            "alg_bytes": byts, "sweeps": sweeps,
            "bound": "hbm" if byts / (HBM_PEAK_GBPS * 1e9) > flops / (peak * 1e12) else "compute"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(w, rhs_np, gpu_iters, samples=3):
    """Oracle (FP64 numpy/scipy, as it stands) on the same input, on a bounded sample:
    one V-cycle and one operator apply at the top level (the work of one MGCG
    iteration), timed single-threaded (median of `samples`) and once with the
    default BLAS thread pool; extrapolated to a whole solve of gpu_iters
    iterations: gpu_iters V-cycles and gpu_iters + 2 applies (initial residual,
    one per iteration, the exit check).  Hierarchy set-up is not timed."""
    import statistics
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import multigrid as mg
    from oracle import operator as op
    g, m = w.grid, w.method
    H = mg.Hierarchy(g, m, patch_mode="fdm", assemble=False)
    f = op.to_lex(rhs_np, g.n, m.P)

    def sample():
        t0 = time.perf_counter()
        H.vcycle(np.zeros_like(f), f)
        t1 = time.perf_counter()
        H.apply(H.L, f)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    with threadpool_limits(1):
        single = [sample() for _ in range(samples)]
    pool = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    multi = sample()
    tv = statistics.median(s[0] for s in single)
    ta = statistics.median(s[1] for s in single)
    t_solve = gpu_iters * tv + (gpu_iters + 2) * ta
    t_multi = gpu_iters * multi[0] + (gpu_iters + 2) * multi[1]
    return {"value": w.n_dof / t_solve, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"extrapolated, not a whole solve: one top-level V-cycle ({tv:.1f} s) and one operator "
                       f"apply ({ta:.2f} s) of the oracle on the same workload, single-threaded, median of "
                       f"{samples}; scaled to the {gpu_iters}-iteration solve ({gpu_iters} V-cycles, "
                       f"{gpu_iters + 2} applies); set-up excluded"),
            "extrapolated": True, "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "single_thread_samples_s": [[round(a, 3), round(b, 3)] for a, b in single],
            "all_threads": {"cores": int(pool), "vcycle_s": round(multi[0], 3), "apply_s": round(multi[1], 3),
                            "value": w.n_dof / t_multi}}


def _solve_entry(S, rhs, x, tol, warmup, steps):
    sec, st, _ = _time_solves(S, rhs, x, tol, warmup, steps, timing=False)
    return sec, {"ms_per_step": sec * 1e3, "iterations": st["iterations"],
                 "true_rel_residual": st["r_true"] / st["r0"] if st["r0"] else 0.0,
                 "converged": st["converged"]}


def _extra_workload(name, args):
    """Mixed precision (the workload's own setting) against the plain FP64 solver on the
    same input; for the P = 32 workload also the learned face weights."""
    import torch
    import synth
    from paper_1603_02524_amd import dgmg
    w = _workload(name)
    n = w.n_dof
    rhs = torch.tensor(synth.rhs_uniform(w.seed, n), dtype=torch.float64, device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    out = {"workload": w.name, "n_dof": n}
    res = {}
    for prec in ("mixed", "fp64"):
        _log(f"{name}: {prec}")
        mw = synth.with_method(w, precision=prec).method
        S = dgmg.Solver(w.grid, mw, max_iter=200)
        if not args.no_autotune:
            S.autotune()
        sec, ent = _solve_entry(S, rhs, x, w.tol, args.warmup, max(2, args.steps // 2))
        ent["value"] = n / sec
        # top-level patch solve: its mean launch time (HIP events, one extra solve)
        # against the method's flop count per unknown, in the handle's precision
        S.kernel_timing(True)
        x.zero_()
        S.solve(rhs, x, w.tol)
        kt = S.kernel_time()
        S.kernel_timing(False)
        L = S.num_levels - 1
        P, n_o, nl = S.level_info(L)
        k_ms = kt["ms"] / max(kt["launches"], 1)
        fl = sweep_flops_per_dof(w.grid.dim, P, n_o, mw.smoother) * nl
        peak = FP64_VALU_PEAK_TFLOPS if prec == "fp64" else FP32_MFMA_PEAK_TFLOPS
        ent["patch_solve"] = {"kernel": _top_kernel(S, mw)[0], "avg_ms": k_ms, "launches": kt["launches"],
                              "flops_per_launch": fl, "achieved_TFLOPs": fl / (k_ms * 1e-3) / 1e12,
                              "peak_TFLOPs": peak, "frac": fl / (k_ms * 1e-3) / 1e12 / peak}
        res[prec] = sec
        out[prec] = ent
        if prec == "mixed" and name == "c5" and w.method.smoother == "FA":
            from paper_1603_02524_amd import learn
            if os.path.exists(learn.DEFAULT_PARAMS):
                params = torch.tensor(learn.load_params(), device="cuda")
                kept, rl, rf = S.apply_mlp(params, probe_iters=4)
                secl, entl = _solve_entry(S, rhs, x, w.tol, args.warmup, max(2, args.steps // 2))
                entl.update({"value": n / secl, "kept": kept, "probe_ratio_learned": rl, "probe_ratio_fixed": rf,
                             "time_per_dof_vs_fixed_mixed": secl / sec})
                out["learned_mixed"] = entl
                res["learned"] = secl
        S.close()
    out["mixed_time_per_dof_vs_fp64"] = res["mixed"] / res["fp64"]
    if "learned" in res:
        out["learned_mixed_time_per_dof_vs_fp64"] = res["learned"] / res["fp64"]
    return out


def _se_step_roofline(S, word, reps=20):
    """One top-level smoothing step of a continuous handle (residual apply, patch
    solves, overlap sum) against max(bytes / HBM peak, flops / FP64 peak): flops of
    the element-local apply 2 D N_P^(D+1) and of the patch solves 4 D n^(D+1)
    (n = N_P + 2 N_O) per element, bytes 3 words per unknown."""
    import torch
    L = S.num_levels - 1
    P, n_o, n = S.level_info(L)
    dim = S.grid.dim
    ne = S.grid.n_elem
    u = torch.rand(n, dtype=torch.float64, device="cuda")
    f = torch.rand(n, dtype=torch.float64, device="cuda")
    S.smooth(L, u, f, 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        S.smooth(L, u, f, 1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    npt = P + 1 + 2 * n_o
    flops = ne * (2.0 * dim * (P + 1) ** (dim + 1) + 4.0 * dim * npt ** (dim + 1))
    byts = 3.0 * word * n
    t_roof = max(byts / (HBM_PEAK_GBPS * 1e9), flops / (FP64_VALU_PEAK_TFLOPS * 1e12)) * 1e3
    return {"ms": ms, "roof_ms": t_roof, "frac": t_roof / ms, "flops": flops, "alg_bytes": byts}


def _se_entry(args):
    """The continuous spectral-element counterpart of EA_l (Sec. 4.3) on the 16^3 P = 8
    grid (FP64 and mixed) against DG EA_l (FP64) on the same grid, and the 2D
    workload of Fig. 6 ((256/P)^2 periodic elements, P = 16) in both discretisations."""
    import torch
    import synth
    from paper_1603_02524_amd import dgmg
    out = {}
    for key, ws in (("se_3d", (synth.se_poisson3d_p8(), synth.with_method(synth.c2_poisson3d_p8(), smoother="EA"))),
                    ("se_fig6_2d_p16", (synth.paper_fig6_2d(16, disc="se"), synth.paper_fig6_2d(16, disc="dg")))):
        ent = {}
        secs = {}
        for w, label in zip(ws, ("se", "dg_ea")):
            n = w.n_dof
            rhs_np = synth.rhs_uniform(w.seed if w.seed is not None else 0, n)
            if all(w.grid.periodic):
                rhs_np = rhs_np - rhs_np.mean()
            rhs = torch.tensor(rhs_np, dtype=torch.float64, device="cuda")
            x = torch.zeros(n, dtype=torch.float64, device="cuda")
            precs = ("fp64", "mixed") if label == "se" and key == "se_3d" else ("fp64",)
            for prec in precs:
                _log(f"{key}: {label} {prec}")
                S = dgmg.Solver(w.grid, synth.with_method(w, precision=prec).method, max_iter=200)
                if not args.no_autotune:
                    S.autotune()
                if label == "se" and prec == "fp64":
                    S.kernel_timing(True)
                sec, e = _solve_entry(S, rhs, x, w.tol, args.warmup, max(2, args.steps // 2))
                e.update({"workload": w.name, "n_dof": n, "value": n / sec})
                if label == "se" and prec == "fp64":
                    kt = S.kernel_time()
                    S.kernel_timing(False)
                    k_ms = kt["ms"] / max(kt["launches"], 1)
                    e["patch_solve"] = {"avg_ms": k_ms, "launches": kt["launches"],
                                        "achieved_TFLOPs": kt["flops"] / max(kt["launches"], 1) / (k_ms * 1e-3) / 1e12,
                                        "frac_fp64_peak": kt["flops"] / max(kt["launches"], 1) / (k_ms * 1e-3) / 1e12
                                        / FP64_VALU_PEAK_TFLOPS}
                    e["smoothing_step"] = _se_step_roofline(S, 8)
                ent[f"{label}_{prec}"] = e
                secs[f"{label}_{prec}"] = sec
                S.close()
        ent["se_time_vs_dg_ea_fp64"] = secs["se_fp64"] / secs["dg_ea_fp64"]
        ent["se_time_per_dof_vs_dg_ea_fp64"] = (secs["se_fp64"] / ent["se_fp64"]["n_dof"]) / (
            secs["dg_ea_fp64"] / ent["dg_ea_fp64"]["n_dof"])
        if "se_mixed" in secs:
            ent["se_mixed_time_vs_se_fp64"] = secs["se_mixed"] / secs["se_fp64"]
        out[key] = ent
    return out


def _batched_entry(args, small=False):
    """64 grids in one batched MGCG (FP32 V-cycle in FP64 PCG; work-list launches
    shared by the grids' smaller levels) against the same grids solved one after
    another, in mixed precision and in FP64.  small: 64 grids of 2^3..6^3
    elements at P in {4, 6, 8} (seed 40), where every level is small enough to
    share launches."""
    import numpy as np
    import torch
    import synth
    from paper_1603_02524_amd import dgmg
    ws = synth.c4_batched(seed=40, n_range=(2, 6), orders=(4, 6, 8)) if small else synth.c4_batched()
    B = dgmg.BatchSolver([(w.grid, w.method) for w in ws], max_iter=200)
    planned, kernels, grid_ops = B.plan_info()
    n = B.n_dof
    rhs = torch.tensor(np.concatenate([synth.rhs_uniform(w.seed, w.n_dof) for w in ws]), device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    if not args.no_autotune:
        B.autotune()
    steps = max(2, args.steps // 2)
    for _ in range(args.warmup):
        x.zero_()
        B.solve(rhs, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        st = B.solve(rhs, x)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    its = [s["iterations"] for s in st]
    out = {"workload": f"batched_{len(ws)}_{'small_' if small else ''}grids_3d_mixed", "grids": len(ws), "n_dof": n,
           "ms_per_step": sec * 1e3, "value": n / sec, "iterations_min_max": [min(its), max(its)],
           "converged": all(s["converged"] for s in st),
           "true_rel_residual_max": max(s["r_true"] / s["r0"] for s in st),
           "plan": {"work_lists": planned, "batched_launches_per_iteration": kernels,
                    "per_grid_ops_per_iteration": grid_ops}}
    B.close()
    for prec in ("mixed", "fp64"):
        _log(f"c4: the same grids one by one, {prec}")
        tot = 0.0
        for w, (a, b) in zip(ws, zip(B.offsets[:-1], B.offsets[1:])):
            S = dgmg.Solver(w.grid, synth.with_method(w, precision=prec).method, max_iter=200)
            if not args.no_autotune:
                S.autotune()
            xs = torch.zeros(b - a, dtype=torch.float64, device="cuda")
            r = rhs[a:b].contiguous()
            s1, _ = _solve_entry(S, r, xs, w.tol, 1, steps)
            tot += s1
            S.close()
        out[f"one_by_one_{prec}_ms"] = tot * 1e3
        out[f"batched_time_per_dof_vs_one_by_one_{prec}"] = sec / tot
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--quick", action="store_true", help="only the 16^3 workload (no 32^3, 8^3 P=32, batch lines)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=3)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run plain device copies of MB MiB (PMC calibration) and exit")
    ap.add_argument("--workload", choices=["c3", "c4", "c4_small", "c5", "se"], default=None,
                    help="only this extra entry (for profiling), printed as its own JSON line: c3, c5 (mixed "
                         "and FP64), c4 / c4_small (batched against one by one), se (continuous counterpart)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the solver "
              "runs on a single MI355X; multi-GPU sharding is a design note only)", file=sys.stderr)
        raise SystemExit(2)

    if args.copy_calibration:
        _copy_calibration(args.copy_calibration)
        return
    if args.workload:
        if args.workload in ("c3", "c5"):
            ent = _extra_workload(args.workload, args)
        elif args.workload in ("c4", "c4_small"):
            ent = _batched_entry(args, small=args.workload == "c4_small")
        else:
            ent = _se_entry(args)
        print(json.dumps({args.workload: ent}), flush=True)
        return

    import torch

    import synth
    from paper_1603_02524_amd import dgmg

    w = _workload("c2")
    g, m = w.grid, w.method
    _log(f"setup {w.name}")
    S = dgmg.Solver(g, m, max_iter=200)
    n = S.n_dof()
    rhs_np = synth.rhs_uniform(w.seed, n)
    rhs = torch.tensor(rhs_np, dtype=torch.float64, device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    tuning = {}
    if not args.no_autotune:
        # patch-solve block shapes per (level, sweep kind); bitwise-neutral, outside the timed region
        _log("autotuning patch-solve block shapes")
        tuning = S.autotune()
    _log("timing FP64 solves")
    sec, st, kt = _time_solves(S, rhs, x, w.tol, args.warmup, args.steps, timing=True)
    _log(f"fp64: {sec * 1e3:.2f} ms per solve, {st['iterations']} iterations")
    true_rel = st["r_true"] / st["r0"]
    if not (st["converged"] and true_rel <= w.tol):
        print(json.dumps({"error": "solve did not reach the tolerance", "stats": st}), file=sys.stderr)
        raise SystemExit(1)
    roof = _dominant_roofline(S, m, kt, 8)
    step = _smoothing_step_roofline(S, m, 8)
    # every smoothed level's step against its own roof (where the V-cycle's time goes)
    steps_by_level = [_smoothing_step_roofline(S, m, 8, level=l) for l in range(S.num_levels - 1, 0, -1)]

    out = {"metric": METRIC, "value": n / sec, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": w.name, "elements": list(g.n), "P": m.P, "n_dof": n,
                      "flux": m.flux, "smoother": f"{m.smoother}_l", "vcycle": "V(1,1)",
                      "precision": m.precision, "tol": w.tol, "seed": w.seed,
                      "iterations": st["iterations"], "true_rel_residual": true_rel,
                      "autotuned_waves": {f"l{l}k{k}": v[0] for (l, k), v in sorted(tuning.items())}},
           "roofline": roof, "smoothing_step": step, "smoothing_steps_by_level": steps_by_level}

    _log("timing mixed-precision solves")
    wm = synth.with_method(w, precision="mixed")
    Sm = dgmg.Solver(wm.grid, wm.method, max_iter=200)
    if not args.no_autotune:
        Sm.autotune()
    xm = torch.zeros(n, dtype=torch.float64, device="cuda")
    secm, entm = _solve_entry(Sm, rhs, xm, w.tol, args.warmup, args.steps)
    entm["value"] = n / secm
    entm["mixed_time_per_dof_vs_fp64"] = secm / sec
    out["mixed"] = entm
    Sm.close()

    if not args.quick:
        out["c3"] = _extra_workload("c3", args)
        out["c5"] = _extra_workload("c5", args)
        _log("c4: batched grids")
        out["c4"] = _batched_entry(args)
        _log("c4: small batched grids")
        out["c4_small"] = _batched_entry(args, small=True)
        out["spectral_element"] = _se_entry(args)

    if not args.no_cpu_baseline:
        _log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = _cpu_baseline(w, rhs_np, st["iterations"], args.cpu_samples)
    S.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
