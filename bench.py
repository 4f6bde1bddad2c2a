"""Benchmark of the MI355X implicit M1 multigrid solver.

Workload: the 2-D hot-wall problem, 1024 x 1024 cells on [0,1]^2, dt = 100 h/c.
Opacity is piecewise constant on 32x32 blocks with log10 sigma_a ~ U[-2,2] and
sigma_s ~ U[0,1]. The x = 0 side is a hot Dirichlet wall; the other sides are
reflective. The solver is plain FP64 and takes 10 implicit Euler steps, each
run to relative residual 1e-8.

One benchmark "step" solves the whole workload (all 10 implicit steps) from the
same initial state, already resident in HBM. The timed region covers
exactly --steps such solves, bracketed by device synchronisation. The reported
value is cell-updates/s = cells * implicit steps / wall time, in millions.

The same JSON line also carries:
  * roofline: the finest-level Jacobi sweep kernel, timed with HIP events on
    the solver's stream; 112 algorithmic bytes per cell;
  * cpu_baseline: the FP64 CPU oracle timed on the host cores over a bounded
    sample of V-cycles of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2208_14703_amd import binding, inputs  # noqa: E402

METRIC = "Mcell-updates/s + time to 1e-8 residual; batched solves/s with p50/p99 latency"
HBM_PEAK_GBS = 8000.0
SWEEP_BYTES_PER_CELL = 112  # v (E,Fx,Fy,T) 32 + b 32 + sigma 16 read, v' 32 written
SOLVER = dict(omega=0.8, levels=0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024, help="grid side (the workload is 1024)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cycles", type=int, default=8, help="oracle V-cycles in the CPU-baseline sample")
    ap.add_argument("--profile-only", action="store_true", help="short run for profilers: no roofline/cpu legs")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="fp64 (the workload's definition) or mixed (FP32 delta-form smoothing)")
    return ap.parse_args()


def sweep_timing(torch, plan, b, v, reps=40):
    """Average duration of the finest-level sweep kernel (HIP events on the plan's stream)."""
    out = torch.empty_like(v)
    for _ in range(3):
        plan.sweep(b, v)
    st = plan.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    src, dst = v.clone(), out
    for _ in range(reps):
        binding.lib().m1_sweep(plan.handle, binding.ctypes.byref(plan._st(b)), binding.ctypes.byref(plan._st(src)),
                               binding.ctypes.byref(plan._st(dst)))
        src, dst = dst, src
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def cpu_baseline(prob, v, sig, run, gpu_cycles_per_step, ncycles):
    import oracle
    o = oracle.Oracle(prob, sig)
    p = oracle.make_params(rtol=run["rtol"], max_cycles=ncycles, **SOLVER)
    t0 = time.perf_counter()
    _, info = o.step(v, 1, p)
    dt = time.perf_counter() - t0
    per_cycle = dt / max(info["cycles"], 1)
    projected = per_cycle * gpu_cycles_per_step * run["steps"]
    cells = prob["nx"] * prob["ny"]
    return {"value": cells * run["steps"] / projected / 1e6, "unit": "Mcell-updates/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{info['cycles']} V-cycles of time step 1 of the same workload in {dt:.1f} s "
                      f"({per_cycle:.2f} s/cycle), projected to the GPU's {gpu_cycles_per_step:.1f} cycles/step "
                      f"x {run['steps']} steps"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    torch.cuda.init()
    prob, v0, sig, run = inputs.hot_wall_2d(n=args.n)
    cells = prob["nx"] * prob["ny"]
    dev_sig = binding.to_device(sig)
    v_init = binding.to_device(v0)
    plan = binding.Plan(prob, dev_sig, dict(rtol=run["rtol"], max_cycles=20000, precision=args.precision, **SOLVER))
    v = torch.empty_like(v_init)

    def one_solve():
        v.copy_(v_init)
        return plan.step(v, run["steps"])

    for _ in range(args.warmup):
        info = one_solve()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(one_solve())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    value = cells * run["steps"] * args.steps / elapsed / 1e6
    cycles = infos[-1]["cycles"]
    status = infos[-1]["status"]
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mcell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f64+f32", "data": "synthetic",
        "config": {"workload": f"hot-wall 2-D {prob['nx']}x{prob['ny']}, {run['steps']} implicit steps, "
                               f"dt=100h/c, block opacity, {args.precision.upper()}, rtol {run['rtol']:g}",
                   "nx": prob["nx"], "ny": prob["ny"], "time_steps": run["steps"], "rtol": run["rtol"],
                   "precision": args.precision, "levels": infos[-1]["levels"], "omega": SOLVER["omega"]},
        "time_to_rtol_ms_per_time_step": round(ms_per_step / run["steps"], 3),
        "cycles_per_time_step": cycles / run["steps"], "solver_status": status,
        "final_rel_residual": infos[-1]["rel_residual"],
    }
    if not args.profile_only:
        b = v_init.clone()
        b[3] *= prob["c_v"]
        t_sweep = sweep_timing(torch, plan, b, v)
        achieved = SWEEP_BYTES_PER_CELL * cells / t_sweep / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                           "kernel": "k_relax<2> (finest-level Jacobi sweep)",
                           "avg_launch_us": round(t_sweep * 1e6, 2)}
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(prob, v0, sig, run, cycles / run["steps"], args.cpu_cycles)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
