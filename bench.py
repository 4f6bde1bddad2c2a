"""Benchmark of the MI355X implicit M1 multigrid solver.

Default line (the headline workload): the 2-D hot-wall problem.
- Grid: 1024 x 1024 cells on [0,1]^2, dt = 100 h/c.
- Opacity: piecewise constant on 32x32 blocks, log10 sigma_a ~ U[-2,2], sigma_s ~ U[0,1].
- Boundaries: a hot Dirichlet wall at x = 0, reflective elsewhere.
- Solver: plain FP64, 10 implicit Euler steps, each run to relative residual 1e-8, with the
  paper's smoothing counts (3 finest sweeps before and after, 3 coarse pseudo-time steps) and
  L_max = 6 levels (coarsest 32^2), the fastest depth of a measured L_max sweep (the solution
  does not depend on it; config.levels reports it).

One benchmark "step" solves the whole workload (all 10 implicit steps) from the same
initial state, already resident in HBM. The timed region covers exactly --steps such
solves, bracketed by device synchronisation. value = cells * implicit steps / wall
time, in millions (Mcell-updates/s).

The same JSON line also carries:
- roofline: the finest-level Jacobi sweep kernel of the cycle, the solve's dominant kernel:
  k_relax2_lds<rows> (two sweeps per launch, the first sweep's iterate kept in LDS), or with
  that launch shape off k_relax_lds<rows, false> (the LDS-staged sweep) or k_relax<2, false,
  true>. It is timed with HIP events on the solver's stream around m1_sweeps launches on a
  4096^2 FP64 plan (the inputs of the 4096^2 lognormal workload: a 1.9 GB working set, far
  beyond the 256 MB Infinity Cache, so the kernel streams from HBM), at 112 algorithmic bytes
  per cell and sweep (the state, right-hand side and opacities read once and the state written
  once per sweep): 224 per cell for the pair, whose own HBM traffic is about half of that,
  since the intermediate iterate stays on chip.
- roofline_kernels: the same measurement for the single staged sweep and for the finest-level
  residual fused with its restriction (k_residual_restrict, m1_residual_restrict: 96 bytes per
  fine cell), both at 4096^2.
- headline_grid_sweep: the pair on the 1024^2 hot wall itself; its working set stays in the
  Infinity Cache, so it gets its rate in bytes of sweep work per second and no HBM fraction.
- traffic: the kernel's FETCH_SIZE + WRITE_SIZE counter bytes per launch, scaled by the same
  counters on a plain copy of known size. They are read from the counter summaries under
  profiles/, and are null when the kernel sources have changed since they were taken.
- c1 / c3: the 1-D Gaussian (N = 256, rtol 1e-10) and the 4096^2 lognormal single solve in
  mixed precision (rtol 1e-8; with the FP64 solve of the same step beside it).
- three_d: the hot wall in 3-D (256^3 cells, 10 implicit steps to 1e-8, FP64) through the 3-D plans, and
  the roofline of their finest-level sweep kernel at 136 algorithmic bytes per cell.
- cpu_baseline: the FP64 CPU oracle on the host cores, over a bounded sample of V-cycles
  of the same workload.
- batched: 256 independent problems of uneven size, seeded 1000+k, side log-uniform in
  {64..512}, one implicit step each to 1e-8. They are solved by the batching engine (one
  launch per level operation) in FP64 and in mixed precision and, for comparison, one by
  one with the plain FP64 path. It reports solves/s and per-problem latency p50/p99.
- serving: a short Poisson request stream through the engine's serving loop (sides 64..2048,
  1..20 steps per request, contrast 10^0..10^6). It reports solves/s and request latency
  p50/p99.

Other modes:
- --workload lognormal: the 4096^2 single solve (mixed or fp64).
- --workload serve: the serving sweep over arrival rates.
- --workload hotwall3d: the 256^3 3-D hot wall (10 steps) and its sweep kernel.
- --profile kernels: only the 4096^2 kernel launches of the roofline entries and a copy kernel
  of known size, for PMC counter runs (kernels3d: the 256^3 3-D sweep and the copy).
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
from paper_2208_14703_amd.profsum import sources_hash  # noqa: E402

METRIC = "Mcell-updates/s + time to 1e-8 residual; batched solves/s with p50/p99 latency"
HBM_PEAK_GBS = 8000.0
SWEEP_BYTES_PER_CELL = 112  # v (E,Fx,Fy,T) 32 + b 32 + sigma 16 read, v' 32 written
RESID_BYTES_PER_CELL = 96   # u 32 + b 32 + sigma 16 read per fine cell; R(u) and R(r) (2 x 32 B) per 4 fine cells
KERNEL_N = 4096             # side of the HBM-resident grid of the kernel measurements
SOLVER = dict(omega=0.8, levels=0)
# Levels (L_max, the paper's own tuning knob: its timing table is a sweep of it) of the two single-problem
# workloads: the fastest depth of a measured sweep. Solutions do not depend on it; cycle counts do.
# Hot wall 1024^2, the pseudo-time step carried from step to step: 5 levels (coarsest 64^2) 112 ms per solve
# (384 cycles), against 116 (6), 126 (7), 133 (8), 139 (9, to side 4) and 156 (4).  Restarted at every step
# instead, 6 levels were fastest (196 ms, 611 cycles; 5 levels took 2661 cycles).  Lognormal 4096^2: 7 levels
# (coarsest 64^2).
WORKLOAD_LEVELS = {"hotwall": 5, "lognormal": 7}
RESET_LEVELS = {"hotwall": 6, "lognormal": 7}  # the fastest depths with the step restarted at every time step
FCYCLE_LEVELS = {"hotwall": 4, "lognormal": 6}  # the fastest depths of F-cycles (a sweep over 4..8 levels)


def sweeps_per_launch():
    """Sweeps per launch of the finest-level sweep kernel the cycle runs (2 with the fused pair on)."""
    return 2 if binding.tune_get("pair_rows") > 0 else 1


def sweep_kernel():
    """Name of the finest-level sweep kernel that m1_sweeps(sweeps_per_launch()) launches under the current
    settings: the fused pair, else the LDS-staged single sweep, else the one-cell sweep."""
    pair, rows = binding.tune_get("pair_rows"), binding.tune_get("sweep_rows")
    if pair > 0:
        return f"k_relax2_lds<{pair}>"
    return f"k_relax_lds<{rows}, false>" if rows > 0 else "k_relax<2, false, true>"


def sweep_tag(pair):
    rows = binding.tune_get("sweep_rows")
    return f"k_relax2_lds{pair}" if pair > 0 else (f"k_relax_lds{rows}" if rows > 0 else "k_relax")


def traffic_file(tag, workload):
    return os.path.join(ROOT, "profiles", f"{tag}_{workload}_traffic.txt")


COPY_ELEMS = 1 << 27  # 1 GiB of float64 per copy launch


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="hotwall", choices=["hotwall", "lognormal", "batch", "serve", "hotwall3d"])
    ap.add_argument("--n", type=int, default=0, help="grid side (default: the workload's own)")
    ap.add_argument("--levels", type=int, default=-1,
                    help="L_max of the hot-wall/lognormal solve (default: the workload's measured fastest; 0: to side 4)")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default: fp64 for hotwall, mixed for lognormal")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cycles", type=int, default=60, help="oracle V-cycles in the CPU-baseline sample")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other dtau reading, C1, C3, 3-D, batched and serving legs")
    ap.add_argument("--batch", type=int, default=256, help="problems in the batched leg")
    ap.add_argument("--requests", type=int, default=48, help="requests per rate in the serving leg")
    ap.add_argument("--rates", default="50", help="comma-separated arrival rates (1/s) for serving")
    ap.add_argument("--arena-gb", type=float, default=64.0, help="engine HBM budget for serving")
    ap.add_argument("--serve-precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--profile", default="none", choices=["none", "kernels", "kernels3d"],
                    help="kernels: only the 4096^2 kernel launches and a copy of known size (for counter runs); "
                         "kernels3d: the same for the 256^3 3-D sweep")
    ap.add_argument("--reps", type=int, default=40, help="sweep launches timed for the roofline")
    ap.add_argument("--stream", default="own", choices=["own", "default"],
                    help="own: run on a created stream (default priority); default: the null stream")
    return ap.parse_args()


def read_traffic(tag: str, workload: str, kernel: str, cells: int):
    """Counter bytes per launch of `kernel` from the committed summary, if the kernel sources are unchanged."""
    try:
        kv = dict(line.split(":", 1) for line in open(traffic_file(tag, workload))
                  if ":" in line and not line.startswith(" "))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if (kv.get("sources_sha256") != sources_hash() or int(kv.get("cells", -1)) != cells
            or kv.get("kernel") != kernel):
        return None
    return float(kv["traffic_bytes_per_launch"])


def time_launches(torch, stream, launch, reps):
    """Average time of one launch: HIP events on `stream` (the plan's) around `reps` back-to-back launches."""
    for _ in range(3):
        launch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        launch()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def sweep_launcher(plan, b, v, n):
    """m1_sweeps(n) between two state buffers (one launch each for n = 1, or n = 2 with the pair on)."""
    L = binding.lib()
    bufs = [v.clone(), v.clone()]
    k = [0]

    def launch():
        src, dst = bufs[k[0]], bufs[1 - k[0]]
        binding._check(L.m1_sweeps(plan.handle, binding.ctypes.byref(plan._st(b)),
                                   binding.ctypes.byref(plan._st(src)), binding.ctypes.byref(plan._st(dst)), n),
                       "m1_sweeps")
        k[0] ^= 1
    return launch


def residual_launcher(plan, b, u):
    """m1_residual_restrict on the finest level: one launch of the fused residual and restriction."""
    L = binding.lib()
    vc, rc = plan.new_state(1), plan.new_state(1)
    args = [binding.ctypes.byref(plan._st(x)) for x in (u, b, vc, rc)]

    def launch():
        binding._check(L.m1_residual_restrict(plan.handle, 0, *args), "m1_residual_restrict")
    return launch


def roofline_entry(kernel, what, bytes_per_launch, t, traffic, grid, residency):
    achieved = bytes_per_launch / t / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": f"{kernel} ({what})",
            "grid": grid, "residency": residency, "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_us": round(t * 1e6, 2)}


def kernel_leg(torch, reps):
    """The cycle's finest-level kernels timed on a 4096^2 FP64 plan (HBM-resident working set)."""
    prob, v0, sig, _ = inputs.lognormal_2d(n=KERNEL_N)
    cells = prob["nx"] * prob["ny"]
    plan = binding.Plan(prob, binding.to_device(sig), dict(precision="fp64", **SOLVER))
    v = binding.to_device(v0)
    b = v.clone()
    b[3] *= prob["c_v"]
    grid = f"{prob['nx']}x{prob['ny']}"
    res = "HBM (lognormal 4096^2 inputs; 1.9 GB working set, beyond the 256 MB Infinity Cache)"
    out = []
    pair = binding.tune_get("pair_rows")
    if pair > 0:
        t = time_launches(torch, plan.stream, sweep_launcher(plan, b, v, 2), reps)
        k = sweep_kernel()
        out.append(roofline_entry(k, "finest-level FP64 Jacobi sweeps, 2 per launch", 2 * SWEEP_BYTES_PER_CELL * cells,
                                  t, read_traffic(sweep_tag(pair), "lognormal4096", k, cells), grid, res))
    binding.tune_set("pair_rows", 0)
    try:
        t = time_launches(torch, plan.stream, sweep_launcher(plan, b, v, 1), reps)
        k = sweep_kernel()
        out.append(roofline_entry(k, "finest-level FP64 Jacobi sweep", SWEEP_BYTES_PER_CELL * cells, t,
                                  read_traffic(sweep_tag(0), "lognormal4096", k, cells), grid, res))
    finally:
        binding.tune_set("pair_rows", pair)
    if binding.tune_get("residual_restrict"):
        t = time_launches(torch, plan.stream, residual_launcher(plan, b, v), reps)
        k = "k_residual_restrict"
        out.append(roofline_entry(k, "finest-level FP64 residual restricted as it is formed", RESID_BYTES_PER_CELL *
                                  cells, t, read_traffic(k, "lognormal4096", k, cells), grid, res))
    del plan
    torch.cuda.empty_cache()
    return out


def copy_timing(torch, reps=10):
    """A plain copy of known size (torch.neg: 8 B read + 8 B written per element)."""
    x = torch.ones(COPY_ELEMS, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(x, out=y)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    return {"bytes": 16 * COPY_ELEMS, "avg_launch_us": round(t * 1e6, 2), "GB_per_s": round(16 * COPY_ELEMS / t / 1e9, 1)}


def cpu_baseline(prob, v, sig, run, gpu_cycles_per_step, ncycles, levels, c1=None):
    import oracle
    o = oracle.Oracle(prob, sig)
    p = oracle.make_params(rtol=run["rtol"], max_cycles=ncycles, **dict(SOLVER, levels=levels))
    t0 = time.perf_counter()
    _, info = o.step(v, 1, p)
    dt = time.perf_counter() - t0
    per_cycle = dt / max(info["cycles"], 1)
    projected = per_cycle * gpu_cycles_per_step * run["steps"]
    cells = prob["nx"] * prob["ny"]
    out = {"value": round(cells * run["steps"] / projected / 1e6, 4), "unit": "Mcell-updates/s",
           "cores": oracle.threads(), "kind": "oracle",
           "sample": f"{info['cycles']} V-cycles of time step 1 of the same workload in {dt:.1f} s "
                     f"({per_cycle:.3f} s/cycle), projected to the GPU's {gpu_cycles_per_step:.1f} cycles/step "
                     f"x {run['steps']} steps (same algorithm, same cycle count)"}
    if c1 is not None:
        out["c1"] = c1_oracle(oracle, c1)
    return out


def c1_oracle(oracle, c1):
    """The 1-D Gaussian solved whole by the oracle on one thread (its own time to rtol), and the GPU result's
    error against the oracle's converged solution (rtol 1e-13)."""
    prob, v, sig, run = inputs.gaussian_1d(n=256)
    o = oracle.Oracle(prob, sig)
    threads = oracle.threads()
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        _, info = o.step(v, run["steps"], oracle.make_params(rtol=run["rtol"], max_cycles=20000, **SOLVER))
        dt = time.perf_counter() - t0
        ref, _ = o.step(v, run["steps"], oracle.make_params(rtol=1e-13, max_cycles=20000, **SOLVER))
    finally:
        oracle.set_threads(threads)
    got = c1.pop("result")
    err = max(np.abs(got[0] - ref[0]).max() / np.abs(ref[0]).max(),
              np.abs(got[1:3] - ref[1:3]).max() / (prob["c"] * np.abs(ref[0]).max()),
              np.abs(got[3] - ref[3]).max() / np.abs(ref[3]).max())
    return {"value": round(prob["nx"] * run["steps"] / dt / 1e6, 5), "unit": "Mcell-updates/s", "cores": 1,
            "kind": "oracle", "time_to_rtol_ms": round(dt * 1e3, 3), "cycles": info["cycles"],
            "sample": "the whole 1-D Gaussian solve (N = 256, rtol 1e-10) on one thread",
            "gpu_error_vs_oracle": float(err)}


def pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def state_rel(a, b, c=1.0):
    """max(|dE|/max|E|, |dF|/(c max|E|), |dT|/max|T|): the parity metric of the tests."""
    a, b = a.double(), b.double()
    sE, sT = b[0].abs().max(), b[3].abs().max()
    return max(float((a[0] - b[0]).abs().max() / sE), float((a[1:3] - b[1:3]).abs().max() / (c * sE)),
               float((a[3] - b[3]).abs().max() / sT))


def timed_solves(torch, plan, v_init, steps, reps):
    """Median wall time of `reps` whole solves (state reset from v_init, synchronised around each)."""
    v = torch.empty_like(v_init)
    times, info = [], None
    for k in range(reps + 1):
        v.copy_(v_init)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = plan.step(v, steps)
        torch.cuda.synchronize()
        if k > 0:  # the first is a warm-up
            times.append(time.perf_counter() - t0)
    return float(np.median(times)), info, v


def c1_leg(torch):
    """The 1-D Gaussian workload (N = 256, one step to rtol 1e-10, FP64)."""
    prob, v0, sig, run = inputs.gaussian_1d(n=256)
    plan = binding.Plan(prob, binding.to_device(sig), dict(rtol=run["rtol"], max_cycles=20000, **SOLVER))
    t, info, v = timed_solves(torch, plan, binding.to_device(v0), run["steps"], 5)
    return {"workload": "1-D Gaussian, N=256 on [0,1], periodic, sigma_a=1, dt=50h/c, FP64, 1 step to rtol 1e-10",
            "Mcell_updates_per_s": round(prob["nx"] * run["steps"] / t / 1e6, 4),
            "time_to_rtol_ms": round(t * 1e3, 3), "cycles": info["cycles"], "levels": info["levels"],
            "status": info["status"], "result": v.cpu().numpy()}


def c3_leg(torch):
    """The 4096^2 lognormal single solve in mixed precision, with the FP64 solve of the same step beside it."""
    prob, v0, sig, run = inputs.lognormal_2d(n=4096)
    cells = prob["nx"] * prob["ny"]
    sd, vd = binding.to_device(sig), binding.to_device(v0)
    out = {"workload": "lognormal 2-D 4096x4096, periodic, |F|=0.9cE, block opacity seed 2, 1 step, dt=100h/c, "
                       "rtol 1e-8"}
    res = {}
    for prec, reps in (("mixed", 3), ("fp64", 1)):
        plan = binding.Plan(prob, sd, dict(rtol=run["rtol"], max_cycles=20000, precision=prec,
                                           **dict(SOLVER, levels=WORKLOAD_LEVELS["lognormal"])))
        t, info, v = timed_solves(torch, plan, vd, run["steps"], reps)
        res[prec] = v
        out[prec] = {"Mcell_updates_per_s": round(cells * run["steps"] / t / 1e6, 2), "time_to_rtol_ms": round(t * 1e3, 2),
                     "cycles": info["cycles"], "levels": info["levels"], "status": info["status"],
                     "rel_residual": info["rel_residual"]}
        del plan
    # W-cycles (Sect. 6.3's alternative shape) in mixed precision, at their fastest depth
    plan = binding.Plan(prob, sd, dict(rtol=run["rtol"], max_cycles=20000, precision="mixed",
                                       **dict(SOLVER, levels=5, cycle="W")))
    t, info, _ = timed_solves(torch, plan, vd, run["steps"], 3)
    del plan
    out["mixed_w_cycles"] = {"levels": 5, "Mcell_updates_per_s": round(cells * run["steps"] / t / 1e6, 2),
                             "time_to_rtol_ms": round(t * 1e3, 2), "cycles": info["cycles"], "status": info["status"]}
    out["mixed_speedup_vs_fp64"] = round(out["fp64"]["time_to_rtol_ms"] / out["mixed"]["time_to_rtol_ms"], 3)
    out["max_rel_diff_mixed_vs_fp64"] = state_rel(res["mixed"], res["fp64"], prob["c"])
    del res
    torch.cuda.empty_cache()
    return out


SWEEP3_BYTES_PER_CELL = 136  # 3-D sweep: u (E, F, T) 40 + b 40 + sigma 16 read, u' 40 written


def three_d_leg(torch, reps):
    """The hot wall in 3-D (256^3 cells, 10 implicit steps to 1e-8, FP64, the deepest hierarchy), one timed
    solve after a one-step warm-up, and the finest-level sweep kernel (m1_sweep3) timed with HIP events."""
    prob, v0, sig, run = inputs.hot_wall_3d(n=256)
    cells = prob["nx"] * prob["ny"] * prob["nz"]
    sd, vd = binding.to_device(sig), binding.to_device(v0)
    plan = binding.Plan3(prob, sd, dict(rtol=run["rtol"], max_cycles=20000, **SOLVER))
    v = vd.clone()
    plan.step(v, 1)
    v.copy_(vd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = plan.step(v, run["steps"])
    torch.cuda.synchronize()
    t = time.perf_counter() - t0

    def variant(extra):
        """The same solve with other solver choices (a fresh plan, timed after it is made)."""
        vplan = binding.Plan3(prob, sd, dict(rtol=run["rtol"], max_cycles=20000, **dict(SOLVER, **extra)))
        v.copy_(vd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        i = vplan.step(v, run["steps"])
        torch.cuda.synchronize()
        tv = time.perf_counter() - t0
        del vplan
        return {"time_to_rtol_ms": round(tv * 1e3, 1), "cycles": i["cycles"], "levels": i["levels"],
                "status": i["status"]}

    out = {"workload": "hot wall 3-D 256^3, 10 implicit steps, dt=100h/c, 8^3 opacity blocks, FP64, rtol 1e-8",
           "Mcell_updates_per_s": round(cells * run["steps"] / t / 1e6, 2), "time_to_rtol_ms": round(t * 1e3, 1),
           "cycles": info["cycles"], "levels": info["levels"], "status": info["status"],
           "dtau_reset": variant(dict(dtau_carry=0)), "w_cycles": variant(dict(cycle="W", levels=4)),
           "f_cycles": variant(dict(cycle="F", levels=5)),
           "roofline": sweep3_entry(torch, plan, prob, vd, reps)}
    del plan, v
    torch.cuda.empty_cache()
    return out


def sweep3_entry(torch, plan, prob, vd, reps):
    """The 3-D finest-level sweep (m1_sweep3) timed with HIP events on the plan's stream."""
    L = binding.lib()
    cells = prob["nx"] * prob["ny"] * prob["nz"]
    b = vd.clone()
    b[4] *= prob["c_v"]
    bufs, k = [vd.clone(), vd.clone()], [0]

    def launch():
        binding._check(L.m1_sweep3(plan.handle, binding.ctypes.byref(plan._st(b)),
                                   binding.ctypes.byref(plan._st(bufs[k[0]])),
                                   binding.ctypes.byref(plan._st(bufs[1 - k[0]]))), "m1_sweep3")
        k[0] ^= 1
    tk = time_launches(torch, plan.stream, launch, reps)
    kname = "k3_staged<1>" if binding.tune_get("stage3") >= 1 else "k3_relax<false>"
    tag = "k3_staged1" if binding.tune_get("stage3") >= 1 else "k3_relax"
    return roofline_entry(kname, "finest-level FP64 Jacobi sweep, 3-D", SWEEP3_BYTES_PER_CELL * cells, tk,
                          read_traffic(tag, "hotwall3d256", kname, cells), "256x256x256", "HBM (2.3 GB working set)")


def kernel3_leg(torch, reps):
    """Only the 3-D sweep kernel on the 256^3 hot wall's plan (for counter runs)."""
    prob, v0, sig, run = inputs.hot_wall_3d(n=256)
    plan = binding.Plan3(prob, binding.to_device(sig), dict(rtol=run["rtol"], max_cycles=20000, **SOLVER))
    entry = sweep3_entry(torch, plan, prob, binding.to_device(v0), reps)
    del plan
    torch.cuda.empty_cache()
    return entry


# ---------------------------------------------------------------------------
# batched leg: many problems of uneven size
# ---------------------------------------------------------------------------
def batch_leg(torch, nprob: int):
    base = dict(rtol=1e-8, max_cycles=20000, **SOLVER)
    cases = [inputs.batch_problem(k) for k in range(nprob)]
    sig_d = [binding.to_device(c[2]) for c in cases]
    v0_d = [binding.to_device(c[1]) for c in cases]
    cells = sum(c[0]["nx"] * c[0]["ny"] for c in cases)

    # the plain FP64 path, one problem after another (plans made before the clock starts)
    plans = [binding.Plan(c[0], s, base) for c, s in zip(cases, sig_d)]
    ws = [v.clone() for v in v0_d]
    plans[0].step(v0_d[0].clone(), 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_info = [p.step(w, 1) for p, w in zip(plans, ws)]
    torch.cuda.synchronize()
    seq_wall = time.perf_counter() - t0
    del plans
    torch.cuda.empty_cache()
    out = {"workload": f"{nprob} problems seeded 1000+k, side log-uniform in 64..512 ({cells / 1e6:.1f} M cells), "
                       f"1 implicit step each to 1e-8",
           "plain_fp64_one_by_one": {"solves_per_s": round(nprob / seq_wall, 2), "wall_s": round(seq_wall, 4),
                                     "all_converged": all(i["status"] == 0 for i in seq_info)}}

    for prec in ("fp64", "mixed"):
        params = dict(base, precision=prec)
        need = sum(binding.Engine.request_bytes(c[0], params) for c in cases)
        E = binding.Engine(need + (256 << 20), params, max_requests=nprob)

        def engine_run(idx):
            vs = [v0_d[i].clone() for i in idx]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tk = [E.submit(cases[i][0], sig_d[i], v, 1) for i, v in zip(idx, vs)]
            pending = set(tk)
            while pending:
                E.run(4)
                pending = {t for t in pending if E.poll(t) is None}
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            infos = [E.poll(t) for t in tk]
            lat = [E.times(t)[2] - E.times(t)[0] for t in tk]
            for t in tk:
                E.release(t)
            return vs, infos, lat, wall

        engine_run(list(range(min(8, nprob))))  # warm-up (module load, first launches)
        vs, infos, lat, wall = engine_run(list(range(nprob)))
        rel = max(state_rel(a, b, c[0]["c"]) for a, b, c in zip(vs, ws, cases))
        res = {"solves_per_s": round(nprob / wall, 2), "wall_s": round(wall, 4),
               "latency_p50_ms": round(pct(lat, 50) * 1e3, 2), "latency_p99_ms": round(pct(lat, 99) * 1e3, 2),
               "Mcell_updates_per_s": round(cells / wall / 1e6, 2),
               "speedup_vs_plain_fp64": round(seq_wall / wall, 3),
               "max_rel_diff_vs_plain_fp64": rel,
               "all_converged": all(i["status"] == 0 for i in infos),
               "cycles_mean": round(float(np.mean([i["cycles"] for i in infos])), 2)}
        if prec == "fp64":
            res["bitwise_equal_to_plain"] = all(torch.equal(a, b) for a, b in zip(vs, ws))
            res["cycle_count_mismatches"] = sum(i["cycles"] != j["cycles"] for i, j in zip(infos, seq_info))
        out[prec] = res
        del E, vs
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# serving leg: a Poisson request stream through the serving loop
# ---------------------------------------------------------------------------
def serve_leg(torch, nreq: int, rate: float, arena_bytes: int, precision: str = "mixed", compare_plain: bool = True,
              seed: int = 7):
    params = dict(rtol=1e-8, max_cycles=20000, precision=precision, **SOLVER)
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for k in range(nreq):
        reqs.append(inputs.serve_request(rng))
        if nreq >= 200 and (k + 1) % 100 == 0:
            print(f"[serve] {k + 1} of {nreq} requests generated", file=sys.stderr, flush=True)
    arr = np.cumsum(np.random.Generator(np.random.PCG64(seed + 1)).exponential(1.0 / rate, nreq))
    sig_d = [binding.to_device(r[2]) for r in reqs]
    v_d = [binding.to_device(r[1]) for r in reqs]
    E = binding.Engine(arena_bytes, params, max_requests=1024)
    # warm-up request (not counted)
    w = inputs.batch_problem(0)
    E.wait(E.submit(w[0], binding.to_device(w[2]), binding.to_device(w[1]), 1))
    torch.cuda.synchronize()
    E.serve_start(4)
    t0 = time.perf_counter()
    tickets = []
    peak = {"pool_in_use": 0, "resident": 0, "pending": 0}
    for i, r in enumerate(reqs):
        d = t0 + arr[i] - time.perf_counter()
        if d > 0:
            time.sleep(d)
        tickets.append(E.submit(r[0], sig_d[i], v_d[i], r[3]["steps"]))
        if i % 8 == 7:  # the pool's use and the queue, sampled as requests arrive
            m = E.memory()
            peak = {k: max(peak[k], m[k]) for k in peak}
            pool_bytes = m["pool_bytes"]
        if nreq >= 200 and (i + 1) % 100 == 0:
            print(f"[serve] rate {rate:g}/s: {i + 1} of {nreq} requests submitted", file=sys.stderr, flush=True)
    infos = [E.wait(t) for t in tickets]
    E.serve_stop()
    tm = [E.times(t) for t in tickets]
    lat = [d - s for s, _, d in tm]
    span = max(d for _, _, d in tm) - min(s for s, _, _ in tm)
    solves = sum(r[3]["steps"] for r in reqs)
    cell_steps = sum(r[0]["nx"] * r[0]["ny"] * r[3]["steps"] for r in reqs)
    # overlap: requests admitted while another request was still running
    adm = sorted((a, d) for _, a, d in tm)
    overlapped = sum(1 for k in range(1, len(adm)) if adm[k][0] < max(d for _, d in adm[:k]))
    ok = all(i["status"] == 0 for i in infos)
    del E
    plain = None
    if compare_plain:
        # the same requests (the first PLAIN_MAX of them), one after another, each on a plain FP64 plan (plans
        # made in the timed region, as a server without the engine would have to)
        base = dict(rtol=1e-8, max_cycles=20000, **SOLVER)
        sub = reqs[:PLAIN_MAX]
        vs = [binding.to_device(r[1]) for r in sub]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r, sd, vd in zip(sub, sig_d, vs):
            binding.Plan(r[0], sd, base).step(vd, r[3]["steps"])
        torch.cuda.synchronize()
        pw = time.perf_counter() - t0
        rel = max(state_rel(a, b, r[0]["c"]) for a, b, r in zip(v_d, vs, sub))
        plain = {"requests": len(sub), "solves_per_s": round(sum(r[3]["steps"] for r in sub) / pw, 2),
                 "wall_s": round(pw, 2), "max_rel_diff_served_vs_plain": rel}
        del vs
    out = {"precision": precision, "rate_per_s": rate, "requests": nreq, "solves": solves,
           "solves_per_s": round(solves / span, 2),
           "requests_per_s": round(nreq / span, 3), "Mcell_updates_per_s": round(cell_steps / span / 1e6, 2),
           "latency_p50_ms": round(pct(lat, 50) * 1e3, 1), "latency_p99_ms": round(pct(lat, 99) * 1e3, 1),
           "admitted_while_others_ran": overlapped, "all_converged": bool(ok), "wall_s": round(span, 2),
           "hbm_pool_peak_gb": round(peak["pool_in_use"] / 2 ** 30, 2),
           "hbm_pool_gb": round(pool_bytes / 2 ** 30, 2) if nreq >= 8 else None,
           "peak_resident": peak["resident"], "peak_waiting": peak["pending"],
           "plain_fp64_one_request_at_a_time": plain}
    if nreq >= 200:
        print("[serve] " + json.dumps(out), file=sys.stderr, flush=True)
    return out


PLAIN_MAX = 200  # requests of the serving stream re-solved one at a time on plain FP64 plans for comparison
SERVE_DESC = ("Poisson stream, side log-uniform in 64..2048, contrast 10^U[0,6], 1..20 steps per request to 1e-8, "
              "state resident in HBM across steps, continuous batching under an HBM budget")


# ---------------------------------------------------------------------------
def fcycle_leg(torch, out, args, prob, dev_sig, v_init, run, precision, cells):
    """The same solve with F-cycles (Sect. 6.3's alternative shape) at their fastest depth, FP64."""
    if precision != "fp64":
        return
    levels = FCYCLE_LEVELS[args.workload]
    plan = binding.Plan(prob, dev_sig, dict(rtol=run["rtol"], max_cycles=20000, precision=precision,
                                            **dict(SOLVER, levels=levels, cycle="F")))
    t, info, _ = timed_solves(torch, plan, v_init, run["steps"], 2)
    del plan
    out["f_cycles"] = {"what": f"F-cycles, {levels} levels, the rest as the headline solve",
                       "value": round(cells * run["steps"] / t / 1e6, 3), "ms_per_step": round(t * 1e3, 3),
                       "cycles_per_time_step": info["cycles"] / run["steps"], "solver_status": info["status"]}


def reset_leg(torch, out, args, prob, dev_sig, v_init, run, precision, cells):
    """The whole solve with the pseudo-time step restarted at 1e-3 in every time step (dtau_carry=0), at that
    reading's own fastest depth."""
    rlevels = RESET_LEVELS[args.workload] if args.levels < 0 else args.levels
    rplan = binding.Plan(prob, dev_sig, dict(rtol=run["rtol"], max_cycles=20000, precision=precision,
                                             **dict(SOLVER, levels=rlevels, dtau_carry=0)))
    t_reset, i_reset, _ = timed_solves(torch, rplan, v_init, run["steps"], 2)
    del rplan
    out["dtau_reset"] = {"what": "the pseudo-time step restarted at 1e-3 in every time step (dtau_carry=0), "
                                 f"{rlevels} levels",
                         "value": round(cells * run["steps"] / t_reset / 1e6, 3),
                         "ms_per_step": round(t_reset * 1e3, 3),
                         "cycles_per_time_step": i_reset["cycles"] / run["steps"], "solver_status": i_reset["status"]}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 (sharding across GPUs is not implemented)"}))
        sys.exit(2)
    import torch
    torch.cuda.init()
    if args.stream == "own":
        # a created stream: launches on the legacy null stream carry extra per-launch overhead
        torch.cuda.set_stream(torch.cuda.Stream())

    if args.workload == "serve":
        legs = [serve_leg(torch, args.requests, float(r), int(args.arena_gb * (1 << 30)), args.serve_precision,
                          compare_plain=(k == 0))
                for k, r in enumerate(args.rates.split(","))]
        best = max(legs, key=lambda x: x["solves_per_s"])
        print(json.dumps({"metric": METRIC, "value": best["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
                          "steps": 1, "warmup": 1, "ms_per_step": round(best["wall_s"] * 1e3, 1),
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                          "dtype": "f64" if args.serve_precision == "fp64" else "f64+f32",
                          "data": "synthetic", "config": {"workload": SERVE_DESC, "arena_gb": args.arena_gb},
                          "rates": legs}), flush=True)
        return

    if args.workload == "hotwall3d":
        leg = three_d_leg(torch, args.reps)
        print(json.dumps({"metric": METRIC, "value": leg["Mcell_updates_per_s"], "unit": "Mcell-updates/s",
                          "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": leg["time_to_rtol_ms"],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "config": {"workload": leg["workload"]}, "roofline": leg["roofline"],
                          "three_d": leg}), flush=True)
        return

    if args.workload == "batch":
        leg = batch_leg(torch, args.batch)
        best = leg["mixed"]
        print(json.dumps({"metric": METRIC, "value": best["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
                          "steps": 1, "warmup": 1, "ms_per_step": round(best["wall_s"] * 1e3, 2),
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
                          "data": "synthetic", "config": {"workload": leg["workload"]}, "batched": leg}), flush=True)
        return

    if args.workload == "lognormal":
        prob, v0, sig, run = inputs.lognormal_2d(n=args.n or 4096)
        precision = args.precision or "mixed"
        desc = (f"lognormal 2-D {prob['nx']}x{prob['ny']}, periodic, |F|=0.9cE, block opacity seed 2, "
                f"1 implicit step, dt=100h/c, {precision}, rtol 1e-8")
    else:
        prob, v0, sig, run = inputs.hot_wall_2d(n=args.n or 1024)
        precision = args.precision or "fp64"
        desc = (f"hot-wall 2-D {prob['nx']}x{prob['ny']}, {run['steps']} implicit steps, dt=100h/c, "
                f"block opacity, {precision.upper()}, rtol {run['rtol']:g}")
    cells = prob["nx"] * prob["ny"]
    dev_sig = binding.to_device(sig)
    v_init = binding.to_device(v0)
    levels = WORKLOAD_LEVELS[args.workload] if args.levels < 0 else args.levels
    plan = binding.Plan(prob, dev_sig, dict(rtol=run["rtol"], max_cycles=20000, precision=precision,
                                            **dict(SOLVER, levels=levels)))
    v = torch.empty_like(v_init)
    b = v_init.clone()
    b[3] *= prob["c_v"]

    if args.profile == "kernels3d":
        del plan
        torch.cuda.empty_cache()
        entry = kernel3_leg(torch, args.reps)
        print(json.dumps({"profile": "kernels3d", "cells": 256 ** 3, "kernels": [entry], "copy": copy_timing(torch)}),
              flush=True)
        return

    if args.profile == "kernels":
        del plan
        torch.cuda.empty_cache()
        entries = kernel_leg(torch, args.reps)
        print(json.dumps({"profile": "kernels", "cells": KERNEL_N * KERNEL_N, "kernels": entries,
                          "copy": copy_timing(torch)}), flush=True)
        return

    def one_solve():
        v.copy_(v_init)
        return plan.step(v, run["steps"])

    for _ in range(args.warmup):
        one_solve()
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
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mcell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if precision == "fp64" else "f64+f32", "data": "synthetic",
        "config": {"workload": desc, "nx": prob["nx"], "ny": prob["ny"], "time_steps": run["steps"],
                   "rtol": run["rtol"], "precision": precision, "levels": infos[-1]["levels"],
                   "omega": SOLVER["omega"]},
        "time_to_rtol_ms_per_time_step": round(ms_per_step / run["steps"], 3),
        "cycles_per_time_step": cycles / run["steps"], "solver_status": infos[-1]["status"],
        "final_rel_residual": infos[-1]["rel_residual"],
        "launch_shapes": {k: binding.tune_get(k) for k in binding.TUNE_ENV},
    }
    # the other reading of the pseudo-time step across time steps: restarted at 1e-3 in every time step
    if not args.no_extras:
        reset_leg(torch, out, args, prob, dev_sig, v_init, run, precision, cells)
        fcycle_leg(torch, out, args, prob, dev_sig, v_init, run, precision, cells)
    # the workload's own finest sweep (cache-resident at 1024^2), then the kernels at an HBM-resident size
    t_own = time_launches(torch, plan.stream, sweep_launcher(plan, b, v_init, sweeps_per_launch()), args.reps)
    cache_resident = SWEEP_BYTES_PER_CELL * cells < (256 << 20)
    own = roofline_entry(sweep_kernel(), f"finest-level FP64 Jacobi sweeps, {sweeps_per_launch()} per launch",
                         SWEEP_BYTES_PER_CELL * sweeps_per_launch() * cells, t_own, None, f"{prob['nx']}x{prob['ny']}",
                         "Infinity Cache (the sweep's working set, 112 B/cell, fits in its 256 MB)"
                         if cache_resident else "HBM")
    del plan
    torch.cuda.empty_cache()
    kernels = kernel_leg(torch, args.reps)
    out["roofline"] = kernels[0]
    out["roofline_kernels"] = kernels[1:]
    if cache_resident:  # HBM does not bound it: its rate, without an HBM fraction
        for key in ("bound", "peak", "frac", "traffic"):
            own.pop(key)
        out["headline_grid_sweep"] = own
    else:
        out["roofline_kernels"].append(own)
    c1 = None
    if args.workload == "hotwall" and not args.no_extras:
        c1 = c1_leg(torch)
        out["c3"] = c3_leg(torch)
        out["three_d"] = three_d_leg(torch, args.reps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, v0, sig, run, cycles / run["steps"], args.cpu_cycles, levels, c1)
    if c1 is not None:
        c1.pop("result", None)
        out["c1"] = c1
    if args.workload == "hotwall" and not args.no_extras:
        out["batched"] = batch_leg(torch, args.batch)
        torch.cuda.empty_cache()
        out["serving"] = {"workload": SERVE_DESC, **serve_leg(torch, args.requests, float(args.rates.split(",")[0]),
                                                              int(args.arena_gb * (1 << 30)), args.serve_precision)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
