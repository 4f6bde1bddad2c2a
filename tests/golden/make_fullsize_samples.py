"""Write tests/golden/fullsize_*.txt: the oracle's converged solutions of the two 2-D timing workloads, at sampled cells.

  * hotwall1024: the hot wall at 1024^2 (paper_2208_14703_amd.inputs.hot_wall_2d), 10 implicit steps;
  * lognormal4096: the lognormal medium at 4096^2 (inputs.lognormal_2d), one implicit step;

each solved by the oracle alone (FP64, multigrid to the deepest hierarchy, omega 0.8, the pseudo-time step carried
from one time step into the next, every step to relative
residual 1e-13 or the rounding floor of A).  Stored per workload: the largest |E| and |T| over the whole grid
(the scales of the parity metric) and (E, Fx, Fy, T) at a 32 x 32 lattice of block centres plus 1024 cells of the
middle row, with 17 significant digits.  The oracle runs on the host's cores for several minutes.

    python tests/golden/make_fullsize_samples.py [hotwall1024|lognormal4096 ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2208_14703_amd import inputs  # noqa: E402

RTOL = 1e-13


def sample_cells(n):
    """32 x 32 block centres and 1024 evenly spaced cells of the middle row, as (j, i) without repeats."""
    lat = (np.arange(32) * n) // 32 + n // 64
    cells = [(int(j), int(i)) for j in lat for i in lat]
    mid = n // 2
    cells += [(mid, int(i)) for i in (np.arange(1024) * n) // 1024]
    seen, out = set(), []
    for c in cells:
        if c not in seen:
            seen.add(c)
            out.append(c)
    return out


def workload(name):
    if name == "hotwall1024":
        return inputs.hot_wall_2d(n=1024)
    if name == "lognormal4096":
        return inputs.lognormal_2d(n=4096)
    raise SystemExit(f"unknown workload {name}")


def main(names):
    for name in names:
        prob, v, sig, run = workload(name)
        o = oracle.Oracle(prob, sig)
        p = oracle.make_params(omega=0.8, rtol=RTOL, max_cycles=40000, dtau_carry=1)
        t0 = time.perf_counter()
        out, info = o.step(v, run["steps"], p)
        dt = time.perf_counter() - t0
        assert info["status"] == 0, info
        n = prob["nx"]
        lines = [f"# {name}: the oracle's converged solution at sampled cells "
                 f"(written by tests/golden/make_fullsize_samples.py, oracle only)",
                 f"# {run['steps']} implicit step(s), FP64, omega 0.8, dtau_im carried from step to step, relative "
                 f"residual {RTOL:g} (or the rounding floor); {info['cycles']} cycles, last relative residual {info['rel_residual']:.3e}, "
                 f"{dt:.0f} s on {oracle.threads()} threads",
                 f"scale {np.abs(out[0]).max():.17e} {np.abs(out[3]).max():.17e}",
                 "# j i E Fx Fy T"]
        for j, i in sample_cells(n):
            lines.append(f"{j} {i} " + " ".join(f"{out[k, j, i]:.17e}" for k in range(4)))
        with open(os.path.join(HERE, f"fullsize_{name}.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
        print(name, info["cycles"], f"{dt:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["hotwall1024", "lognormal4096"])
