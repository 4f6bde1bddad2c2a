"""Write tests/golden/beam_peaks.txt: reference values of the Sect. 5.1 beam, computed by the oracle only.

For the beam recipe (paper_2208_14703_amd.inputs.beam_2d) at 128^2 and 129^2 cells:
  * the explicit steady states (CFL 0.45, run until a step changes E by at most 1e-13 of its maximum) with the
    Rusanov flux (wave speeds +-c, the implicit scheme's flux) and with the HLL flux at the M1 wave speeds;
  * the implicit solution of one step at CFL 2000 (the oracle's multigrid at 128^2, plain Jacobi at 129^2, whose
    odd sides do not coarsen), relative residual 1e-11;
and, for each, the largest E on the horizontal cut at mid height (y = 0: the middle row of 129^2, the mean of the
two middle rows of 128^2).

    python tests/golden/make_beam_peaks.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2208_14703_amd import inputs  # noqa: E402


def cut_peak(v):
    n = v.shape[1]
    row = v[0, n // 2] if n % 2 else 0.5 * (v[0, n // 2 - 1] + v[0, n // 2])
    return float(row.max())


def main():
    lines = ["# Sect. 5.1 beam: largest E on the cut y = 0 (written by tests/golden/make_beam_peaks.py, oracle only)",
             "# n  solution  cycles_or_steps  peak"]
    for n in (128, 129):
        prob, v, sig, _ = inputs.beam_2d(n=n)
        o = oracle.Oracle(prob, sig)
        for name, hll in (("explicit_rusanov", False), ("explicit_hll", True)):
            out, steps = o.explicit_run(v, hll=hll, dt=0.45 * prob["hx"] / prob["c"], max_steps=400000, tol=1e-13)
            assert steps < 400000
            lines.append(f"{n} {name} {steps} {cut_peak(out):.12e}")
            print(lines[-1], flush=True)
        p = oracle.make_params(omega=0.8, rtol=1e-11, max_cycles=400000, levels=1 if n % 2 else 0)
        out, info = o.step(v, 1, p)
        assert info["status"] == 0
        lines.append(f"{n} implicit_cfl2000 {info['cycles']} {cut_peak(out):.12e}")
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "beam_peaks.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
