"""W- and F-cycles of the three-dimensional plans against the 3-D oracle (GPU, through the C ABI).

The alternatives to the V-cycle that Sect. 6.3 names, run by the 3-D plans as a
recursion over the coarse FAS problems:

* three cycles of each shape in a row against the oracle's recursion (1e-11 of
  the state's scale) on grids of three levels with every side kind, unequal
  sides and unequal cell sizes, the finest levels wide enough for the staged
  kernels and the coarsest not;
* on two levels W and F equal, to the bit, a V-cycle with twice the coarse
  pseudo-time steps (the oracle's pin, here on the device's own launches);
* converged time steps (both sides at 1e-13: 1e-10, cycle counts within one per
  step) of the 32^3 hot wall, both shapes;
* a plan of one level runs the shapes as its sweeps;
* at the cycle cap the state is the oracle's after that many cycles (the last
  cycle enqueued only measures the residual of the one before), with the
  iterate in either buffer.
"""
import numpy as np
import pytest

import oracle
from paper_2208_14703_amd import binding, inputs
from tests.gpu_util import announce, to_dev, to_host

pytestmark = pytest.mark.gpu

OMEGA = 0.8
MIXED = ("dirichlet", "reflective", "neumann", "reflective", "periodic", "periodic")
ALLKINDS = ("dirichlet", "neumann", "reflective", "reflective", "neumann", "dirichlet")
CASES = {
    "mixed32x24x16": (32, 24, 16, MIXED),
    "all64x16x16": (64, 16, 16, ALLKINDS),
    "periodic40x24x16": (40, 24, 16, ("periodic",) * 6),
}


def rel3(got, ref, c):
    sE = np.abs(ref[0]).max()
    return max(np.abs(got[0] - ref[0]).max() / sE, np.abs(got[1:4] - ref[1:4]).max() / (c * sE),
               np.abs(got[4] - ref[4]).max() / np.abs(ref[4]).max())


def problem(case, seed=7, cfl=40.0):
    nx, ny, nz, bcs = CASES[case]
    prob, v, sig = inputs.random_problem3(seed, nx, ny, nz, bc_kinds=bcs, cfl=cfl, log10_sa=(-3, 2), wall_E=5.0)
    prob["hy"], prob["hz"] = prob["hx"] * 1.25, prob["hx"] * 0.8
    return prob, v, sig


@pytest.mark.parametrize("kind", ["W", "F"])
@pytest.mark.parametrize("case", list(CASES))
def test_cycles_match_oracle(case, kind):
    announce("3-D cycles", case, kind)
    prob, v, sig = problem(case)
    o = oracle.Oracle3(prob, sig)
    params = dict(omega=OMEGA, cycle=kind)
    P = binding.Plan3(prob, to_dev(sig), params)
    assert P.levels == o.num_levels(oracle.make_params(**params)) == 3
    b = o.rhs(v)
    vd, vn = to_dev(v), to_dev(v)
    ref = v
    for cyc, dtau in enumerate((1e-3, 0.3, 5.0)):
        P.vcycle(vd, vn, dtau)
        ref = o.cycle(b, ref, dtau, kind, oracle.make_params(omega=OMEGA))
        err = rel3(to_host(vd), ref, prob["c"])
        assert err <= 1e-11, (cyc, err)
    # the shapes differ from the V-cycle on three levels
    vv = to_dev(v)
    binding.Plan3(prob, to_dev(sig), dict(omega=OMEGA)).vcycle(vv, vn, 1e-3)
    vw = to_dev(v)
    P.vcycle(vw, vn, 1e-3)
    assert not np.array_equal(to_host(vv), to_host(vw))


@pytest.mark.parametrize("m", [1, 2])
def test_two_levels_are_v_with_twice_the_coarse_steps(m):
    announce("3-D two-level cycles", m)
    prob, v, sig = problem("mixed32x24x16", seed=8)
    sd = to_dev(sig)
    want = to_dev(v)
    vn = to_dev(v)
    binding.Plan3(prob, sd, dict(omega=OMEGA, levels=2, pseudo_steps=2 * m)).vcycle(want, vn, 0.05)
    for kind in "WF":
        got = to_dev(v)
        binding.Plan3(prob, sd, dict(omega=OMEGA, levels=2, pseudo_steps=m, cycle=kind)).vcycle(got, vn, 0.05)
        np.testing.assert_array_equal(to_host(got), to_host(want))


@pytest.mark.parametrize("kind", ["W", "F"])
def test_converged_steps_match_oracle(kind):
    announce("3-D cycle steps", kind)
    prob, v, sig, _ = inputs.hot_wall_3d(n=32, block=4)
    nsteps = 2
    params = dict(omega=OMEGA, rtol=1e-13, max_cycles=20000, cycle=kind)
    o = oracle.Oracle3(prob, sig)
    ref, io = o.step(v, nsteps, oracle.make_params(**params))
    assert io["status"] == 0
    P = binding.Plan3(prob, to_dev(sig), params)
    assert P.levels == 4
    vd = to_dev(v)
    info = P.step(vd, nsteps)
    assert info["status"] == 0, info
    err = rel3(to_host(vd), ref, prob["c"])
    print(f"{kind}: cycles gpu/oracle {info['cycles']} {io['cycles']}, error {err:.2e}")
    assert err <= 1e-10
    assert abs(info["cycles"] - io["cycles"]) <= nsteps


def test_one_level_plan():
    announce("3-D cycles on one level")
    prob = inputs.grid_problem3(1, 1, 1, 5.0, [dict(kind="periodic")] * 6)
    v = np.array([2.0, 0.3, -0.2, 0.1, 1.2]).reshape(5, 1, 1, 1)
    sig = np.zeros((2, 1, 1, 1))
    sig[0] = 2.0
    o = oracle.Oracle3(prob, sig)
    for kind in "WF":
        params = dict(omega=OMEGA, rtol=1e-13, cycle=kind)
        ref, io = o.step(v, 2, oracle.make_params(**params))
        P = binding.Plan3(prob, to_dev(sig), params)
        assert P.levels == 1
        vd = to_dev(v)
        info = P.step(vd, 2)
        assert info["status"] == io["status"] == 0
        assert rel3(to_host(vd), ref, prob["c"]) <= 1e-12


@pytest.mark.parametrize("levels,nu0", [(0, 3), (1, 3), (1, 2)])
def test_cycle_cap_returns_the_last_full_cycle(levels, nu0):
    """Each cycle's first sweep measures the previous result's residual, so the last cycle enqueued only
    measures: at the cycle cap the state is the one after max_cycles full cycles, wherever the sweeps left
    it (one level with an odd nu0 moves it to the partner buffer every cycle)."""
    announce("3-D cycle cap", levels, nu0)
    prob, v, sig = problem("mixed32x24x16", seed=9)
    o = oracle.Oracle3(prob, sig)
    for kind in "VW":
        for cap in (1, 4, 5):
            params = dict(omega=OMEGA, rtol=1e-30, max_cycles=cap, cycle=kind, levels=levels, nu0=nu0)
            ref, io = o.step(v, 1, oracle.make_params(**params))
            P = binding.Plan3(prob, to_dev(sig), params)
            vd = to_dev(v)
            info = P.step(vd, 1)
            assert info["status"] == io["status"] == 3 and info["cycles"] == io["cycles"] == cap, (info, io)
            err = rel3(to_host(vd), ref, prob["c"])
            assert err <= 1e-11, (kind, cap, err)
