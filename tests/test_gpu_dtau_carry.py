"""The implicit pseudo-time step across time steps, both readings (GPU, through the C ABI).

The overall algorithm of Appendix A computes one time step and does not set the
pseudo-time step among its first steps; Sect. 5 gives only its initial value,
1e-3.  With dtau_carry = 1 (the default) a call's time steps hand the step on,
with dtau_carry = 0 every time step restarts it at dtau_im0.

* Against the oracle in both readings: three time steps of a 2-D hot wall and
  two of a 3-D problem, solved to 1e-13: the state within 1e-10, the cycle
  count within one per step.
* Splitting: n steps in one call give, to the bit, the results of n calls of one
  step each, every call started at the dtau the previous one ended with
  (carry) or at dtau_im0 (no carry): 2-D FP64, 2-D mixed precision, 3-D.
* Engines: requests of both readings in one batch give, to the bit, their
  results solved alone.
"""
import numpy as np
import pytest

import oracle
from paper_2208_14703_amd import binding, inputs
from tests.gpu_util import announce, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

OMEGA = 0.8


def hot_wall(n=96):
    prob, v, sig, _ = inputs.hot_wall_2d(n=n)
    return prob, v, sig


@pytest.mark.parametrize("carry", [1, 0])
def test_steps_match_the_oracle(carry):
    announce("dtau carry vs oracle", carry)
    prob, v, sig = hot_wall()
    params = dict(omega=OMEGA, rtol=1e-13, max_cycles=20000, dtau_carry=carry)
    ref, io = oracle.Oracle(prob, sig).step(v, 3, oracle.make_params(**params))
    P = binding.Plan(prob, to_dev(sig), params)
    vd = to_dev(v)
    info = P.step(vd, 3)
    assert info["status"] == io["status"] == 0
    err = rel_err(to_host(vd), ref, prob["c"])
    print(f"2-D carry {carry}: cycles gpu/oracle {info['cycles']} {io['cycles']}, error {err:.2e}")
    assert err <= 1e-10
    assert abs(info["cycles"] - io["cycles"]) <= 3
    prob3, v3, sig3, _ = inputs.hot_wall_3d(n=16, block=4)
    ref3, io3 = oracle.Oracle3(prob3, sig3).step(v3, 2, oracle.make_params(**params))
    P3 = binding.Plan3(prob3, to_dev(sig3), params)
    vd3 = to_dev(v3)
    i3 = P3.step(vd3, 2)
    assert i3["status"] == io3["status"] == 0
    g3 = to_host(vd3)
    sE = np.abs(ref3[0]).max()
    err3 = max(np.abs(g3[0] - ref3[0]).max() / sE, np.abs(g3[1:4] - ref3[1:4]).max() / (prob3["c"] * sE),
               np.abs(g3[4] - ref3[4]).max() / np.abs(ref3[4]).max())
    print(f"3-D carry {carry}: cycles gpu/oracle {i3['cycles']} {io3['cycles']}, error {err3:.2e}")
    assert err3 <= 1e-10
    assert abs(i3["cycles"] - io3["cycles"]) <= 2


def split_runs(make_plan, v, nsteps, carry, dtau0=1e-3):
    """nsteps in one call, and nsteps calls of one step each (fresh plans, each started where the last ended)."""
    P = make_plan(dict(dtau_carry=carry))
    vd = to_dev(v)
    whole = P.step(vd, nsteps)
    got_whole = to_host(vd)
    vs = to_dev(v)
    dtau, cycles = dtau0, 0
    for _ in range(nsteps):
        info = make_plan(dict(dtau_carry=carry, dtau_im0=dtau)).step(vs, 1)
        assert info["status"] == 0
        cycles += info["cycles"]
        if carry:
            dtau = info["dtau"]
    return got_whole, whole, to_host(vs), cycles, info["dtau"]


@pytest.mark.parametrize("form", ["fp64", "mixed", "3d"])
@pytest.mark.parametrize("carry", [1, 0])
def test_one_call_equals_single_steps(form, carry):
    announce("dtau carry splitting", form, carry)
    base = dict(omega=OMEGA, rtol=1e-9, max_cycles=5000)
    if form == "3d":
        prob, v, sig, _ = inputs.hot_wall_3d(n=32, block=4)
        sd = to_dev(sig)
        make = lambda extra: binding.Plan3(prob, sd, dict(base, **extra))  # noqa: E731
    else:
        prob, v, sig = hot_wall(128)
        sd = to_dev(sig)
        make = lambda extra: binding.Plan(prob, sd, dict(base, precision=form, **extra))  # noqa: E731
    got_whole, whole, got_split, cycles, last_dtau = split_runs(make, v, 3, carry)
    print(f"{form} carry {carry}: cycles {whole['cycles']}, final dtau {whole['dtau']:.4g}")
    assert whole["status"] == 0
    np.testing.assert_array_equal(got_whole, got_split)
    assert whole["cycles"] == cycles and whole["dtau"] == last_dtau


def test_engine_runs_both_readings():
    announce("dtau carry in engines")
    base = dict(omega=OMEGA, rtol=1e-8)
    E = binding.Engine(1 << 30, base, max_requests=16)
    cases = []
    for k in range(6):
        prob, v, sig = inputs.random_problem(500 + k, 2, 64 + 32 * (k % 3), 64, cfl=100.0, log10_sa=(-3, 3),
                                             fmax=0.95, block=16)
        params = dict(base, dtau_carry=k % 2)
        vd = to_dev(v)
        cases.append((prob, v, sig, params, vd, E.submit(prob, to_dev(sig), vd, 3, params)))
    for prob, v, sig, params, vd, t in cases:
        info = E.wait(t)
        P = binding.Plan(prob, to_dev(sig), params)
        va = to_dev(v)
        ia = P.step(va, 3)
        assert info["status"] == ia["status"] == 0
        assert info["cycles"] == ia["cycles"] and info["dtau"] == ia["dtau"], (params["dtau_carry"], info, ia)
        np.testing.assert_array_equal(to_host(vd), to_host(va))
