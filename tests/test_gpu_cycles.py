"""W- and F-cycles (Sect. 6.3) on the GPU against the oracle's.

* One cycle at a time, three in a row with changing pseudo-time steps, on 2-D
  workloads of four and five levels, a 2-D side-condition mix, 1-D, with the
  fused residual-restriction launch and without, and with two Jacobi sweeps per
  pseudo-time step: 1e-11 of the state's scale (the V-cycle's bar).
* Converged time steps (rtol 1e-13) within 1e-10, with the cycle count of the
  oracle's up to a rounding flip of the last stopping test; the same step with
  recorded (hipGraph) cycles and with plain launches, bitwise.
* W and F are FP64 only: mixed-precision plans and engines reject them.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2208_14703_amd import binding, inputs
from tests.gpu_util import announce, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

OMEGA = 0.8


def case_problem(case):
    if case == "hot64":
        prob, v, sig, _ = inputs.hot_wall_2d(n=64)
    elif case == "logn128":
        prob, v, sig, _ = inputs.lognormal_2d(n=128)
    elif case == "gauss256":
        prob, v, sig, _ = inputs.gaussian_1d(n=256)
    else:
        prob, v, sig = inputs.random_problem(7, 2, 96, 80, bc_kinds=("dirichlet", "reflective", "periodic",
                                                                   "periodic"), cfl=80.0)
    return prob, v, sig


@pytest.mark.parametrize("kind", ["W", "F"])
@pytest.mark.parametrize("case,fused,nu_l", [("hot64", 1, 1), ("logn128", 1, 1), ("logn128", 0, 1),
                                             ("mixed96x80", 1, 1), ("mixed96x80", 1, 2), ("gauss256", 1, 1)])
def test_cycle_parity(kind, case, fused, nu_l):
    announce("cycle", kind, case, fused, nu_l)
    prob, v, sig = case_problem(case)
    o = oracle.Oracle(prob, sig)
    params = dict(omega=OMEGA, cycle=kind, nu_l=nu_l)
    old = binding.tune_get("residual_restrict")
    binding.tune_set("residual_restrict", fused)
    try:
        P = binding.Plan(prob, to_dev(sig), params)
        assert P.levels >= 4 or prob["dim"] == 1
        b = o.rhs(v)
        vd, vn = to_dev(v), to_dev(v)
        ref = v
        for cyc, dtau in enumerate((1e-3, 0.3, 5.0)):
            P.vcycle(vd, vn, dtau)
            ref = o.vcycle(b, ref, dtau, params=oracle.make_params(**params))
            err = rel_err(to_host(vd), ref, prob["c"])
            assert err <= 1e-11, (cyc, err)
    finally:
        binding.tune_set("residual_restrict", old)


@pytest.mark.parametrize("kind", ["W", "F"])
@pytest.mark.parametrize("case", ["hot128", "gauss256"])
def test_converged_step_parity(kind, case):
    announce("cycle step", kind, case)
    if case == "hot128":
        prob, v, sig, _ = inputs.hot_wall_2d(n=128)
    else:
        prob, v, sig, _ = inputs.gaussian_1d(n=256)
    rtol = 1e-13
    o = oracle.Oracle(prob, sig)
    ref, info_o = o.step(v, 1, oracle.make_params(omega=OMEGA, rtol=rtol, max_cycles=40000, cycle=kind))
    assert info_o["status"] == 0
    results = {}
    old = binding.tune_get("graphs")
    try:
        for graphs in (1, 0):
            binding.tune_set("graphs", graphs)
            P = binding.Plan(prob, to_dev(sig), dict(omega=OMEGA, rtol=rtol, max_cycles=40000, cycle=kind))
            vd = to_dev(v)
            info = P.step(vd, 1)
            assert info["status"] == 0 and info["rel_residual"] <= 1e-11, info
            results[graphs] = (to_host(vd), info["cycles"])
    finally:
        binding.tune_set("graphs", old)
    got, cycles = results[1]
    np.testing.assert_array_equal(got, results[0][0])
    assert cycles == results[0][1]
    assert rel_err(got, ref, prob["c"]) <= 1e-10
    print(f"{kind} {case}: cycles gpu/oracle {cycles} {info_o['cycles']}", flush=True)
    assert abs(cycles - info_o["cycles"]) <= 1


@pytest.mark.parametrize("kind", ["W", "F"])
def test_mixed_precision_and_engines_reject_w_and_f(kind):
    announce("cycle rejections", kind)
    prob, v, sig, _ = inputs.hot_wall_2d(n=64)
    with pytest.raises(binding.M1Error) as e:
        binding.Plan(prob, to_dev(sig), dict(omega=OMEGA, cycle=kind, precision="mixed"))
    assert "M1_ERR_ARG" in str(e.value)
    p = binding.make_params(binding.default_params(omega=OMEGA, cycle=kind))
    arena = ctypes.c_void_p(256)  # never dereferenced: the parameters are checked first
    out = ctypes.c_void_p()
    st = binding.lib().m1_engine_create(ctypes.byref(p), arena, 1 << 20, 4, None, ctypes.byref(out))
    assert st == 1 and not out.value  # M1_ERR_ARG
