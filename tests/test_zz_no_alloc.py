"""m1_step_static, the allocation-free time step: a plan over the library's
static device array (no hipMalloc, no pinned host memory, no graphs).  Its
results must equal m1_step's on a plan with a caller workspace, to the bit, on
consecutive calls that reuse the array with different (smaller) problems and
precisions; sizes beyond the array are refused before anything runs."""
import numpy as np
import pytest

from paper_2208_14703_amd import binding, inputs
from tests.gpu_util import announce, to_dev, to_host

pytestmark = pytest.mark.gpu


def with_plan(prob, v, sig, steps, params):
    P = binding.Plan(prob, to_dev(sig), params)
    vd = to_dev(v)
    info = P.step(vd, steps)
    return to_host(vd), info


def static(prob, v, sig, steps, params):
    vd = to_dev(v)
    info = binding.step_static(prob, to_dev(sig), vd, steps, params)
    return to_host(vd), info


CALLS = [
    # (dim, nx, ny, steps, precision): each call smaller than the one before it
    (2, 512, 256, 2, "fp64"),
    (2, 160, 96, 2, "mixed"),
    (2, 64, 48, 3, "fp64"),
    (1, 96, 1, 2, "fp64"),
]


def test_static_step_matches_plan_step_on_consecutive_calls():
    for k, (dim, nx, ny, steps, prec) in enumerate(CALLS):
        announce("m1_step_static", dim, nx, ny, steps, prec)
        bcs = ("dirichlet", "reflective", "periodic", "periodic") if dim == 2 else ("periodic",) * 4
        prob, v, sig = inputs.random_problem(600 + k, dim, nx, ny, bc_kinds=bcs, cfl=80.0, log10_sa=(-3, 3),
                                             fmax=0.95, block=8)
        params = dict(omega=0.8, rtol=1e-10, precision=prec)
        ref, iref = with_plan(prob, v, sig, steps, params)
        got, info = static(prob, v, sig, steps, params)
        assert iref["status"] == 0 and info["status"] == 0, (iref, info)
        assert (info["cycles"], info["steps_done"], info["rel_residual"]) == \
            (iref["cycles"], iref["steps_done"], iref["rel_residual"])
        np.testing.assert_array_equal(got.view(np.int64), ref.view(np.int64))


def test_static_step_refuses_sizes_beyond_its_array():
    announce("m1_step_static: size limit")
    prob, v, sig = inputs.random_problem(650, 2, 1024, 1024, cfl=80.0, block=32)
    vd = to_dev(v)
    with pytest.raises(binding.M1Error) as ei:
        binding.step_static(prob, to_dev(sig), vd, 1, dict(omega=0.8))
    assert ei.value.status == 4  # M1_ERR_WORKSPACE
    np.testing.assert_array_equal(to_host(vd), v)
    # the array still serves a call that fits, and a non-admissible input is reported as by m1_step
    prob, v, sig = inputs.random_problem(651, 2, 64, 64, cfl=80.0)
    bad = v.copy()
    bad[0, 5, 7] = -1.0
    vd = to_dev(bad)
    with pytest.raises(binding.M1Error) as ei:
        binding.step_static(prob, to_dev(sig), vd, 1, dict(omega=0.8))
    assert ei.value.status == 2
    np.testing.assert_array_equal(to_host(vd), bad)
    got, info = static(prob, v, sig, 1, dict(omega=0.8))
    ref, iref = with_plan(prob, v, sig, 1, dict(omega=0.8))
    np.testing.assert_array_equal(got, ref)
