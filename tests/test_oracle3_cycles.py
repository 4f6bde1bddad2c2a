"""Pins of the three-dimensional oracle's W- and F-cycles (CPU only).

The paper names W- and F-cycles as alternatives to its V-cycle (Sect. 6.3).
The 3-D oracle writes every shape as one recursion over the coarse FAS
problems, as the 2-D oracle does; its V-cycle (Appendix A) is also written as
the loop over levels.  Pins:

* the recursion with one visit per level (V) equals the loop form bitwise on
  grids of two to four levels and every side kind;
* on two levels a W-cycle visits the coarse problem twice and an F-cycle runs
  an F-visit then a V-visit of it; both equal a V-cycle with twice the
  pseudo-time steps on the coarse level, bitwise, and the shape field of the
  parameters selects the same cycles;
* on three or more levels the three shapes differ and keep every iterate
  admissible;
* a state that solves the step's system is left in place by W- and F-cycles,
  and time steps with them satisfy the equations of the independent numpy
  operator (oracle/dense3.py) to the rounding floor, as the V-cycle's do.
"""
import numpy as np
import pytest

import oracle
from oracle import dense3
from paper_2208_14703_amd import inputs

BCS = [("periodic",) * 6, ("dirichlet", "reflective", "neumann", "reflective", "periodic", "periodic"),
       ("dirichlet", "neumann", "reflective", "reflective", "neumann", "dirichlet")]


def admissible3(v, c):
    F = np.sqrt(v[1] ** 2 + v[2] ** 2 + v[3] ** 2)
    return bool(np.all(v[0] > 0) and np.all(v[4] > 0) and np.all(F <= c * v[0] * (1 + 1e-14)))


def problem(seed, nx, ny, nz, bcs, cfl=100.0):
    prob, v, sig = inputs.random_problem3(seed, nx, ny, nz, bc_kinds=bcs, cfl=cfl, log10_sa=(-3, 2))
    o = oracle.Oracle3(prob, sig)
    b = o.rhs(v)
    u = inputs.random_state3(np.random.default_rng(seed + 1), nz, ny, nx, fmax=0.9)
    u[4] = np.random.default_rng(seed + 2).uniform(0.5, 1.5, size=u[4].shape)
    return prob, o, b, u


@pytest.mark.parametrize("nx,ny,nz,levels", [(16, 16, 16, 0), (16, 8, 8, 2), (32, 16, 16, 4)])
def test_recursive_v_equals_the_loop_form(nx, ny, nz, levels):
    for k, bcs in enumerate(BCS):
        prob, o, b, u = problem(800 + k, nx, ny, nz, bcs)
        p = oracle.make_params(omega=0.8, levels=levels)
        assert o.num_levels(p) >= 2
        for dtau in (1e-3, 0.3):
            np.testing.assert_array_equal(o.cycle(b, u, dtau, "V", p), o.vcycle(b, u, dtau, p))


@pytest.mark.parametrize("m", [1, 3])
def test_two_level_w_and_f_are_v_with_twice_the_coarse_steps(m):
    for k, bcs in enumerate(BCS):
        prob, o, b, u = problem(820 + k, 12, 8, 8, bcs)
        p = oracle.make_params(omega=0.8, levels=2, pseudo_steps=m)
        want = o.vcycle(b, u, 0.05, oracle.make_params(omega=0.8, levels=2, pseudo_steps=2 * m))
        np.testing.assert_array_equal(o.cycle(b, u, 0.05, "W", p), want)
        np.testing.assert_array_equal(o.cycle(b, u, 0.05, "F", p), want)
        for kind in "WF":
            np.testing.assert_array_equal(
                o.vcycle(b, u, 0.05, oracle.make_params(omega=0.8, levels=2, pseudo_steps=m, cycle=kind)), want)


def test_shapes_differ_on_more_levels_and_stay_admissible():
    prob, o, b, u = problem(840, 32, 16, 16, BCS[1])
    p = oracle.make_params(omega=0.8)
    assert o.num_levels(p) >= 3
    out = {kind: o.cycle(b, u, 0.05, kind, p) for kind in "VWF"}
    for kind, x in out.items():
        assert admissible3(x, prob["c"]), kind
    assert not np.array_equal(out["V"], out["W"]) and not np.array_equal(out["V"], out["F"])
    assert not np.array_equal(out["W"], out["F"])


@pytest.mark.parametrize("kind", ["W", "F"])
def test_steps_solve_the_system_and_its_solution_is_a_fixed_point(kind):
    prob, v, sig = inputs.random_problem3(850, 16, 16, 16, bc_kinds=BCS[1], cfl=20.0, log10_sa=(-2, 1), wall_E=3.0)
    o = oracle.Oracle3(prob, sig)
    b = o.rhs(v)
    tight = dict(omega=0.8, rtol=1e-14, max_cycles=20000)
    assert o.num_levels(oracle.make_params(**tight)) == 3
    got, info = o.step(v, 1, oracle.make_params(cycle=kind, **tight))
    assert info["status"] == 0
    vref, iv = o.step(v, 1, oracle.make_params(**tight))
    scale = np.abs(vref).max()
    # the equations of the independent numpy operator hold at both solutions
    for x in (got, vref):
        assert np.abs(dense3.apply_A3(x, sig, prob) - b).max() <= 1e-11 * np.abs(b).max()
    np.testing.assert_allclose(got, vref, rtol=0, atol=1e-11 * scale)
    # and one more cycle of the shape does not move the solution
    np.testing.assert_allclose(o.cycle(b, vref, 0.1, kind, oracle.make_params(omega=0.8)), vref, rtol=0,
                               atol=1e-11 * scale)
    print(f"{kind}: {info['cycles']} cycles, V: {iv['cycles']}")
