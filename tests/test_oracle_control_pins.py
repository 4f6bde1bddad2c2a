"""Pins of the oracle's speed-only rules (CPU only).

These rules change how fast the cycle converges, not its answer, so no
converged-solution test can catch a wrong factor in them.  Each is pinned here
against what the paper prints or against an independent construction:

* pseudo-time step adaptation (Appendix A, Algorithm 4; Sect. 5: initial step
  1e-3): the time-step driver is written out again in the test from the printed
  rule -- x1.1 when the residual change exceeds eps_inc, /2 when it is below
  eps_dec, set to 1e-3 once before the first time step (the overall algorithm
  does not set it at the start of a step) or, in the other reading, again at
  every time step -- with the oracle's V-cycle as a step, and
  its iterates and final step must equal those of ``or_step``; both the signed
  reading and the literal |r_k - r_{k-1}| / r_0 form, with thresholds that make
  both branches fire;
* the explicit sub-steps of a pseudo-time step (Algorithm 3, the explicit
  formula for the sub-step length of Sect. 4.3): each cell's pseudo time equals
  min(dtau, tau* (1 - (1 - eta)^K)) with tau* found by bisection on the
  admissibility predicate (the sub-steps move along one ray, each taking eta of
  what is left);
* a whole pseudo-time step on a one-cell periodic grid, where the implicit
  Jacobi step has a closed form;
* the admissibility-restoring correction (eq. prolongatedSol): the blend is
  u + theta (w - u) with theta = eta tau*(u, w - u), tau* again by bisection.
"""
import numpy as np
import pytest

import oracle
from paper_2208_14703_amd import inputs

# Sect. 5: initial implicit pseudo-time step; Appendix A: growth and decrease factors
DTAU0 = 1e-3
GROW, SHRINK = 1.1, 0.5


def bisect_ray(c, w, s, hi=1e8, iters=300):
    """Largest tau with w + tau s admissible, by bisection on the predicate only."""
    if oracle.admissible(c, w + hi * s):
        return np.inf
    lo = 0.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if oracle.admissible(c, w + mid * s):
            lo = mid
        else:
            hi = mid
    return lo


# ------------------------------------------------------------------ dtau adaptation
def printed_rule(rule, dtau, r0, rprev, r, eps_inc, eps_dec, dmin, dmax):
    if rule == "literal":
        change = abs(r - rprev) / r0          # as printed in the overall algorithm
    else:
        change = (rprev - r) / rprev          # signed relative decrease (the reading used by default)
    if change > eps_inc:
        dtau = GROW * dtau
    if change < eps_dec:
        dtau = dtau / 2.0
    return min(max(dtau, dmin), dmax)


def driver(o, v, nsteps, p, rule, max_cycles, carry=True):
    """The overall algorithm's time-step loop, written out from the paper with
    the oracle's V-cycle, residual and norm as its steps.  The pseudo-time step
    is initialised once, before the time loop (carry); carry=False restarts it
    at every time step."""
    v = v.copy()
    dtaus, rels = [], []
    dtau = DTAU0
    for _ in range(nsteps):
        b = o.rhs(v)
        if not carry:
            dtau = DTAU0
        r0 = o.norm(o.residual(b, v))
        rprev = r0
        for _k in range(max_cycles):
            dtaus.append(dtau)
            v = o.vcycle(b, v, dtau, p)
            r = o.norm(o.residual(b, v))
            rels.append(r / r0)
            dtau = printed_rule(rule, dtau, r0, rprev, r, p.eps_inc, p.eps_dec, p.dtau_min, p.dtau_max)
            rprev = r
            if r / r0 <= p.rtol:
                break
    return v, dtau, dtaus, rels


@pytest.mark.parametrize("rule,eps_inc,eps_dec,both", [("signed", 0.05, 0.0, False), ("signed", 0.5, 0.3, True),
                                                        ("literal", 0.02, 0.005, True)])
def test_dtau_adaptation_follows_the_printed_rule(rule, eps_inc, eps_dec, both):
    """The paper gives no values for eps_inc / eps_dec; the defaults (0.05, 0) only
    grow the step on this case, the others make both branches fire."""
    prob, v, sig = inputs.random_problem(901, 2, 16, 16, bc_kinds=("dirichlet", "reflective", "periodic", "periodic"),
                                         cfl=60.0, fmax=0.99, log10_sa=(-3, 2))
    o = oracle.Oracle(prob, sig)
    cycles = 14
    p = oracle.make_params(omega=0.8, rtol=1e-30, max_cycles=cycles, dtau_rule=rule, eps_inc=eps_inc,
                           eps_dec=eps_dec)
    assert p.dtau_im0 == DTAU0  # the default initial step is the paper's
    got, info = o.step(v, 2, p)
    assert info["status"] == 3  # stopped at the cycle cap, within the first step
    ref, dtau_ref, dtaus, rels = driver(o, v, 1, p, rule, cycles)
    np.testing.assert_array_equal(got, ref)
    assert info["dtau"] == dtau_ref
    np.testing.assert_array_equal(info["history"], np.array(rels))
    # the run exercises the branches of the rule, so a wrong factor or test in either is seen
    ratios = np.array(dtaus[1:] + [dtau_ref]) / np.array(dtaus)
    assert np.any(np.isclose(ratios, GROW)), ratios
    assert np.any(np.isclose(ratios, SHRINK)) == both, ratios


@pytest.mark.parametrize("carry", [1, 0])
def test_dtau_across_time_steps(carry):
    """carry=1: each time step's first cycle runs with the step the previous one
    ended with; carry=0: with the initial step again."""
    prob, v, sig = inputs.random_problem(902, 2, 16, 16, cfl=30.0)
    o = oracle.Oracle(prob, sig)
    p = oracle.make_params(omega=0.8, rtol=1e-6, max_cycles=500, eps_inc=0.05, eps_dec=0.0, dtau_carry=carry)
    got, info = o.step(v, 3, p)
    assert info["status"] == 0
    ref, dtau_ref, dtaus, rels = driver(o, v, 3, p, "signed", 500, carry=bool(carry))
    np.testing.assert_array_equal(got, ref)
    assert info["dtau"] == dtau_ref and info["cycles"] == len(dtaus)
    np.testing.assert_array_equal(info["history"], np.array(rels))
    starts = [0]
    for k in range(1, len(rels)):
        if rels[k - 1] <= p.rtol:
            starts.append(k)
    assert len(starts) == 3 and dtaus[0] == DTAU0
    if carry:  # the step grew during the previous time step (eps_dec = 0 never halves it) and runs on
        assert all(dtaus[k] > DTAU0 for k in starts[1:])
    else:
        assert all(dtaus[k] == DTAU0 for k in starts)
    assert any(d != DTAU0 for d in dtaus)


# ------------------------------------------------------------------ sub-steps
@pytest.mark.parametrize("eta,K", [(0.9, 4), (0.5, 2), (0.7, 1), (0.9, 6)])
def test_pseudo_time_of_each_cell_is_the_closed_form(eta, K):
    rng = np.random.default_rng(7)
    prob, v, sig = inputs.random_problem(903, 2, 8, 6, cfl=10.0, fmax=1.0)
    o = oracle.Oracle(prob, sig)
    c = prob["c"]
    p = oracle.make_params(eta=eta, sub_steps=K)
    # sources pointing anywhere: some rays leave the admissible set, some never do
    f = rng.normal(size=v.shape) * np.array([1.0, c, c, 1.0])[:, None, None] * v[0] * rng.choice([0.1, 3.0, 30.0])
    f[:, 0, 0] = np.array([1.0, 0.0, 0.0, 1.0])  # a source that keeps the state admissible forever
    for dtau in (1e-3, 0.05, 1.0, 1e3):
        taus, ut = o.pseudo_time(f, v, dtau, p)
        nfree = 0
        for j in range(v.shape[1]):
            for i in range(v.shape[2]):
                s = f[:, j, i].copy()
                s[3] /= prob["c_v"]
                ts = bisect_ray(c, v[:, j, i], s)
                want = dtau if np.isinf(ts) else min(dtau, ts * (1.0 - (1.0 - eta) ** K))
                nfree += np.isinf(ts)
                assert taus[j, i] == pytest.approx(want, rel=1e-9), (dtau, j, i, taus[j, i], want, ts)
                np.testing.assert_allclose(ut[:, j, i], v[:, j, i] + taus[j, i] * s, rtol=1e-13,
                                           atol=1e-13 * abs(v[0, j, i]))
        assert nfree >= 1
        if dtau >= 1.0:  # large pseudo-time steps are ray-limited somewhere
            assert np.any(taus < dtau)


@pytest.mark.parametrize("local", [1, 0])
def test_one_cell_pseudo_step_closed_form(local):
    """One periodic cell in 1-D, no opacity: each neighbour is the cell itself, so the
    Jacobi step of (M + tau A)(u) = M u~ started from u reads
    u' (1 + tau (1 + alpha)) = u~ + tau alpha u  for E and F, and
    T' (1 + tau) = T~  for the decoupled gas row, with u~ = u + tau_i M^{-1} f."""
    cfl, eta, K = 7.0, 0.9, 4
    prob = inputs.grid_problem(1, 1, 1, cfl, inputs.bc_all("periodic"), c=1.3, c_v=2.0)
    o = oracle.Oracle(prob)
    c, cv, alpha = prob["c"], prob["c_v"], cfl
    p = oracle.make_params(eta=eta, sub_steps=K, pseudo_local=local)
    u = np.array([2.0, 0.8 * c * 2.0, 0.0, 1.5]).reshape(4, 1, 1)
    for fE, fF, dtau in [(1.0, 0.0, 0.3), (-1.0, 0.0, 5.0), (0.2, 5.0, 1.0), (0.0, -4.0, 1e-2), (3.0, 3.0, 2.0)]:
        f = np.array([fE, fF, 0.0, -0.5]).reshape(4, 1, 1)
        s = f[:, 0, 0] / np.array([1.0, 1.0, 1.0, cv])
        ts = bisect_ray(c, u[:, 0, 0], s)
        tau_i = dtau if np.isinf(ts) else min(dtau, ts * (1 - (1 - eta) ** K))
        ut = u[:, 0, 0] + tau_i * s
        tau = tau_i if local else dtau
        want = np.empty(4)
        want[:3] = (ut[:3] + tau * alpha * u[:3, 0, 0]) / (1.0 + tau * (1.0 + alpha))
        want[3] = ut[3] / (1.0 + tau)
        got = o.pseudo_step(f, u, dtau, p)[:, 0, 0]
        np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-12)


# ------------------------------------------------------------------ projection
def test_projection_blend_is_eta_times_the_ray_length():
    rng = np.random.default_rng(11)
    for eta in (0.9, 0.5):
        p = oracle.make_params(eta=eta)
        prob, v, sig = inputs.random_problem(904, 2, 10, 10, fmax=1.0)
        o = oracle.Oracle(prob, sig)
        c = prob["c"]
        w = v + rng.normal(size=v.shape) * v[0] * np.array([1.0, c, c, 0.5])[:, None, None] * 0.9
        out = o.project(v, w, p)
        nproj = 0
        for j in range(10):
            for i in range(10):
                if oracle.admissible(c, w[:, j, i]):
                    np.testing.assert_array_equal(out[:, j, i], w[:, j, i])
                    continue
                nproj += 1
                d = w[:, j, i] - v[:, j, i]
                theta = eta * bisect_ray(c, v[:, j, i], d)
                assert theta < 1.0
                np.testing.assert_allclose(out[:, j, i], v[:, j, i] + theta * d, rtol=1e-9,
                                           atol=1e-9 * np.abs(d).max())
        assert nproj >= 10
