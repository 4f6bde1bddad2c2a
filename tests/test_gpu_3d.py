"""The three-dimensional method on the GPU against the 3-D oracle (through the C ABI).

* Per operation on the finest and the first coarse level -- A, a relaxed Jacobi
  sweep, pseudo-time steps in both readings of the local step, the restriction
  and the correction with projection: 1e-13 of the state's scale (1e-12 for the
  pseudo-time step), on grids with every side kind, unequal and non-power-of-two
  sides and unequal cell sizes.
* Three V-cycles in a row (1e-11) and converged time steps (both sides at
  1e-13: 1e-10, cycle counts within one).
* Edge cases: one cell, zero steps, a non-admissible input cell (its index is
  reported), a negative opacity, parameter choices the 3-D plans do not take.
* The staged launch shapes give the one-cell kernels' bits: the apply, sweep and
  pseudo-time step staged per z-plane, and the correction with its coarse
  differences staged per tile (also whole steps, with equal cycle counts);
  every operation staged on grids one or two cells thick, whose staged
  sweeps launch more blocks (and norm partials) than 256-cell blocks would.
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
    "mixed16x12x8": (16, 12, 8, MIXED),
    "all8": (8, 8, 8, ALLKINDS),
    "periodic20x8x16": (20, 8, 16, ("periodic",) * 6),
}


def rel3(got, ref, c):
    sE = np.abs(ref[0]).max()
    return max(np.abs(got[0] - ref[0]).max() / sE, np.abs(got[1:4] - ref[1:4]).max() / (c * sE),
               np.abs(got[4] - ref[4]).max() / np.abs(ref[4]).max())


def problem(case, seed=3, cfl=40.0):
    nx, ny, nz, bcs = CASES[case]
    prob, v, sig = inputs.random_problem3(seed, nx, ny, nz, bc_kinds=bcs, cfl=cfl, log10_sa=(-3, 2), wall_E=5.0)
    prob["hy"], prob["hz"] = prob["hx"] * 1.25, prob["hx"] * 0.8
    return prob, v, sig


@pytest.mark.parametrize("case", list(CASES))
def test_operations_match_oracle(case):
    announce("3-D operations", case)
    prob, v, sig = problem(case)
    c = prob["c"]
    o = oracle.Oracle3(prob, sig)
    P = binding.Plan3(prob, to_dev(sig), dict(omega=OMEGA))
    assert P.levels == o.num_levels(oracle.make_params())
    rng = np.random.default_rng(4)
    u = inputs.random_state3(rng, prob["nz"], prob["ny"], prob["nx"], c=c, fmax=0.9)
    u[4] = rng.uniform(0.5, 1.5, size=u[4].shape)
    assert rel3(to_host(P.apply_A(0, to_dev(u))), o.apply_A(u), c) <= 1e-13
    b = o.rhs(v)
    assert rel3(to_host(P.sweep(to_dev(b), to_dev(u))), o.sweep(b, u, OMEGA), c) <= 1e-13
    f = o.apply_A(v) * 1.05
    for local in (1, 0):
        p = oracle.make_params(pseudo_local=local)
        Pl = P if local else binding.Plan3(prob, to_dev(sig), dict(omega=OMEGA, pseudo_local=0))
        for dtau in (1e-3, 0.5, 50.0):
            got = to_host(Pl.pseudo_step(0, dtau, to_dev(f), to_dev(u)))
            assert rel3(got, o.pseudo_step(f, u, dtau, p), c) <= 1e-12, (local, dtau)
    if P.levels > 1:
        g1 = o.coarse_grid()
        s1 = o.restrict(sig)
        u1 = o.restrict(u)
        assert rel3(to_host(P.restrict(0, to_dev(u))), u1, c) <= 1e-14
        assert rel3(to_host(P.apply_A(1, to_dev(u1))), o.apply_A(u1, sigma=s1, g=g1), c) <= 1e-13
        f1 = o.apply_A(u1, sigma=s1, g=g1) * 0.97
        p = oracle.make_params()
        got = to_host(P.pseudo_step(1, 0.3, to_dev(f1), to_dev(u1)))
        assert rel3(got, o.pseudo_step(f1, u1, 0.3, p, sigma=s1, g=g1), c) <= 1e-12
        uc = u1 * (1.0 + 0.6 * rng.normal(size=u1.shape))  # large coarse changes: the projection acts somewhere
        w = u + o.prolong(uc - u1)
        ref = o.project(u, w, p)
        got = to_host(P.prolong_project(0, to_dev(u), to_dev(uc), to_dev(u1)))
        assert rel3(got, ref, c) <= 1e-13
        assert not np.array_equal(ref, w)


@pytest.mark.parametrize("case", list(CASES))
def test_vcycles_match_oracle(case):
    announce("3-D vcycles", case)
    prob, v, sig = problem(case, seed=5)
    o = oracle.Oracle3(prob, sig)
    P = binding.Plan3(prob, to_dev(sig), dict(omega=OMEGA))
    b = o.rhs(v)
    vd, vn = to_dev(v), to_dev(v)
    ref = v
    for cyc, dtau in enumerate((1e-3, 0.3, 5.0)):
        P.vcycle(vd, vn, dtau)
        ref = o.vcycle(b, ref, dtau, oracle.make_params(omega=OMEGA))
        assert rel3(to_host(vd), ref, prob["c"]) <= 1e-11, cyc


@pytest.mark.parametrize("case", ["mixed16x12x8", "hot32", "periodic20x8x16"])
def test_converged_steps_match_oracle(case):
    announce("3-D steps", case)
    if case == "hot32":
        prob, v, sig, _ = inputs.hot_wall_3d(n=32, block=4)
        nsteps = 2
    else:
        prob, v, sig = problem(case, seed=6, cfl=20.0)
        nsteps = 1
    params = dict(omega=OMEGA, rtol=1e-13, max_cycles=20000)
    o = oracle.Oracle3(prob, sig)
    ref, io = o.step(v, nsteps, oracle.make_params(**params))
    assert io["status"] == 0
    P = binding.Plan3(prob, to_dev(sig), params)
    vd = to_dev(v)
    info = P.step(vd, nsteps)
    assert info["status"] == 0, info
    err = rel3(to_host(vd), ref, prob["c"])
    print(f"{case}: cycles gpu/oracle {info['cycles']} {io['cycles']}, error {err:.2e}")
    assert err <= 1e-10
    assert abs(info["cycles"] - io["cycles"]) <= nsteps


def test_edge_cases():
    announce("3-D edge cases")
    prob = inputs.grid_problem3(1, 1, 1, 5.0, [dict(kind="periodic")] * 6)
    v = np.array([2.0, 0.3, -0.2, 0.1, 1.2]).reshape(5, 1, 1, 1)
    sig = np.zeros((2, 1, 1, 1))
    sig[0] = 2.0
    o = oracle.Oracle3(prob, sig)
    ref, io = o.step(v, 3, oracle.make_params(omega=OMEGA, rtol=1e-13))
    P = binding.Plan3(prob, to_dev(sig), dict(omega=OMEGA, rtol=1e-13))
    assert P.levels == 1
    vd = to_dev(v)
    info = P.step(vd, 3)
    assert info["status"] == 0 and io["status"] == 0
    assert rel3(to_host(vd), ref, prob["c"]) <= 1e-12
    assert P.step(vd, 0)["cycles"] == 0
    # a non-admissible input cell
    prob, v, sig = problem("all8")
    v[1, 3, 2, 5] = 2.0 * prob["c"] * v[0, 3, 2, 5]
    P = binding.Plan3(prob, to_dev(sig), dict(omega=OMEGA))
    with pytest.raises(binding.M1Error) as e:
        P.step(to_dev(v), 1)
    assert e.value.status == 2 and f"'first_bad_cell': {(3 * 8 + 2) * 8 + 5}" in str(e.value)
    # a negative opacity, and parameter choices the 3-D plans reject
    bad = sig.copy()
    bad[0, 1, 1, 1] = -1.0
    with pytest.raises(binding.M1Error):
        binding.Plan3(prob, to_dev(bad), dict(omega=OMEGA))
    for extra in (dict(precision="mixed"), dict(cycle=3), dict(transfer="mean"), dict(nu_l=2),
                  dict(smoother="rbgs")):
        with pytest.raises(binding.M1Error):
            binding.Plan3(prob, to_dev(sig), dict(omega=OMEGA, **extra))


STAGE_SHAPES = [(100, 6, 20, ALLKINDS), (70, 9, 17, ("periodic",) * 6), (64, 8, 16, MIXED),
                (33, 5, 3, ("periodic", "periodic", "dirichlet", "neumann", "reflective", "dirichlet"))]


@pytest.mark.parametrize("shape", range(len(STAGE_SHAPES)))
def test_staged_operations_equal_the_one_cell_forms(shape):
    """The staged (2.5-D blocked) apply, sweep and pseudo-time step give the one-cell kernels' bits on ragged
    tiles, periodic and non-periodic sides and chunks of z-planes that do not divide the grid; whole steps give
    the same bits and cycle counts."""
    nx, ny, nz, bcs = STAGE_SHAPES[shape]
    announce("3-D staged vs one-cell", nx, ny, nz)
    prob, v, sig = inputs.random_problem3(40 + shape, nx, ny, nz, bc_kinds=bcs, cfl=30.0, log10_sa=(-3, 2),
                                          wall_E=5.0)
    rng = np.random.default_rng(shape)
    u = inputs.random_state3(rng, nz, ny, nx, c=prob["c"], fmax=0.95)
    u[4] = rng.uniform(0.5, 1.5, size=u[4].shape)
    o = oracle.Oracle3(prob, sig)
    b, f = o.rhs(v), o.apply_A(v) * 1.05
    old = binding.tune_get("stage3")
    res = {}
    try:
        for staged in (2, 0):  # every staged form, then none
            binding.tune_set("stage3", staged)
            P = binding.Plan3(prob, to_dev(sig), dict(omega=OMEGA, rtol=1e-12, max_cycles=5000))
            vd = to_dev(v)
            info = P.step(vd, 1)
            res[staged] = (to_host(P.apply_A(0, to_dev(u))), to_host(P.sweep(to_dev(b), to_dev(u))),
                           to_host(P.pseudo_step(0, 0.7, to_dev(f), to_dev(u))), to_host(vd), info["cycles"])
    finally:
        binding.tune_set("stage3", old)
    for a, c in zip(res[2][:4], res[0][:4]):
        np.testing.assert_array_equal(a, c)
    assert res[2][4] == res[0][4]
    assert rel3(res[2][1], o.sweep(b, u, OMEGA), prob["c"]) <= 1e-13


PROLONG_SHAPES = [(100, 12, 10, ALLKINDS), (72, 18, 14, ("periodic",) * 6), (8, 8, 8, MIXED),
                  (66, 10, 8, ("periodic", "periodic", "neumann", "dirichlet", "periodic", "periodic"))]


@pytest.mark.parametrize("shape", range(len(PROLONG_SHAPES)))
def test_staged_prolongation_equals_the_one_cell_form(shape):
    """The correction with the coarse differences of a tile staged in LDS gives the one-thread-per-fine-cell
    kernel's bits on coarse tiles cut by the grid's end in every axis, periodic and other sides; whole steps
    give the same bits and cycle counts."""
    nx, ny, nz, bcs = PROLONG_SHAPES[shape]
    announce("3-D staged prolongation", nx, ny, nz)
    prob, v, sig = inputs.random_problem3(60 + shape, nx, ny, nz, bc_kinds=bcs, cfl=30.0, log10_sa=(-3, 2),
                                          wall_E=5.0)
    rng = np.random.default_rng(70 + shape)
    u = inputs.random_state3(rng, nz, ny, nx, c=prob["c"], fmax=0.9)
    u[4] = rng.uniform(0.5, 1.5, size=u[4].shape)
    o = oracle.Oracle3(prob, sig)
    u1 = o.restrict(u)
    uc = u1 * (1.0 + 0.6 * rng.normal(size=u1.shape))  # large coarse changes: the projection acts somewhere
    old = binding.tune_get("prolong3_lds")
    res = {}
    try:
        for lds in (1, 0):
            binding.tune_set("prolong3_lds", lds)
            P = binding.Plan3(prob, to_dev(sig), dict(omega=OMEGA, rtol=1e-12, max_cycles=5000))
            assert P.levels >= 2
            vd = to_dev(v)
            info = P.step(vd, 1)
            res[lds] = (to_host(P.prolong_project(0, to_dev(u), to_dev(uc), to_dev(u1))), to_host(vd), info["cycles"])
    finally:
        binding.tune_set("prolong3_lds", old)
    np.testing.assert_array_equal(res[1][0], res[0][0])
    np.testing.assert_array_equal(res[1][1], res[0][1])
    assert res[1][2] == res[0][2]
    ref = o.project(u, u + o.prolong(uc - u1), oracle.make_params())
    assert rel3(res[1][0], ref, prob["c"]) <= 1e-13
    assert not np.array_equal(ref, u + o.prolong(uc - u1))


@pytest.mark.parametrize("shape", [(1024, 1, 1), (2048, 2, 1), (512, 1, 17)])
def test_staged_sweeps_on_thin_grids(shape):
    """Staged sweeps on levels one or two cells thick launch more blocks than the one-cell kernels' 256-cell
    blocks; the first sweep of each cycle writes one norm partial per block, so the plan holds as many.  Whole
    steps against the oracle with every stencil operation staged."""
    nx, ny, nz = shape
    announce("3-D staged thin grid", nx, ny, nz)
    prob, v, sig = inputs.random_problem3(80 + nx + ny + nz, nx, ny, nz, bc_kinds=MIXED, cfl=20.0, log10_sa=(-3, 2),
                                          wall_E=5.0)
    params = dict(omega=OMEGA, rtol=1e-12, max_cycles=20000)
    ref, io = oracle.Oracle3(prob, sig).step(v, 2, oracle.make_params(**params))
    assert io["status"] == 0
    old = binding.tune_get("stage3")
    try:
        got = {}
        for staged in (2, 0):
            binding.tune_set("stage3", staged)
            P = binding.Plan3(prob, to_dev(sig), params)
            vd = to_dev(v)
            info = P.step(vd, 2)
            assert info["status"] == 0, info
            assert abs(info["cycles"] - io["cycles"]) <= 2, (staged, info["cycles"], io["cycles"])
            got[staged] = to_host(vd)
            assert rel3(got[staged], ref, prob["c"]) <= 1e-10, staged
    finally:
        binding.tune_set("stage3", old)
    assert rel3(got[2], got[0], prob["c"]) <= 1e-12
