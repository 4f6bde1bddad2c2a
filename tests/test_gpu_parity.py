"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Cases:
  * per operation (A, relaxed Jacobi sweep, pseudo-time step, restriction,
    prolongation with projection), 1e-13 relative;
  * one V-cycle, 1e-11;
  * converged time steps, 1e-10 relative in E and F (both sides at relative
    residual 1e-13);
  * full-size checks of the 1024^2 hot-wall workload (oracle residual of the GPU
    solution, a full-grid sweep compared element by element);
  * edge cases: ragged sizes, 1x1 grids, zero steps, non-admissible input, bad
    opacities, the cycle cap, determinism.
"""
import numpy as np
import pytest

import oracle
from paper_2208_14703_amd import binding, inputs
from tests.gpu_util import announce, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

OMEGA = 0.8


def plan_for(prob, sig, **params):
    params.setdefault("omega", OMEGA)
    return binding.Plan(prob, to_dev(sig), params)


def oracle_params(**kw):
    kw.setdefault("omega", OMEGA)
    return oracle.make_params(**kw)


BC_SETS = {
    "periodic": ("periodic",) * 4,
    "mixed": ("dirichlet", "reflective", "neumann", "reflective"),
    "wall": ("dirichlet", "reflective", "reflective", "reflective"),
}


# ------------------------------------------------------------------ single operations
@pytest.mark.parametrize("dim,nx,ny", [(2, 100, 37), (2, 64, 64), (1, 1000, 1), (2, 1, 1), (2, 3, 5)])
@pytest.mark.parametrize("bcs", ["periodic", "mixed"])
def test_apply_and_sweep_parity(dim, nx, ny, bcs):
    announce("apply/sweep", dim, nx, ny, bcs)
    kinds = BC_SETS[bcs]
    prob, v, sig = inputs.random_problem(1, dim, nx, ny, bc_kinds=kinds, cfl=40.0, fmax=1.0)
    o = oracle.Oracle(prob, sig)
    P = plan_for(prob, sig, levels=1)
    vd = to_dev(v)
    A = to_host(P.apply_A(0, vd))
    Ao = o.apply_A(v)
    scale = np.abs(Ao).max()
    assert np.abs(A - Ao).max() <= 1e-13 * scale
    b = o.rhs(inputs.random_problem(2, dim, nx, ny, bc_kinds=kinds, cfl=40.0)[1])
    for omega in (1.0, OMEGA):
        P2 = plan_for(prob, sig, levels=1, omega=omega)
        g = to_host(P2.sweep(to_dev(b), vd))
        assert rel_err(g, o.sweep(b, v, omega), prob["c"]) <= 1e-13
    norm, r = P.residual(vd, to_dev(b / np.array([1, 1, 1, prob["c_v"]])[:, None, None]), want_r=True)
    ro = o.residual(b, v)
    assert np.abs(to_host(r) - ro).max() <= 1e-13 * np.abs(Ao).max()
    assert norm == pytest.approx(o.norm(ro), rel=1e-12)


@pytest.mark.parametrize("nx,ny", [(100, 37), (64, 64), (1, 1), (3, 5), (130, 70), (65, 9), (64, 17)])
@pytest.mark.parametrize("bcs", ["periodic", "mixed", "wall"])
def test_lds_sweep_matches_one_cell_sweep(nx, ny, bcs):
    """The LDS-staged finest sweep (64 x rows tiles, every closure evaluated
    once) gives the one-cell-per-thread sweep's result to the bit: ragged tiles
    in both directions, one-cell domains, every kind of side."""
    announce("lds sweep", nx, ny, bcs)
    kinds = BC_SETS[bcs]
    prob, v, sig = inputs.random_problem(4, 2, nx, ny, bc_kinds=kinds, cfl=40.0, fmax=1.0)
    b = oracle.Oracle(prob, sig).rhs(inputs.random_problem(5, 2, nx, ny, bc_kinds=kinds, cfl=40.0)[1])
    vd, bd = to_dev(v), to_dev(b)
    old = binding.tune_get("sweep_rows")
    try:
        res = {}
        for rows in (0, 4, 8, 16):
            binding.tune_set("sweep_rows", rows)
            for omega in (1.0, OMEGA):
                P = plan_for(prob, sig, levels=1, omega=omega)
                res[rows, omega] = to_host(P.sweep(bd, vd))
    finally:
        binding.tune_set("sweep_rows", old)
    for rows in (4, 8, 16):
        for omega in (1.0, OMEGA):
            np.testing.assert_array_equal(res[rows, omega], res[0, omega])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nx,ny", [(100, 37), (64, 64), (1, 1), (3, 5), (130, 70), (65, 9), (64, 17), (200, 3)])
@pytest.mark.parametrize("bcs", ["periodic", "mixed", "wall", "xper"])
def test_sweep_pair_matches_two_sweeps(nx, ny, bcs, precision):
    """Two finest sweeps in one launch (the first sweep's iterate kept in LDS,
    its ring of ghosts rebuilt from it) give the sweeps launched one by one, to
    the bit, in FP64 and for the mixed-precision correction sweeps: one-level
    cycles of 2, 3 and 4 sweeps (FP64: one pair, a pair and a single, two
    pairs; mixed, whose first sweep starts from a zero correction: a single,
    then pairs) on ragged tiles, one-cell domains and every kind of side,
    periodic in one direction only included."""
    announce("sweep pair", nx, ny, bcs, precision)
    kinds = BC_SETS.get(bcs, ("periodic", "periodic", "dirichlet", "reflective"))
    prob, v, sig = inputs.random_problem(6, 2, nx, ny, bc_kinds=kinds, cfl=40.0, fmax=1.0)
    vn = inputs.random_problem(7, 2, nx, ny, bc_kinds=kinds, cfl=40.0)[1]
    vnd = to_dev(vn)
    old = binding.tune_get("pair_rows")
    try:
        res = {}
        for rows in (0, 4, 8, 16):
            binding.tune_set("pair_rows", rows)
            for nu0 in (2, 3, 4):
                for omega in (1.0, OMEGA):
                    P = plan_for(prob, sig, levels=1, omega=omega, nu0=nu0, precision=precision)
                    vd = to_dev(v)
                    P.vcycle(vd, vnd, 0.5)
                    res[rows, nu0, omega] = to_host(vd)
    finally:
        binding.tune_set("pair_rows", old)
    for (rows, nu0, omega), x in res.items():
        assert np.all(np.isfinite(x))
        np.testing.assert_array_equal(x, res[0, nu0, omega])


@pytest.mark.parametrize("case", ["hot1024", "periodic1024x768"])
def test_sweep_pair_full_size(case):
    """At the benchmark's size (1024^2 hot wall: a Dirichlet wall and
    reflective sides) and on a periodic 1024 x 768 grid, two and three
    sweeps through m1_sweeps are the same to the bit with the pair launch off
    and at 4, 8 and 16 tile rows."""
    announce("sweep pair full size", case)
    if case == "hot1024":
        prob, v, sig, _ = inputs.hot_wall_2d(n=1024)
        w = v.copy()
        w[0] *= 1.5  # a right-hand side away from the state
    else:
        prob, v, sig = inputs.random_problem(41, 2, 1024, 768, cfl=100.0, block=32)
        w = inputs.random_problem(42, 2, 1024, 768, cfl=100.0, block=32)[1]
    b = w.copy()
    b[3] *= prob["c_v"]
    vd, bd = to_dev(v), to_dev(b)
    P = plan_for(prob, sig, levels=1)
    old = binding.tune_get("pair_rows")
    try:
        res = {}
        for rows in (0, 4, 8, 16):
            binding.tune_set("pair_rows", rows)
            for n in (2, 3):
                res[rows, n] = to_host(P.sweeps(bd, vd, n))
    finally:
        binding.tune_set("pair_rows", old)
    for (rows, n), x in res.items():
        np.testing.assert_array_equal(x, res[0, n])


@pytest.mark.parametrize("levels,nu0,sweep_rows", [(1, 3, 4), (1, 2, 4), (1, 1, 4), (0, 2, 0), (0, 4, 0),
                                                    (0, 3, 4), (0, 2, 4)])
def test_step_result_with_and_without_sweep_pairs(levels, nu0, sweep_rows):
    """m1_step returns the same result, to the bit and with the same cycle
    counts, with the two-sweep launch on and off.  The launches per cycle
    differ (one for two sweeps), so the buffer holding the iterate after a
    cycle differs too: one-level cycles with odd and even sweep counts, and
    full cycles with the correction not fused into the first post-sweep
    (staged sweeps off) and even counts, over two steps."""
    announce("step with sweep pairs", levels, nu0, sweep_rows)
    prob, v, sig = inputs.random_problem(21, 2, 96, 80, cfl=2.0 if levels == 1 else 50.0, block=8)
    old = {k: binding.tune_get(k) for k in ("pair_rows", "sweep_rows")}
    try:
        res = {}
        for pair in (0, 8):
            binding.tune_set("pair_rows", pair)
            binding.tune_set("sweep_rows", sweep_rows)
            P = plan_for(prob, sig, levels=levels, nu0=nu0, rtol=1e-8, max_cycles=20000)
            vd = to_dev(v)
            info = P.step(vd, 2)
            res[pair] = (to_host(vd), info["cycles"], info["status"])
    finally:
        for k, val in old.items():
            binding.tune_set(k, val)
    assert res[0][2] == 0 and res[8][2] == 0
    assert res[0][1] == res[8][1]
    np.testing.assert_array_equal(res[8][0], res[0][0])


@pytest.mark.parametrize("omega", [1.0, OMEGA])
def test_local_solve_extremes(omega):
    """One sweep against the oracle, cell by cell, where the local Newton
    solve is hardest: absorption opacity log-uniform over 1e-8 .. 1e8 per
    cell (the quartic from linear- to T^4-dominated), temperatures over
    1e-2 .. 1e2, and a right-hand side drawn independently, so that the
    guess (the current temperature) is far below or far above the root and
    the upper bound both starts and clamps the iteration.  Per-cell relative
    error <= 1e-12 in E and T (F scaled by cE + |F|)."""
    announce("local solve extremes", omega)
    nx = ny = 96
    prob, v, sig = inputs.random_problem(31, 2, nx, ny, cfl=50.0, block=1)
    rng = np.random.default_rng(32)
    sig[0] = 10.0 ** rng.uniform(-8.0, 8.0, size=(ny, nx))
    v[3] = 10.0 ** rng.uniform(-2.0, 2.0, size=(ny, nx))
    w = inputs.random_problem(33, 2, nx, ny, cfl=50.0, block=1)[1]
    w[3] = 10.0 ** rng.uniform(-2.0, 2.0, size=(ny, nx))
    o = oracle.Oracle(prob, sig)
    b = o.rhs(w)
    ref = o.sweep(b, v, omega)
    P = plan_for(prob, sig, levels=1, omega=omega)
    got = to_host(P.sweep(to_dev(b), to_dev(v)))
    assert np.all(np.isfinite(got))
    c = prob["c"]
    eE = np.abs(got[0] - ref[0]) / np.abs(ref[0])
    eF = np.abs(got[1:3] - ref[1:3]) / (c * np.abs(ref[0]) + np.abs(ref[1:3]))
    eT = np.abs(got[3] - ref[3]) / np.abs(ref[3])
    assert eE.max() <= 1e-12 and eF.max() <= 1e-12 and eT.max() <= 1e-12, (eE.max(), eF.max(), eT.max())


@pytest.mark.parametrize("nx,ny,bcs", [(100, 37, "mixed"), (64, 64, "periodic"), (130, 70, "wall"), (3, 5, "xper"),
                                        (260, 52, "periodic"), (200, 90, "mixed")])
def test_sweeps_match_chained_sweeps(nx, ny, bcs):
    """m1_sweeps(n) -- fused pairs, and one single sweep for odd n -- gives n
    chained m1_sweep calls to the bit, with the pair launch on and off, and
    leaves its input alone; two sweeps agree with the oracle's two sweeps.
    The wider grids hold tiles whose halo touches no side (their kernels skip
    the side logic) beside tiles on every side."""
    announce("sweeps", nx, ny, bcs)
    kinds = BC_SETS.get(bcs, ("periodic", "periodic", "dirichlet", "reflective"))
    prob, v, sig = inputs.random_problem(8, 2, nx, ny, bc_kinds=kinds, cfl=40.0, fmax=1.0)
    o = oracle.Oracle(prob, sig)
    b = o.rhs(inputs.random_problem(9, 2, nx, ny, bc_kinds=kinds, cfl=40.0)[1])
    vd, bd = to_dev(v), to_dev(b)
    P = plan_for(prob, sig, levels=1)
    chain = [vd]
    for _ in range(5):
        chain.append(P.sweep(bd, chain[-1]))
    old = binding.tune_get("pair_rows")
    try:
        for rows in (0, 8):
            binding.tune_set("pair_rows", rows)
            for n in range(1, 6):
                np.testing.assert_array_equal(to_host(P.sweeps(bd, vd, n)), to_host(chain[n]))
    finally:
        binding.tune_set("pair_rows", old)
    np.testing.assert_array_equal(to_host(vd), v)
    two = o.sweep(b, o.sweep(b, v, OMEGA), OMEGA)
    assert rel_err(to_host(chain[2]), two, prob["c"]) <= 2e-13


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nx,ny", [(96, 80), (100, 36), (66, 10), (130, 70), (64, 64), (258, 130)])
@pytest.mark.parametrize("bcs", ["periodic", "mixed", "wall"])
def test_fused_residual_restriction_matches_two_kernels(nx, ny, bcs, precision):
    """The finest residual restricted as it is formed (one launch) gives the
    stored-then-restricted path's cycle to the bit: odd coarse sizes, ragged
    coarse tiles, periodic wrap and dropped points at every kind of side, and
    tiles that touch no side (258 x 130: three columns of them); one V-cycle and
    a whole time step."""
    announce("fused residual/restriction", nx, ny, bcs, precision)
    kinds = BC_SETS[bcs]
    prob, v, sig = inputs.random_problem(6, 2, nx, ny, bc_kinds=kinds, cfl=60.0, fmax=0.9)
    vn = inputs.random_problem(7, 2, nx, ny, bc_kinds=kinds, cfl=60.0, fmax=0.9)[1]
    old = binding.tune_get("residual_restrict")
    res = {}
    try:
        for on in (0, 1):
            binding.tune_set("residual_restrict", on)
            P = plan_for(prob, sig, rtol=1e-10, max_cycles=20000, precision=precision)
            assert P.levels >= 2
            vd = to_dev(v)
            P.vcycle(vd, to_dev(vn), 1e-2)
            w = to_dev(v)
            info = P.step(w, 1)
            res[on] = (to_host(vd), to_host(w), info["cycles"])
    finally:
        binding.tune_set("residual_restrict", old)
    np.testing.assert_array_equal(res[1][0], res[0][0])
    np.testing.assert_array_equal(res[1][1], res[0][1])
    assert res[1][2] == res[0][2]


@pytest.mark.parametrize("dim,n", [(2, 64), (1, 512)])
@pytest.mark.parametrize("local", [1, 0])
def test_pseudo_step_parity(dim, n, local):
    announce("pseudo", dim, n, local)
    prob, v, sig = inputs.random_problem(3, dim, n, n, bc_kinds=BC_SETS["mixed"], cfl=60.0)
    o = oracle.Oracle(prob, sig)
    P = plan_for(prob, sig, pseudo_local=local)
    op = oracle_params(pseudo_local=local)
    g1 = o.coarse_grid()
    sig1 = o.restrict(sig)
    v1 = o.restrict(v)
    rng = np.random.default_rng(4)
    f = o.apply_A(v1, sigma=sig1, g=g1) + rng.normal(size=v1.shape) * np.abs(v1).max() * 3
    if dim == 1:
        f[2] = 0.0
    for dtau in (1e-3, 0.7, 50.0):
        got = to_host(P.pseudo_step(1, dtau, to_dev(f), to_dev(v1)))
        ref = o.pseudo_step(f, v1, dtau, params=op, sigma=sig1, g=g1)
        assert rel_err(got, ref, prob["c"]) <= 1e-12, dtau


@pytest.mark.parametrize("dim,n", [(2, 64), (1, 256)])
@pytest.mark.parametrize("bcs", ["periodic", "mixed"])
def test_restrict_and_prolong_project_parity(dim, n, bcs):
    announce("transfer", dim, n, bcs)
    prob, v, sig = inputs.random_problem(5, dim, n, n, bc_kinds=BC_SETS[bcs], cfl=10.0)
    o = oracle.Oracle(prob, sig)
    P = plan_for(prob, sig)
    got = to_host(P.restrict(0, to_dev(v)))
    assert rel_err(got, o.restrict(v), prob["c"]) <= 1e-15
    vc = o.restrict(v)
    rng = np.random.default_rng(6)
    uc = vc + rng.normal(size=vc.shape) * vc[0] * 0.7
    if dim == 1:
        uc[2] = 0.0
    w = v + o.prolong(uc - vc)
    ref = o.project(v, w, params=oracle_params())
    got = to_host(P.prolong_project(0, to_dev(v), to_dev(uc), to_dev(vc)))
    assert rel_err(got, ref, prob["c"]) <= 1e-13


@pytest.mark.parametrize("dim,nx,ny", [(2, 96, 80), (2, 136, 72), (2, 64, 64), (1, 512, 1)])
@pytest.mark.parametrize("bcs", ["periodic", "mixed", "wall"])
def test_residual_restriction_parity(dim, nx, ny, bcs):
    """m1_residual_restrict against the oracle's restriction of u and of
    rhs - A_l(u), on the finest level (rhs = b) and on level 1 (its own
    opacities and spacing), fused (one launch) and stored-then-restricted."""
    announce("residual restriction", dim, nx, ny, bcs)
    prob, v, sig = inputs.random_problem(8, dim, nx, ny, bc_kinds=BC_SETS[bcs], cfl=60.0, fmax=0.95)
    o = oracle.Oracle(prob, sig)
    rng = np.random.default_rng(9)
    u = v.copy()  # another admissible state: E and F scaled together (f unchanged), T perturbed
    u[:3] *= np.exp(rng.normal(size=u[0].shape) * 0.2)
    u[3] *= np.exp(rng.normal(size=u[0].shape) * 0.1)
    b = o.rhs(v)
    g1, sig1 = o.coarse_grid(), o.restrict(sig)
    u1 = o.restrict(u)
    f1 = o.apply_A(o.restrict(v), sigma=sig1, g=g1) + rng.normal(size=u1.shape) * np.abs(u1).max()
    if dim == 1:
        f1[2] = 0.0
    refs = [(o.restrict(u), o.restrict(b - o.apply_A(u))),
            (o.restrict(u1, g=g1), o.restrict(f1 - o.apply_A(u1, sigma=sig1, g=g1), g=g1))]
    old = binding.tune_get("residual_restrict")
    try:
        for fused in (1, 0):
            binding.tune_set("residual_restrict", fused)
            P = plan_for(prob, sig)
            assert P.levels >= 3
            for level, (uu, rhs) in enumerate(((u, b), (u1, f1))):
                vc, rc = P.residual_restrict(level, to_dev(uu), to_dev(rhs))
                assert rel_err(to_host(vc), refs[level][0], prob["c"]) <= 1e-14
                rscale = np.abs(refs[level][1]).max()
                assert np.abs(to_host(rc) - refs[level][1]).max() <= 1e-12 * rscale, (fused, level)
    finally:
        binding.tune_set("residual_restrict", old)


# ------------------------------------------------------------------ one V-cycle
@pytest.mark.parametrize("case", ["hot64", "logn64", "gauss256", "mixed32x64"])
def test_vcycle_parity(case):
    announce("vcycle", case)
    if case == "hot64":
        prob, v, sig, _ = inputs.hot_wall_2d(n=64)
    elif case == "logn64":
        prob, v, sig, _ = inputs.lognormal_2d(n=64)
    elif case == "gauss256":
        prob, v, sig, _ = inputs.gaussian_1d(n=256)
    else:
        prob, v, sig = inputs.random_problem(7, 2, 64, 64, bc_kinds=BC_SETS["mixed"], cfl=80.0)
    o = oracle.Oracle(prob, sig)
    P = plan_for(prob, sig)
    b = o.rhs(v)
    vd, vn = to_dev(v), to_dev(v)
    ref = v
    for cyc, dtau in enumerate((1e-3, 0.3, 5.0)):
        P.vcycle(vd, vn, dtau)
        ref = o.vcycle(b, ref, dtau, params=oracle_params())
        err = rel_err(to_host(vd), ref, prob["c"])
        assert err <= 1e-11, (cyc, err)


@pytest.mark.parametrize("m,nu_l,nu0,tiled", [(1, 1, 3, 1), (2, 1, 3, 1), (4, 1, 3, 1), (3, 2, 3, 1), (2, 2, 2, 1),
                                              (3, 1, 2, 1), (1, 1, 1, 1), (2, 1, 3, 0), (3, 1, 2, 0)])
def test_vcycle_parity_smoothing_counts(m, nu_l, nu0, tiled):
    """Three V-cycles against the oracle's with other smoothing counts than
    the paper's: pseudo-time steps per coarse smoothing m = 1, 2, 4, two
    Jacobi sweeps per pseudo-time step, even and odd finest-level sweep
    counts, with the one-launch smoothing legs (m <= 3) and without; each
    count changes which buffers the legs end in."""
    announce("vcycle smoothing counts", m, nu_l, nu0, tiled)
    prob, v, sig = inputs.random_problem(7, 2, 128, 128, bc_kinds=BC_SETS["mixed"], cfl=80.0, block=8)
    params = dict(pseudo_steps=m, nu_l=nu_l, nu0=nu0)
    o = oracle.Oracle(prob, sig)
    old = binding.tune_get("tiled_max_cells")
    binding.tune_set("tiled_max_cells", 65536 if tiled else 0)
    try:
        P = plan_for(prob, sig, **params)  # the tiled bound is read when the plan is created
    finally:
        binding.tune_set("tiled_max_cells", old)
    b = o.rhs(v)
    vd, vn = to_dev(v), to_dev(v)
    ref = v
    for cyc, dtau in enumerate((1e-3, 0.3, 5.0)):
        P.vcycle(vd, vn, dtau)
        ref = o.vcycle(b, ref, dtau, params=oracle_params(**params))
        err = rel_err(to_host(vd), ref, prob["c"])
        assert err <= 1e-11, (cyc, err)


# ------------------------------------------------------------------ converged solves
@pytest.mark.parametrize("case", ["gauss256", "hot128", "logn128", "mixed64_2steps", "gauss256_jacobi"])
def test_converged_step_parity(case):
    announce("converged", case)
    steps, levels = 1, 0
    if case.startswith("gauss256"):
        prob, v, sig, _ = inputs.gaussian_1d(n=256)
        if case.endswith("jacobi"):
            levels = 1
    elif case == "hot128":
        prob, v, sig, _ = inputs.hot_wall_2d(n=128)
    elif case == "logn128":
        prob, v, sig, _ = inputs.lognormal_2d(n=128)
    else:
        prob, v, sig = inputs.random_problem(8, 2, 64, 64, bc_kinds=BC_SETS["mixed"], cfl=50.0)
        steps = 2
    rtol = 1e-13
    o = oracle.Oracle(prob, sig)
    ref, info_o = o.step(v, steps, oracle_params(rtol=rtol, levels=levels, max_cycles=40000))
    assert info_o["status"] == 0
    P = plan_for(prob, sig, rtol=rtol, levels=levels, max_cycles=40000)
    vd = to_dev(v)
    info = P.step(vd, steps)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-11  # rtol, or the rounding floor of A
    got = to_host(vd)
    sE = np.abs(ref[0]).max()
    assert np.abs(got[0] - ref[0]).max() / sE <= 1e-10
    assert np.abs(got[1:3] - ref[1:3]).max() / (prob["c"] * sE) <= 1e-10
    assert np.abs(got[3] - ref[3]).max() / np.abs(ref[3]).max() <= 1e-10
    print("cycles gpu/oracle", info["cycles"], info_o["cycles"], flush=True)


@pytest.mark.parametrize("case", ["gauss256", "hot128", "logn128", "hot128_literal", "hot128_paper"])
def test_cycle_counts_match_oracle(case):
    # same algorithm and readings on both sides: the cycle count to the workload's
    # tolerance agrees up to a rounding flip of the last stopping test
    announce("cycle counts", case)
    extra = {}
    if case == "gauss256":
        prob, v, sig, run = inputs.gaussian_1d(n=256)
    elif case.startswith("hot128"):
        prob, v, sig, run = inputs.hot_wall_2d(n=128)
        if case.endswith("literal"):
            extra = dict(dtau_rule="literal", eps_inc=1e-3, eps_dec=1e-5)
        if case.endswith("paper"):
            extra = dict(omega=1.0, max_cycles=3000)
    else:
        prob, v, sig, run = inputs.lognormal_2d(n=128)
    o = oracle.Oracle(prob, sig)
    ref, info_o = o.step(v, 1, oracle_params(rtol=run["rtol"], **extra))
    P = plan_for(prob, sig, rtol=run["rtol"], **extra)
    vd = to_dev(v)
    info = P.step(vd, 1)
    assert info["status"] == info_o["status"] == 0
    assert abs(info["cycles"] - info_o["cycles"]) <= 1, (info["cycles"], info_o["cycles"])
    assert info["dtau"] == pytest.approx(info_o["dtau"], rel=0.25)


# ------------------------------------------------------------------ full-size workload checks
def test_full_size_hot_wall_solution_satisfies_oracle_residual():
    announce("full 1024 hot wall, 1 step")
    prob, v, sig, run = inputs.hot_wall_2d(n=1024)
    P = plan_for(prob, sig, rtol=run["rtol"])
    vd = to_dev(v)
    info = P.step(vd, 1)
    assert info["status"] == 0
    got = to_host(vd)
    o = oracle.Oracle(prob, sig)
    b = o.rhs(v)
    rel = o.norm(o.residual(b, got)) / o.norm(o.residual(b, v))
    assert rel <= 1.001 * run["rtol"], rel
    E, F2, T = got[0], got[1] ** 2 + got[2] ** 2, got[3]
    assert np.all(E > 0) and np.all(T > 0) and np.all(np.sqrt(F2) <= prob["c"] * E * (1 + 1e-12))
    # one sweep of the full grid, element by element
    sw = to_host(P.sweep(to_dev(b), vd))
    assert rel_err(sw, o.sweep(b, got, OMEGA), prob["c"]) <= 1e-13


# ------------------------------------------------------------------ edge cases
def test_zero_steps_and_equilibrium():
    announce("edge: zero steps / equilibrium")
    prob = inputs.grid_problem(2, 32, 32, 50.0, inputs.bc_all("periodic"))
    v = np.zeros((4, 32, 32))
    v[0], v[3] = 1.0, 1.0
    sig = np.ones((2, 32, 32))
    P = plan_for(prob, sig)
    vd = to_dev(v)
    info = P.step(vd, 0)
    assert info["status"] == 0 and info["cycles"] == 0
    np.testing.assert_array_equal(to_host(vd), v)
    info = P.step(vd, 2)
    assert info["status"] == 0 and info["cycles"] == 0   # residual at the rounding level of A
    np.testing.assert_array_equal(to_host(vd), v)


def test_non_admissible_input_is_rejected_untouched():
    announce("edge: non-admissible input")
    prob, v, sig = inputs.random_problem(9, 2, 64, 48, cfl=10.0)
    v[0, 10, 7] = -1.0                      # cell 10*64 + 7 = 647
    v[1, 20, 3] = 5 * v[0, 20, 3]           # |F| > cE at a later cell
    P = plan_for(prob, sig, levels=1)
    vd = to_dev(v)
    with pytest.raises(binding.M1Error) as ei:
        P.step(vd, 1)
    assert ei.value.status == 2 and "647" in str(ei.value)
    np.testing.assert_array_equal(to_host(vd), v)
    v2 = inputs.random_problem(9, 2, 64, 48, cfl=10.0)[1]
    v2[3, 0, 5] = np.nan
    with pytest.raises(binding.M1Error):
        P.step(to_dev(v2), 1)


def test_bad_opacity_and_arguments_rejected():
    announce("edge: bad opacity / arguments")
    prob, v, sig = inputs.random_problem(10, 2, 32, 32)
    bad = sig.copy()
    bad[1, 3, 3] = -1.0
    with pytest.raises(binding.M1Error) as ei:
        plan_for(prob, bad)
    assert ei.value.status == 1
    odd = inputs.random_problem(10, 2, 30, 32)
    with pytest.raises(binding.M1Error):
        plan_for(odd[0], odd[2], levels=4)   # 30 cannot be halved three times


def test_cycle_cap_reports_no_convergence_with_admissible_state():
    announce("edge: max_cycles")
    prob, v, sig, _ = inputs.hot_wall_2d(n=64)
    P = plan_for(prob, sig, max_cycles=2, rtol=1e-12)
    vd = to_dev(v)
    info = P.step(vd, 1)
    assert info["status"] == 3 and info["cycles"] == 2
    got = to_host(vd)
    assert np.all(got[0] > 0) and np.all(got[3] > 0)
    assert np.all(np.sqrt(got[1] ** 2 + got[2] ** 2) <= prob["c"] * got[0] * (1 + 1e-12))


def test_deterministic():
    announce("edge: determinism")
    prob, v, sig, _ = inputs.lognormal_2d(n=128)
    outs = []
    for _ in range(2):
        P = plan_for(prob, sig)
        vd = to_dev(v)
        P.step(vd, 1)
        outs.append(to_host(vd))
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("bcs", ["periodic", "mixed", "wall"])
def test_tiled_smoothing_legs_match_one_step_kernels(bcs):
    """The LDS-tiled smoothing legs give the one-step kernels' results to the
    bit.  96x64 is not a power of two and its 48x32 level is tiled while 24x16
    is not (12x8 runs in the tail); every kind of side.  The solution also
    meets the oracle's."""
    announce("tiled legs", bcs)
    prob, v, sig = inputs.random_problem(21, 2, 96, 64, bc_kinds=BC_SETS[bcs], cfl=50.0, block=8)
    res = {}
    old = binding.tune_get("tiled_max_cells")
    try:
        for tiled in (65536, 0):
            binding.tune_set("tiled_max_cells", tiled)
            P = plan_for(prob, sig, rtol=1e-12, max_cycles=20000)
            assert P.level_dims(1) == (48, 32)
            vd = to_dev(v)
            info = P.step(vd, 2)
            assert info["status"] == 0
            res[tiled] = (to_host(vd), info)
    finally:
        binding.tune_set("tiled_max_cells", old)
    np.testing.assert_array_equal(res[65536][0], res[0][0])
    assert res[65536][1]["cycles"] == res[0][1]["cycles"]
    ref, info_o = oracle.Oracle(prob, sig).step(v, 2, oracle_params(rtol=1e-12, max_cycles=20000))
    assert info_o["status"] == 0
    assert rel_err(res[65536][0], ref, prob["c"]) <= 1e-9


@pytest.mark.parametrize("bcs", ["periodic", "mixed", "wall", "xper"])
def test_staged_pseudo_steps_match_one_cell(bcs):
    """The LDS-staged coarse pseudo-time step (2-D levels of at least 512 K
    cells, while the staged sweeps are on) gives the one-cell step's results
    to the bit: whole 2048 x 1024 FP64 solves, whose 1024 x 512 level takes the
    staged step, end in the same bits and cycles with sweep_rows 8 (staged)
    and 0 (one cell per thread)."""
    announce("staged pseudo steps", bcs)
    kinds = BC_SETS.get(bcs, ("periodic", "periodic", "dirichlet", "reflective"))
    prob, v, sig = inputs.random_problem(41, 2, 2048, 1024, bc_kinds=kinds, cfl=80.0, fmax=0.9)
    old = {k: binding.tune_get(k) for k in ("sweep_rows", "tiled_max_cells")}
    res = {}
    try:
        binding.tune_set("tiled_max_cells", 0)
        for rows in (0, 8):
            binding.tune_set("sweep_rows", rows)
            P = plan_for(prob, sig, rtol=1e-9, max_cycles=400)
            vd = to_dev(v)
            info = P.step(vd, 2)
            res[rows] = (to_host(vd), info)
    finally:
        for k, x in old.items():
            binding.tune_set(k, x)
    (a, ia), (b, ib) = res[0], res[8]
    assert ia["status"] == 0, ia
    assert (ia["cycles"], ia["rel_residual"]) == (ib["cycles"], ib["rel_residual"])
    np.testing.assert_array_equal(a.view(np.int64), b.view(np.int64))
