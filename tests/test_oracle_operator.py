"""Pins of the oracle's discrete operator and converged solve, against closed forms (CPU only).

Each test fixes a special case whose answer is known without the oracle:
  * the equilibrium fixed point;
  * free streaming, which reduces to implicit upwind and is solved by numpy.linalg;
  * a 2-D beam, which reduces to upwind plus transverse Rusanov diffusion (scipy sparse solve);
  * the thick scattering limit, the discrete heat equation;
  * a uniform gas-radiation exchange, solved by scipy's brentq;
  * conservation of E + C_v T;
  * a dense Newton solve on tiny grids (independent numpy operator).
A dropped term, a wrong sign or a transposed index in the oracle fails at least one.
"""
import numpy as np
import pytest
import scipy.optimize
import scipy.sparse
import scipy.sparse.linalg

import oracle
from oracle import dense
from paper_2208_14703_amd import inputs

EPS = np.finfo(float).eps


def solve(prob, v, sig, rtol=1e-13, **kw):
    o = oracle.Oracle(prob, sig)
    kw.setdefault("omega", 0.8)
    out, info = o.step(v, 1, oracle.make_params(rtol=rtol, max_cycles=20000, **kw))
    assert info["status"] == 0, info
    return o, out, info


# ------------------------------------------------------------------ equilibrium
@pytest.mark.parametrize("bc", ["periodic", "reflective", "neumann"])
def test_equilibrium_is_a_fixed_point(bc):
    prob = inputs.grid_problem(2, 16, 8, 30.0, inputs.bc_all(bc), a_r=0.7, c_v=2.0, c=1.5)
    rng = np.random.default_rng(3)
    sig = inputs.block_opacity(rng, 8, 16, 4, (-2, 2), (0, 1))
    T = 1.3
    v = np.zeros((4, 8, 16))
    v[0] = prob["a_r"] * T ** 4
    v[3] = T
    o = oracle.Oracle(prob, sig)
    b = o.rhs(v)
    r = o.residual(b, v)
    assert np.abs(r).max() <= 8 * EPS * v[0].max() * 100  # alpha ~ 100: rounding of a E - S_E
    np.testing.assert_allclose(o.sweep(b, v, 1.0), v, rtol=8 * EPS * 100, atol=8 * EPS * 100)
    p = oracle.make_params(levels=0)
    np.testing.assert_allclose(o.vcycle(b, v, 1e-3, p), v, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------------ free streaming (linear special case)
@pytest.mark.parametrize("direction", [+1, -1])
def test_free_streaming_1d_is_implicit_upwind(direction):
    # sigma = 0 and F = +-cE everywhere: the closure gives P = E, the right (left)
    # operator vanishes and the E row is implicit upwind; F = +-cE is preserved.
    n, cfl = 64, 7.5
    prob = inputs.grid_problem(1, n, 1, cfl, inputs.bc_all("periodic"))
    x = (np.arange(n) + 0.5) / n
    En = 1.0 + 0.8 * np.exp(-((x - 0.3) ** 2) / 0.005)
    v = np.zeros((4, 1, n))
    v[0, 0], v[1, 0], v[3] = En, direction * En, 1.0
    sig = np.zeros((2, 1, n))
    _, out, _ = solve(prob, v, sig)
    alpha = cfl
    M = (1 + alpha) * np.eye(n) - alpha * np.roll(np.eye(n), -direction, axis=1)  # couples E_{i-direction}
    E_ref = np.linalg.solve(M, En)
    np.testing.assert_allclose(out[0, 0], E_ref, rtol=1e-12, atol=0)
    np.testing.assert_allclose(out[1, 0], direction * E_ref, rtol=1e-12, atol=0)


def test_free_streaming_jacobi_sweep_is_classical_jacobi():
    # In the linear special case one nonlinear Jacobi sweep is one classical
    # Jacobi iteration of the upwind matrix (remark after the rows of A, Sect. 3.1).
    n, alpha = 32, 5.0
    prob = inputs.grid_problem(1, n, 1, alpha, inputs.bc_all("periodic"))
    rng = np.random.default_rng(4)
    En = rng.uniform(1, 2, n)
    Ek = rng.uniform(1, 2, n)
    v = np.zeros((4, 1, n))
    v[0, 0], v[1, 0], v[3] = Ek, Ek, 1.0
    b = np.zeros((4, 1, n))
    b[0, 0], b[1, 0], b[3] = En, En, 1.0
    o = oracle.Oracle(prob, np.zeros((2, 1, n)))
    out = o.sweep(b, v, 1.0)
    np.testing.assert_allclose(out[0, 0], (En + alpha * np.roll(Ek, 1)) / (1 + alpha), rtol=1e-14)


def test_free_streaming_2d_beam_along_x():
    # F = (cE, 0): x is pure upwind, y keeps the Rusanov diffusion (alpha_y / 2).
    nx, ny, cfl = 16, 8, 6.0
    prob = inputs.grid_problem(2, nx, ny, cfl, inputs.bc_all("periodic"), length=1.0)
    prob["hy"] = prob["hx"] / 2  # anisotropic cells: alpha_y = 2 alpha_x catches an x/y swap
    ax, ay = prob["c"] * prob["dt"] / prob["hx"], prob["c"] * prob["dt"] / prob["hy"]
    rng = np.random.default_rng(5)
    En = rng.uniform(1, 3, (ny, nx))
    v = np.zeros((4, ny, nx))
    v[0], v[1], v[3] = En, En, 1.0
    _, out, _ = solve(prob, v, np.zeros((2, ny, nx)))
    N = nx * ny
    idx = np.arange(N).reshape(ny, nx)
    A = scipy.sparse.lil_matrix((N, N))
    for j in range(ny):
        for i in range(nx):
            k = idx[j, i]
            A[k, k] += 1 + ax + ay
            A[k, idx[j, (i - 1) % nx]] -= ax
            A[k, idx[(j - 1) % ny, i]] -= ay / 2
            A[k, idx[(j + 1) % ny, i]] -= ay / 2
    E_ref = scipy.sparse.linalg.spsolve(A.tocsr(), En.ravel()).reshape(ny, nx)
    np.testing.assert_allclose(out[0], E_ref, rtol=1e-12)
    np.testing.assert_allclose(out[1], E_ref, rtol=1e-12)
    assert np.abs(out[2]).max() <= 1e-12 * E_ref.max()


# ------------------------------------------------------------------ thick limits
def test_thick_scattering_limit_is_discrete_heat_equation():
    # sigma_s -> infinity, sigma_a = 0: F = O(1/sigma_s) and E solves
    # (1 + a) E_i - (a/2)(E_{i-1} + E_{i+1}) = E^n_i  (the scheme is not
    # asymptotic preserving; the error must fall like 1/sigma_s).
    n, cfl = 32, 4.0
    prob = inputs.grid_problem(1, n, 1, cfl, inputs.bc_all("periodic"))
    x = (np.arange(n) + 0.5) / n
    En = 1.0 + 0.5 * np.sin(2 * np.pi * x)
    v = np.zeros((4, 1, n))
    v[0, 0], v[3] = En, 1.0
    M = (1 + cfl) * np.eye(n) - cfl / 2 * (np.roll(np.eye(n), 1, axis=1) + np.roll(np.eye(n), -1, axis=1))
    E_ref = np.linalg.solve(M, En)
    errs = []
    for ss in (1e3, 1e4, 1e5):
        sig = np.zeros((2, 1, n))
        sig[1] = ss
        _, out, _ = solve(prob, v, sig)
        errs.append(np.abs(out[0, 0] - E_ref).max())
        assert np.abs(out[1, 0]).max() < 50.0 / (ss * prob["dt"])
    assert errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5


def test_thick_absorption_limit_reaches_equilibrium():
    n, cfl = 16, 3.0
    prob = inputs.grid_problem(1, n, 1, cfl, inputs.bc_all("periodic"))
    rng = np.random.default_rng(6)
    v = np.zeros((4, 1, n))
    v[0, 0], v[3, 0] = rng.uniform(0.5, 2, n), rng.uniform(0.5, 1.5, n)
    gaps = []
    for sa in (1e2, 1e3, 1e4):
        sig = np.zeros((2, 1, n))
        sig[0] = sa
        _, out, _ = solve(prob, v, sig)
        gaps.append(np.abs(out[0, 0] - prob["a_r"] * out[3, 0] ** 4).max() / out[0, 0].max())
    assert gaps[1] < gaps[0] / 5 and gaps[2] < gaps[1] / 5


def test_uniform_gas_radiation_exchange_matches_brentq():
    # No gradients: each cell is E + ka (E - a_r T^4) = E^n, C_v T + ka (a_r T^4 - E) = C_v T^n.
    # Eliminate E and find T with a library root finder.
    prob = inputs.grid_problem(2, 8, 8, 10.0, inputs.bc_all("periodic"), a_r=0.3, c_v=2.5)
    En, Tn, sa = 3.0, 0.6, 7.0
    v = np.zeros((4, 8, 8))
    v[0], v[3] = En, Tn
    sig = np.zeros((2, 8, 8))
    sig[0] = sa
    _, out, _ = solve(prob, v, sig, rtol=1e-14)
    ka, ar, cv = prob["c"] * prob["dt"] * sa, prob["a_r"], prob["c_v"]

    def g(T):
        E = (En + ka * ar * T ** 4) / (1 + ka)
        return cv * T + ka * (ar * T ** 4 - E) - cv * Tn

    T = scipy.optimize.brentq(g, 1e-6, 10.0, xtol=1e-16, rtol=4 * EPS)
    E = (En + ka * ar * T ** 4) / (1 + ka)
    np.testing.assert_allclose(out[3], T, rtol=1e-12)
    np.testing.assert_allclose(out[0], E, rtol=1e-12)


# ------------------------------------------------------------------ conservation
@pytest.mark.parametrize("bc", ["periodic", "reflective"])
def test_operator_conserves_total_energy(bc):
    # Fluxes telescope and the exchange terms cancel between the E and T rows, so
    # sum(A_E + A_T) = sum(E + C_v T) for ANY state (periodic or reflective walls).
    prob, v, sig = inputs.random_problem(7, 2, 16, 16, bc_kinds=(bc,) * 4, cfl=30.0)
    o = oracle.Oracle(prob, sig)
    Av = o.apply_A(v)
    total = (v[0] + prob["c_v"] * v[3]).sum()
    assert abs((Av[0] + Av[3]).sum() - total) <= 1e-13 * 60 * total


@pytest.mark.parametrize("bc", ["periodic", "reflective"])
def test_solution_conserves_total_energy(bc):
    prob, v, sig = inputs.random_problem(8, 2, 16, 16, bc_kinds=(bc,) * 4, cfl=30.0)
    o, out, _ = solve(prob, v, sig)
    before = (v[0] + prob["c_v"] * v[3]).sum()
    after = (out[0] + prob["c_v"] * out[3]).sum()
    assert abs(after - before) <= 1e-10 * before


# ------------------------------------------------------------------ dense Newton on tiny grids
def test_dense_operator_matches_oracle_operator():
    for seed, dim, n, bcs in [(10, 1, 8, ("periodic",) * 4), (11, 2, 6, ("reflective", "dirichlet", "neumann", "periodic")),
                              (12, 2, 8, ("dirichlet", "reflective", "reflective", "reflective"))]:
        bcs = list(bcs)
        if bcs[2] == "periodic" or bcs[3] == "periodic":
            bcs[2] = bcs[3] = "periodic"
        prob, v, sig = inputs.random_problem(seed, dim, n, n, bc_kinds=bcs, cfl=15.0)
        o = oracle.Oracle(prob, sig)
        np.testing.assert_allclose(dense.apply_A(v, sig, prob), o.apply_A(v), rtol=1e-13, atol=1e-13 * np.abs(v).max() * 30)


CASES = [
    (20, 1, 8, ("periodic",) * 4, (-2, 1)),
    (21, 1, 16, ("dirichlet", "reflective", "periodic", "periodic"), (-2, 1)),
    (22, 1, 16, ("neumann", "dirichlet", "periodic", "periodic"), (-9, -9)),
    (23, 2, 4, ("periodic",) * 4, (-2, 1)),
    (24, 2, 8, ("reflective", "dirichlet", "neumann", "reflective"), (-2, 1)),
    (25, 2, 8, ("dirichlet", "reflective", "periodic", "periodic"), (-9, -9)),
]


@pytest.mark.parametrize("seed,dim,n,bcs,lsa", CASES)
def test_cycle_reaches_dense_newton_root(seed, dim, n, bcs, lsa):
    prob, v, sig = inputs.random_problem(seed, dim, n, n, bc_kinds=bcs, cfl=8.0, log10_sa=lsa, fmax=0.6)
    o, out, _ = solve(prob, v, sig, rtol=1e-14)
    b = o.rhs(v)
    ref, res = dense.newton_solve(v, b, sig, prob)
    assert o.norm(o.residual(b, ref)) <= 1e-15 * o.norm(o.residual(b, v))
    scale = np.abs(ref[0]).max()
    np.testing.assert_allclose(out[0], ref[0], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(out[1:3], ref[1:3], rtol=0, atol=1e-12 * prob["c"] * scale)
    np.testing.assert_allclose(out[3], ref[3], rtol=1e-12)
