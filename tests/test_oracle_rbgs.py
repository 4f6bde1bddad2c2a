"""Pins of the oracle's red-black nonlinear Gauss-Seidel smoother (CPU only).

The paper names Gauss-Seidel as the alternative to the Jacobi smoother
(Sect. 6.3).  The red-black form updates the cells with i + j even from the
old iterate, then the others from that intermediate state.

* Prop. 1 carries over: each cell's update is the local solve of a Jacobi
  sweep with admissible neighbours, so every iterate stays admissible (also at
  f = 1, with relaxation or without).
* Young's theorem for a 2-cyclic (red-black) ordering: on the linearised
  system the asymptotic contraction factor of Gauss-Seidel is the square of
  Jacobi's, rho_GS = rho_J^2.  Near the diffusion limit (small flux, where the
  closure is nearly linear) the measured 2-D rates satisfy log rho_GS /
  log rho_J = 2 within the window's noise (1.91 .. 2.01 observed); a sweep
  that read the old iterate in its second half (plain Jacobi) gives 1.
* The fixed point does not depend on the smoother: a multigrid solve with
  red-black sweeps reaches the dense Newton root and the Jacobi-smoothed
  solution.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2208_14703_amd import inputs


def admissible(v, c):
    return bool(np.all(v[0] > 0) and np.all(v[3] > 0) and np.all(np.hypot(v[1], v[2]) <= c * v[0] * (1 + 4e-16 * 4)))


@pytest.mark.parametrize("fixed_f", [None, 1.0])
@pytest.mark.parametrize("omega", [1.0, 0.8])
def test_rb_sweep_keeps_admissibility(fixed_f, omega):
    for seed in range(4):
        bcs = [("periodic",) * 4, ("dirichlet", "reflective", "neumann", "reflective")][seed % 2]
        prob, v, sig = inputs.random_problem(500 + seed, 2, 12, 10, bc_kinds=bcs, cfl=300.0, fixed_f=fixed_f,
                                             log10_sa=(-3, 2))
        o = oracle.Oracle(prob, sig)
        b = o.rhs(v)
        u = inputs.random_state(np.random.default_rng(seed), 10, 12, fmax=1.0)
        for _ in range(6):
            u = o.rb_sweep(b, u, omega)
            assert admissible(u, prob["c"])


def contraction(o, b, v, sweep, n):
    """Asymptotic contraction factor of the residual over the last half of n sweeps."""
    norms = []
    u = v.copy()
    for _ in range(n):
        u = sweep(b, u)
        norms.append(o.norm(o.residual(b, u)))
    h = n // 2
    return (norms[-1] / norms[h]) ** (1.0 / (n - 1 - h))


@pytest.mark.parametrize("dim,nx,ny,nj", [(2, 16, 16, 100), (2, 24, 16, 120)])
def test_red_black_squares_the_jacobi_contraction(dim, nx, ny, nj):
    # thick scattering, no absorption: the discrete heat equation regime, flux small, closure nearly linear
    bcs = ("periodic",) * 4
    prob = inputs.grid_problem(dim, nx, ny, 2.0, [dict(kind=k) for k in bcs])
    ny_ = prob["ny"]
    sig = np.zeros((2, ny_, nx))
    sig[1] = 200.0
    rng = np.random.default_rng(2)
    v = np.zeros((4, ny_, nx))
    v[0] = 1.0 + 0.1 * rng.normal(size=(ny_, nx))
    v[3] = 1.0
    o = oracle.Oracle(prob, sig)
    b = o.rhs(v)
    rho_j = contraction(o, b, v, lambda bb, u: o.sweep(bb, u, 1.0), nj)
    rho_gs = contraction(o, b, v, lambda bb, u: o.rb_sweep(bb, u, 1.0), nj // 2)
    assert 0.5 < rho_j < 1.0
    ratio = np.log(rho_gs) / np.log(rho_j)  # 2 in the linear limit; the measured windows give 1.91 .. 2.01
    assert 1.85 < ratio < 2.15, (rho_j, rho_gs, ratio)


def test_rb_smoothed_solve_reaches_the_same_solution():
    prob, v, sig = inputs.random_problem(520, 2, 8, 8, bc_kinds=("dirichlet", "reflective", "periodic", "periodic"),
                                         cfl=20.0)
    o = oracle.Oracle(prob, sig)
    rb, info = o.step(v, 1, oracle.make_params(omega=1.0, rtol=1e-14, max_cycles=20000, smoother="rbgs"))
    assert info["status"] == 0
    jac, _ = o.step(v, 1, oracle.make_params(omega=0.8, rtol=1e-14, max_cycles=20000))
    root, _ = dense.newton_solve(v, o.rhs(v), sig, prob)
    scale = np.abs(root).max()
    np.testing.assert_allclose(rb, root, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(rb, jac, rtol=0, atol=1e-12 * scale)
