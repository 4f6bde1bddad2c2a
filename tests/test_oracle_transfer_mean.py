"""Pins of the oracle's alternative grid-transfer pair (CPU only).

Sect. 6.3 names the restriction and prolongation operators as a choice that
changes the speed of the method.  The alternative built here is the one native
to cell-centred finite volumes: coarse cell I is the union of fine cells 2I and
2I+1 along each axis, the prolongation gives both its value (piecewise
constant) and the restriction is R = 2^-d P^T, the mean of the 2^d cells, as
Sect. 4.2 builds its full-weighting R from its P.  Pins:

* both operators against brute force (numpy reshape-mean and repeat) on 1-D and
  2-D grids of every side kind (they read no ghost);
* R = P^T / 2^d exactly and R P = I (the coarse values come back);
* rows are convex (admissible states stay admissible);
* cycles with the pair keep admissibility, differ from full weighting, leave the
  discrete solution fixed and converge to the dense Newton root: the transfer
  changes how fast the cycle converges, not its answer.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2208_14703_amd import inputs

BCS = [("periodic",) * 4, ("dirichlet", "reflective", "neumann", "reflective")]


def grid(dim, nx, ny, bcs):
    prob = inputs.grid_problem(dim, nx, ny if dim == 2 else 1, 5.0, [dict(kind=k) for k in bcs])
    return oracle.Oracle(prob)


def matrices(o, dim, nx, ny):
    nyf = ny if dim == 2 else 1
    nyc = ny // 2 if dim == 2 else 1
    nf, nc = nx * nyf, (nx // 2) * nyc
    P, R = np.zeros((nf, nc)), np.zeros((nc, nf))
    for m in range(nc):
        x = np.zeros((1, nyc, nx // 2))
        x.flat[m] = 1.0
        P[:, m] = o.prolong(x, transfer="mean").ravel()
    for m in range(nf):
        x = np.zeros((1, nyf, nx))
        x.flat[m] = 1.0
        R[:, m] = o.restrict(x, transfer="mean").ravel()
    return P, R


@pytest.mark.parametrize("bcs", BCS)
@pytest.mark.parametrize("dim,nx,ny", [(1, 16, 1), (2, 12, 8)])
def test_mean_and_constant_against_brute_force(dim, nx, ny, bcs):
    o = grid(dim, nx, ny, bcs)
    rng = np.random.default_rng(3)
    nyf = ny if dim == 2 else 1
    x = rng.normal(size=(3, nyf, nx))
    if dim == 2:
        want = x.reshape(3, ny // 2, 2, nx // 2, 2).mean(axis=(2, 4))
    else:
        want = x.reshape(3, 1, nx // 2, 2).mean(axis=3)
    np.testing.assert_allclose(o.restrict(x, transfer="mean"), want, rtol=1e-15, atol=1e-15)
    xc = rng.normal(size=want.shape)
    up = np.repeat(xc, 2, axis=2)
    if dim == 2:
        up = np.repeat(up, 2, axis=1)
    np.testing.assert_array_equal(o.prolong(xc, transfer="mean"), up)


@pytest.mark.parametrize("bcs", BCS)
@pytest.mark.parametrize("dim,nx,ny", [(1, 16, 1), (2, 8, 8)])
def test_restriction_is_scaled_transpose_and_inverts_the_prolongation(dim, nx, ny, bcs):
    o = grid(dim, nx, ny, bcs)
    P, R = matrices(o, dim, nx, ny)
    np.testing.assert_array_equal(R, P.T / 2 ** dim)
    np.testing.assert_array_equal(R @ P, np.eye(R.shape[0]))
    for M in (P, R):
        assert np.all(M >= 0)
        np.testing.assert_array_equal(M.sum(axis=1), 1.0)


def test_pair_differs_from_full_weighting():
    o = grid(2, 8, 8, BCS[1])
    x = np.random.default_rng(4).normal(size=(1, 8, 8))
    assert np.abs(o.restrict(x, transfer="mean") - o.restrict(x)).max() > 1e-3
    xc = np.random.default_rng(5).normal(size=(1, 4, 4))
    assert np.abs(o.prolong(xc, transfer="mean") - o.prolong(xc)).max() > 1e-3


@pytest.mark.parametrize("cycle", ["V", "W"])
def test_cycles_with_the_pair_reach_the_newton_root(cycle):
    prob, v, sig = inputs.random_problem(760, 2, 16, 16, bc_kinds=BCS[1], cfl=50.0, log10_sa=(-3, 2))
    o = oracle.Oracle(prob, sig)
    b = o.rhs(v)
    p = oracle.make_params(omega=0.8, transfer="mean", cycle=cycle)
    u = o.vcycle(b, v, 0.05, p)
    assert np.all(u[0] > 0) and np.all(np.hypot(u[1], u[2]) <= prob["c"] * u[0] * (1 + 1e-14))
    assert np.abs(u - o.vcycle(b, v, 0.05, oracle.make_params(omega=0.8, cycle=cycle))).max() > 1e-8
    root, _ = dense.newton_solve(v, b, sig, prob)
    scale = np.abs(root).max()
    np.testing.assert_allclose(o.vcycle(b, root, 0.1, p), root, rtol=0, atol=1e-12 * scale)
    got, info = o.step(v, 1, oracle.make_params(omega=0.8, rtol=1e-14, max_cycles=20000, transfer="mean",
                                                 cycle=cycle))
    assert info["status"] == 0
    np.testing.assert_allclose(got, root, rtol=0, atol=1e-12 * scale)
    print(f"{cycle} with the mean/constant pair: {info['cycles']} cycles")
