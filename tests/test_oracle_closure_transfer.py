"""Pins of the oracle's single-cell closure and grid-transfer operators (CPU only).

The closure is pinned by its printed special values and by invariants:
  * chi(0) = 1/3 and chi(1) = 1;
  * the free-streaming and isotropic limits;
  * covariance under rotations of F;
  * unit trace of the full 3-D tensor.
The transfer operators are pinned by the matrices and stencils printed in
Sect. 4.2 (tests/golden/*).
"""
import os

import numpy as np
import pytest

import oracle
from paper_2208_14703_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    factor, rows, blocks, cur = 1.0, [], {}, None
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line.startswith("# factor"):
            factor = float(line.split()[-1])
        elif line.startswith("# ") and "_" in line and len(line.split()) == 2:
            cur = line.split()[1]
            blocks[cur] = []
        elif line and not line.startswith("#"):
            vals = [float(x) for x in line.split()]
            (blocks[cur] if cur else rows).append(vals)
    if blocks:
        return {k: factor * np.array(v) for k, v in blocks.items()}
    return factor * np.array(rows)


# ---------------------------------------------------------------- closure (Sect. 2.1)
def test_chi_special_values():
    assert oracle.chi(0.0) == pytest.approx(1.0 / 3.0, abs=1e-16)
    assert oracle.chi(1.0) == pytest.approx(1.0, abs=1e-16)
    f = np.linspace(0, 1, 101)
    chi = np.array([oracle.chi(x) for x in f])
    assert np.all(np.diff(chi) > 0)           # monotone between the diffusion and free-streaming limits
    assert np.all((chi >= 1 / 3 - 1e-16) & (chi <= 1 + 1e-16))


def test_closure_isotropic_limit():
    P = oracle.closure(2.5, 0.0, 0.0, c=3.0)
    np.testing.assert_allclose(P, [2.5 / 3, 0.0, 2.5 / 3], rtol=1e-15, atol=0)


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.1, np.pi / 2, 2.7, 4.0])
def test_closure_free_streaming_limit(theta):
    # f = 1: the pressure is E n (x) n (a beam), whatever the direction.
    c, E = 2.0, 1.7
    n = np.array([np.cos(theta), np.sin(theta)])
    P = oracle.closure(E, c * E * n[0], c * E * n[1], c=c)
    np.testing.assert_allclose(P, E * np.array([n[0] ** 2, n[0] * n[1], n[1] ** 2]), rtol=0, atol=4e-16 * E)


def test_closure_one_dimensional_is_chi_E():
    rng = np.random.default_rng(0)
    for _ in range(50):
        E, f, c = rng.lognormal(), rng.uniform(0, 1), rng.uniform(0.5, 2)
        P = oracle.closure(E, f * c * E, 0.0, c=c)
        assert P[0] == pytest.approx(oracle.chi(f) * E, rel=1e-14)
        assert P[1] == 0.0
        assert P[2] == pytest.approx(0.5 * (1 - oracle.chi(f)) * E, rel=1e-14)


def test_closure_rotation_covariance_and_trace():
    rng = np.random.default_rng(1)
    for _ in range(200):
        E, f, th, rot, c = rng.lognormal(), rng.uniform(0, 1), rng.uniform(0, 6.3), rng.uniform(0, 6.3), 1.3
        F = f * c * E * np.array([np.cos(th), np.sin(th)])
        R = np.array([[np.cos(rot), -np.sin(rot)], [np.sin(rot), np.cos(rot)]])
        p = oracle.closure(E, F[0], F[1], c=c)
        P = np.array([[p[0], p[1]], [p[1], p[2]]])
        q = oracle.closure(E, *(R @ F), c=c)
        Q = np.array([[q[0], q[1]], [q[1], q[2]]])
        np.testing.assert_allclose(Q, R @ P @ R.T, rtol=0, atol=1e-14 * E)
        # full 3-D tensor: Pzz = (1 - chi)/2 E, trace = E
        assert p[0] + p[2] + 0.5 * (1 - oracle.chi(f)) * E == pytest.approx(E, rel=1e-14)


# ---------------------------------------------------------------- grid transfer (Sect. 4.2)
def transfer_matrices(dim, n, bc="periodic"):
    """Dense P (fine x coarse) and R (coarse x fine) from the oracle, by unit vectors."""
    prob = inputs.grid_problem(dim, n, n, 1.0, inputs.bc_all(bc))
    o = oracle.Oracle(prob)
    nyf = n if dim == 2 else 1
    nyc = n // 2 if dim == 2 else 1
    nf, nc = n * nyf, (n // 2) * nyc
    P = np.zeros((nf, nc))
    R = np.zeros((nc, nf))
    for m in range(nc):
        x = np.zeros((1, nyc, n // 2))
        x.flat[m] = 1.0
        P[:, m] = o.prolong(x).ravel()
    for m in range(nf):
        x = np.zeros((1, nyf, n))
        x.flat[m] = 1.0
        R[:, m] = o.restrict(x).ravel()
    return P, R


def test_printed_prolongation_and_restriction_matrices():
    # With 8 fine / 4 coarse periodic cells and coarse cell 0 held at zero, fine
    # cells 1..7 and coarse cells 1..3 are exactly the printed example.
    P, R = transfer_matrices(1, 8)
    np.testing.assert_array_equal(P[1:8, 1:4], load_golden("prolongation_7x3.txt"))
    np.testing.assert_array_equal(R[1:4, 1:8], load_golden("restriction_3x7.txt"))


@pytest.mark.parametrize("dim,n", [(1, 16), (2, 8)])
def test_periodic_restriction_is_scaled_transpose(dim, n):
    P, R = transfer_matrices(dim, n)
    np.testing.assert_array_equal(R, P.T / 2 ** dim)


def test_2d_restriction_stencil_and_prolongation_weights():
    n = 8
    P, R = transfer_matrices(2, n)
    # interior coarse cell (I, J) = (2, 2): weights on fine (3..5) x (3..5)
    I = J = 2
    w = R[J * (n // 2) + I].reshape(n, n)[2 * J - 1:2 * J + 2, 2 * I - 1:2 * I + 2]
    np.testing.assert_array_equal(w, load_golden("restriction_2d_stencil.txt"))
    gold = load_golden("prolongation_2d_weights.txt")
    coarse = [(I, J), (I + 1, J), (I, J + 1), (I + 1, J + 1)]
    for key, (di, dj) in {"ieven_jeven": (0, 0), "iodd_jeven": (1, 0), "ieven_jodd": (0, 1),
                          "iodd_jodd": (1, 1)}.items():
        row = P[(2 * J + dj) * n + (2 * I + di)]
        got = [row[cj * (n // 2) + ci] for ci, cj in coarse]
        np.testing.assert_array_equal(got, gold[key][0])
        assert row.sum() == 1.0


@pytest.mark.parametrize("bc", ["reflective", "neumann", "dirichlet"])
@pytest.mark.parametrize("dim", [1, 2])
def test_nonperiodic_transfer_is_convex(dim, bc):
    # Away from periodic wrap a dropped stencil point renormalises the others:
    # every row has nonnegative weights summing to one (constants are preserved,
    # admissible states stay admissible).
    P, R = transfer_matrices(dim, 16 if dim == 1 else 8, bc)
    for M in (P, R):
        assert np.all(M >= 0)
        np.testing.assert_allclose(M.sum(axis=1), 1.0, rtol=0, atol=1e-15)
