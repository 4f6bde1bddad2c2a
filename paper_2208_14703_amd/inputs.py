"""Seeded synthetic inputs for the implicit M1 solver.

This module is the only code shared by the GPU path and the CPU oracle. It holds
no arithmetic of the method itself, only problem descriptions: grids, time steps,
boundary conditions, opacity fields and initial states. Every draw comes from
``numpy.random.Generator(PCG64(seed))`` in a fixed order:
  1. per-block sigma_a (row-major over blocks);
  2. per-block sigma_s;
  3. per-cell E;
  4. per-cell flux angle;
  5. per-cell reduced flux |F|/(cE).
Inputs are generated once on the host, so both sides see identical bits.

A problem is a dict with these keys:
  dim, nx, ny, hx, hy, dt, c, a_r, c_v;
  bc: four dicts {kind, E, Fx, Fy} for the sides x-, x+, y-, y+.
The state is a float64 array of shape (4, ny, nx) holding E, Fx, Fy, T.
The opacity is a float64 array of shape (2, ny, nx) holding sigma_a, sigma_s.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def bc_all(kind: str, **wall) -> list:
    return [dict(kind=kind, **wall) for _ in range(4)]


def grid_problem(dim: int, nx: int, ny: int, cfl: float, bc: list, c: float = 1.0, a_r: float = 1.0,
                 c_v: float = 1.0, length: float = 1.0) -> dict:
    """Uniform grid on [0, length]^dim with dt = cfl * h / c (h = hx)."""
    hx = length / nx
    hy = length / ny if dim == 2 else hx
    return dict(dim=dim, nx=nx, ny=ny if dim == 2 else 1, hx=hx, hy=hy, dt=cfl * hx / c, c=c, a_r=a_r, c_v=c_v,
                bc=[dict(b) for b in bc])


def block_opacity(rng: np.random.Generator, ny: int, nx: int, block: int, log10_sa: tuple, ss: tuple) -> np.ndarray:
    """Piecewise-constant opacity on block x block cells.

    log10(sigma_a) ~ U[log10_sa] and sigma_s ~ U[ss], drawn per block. All
    sigma_a blocks are drawn first, in row-major order, then all sigma_s blocks.
    """
    by, bx = max(1, -(-ny // block)), max(1, -(-nx // block))
    la = rng.uniform(log10_sa[0], log10_sa[1], size=(by, bx))
    s = rng.uniform(ss[0], ss[1], size=(by, bx))
    sig = np.empty((2, ny, nx))
    sig[0] = np.repeat(np.repeat(10.0 ** la, block, axis=0), block, axis=1)[:ny, :nx]
    sig[1] = np.repeat(np.repeat(s, block, axis=0), block, axis=1)[:ny, :nx]
    return sig


def random_state(rng: np.random.Generator, ny: int, nx: int, c: float = 1.0, fmax: float = 0.95, fixed_f=None,
                 dim: int = 2, T: float = 1.0) -> np.ndarray:
    """Admissible state with E ~ lognormal(0,1), a random angle, and |F|/(cE) ~ U[0, fmax].

    Pass ``fixed_f`` to use the same reduced flux in every cell instead. In 1-D
    the flux points along +-x and Fy = 0.
    """
    v = np.empty((4, ny, nx))
    v[0] = rng.lognormal(0.0, 1.0, size=(ny, nx))
    th = rng.uniform(0.0, 2.0 * np.pi, size=(ny, nx))
    f = np.full((ny, nx), float(fixed_f)) if fixed_f is not None else rng.uniform(0.0, fmax, size=(ny, nx))
    if dim == 1:
        v[1] = np.where(np.cos(th) >= 0, 1.0, -1.0) * f * c * v[0]
        v[2] = 0.0
    else:
        v[1] = f * c * v[0] * np.cos(th)
        v[2] = f * c * v[0] * np.sin(th)
    v[3] = T
    return v


# --------------------------------------------------------------------------------------------
# The benchmark workloads (sizes overridable so the same recipe also gives small parity cases)
# --------------------------------------------------------------------------------------------

def gaussian_1d(n: int = 256, cfl: float = 50.0):
    """1-D Gaussian pulse: N cells on [0,1], c = a_r = C_v = 1, sigma_a = 1, sigma_s = 0.

    Initial state: E = 1 + 0.5 exp(-(x-0.5)^2 / (2*0.05^2)) at the cell centres,
    F = 0, T = 1. Boundaries are periodic and dt = 50 h/c. Solved for one step to
    relative residual 1e-10.
    """
    prob = grid_problem(1, n, 1, cfl, bc_all("periodic"))
    x = (np.arange(n) + 0.5) / n
    v = np.zeros((4, 1, n))
    v[0, 0] = 1.0 + 0.5 * np.exp(-((x - 0.5) ** 2) / (2 * 0.05 ** 2))
    v[3] = 1.0
    sig = np.zeros((2, 1, n))
    sig[0] = 1.0
    return prob, v, sig, dict(steps=1, rtol=1e-10)


def hot_wall_2d(n: int = 1024, seed: int = 1, cfl: float = 100.0, block: int = 32):
    """2-D hot-wall problem on [0,1]^2: n x n cells, dt = 100 h/c.

    Opacity is piecewise constant on 32x32-cell blocks, with log10 sigma_a ~ U[-2,2]
    and sigma_s ~ U[0,1]. The interior starts cold at E = a_r, F = 0, T = 1. The
    x = 0 side is a Dirichlet wall with E = a_r*1e4 and F = 0; the other sides
    are reflective. Run for 10 implicit steps to relative residual 1e-8.
    """
    bc = [dict(kind="dirichlet", E=1.0e4, Fx=0.0, Fy=0.0)] + [dict(kind="reflective") for _ in range(3)]
    prob = grid_problem(2, n, n, cfl, bc)
    rng = _rng(seed)
    sig = block_opacity(rng, n, n, block, (-2.0, 2.0), (0.0, 1.0))
    v = np.zeros((4, n, n))
    v[0] = prob["a_r"]
    v[3] = 1.0
    return prob, v, sig, dict(steps=10, rtol=1e-8)


def lognormal_2d(n: int = 4096, seed: int = 2, cfl: float = 100.0, block: int = 32):
    """2-D single solve on [0,1]^2: n x n cells, dt = 100 h/c, periodic sides.

    Opacity uses the hot-wall block recipe with seed 2. The initial state has
    E ~ lognormal(0,1) per cell, F = 0.9 c E along a uniformly random direction,
    and T = 1. Solved to relative residual 1e-8.
    """
    prob = grid_problem(2, n, n, cfl, bc_all("periodic"))
    rng = _rng(seed)
    sig = block_opacity(rng, n, n, block, (-2.0, 2.0), (0.0, 1.0))
    v = random_state(rng, n, n, c=prob["c"], fixed_f=0.9)
    return prob, v, sig, dict(steps=1, rtol=1e-8)


def beam_2d(n: int = 128, cfl: float = 2000.0, t0: float = 0.3, t_beam: float = 1.0):
    """The beam of Sect. 5.1: free streaming (no opacity) on [-1, 1]^2 with n x n cells.

    Temperatures are in units of 1000 K with a_r = c = 1: the ambient radiation
    has T_r = 0.3 (300 K), E = a_r T_r^4, F = 0; a beam of T_r = 1 (1000 K) with
    reduced flux f = 1 at 45 degrees enters through x = -1, y in [-0.875, -0.75]
    (the fractions [0.0625, 0.125] of that side); the rest of that side holds the
    ambient radiation (its ghost is (E_0, 0)), and the other sides copy the
    adjacent cell (outflow).  The gas, with no
    opacity, is decoupled (T = 1).  dt = cfl h / c: one implicit step of
    cfl 2000 reaches the steady state.
    """
    e_beam = t_beam ** 4
    f = e_beam / np.sqrt(2.0)  # |F| = c E at 45 degrees (c = 1)
    bc = [dict(kind="inflow", E=e_beam, Fx=f, Fy=f, lo=0.0625, hi=0.125, Eo=t0 ** 4)] + [dict(kind="neumann")] * 3
    prob = grid_problem(2, n, n, cfl, bc, length=2.0)
    v = np.zeros((4, n, n))
    v[0] = t0 ** 4
    v[3] = 1.0
    return prob, v, np.zeros((2, n, n)), dict(steps=1, rtol=1e-8)


def riemann_2d(n: int = 256, cfl: float = 2000.0, t0: float = 1.0):
    """The periodic 2-D Riemann problem of Sect. 5.2 on [0, 1]^2 with n x n cells.

    T_r = t0 (1000 K in units of 1000 K) everywhere, so E = a_r t0^4, and
    F = (1 - 1e-8) c E F_hat with F_hat = (1, 0) in the lower-left quadrant,
    (0, -1) lower-right, (0, 1) upper-left and (-1, 0) upper-right; no opacity,
    periodic sides, dt = cfl h / c.
    """
    prob = grid_problem(2, n, n, cfl, bc_all("periodic"))
    E = t0 ** 4
    a = (1.0 - 1e-8) * prob["c"] * E
    h = n // 2
    v = np.zeros((4, n, n))
    v[0] = E
    v[3] = 1.0
    v[1, :h, :h] = a    # lower-left: +x
    v[2, :h, h:] = -a   # lower-right: -y
    v[2, h:, :h] = a    # upper-left: +y
    v[1, h:, h:] = -a   # upper-right: -x
    return prob, v, np.zeros((2, n, n)), dict(steps=1, rtol=5e-3)


def batch_problem(k: int, sides=(64, 128, 256, 512), cfl: float = 100.0, block: int = 32):
    """Problem k of the batched workload, seeded with 1000 + k.

    The side is drawn log-uniformly from {64, ..., 512}. Opacity is on blocks
    with log10 sigma_a ~ U[-3,3] and sigma_s ~ U[0,1]. The state is a random
    admissible (E, F) with |F|/(cE) ~ U[0, 0.95] and T = 1. Sides are periodic.
    """
    rng = _rng(1000 + k)
    n = int(sides[rng.integers(0, len(sides))])
    prob = grid_problem(2, n, n, cfl, bc_all("periodic"))
    sig = block_opacity(rng, n, n, block, (-3.0, 3.0), (0.0, 1.0))
    v = random_state(rng, n, n, c=prob["c"], fmax=0.95)
    return prob, v, sig, dict(steps=1, rtol=1e-8)


def serve_request(rng: np.random.Generator, sides=(64, 128, 256, 512, 1024, 2048), max_steps: int = 20,
                  cfl: float = 100.0, block: int = 32):
    """One serving request: a log-uniform side, opacity contrast 10^C with C ~ U[0,6], and 1..20 steps."""
    n = int(sides[rng.integers(0, len(sides))])
    contrast = rng.uniform(0.0, 6.0)
    steps = int(rng.integers(1, max_steps + 1))
    prob = grid_problem(2, n, n, cfl, bc_all("periodic"))
    sig = block_opacity(rng, n, n, block, (-contrast / 2, contrast / 2), (0.0, 1.0))
    v = random_state(rng, n, n, c=prob["c"], fmax=0.95)
    return prob, v, sig, dict(steps=steps, rtol=1e-8)


def random_problem(seed: int, dim: int, nx: int, ny: int, bc_kinds=("periodic",) * 4, cfl: float = 20.0,
                   log10_sa=(-2.0, 1.0), ss=(0.0, 1.0), fmax: float = 0.95, fixed_f=None, block: int = 4,
                   c: float = 1.0, a_r: float = 1.0, c_v: float = 1.0, wall_E: float = 10.0):
    """Small random problem for tests: random admissible state, block opacity and any boundary mix.

    Dirichlet sides get the wall state (wall_E, 0.3 c wall_E, 0).
    """
    rng = _rng(seed)
    bc = []
    for kind in bc_kinds:
        if kind == "dirichlet":
            bc.append(dict(kind=kind, E=wall_E, Fx=0.3 * c * wall_E, Fy=0.0))
        else:
            bc.append(dict(kind=kind))
    prob = grid_problem(dim, nx, ny, cfl, bc, c=c, a_r=a_r, c_v=c_v)
    ny_ = prob["ny"]
    sig = block_opacity(rng, ny_, nx, block, log10_sa, ss)
    v = random_state(rng, ny_, nx, c=c, fmax=fmax, fixed_f=fixed_f, dim=dim)
    v[3] = rng.uniform(0.5, 1.5, size=(ny_, nx))
    return prob, v, sig


# ---------------------------------------------------------------------------- three dimensions
# A 3-D problem is a dict with keys nx, ny, nz, hx, hy, hz, dt, c, a_r, c_v and bc: six dicts {kind, E, Fx, Fy,
# Fz} for the sides x-, x+, y-, y+, z-, z+.  States have shape (5, nz, ny, nx) holding E, Fx, Fy, Fz, T;
# opacities (2, nz, ny, nx).
def grid_problem3(nx: int, ny: int, nz: int, cfl: float, bc: list, c: float = 1.0, a_r: float = 1.0,
                  c_v: float = 1.0, length: float = 1.0) -> dict:
    """Uniform grid on [0, length]^3 with dt = cfl * hx / c."""
    hx, hy, hz = length / nx, length / ny, length / nz
    return dict(nx=nx, ny=ny, nz=nz, hx=hx, hy=hy, hz=hz, dt=cfl * hx / c, c=c, a_r=a_r, c_v=c_v,
                bc=[dict(b) for b in bc])


def block_opacity3(rng: np.random.Generator, nz: int, ny: int, nx: int, block: int, log10_sa: tuple,
                   ss: tuple) -> np.ndarray:
    """Piecewise-constant opacity on block^3 cells: all sigma_a blocks first (z, y, x order), then sigma_s."""
    bz, by, bx = (max(1, -(-m // block)) for m in (nz, ny, nx))
    la = rng.uniform(log10_sa[0], log10_sa[1], size=(bz, by, bx))
    s = rng.uniform(ss[0], ss[1], size=(bz, by, bx))

    def expand(a):
        return np.repeat(np.repeat(np.repeat(a, block, axis=0), block, axis=1), block, axis=2)[:nz, :ny, :nx]

    sig = np.empty((2, nz, ny, nx))
    sig[0] = expand(10.0 ** la)
    sig[1] = expand(s)
    return sig


def random_state3(rng: np.random.Generator, nz: int, ny: int, nx: int, c: float = 1.0, fmax: float = 0.95,
                  fixed_f=None, T: float = 1.0) -> np.ndarray:
    """Admissible 3-D state: E ~ lognormal(0,1), a direction uniform on the sphere, |F|/(cE) ~ U[0, fmax]."""
    v = np.empty((5, nz, ny, nx))
    v[0] = rng.lognormal(0.0, 1.0, size=(nz, ny, nx))
    d = rng.normal(size=(3, nz, ny, nx))
    d /= np.linalg.norm(d, axis=0)
    f = np.full((nz, ny, nx), float(fixed_f)) if fixed_f is not None else rng.uniform(0.0, fmax, size=(nz, ny, nx))
    v[1:4] = d * f * c * v[0]
    v[4] = T
    return v


def random_problem3(seed: int, nx: int, ny: int, nz: int, bc_kinds=("periodic",) * 6, cfl: float = 20.0,
                    log10_sa=(-2.0, 1.0), ss=(0.0, 1.0), fmax: float = 0.95, fixed_f=None, block: int = 2,
                    c: float = 1.0, wall_E: float = 10.0):
    """Small random 3-D problem for tests; Dirichlet sides get the wall state (wall_E, 0.3 c wall_E, 0, 0)."""
    rng = _rng(seed)
    bc = [dict(kind=k, E=wall_E, Fx=0.3 * c * wall_E, Fy=0.0, Fz=0.0) if k == "dirichlet" else dict(kind=k)
          for k in bc_kinds]
    prob = grid_problem3(nx, ny, nz, cfl, bc, c=c)
    sig = block_opacity3(rng, nz, ny, nx, block, log10_sa, ss)
    v = random_state3(rng, nz, ny, nx, c=c, fmax=fmax, fixed_f=fixed_f)
    v[4] = rng.uniform(0.5, 1.5, size=(nz, ny, nx))
    return prob, v, sig


def hot_wall_3d(n: int = 256, seed: int = 1, cfl: float = 100.0, block: int = 8, steps: int = 10):
    """The hot-wall problem in 3-D on [0,1]^3: n^3 cells, dt = 100 h/c, opacity piecewise constant on block^3
    cells (log10 sigma_a ~ U[-2,2], sigma_s ~ U[0,1]), cold interior E = a_r, F = 0, T = 1, a Dirichlet wall
    E = a_r*1e4, F = 0 at x = 0 and reflective sides elsewhere; implicit steps to relative residual 1e-8."""
    bc = [dict(kind="dirichlet", E=1.0e4, Fx=0.0, Fy=0.0, Fz=0.0)] + [dict(kind="reflective") for _ in range(5)]
    prob = grid_problem3(n, n, n, cfl, bc)
    rng = _rng(seed)
    sig = block_opacity3(rng, n, n, n, block, (-2.0, 2.0), (0.0, 1.0))
    v = np.zeros((5, n, n, n))
    v[0] = prob["a_r"]
    v[4] = 1.0
    return prob, v, sig, dict(steps=steps, rtol=1e-8)
