"""TEST INFRASTRUCTURE ONLY -- dense Newton check on tiny grids.

An independent numpy form of the implicit M1 operator A (written apart from
``m1_oracle.c``: vectorised over ghost-padded arrays, closure written through
f^2 so that it is analytic), its Jacobian by the complex-step derivative, and a
Newton solver for A(v) = b.  On tiny grids the Newton root is the reference the
multigrid cycle must reach (uniqueness of the solution, Sect. 3.1).
"""
from __future__ import annotations

import numpy as np


def closure(E, Fx, Fy, c):
    """M1 closure (Sect. 2.1) as an analytic function of (E, F).

    With f^2 = |F|^2/(cE)^2 and s = sqrt(4 - 3 f^2):
      chi = (3 + 4 f^2)/(5 + 2 s),  (1 - chi)/2 E is the isotropic part and
      (3 chi - 1)/2 E n_i n_j = (3 chi - 1)/(2 f^2) F_i F_j /(c^2 E),
    where (3 chi - 1)/(2 f^2) = 3/(2 + s) removes the 0/0 at F = 0.
    """
    f2 = (Fx * Fx + Fy * Fy) / (c * E) ** 2
    s = np.sqrt(4.0 - 3.0 * f2)
    chi = (3.0 + 4.0 * f2) / (5.0 + 2.0 * s)
    iso = 0.5 * (1.0 - chi) * E
    aniso = 3.0 / (2.0 + s) / (c * c * E)
    return iso + aniso * Fx * Fx, aniso * Fx * Fy, iso + aniso * Fy * Fy


def _pad(U, prob):
    """Ghost-padded copy of U = (E, Fx, Fy) with one ghost layer per side."""
    _, ny, nx = U.shape
    P = np.zeros((3, ny + 2, nx + 2), dtype=U.dtype)
    P[:, 1:-1, 1:-1] = U
    sides = [
        (0, (slice(None), slice(1, -1), 0), (slice(None), slice(None), -1), (slice(None), slice(None), 0), 1),
        (1, (slice(None), slice(1, -1), -1), (slice(None), slice(None), 0), (slice(None), slice(None), -1), 1),
        (2, (slice(None), 0, slice(1, -1)), (slice(None), -1, slice(None)), (slice(None), 0, slice(None)), 2),
        (3, (slice(None), -1, slice(1, -1)), (slice(None), 0, slice(None)), (slice(None), -1, slice(None)), 2),
    ]
    for side, dst, wrap_src, own_src, normal in sides:
        if side >= 2 and prob["dim"] == 1:
            continue
        bc = prob["bc"][side]
        kind = bc["kind"]
        if kind == "periodic":
            P[dst] = U[wrap_src]
        elif kind in ("reflective", "neumann"):
            P[dst] = U[own_src]
            if kind == "reflective":
                P[(normal,) + dst[1:]] *= -1.0
        elif kind == "dirichlet":
            P[(0,) + dst[1:]] = bc["E"]
            P[(1,) + dst[1:]] = bc["Fx"]
            P[(2,) + dst[1:]] = bc["Fy"]
        elif kind == "inflow":  # wall state where the boundary cell's centre is in [lo, hi] of the side, else (Eo, 0)
            P[(0,) + dst[1:]] = bc["Eo"]
            P[(1,) + dst[1:]] = 0.0
            P[(2,) + dst[1:]] = 0.0
            n = ny if side < 2 else nx
            centres = (np.arange(n) + 0.5) / n
            on = (centres >= bc["lo"]) & (centres <= bc["hi"])
            for q, key in enumerate(("E", "Fx", "Fy")):
                row = P[(q,) + dst[1:]]
                row[on] = bc[key]
                P[(q,) + dst[1:]] = row
        else:
            raise ValueError(kind)
    return P


def apply_A(v, sigma, prob):
    """A(v) of the implicit HLL (Rusanov) system with implicit sources, any dtype (complex allowed)."""
    c, dt, ar, cv = prob["c"], prob["dt"], prob["a_r"], prob["c_v"]
    E, Fx, Fy, T = v[0], v[1], v[2], v[3]
    Pd = _pad(np.stack([E, Fx, Fy]), prob)
    kx = dt / (2.0 * prob["hx"])
    a = 1.0 + c * dt / prob["hx"]

    def flux_x(U):
        Pxx, Pxy, _ = closure(U[0], U[1], U[2], c)
        return np.stack([U[1], c * c * Pxx, c * c * Pxy])

    def flux_y(U):
        _, Pxy, Pyy = closure(U[0], U[1], U[2], c)
        return np.stack([U[2], c * c * Pxy, c * c * Pyy])

    Ul = Pd[:, 1:-1, :-2]
    Ur = Pd[:, 1:-1, 2:]
    S = kx * (c * Ul + flux_x(Ul)) + kx * (c * Ur - flux_x(Ur))
    if prob["dim"] == 2:
        ky = dt / (2.0 * prob["hy"])
        a = a + c * dt / prob["hy"]
        Ud = Pd[:, :-2, 1:-1]
        Uu = Pd[:, 2:, 1:-1]
        S = S + ky * (c * Ud + flux_y(Ud)) + ky * (c * Uu - flux_y(Uu))
    ka = c * dt * sigma[0]
    ks = c * dt * sigma[1]
    out = np.zeros_like(v)
    T4 = T ** 4
    out[0] = a * E - S[0] + ka * (E - ar * T4)
    out[1] = a * Fx - S[1] + (ka + ks) * Fx
    if prob["dim"] == 2:
        out[2] = a * Fy - S[2] + (ka + ks) * Fy
    out[3] = cv * T + ka * (ar * T4 - E)
    return out


def _fields(prob):
    return [0, 1, 2, 3] if prob["dim"] == 2 else [0, 1, 3]


def newton_solve(v0, b, sigma, prob, tol=1e-15, maxit=60):
    """Newton's method for A(v) = b with a complex-step Jacobian and backtracking on |A(v) - b|."""
    fields = _fields(prob)
    shape = v0.shape
    ncell = shape[1] * shape[2]

    def pack(v):
        return np.concatenate([v[f].ravel() for f in fields])

    def unpack(x, dtype=float):
        v = np.zeros(shape, dtype=dtype)
        for m, f in enumerate(fields):
            v[f] = x[m * ncell:(m + 1) * ncell].reshape(shape[1:])
        return v

    def F(x):
        return pack(apply_A(unpack(x, x.dtype), sigma, prob) - b)

    x = pack(v0).astype(float)
    n = x.size
    h = 1e-30
    res = np.linalg.norm(F(x))
    for _ in range(maxit):
        J = np.empty((n, n))
        for m in range(n):
            xc = x.astype(complex)
            xc[m] += 1j * h
            J[:, m] = F(xc).imag / h
        dx = np.linalg.solve(J, -F(x))
        step = 1.0
        while step > 1e-8:
            xn = x + step * dx
            vn = unpack(xn)
            if np.all(vn[0] > 0) and np.all(vn[3] > 0):
                rn = np.linalg.norm(F(xn))
                if rn < res or rn < tol * (1.0 + np.linalg.norm(pack(b))):
                    break
            step *= 0.5
        x, res = xn, rn
        if np.linalg.norm(step * dx) <= tol * np.linalg.norm(x):
            break
    return unpack(x), res
