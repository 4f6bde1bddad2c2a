"""TEST INFRASTRUCTURE ONLY -- dense Newton check of the three-dimensional operator on tiny grids.

An independent numpy form of the 3-D implicit M1 operator A (vectorised over ghost-padded arrays, the
closure written through f^2 so that it is analytic; written apart from ``m1_oracle3.c``), its Jacobian by
the complex-step derivative, and a Newton solver for A(v) = b.  States have shape (5, nz, ny, nx) holding
E, Fx, Fy, Fz, T.
"""
from __future__ import annotations

import numpy as np


def closure3(E, F, c):
    """M1 pressure tensor (Sect. 2.1) as an analytic function of (E, F): a dict keyed by (row, column)."""
    f2 = (F[0] * F[0] + F[1] * F[1] + F[2] * F[2]) / (c * E) ** 2
    s = np.sqrt(4.0 - 3.0 * f2)
    chi = (3.0 + 4.0 * f2) / (5.0 + 2.0 * s)
    iso = 0.5 * (1.0 - chi) * E
    aniso = 3.0 / (2.0 + s) / (c * c * E)  # (3 chi - 1)/(2 f^2) / (c^2 E)
    return {(a, b): (iso if a == b else 0.0) + aniso * F[a] * F[b] for a in range(3) for b in range(3)}


def _pad3(U, prob):
    """(E, Fx, Fy, Fz) with one ghost layer on each of the six sides (axes of U: field, z, y, x)."""
    P = np.pad(U, ((0, 0), (1, 1), (1, 1), (1, 1)))
    P = P.astype(U.dtype)
    for side, bc in enumerate(prob["bc"]):
        axis = 3 - side // 2            # x sides pad array axis 3, y axis 2, z axis 1
        lo = side % 2 == 0
        ghost = [slice(1, -1)] * 3
        ghost[axis - 1] = 0 if lo else -1
        kind = bc["kind"]
        if kind == "periodic":
            src = [slice(1, -1)] * 3
            src[axis - 1] = -2 if lo else 1
            P[(slice(None),) + tuple(ghost)] = P[(slice(None),) + tuple(src)]
        elif kind in ("reflective", "neumann"):
            src = [slice(1, -1)] * 3
            src[axis - 1] = 1 if lo else -2
            P[(slice(None),) + tuple(ghost)] = P[(slice(None),) + tuple(src)]
            if kind == "reflective":
                normal = 1 + side // 2      # the flux component normal to the side
                P[(normal,) + tuple(ghost)] *= -1.0
        elif kind == "dirichlet":
            for q, key in enumerate(("E", "Fx", "Fy", "Fz")):
                P[(q,) + tuple(ghost)] = bc.get(key, 0.0)
        else:
            raise ValueError(kind)
    return P


def apply_A3(v, sigma, prob):
    """A(v) of the 3-D implicit Rusanov system with implicit sources (any dtype, complex allowed)."""
    c, dt, ar, cv = prob["c"], prob["dt"], prob["a_r"], prob["c_v"]
    E, T = v[0], v[4]
    Pd = _pad3(np.stack([v[0], v[1], v[2], v[3]]), prob)
    inner = (slice(1, -1),) * 3
    S = np.zeros((4,) + E.shape, dtype=v.dtype)
    a = 1.0
    for axis, h in enumerate((prob["hx"], prob["hy"], prob["hz"])):
        k = dt / (2.0 * h)
        a = a + c * dt / h
        arr = 3 - axis
        for shift, sign in ((-1, 1.0), (1, -1.0)):   # lower neighbour with L (+G), upper with R (-G)
            idx = list(inner)
            idx[arr - 1] = slice(1 + shift, Pd.shape[arr] - 1 + shift)
            U = Pd[(slice(None),) + tuple(idx)]
            Pt = closure3(U[0], U[1:4], c)
            G = np.stack([U[1 + axis]] + [c * c * Pt[(m, axis)] for m in range(3)])
            S = S + k * (c * U + sign * G)
    ka = c * dt * sigma[0]
    ks = c * dt * sigma[1]
    out = np.zeros_like(v)
    T4 = T ** 4
    out[0] = a * E - S[0] + ka * (E - ar * T4)
    for m in range(1, 4):
        out[m] = a * v[m] - S[m] + (ka + ks) * v[m]
    out[4] = cv * T + ka * (ar * T4 - E)
    return out


def newton_solve3(v0, b, sigma, prob, tol=1e-15, maxit=60):
    """Newton's method for A(v) = b with a complex-step Jacobian and backtracking on |A(v) - b|."""
    shape = v0.shape
    n = v0.size
    h = 1e-30

    def F(x):
        return (apply_A3(x.reshape(shape), sigma, prob) - b).ravel()

    x = v0.astype(float).ravel()
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
            vn = xn.reshape(shape)
            if np.all(vn[0] > 0) and np.all(vn[4] > 0):
                rn = np.linalg.norm(F(xn))
                if rn < res or rn < tol * (1.0 + np.linalg.norm(b)):
                    break
            step *= 0.5
        x, res = xn, rn
        if np.linalg.norm(step * dx) <= tol * np.linalg.norm(x):
            break
    return x.reshape(shape), res
