"""Initial and reference states (conserved variables rho, rho u, rho v, E).

These are inputs: closed-form flow fields evaluated at given points.  The
state layout matches the solver's: an array (K, 4, Np) of float64.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


def primitive_to_conserved(rho, u, v, p, gamma=GAMMA):
    rho, u, v, p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (rho, u, v, p)))
    axis = -2 if rho.ndim >= 1 else 0
    return np.stack([rho, rho * u, rho * v,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)], axis=axis)


def freestream_state(mach: float, alpha_deg: float = 0.0, gamma=GAMMA):
    """(rho, rho u, rho v, E) with rho=1, sound speed 1, velocity M(cos a, sin a)."""
    a = np.deg2rad(alpha_deg)
    u = mach * np.cos(a)
    v = mach * np.sin(a)
    p = 1.0 / gamma
    return np.array([1.0, u, v, p / (gamma - 1.0) + 0.5 * (u * u + v * v)])


def cylinder_potential(x, y, mach: float, radius: float = 1.0, gamma=GAMMA):
    """Wall-compatible start for flow past a cylinder of the given radius at
    the origin: the incompressible potential-flow velocity (freestream
    (mach, 0), zero normal velocity on the wall) with density and pressure
    from the isentropic energy relation c^2 = 1 + (gamma-1)/2 (M^2 - |v|^2)
    (rho = c^(2/(gamma-1)), p = rho^gamma / gamma; freestream rho = c = 1)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r2 = (x * x + y * y) / (radius * radius)
    th = np.arctan2(y, x)
    ur = mach * (1.0 - 1.0 / r2) * np.cos(th)
    ut = -mach * (1.0 + 1.0 / r2) * np.sin(th)
    u = ur * np.cos(th) - ut * np.sin(th)
    v = ur * np.sin(th) + ut * np.cos(th)
    c2 = 1.0 + 0.5 * (gamma - 1.0) * (mach * mach - (u * u + v * v))
    if np.any(c2 <= 0):
        raise ValueError("Mach number too high for the isentropic potential start")
    rho = c2 ** (1.0 / (gamma - 1.0))
    return primitive_to_conserved(rho, u, v, rho ** gamma / gamma, gamma)


def _panel_velocity(px, py, ax, ay, bx, by):
    """Velocity at points (px, py) [n] induced by unit-strength constant
    source and vortex sheets on panels A -> B [m]: two arrays (n, m, 2).
    Panel-local frame: x along A -> B, y to its left; for a source sheet
    u = ln(rA / rB) / 2pi, v = theta / 2pi, for a (counter-clockwise) vortex
    sheet u = -theta / 2pi, v = ln(rA / rB) / 2pi, theta the signed angle
    the panel subtends at the point."""
    tx, ty = bx - ax, by - ay
    L = np.hypot(tx, ty)
    tx, ty = tx / L, ty / L
    dx, dy = px[:, None] - ax[None, :], py[:, None] - ay[None, :]
    xl = dx * tx[None, :] + dy * ty[None, :]
    yl = -dx * ty[None, :] + dy * tx[None, :]
    rA2 = xl * xl + yl * yl
    rB2 = (xl - L[None, :]) ** 2 + yl * yl
    lnr = 0.5 * np.log(rA2 / rB2)
    theta = np.arctan2(yl, xl - L[None, :]) - np.arctan2(yl, xl)
    theta = np.where(theta > np.pi, theta - 2 * np.pi, np.where(theta < -np.pi, theta + 2 * np.pi, theta))
    k = 1.0 / (2.0 * np.pi)
    us, vs = k * lnr, k * theta
    uv, vv = -k * theta, k * lnr
    src = np.stack([us * tx - vs * ty, us * ty + vs * tx], axis=-1)
    vor = np.stack([uv * tx - vv * ty, uv * ty + vv * tx], axis=-1)
    return src, vor


def airfoil_panels(mach: float, alpha_deg: float, t: float = 0.12, n_panels: int = 400):
    """Hess-Smith panel solution of incompressible potential flow past the
    symmetric 4-digit airfoil (chord 1, closed trailing edge): a constant
    source strength per panel plus one vortex strength on every panel, from
    zero normal velocity at the panel midpoints and equal speeds on the two
    panels at the trailing edge (Kutta).  Returns (panel end points,
    sources, vortex strength, freestream velocity)."""
    from .meshes import naca_point
    beta = 2 * np.pi * np.arange(n_panels + 1) / n_panels
    pts = naca_point(np.mod(beta, 2 * np.pi), t)          # TE, upper surface, LE, lower surface, TE
    ax, ay, bx, by = pts[:-1, 0], pts[:-1, 1], pts[1:, 0], pts[1:, 1]
    L = np.hypot(bx - ax, by - ay)
    tx, ty = (bx - ax) / L, (by - ay) / L
    nx, ny = ty, -tx                                        # outward: the traversal is counter-clockwise
    a = np.deg2rad(alpha_deg)
    Vinf = np.array([mach * np.cos(a), mach * np.sin(a)])
    # control points just outside the midpoints (the fluid side of each sheet)
    cx = 0.5 * (ax + bx) + 1e-10 * nx
    cy = 0.5 * (ay + by) + 1e-10 * ny
    src, vor = _panel_velocity(cx, cy, ax, ay, bx, by)
    m = n_panels
    A = np.zeros((m + 1, m + 1))
    rhs = np.zeros(m + 1)
    A[:m, :m] = src[..., 0] * nx[:, None] + src[..., 1] * ny[:, None]
    A[:m, m] = (vor[..., 0] * nx[:, None] + vor[..., 1] * ny[:, None]).sum(axis=1)
    rhs[:m] = -(Vinf[0] * nx + Vinf[1] * ny)
    # Kutta: V.t on the first panel + V.t on the last panel = 0
    for i in (0, m - 1):
        A[m, :m] += src[i, :, 0] * tx[i] + src[i, :, 1] * ty[i]
        A[m, m] += (vor[i, :, 0] * tx[i] + vor[i, :, 1] * ty[i]).sum()
        rhs[m] -= Vinf[0] * tx[i] + Vinf[1] * ty[i]
    sol = np.linalg.solve(A, rhs)
    return (ax, ay, bx, by), sol[:m], sol[m], Vinf


def airfoil_velocity(x, y, panels, q, g, Vinf, chunk: int = 4096, standoff: float = 2e-3):
    """Velocity (u, v) of the panel solution at points (x, y).  A point
    closer than ``standoff`` to its nearest panel (the surface nodes of a
    mesh, which may coincide with panel end points, where the sheets' log
    terms are singular) takes the velocity at ``standoff`` outside it."""
    from scipy.spatial import cKDTree
    ax, ay, bx, by = panels
    px, py = np.ravel(x).astype(np.float64), np.ravel(y).astype(np.float64)
    L = np.hypot(bx - ax, by - ay)
    tx, ty = (bx - ax) / L, (by - ay) / L
    nx, ny = ty, -tx
    _, j = cKDTree(np.c_[0.5 * (ax + bx), 0.5 * (ay + by)]).query(np.c_[px, py])
    d = (px - ax[j]) * nx[j] + (py - ay[j]) * ny[j]
    near = d < standoff
    px = np.where(near, px + (standoff - d) * nx[j], px)
    py = np.where(near, py + (standoff - d) * ny[j], py)
    u = np.empty_like(px)
    v = np.empty_like(py)
    for i in range(0, px.size, chunk):
        src, vor = _panel_velocity(px[i:i + chunk], py[i:i + chunk], ax, ay, bx, by)
        vel = np.einsum("nmk,m->nk", src, q) + g * vor.sum(axis=1)
        u[i:i + chunk] = Vinf[0] + vel[:, 0]
        v[i:i + chunk] = Vinf[1] + vel[:, 1]
    return u.reshape(np.shape(x)), v.reshape(np.shape(y))


def airfoil_potential(x, y, mach: float, alpha_deg: float, t: float = 0.12, n_panels: int = 400,
                      gamma=GAMMA):
    """Wall-compatible start for flow past the airfoil: the incompressible
    potential-flow velocity of the panel solution, with density and pressure
    from the isentropic energy relation as for the cylinder start."""
    panels, q, g, Vinf = airfoil_panels(mach, alpha_deg, t, n_panels)
    u, v = airfoil_velocity(x, y, panels, q, g, Vinf)
    c2 = 1.0 + 0.5 * (gamma - 1.0) * (mach * mach - (u * u + v * v))
    if np.any(c2 <= 0):
        raise ValueError("Mach number too high for the isentropic potential start")
    rho = c2 ** (1.0 / (gamma - 1.0))
    return np.ascontiguousarray(primitive_to_conserved(rho, u, v, rho ** gamma / gamma, gamma))


def wall_damped(x, y, wall_x, wall_y, q, delta: float = 0.2, gamma=GAMMA):
    """Smooth start for flow past a body: the freestream q with its velocity
    scaled by 1 - exp(-(d / delta)^2), d the distance to the nearest of the
    given wall points, at the freestream density and pressure.  The fluid at
    the wall starts at rest (compatible with the slip wall) and the flow
    reaches the freestream a few delta away, so the start launches no
    impulsive wave from the wall."""
    from scipy.spatial import cKDTree
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d, _ = cKDTree(np.c_[np.ravel(wall_x), np.ravel(wall_y)]).query(np.c_[x.ravel(), y.ravel()])
    f = 1.0 - np.exp(-(d.reshape(x.shape) / delta) ** 2)
    q = np.asarray(q, dtype=np.float64)
    rho, u, v = q[0], q[1] / q[0], q[2] / q[0]
    p = (gamma - 1.0) * (q[3] - 0.5 * rho * (u * u + v * v))
    return np.ascontiguousarray(primitive_to_conserved(rho + 0 * x, u * f, v * f, p + 0 * x, gamma))


def uniform(shape_KNp, q):
    """Fill (K,4,Np) with the constant state q (4,)."""
    K, Np = shape_KNp
    return np.ascontiguousarray(np.broadcast_to(np.asarray(q, dtype=np.float64)[None, :, None],
                                                (K, 4, Np)).copy())


def isentropic_vortex(x, y, t=0.0, beta=5.0, x0=5.0, y0=5.0, L=10.0,
                      u_inf=1.0, gamma=GAMMA):
    """Isentropic vortex advected with (u_inf, 0) on a periodic box of side L.

    Velocity perturbation beta*(-ybar, xbar)*exp(1-r^2)/(2 pi) and temperature
    drop (gamma-1) beta^2 exp(2(1-r^2))/(16 gamma pi^2); p = rho^gamma.  This
    pair satisfies radial equilibrium exactly, so the field is a steady vortex
    carried by the uniform flow.  xbar is wrapped to the nearest periodic
    image of the moving centre.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xb = x - x0 - u_inf * t
    xb = xb - L * np.round(xb / L)
    yb = y - y0
    r2 = xb * xb + yb * yb
    e1 = np.exp(1.0 - r2)
    u = u_inf - beta * yb * e1 / (2 * np.pi)
    v = beta * xb * e1 / (2 * np.pi)
    T = 1.0 - (gamma - 1.0) * beta * beta * e1 * e1 / (16.0 * gamma * np.pi ** 2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return np.ascontiguousarray(primitive_to_conserved(rho, u, v, p, gamma))
