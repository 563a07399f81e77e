"""Exact solutions of the paper's smooth accuracy tests (Examples 3.1, 3.2, 3.8, 3.9),
evaluated at cell centres.  Burgers' solutions follow the characteristics
(u is constant along x - u t), solved by Newton's method to machine precision."""
import numpy as np


def burgers_1d(x, t):
    """u_t + (u^2/2)_x = 0, u0 = 0.5 + sin(pi x): u = u0(x - u t)."""
    u = 0.5 + np.sin(np.pi * x)
    for _ in range(60):
        g = u - (0.5 + np.sin(np.pi * (x - u * t)))
        u = u - g / (1 + np.pi * np.cos(np.pi * (x - u * t)) * t)
    return u


def burgers_2d(x, y, t):
    """u_t + (u^2/2)_x + (u^2/2)_y = 0, u0 = 0.5 + sin(pi (x + y)/2): u = u0(x - u t, y - u t)."""
    s = x + y
    u = 0.5 + np.sin(np.pi * s / 2)
    for _ in range(60):
        g = u - (0.5 + np.sin(np.pi * (s - 2 * u * t) / 2))
        u = u - g / (1 + np.pi * np.cos(np.pi * (s - 2 * u * t) / 2) * t)
    return u


def density_wave_1d(x, t):
    """Euler, rho0 = 1 + 0.2 sin(pi x), u = p = 1: rho = rho0(x - t)."""
    return 1 + 0.2 * np.sin(np.pi * (x - t))


def density_wave_2d(x, y, t):
    """Euler, rho0 = 1 + 0.2 sin(pi (x + y)), u = v = p = 1: rho = rho0(x - t, y - t)."""
    return 1 + 0.2 * np.sin(np.pi * (x + y - 2 * t))


def riemann_euler(WL, WR, xi, gamma=1.4):
    """Exact solution (rho, u, p) of the 1D Euler Riemann problem with left/right primitive
    states WL, WR, sampled at xi = x / t (self-similar).  The star pressure is the root
    of f_L(p) + f_R(p) + u_R - u_L = 0, f_K being the shock (Rankine-Hugoniot) branch for
    p > p_K and the isentropic rarefaction branch otherwise; Newton's method from the
    two-rarefaction guess converges to machine precision.  Vacuum is not handled."""
    g = gamma
    rL, uL, pL = (float(v) for v in WL)
    rR, uR, pR = (float(v) for v in WR)
    aL, aR = np.sqrt(g * pL / rL), np.sqrt(g * pR / rR)
    z = (g - 1) / (2 * g)

    def f(p, r, pk, a):
        if p > pk:
            A, B = 2 / ((g + 1) * r), (g - 1) / (g + 1) * pk
            q = np.sqrt(A / (p + B))
            return (p - pk) * q, q * (1 - 0.5 * (p - pk) / (p + B))
        return 2 * a / (g - 1) * ((p / pk) ** z - 1), (p / pk) ** (-(g + 1) / (2 * g)) / (r * a)

    p = ((aL + aR - 0.5 * (g - 1) * (uR - uL)) / (aL / pL ** z + aR / pR ** z)) ** (1 / z)
    for _ in range(100):
        fl, dl = f(p, rL, pL, aL)
        fr, dr = f(p, rR, pR, aR)
        step = (fl + fr + uR - uL) / (dl + dr)
        p = max(p - step, 1e-14)
        if abs(step) < 1e-15 * p:
            break
    fl, _ = f(p, rL, pL, aL)
    fr, _ = f(p, rR, pR, aR)
    us = 0.5 * (uL + uR) + 0.5 * (fr - fl)
    g6 = (g - 1) / (g + 1)

    xi = np.asarray(xi, dtype=np.float64)
    out = np.empty((3,) + xi.shape)
    for idx, s in np.ndenumerate(xi):
        if s <= us:
            r, u, pk, a, sg = rL, uL, pL, aL, 1.0
        else:  # mirror the right side onto the left-side formulas
            r, u, pk, a, sg = rR, -uR, pR, aR, -1.0
        s_, u_star = sg * s, sg * us
        if p > pk:
            shock = u - a * np.sqrt((g + 1) / (2 * g) * p / pk + z)
            if s_ <= shock:
                W = (r, u, pk)
            else:
                W = (r * (p / pk + g6) / (g6 * p / pk + 1), u_star, p)
        else:
            head, tail = u - a, u_star - a * (p / pk) ** z
            if s_ <= head:
                W = (r, u, pk)
            elif s_ >= tail:
                W = (r * (p / pk) ** (1 / g), u_star, p)
            else:
                c = 2 / (g + 1) * (a + 0.5 * (g - 1) * (u - s_))
                W = (r * (c / a) ** (2 / (g - 1)), 2 / (g + 1) * (a + 0.5 * (g - 1) * u + s_),
                     pk * (c / a) ** (2 * g / (g - 1)))
        out[0][idx], out[1][idx], out[2][idx] = W[0], sg * W[1], W[2]
    return out


def riemann_cell_averages(WL, WR, x0, lo, hi, n, t, sub=32, gamma=1.4):
    """Cell averages of the exact Riemann solution (discontinuity at x0 at t = 0) on n
    uniform cells of [lo, hi]: conserved variables averaged with a sub-point midpoint rule."""
    dx = (hi - lo) / n
    xs = lo + (np.arange(n * sub) + 0.5) * dx / sub
    rho, u, p = riemann_euler(WL, WR, (xs - x0) / t, gamma)
    U = np.stack([rho, rho * u, p / (gamma - 1) + 0.5 * rho * u * u])
    return U.reshape(3, n, sub).mean(axis=2)
