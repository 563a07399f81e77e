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
