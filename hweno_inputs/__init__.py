"""Seeded synthetic initial states for the L-HWENO hot path.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
no arithmetic of the numerical method itself: it only samples initial data on a
uniform cell-centred grid (point values of the solution and of its first
derivatives), converts primitive Euler variables to conserved ones and records
the grid geometry.

State layout (all generators): a float64 numpy array ``S[nf, ny, nx]``, x
fastest, ``ny == 1`` in one dimension.  The fields are the m conserved
components U, then their x-derivatives U_x, then (2D only) their
y-derivatives U_y, so ``nf = m * (1 + dim)``.  Derivatives of discontinuous
data are zero (pointwise derivative of piecewise-constant data); derivatives of
smooth data are the analytic ones.

Random numbers come from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

GAMMA_GAS = 1.4

PERIODIC = 0
OUTFLOW = 1
REFLECT = 2
EDGES = 3   # each side of the direction described in Workload.edges

SEG_OUTFLOW, SEG_REFLECT, SEG_STATE = 0, 1, 2


@dataclass
class Workload:
    """One initial state plus the geometry and physics it belongs to."""

    S: np.ndarray            # [nf, ny, nx] float64
    dim: int                 # 1 or 2
    physics: str             # "linadv" | "burgers" | "euler"
    dx: float
    dy: float
    bc_x: int
    bc_y: int
    lo: tuple = (0.0, 0.0)
    hi: tuple = (1.0, 1.0)
    gamma_gas: float = GAMMA_GAS
    adv_speed: tuple = (1.0, 1.0)
    name: str = ""
    info: dict = field(default_factory=dict)
    # sides x_lo, x_hi, y_lo, y_hi where a bc is EDGES: each
    # ((kind_0, kind_1), (s0, s1, s2), (state_0, state_1)); a ghost cell at
    # position pos along the side, d beyond it, at time t takes segment 0 when
    # pos < s0 + s1 t + s2 d (conserved states, zero derivatives for SEG_STATE)
    edges: Optional[tuple] = None
    # (i_s, j_s): cells i >= i_s, j < j_s are solid (a step against the bottom-right corner)
    obstacle: Optional[tuple] = None

    @property
    def nx(self) -> int:
        return self.S.shape[2]

    @property
    def ny(self) -> int:
        return self.S.shape[1]

    @property
    def m(self) -> int:
        return self.S.shape[0] // (1 + self.dim)


def centers(n: int, lo: float, hi: float) -> np.ndarray:
    """Cell centres x_i = lo + (i + 1/2) dx of n uniform cells on [lo, hi]."""
    dx = (hi - lo) / n
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * dx


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# primitive -> conserved (definition of the Euler state, not of the scheme)
# ---------------------------------------------------------------------------

def conserved_1d(rho, u, p, gamma=GAMMA_GAS):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def conserved_2d(rho, u, v, p, gamma=GAMMA_GAS):
    return np.stack([rho, rho * u, rho * v,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


# ---------------------------------------------------------------------------
# scalar problems
# ---------------------------------------------------------------------------

def scalar_sine_1d(n: int, physics: str = "linadv", lo=0.0, hi=2.0,
                   a: float = 1.0) -> Workload:
    """u0 = 0.5 + sin(pi x) on [lo, hi] periodic; v0 = pi cos(pi x)."""
    x = centers(n, lo, hi)
    S = np.zeros((2, 1, n))
    S[0, 0] = 0.5 + np.sin(np.pi * x)
    S[1, 0] = np.pi * np.cos(np.pi * x)
    return Workload(S, 1, physics, (hi - lo) / n, 1.0, PERIODIC, PERIODIC,
                    (lo, 0.0), (hi, 1.0), adv_speed=(a, 0.0),
                    name=f"{physics}1d_sine_{n}")


def scalar_sine_2d(nx: int, ny: int, physics: str = "burgers", lo=0.0, hi=4.0,
                   a=(1.0, 1.0)) -> Workload:
    """u0 = 0.5 + sin(pi (x + y) / 2) on [lo, hi]^2 periodic, with derivatives."""
    x = centers(nx, lo, hi)[None, :]
    y = centers(ny, lo, hi)[:, None]
    arg = np.pi * (x + y) / 2.0
    S = np.zeros((3, ny, nx))
    S[0] = 0.5 + np.sin(arg)
    S[1] = 0.5 * np.pi * np.cos(arg)
    S[2] = 0.5 * np.pi * np.cos(arg)
    return Workload(S, 2, physics, (hi - lo) / nx, (hi - lo) / ny, PERIODIC,
                    PERIODIC, (lo, lo), (hi, hi), adv_speed=tuple(a),
                    name=f"{physics}2d_sine_{nx}x{ny}")


def scalar_random_2d(nx: int, ny: int, seed: int, physics="linadv",
                     a=(1.0, -0.5)) -> Workload:
    """Rough random scalar data (values and derivatives U[-1, 1]) on [0,1]^2."""
    g = rng(seed)
    S = g.uniform(-1.0, 1.0, size=(3, ny, nx))
    return Workload(S, 2, physics, 1.0 / nx, 1.0 / ny, PERIODIC, PERIODIC,
                    adv_speed=tuple(a), name=f"{physics}2d_random_{nx}x{ny}_s{seed}")


def scalar_random_1d(n: int, seed: int, physics="linadv", a=1.0) -> Workload:
    g = rng(seed)
    S = g.uniform(-1.0, 1.0, size=(2, 1, n))
    return Workload(S, 1, physics, 1.0 / n, 1.0, PERIODIC, PERIODIC,
                    adv_speed=(a, 0.0), name=f"{physics}1d_random_{n}_s{seed}")


# ---------------------------------------------------------------------------
# 1D Euler
# ---------------------------------------------------------------------------

def euler1d_smooth(n: int, lo=0.0, hi=2.0, amp=0.2) -> Workload:
    """Density wave rho = 1 + amp sin(pi x), u = 1, p = 1 on [lo, hi] periodic."""
    x = centers(n, lo, hi)
    rho = 1.0 + amp * np.sin(np.pi * x)
    rho_x = amp * np.pi * np.cos(np.pi * x)
    u = np.ones_like(x)
    p = np.ones_like(x)
    U = conserved_1d(rho, u, p)
    # u and p constant: m_x = rho_x, E_x = rho_x / 2
    D = np.stack([rho_x, rho_x, 0.5 * rho_x])
    S = np.concatenate([U, D])[:, None, :]
    return Workload(S, 1, "euler", (hi - lo) / n, 1.0, PERIODIC, PERIODIC,
                    (lo, 0.0), (hi, 1.0), name=f"euler1d_smooth_{n}")


def euler1d_piecewise(n: int, seed: int, lo=0.0, hi=2.0) -> Workload:
    """Piecewise-constant data with k ~ U{1..5} jumps at sorted uniform points.

    Each of the k+1 pieces draws rho ~ U[0.1, 2], u ~ U[-1, 1], p ~ U[0.1, 5];
    derivatives are zero.  Periodic, so the seam is one more jump unless the
    end states agree.
    """
    g = rng(seed)
    k = int(g.integers(1, 6))
    cuts = np.sort(g.uniform(lo, hi, size=k))
    rho = g.uniform(0.1, 2.0, size=k + 1)
    u = g.uniform(-1.0, 1.0, size=k + 1)
    p = g.uniform(0.1, 5.0, size=k + 1)
    x = centers(n, lo, hi)
    piece = np.searchsorted(cuts, x)
    U = conserved_1d(rho[piece], u[piece], p[piece])
    S = np.concatenate([U, np.zeros_like(U)])[:, None, :]
    return Workload(S, 1, "euler", (hi - lo) / n, 1.0, PERIODIC, PERIODIC,
                    (lo, 0.0), (hi, 1.0), name=f"euler1d_piecewise_{n}_s{seed}",
                    info={"jumps": k})


def _riemann_1d(n, lo, hi, cuts, states, bc, name):
    """Piecewise-constant (rho, u, p) states separated at ``cuts``; zero derivatives."""
    x = centers(n, lo, hi)
    piece = np.searchsorted(np.asarray(cuts), x)
    st = np.asarray(states, dtype=np.float64)
    U = conserved_1d(st[piece, 0], st[piece, 1], st[piece, 2])
    S = np.concatenate([U, np.zeros_like(U)])[:, None, :]
    return Workload(S, 1, "euler", (hi - lo) / n, 1.0, bc, bc, (lo, 0.0), (hi, 1.0), name=name)


def lax_1d(n: int) -> Workload:
    """Lax shock tube (Example 3.5): (0.445, 0.698, 3.528) for x < 0, (0.5, 0, 0.571)
    for x > 0 on [-0.5, 0.5] with outflow boundaries; the paper runs it to T = 0.16."""
    return _riemann_1d(n, -0.5, 0.5, [0.0], [(0.445, 0.698, 3.528), (0.5, 0.0, 0.571)],
                       OUTFLOW, f"lax_{n}")


def blast_waves_1d(n: int) -> Workload:
    """Two interacting blast waves (Example 3.7): rho = 1, u = 0, p = 1000 / 0.01 / 100
    on (0, 0.1) / (0.1, 0.9) / (0.9, 1), reflecting walls at both ends; T = 0.038."""
    return _riemann_1d(n, 0.0, 1.0, [0.1, 0.9], [(1.0, 0.0, 1e3), (1.0, 0.0, 1e-2), (1.0, 0.0, 1e2)],
                       REFLECT, f"blast_waves_{n}")


def shu_osher_1d(n: int) -> Workload:
    """Shock / entropy-wave interaction (Example 3.6): (3.857143, 2.629369, 10.333333)
    for x < -4, (1 + 0.2 sin 5x, 0, 1) for x >= -4, on [-5, 5] with outflow
    boundaries; T = 1.8.  Derivatives: those of the smooth piece, zero elsewhere."""
    lo, hi = -5.0, 5.0
    x = centers(n, lo, hi)
    left = x < -4.0
    rho = np.where(left, 3.857143, 1.0 + 0.2 * np.sin(5.0 * x))
    u = np.where(left, 2.629369, 0.0)
    p = np.where(left, 10.333333, 1.0)
    U = conserved_1d(rho, u, p)
    # right piece: u = 0, p = 1, so m_x = E_x = 0 and only rho_x = cos(5x) is nonzero
    D = np.zeros_like(U)
    D[0] = np.where(left, 0.0, np.cos(5.0 * x))
    S = np.concatenate([U, D])[:, None, :]
    return Workload(S, 1, "euler", (hi - lo) / n, 1.0, OUTFLOW, OUTFLOW, (lo, 0.0), (hi, 1.0),
                    name=f"shu_osher_{n}")


# ---------------------------------------------------------------------------
# 2D Euler
# ---------------------------------------------------------------------------

def normal_shock_states(mach: float, rho1: float, p1: float, gamma=GAMMA_GAS):
    """Rankine-Hugoniot states of a normal shock of Mach number ``mach`` moving
    into gas at rest (rho1, p1): (shock speed, rho2, normal velocity u2, p2)."""
    c1 = np.sqrt(gamma * p1 / rho1)
    s = mach * c1
    m2 = mach * mach
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    u2 = s * (1.0 - rho1 / rho2)
    return s, rho2, u2, p2


def double_mach(nx: int, ny: int) -> Workload:
    """Double Mach reflection (Example 3.11) on [0, 4] x [0, 1], T = 0.2: a Mach 10
    shock into (rho, u, v, p) = (1.4, 0, 0, 1), through (1/6, 0) at 60 degrees to
    the x axis, moving along its normal n = (sin 60, -cos 60).  Post-shock state from
    the Rankine-Hugoniot relations (rho = 8, |u| = 8.25, p = 116.5).  Boundaries:
    post-shock inflow on the left; outflow on the right; on the bottom post-shock
    inflow for x < 1/6 and a wall beyond; on the top the exact shock, which meets
    the height y = 1 + d of a ghost centre at x = 1/6 + y / sqrt(3) + s t / sin 60."""
    lo, hi = (0.0, 0.0), (4.0, 1.0)
    x = centers(nx, lo[0], hi[0])[None, :]
    y = centers(ny, lo[1], hi[1])[:, None]
    s, rho2, u2, p2 = normal_shock_states(10.0, 1.4, 1.0)
    nrm = (np.sin(np.pi / 3.0), -np.cos(np.pi / 3.0))
    x0, r3 = 1.0 / 6.0, np.sqrt(3.0)
    post = (rho2, u2 * nrm[0], u2 * nrm[1], p2)
    pre = (1.4, 0.0, 0.0, 1.0)
    behind = x < x0 + y / r3
    prim = [np.where(behind, a, b) * np.ones((ny, nx)) for a, b in zip(post, pre)]
    U = conserved_2d(*prim)
    S = np.concatenate([U, np.zeros_like(U), np.zeros_like(U)])
    post_c = tuple(float(v[0, 0]) for v in conserved_2d(*[np.full((1, 1), q) for q in post]))
    pre_c = tuple(float(v[0, 0]) for v in conserved_2d(*[np.full((1, 1), q) for q in pre]))
    inflow = ((SEG_STATE, SEG_STATE), (0.0, 0.0, 0.0), (post_c, post_c))
    outflow = ((SEG_OUTFLOW, SEG_OUTFLOW), (0.0, 0.0, 0.0), (pre_c, pre_c))
    bottom = ((SEG_STATE, SEG_REFLECT), (x0, 0.0, 0.0), (post_c, pre_c))
    top = ((SEG_STATE, SEG_STATE), (x0 + hi[1] / r3, s / nrm[0], 1.0 / r3), (post_c, pre_c))
    return Workload(S, 2, "euler", (hi[0] - lo[0]) / nx, (hi[1] - lo[1]) / ny, EDGES, EDGES,
                    lo, hi, name=f"double_mach_{nx}x{ny}",
                    info={"t_end": 0.2, "shock_speed": s, "post": post, "pre": pre},
                    edges=(inflow, outflow, bottom, top))

def forward_step(nx: int, ny: int) -> Workload:
    """Forward-facing step (Example 3.12): a wind tunnel [0, 3] x [0, 1] with a step
    from x = 0.6 to the exit, 0.2 high, filled with a right-going Mach 3 flow
    (rho, u, v, p) = (1.4, 3, 0, 1); inflow of that state on the left, outflow on the
    right, walls on the bottom, the top and the step; T = 4.  nx and ny must be
    multiples of 5 so that the step's faces fall on cell faces."""
    if nx % 5 or ny % 5:
        raise ValueError("nx and ny must be multiples of 5")
    lo, hi = (0.0, 0.0), (3.0, 1.0)
    free = (1.4, 3.0, 0.0, 1.0)
    U = conserved_2d(*[np.full((ny, nx), q) for q in free])
    S = np.concatenate([U, np.zeros_like(U), np.zeros_like(U)])
    q = tuple(float(v[0, 0]) for v in conserved_2d(*[np.full((1, 1), c) for c in free]))
    inflow = ((SEG_STATE, SEG_STATE), (0.0, 0.0, 0.0), (q, q))
    outflow = ((SEG_OUTFLOW, SEG_OUTFLOW), (0.0, 0.0, 0.0), (q, q))
    return Workload(S, 2, "euler", (hi[0] - lo[0]) / nx, (hi[1] - lo[1]) / ny, EDGES, REFLECT,
                    lo, hi, name=f"forward_step_{nx}x{ny}", info={"t_end": 4.0, "free": free},
                    edges=(inflow, outflow, outflow, outflow), obstacle=(nx // 5, ny // 5))


def euler2d_quadrants(nx: int, ny: int, seed: int, bc=OUTFLOW) -> Workload:
    """Four constant quadrants of [0,1]^2 split at x = 1/2, y = 1/2.

    Each quadrant draws rho ~ U[0.1, 2], u, v ~ U[-1, 1], p ~ U[0.1, 2];
    derivatives are zero; outflow boundaries by default.
    """
    g = rng(seed)
    rho = g.uniform(0.1, 2.0, size=4)
    u = g.uniform(-1.0, 1.0, size=4)
    v = g.uniform(-1.0, 1.0, size=4)
    p = g.uniform(0.1, 2.0, size=4)
    x = centers(nx, 0.0, 1.0)[None, :]
    y = centers(ny, 0.0, 1.0)[:, None]
    q = (x >= 0.5).astype(np.int64) + 2 * (y >= 0.5).astype(np.int64)
    U = conserved_2d(rho[q], u[q], v[q], p[q])
    S = np.concatenate([U, np.zeros_like(U), np.zeros_like(U)])
    return Workload(S, 2, "euler", 1.0 / nx, 1.0 / ny, bc, bc,
                    name=f"euler2d_quadrants_{nx}x{ny}_s{seed}")


def euler2d_wave(nx: int, ny: int, lo=0.0, hi=2.0, amp=0.2, k=1.0,
                 phase=0.0, u0=1.0, v0=1.0, p0=1.0) -> Workload:
    """rho = 1 + amp sin(k pi (x + y) + phase), u = u0, v = v0, p = p0, periodic.

    With k = 1 on [0, 2]^2 this is the 2D density wave; with k = 2 on
    [0, 1]^2 it is the smooth instance type of the batched workload.
    """
    x = centers(nx, lo, hi)[None, :]
    y = centers(ny, lo, hi)[:, None]
    arg = k * np.pi * (x + y) + phase
    rho = 1.0 + amp * np.sin(arg) + 0.0 * (x + y)
    drho = amp * k * np.pi * np.cos(arg) + 0.0 * (x + y)
    one = np.ones_like(rho)
    U = conserved_2d(rho, u0 * one, v0 * one, p0 * one)
    # velocities and pressure constant: m_d = u0 rho_d, n_d = v0 rho_d,
    # E_d = (u0^2 + v0^2)/2 rho_d, and rho_x = rho_y = drho
    D = np.stack([drho, u0 * drho, v0 * drho, 0.5 * (u0 * u0 + v0 * v0) * drho])
    S = np.concatenate([U, D, D])
    return Workload(S, 2, "euler", (hi - lo) / nx, (hi - lo) / ny, PERIODIC,
                    PERIODIC, (lo, lo), (hi, hi), name=f"euler2d_wave_{nx}x{ny}")


def euler2d_random_smooth(nx: int, ny: int, seed: int, bc=PERIODIC) -> Workload:
    """Smooth but non-trivial periodic 2D Euler data on [0,1]^2 (all fields vary)."""
    g = rng(seed)
    x = centers(nx, 0.0, 1.0)[None, :]
    y = centers(ny, 0.0, 1.0)[:, None]
    tp = 2.0 * np.pi

    def wave(base, amp):
        kx, ky = g.integers(1, 3, size=2)
        ph = g.uniform(0.0, tp)
        arg = tp * (kx * x + ky * y) + ph
        return (base + amp * np.sin(arg),
                amp * tp * kx * np.cos(arg), amp * tp * ky * np.cos(arg))

    r, rx, ry = wave(1.0, 0.2)
    u, ux, uy = wave(0.3, 0.3)
    v, vx, vy = wave(-0.2, 0.3)
    p, px, py = wave(1.0, 0.2)
    gm1 = GAMMA_GAS - 1.0
    U = conserved_2d(r, u, v, p)

    def dcons(rd, ud, vd, pd):
        return np.stack([rd, rd * u + r * ud, rd * v + r * vd,
                         pd / gm1 + 0.5 * rd * (u * u + v * v) + r * (u * ud + v * vd)])

    S = np.concatenate([U, dcons(rx, ux, vx, px), dcons(ry, uy, vy, py)])
    return Workload(S, 2, "euler", 1.0 / nx, 1.0 / ny, bc, bc,
                    name=f"euler2d_rsmooth_{nx}x{ny}_s{seed}")


def euler2d_rough(nx: int, ny: int, seed: int, bc=OUTFLOW) -> Workload:
    """Admissible random cell data with random derivatives (stress input)."""
    g = rng(seed)
    rho = g.uniform(0.2, 2.0, size=(ny, nx))
    u = g.uniform(-1.0, 1.0, size=(ny, nx))
    v = g.uniform(-1.0, 1.0, size=(ny, nx))
    p = g.uniform(0.5, 2.0, size=(ny, nx))
    U = conserved_2d(rho, u, v, p)
    D1 = g.uniform(-1.0, 1.0, size=U.shape) * nx * 0.05
    D2 = g.uniform(-1.0, 1.0, size=U.shape) * ny * 0.05
    S = np.concatenate([U, D1, D2])
    return Workload(S, 2, "euler", 1.0 / nx, 1.0 / ny, bc, bc,
                    name=f"euler2d_rough_{nx}x{ny}_s{seed}")


def roughened(w: Workload, seed: int, amp: float = 0.2, slope: float = 0.05) -> Workload:
    """A copy of a 2D Euler workload with seeded cell-by-cell noise (stress input
    with structure in every stencil and next to every side): rho and p multiplied
    by U[1 - amp, 1 + amp], each velocity component shifted by amp * U[-1, 1] times
    the local sound speed, and random derivative fields of size slope * n as in
    euler2d_rough.  Geometry, boundaries, edges and obstacle are kept."""
    g = rng(seed)
    ny, nx = w.ny, w.nx
    rho, mx, my, E = (w.S[c] for c in range(4))
    u, v = mx / rho, my / rho
    p = (w.gamma_gas - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    c = np.sqrt(w.gamma_gas * p / rho)
    rho = rho * g.uniform(1.0 - amp, 1.0 + amp, size=(ny, nx))
    p = p * g.uniform(1.0 - amp, 1.0 + amp, size=(ny, nx))
    u = u + amp * c * g.uniform(-1.0, 1.0, size=(ny, nx))
    v = v + amp * c * g.uniform(-1.0, 1.0, size=(ny, nx))
    U = conserved_2d(rho, u, v, p, w.gamma_gas)
    D1 = g.uniform(-1.0, 1.0, size=U.shape) * nx * slope
    D2 = g.uniform(-1.0, 1.0, size=U.shape) * ny * slope
    return Workload(np.concatenate([U, D1, D2]), 2, "euler", w.dx, w.dy, w.bc_x, w.bc_y,
                    w.lo, w.hi, w.gamma_gas, w.adv_speed, name=f"{w.name}_rough_s{seed}",
                    info=dict(w.info), edges=w.edges, obstacle=w.obstacle)


# ---------------------------------------------------------------------------
# batched uneven 2D Euler instances
# ---------------------------------------------------------------------------

def batched_instances(n_inst: int, seed: int, side_lo=64, side_hi=512,
                      sizes: Optional[List[tuple]] = None) -> List[Workload]:
    """Independent 2D Euler instances on [0,1]^2 with uneven grids.

    Sides nx, ny ~ U{side_lo..side_hi} independently (unless ``sizes`` is
    given).  Instance type ~ Bernoulli(1/2): four-quadrant data (outflow) or
    a smooth wave rho = 1 + A sin(2 pi (x + y) + phi), A ~ U[0.05, 0.2],
    phi ~ U[0, 2 pi), u = v = p = 1 (periodic).
    """
    g = rng(seed)
    out = []
    for k in range(n_inst):
        if sizes is None:
            nx = int(g.integers(side_lo, side_hi + 1))
            ny = int(g.integers(side_lo, side_hi + 1))
        else:
            nx, ny = sizes[k]
        if g.uniform() < 0.5:
            w = euler2d_quadrants(nx, ny, seed=int(g.integers(0, 2**31)))
        else:
            amp = float(g.uniform(0.05, 0.2))
            ph = float(g.uniform(0.0, 2.0 * np.pi))
            w = euler2d_wave(nx, ny, lo=0.0, hi=1.0, amp=amp, k=2.0, phase=ph)
        w.name = f"inst{k}_" + w.name
        out.append(w)
    return out


# ---------------------------------------------------------------------------
# adjoint workload
# ---------------------------------------------------------------------------

def adjoint_pair(n: int, seed: int):
    """Initial smooth state U0 and a seed-perturbed state whose rollout is the target.

    U0: rho = 1 + 0.2 sin(2 pi (x + y)), u = v = p = 1 on [0,1]^2 periodic.
    Perturbation of the density: 0.02 sum_k a_k sin(2 pi (kx x + ky y) + phi_k),
    k = 1..3, a_k ~ U[0.5, 1], (kx, ky) ~ U{1..3}^2, phi_k ~ U[0, 2 pi).
    """
    g = rng(seed)
    base = euler2d_wave(n, n, lo=0.0, hi=1.0, amp=0.2, k=2.0)
    x = centers(n, 0.0, 1.0)[None, :]
    y = centers(n, 0.0, 1.0)[:, None]
    tp = 2.0 * np.pi
    drho = np.zeros((n, n))
    drho_x = np.zeros((n, n))
    drho_y = np.zeros((n, n))
    for _ in range(3):
        a = g.uniform(0.5, 1.0)
        kx, ky = g.integers(1, 4, size=2)
        ph = g.uniform(0.0, tp)
        arg = tp * (kx * x + ky * y) + ph
        drho += 0.02 * a * np.sin(arg)
        drho_x += 0.02 * a * tp * kx * np.cos(arg)
        drho_y += 0.02 * a * tp * ky * np.cos(arg)
    pert = base.S.copy()
    # u = v = 1 and p = 1 stay: m = rho, n = rho, E = 1/(g-1) + rho
    for c, s in ((0, 1.0), (1, 1.0), (2, 1.0), (3, 1.0)):
        pert[c] += s * drho
        pert[4 + c] += s * drho_x
        pert[8 + c] += s * drho_y
    target = Workload(pert, 2, "euler", base.dx, base.dy, PERIODIC, PERIODIC,
                      base.lo, base.hi, name=f"adjoint_target_{n}_s{seed}")
    return base, target
