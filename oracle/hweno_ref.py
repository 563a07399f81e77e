"""Plain, slow FP64 CPU oracle of the L-HWENO hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import or run this module.  It shares no code with the
HIP library and imports nothing from the product package.

Source: Zhang & Zhao, "A fifth-order finite difference HWENO scheme combined
with limiter for hyperbolic conservation laws" (arXiv 2207.05258).  Every
function names the passage it follows.  Tensors are torch float64 on the CPU,
so that torch autograd of this forward (with the wave speeds and the time step
held fixed) serves as the oracle adjoint.

State layout: ``S[nf, ny, nx]`` with the m conserved components U, then U_x,
then (2D) U_y; ``ny == 1`` in one dimension.

Readings of passages the paper leaves open (each listed in the design notes):
  * beta_2 of the quadratic on {x_i, x_{i+1}} is taken from its definition
    (eq. GHYZ); the printed explicit form has f_{i-1} where the definition
    gives f_{i+1}.
  * The "-" reconstruction is the mirror image of the "+" one about
    x_{i+1/2}: indices reflected, derivative data negated, and the returned
    derivative negated.
  * The global Lax-Friedrichs speed is one scalar per direction, the maximum
    of |f'(u)| (Euler: |u_d| + c) over the grid of the state the operator is
    evaluated on, recomputed at every Runge-Kutta stage.
  * Characteristic decomposition uses the Roe average of the two cells next
    to the interface; right eigenvectors scaled as documented in
    ``Euler.right_eigenvectors``; L = R^{-1} by a numerical inverse; both the
    split fluxes and the split derivative fluxes are projected.
  * The limiter acts component by component on the conserved variables:
    U_x along x, U_y along y.  An optional variant (``limiter_characteristic``)
    limits the characteristic fields of each cell's own state instead.
  * The mixed fluxes use the step sizes of eq. (ode2H): the y-differences of
    xi-hat are divided by dy and the x-differences of eta-hat by dx.
  * Outflow boundaries copy the nearest interior value of every field.
  * Reflecting walls (Euler, Example 3.7) fill ghost cells with the mirror
    image of the interior, with the wall-normal momentum and the derivatives
    along the wall normal negated.
  * The step of Example 3.12 is an obstacle of solid cells (i >= i_s, j < j_s)
    whose faces are walls: for the fluxes and the limiter along x a solid cell
    holds the mirror image of the fluid across the front face, along y the
    mirror image across the top face.  Solid cells keep their state.  The
    paper treats the step corner "as in" its reference, which is not at hand:
    no corner correction is applied.
  * Edge-described sides (the boundaries of Example 3.11): a side is cut in
    two segments at split = s0 + s1 t + s2 d along it (d: distance of the
    ghost centre beyond the side).  A segment is an outflow copy, a wall, or
    an inflow holding a prescribed state with zero derivatives ("exact
    post-shock condition", "exact motion of the shock").  Each Runge-Kutta
    stage reads the ghosts at the time of its input state: t, t + dt,
    t + dt/2.

Parity unpinned (documented choices with nothing in the paper to check them
against): the component-wise limiter for systems, and the zero derivatives in
the ghost cells of inflow segments (pinned only where an edge reduces to a
plain boundary or a state that is already uniform).  The characteristic
limiter variant is pinned only through its special cases (linear weights, data
along one eigenvector).  The outflow copy is pinned by the domain it stands
for: repeating the edge cells outward leaves the operator and the limiter of
the original cells unchanged, and a step of data that are constant next to an
outflow side equals the step of the domain extended by that constant.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import torch

DTYPE = torch.float64

PERIODIC = 0
OUTFLOW = 1
REFLECT = 2   # solid wall: mirror image, wall-normal momentum and normal derivatives odd
EDGES = 3     # each side of the direction described by an Edge

SEG_OUTFLOW, SEG_REFLECT, SEG_STATE = 0, 1, 2


@dataclass(frozen=True)
class Edge:
    """One side of the domain cut in two segments (Example 3.11's boundaries).

    A ghost cell at position ``pos`` along the side (measured from the domain's
    low corner, cell centres at (j + 1/2) h) and distance ``d`` beyond it takes
    segment 0 when pos < split[0] + split[1] t + split[2] d, else segment 1.
    Kinds: SEG_OUTFLOW (copy), SEG_REFLECT (wall), SEG_STATE (``state[s]``,
    conserved variables, with zero derivatives)."""

    kind: Tuple[int, int] = (SEG_OUTFLOW, SEG_OUTFLOW)
    split: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    state: Tuple[Tuple[float, ...], Tuple[float, ...]] = ((0.0,) * 4, (0.0,) * 4)


@dataclass
class Problem:
    """Parameters of one discretised problem (Section 3 defaults)."""

    dim: int = 1
    physics: str = "linadv"          # "linadv" | "burgers" | "euler"
    dx: float = 1.0
    dy: float = 1.0
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    gamma_gas: float = 1.4
    adv_speed: Tuple[float, float] = (1.0, 1.0)
    lin_w: Tuple[float, float, float] = (0.98, 0.01, 0.01)   # gamma_0..2
    lim_w: Tuple[float, float, float] = (0.98, 0.01, 0.01)   # d_0..2
    eps: float = 1e-6
    cfl: float = 0.6
    characteristic: bool = True
    limiter_on: bool = True
    # Euler only: apply the limiter to local characteristic fields of each cell
    # instead of component by component (a variant; the paper does not say)
    limiter_characteristic: bool = False
    # sides x_lo, x_hi, y_lo, y_hi, read where bc_x / bc_y is EDGES
    edges: Optional[Tuple[Edge, Edge, Edge, Edge]] = None
    # (i_s, j_s): the cells i >= i_s, j < j_s are solid (the step of Example 3.12)
    obstacle: Optional[Tuple[int, int]] = None
    # test-only switches: force the nonlinear weights to the linear ones
    linear_recon: bool = False
    linear_limiter: bool = False

    @property
    def m(self) -> int:
        if self.physics == "euler":
            return 3 if self.dim == 1 else 4
        return 1

    @property
    def nf(self) -> int:
        return self.m * (1 + self.dim)


def problem_from_workload(w, **kw) -> Problem:
    obstacle = getattr(w, "obstacle", None)
    if obstacle is not None and "obstacle" not in kw:
        kw["obstacle"] = tuple(obstacle)
    edges = getattr(w, "edges", None)
    if edges is not None and "edges" not in kw:
        kw["edges"] = tuple(Edge(kind=tuple(e[0]), split=tuple(e[1]),
                                 state=(tuple(e[2][0]), tuple(e[2][1]))) for e in edges)
    return Problem(dim=w.dim, physics=w.physics, dx=w.dx, dy=w.dy,
                   bc_x=w.bc_x, bc_y=w.bc_y, gamma_gas=w.gamma_gas,
                   adv_speed=tuple(w.adv_speed), **kw)


# ===========================================================================
# Section 2.1: Hermite reconstruction of the "+" flux at x_{i+1/2}
# Data: f_{i-1}, f_i, f_{i+1} (split point fluxes) and H_l = dx * h_l.
# ===========================================================================

def hermite_values(fm, f0, fp, Hm, H0, Hp):
    """p_0, p_1, p_2 at x_{i+1/2} (Section 2.1, the values following eq. HWEp12)."""
    p0 = 11.0 / 60.0 * fm + 19.0 / 30.0 * f0 + 11.0 / 60.0 * fp \
        + (Hm + 10.0 * H0 - Hp) / 20.0
    p1 = fm / 6.0 + 5.0 / 6.0 * f0 + 2.0 / 3.0 * H0
    p2 = 5.0 / 6.0 * f0 + fp / 6.0 + H0 / 3.0
    return p0, p1, p2


def quintic_coefficients(fm, f0, fp, Hm, H0, Hp):
    """a_1..a_5 of p_0 in the scaled variable (x - x_i)/dx (Section 2.1)."""
    a1 = 19.0 / 192.0 * Hm + 79.0 / 48.0 * H0 + 19.0 / 192.0 * Hp \
        + 27.0 / 64.0 * (fm - fp)
    a2 = 3.0 / 8.0 * Hm - 3.0 / 8.0 * Hp + 5.0 / 4.0 * (fm - 2.0 * f0 + fp)
    a3 = -(11.0 / 24.0 * Hm + 17.0 / 6.0 * H0 + 11.0 / 24.0 * Hp) \
        + 15.0 / 8.0 * (fp - fm)
    a4 = 0.25 * Hp - 0.25 * Hm - 0.5 * (fm - 2.0 * f0 + fp)
    a5 = 0.25 * Hm + H0 + 0.25 * Hp + 0.75 * (fm - fp)
    return a1, a2, a3, a4, a5


def smoothness_indicators(fm, f0, fp, Hm, H0, Hp):
    """beta_0, beta_1, beta_2 (eq. GHYZ / GHYZP; beta_2 from its definition)."""
    a1, a2, a3, a4, a5 = quintic_coefficients(fm, f0, fp, Hm, H0, Hp)
    b0 = (a1 + a3 / 4.0 + a5 / 16.0) ** 2 \
        + 13.0 / 3.0 * (a2 + 63.0 / 130.0 * a4) ** 2 \
        + 781.0 / 20.0 * (a3 + 8825.0 / 10934.0 * a5) ** 2 \
        + 1421461.0 / 2275.0 * a4 ** 2 \
        + 21520059541.0 / 1377684.0 * a5 ** 2
    b1 = H0 ** 2 + 13.0 / 3.0 * (H0 - f0 + fm) ** 2
    b2 = H0 ** 2 + 13.0 / 3.0 * (H0 + f0 - fp) ** 2
    return b0, b1, b2


def nonlinear_weights(b0, b1, b2, lin, eps):
    """omega_l from tau (eq. tau-fh) and the normalised bar-omega (Section 2.1)."""
    tau = 0.25 * ((b0 - b1).abs() + (b0 - b2).abs()) ** 2
    w0 = lin[0] * (1.0 + tau / (b0 + eps))
    w1 = lin[1] * (1.0 + tau / (b1 + eps))
    w2 = lin[2] * (1.0 + tau / (b2 + eps))
    s = w0 + w1 + w2
    return w0 / s, w1 / s, w2 / s


def hweno_plus(fm, f0, fp, Hm, H0, Hp, lin, eps, linear=False):
    """Nonlinear HWENO value f-hat^+_{i+1/2} (Section 2.1, final combination).

    With ``linear=True`` the nonlinear weights are replaced by the linear
    ones, which reduces the combination to p_0 (test switch).
    """
    p0, p1, p2 = hermite_values(fm, f0, fp, Hm, H0, Hp)
    if linear:
        w0, w1, w2 = lin
    else:
        b0, b1, b2 = smoothness_indicators(fm, f0, fp, Hm, H0, Hp)
        w0, w1, w2 = nonlinear_weights(b0, b1, b2, lin, eps)
    g0, g1, g2 = lin
    return w0 * (p0 / g0 - g1 / g0 * p1 - g2 / g0 * p2) + w1 * p1 + w2 * p2


def quintic_derivative(fm, f0, fp, hm, h0, hp, dx):
    """p_0'(x_{i+1/2}) (Section 2.1): the linear derivative-equation flux h-hat^+."""
    return (fm - 8.0 * f0 + 7.0 * fp) / (4.0 * dx) + (hm - 2.0 * h0 - 5.0 * hp) / 12.0


def hweno_minus(f_i, f_ip1, f_ip2, H_i, H_ip1, H_ip2, lin, eps, linear=False):
    """f-hat^-_{i+1/2}: the "+" procedure mirrored about x_{i+1/2} (Section 2.1).

    Reflection maps cell i+1 to the centre, i+2 to the upwind side and i to
    the downwind side; derivative data change sign under the reflection.
    """
    return hweno_plus(f_ip2, f_ip1, f_i, -H_ip2, -H_ip1, -H_i, lin, eps, linear)


def quintic_derivative_minus(f_i, f_ip1, f_ip2, h_i, h_ip1, h_ip2, dx):
    """h-hat^-_{i+1/2}: mirrored p_0' (derivative of the reflected polynomial negated)."""
    return -quintic_derivative(f_ip2, f_ip1, f_i, -h_ip2, -h_ip1, -h_i, dx)


# ===========================================================================
# Section 2.2: HWENO limiter for the derivative at x_i
# Inputs u_{i-1}, u_i, u_{i+1}, v_{i-1}, v_{i+1}; v_i is not used.
# ===========================================================================

def limiter_candidates(um, u0, up, vm, vp, dx):
    """q_0'(x_i), q_1'(x_i), q_2'(x_i) (Section 2.2)."""
    q0 = 3.0 / (4.0 * dx) * (up - um) - 0.25 * (vm + vp)
    q1 = (u0 - um) / dx
    q2 = (up - u0) / dx
    return q0, q1, q2


def limiter_smoothness(um, u0, up, vm, vp, dx):
    """beta_0..2 of q_0, q_1, q_2 (eq. GHYZ-q and its explicit form)."""
    a1 = -dx / 4.0 * (vm + vp) + 0.75 * (up - um)
    a2 = dx / 4.0 * (vm - vp) + um - 2.0 * u0 + up
    a3 = dx / 4.0 * (vm + vp) + 0.25 * (um - up)
    a4 = dx / 4.0 * (vp - vm) - 0.5 * (um - 2.0 * u0 + up)
    b0 = (a1 + a3 / 4.0) ** 2 + 13.0 / 3.0 * (a2 + 63.0 / 130.0 * a4) ** 2 \
        + 781.0 / 20.0 * a3 ** 2 + 1421461.0 / 2275.0 * a4 ** 2
    b1 = (u0 - um) ** 2
    b2 = (u0 - up) ** 2
    return b0, b1, b2


def limit_derivative(um, u0, up, vm, vp, dx, d, eps, linear=False):
    """Modified derivative v-tilde_i (Section 2.2, final combination)."""
    q0, q1, q2 = limiter_candidates(um, u0, up, vm, vp, dx)
    if linear:
        l0, l1, l2 = d
    else:
        b0, b1, b2 = limiter_smoothness(um, u0, up, vm, vp, dx)
        l0, l1, l2 = nonlinear_weights(b0, b1, b2, d, eps)
    d0, d1, d2 = d
    return l0 * (q0 / d0 - d1 / d0 * q1 - d2 / d0 * q2) + l1 * q1 + l2 * q2


# ===========================================================================
# Physics: fluxes, chain-rule derivative fluxes, wave speeds, eigenvectors
# (eq. EQ1 / EQ3 definitions of h, xi, eta, theta; eqs. euler1 / euler2)
# Component index is the LAST axis in this section.
# ===========================================================================

class Scalar:
    """f(u) = a_x u, g(u) = a_y u (linear advection) or u^2/2 (Burgers)."""

    def __init__(self, prob: Problem):
        self.prob = prob

    def flux(self, U, d):
        if self.prob.physics == "linadv":
            return self.prob.adv_speed[d] * U
        return 0.5 * U * U

    def jvp(self, U, D, d):
        """f'(u) D: h = f'(u) v, xi = g'(u) v, eta = f'(u) w, theta = g'(u) w."""
        if self.prob.physics == "linadv":
            return self.prob.adv_speed[d] * D
        return U * D

    def speed(self, U, d):
        if self.prob.physics == "linadv":
            return torch.full_like(U[..., 0], abs(self.prob.adv_speed[d]))
        return U[..., 0].abs()

    def right_eigenvectors(self, UL, UR, d):
        return torch.ones(UL.shape[:-1] + (1, 1), dtype=DTYPE)


class Euler:
    """Compressible Euler, E = p/(gamma-1) + rho |vel|^2 / 2 (eqs. euler1, euler2)."""

    def __init__(self, prob: Problem):
        self.g = prob.gamma_gas
        self.dim = prob.dim

    def _prim(self, U):
        rho = U[..., 0]
        u = U[..., 1] / rho
        if self.dim == 1:
            v = torch.zeros_like(u)
            E = U[..., 2]
        else:
            v = U[..., 2] / rho
            E = U[..., 3]
        p = (self.g - 1.0) * (E - 0.5 * rho * (u * u + v * v))
        return rho, u, v, E, p

    def flux(self, U, d):
        rho, u, v, E, p = self._prim(U)
        if self.dim == 1:
            return torch.stack([rho * u, rho * u * u + p, u * (E + p)], -1)
        if d == 0:
            return torch.stack([rho * u, rho * u * u + p, rho * u * v, u * (E + p)], -1)
        return torch.stack([rho * v, rho * u * v, rho * v * v + p, v * (E + p)], -1)

    def jvp(self, U, D, d):
        """dF_d/dU . D by the chain rule (D = derivative of U along some direction)."""
        rho, u, v, E, p = self._prim(U)
        gm1 = self.g - 1.0
        r_s = D[..., 0]
        m_s = D[..., 1]
        if self.dim == 1:
            n_s = torch.zeros_like(r_s)
            E_s = D[..., 2]
        else:
            n_s = D[..., 2]
            E_s = D[..., 3]
        u_s = (m_s - u * r_s) / rho
        v_s = (n_s - v * r_s) / rho
        p_s = gm1 * (E_s - u * m_s - v * n_s + 0.5 * (u * u + v * v) * r_s)
        m = rho * u
        n = rho * v
        if self.dim == 1:
            return torch.stack([m_s, m_s * u + m * u_s + p_s,
                                u_s * (E + p) + u * (E_s + p_s)], -1)
        if d == 0:
            return torch.stack([m_s, m_s * u + m * u_s + p_s, m_s * v + m * v_s,
                                u_s * (E + p) + u * (E_s + p_s)], -1)
        return torch.stack([n_s, n_s * u + n * u_s, n_s * v + n * v_s + p_s,
                            v_s * (E + p) + v * (E_s + p_s)], -1)

    def speed(self, U, d):
        rho, u, v, E, p = self._prim(U)
        c = torch.sqrt(self.g * p / rho)
        return (u if d == 0 else v).abs() + c

    def roe_average(self, UL, UR):
        rL, uL, vL, EL, pL = self._prim(UL)
        rR, uR, vR, ER, pR = self._prim(UR)
        sL = torch.sqrt(rL)
        sR = torch.sqrt(rR)
        HL = (EL + pL) / rL
        HR = (ER + pR) / rR
        u = (sL * uL + sR * uR) / (sL + sR)
        v = (sL * vL + sR * vR) / (sL + sR)
        H = (sL * HL + sR * HR) / (sL + sR)
        c = torch.sqrt((self.g - 1.0) * (H - 0.5 * (u * u + v * v)))
        return u, v, H, c

    def right_eigenvectors(self, UL, UR, d):
        """Columns = right eigenvectors of dF_d/dU at the Roe average.

        x: (1, u-c, v, H-uc), (1, u, v, q^2/2), (0, 0, 1, v), (1, u+c, v, H+uc);
        y: (1, u, v-c, H-vc), (1, u, v, q^2/2), (0, 1, 0, u), (1, u, v+c, H+vc);
        1D drops the v rows/columns.
        """
        u, v, H, c = self.roe_average(UL, UR)
        one = torch.ones_like(u)
        zero = torch.zeros_like(u)
        q2 = 0.5 * (u * u + v * v)
        if self.dim == 1:
            cols = [torch.stack([one, u - c, H - u * c], -1),
                    torch.stack([one, u, q2], -1),
                    torch.stack([one, u + c, H + u * c], -1)]
        elif d == 0:
            cols = [torch.stack([one, u - c, v, H - u * c], -1),
                    torch.stack([one, u, v, q2], -1),
                    torch.stack([zero, zero, one, v], -1),
                    torch.stack([one, u + c, v, H + u * c], -1)]
        else:
            cols = [torch.stack([one, u, v - c, H - v * c], -1),
                    torch.stack([one, u, v, q2], -1),
                    torch.stack([zero, one, zero, u], -1),
                    torch.stack([one, u, v + c, H + v * c], -1)]
        return torch.stack(cols, -1)


def physics_of(prob: Problem):
    return Euler(prob) if prob.physics == "euler" else Scalar(prob)


# ===========================================================================
# Grid helpers
# ===========================================================================

def _pad(A, axis, bc, width=2, parity=None):
    """Ghost cells along ``axis`` of A = [components, ny, nx]: periodic wrap, copy
    of the nearest interior value, or (REFLECT) the mirror image across the wall,
    ghost k taking interior cell k (k = 1, 2 counted from the wall) times the
    component's parity (+1 even, -1 odd) under the reflection."""
    n = A.shape[axis]
    k = torch.arange(-width, n + width)
    if bc == PERIODIC:
        return A.index_select(axis, k % n)
    if bc == OUTFLOW:
        return A.index_select(axis, torch.clamp(k, 0, n - 1))
    if n < width:
        raise ValueError("a reflecting wall needs at least as many cells as ghost cells")
    mirror = torch.where(k < 0, -1 - k, torch.where(k >= n, 2 * n - 1 - k, k))
    out = A.index_select(axis, mirror)
    ghost = ((k < 0) | (k >= n)).to(A.dtype)
    shape = [1] * A.dim()
    shape[axis] = k.numel()
    p = torch.as_tensor(parity, dtype=A.dtype).view([-1] + [1] * (A.dim() - 1))
    # interior points keep their values; ghosts are multiplied by the parity
    return out * (1 - ghost.view(shape) + ghost.view(shape) * p)


def _pad_edges(A, axis, prob, d, role, t, width=2):
    """Ghost cells along ``axis`` (direction d) of A = [components, ny, nx] for a
    direction under EDGES.  ``role``: "U" (conserved variables), "n" (their
    derivative along d) or "t" (across d), which decides what a wall's parity
    and an inflow's zero derivative do to A."""
    n = A.shape[axis]
    lo, hi = prob.edges[2 * d], prob.edges[2 * d + 1]
    wall_lo, wall_hi = SEG_REFLECT in lo.kind, SEG_REFLECT in hi.kind
    if (wall_lo or wall_hi) and n < width:
        raise ValueError("a reflecting wall needs at least as many cells as ghost cells")
    k = torch.arange(-width, n + width)
    src = torch.where(k < 0, (-1 - k) if wall_lo else torch.zeros_like(k),
                      torch.where(k >= n, (2 * n - 1 - k) if wall_hi else torch.full_like(k, n - 1), k))
    out = A.index_select(axis, src).clone()
    # tangential coordinates of the cells along the side
    t_axis = 1 if axis == 2 else 2
    h_t = prob.dy if axis == 2 else prob.dx
    h_d = prob.dx if axis == 2 else prob.dy
    pos = (torch.arange(A.shape[t_axis], dtype=DTYPE) + 0.5) * h_t
    if prob.physics == "euler":
        pu, pn, pt = _parities(prob, d)
        par = {"U": pu, "n": pn, "t": pt}[role]
    else:
        par = None
    for layer in range(1, width + 1):
        depth = (layer - 0.5) * h_d
        for side, e, g in ((0, lo, width - layer), (1, hi, n + width - 1 + layer)):
            split = e.split[0] + e.split[1] * t + e.split[2] * depth
            seg1 = pos >= split                      # segment of each ghost cell along the side
            ghost = out.narrow(axis, g, 1)           # view [m, 1, n_t] or [m, n_t, 1]
            for sg, mask in ((0, ~seg1), (1, seg1)):
                if not bool(mask.any()):
                    continue
                shape = [1, 1, 1]
                shape[t_axis] = -1
                msk = mask.view(shape)
                if e.kind[sg] == SEG_REFLECT:
                    p = torch.as_tensor(par, dtype=A.dtype).view(-1, 1, 1)
                    ghost.copy_(torch.where(msk, ghost * p, ghost))
                elif e.kind[sg] == SEG_STATE:
                    if role == "U":
                        val = torch.as_tensor(e.state[sg][:A.shape[0]], dtype=A.dtype).view(-1, 1, 1)
                    else:
                        val = torch.zeros(A.shape[0], 1, 1, dtype=A.dtype)
                    ghost.copy_(torch.where(msk, val.expand_as(ghost), ghost))
    return out


def _solid(prob, ny, nx):
    """Mask [ny, nx] of the obstacle's solid cells (all False without one)."""
    m = torch.zeros(ny, nx, dtype=torch.bool)
    if prob.obstacle is not None:
        i_s, j_s = prob.obstacle
        m[:j_s, i_s:] = True
    return m


def _obstacle_image(A, prob, d, role):
    """A = [components, ny, nx] with every solid cell replaced by the mirror image
    of the fluid across the obstacle's face normal to direction d (the front face
    x = i_s dx for d = 0, the top face y = j_s dy for d = 1), times the parity of
    ``role`` ("U", "n": derivative along d, "t": across d) under that reflection.
    Solid cells deeper than the fluid can mirror take a clamped copy; no stencil
    of a fluid cell reaches them."""
    if prob.obstacle is None:
        return A
    i_s, j_s = prob.obstacle
    ny, nx = A.shape[1], A.shape[2]
    jj, ii = torch.meshgrid(torch.arange(ny), torch.arange(nx), indexing="ij")
    if d == 0:
        src_j, src_i = jj, (2 * i_s - 1 - ii).clamp(0, nx - 1)
    else:
        src_j, src_i = (2 * j_s - 1 - jj).clamp(0, ny - 1), ii
    pu, pn, pt = _parities(prob, d)
    par = torch.as_tensor({"U": pu, "n": pn, "t": pt}[role], dtype=A.dtype).view(-1, 1, 1)
    return torch.where(_solid(prob, ny, nx), A[:, src_j, src_i] * par, A)


def _parities(prob, d):
    """Parities of (U, derivative along d, derivative across d) under reflection
    across a wall normal to direction d: the momentum component normal to the
    wall is odd, a derivative along d flips the parity of its component."""
    if prob.physics != "euler":
        raise ValueError("reflecting walls are defined for the Euler equations only")
    pu = [1.0] * prob.m
    pu[1 + d] = -1.0
    return pu, [-q for q in pu], pu


def _split(S, prob):
    m = prob.m
    U = S[:m]
    V = S[m:2 * m]
    W = S[2 * m:3 * m] if prob.dim == 2 else None
    return U, V, W


def max_speeds(S, prob) -> Tuple[float, float]:
    """alpha_d = max over the grid of |f_d'(u)| (global LF speed, Section 2.1)."""
    phys = physics_of(prob)
    U = _split(S, prob)[0].movedim(0, -1)
    fluid = ~_solid(prob, U.shape[0], U.shape[1])    # solid cells enter no speed
    ax = float(phys.speed(U, 0)[fluid].max())
    ay = float(phys.speed(U, 1)[fluid].max()) if prob.dim == 2 else 0.0
    return ax, ay


# ===========================================================================
# Semi-discrete operator (eqs. odeH, ode2H; Remarks 2.1 and 2.2)
# ===========================================================================

def _direction_fluxes(U, Dn, Dt, prob, d, alpha, t=0.0):
    """Interface fluxes along direction d for interfaces -1/2 .. n-1/2.

    U, Dn (derivative along d), Dt (derivative across d, or None): [m, ny, nx];
    t: time of the state (read by edge-described sides).
    Returns (f-hat, h-hat, mixed-hat), each with the component axis first.
    """
    phys = physics_of(prob)
    axis = 2 if d == 0 else 1
    bc = prob.bc_x if d == 0 else prob.bc_y
    dd = prob.dx if d == 0 else prob.dy
    n = U.shape[axis]
    pu, pn, pt = _parities(prob, d) if bc == REFLECT else (None, None, None)

    def pad(A, par, role):
        if bc == EDGES:
            return _pad_edges(A, axis, prob, d, role, t)
        return _pad(A, axis, bc, parity=par)
    Up = pad(U, pu, "U").movedim(0, -1)
    Dnp = pad(Dn, pn, "n").movedim(0, -1)
    cax = axis - 1   # grid axis once the component axis has moved last

    def at(A, k):    # stencil point i-1+k of the interfaces i+1/2, i = -1..n-1
        return A.narrow(cax, k, n + 1)

    F = phys.flux(Up, d)
    AD = phys.jvp(Up, Dnp, d)

    # global Lax-Friedrichs splitting (Section 2.1), conserved components
    fP = [0.5 * (at(F, k) + alpha * at(Up, k)) for k in range(4)]
    fM = [0.5 * (at(F, k) - alpha * at(Up, k)) for k in range(4)]
    hP = [0.5 * (at(AD, k) + alpha * at(Dnp, k)) for k in range(4)]
    hM = [0.5 * (at(AD, k) - alpha * at(Dnp, k)) for k in range(4)]

    # nonlinear flux in local characteristic fields (Remarks 2.1 / 2.2)
    if prob.characteristic and prob.m > 1:
        R = phys.right_eigenvectors(at(Up, 1), at(Up, 2), d)
        L = torch.linalg.inv(R)

        def proj(X):
            return (L @ X.unsqueeze(-1)).squeeze(-1)
    else:
        R = None

        def proj(X):
            return X
    cfP = [proj(x) for x in fP]
    cfM = [proj(x) for x in fM]
    cHP = [dd * proj(x) for x in hP]
    cHM = [dd * proj(x) for x in hM]
    lin, eps, lr = prob.lin_w, prob.eps, prob.linear_recon
    fhat_c = hweno_plus(cfP[0], cfP[1], cfP[2], cHP[0], cHP[1], cHP[2], lin, eps, lr) \
        + hweno_minus(cfM[1], cfM[2], cfM[3], cHM[1], cHM[2], cHM[3], lin, eps, lr)
    fhat = (R @ fhat_c.unsqueeze(-1)).squeeze(-1) if R is not None else fhat_c

    # linear derivative-equation flux, component by component
    hhat = quintic_derivative(fP[0], fP[1], fP[2], hP[0], hP[1], hP[2], dd) \
        + quintic_derivative_minus(fM[1], fM[2], fM[3], hM[1], hM[2], hM[3], dd)

    mixed = None
    if Dt is not None:
        Dtp = pad(Dt, pt, "t").movedim(0, -1)
        AT = phys.jvp(Up, Dtp, d)
        # eq. (mixed): central four-point value, no splitting
        mixed = (-at(AT, 0) + 7.0 * at(AT, 1) + 7.0 * at(AT, 2) - at(AT, 3)) / 12.0
        mixed = mixed.movedim(-1, 0)
    return fhat.movedim(-1, 0), hhat.movedim(-1, 0), mixed


def _difference(Fh, axis, h):
    n = Fh.shape[axis] - 1
    return -(Fh.narrow(axis, 1, n) - Fh.narrow(axis, 0, n)) / h


def rhs(S, prob: Problem, alpha: Optional[Tuple[float, float]] = None, t: float = 0.0):
    """Semi-discrete right-hand side L(S) (eqs. odeH and ode2H) of the state at time t."""
    if alpha is None:
        alpha = max_speeds(S, prob)
    U, V, W = _split(S, prob)
    img = _obstacle_image
    fh, hh, eh = _direction_fluxes(img(U, prob, 0, "U"), img(V, prob, 0, "n"),
                                   None if W is None else img(W, prob, 0, "t"), prob, 0, alpha[0], t)
    LU = _difference(fh, 2, prob.dx)
    LV = _difference(hh, 2, prob.dx)
    if prob.dim == 1:
        return torch.cat([LU, LV])
    LW = _difference(eh, 2, prob.dx)
    gh, th, xh = _direction_fluxes(img(U, prob, 1, "U"), img(W, prob, 1, "n"),
                                   img(V, prob, 1, "t"), prob, 1, alpha[1], t)
    LU = LU + _difference(gh, 1, prob.dy)
    LW = LW + _difference(th, 1, prob.dy)
    LV = LV + _difference(xh, 1, prob.dy)
    L = torch.cat([LU, LV, LW])
    # solid cells: zero right-hand side
    return torch.where(_solid(prob, S.shape[1], S.shape[2]), torch.zeros_like(L), L)


def limited_derivatives(S, prob: Problem, t: float = 0.0):
    """Limited derivatives: U_x along x (and U_y along y) by Section 2.2, of the
    state at time t."""
    U, V, W = _split(S, prob)
    d, eps, lin = prob.lim_w, prob.eps, prob.linear_limiter

    char = prob.limiter_characteristic and prob.physics == "euler"
    phys = physics_of(prob) if char else None

    def along(D, axis, bc, h):
        n = U.shape[axis]
        dr = 0 if axis == 2 else 1
        Ui, D = _obstacle_image(U, prob, dr, "U"), _obstacle_image(D, prob, dr, "n")
        pu, pn, _ = _parities(prob, dr) if bc == REFLECT else (None, None, None)
        if bc == EDGES:
            Up = _pad_edges(Ui, axis, prob, dr, "U", t, 1)
            Dp = _pad_edges(D, axis, prob, dr, "n", t, 1)
        else:
            Up = _pad(Ui, axis, bc, 1, parity=pu)
            Dp = _pad(D, axis, bc, 1, parity=pn)
        um, u0, up = (Up.narrow(axis, k, n) for k in range(3))
        vm, vp = Dp.narrow(axis, 0, n), Dp.narrow(axis, 2, n)
        if not char:
            return limit_derivative(um, u0, up, vm, vp, h, d, eps, lin)
        # characteristic variant: every stencil value is projected with the left
        # eigenvectors of dF_d/dU at the cell's own state, the scalar limiter acts
        # on each characteristic field, and the right eigenvectors map back
        R = phys.right_eigenvectors(u0.movedim(0, -1), u0.movedim(0, -1), dr)
        Li = torch.linalg.inv(R)

        def proj(A):
            return (Li @ A.movedim(0, -1).unsqueeze(-1)).squeeze(-1).movedim(-1, 0)

        z = limit_derivative(proj(um), proj(u0), proj(up), proj(vm), proj(vp), h, d, eps, lin)
        return (R @ z.movedim(0, -1).unsqueeze(-1)).squeeze(-1).movedim(-1, 0)

    out = [along(V, 2, prob.bc_x, prob.dx)]
    if prob.dim == 2:
        out.append(along(W, 1, prob.bc_y, prob.dy))
    D = torch.cat(out)
    # solid cells keep their derivatives
    return torch.where(_solid(prob, S.shape[1], S.shape[2]), S[prob.m:], D)


def hat(S, prob: Problem, t: float = 0.0):
    """(U, limited derivatives), or S itself with the limiter switched off."""
    if not prob.limiter_on:
        return S
    return torch.cat([S[:prob.m], limited_derivatives(S, prob, t)])


def cfl_dt(alpha, prob: Problem) -> float:
    """Time step from the CFL number: 1D cfl dx / a_x, 2D cfl / (a_x/dx + a_y/dy)."""
    if prob.dim == 1:
        return prob.cfl * prob.dx / alpha[0]
    return prob.cfl / (alpha[0] / prob.dx + alpha[1] / prob.dy)


def rk3_step(S, prob: Problem, dt: Optional[float] = None, alphas=None, t: float = 0.0):
    """One SSP-RK3 step with limited derivatives in the update only (Section 2.2).

    ``alphas``: optional per-stage wave speeds (replay); otherwise each stage
    computes them from its own state.  ``t``: time of S; the stage inputs sit
    at t, t + dt and t + dt/2 (what edge-described sides read).
    Returns (S^{n+1}, dt, alphas).
    """
    a = [None, None, None] if alphas is None else list(alphas)
    a[0] = a[0] if a[0] is not None else max_speeds(S, prob)
    if dt is None:
        dt = cfl_dt(a[0], prob)
    t1, t2 = t + dt, t + 0.5 * dt
    solid = _solid(prob, S.shape[1], S.shape[2])

    def keep(X):     # the obstacle's solid cells keep their state exactly
        return torch.where(solid, S, X) if prob.obstacle is not None else X
    H0 = hat(S, prob, t)
    S1 = keep(H0 + dt * rhs(S, prob, a[0], t))
    a[1] = a[1] if a[1] is not None else max_speeds(S1, prob)
    S2 = keep(0.75 * H0 + 0.25 * (hat(S1, prob, t1) + dt * rhs(S1, prob, a[1], t1)))
    a[2] = a[2] if a[2] is not None else max_speeds(S2, prob)
    S3 = keep(H0 / 3.0 + 2.0 / 3.0 * (hat(S2, prob, t2) + dt * rhs(S2, prob, a[2], t2)))
    return S3, dt, a


def run(S, prob: Problem, t_end: float, dt_rule=None, max_steps=10 ** 7):
    """Advance to t_end; ``dt_rule(alpha) -> dt`` overrides the CFL rule; last step clipped."""
    t = 0.0
    steps = 0
    while t < t_end - 1e-14 * max(1.0, t_end) and steps < max_steps:
        a0 = max_speeds(S, prob)
        dt = dt_rule(a0) if dt_rule is not None else cfl_dt(a0, prob)
        dt = min(dt, t_end - t)
        S, _, _ = rk3_step(S, prob, dt, [a0, None, None], t)
        t += dt
        steps += 1
    return S, steps


def as_tensor(S) -> torch.Tensor:
    return torch.as_tensor(S, dtype=DTYPE)
