"""Pins of the oracle's nonlinear selection and of its outflow ghost copy.

Section 2.1 builds the nonlinear weights from the smoothness indicators through
tau (eq. tau-fh) and bar-omega_l = gamma_l (1 + tau / (beta_l + eps)); Section
2.2 builds the limiter's lambda the same way.  The point of these weights is
that a stencil crossed by a jump hands the result to the candidate whose
stencil is smooth.  The tests below place a jump on one side of the stencil and
require the oracle's value to be that candidate's, which is fitted here from
its defining conditions in exact arithmetic (tests/exact_poly.py), not taken
from the oracle.  The allowed deviation is derived from the weight formula: for
the smooth candidate s and any other l,

    omega_l <= bar-omega_l / bar-omega_s
            <= (gamma_l / gamma_s) (beta_s + eps) (1 / tau + 1 / (beta_l + eps)),

and tau >= (beta_a - beta_b)^2 / 4 for the two quadratics a, b (triangle
inequality on |beta_0 - beta_1| + |beta_0 - beta_2|), with every beta from the
exact integral definition (eq. GHYZ / GHYZ-q).  Each case also checks that the
bound is far below the distance to the other candidates, so that exchanging
beta_1 and beta_2, or the two quadratic candidates, or taking the wrong side's
data for the mirrored reconstruction, fails.

The outflow pins: the boundary copies the nearest interior value of every field
into the ghost cells, so a domain whose outermost cells are repeated outward
gives, on its own cells, exactly the operator and the limiter of the extended
domain; and when the data are constant for several cells next to an outflow
side, a whole SSP-RK3 step equals that of the domain extended by the constant
(nothing reaches the side within one step).
"""
import random
from fractions import Fraction as Fr

import pytest
import torch

from oracle import hweno_ref as o
from tests import exact_poly as ep

EPS = 1e-6
WEIGHT_SETS = [(0.98, 0.01, 0.01), (0.6, 0.2, 0.2), (1 / 3, 1 / 3, 1 / 3)]


def _t(x):
    return torch.tensor(float(x), dtype=torch.float64)


def _selection_bound(s, beta, cand, lin, eps):
    """Upper bound of |combination - cand[s]| from the weight formula (module docstring).

    beta: exact beta_0..2; cand: the three values the weights multiply (the
    first one being (p_0 - gamma_1 p_1 - gamma_2 p_2) / gamma_0); s: index of the
    smooth candidate (1 or 2)."""
    other = 3 - s
    tau_lo = 0.25 * (beta[other] - beta[s]) ** 2
    total = 0.0
    for l in range(3):
        if l == s:
            continue
        ratio = (lin[l] / lin[s]) * (beta[s] + eps) * (1.0 / tau_lo + 1.0 / (beta[l] + eps))
        total += ratio * abs(cand[l] - cand[s])
    return total


def _smooth_cells(rnd, scale):
    """A small quadratic c0 + c1 xi + c2 xi^2 (scaled coordinate) with coefficients of size ~scale."""
    return [Fr(rnd.randint(-9, 9), 10) * scale for _ in range(3)]


def _avg(c, l):
    return sum(r * ck for r, ck in zip(ep.cell_average_row(l, len(c) - 1), c))


def _davg(c, l):
    return sum(r * ck for r, ck in zip(ep.derivative_average_row(l, len(c) - 1), c))


@pytest.mark.parametrize("lin", WEIGHT_SETS)
@pytest.mark.parametrize("jump", [Fr(1), Fr(-3), Fr(10)])
@pytest.mark.parametrize("side", ["right", "left"])
@pytest.mark.parametrize("seed", range(3))
def test_plus_reconstruction_takes_the_smooth_quadratic(lin, jump, side, seed):
    """f-hat^+ at x_{i+1/2} from cells i-1, i, i+1 with a jump between i and i+1
    ("right") is p_1, the quadratic with the averages of cells i-1, i and the
    derivative average of cell i; with the jump between i-1 and i ("left") it is
    p_2, the quadratic on cells i, i+1 (Section 2.1)."""
    rnd = random.Random(1000 + seed)
    c = _smooth_cells(rnd, Fr(1, 1000))
    # smooth data from the quadratic on the smooth side, a jump on the other
    f = {l: _avg(c, l) for l in (-1, 0, 1)}
    H = {l: _davg(c, l) for l in (-1, 0, 1)}
    jumped = 1 if side == "right" else -1
    f[jumped] += jump
    H[jumped] = Fr(rnd.randint(-9, 9), 10)        # arbitrary derivative datum in the jumped cell
    q0 = ep.fit_averages(f, H, 5)
    q1 = ep.fit_averages({-1: f[-1], 0: f[0]}, {0: H[0]}, 2)
    q2 = ep.fit_averages({0: f[0], 1: f[1]}, {0: H[0]}, 2)
    half = Fr(1, 2)
    p = [float(ep.evaluate(q, half)) for q in (q0, q1, q2)]
    beta = [float(ep.smoothness(q)) for q in (q0, q1, q2)]
    cand = [(p[0] - lin[1] * p[1] - lin[2] * p[2]) / lin[0], p[1], p[2]]
    s = 1 if side == "right" else 2
    bound = _selection_bound(s, beta, cand, lin, EPS)
    # the bound separates the right answer from every wrong candidate by far
    assert bound < 1e-3 * min(abs(p[0] - p[s]), abs(p[3 - s] - p[s]))
    got = float(o.hweno_plus(*[_t(f[l]) for l in (-1, 0, 1)], *[_t(H[l]) for l in (-1, 0, 1)],
                             lin, EPS))
    assert abs(got - p[s]) <= bound * (1 + 1e-9) + 1e-15, (got, p, bound)


@pytest.mark.parametrize("lin", WEIGHT_SETS)
@pytest.mark.parametrize("jump", [Fr(1), Fr(-4)])
@pytest.mark.parametrize("where", ["i|i+1", "i+1|i+2"])
@pytest.mark.parametrize("seed", range(3))
def test_minus_reconstruction_takes_the_smooth_quadratic(lin, jump, where, seed):
    """f-hat^-_{i+1/2} (the mirror image of the "+" procedure, centred on cell i+1)
    from cells i, i+1, i+2.  A jump between i and i+1 leaves the quadratic with the
    averages of cells i+1, i+2 and the derivative average of cell i+1; a jump
    between i+1 and i+2 leaves the quadratic on cells i, i+1 (same derivative
    datum).  Values at the interface x_{i+1/2}, the left edge of cell i+1.
    Coordinates here are centred on cell i+1: cells i, i+1, i+2 are -1, 0, 1."""
    rnd = random.Random(2000 + seed)
    c = _smooth_cells(rnd, Fr(1, 1000))
    g = {l: _avg(c, l) for l in (-1, 0, 1)}
    k = {l: _davg(c, l) for l in (-1, 0, 1)}
    jumped = -1 if where == "i|i+1" else 1
    g[jumped] += jump
    k[jumped] = Fr(rnd.randint(-9, 9), 10)
    q0 = ep.fit_averages(g, k, 5)
    q_up = ep.fit_averages({0: g[0], 1: g[1]}, {0: k[0]}, 2)     # cells i+1, i+2
    q_dn = ep.fit_averages({-1: g[-1], 0: g[0]}, {0: k[0]}, 2)   # cells i, i+1
    edge = Fr(-1, 2)
    p = [float(ep.evaluate(q, edge)) for q in (q0, q_up, q_dn)]
    beta = [float(ep.smoothness(q)) for q in (q0, q_up, q_dn)]
    cand = [(p[0] - lin[1] * p[1] - lin[2] * p[2]) / lin[0], p[1], p[2]]
    s = 1 if where == "i|i+1" else 2
    bound = _selection_bound(s, beta, cand, lin, EPS)
    assert bound < 1e-3 * min(abs(p[0] - p[s]), abs(p[3 - s] - p[s]))
    got = float(o.hweno_minus(*[_t(g[l]) for l in (-1, 0, 1)], *[_t(k[l]) for l in (-1, 0, 1)],
                              lin, EPS))
    assert abs(got - p[s]) <= bound * (1 + 1e-9) + 1e-15, (got, p, bound)


@pytest.mark.parametrize("d", WEIGHT_SETS)
@pytest.mark.parametrize("jump", [Fr(1), Fr(-5)])
@pytest.mark.parametrize("side", ["right", "left"])
@pytest.mark.parametrize("seed", range(3))
def test_limiter_takes_the_one_sided_difference(d, jump, side, seed):
    """v-tilde_i (Section 2.2) from u_{i-1}, u_i, u_{i+1}, v_{i-1}, v_{i+1}: with a
    jump between i and i+1 it is q_1' = (u_i - u_{i-1})/dx, the derivative of the
    line through the two smooth points; with the jump between i-1 and i it is
    q_2' = (u_{i+1} - u_i)/dx."""
    rnd = random.Random(3000 + seed)
    c = _smooth_cells(rnd, Fr(1, 1000))
    dx = Fr(1, 4)
    # point data u(l) = c(l), derivative data V = dx v = c'(l) in the scaled coordinate
    dc = ep.derivative(c)
    u = {l: ep.evaluate(c, l) for l in (-1, 0, 1)}
    V = {l: ep.evaluate(dc, l) for l in (-1, 1)}
    jumped = 1 if side == "right" else -1
    u[jumped] += jump
    V[jumped] = Fr(rnd.randint(-9, 9), 10)
    q0 = ep.fit_points(u, V, 4)
    q1 = ep.fit_points({-1: u[-1], 0: u[0]}, {}, 1)
    q2 = ep.fit_points({0: u[0], 1: u[1]}, {}, 1)
    # candidates as derivatives at x_i per unit x
    qv = [float(ep.evaluate(ep.derivative(q), 0) / dx) for q in (q0, q1, q2)]
    beta = [float(ep.smoothness(q)) for q in (q0, q1, q2)]
    cand = [(qv[0] - d[1] * qv[1] - d[2] * qv[2]) / d[0], qv[1], qv[2]]
    s = 1 if side == "right" else 2
    bound = _selection_bound(s, beta, cand, d, EPS)
    assert bound < 1e-3 * min(abs(qv[0] - qv[s]), abs(qv[3 - s] - qv[s]))
    got = float(o.limit_derivative(_t(u[-1]), _t(u[0]), _t(u[1]), _t(V[-1] / dx), _t(V[1] / dx),
                                   float(dx), d, EPS))
    assert abs(got - qv[s]) <= bound * (1 + 1e-9) + 1e-15, (got, qv, bound)


def test_selection_fails_with_exchanged_indicators():
    """The pin above has teeth: the same combination with beta_1 and beta_2
    exchanged lands on the other quadratic, outside the bound."""
    rnd = random.Random(7)
    c = _smooth_cells(rnd, Fr(1, 1000))
    f = {l: _avg(c, l) for l in (-1, 0, 1)}
    H = {l: _davg(c, l) for l in (-1, 0, 1)}
    f[1] += 1
    args = [_t(f[l]) for l in (-1, 0, 1)] + [_t(H[l]) for l in (-1, 0, 1)]
    lin = WEIGHT_SETS[0]
    p0, p1, p2 = o.hermite_values(*args)
    b0, b1, b2 = o.smoothness_indicators(*args)
    w0, w1, w2 = o.nonlinear_weights(b0, b2, b1, lin, EPS)      # exchanged
    wrong = w0 * (p0 / lin[0] - lin[1] / lin[0] * p1 - lin[2] / lin[0] * p2) + w1 * p1 + w2 * p2
    right = o.hweno_plus(*args, lin, EPS)
    assert abs(float(right - p1)) < 1e-4 * abs(float(p2 - p1))
    assert abs(float(wrong - p1)) > 0.5 * abs(float(p2 - p1))


# ---------------------------------------------------------------------------
# outflow ghost copy
# ---------------------------------------------------------------------------

def _extend(A, axis, lo, hi):
    """A with its first slice repeated lo times before and its last slice hi times after."""
    n = A.shape[axis]
    parts = [A.narrow(axis, 0, 1)] * lo + [A] + [A.narrow(axis, n - 1, 1)] * hi
    return torch.cat(parts, axis)


def _random_state(prob, ny, nx, seed):
    """Admissible rough Euler data (or Burgers data) with random derivative fields."""
    g = torch.Generator().manual_seed(seed)
    m = prob.m
    S = torch.zeros(prob.nf, ny, nx, dtype=torch.float64)
    if prob.physics == "euler":
        rho = 0.5 + torch.rand(ny, nx, generator=g, dtype=torch.float64)
        vel = [torch.rand(ny, nx, generator=g, dtype=torch.float64) - 0.5 for _ in range(prob.dim)]
        p = 0.5 + torch.rand(ny, nx, generator=g, dtype=torch.float64)
        S[0] = rho
        for k, v in enumerate(vel):
            S[1 + k] = rho * v
        S[m - 1] = p / (prob.gamma_gas - 1) + 0.5 * rho * sum(v * v for v in vel)
    else:
        S[0] = torch.rand(ny, nx, generator=g, dtype=torch.float64) - 0.3
    S[m:] = torch.randn(prob.nf - m, ny, nx, generator=g, dtype=torch.float64) * 0.3
    return S


CASES = [
    ("burgers", 1, 23, 1),
    ("euler", 1, 29, 1),
    ("euler", 2, 19, 14),
]


@pytest.mark.parametrize("physics,dim,nx,ny", CASES)
@pytest.mark.parametrize("seed", range(2))
def test_outflow_equals_the_domain_extended_by_its_edge_cells(physics, dim, nx, ny, seed):
    """Outflow ghosts are copies of the nearest interior cell (all fields): the
    operator and the limiter of any state equal, on its own cells, those of the
    domain with its edge cells repeated outward (ext >= 2 cells per side, so that
    the wider domain's own ghosts lie beyond every stencil that reaches the
    original cells).  A ghost copied from the second cell, a mirror, or zero
    ghost derivatives would differ."""
    prob = o.Problem(dim=dim, physics=physics, dx=0.1, dy=0.13, bc_x=o.OUTFLOW,
                     bc_y=o.OUTFLOW if dim == 2 else o.PERIODIC)
    S = _random_state(prob, ny, nx, seed)
    ext = 3
    E = _extend(S, 2, ext, ext)
    if dim == 2:
        E = _extend(E, 1, ext, ext)
    alpha = o.max_speeds(S, prob)
    # the wider domain holds only copies of the original cells: the same speeds
    assert o.max_speeds(E, prob) == alpha
    inner = (slice(None), slice(ext, ext + ny) if dim == 2 else slice(None), slice(ext, ext + nx))
    L = o.rhs(S, prob, alpha)
    LE = o.rhs(E, prob, alpha)
    assert torch.equal(L, LE[inner])
    D = o.limited_derivatives(S, prob)
    DE = o.limited_derivatives(E, prob)
    assert torch.equal(D, DE[inner])
    # a ghost copied from the second cell from the side differs (the pin has teeth)
    wrong = torch.cat([S.narrow(2, 1, 1), S.narrow(2, 1, 1), S, S.narrow(2, nx - 2, 1),
                       S.narrow(2, nx - 2, 1)], 2)
    if dim == 2:
        wrong = _extend(wrong, 1, 2, 2)
    inner2 = (slice(None), slice(2, 2 + ny) if dim == 2 else slice(None), slice(2, 2 + nx))
    assert not torch.equal(L, o.rhs(wrong, prob, alpha)[inner2])


@pytest.mark.parametrize("physics,dim,nx,ny", CASES)
def test_outflow_step_with_constant_data_near_the_sides(physics, dim, nx, ny):
    """When the data are constant (derivatives zero) for K = 8 cells next to each
    outflow side, one SSP-RK3 step equals, on the original cells, the step of the
    domain extended by that constant: each stage moves the non-constant front by
    two cells (the flux stencil), so after three stages it stays clear of the
    last three cells, whose ghosts the copy fills with the constant the wider
    domain holds (Section 2.2 time stepping, outflow reading of the boundary)."""
    prob = o.Problem(dim=dim, physics=physics, dx=0.1, dy=0.13, bc_x=o.OUTFLOW,
                     bc_y=o.OUTFLOW if dim == 2 else o.PERIODIC)
    K, ext = 8, 6
    S = _random_state(prob, ny + (2 * K if dim == 2 else 0), nx + 2 * K, 5)
    m = prob.m
    # constant edge bands: every cell within K of an outflow side takes the state
    # of one interior cell, with zero derivatives
    ref = S[:, (S.shape[1] - 1) // 2, (S.shape[2] - 1) // 2].clone()
    ref[m:] = 0.0
    band = torch.zeros(S.shape[1:], dtype=torch.bool)
    band[:, :K] = True
    band[:, -K:] = True
    if dim == 2:
        band[:K, :] = True
        band[-K:, :] = True
    S = torch.where(band, ref.view(-1, 1, 1), S)
    ny2, nx2 = S.shape[1], S.shape[2]
    E = _extend(S, 2, ext, ext)
    if dim == 2:
        E = _extend(E, 1, ext, ext)
    inner = (slice(None), slice(ext, ext + ny2) if dim == 2 else slice(None), slice(ext, ext + nx2))
    S1, dt, a = o.rk3_step(S, prob)
    E1, dtE, aE = o.rk3_step(E, prob)
    assert dt == dtE and a == aE
    assert torch.equal(S1, E1[inner])
    # the front did move: the step changed cells inside the bands' inner edges
    assert not torch.equal(S1, S)
