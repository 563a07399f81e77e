"""Pins of the oracle's edge-described sides (the boundaries of Example 3.11).

Each test compares against something built without the edge rule:
  * edges whose segments are all walls, or all outflow copies, are the plain
    reflecting / outflow boundaries, which have their own pins;
  * a uniform flow along a channel (inflow of the same state, outflow, walls
    parallel to the flow) is an exact steady solution: the operator vanishes;
  * a contact discontinuity (uniform velocity and pressure, density jump along
    a straight line) is advected exactly by the Euler equations.  Its ghost cells
    described by moving, depth-dependent splits must be the exact solution in a
    domain two cells wider on every side, so the operator and the limiter on the
    small domain equal those of the wide domain on the same cells.
"""
import math

import numpy as np
import pytest
import torch

import hweno_inputs as hi
from oracle import hweno_ref as o

GAM = 1.4


def _cons(rho, u, v, p):
    return (rho, rho * u, rho * v, p / (GAM - 1.0) + 0.5 * rho * (u * u + v * v))


def _edge(kinds, split=(0.0, 0.0, 0.0), states=((1.0, 0.0, 0.0, 2.5),) * 2):
    return o.Edge(kind=tuple(kinds), split=tuple(split), state=tuple(tuple(s) for s in states))


def _smooth(nx=20, ny=18):
    w = hi.euler2d_random_smooth(nx, ny, 3)
    return o.as_tensor(w.S), w


def test_all_wall_and_all_outflow_edges_are_the_plain_boundaries():
    S, w = _smooth()
    base = dict(dim=2, physics="euler", dx=w.dx, dy=w.dy)
    plain = o.Problem(bc_x=o.REFLECT, bc_y=o.OUTFLOW, **base)
    wall = _edge((o.SEG_REFLECT, o.SEG_REFLECT), (0.3, 1.0, 0.2))
    out = _edge((o.SEG_OUTFLOW, o.SEG_OUTFLOW), (0.5, -2.0, 0.7))
    edged = o.Problem(bc_x=o.EDGES, bc_y=o.EDGES, edges=(wall, wall, out, out), **base)
    a = o.max_speeds(S, plain)
    for t in (0.0, 0.13):
        assert torch.equal(o.rhs(S, edged, a, t), o.rhs(S, plain, a))
        assert torch.equal(o.limited_derivatives(S, edged, t), o.limited_derivatives(S, plain))
    s1, _, _ = o.rk3_step(S, plain)
    s2, _, _ = o.rk3_step(S, edged, t=0.4)
    assert torch.equal(s1, s2)


def test_uniform_channel_flow_is_stationary():
    nx, ny = 24, 12
    q = _cons(1.3, 0.7, 0.0, 2.0)
    U = torch.tensor(q, dtype=torch.float64).view(4, 1, 1).expand(4, ny, nx)
    S = torch.cat([U, torch.zeros(8, ny, nx, dtype=torch.float64)])
    inflow = _edge((o.SEG_STATE, o.SEG_STATE), (0.0, 0.0, 0.0), (q, q))
    out = _edge((o.SEG_OUTFLOW, o.SEG_OUTFLOW))
    # bottom: inflow of the same state up to x = 0.4, then a wall; top: a wall
    bottom = _edge((o.SEG_STATE, o.SEG_REFLECT), (0.4, 0.0, 0.0), (q, q))
    top = _edge((o.SEG_REFLECT, o.SEG_REFLECT))
    prob = o.Problem(dim=2, physics="euler", dx=1.0 / nx, dy=0.5 / ny, bc_x=o.EDGES,
                     bc_y=o.EDGES, edges=(inflow, out, bottom, top))
    L = o.rhs(S, prob, None, 0.25)
    assert float(L.abs().max()) <= 1e-12 * max(abs(x) for x in q) * nx
    S1, _, _ = o.rk3_step(S, prob, t=0.25)
    assert float((S1 - S).abs().max()) <= 1e-13 * max(abs(x) for x in q)


def _contact(theta, c, vel, rhos, p, lo, n, h, t, pad):
    """Cell-centre data of the advected contact on a grid of n = (nx, ny) cells of
    size h from lo, with ``pad`` extra cells on every side."""
    nx, ny = n
    xs = lo[0] + (np.arange(-pad, nx + pad) + 0.5) * h[0]
    ys = lo[1] + (np.arange(-pad, ny + pad) + 0.5) * h[1]
    X, Y = np.meshgrid(xs, ys)
    w = vel[0] * math.cos(theta) + vel[1] * math.sin(theta)
    A = X * math.cos(theta) + Y * math.sin(theta) < c + w * t
    qa, qb = _cons(rhos[0], vel[0], vel[1], p), _cons(rhos[1], vel[0], vel[1], p)
    U = np.stack([np.where(A, qa[k], qb[k]) for k in range(4)])
    return torch.cat([torch.as_tensor(U), torch.zeros(8, *U.shape[1:], dtype=torch.float64)])


@pytest.mark.parametrize("theta_deg", [50.0, 125.0])
def test_moving_oblique_contact_ghosts_equal_a_wider_domain(theta_deg):
    theta = math.radians(theta_deg)
    nx, ny, Lx, Ly = 24, 20, 1.0, 1.0
    h = (Lx / nx, Ly / ny)
    vel, rhos, p, t = (0.3, -0.2), (1.0, 0.4), 1.0, 0.37
    ct, st = math.cos(theta), math.sin(theta)
    c = 0.55 if theta_deg < 90 else 0.25
    w = vel[0] * ct + vel[1] * st
    qa, qb = _cons(rhos[0], vel[0], vel[1], p), _cons(rhos[1], vel[0], vel[1], p)
    # side-by-side: the region x cos + y sin < c + w t holds state A; on each side the
    # boundary of that region, solved for the coordinate along the side, is the split,
    # and segment 0 (before the split) is A where the coordinate's coefficient is > 0
    def side(s0, s1, s2, coef):
        kinds = (o.SEG_STATE, o.SEG_STATE)
        states = (qa, qb) if coef > 0 else (qb, qa)
        return _edge(kinds, (s0, s1, s2), states)
    left = side(c / st, w / st, ct / st, st)                       # x = -d
    right = side((c - Lx * ct) / st, w / st, -ct / st, st)         # x = Lx + d
    bottom = side(c / ct, w / ct, st / ct, ct)                     # y = -d
    top = side((c - Ly * st) / ct, w / ct, -st / ct, ct)           # y = Ly + d
    small = _contact(theta, c, vel, rhos, p, (0.0, 0.0), (nx, ny), h, t, 0)
    wide = _contact(theta, c, vel, rhos, p, (0.0, 0.0), (nx, ny), h, t, 2)
    # both states occur inside the small domain
    assert 0 < int((small[0] == rhos[0]).sum()) < nx * ny
    ps = o.Problem(dim=2, physics="euler", dx=h[0], dy=h[1], bc_x=o.EDGES, bc_y=o.EDGES,
                   edges=(left, right, bottom, top))
    pw = o.Problem(dim=2, physics="euler", dx=h[0], dy=h[1], bc_x=o.OUTFLOW, bc_y=o.OUTFLOW)
    a = o.max_speeds(small, ps)
    inner = (slice(None), slice(2, 2 + ny), slice(2, 2 + nx))
    Ls, Lw = o.rhs(small, ps, a, t), o.rhs(wide, pw, a)[inner]
    scale = float(Lw.abs().max())
    assert scale > 0
    assert float((Ls - Lw).abs().max()) <= 1e-13 * scale
    Ds = o.limited_derivatives(small, ps, t)
    Dw = o.limited_derivatives(wide, pw)[inner]
    assert float((Ds - Dw).abs().max()) <= 1e-13 * (float(Dw.abs().max()) + 1.0)
    # the same sides read at another time do not give the wide domain's operator
    assert float((o.rhs(small, ps, a, t + 0.2) - Lw).abs().max()) > 1e-3 * scale


def test_double_mach_initial_state_is_consistent_with_its_edges():
    """At t = 0 the top side's split is where the shock line crosses each ghost row,
    and the left side holds the post-shock state the interior holds near it."""
    w = hi.double_mach(48, 12)
    prob = o.problem_from_workload(w)
    S = o.as_tensor(w.S)
    # the operator vanishes on every cell whose stencils (three cells either way,
    # ghosts included) see one state only: the inflow, wall and top ghosts continue
    # the data there; next to the shock it does not vanish
    x = (np.arange(w.nx) + 0.5) * w.dx
    y = (np.arange(-3, w.ny + 3) + 0.5) * w.dy
    xs = np.concatenate([np.full(3, -1.0), x, np.full(3, 9.0)])
    behind = xs[None, :] < 1.0 / 6.0 + y[:, None] / math.sqrt(3.0)
    uniform = np.ones((w.ny, w.nx), dtype=bool)
    for dj in range(-3, 4):
        for di in range(-3, 4):
            uniform &= behind[3 + dj:3 + dj + w.ny, 3 + di:3 + di + w.nx] == behind[3:-3, 3:-3]
    # the bottom wall beyond x = 1/6 mirrors the pre-shock state, which is at rest
    assert uniform.sum() > w.nx * w.ny // 2
    L = o.rhs(S, prob, None, 0.0)
    Lu = L[:, torch.as_tensor(uniform)]
    assert float(Lu.abs().max()) <= 1e-12 * float(L.abs().max())
    assert float(L[:, torch.as_tensor(~uniform)].abs().max()) > 1e-3 * float(L.abs().max())
    # the shock crosses the top row's ghost cells where the interior line continues
    top = prob.edges[3]
    x_top = 1.0 / 6.0 + 1.0 / math.sqrt(3.0)
    assert top.split[0] == pytest.approx(x_top, rel=1e-15)
    assert top.split[2] == pytest.approx(1.0 / math.sqrt(3.0), rel=1e-15)
    assert top.split[1] == pytest.approx(10.0 / math.sin(math.pi / 3.0), rel=1e-14)


# ---------------------------------------------------------------------------
# The obstacle of Example 3.12 (solid cells i >= i_s, j < j_s, faces are walls)
# ---------------------------------------------------------------------------

def _x_edges(qa):
    """x sides without a split: an inflow on the left, an outflow on the right."""
    return (_edge((o.SEG_STATE, o.SEG_STATE), (0.0, 0.0, 0.0), (qa, qa)),
            _edge((o.SEG_OUTFLOW, o.SEG_OUTFLOW)))


def test_obstacle_across_the_whole_height_is_a_wall_on_the_right():
    S, w = _smooth(22, 14)
    i_s = 15
    qa = _cons(1.1, 0.4, -0.1, 2.0)
    lo, hi_ = _x_edges(qa)
    base = dict(dim=2, physics="euler", dx=w.dx, dy=w.dy, bc_y=o.OUTFLOW)
    pa = o.Problem(bc_x=o.EDGES, edges=(lo, hi_, hi_, hi_), obstacle=(i_s, w.ny), **base)
    wall = _edge((o.SEG_REFLECT, o.SEG_REFLECT))
    pb = o.Problem(bc_x=o.EDGES, edges=(lo, wall, hi_, hi_), **base)
    Sb = S[:, :, :i_s].contiguous()
    a = o.max_speeds(S, pa)
    assert a == o.max_speeds(Sb, pb)      # solid cells enter no speed
    La, Lb = o.rhs(S, pa, a), o.rhs(Sb, pb, a)
    assert torch.equal(La[:, :, :i_s], Lb)
    assert float(La[:, :, i_s:].abs().max()) == 0.0
    Da, Db = o.limited_derivatives(S, pa), o.limited_derivatives(Sb, pb)
    assert torch.equal(Da[:, :, :i_s], Db)
    assert torch.equal(Da[:, :, i_s:], S[4:, :, i_s:])    # solid cells keep their derivatives
    Sa1, _, _ = o.rk3_step(S, pa)
    Sb1, _, _ = o.rk3_step(Sb, pb)
    assert torch.equal(Sa1[:, :, :i_s], Sb1)
    assert torch.equal(Sa1[:, :, i_s:], S[:, :, i_s:])


def test_obstacle_across_the_whole_width_is_a_wall_below():
    S, w = _smooth(16, 20)
    j_s = 6
    qa = _cons(1.1, 0.4, -0.1, 2.0)
    lo, hi_ = _x_edges(qa)
    out = _edge((o.SEG_OUTFLOW, o.SEG_OUTFLOW))
    base = dict(dim=2, physics="euler", dx=w.dx, dy=w.dy, bc_x=o.EDGES)
    pa = o.Problem(bc_y=o.OUTFLOW, edges=(lo, hi_, out, out), obstacle=(0, j_s), **base)
    wall = _edge((o.SEG_REFLECT, o.SEG_REFLECT))
    pb = o.Problem(bc_y=o.EDGES, edges=(lo, hi_, wall, out), **base)
    Sb = S[:, j_s:, :].contiguous()
    a = o.max_speeds(S, pa)
    assert a == o.max_speeds(Sb, pb)
    assert torch.equal(o.rhs(S, pa, a)[:, j_s:, :], o.rhs(Sb, pb, a))
    assert torch.equal(o.limited_derivatives(S, pa)[:, j_s:, :], o.limited_derivatives(Sb, pb))
    Sa1, _, _ = o.rk3_step(S, pa)
    Sb1, _, _ = o.rk3_step(Sb, pb)
    assert torch.equal(Sa1[:, j_s:, :], Sb1)


def test_gas_at_rest_around_a_step_is_stationary():
    nx, ny = 20, 14
    q = _cons(1.2, 0.0, 0.0, 1.5)
    U = torch.tensor(q, dtype=torch.float64).view(4, 1, 1).expand(4, ny, nx)
    S = torch.cat([U, torch.zeros(8, ny, nx, dtype=torch.float64)])
    wall = _edge((o.SEG_REFLECT, o.SEG_REFLECT))
    prob = o.Problem(dim=2, physics="euler", dx=0.1, dy=0.07, bc_x=o.EDGES, bc_y=o.REFLECT,
                     edges=(wall, wall, wall, wall), obstacle=(8, 4))
    assert float(o.rhs(S, prob).abs().max()) <= 1e-13
    S1, _, _ = o.rk3_step(S, prob)
    assert float((S1 - S).abs().max()) <= 1e-14


def test_forward_step_initial_operator_vanishes_away_from_the_front_face():
    """The free stream is uniform and parallel to every wall but the step's front face:
    the operator vanishes except on the fluid cells within three cells of that face."""
    w = hi.forward_step(60, 20)
    prob = o.problem_from_workload(w)
    S = o.as_tensor(w.S)
    i_s, j_s = w.obstacle
    L = o.rhs(S, prob)
    near = torch.zeros(w.ny, w.nx, dtype=torch.bool)
    near[:j_s, i_s - 3:i_s] = True
    assert float(L[:, ~near].abs().max()) <= 1e-12
    assert float(L[:, near].abs().max()) > 1.0


def test_stages_read_the_sides_at_the_ssp_rk3_abscissae(monkeypatch):
    """The time each stage hands to the operator and the limiter is t + c_k dt with c
    the row sums of the Butcher matrix of SSP-RK3 in Shu-Osher form (a_21 = 1,
    a_31 = a_32 = 1/4): c = (0, 1, 1/2)."""
    A = [[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.25, 0.25, 0.0]]
    c = [sum(row) for row in A]
    w = hi.double_mach(24, 8)
    prob = o.problem_from_workload(w)
    S = o.as_tensor(w.S)
    seen = {"rhs": [], "lim": []}
    rhs0, lim0 = o.rhs, o.limited_derivatives

    def rhs(S_, p, a=None, t=0.0):
        seen["rhs"].append(t)
        return rhs0(S_, p, a, t)

    def lim(S_, p, t=0.0):
        seen["lim"].append(t)
        return lim0(S_, p, t)
    monkeypatch.setattr(o, "rhs", rhs)
    monkeypatch.setattr(o, "limited_derivatives", lim)
    t0, dt = 0.013, 1.7e-3
    o.rk3_step(S, prob, dt, t=t0)
    want = [t0 + ck * dt for ck in c]
    assert seen["rhs"] == pytest.approx(want, rel=0, abs=1e-18)
    assert seen["lim"] == pytest.approx(want, rel=0, abs=1e-18)
