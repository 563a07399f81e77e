"""Pins of the oracle's reconstruction and limiter formulas against their definitions.

Each quantity the oracle computes from an explicit formula of Sections 2.1 and
2.2 is recomputed here from the defining Hermite conditions and integrals in
exact rational arithmetic (tests/exact_poly.py), or checked on polynomial data
where the paper fixes the exact answer.
"""
import random
from fractions import Fraction as Fr

import pytest
import torch

from oracle import hweno_ref as o
from tests import exact_poly as ep


def _t(x):
    return torch.tensor(float(x), dtype=torch.float64)


def _rand_data(rnd, n=6):
    return [Fr(rnd.randint(-40, 40), rnd.randint(1, 9)) for _ in range(n)]


def _close(a, b, rel=1e-12, abs_=1e-12):
    a = float(a)
    b = float(b)
    return abs(a - b) <= abs_ + rel * max(abs(a), abs(b))


@pytest.mark.parametrize("seed", range(8))
def test_hermite_values_and_indicators_match_definition(seed):
    """p0, p1, p2, p0', a1..a5 and beta0..2 against eqs. HWEp0, HWEp12, GHYZ."""
    rnd = random.Random(seed)
    fm, f0, fp, Hm, H0, Hp = _rand_data(rnd)
    q0 = ep.fit_averages({-1: fm, 0: f0, 1: fp}, {-1: Hm, 0: H0, 1: Hp}, 5)
    q1 = ep.fit_averages({-1: fm, 0: f0}, {0: H0}, 2)
    q2 = ep.fit_averages({0: f0, 1: fp}, {0: H0}, 2)
    args = [_t(v) for v in (fm, f0, fp, Hm, H0, Hp)]
    p0, p1, p2 = o.hermite_values(*args)
    half = Fr(1, 2)
    assert _close(p0, ep.evaluate(q0, half))
    assert _close(p1, ep.evaluate(q1, half))
    assert _close(p2, ep.evaluate(q2, half))
    # monomial coefficients a_1..a_5 of p0 in xi
    for a, c in zip(o.quintic_coefficients(*args), q0[1:]):
        assert _close(a, c)
    b0, b1, b2 = o.smoothness_indicators(*args)
    assert _close(b0, ep.smoothness(q0), rel=1e-11)
    assert _close(b1, ep.smoothness(q1))
    assert _close(b2, ep.smoothness(q2))
    # h-hat^+ = p0'(x_{i+1/2}); with dx = 1 the scaled derivative is the x-derivative
    dq0 = ep.derivative(q0)
    assert _close(o.quintic_derivative(*args, 1.0), ep.evaluate(dq0, half))


def test_printed_beta2_differs_from_definition():
    """The explicit beta2 as printed (with f_{i-1}) is not the integral definition."""
    fm, f0, fp, H0 = Fr(3), Fr(1), Fr(-2), Fr(1, 2)
    q2 = ep.fit_averages({0: f0, 1: fp}, {0: H0}, 2)
    printed = H0 ** 2 + Fr(13, 3) * (H0 + f0 - fm) ** 2
    corrected = H0 ** 2 + Fr(13, 3) * (H0 + f0 - fp) ** 2
    assert ep.smoothness(q2) == corrected
    assert ep.smoothness(q2) != printed


@pytest.mark.parametrize("deg", range(0, 7))
def test_quintic_exact_up_to_degree_five(deg):
    """p0 and p0' at x_{i+1/2} reproduce cell-average data of any polynomial of degree <= 5."""
    rnd = random.Random(100 + deg)
    c = [Fr(rnd.randint(-9, 9), rnd.randint(1, 5)) for _ in range(deg + 1)]
    c[-1] = c[-1] or Fr(1)
    dc = ep.derivative(c)
    avg = [sum(r * ck for r, ck in zip(ep.cell_average_row(l, deg), c)) for l in (-1, 0, 1)]
    H = [sum(r * ck for r, ck in zip(ep.derivative_average_row(l, deg), c)) for l in (-1, 0, 1)]
    args = [_t(v) for v in avg + H]
    p0, p1, p2 = o.hermite_values(*args)
    exact = ep.evaluate(c, Fr(1, 2))
    dexact = ep.evaluate(dc, Fr(1, 2)) if dc else Fr(0)
    if deg <= 5:
        assert _close(p0, exact, abs_=1e-12)
        assert _close(o.quintic_derivative(*args, 1.0), dexact, abs_=1e-12)
    else:
        assert not _close(p0, exact, abs_=1e-9)
    if deg <= 2:
        assert _close(p1, exact, abs_=1e-12) and _close(p2, exact, abs_=1e-12)
        # nonlinear combination is exact for degree <= 2 whatever the weights
        for lin in [(0.98, 0.01, 0.01), (1 / 3, 1 / 3, 1 / 3), (0.01, 0.495, 0.495)]:
            assert _close(o.hweno_plus(*args, lin, 1e-6), exact, abs_=1e-11)
    elif deg == 3:
        assert not _close(p1, exact, abs_=1e-9)


def test_nonlinear_combination_is_p0_for_equal_indicators():
    """tau = 0 (all beta equal) leaves omega = gamma, so f-hat = p0."""
    # constant data: all beta are zero
    args = [_t(v) for v in (2.0, 2.0, 2.0, 0.0, 0.0, 0.0)]
    p0 = o.hermite_values(*args)[0]
    assert float(o.hweno_plus(*args, (0.5, 0.3, 0.2), 1e-6)) == pytest.approx(float(p0), abs=1e-15)
    # linear switch: omega forced to gamma
    rnd = random.Random(7)
    args = [_t(v) for v in _rand_data(rnd)]
    p0 = o.hermite_values(*args)[0]
    assert _close(o.hweno_plus(*args, (0.6, 0.3, 0.1), 1e-6, linear=True), p0)


def test_nonlinear_weights_sum_to_one_and_are_positive():
    g = torch.Generator().manual_seed(3)
    b = torch.rand(3, 1000, generator=g, dtype=torch.float64) ** 4 * 10.0
    w = o.nonlinear_weights(b[0], b[1], b[2], (0.98, 0.01, 0.01), 1e-6)
    s = w[0] + w[1] + w[2]
    assert torch.allclose(s, torch.ones_like(s), atol=1e-14)
    assert all((x > 0).all() for x in w)


def test_nonlinear_weights_see_each_indicator_plus_epsilon():
    """In the weights of Section 2.1 (eq. tau-fh and the normalised bar-omega) an
    indicator enters only as beta_l + eps, and tau only through differences of
    indicators; so raising every beta_l by s and lowering eps by s changes no weight.
    Indicators near eps, where eps matters, on three weight sets."""
    g = torch.Generator().manual_seed(5)
    eps = 1e-6
    b = 10.0 ** (torch.rand(3, 2000, generator=g, dtype=torch.float64) * 4 - 8)   # 1e-8..1e-4
    for lin in ((0.98, 0.01, 0.01), (0.5, 0.3, 0.2), (0.1, 0.45, 0.45)):
        w = o.nonlinear_weights(b[0], b[1], b[2], lin, eps)
        for shift in (2e-7, 7e-7):
            v = o.nonlinear_weights(b[0] + shift, b[1] + shift, b[2] + shift, lin, eps - shift)
            for x, y in zip(w, v):
                assert torch.allclose(x, y, rtol=1e-12, atol=0), (lin, shift)


def test_mirror_reconstruction_is_reflection():
    """f-hat^- from data at i..i+2 equals the '+' value of the reflected data (Section 2.1)."""
    rnd = random.Random(11)
    g = [Fr(rnd.randint(-30, 30), 7) for _ in range(3)]   # f^- at i, i+1, i+2
    k = [Fr(rnd.randint(-30, 30), 5) for _ in range(3)]   # dx h^- at i, i+1, i+2
    # reflected polynomial r(s) = p(1 - s) about the interface s = 1/2 (cells i, i+1, i+2
    # become 1, 0, -1); averages of p' change sign under the reflection.
    q = ep.fit_averages({1: g[0], 0: g[1], -1: g[2]}, {1: -k[0], 0: -k[1], -1: -k[2]}, 5)
    # polynomial p in the original frame centred at i+1: p(s') with cells i=-1, i+1=0, i+2=1
    p = ep.fit_averages({-1: g[0], 0: g[1], 1: g[2]}, {-1: k[0], 0: k[1], 1: k[2]}, 5)
    val = o.hweno_minus(*[_t(v) for v in g + k], (0.98, 0.01, 0.01), 1e-6, linear=True)
    # the mirrored quintic is the same polynomial: its value at the interface
    # (left edge of cell i+1) equals p(-1/2) and q(1/2)
    assert _close(val, ep.evaluate(q, Fr(1, 2)))
    assert _close(val, ep.evaluate(p, Fr(-1, 2)))
    # derivative flux: p'(-1/2) in the original frame
    dval = o.quintic_derivative_minus(*[_t(v) for v in g + k], 1.0)
    assert _close(dval, ep.evaluate(ep.derivative(p), Fr(-1, 2)))


# ---------------------------------------------------------------------------
# limiter (Section 2.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_limiter_matches_definition(seed):
    rnd = random.Random(200 + seed)
    um, u0, up, Vm, Vp = _rand_data(rnd, 5)   # V = dx * v
    q0 = ep.fit_points({-1: um, 0: u0, 1: up}, {-1: Vm, 1: Vp}, 4)
    q1 = ep.fit_points({-1: um, 0: u0}, {}, 1)
    q2 = ep.fit_points({0: u0, 1: up}, {}, 1)
    args = [_t(v) for v in (um, u0, up, Vm, Vp)]
    c0, c1, c2 = o.limiter_candidates(*args, 1.0)
    assert _close(c0, ep.evaluate(ep.derivative(q0), 0))
    assert _close(c1, ep.evaluate(ep.derivative(q1), 0))
    assert _close(c2, ep.evaluate(ep.derivative(q2), 0))
    b0, b1, b2 = o.limiter_smoothness(*args, 1.0)
    assert _close(b0, ep.smoothness(q0), rel=1e-11)
    assert _close(b1, ep.smoothness(q1))
    assert _close(b2, ep.smoothness(q2))


@pytest.mark.parametrize("deg", range(0, 6))
def test_limiter_exactness(deg):
    """q0' exact for point data of degree <= 4; v-tilde exact for degree <= 1, any weights."""
    rnd = random.Random(300 + deg)
    c = [Fr(rnd.randint(-9, 9), rnd.randint(1, 5)) for _ in range(deg + 1)]
    c[-1] = c[-1] or Fr(1)
    dc = ep.derivative(c) or [Fr(0)]
    dx = 0.25
    # point data at x = l * dx with u(x) = sum c_k (x/dx)^k
    u = [float(ep.evaluate(c, l)) for l in (-1, 0, 1)]
    v = [float(ep.evaluate(dc, l)) / dx for l in (-1, 1)]
    exact = float(ep.evaluate(dc, 0)) / dx
    q0 = o.limiter_candidates(_t(u[0]), _t(u[1]), _t(u[2]), _t(v[0]), _t(v[1]), dx)[0]
    if deg <= 4:
        assert _close(q0, exact, rel=1e-12, abs_=1e-11)
    else:
        assert not _close(q0, exact, rel=1e-9, abs_=1e-9)
    if deg <= 1:
        for d in [(0.98, 0.01, 0.01), (0.01, 0.495, 0.495)]:
            vt = o.limit_derivative(_t(u[0]), _t(u[1]), _t(u[2]), _t(v[0]), _t(v[1]), dx, d, 1e-6)
            assert _close(vt, exact, abs_=1e-11)


def test_limiter_accuracy_order_four():
    """max |v-tilde - v| = O(dx^4) on smooth data (Section 2.2)."""
    errs = []
    for n in (20, 40, 80, 160):
        x = (torch.arange(n, dtype=torch.float64) + 0.5) * (2.0 / n)
        dx = 2.0 / n
        u = torch.sin(torch.pi * x) + 0.3 * torch.cos(2 * torch.pi * x)
        v = torch.pi * torch.cos(torch.pi * x) - 0.6 * torch.pi * torch.sin(2 * torch.pi * x)
        vt = o.limit_derivative(u.roll(1), u, u.roll(-1), v.roll(1), v.roll(-1), dx,
                                (0.98, 0.01, 0.01), 1e-6)
        errs.append(float((vt - v).abs().max()))
    import math
    orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert min(orders[1:]) > 3.7, (errs, orders)
