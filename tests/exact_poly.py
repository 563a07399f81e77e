"""Exact rational polynomial fitting, used to pin the oracle to the definitions.

The Hermite polynomials of Section 2.1 (eqs. HWEp0, HWEp12) and Section 2.2 are
built here directly from their defining conditions by solving the linear
systems in ``fractions.Fraction`` arithmetic, and the smoothness indicators
from their integral definitions (eqs. GHYZ, GHYZ-q).  Nothing here is taken
from the explicit formulas the oracle implements.

Coordinates are scaled: xi = (x - x_i) / dx, so cell I_{i+l} is
[l - 1/2, l + 1/2], the interface x_{i+1/2} is xi = 1/2, and a derivative
datum h (per unit x) enters as H = dx * h.
"""
from fractions import Fraction as Fr


def solve(A, b):
    """Gaussian elimination with exact fractions (A square, nonsingular)."""
    n = len(A)
    M = [list(map(Fr, row)) + [Fr(bv)] for row, bv in zip(A, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [a - f * c for a, c in zip(M[r], M[col])]
    return [M[r][n] / M[r][r] for r in range(n)]


def antideriv_at(c, x):
    return sum(ck * Fr(x) ** (k + 1) / (k + 1) for k, ck in enumerate(c))


def evaluate(c, x):
    return sum(ck * Fr(x) ** k for k, ck in enumerate(c))


def derivative(c):
    return [k * ck for k, ck in enumerate(c)][1:]


def cell_average_row(l, deg):
    """Row of coefficients of avg_{[l-1/2, l+1/2]} xi^k, k = 0..deg."""
    a, b = Fr(2 * l - 1, 2), Fr(2 * l + 1, 2)
    return [(b ** (k + 1) - a ** (k + 1)) / (k + 1) for k in range(deg + 1)]


def derivative_average_row(l, deg):
    """Row for p(l + 1/2) - p(l - 1/2) (= dx times the average of p' on I_{i+l})."""
    a, b = Fr(2 * l - 1, 2), Fr(2 * l + 1, 2)
    return [b ** k - a ** k for k in range(deg + 1)]


def fit_averages(avg, davg, deg):
    """Polynomial (coefficients in xi) with given cell averages and derivative averages.

    avg: {l: value}, davg: {l: H value}; the number of conditions is deg + 1.
    """
    rows, rhs = [], []
    for l, val in avg.items():
        rows.append(cell_average_row(l, deg))
        rhs.append(val)
    for l, val in davg.items():
        rows.append(derivative_average_row(l, deg))
        rhs.append(val)
    assert len(rows) == deg + 1
    return solve(rows, rhs)


def fit_points(vals, dvals, deg):
    """Polynomial with given point values p(l) and scaled derivatives p'(l) (= dx v_l)."""
    rows, rhs = [], []
    for l, val in vals.items():
        rows.append([Fr(l) ** k for k in range(deg + 1)])
        rhs.append(val)
    for l, val in dvals.items():
        rows.append([k * Fr(l) ** (k - 1) if k > 0 else Fr(0) for k in range(deg + 1)])
        rhs.append(val)
    assert len(rows) == deg + 1
    return solve(rows, rhs)


def smoothness(c):
    """sum_{a=1..deg} integral over [-1/2, 1/2] of (p^(a))^2 in scaled coordinates.

    In x this is sum_a int_{I_i} dx^(2a-1) (d^a p / dx^a)^2 dx.
    """
    total = Fr(0)
    d = derivative(c)
    while d:
        sq = [Fr(0)] * (2 * len(d) - 1)
        for i, a in enumerate(d):
            for j, b in enumerate(d):
                sq[i + j] += a * b
        total += antideriv_at(sq, Fr(1, 2)) - antideriv_at(sq, Fr(-1, 2))
        d = derivative(d)
    return total
