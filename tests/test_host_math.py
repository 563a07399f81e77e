"""The kernels' arithmetic (hweno_math.h, built for the host, where its
reciprocals and square roots are the exact library ones) against the oracle's
literal formulas, on seeded data: the reconstruction and the limiter (Sections
2.1 / 2.2) from smooth to discontinuous data over many decades of magnitude --
the rearranged combinations (FP64: numerator and denominator times the product
of the three beta_l + eps, epsilon starting the indicator sums; FP32: one
reciprocal per weight) compute the same function -- and, for 2D Euler, the
point fluxes with their chain-rule products (eq. EQ3) and the closed-form
characteristic projection (Remarks 2.1/2.2: L x solves R w = x for the oracle's
right eigenvectors at the Roe average, and R L x = x); and the hand-written
reverse-mode derivatives of the reconstruction, the limiter and the point fluxes
(hweno_adjoint.h) against torch autograd through the oracle's formulas; and the
characteristic limiter variant and its reverse against the oracle's (one periodic
3-cell row per stencil).
Bounds, relative to the data's scale (for the point fluxes the largest
component of each output vector, for the projection |x| times the condition
number of R): FP64 1e-13, FP32 2e-6 (5e-6 for the point fluxes: a few FP32 ulps
of the largest term).  FP32 data stay within six decades of their scale: beyond
that tau = O(beta^2) leaves the FP32 range."""
import hashlib
import os
import subprocess

import numpy as np
import pytest
import torch

from oracle import hweno_ref as o

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
SRC = ["tests/host/math_host.cpp", "paper_2207_05258_amd/csrc/hweno_math.h",
       "paper_2207_05258_amd/csrc/hweno_adjoint.h"]
LIN = (0.98, 0.01, 0.01)   # the paper's linear weights gamma
LIM = (0.98, 0.01, 0.01)   # and d
EPS = 1e-6
GAMMA = 1.4


def _exe():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    h = hashlib.sha256()
    for s in SRC:
        with open(os.path.join(ROOT, s), "rb") as fh:
            h.update(fh.read())
    out = os.path.join("/tmp", "hweno_math_host", h.hexdigest()[:16])
    exe = os.path.join(out, "math_host")
    if not os.path.exists(exe):
        os.makedirs(out, exist_ok=True)
        cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               os.path.join(ROOT, SRC[0]), "-o", exe + ".tmp"]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
        os.replace(exe + ".tmp", exe)
    return exe


def _run(op, prec, rows):
    args = [_exe()] + [repr(x) for x in LIN + LIM] + [repr(EPS), repr(GAMMA)]
    text = "".join(f"{op} {prec} " + " ".join(repr(float(x)) for x in r) + "\n" for r in rows)
    r = subprocess.run(args, input=text, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = np.array([[float(x) for x in ln.split()] for ln in r.stdout.splitlines()])
    assert out.shape[0] == len(rows)
    return out[:, 0] if out.shape[1] == 1 else out


def _data(seed, n=4000, decades=4, jumps=6):
    """Six-value stencils: smooth (small differences around a level), kinked,
    discontinuous (one jump of up to `jumps` decades) and all-zero-derivative
    rows, at levels from 10^-decades to 10^decades."""
    g = np.random.default_rng(seed)
    level = 10.0 ** g.uniform(-decades, decades, n)
    base = g.uniform(-1, 1, (n, 6)) * level[:, None]
    kind = g.integers(0, 4, n)
    smooth = level[:, None] * (1 + 1e-3 * g.standard_normal((n, 6)))
    rows = np.where((kind == 0)[:, None], smooth, base)
    jump = 10.0 ** g.uniform(0, jumps, n)
    rows[kind == 2, 2] *= jump[kind == 2]
    rows[kind == 3, 3:] = 0.0
    return rows


# FP32 data stay where tau = O(beta^2) is in range: beta_0 carries weights up to
# 1.6e4 on squared data, so values within about 1e6 of the data's scale
FP32_RANGE = dict(decades=2, jumps=3)


def _scale(rows):
    return np.abs(rows).max(axis=1)


@pytest.mark.parametrize("prec,tol", [("d", 1e-13), ("f", 2e-6)])
def test_reconstruction_matches_the_oracle(prec, tol):
    rows = _data(11) if prec == "d" else _data(11, **FP32_RANGE)
    if prec == "f":
        rows = rows.astype(np.float32).astype(np.float64)
    got = _run("r", prec, rows)
    t = torch.as_tensor(rows, dtype=torch.float64)
    ref = o.hweno_plus(t[:, 0], t[:, 1], t[:, 2], t[:, 3], t[:, 4], t[:, 5], LIN, EPS).numpy()
    err = np.abs(got - ref) / _scale(rows)
    assert err.max() <= tol, (err.max(), rows[err.argmax()])


@pytest.mark.parametrize("prec,tol", [("d", 1e-13), ("f", 2e-6)])
def test_limiter_matches_the_oracle(prec, tol):
    rows = _data(12) if prec == "d" else _data(12, **FP32_RANGE)
    g = np.random.default_rng(13)
    rows[:, 5] = 10.0 ** g.uniform(-3, -1, len(rows))    # the cell size h
    if prec == "f":
        rows = rows.astype(np.float32).astype(np.float64)
    got = _run("l", prec, rows)
    t = torch.as_tensor(rows, dtype=torch.float64)
    ref = o.limit_derivative(t[:, 0], t[:, 1], t[:, 2], t[:, 3], t[:, 4], t[:, 5], LIM,
                             EPS).numpy()
    # the limited derivative is O(data / h + derivatives)
    scale = np.maximum(np.abs(rows[:, :3]).max(axis=1) / rows[:, 5], np.abs(rows[:, 3:5]).max(axis=1))
    err = np.abs(got - ref) / scale
    assert err.max() <= tol, (err.max(), rows[err.argmax()])


def _states(g, n):
    """Admissible 2D Euler states: density 1e-2..1e2, velocity up to Mach ~3,
    pressure 1e-2..1e3."""
    rho = 10.0 ** g.uniform(-2, 2, n)
    p = 10.0 ** g.uniform(-2, 3, n)
    c = np.sqrt(GAMMA * p / rho)
    u = g.uniform(-3, 3, n) * c
    v = g.uniform(-3, 3, n) * c
    E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E], 1)


class _Prob:
    gamma_gas = GAMMA
    dim = 2


@pytest.mark.parametrize("prec,tol", [("d", 1e-13), ("f", 5e-6)])
def test_point_fluxes_match_the_oracle(prec, tol):
    g = np.random.default_rng(21)
    n = 2000
    U = _states(g, n)
    D = g.standard_normal((n, 8)) * np.abs(U).max(1, keepdims=True)
    rows = np.concatenate([U, D], 1)
    if prec == "f":
        rows = rows.astype(np.float32).astype(np.float64)
    got = _run("p", prec, rows)
    t = torch.as_tensor(rows, dtype=torch.float64)
    eu = o.Euler(_Prob())
    ref = torch.cat([eu.flux(t[:, :4], 0), eu.jvp(t[:, :4], t[:, 4:8], 0),
                     eu.jvp(t[:, :4], t[:, 8:], 0)], 1).numpy()
    # relative to the largest component of each output vector (F, A Dn, A Dt)
    scale = np.abs(ref).reshape(-1, 3, 4).max(2, keepdims=True).repeat(4, 2).reshape(-1, 12)
    err = np.abs(got - ref) / scale
    assert err.max() <= tol, (err.max(), np.unravel_index(err.argmax(), err.shape))


@pytest.mark.parametrize("prec,tol", [("d", 1e-13), ("f", 2e-6)])
def test_characteristic_projection_inverts_the_right_eigenvectors(prec, tol):
    g = np.random.default_rng(22)
    n = 2000
    UL, UR = _states(g, n), _states(g, n)
    x = g.standard_normal((n, 4)) * np.abs(UL).max(1, keepdims=True)
    rows = np.concatenate([UL, UR, x], 1)
    if prec == "f":
        rows = rows.astype(np.float32).astype(np.float64)
    got = _run("e", prec, rows)
    t = torch.as_tensor(rows, dtype=torch.float64)
    R = o.Euler(_Prob()).right_eigenvectors(t[:, :4], t[:, 4:8], 0)
    w_ref = torch.linalg.solve(R, t[:, 8:]).numpy()
    xs = np.abs(rows[:, 8:]).max(1, keepdims=True)
    cond = torch.linalg.cond(R).numpy()[:, None]
    err_w = np.abs(got[:, :4] - w_ref) / (xs * cond)
    err_x = np.abs(got[:, 4:] - rows[:, 8:]) / (xs * cond)
    assert err_w.max() <= tol, err_w.max()
    assert err_x.max() <= tol, err_x.max()


def _grad(fn, rows):
    t = torch.as_tensor(rows, dtype=torch.float64).clone().requires_grad_(True)
    fn(t).sum().backward()
    return t.grad.numpy()


def test_reconstruction_and_limiter_adjoints_match_autograd():
    rows = _data(31)
    got = _run("R", "d", rows)
    ref = _grad(lambda t: o.hweno_plus(t[:, 0], t[:, 1], t[:, 2], t[:, 3], t[:, 4], t[:, 5], LIN, EPS),
                rows)
    # gradients of a function O(1) in the data's units: compare relative to the largest entry
    err = np.abs(got - ref) / np.abs(ref).max(1, keepdims=True)
    assert err.max() <= 1e-11, err.max()
    rows = _data(32)
    rows[:, 5] = 10.0 ** np.random.default_rng(33).uniform(-3, -1, len(rows))
    got = _run("L", "d", rows)
    ref = _grad(lambda t: o.limit_derivative(t[:, 0], t[:, 1], t[:, 2], t[:, 3], t[:, 4],
                                             t[:, 5].detach(), LIM, EPS), rows)[:, :5]
    err = np.abs(got - ref) / np.abs(ref).max(1, keepdims=True)
    assert err.max() <= 1e-11, err.max()


def test_point_flux_adjoint_matches_autograd():
    g = np.random.default_rng(34)
    n = 2000
    U = _states(g, n)
    D = g.standard_normal((n, 8)) * np.abs(U).max(1, keepdims=True)
    gout = g.standard_normal((n, 12))
    rows = np.concatenate([U, D, gout], 1)
    got = _run("P", "d", rows)
    t = torch.as_tensor(rows[:, :12], dtype=torch.float64).clone().requires_grad_(True)
    eu = o.Euler(_Prob())
    out = torch.cat([eu.flux(t[:, :4], 0), eu.jvp(t[:, :4], t[:, 4:8], 0),
                     eu.jvp(t[:, :4], t[:, 8:], 0)], 1)
    (out * torch.as_tensor(gout)).sum().backward()
    ref = t.grad.numpy()
    err = np.abs(got - ref) / np.abs(ref).max(1, keepdims=True)
    assert err.max() <= 1e-11, err.max()


H_CHAR = 1.0 / 64.0


def _char_rows(seed, n=1500):
    """Characteristic-limiter stencils of 2D Euler: three admissible states (the
    neighbours close to the centre in half the rows, independent in the others)
    and the two neighbours' x-derivatives, about |U| / h in size."""
    g = np.random.default_rng(seed)
    u0 = _states(g, n)
    um, up = _states(g, n), _states(g, n)
    near = g.random(n) < 0.5
    for a in (um, up):
        a[near] = u0[near] * (1.0 + 0.02 * g.uniform(-1, 1, (int(near.sum()), 1)))
    sc = np.abs(u0).max(1, keepdims=True) / H_CHAR
    vm = g.standard_normal((n, 4)) * sc * 0.1
    vp = g.standard_normal((n, 4)) * sc * 0.1
    return np.concatenate([um, u0, up, vm, vp, np.full((n, 1), H_CHAR)], 1)


def _oracle_char_grid(rows):
    """One periodic 3-cell row per stencil; cell 1's x-limiter reads exactly it."""
    n = len(rows)
    S = torch.zeros(12, n, 3, dtype=torch.float64)
    t = torch.as_tensor(rows, dtype=torch.float64)
    for k in range(3):
        S[:4, :, k] = t[:, 4 * k:4 * k + 4].T
    S[4:8, :, 0] = t[:, 12:16].T
    S[4:8, :, 2] = t[:, 16:20].T
    prob = o.Problem(dim=2, physics="euler", dx=H_CHAR, dy=H_CHAR, lim_w=LIM, eps=EPS,
                     gamma_gas=GAMMA, limiter_characteristic=True)
    return S, prob


@pytest.mark.parametrize("prec,tol", [("d", 1e-13), ("f", 2e-6)])
def test_characteristic_limiter_matches_the_oracle(prec, tol):
    """The characteristic limiter variant (each stencil vector projected on the left
    eigenvectors of the cell's own state, the scalar Section 2.2 limiter per field,
    back with the right eigenvectors) against the oracle's, relative to |U| / h times
    the condition number of the cell's eigenvectors."""
    rows = _char_rows(41)
    if prec == "f":
        rows = rows.astype(np.float32).astype(np.float64)
    got = _run("c", prec, rows)
    S, prob = _oracle_char_grid(rows)
    ref = o.limited_derivatives(S, prob)[:4, :, 1].T.numpy()
    u0 = torch.as_tensor(rows[:, 4:8])
    cond = torch.linalg.cond(o.Euler(prob).right_eigenvectors(u0, u0, 0)).numpy()
    scale = (np.abs(rows[:, :12]).max(1) / H_CHAR + np.abs(rows[:, 12:20]).max(1)) * cond
    err = np.abs(got - ref) / scale[:, None]
    assert err.max() <= tol, (err.max(), np.unravel_index(err.argmax(), err.shape))


def test_characteristic_limiter_adjoint_matches_autograd():
    """The reverse of the characteristic limiter (through the cell's eigen-system, the
    projections and the scalar limiters) against torch autograd through the oracle,
    relative to the largest entry times the condition number of the cell's right
    eigenvectors (the oracle inverts them numerically; where the sound speed is small
    the two sides differ by up to 1e-9 of the largest entry, 3e-12 once scaled)."""
    rows = _char_rows(42, 800)
    gout = np.random.default_rng(43).standard_normal((len(rows), 4))
    got = _run("C", "d", np.concatenate([rows, gout], 1))
    S, prob = _oracle_char_grid(rows)
    X = S.clone().requires_grad_(True)
    (o.limited_derivatives(X, prob)[:4, :, 1] * torch.as_tensor(gout).T).sum().backward()
    G = X.grad
    ref = np.concatenate([G[:4, :, 0].T, G[:4, :, 1].T, G[:4, :, 2].T, G[4:8, :, 0].T,
                          G[4:8, :, 2].T], 1)
    u0 = torch.as_tensor(rows[:, 4:8])
    cond = torch.linalg.cond(o.Euler(prob).right_eigenvectors(u0, u0, 0)).numpy()
    err = np.abs(got - ref) / (np.abs(ref).max(1, keepdims=True) * cond[:, None])
    assert err.max() <= 1e-11, (err.max(), np.unravel_index(err.argmax(), err.shape))
