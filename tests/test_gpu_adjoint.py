"""Discrete adjoint: the hand-written GPU VJPs against torch autograd through
the CPU oracle (speeds and time steps held fixed), against central finite
differences of the GPU forward pass (replayed), and across checkpoint
segments of the differentiable rollout."""
import sys

import numpy as np
import pytest
import torch

import hweno_inputs as hi
from oracle import hweno_ref as o
from tests import parity as P

pytestmark = pytest.mark.gpu

h = pytest.importorskip("paper_2207_05258_amd")


def announce(*what):
    print("\n[case]", *what, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    h.lib()
    yield
    torch.cuda.synchronize()


def rel_err(a, b):
    a = a.detach().cpu().to(torch.float64)
    b = b.detach().cpu().to(torch.float64)
    return float((a - b).abs().max()) / max(float(b.abs().max()), 1e-300)


def oracle_rhs_vjp(S, op, alpha, mu_L, mu_lim):
    X = S.clone().requires_grad_(True)
    loss = (o.rhs(X, op, alpha) * mu_L).sum()
    if mu_lim is not None:
        loss = loss + (o.limited_derivatives(X, op) * mu_lim).sum()
    loss.backward()
    return X.grad


def oracle_step_vjp(S, op, alphas, dt, lam):
    X = S.clone().requires_grad_(True)
    Y, _, _ = o.rk3_step(X, op, dt, alphas)
    (Y * lam).sum().backward()
    return X.grad


CASES = {
    "euler2d_rough_outflow_33x21": lambda: hi.euler2d_rough(33, 21, 1),
    "euler2d_rough_periodic_20x37": lambda: hi.euler2d_rough(20, 37, 2, bc=hi.PERIODIC),
    "euler2d_quadrants_periodic_24x18": lambda: hi.euler2d_quadrants(24, 18, 3, bc=hi.PERIODIC),
    "euler2d_rsmooth_32x32": lambda: hi.euler2d_random_smooth(32, 32, 4),
    "euler1d_piecewise_301": lambda: hi.euler1d_piecewise(301, 5),
    "euler1d_smooth_64": lambda: hi.euler1d_smooth(64),
    "burgers2d_sine_19x23": lambda: hi.scalar_sine_2d(19, 23, "burgers"),
    "linadv1d_random_270": lambda: hi.scalar_random_1d(270, 6, "linadv", a=-0.8),
    "linadv2d_random_17x40": lambda: hi.scalar_random_2d(17, 40, 7, "linadv", a=(0.6, -1.1)),
    "euler2d_rough_reflect_26x19": lambda: hi.euler2d_rough(26, 19, 16, bc=hi.REFLECT),
    "euler1d_piecewise_reflect_150": lambda: _reflect(hi.euler1d_piecewise(150, 17)),
}


def _reflect(w):
    w.bc_x = hi.REFLECT
    return w


def _mus(w, seed, dtype=torch.float64):
    g = torch.Generator().manual_seed(seed)
    m = w.m
    mu_L = torch.randn(w.S.shape, dtype=torch.float64, generator=g)
    mu_lim = torch.randn((m * w.dim,) + w.S.shape[1:], dtype=torch.float64, generator=g)
    return mu_L, mu_lim


@pytest.mark.parametrize("characteristic", [True, False], ids=["char", "comp"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_rhs_adjoint_matches_oracle_autograd(case, characteristic):
    w = CASES[case]()
    if w.physics != "euler" and not characteristic:
        pytest.skip("component-wise differs only for systems")
    announce("rhs adjoint", case, characteristic)
    Sg = P.to_gpu(w, torch.float64)
    S = P.exact_input(Sg)
    prob = P.gpu_problem(w, torch.float64, characteristic=characteristic)
    op = P.oracle_problem(w, characteristic=characteristic)
    alpha = o.max_speeds(S, op)
    mu_L, mu_lim = _mus(w, 11)
    ref = oracle_rhs_vjp(S, op, alpha, mu_L, mu_lim)
    got = h.rhs_adjoint(Sg, prob, torch.tensor(alpha, dtype=torch.float64), mu_L.cuda(), mu_lim.cuda())
    assert rel_err(got, ref) < 1e-11, rel_err(got, ref)
    # without the limiter term, and accumulating into an existing buffer
    ref2 = oracle_rhs_vjp(S, op, alpha, mu_L, None)
    base = torch.randn(Sg.shape, dtype=torch.float64, device="cuda")
    got2 = h.rhs_adjoint(Sg, prob, torch.tensor(alpha, dtype=torch.float64), mu_L.cuda(), None, base.clone())
    assert rel_err(got2 - base, ref2) < 1e-11


def test_rhs_adjoint_fp32():
    w = hi.euler2d_rough(40, 25, 8)
    announce("rhs adjoint fp32")
    Sg = P.to_gpu(w, torch.float32)
    S = P.exact_input(Sg)
    prob = P.gpu_problem(w, torch.float32)
    op = P.oracle_problem(w)
    alpha = o.max_speeds(S, op)
    mu_L, mu_lim = _mus(w, 3)
    ref = oracle_rhs_vjp(S, op, alpha, mu_L, mu_lim)
    got = h.rhs_adjoint(Sg, prob, torch.tensor(alpha, dtype=torch.float64), mu_L.float().cuda(), mu_lim.float().cuda())
    assert rel_err(got, ref) < 2e-4


# tiny 2D grids: the step adjoint folds only the two-cell boundary bands in a
# separate pass; at nx or ny = 4 the bands cover the whole grid
TINY = {
    "euler2d_rough_periodic_4x4": lambda: hi.euler2d_rough(4, 4, 12, bc=hi.PERIODIC),
    "euler2d_rough_outflow_5x4": lambda: hi.euler2d_rough(5, 4, 13),
    "euler2d_rough_periodic_4x7": lambda: hi.euler2d_rough(4, 7, 14, bc=hi.PERIODIC),
    "euler2d_rough_outflow_6x5": lambda: hi.euler2d_rough(6, 5, 15),
    "burgers2d_sine_5x6": lambda: hi.scalar_sine_2d(5, 6, "burgers"),
    "euler2d_rough_reflect_4x6": lambda: hi.euler2d_rough(4, 6, 18, bc=hi.REFLECT),
}


@pytest.mark.parametrize("limiter_on", [True, False], ids=["lim", "nolim"])
@pytest.mark.parametrize("case", ["euler2d_rough_outflow_33x21", "euler2d_rsmooth_32x32",
                                  "euler1d_piecewise_301", "burgers2d_sine_19x23",
                                  "linadv1d_random_270", "euler2d_rough_reflect_26x19",
                                  "euler1d_piecewise_reflect_150"] + sorted(TINY))
def test_step_adjoint_matches_oracle_autograd(case, limiter_on):
    w = (CASES.get(case) or TINY[case])()
    announce("step adjoint", case, limiter_on)
    Sg = P.to_gpu(w, torch.float64)
    S0 = Sg.clone()
    S = P.exact_input(Sg)
    prob = P.gpu_problem(w, torch.float64, limiter_on=limiter_on)
    op = P.oracle_problem(w, limiter_on=limiter_on)
    st = h.Stepper(prob)
    tape = torch.zeros(h.CTRL_LEN, dtype=torch.float64, device="cuda")
    st.step(Sg, tape=tape)
    tp = tape.cpu()
    alphas = [(float(tp[0]), float(tp[1])), (float(tp[2]), float(tp[3])),
              (float(tp[4]), float(tp[5]))]
    lam = torch.randn(Sg.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(5))
    ref = oracle_step_vjp(S, op, alphas, float(tp[6]), lam)
    got = lam.clone().cuda()
    h.step_adjoint(prob, S0, st, tape, got, h.adjoint_workspace(prob))
    assert rel_err(got, ref) < 1e-11, rel_err(got, ref)


CHAR_LIM = ["euler2d_rough_outflow_33x21", "euler2d_rough_periodic_20x37", "euler1d_piecewise_301",
            "euler2d_rough_reflect_26x19", "euler1d_piecewise_reflect_150"]


@pytest.mark.parametrize("case", CHAR_LIM)
def test_rhs_adjoint_characteristic_limiter(case):
    """The limiter variant on characteristic fields, differentiated through the cell's
    eigen-system, against autograd through the oracle's variant."""
    w = CASES[case]()
    announce("rhs adjoint characteristic limiter", case)
    Sg = P.to_gpu(w, torch.float64)
    S = P.exact_input(Sg)
    prob = P.gpu_problem(w, torch.float64, limiter_characteristic=True)
    op = P.oracle_problem(w, limiter_characteristic=True)
    alpha = o.max_speeds(S, op)
    mu_L, mu_lim = _mus(w, 21)
    ref = oracle_rhs_vjp(S, op, alpha, mu_L, mu_lim)
    got = h.rhs_adjoint(Sg, prob, torch.tensor(alpha, dtype=torch.float64), mu_L.cuda(), mu_lim.cuda())
    assert rel_err(got, ref) < 1e-11, rel_err(got, ref)
    # the limiter term alone
    zero = torch.zeros_like(mu_L)
    ref3 = oracle_rhs_vjp(S, op, alpha, zero, mu_lim)
    got3 = h.rhs_adjoint(Sg, prob, torch.tensor(alpha, dtype=torch.float64), zero.cuda(), mu_lim.cuda())
    assert rel_err(got3, ref3) < 1e-11, rel_err(got3, ref3)


@pytest.mark.parametrize("case", ["euler2d_rough_outflow_33x21", "euler1d_piecewise_301",
                                  "euler2d_rough_reflect_26x19", "euler2d_rough_periodic_4x4",
                                  "euler2d_rough_reflect_4x6"])
def test_step_adjoint_characteristic_limiter(case):
    w = (CASES.get(case) or TINY[case])()
    announce("step adjoint characteristic limiter", case)
    Sg = P.to_gpu(w, torch.float64)
    S0 = Sg.clone()
    S = P.exact_input(Sg)
    prob = P.gpu_problem(w, torch.float64, limiter_characteristic=True)
    op = P.oracle_problem(w, limiter_characteristic=True)
    st = h.Stepper(prob)
    tape = torch.zeros(h.CTRL_LEN, dtype=torch.float64, device="cuda")
    st.step(Sg, tape=tape)
    tp = tape.cpu()
    alphas = [(float(tp[0]), float(tp[1])), (float(tp[2]), float(tp[3])),
              (float(tp[4]), float(tp[5]))]
    lam = torch.randn(Sg.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(6))
    ref = oracle_step_vjp(S, op, alphas, float(tp[6]), lam)
    got = lam.clone().cuda()
    h.step_adjoint(prob, S0, st, tape, got, h.adjoint_workspace(prob))
    assert rel_err(got, ref) < 1e-11, rel_err(got, ref)


def _loss(S, target, dx, dy):
    return 0.5 * dx * dy * ((S[0] - target[0]) ** 2).sum()


def test_rollout_gradient_matches_oracle_across_checkpoints():
    base, target = hi.adjoint_pair(24, 0)
    announce("rollout vs oracle")
    prob = P.gpu_problem(base, torch.float64)
    U0 = P.to_gpu(base, torch.float64).requires_grad_(True)
    tgt = P.to_gpu(target, torch.float64)
    SN = h.Rollout.apply(U0, prob, 7, 3, None)       # segments of 3, 3, 1 steps
    tapes = h.Rollout.last_tapes.cpu()
    _loss(SN, tgt, base.dx, base.dy).backward()
    # oracle: the same 7 steps with the taped speeds and dt, differentiated by autograd
    X = P.exact_input(U0.detach()).requires_grad_(True)
    S = X
    op = P.oracle_problem(base)
    for n in range(7):
        t = tapes[n]
        S, _, _ = o.rk3_step(S, op, float(t[6]), [(float(t[0]), float(t[1])),
                                                   (float(t[2]), float(t[3])),
                                                   (float(t[4]), float(t[5]))])
    _loss(S, P.exact_input(tgt), base.dx, base.dy).backward()
    assert rel_err(U0.grad, X.grad) < 1e-10, rel_err(U0.grad, X.grad)


def test_rollout_keep_all_equals_checkpointed_replay():
    """Keeping every step's states (ckpt=0), checkpointing with overlapped replay and the
    automatic choice give bitwise the same gradient: the step adjoints see the same inputs."""
    base, target = hi.adjoint_pair(40, 3)
    announce("rollout keep-all vs checkpointed")
    prob = P.gpu_problem(base, torch.float64)
    tgt = P.to_gpu(target, torch.float64)
    grads, finals = {}, {}
    # 4: segments of 4, 4, 3 (the newest kept by the forward); 1: ten replayed
    # single steps and one kept; 20: one segment, kept whole
    for ck in (0, 4, 1, 20, None):
        X = P.to_gpu(base, torch.float64).requires_grad_(True)
        SN = h.Rollout.apply(X, prob, 11, ck, None)
        _loss(SN, tgt, base.dx, base.dy).backward()
        grads[ck], finals[ck] = X.grad.clone(), SN.detach().clone()
    for ck in (4, 1, 20, None):
        assert torch.equal(finals[ck], finals[0]), ck
        assert torch.equal(grads[ck], grads[0]), (ck, rel_err(grads[ck], grads[0]))
    stride = (h.workspace_bytes(prob) + 255) // 256 * 256
    assert h.rollout_bytes_kept(prob, 11) == 11 * (stride + 12 * 40 * 40 * 8)


def test_rollout_gradient_matches_finite_differences():
    base, target = hi.adjoint_pair(32, 1)
    announce("rollout vs finite differences")
    prob = P.gpu_problem(base, torch.float64)
    U0 = P.to_gpu(base, torch.float64)
    tgt = P.to_gpu(target, torch.float64)
    X = U0.clone().requires_grad_(True)
    SN = h.Rollout.apply(X, prob, 20, 7, None)
    tapes = h.Rollout.last_tapes.clone()
    _loss(SN, tgt, base.dx, base.dy).backward()
    g = torch.Generator().manual_seed(9)
    for k in range(3):
        d = torch.randn(U0.shape, dtype=torch.float64, generator=g).cuda()
        if k == 0:
            d[4:] = 0.0     # perturb the solution fields only
        eps = 1e-5
        jp = _loss(h.rollout_replay(U0 + eps * d, prob, tapes), tgt, base.dx, base.dy)
        jm = _loss(h.rollout_replay(U0 - eps * d, prob, tapes), tgt, base.dx, base.dy)
        fd = float((jp - jm) / (2 * eps))
        an = float((X.grad * d).sum())
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-12), (k, an, fd)


def test_step_dot_product_identity():
    """<J d, l> = <d, J^T l> with J d from central differences of the replayed step."""
    w = hi.euler2d_rough(28, 19, 4)
    announce("dot product")
    prob = P.gpu_problem(w, torch.float64)
    S0 = P.to_gpu(w, torch.float64)
    st = h.Stepper(prob)
    tape = torch.zeros(h.CTRL_LEN, dtype=torch.float64, device="cuda")
    S1 = S0.clone()
    st.step(S1, tape=tape)
    g = torch.Generator().manual_seed(2)
    d = torch.randn(S0.shape, dtype=torch.float64, generator=g).cuda()
    lam = torch.randn(S0.shape, dtype=torch.float64, generator=g).cuda()
    eps = 1e-6
    Jd = (h.rollout_replay(S0 + eps * d, prob, tape[None]) -
          h.rollout_replay(S0 - eps * d, prob, tape[None])) / (2 * eps)
    JT = lam.clone()
    h.step_adjoint(prob, S0, st, tape, JT, h.adjoint_workspace(prob))
    lhs = float((Jd * lam).sum())
    rhs = float((d * JT).sum())
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)


def test_rollout_fp32_close_to_fp64():
    base, target = hi.adjoint_pair(64, 2)
    announce("rollout fp32 vs fp64")
    grads = {}
    for dtype in (torch.float64, torch.float32):
        prob = P.gpu_problem(base, dtype)
        X = P.to_gpu(base, dtype).requires_grad_(True)
        SN = h.Rollout.apply(X, prob, 30, 10, None)
        _loss(SN, P.to_gpu(target, dtype), base.dx, base.dy).backward()
        grads[dtype] = X.grad[:4].double()
    assert rel_err(grads[torch.float32], grads[torch.float64]) < 1e-3


def test_rollout_at_full_size_512_200_steps():
    """The adjoint configuration as the bench times it: 512^2 2D Euler, 200 steps, a
    checkpoint every 20, loss = L2 mismatch of the final density.  The FP64 gradient
    agrees with central differences of the replayed FP64 rollout along random
    directions to 1e-6 (measured: 2e-10 to 3e-9 at eps = 1e-5); the FP32 gradient
    is within 1e-3 of the FP64 one, relative to its largest entry (measured: 6.5e-5);
    and in FP32 keeping every step's states gives bitwise the checkpointed gradient."""
    base, target = hi.adjoint_pair(512, 0)
    announce("rollout 512^2, 200 steps, checkpoint every 20")
    grads = {}
    for dtype in (torch.float64, torch.float32):
        prob = P.gpu_problem(base, dtype)
        X = P.to_gpu(base, dtype).requires_grad_(True)
        SN = h.Rollout.apply(X, prob, 200, 20, None)
        if dtype == torch.float64:
            tapes = h.Rollout.last_tapes.clone()
        _loss(SN, P.to_gpu(target, dtype), base.dx, base.dy).backward()
        grads[dtype] = X.grad.detach().clone()
    assert rel_err(grads[torch.float32], grads[torch.float64]) < 1e-3, \
        rel_err(grads[torch.float32], grads[torch.float64])
    prob = P.gpu_problem(base, torch.float64)
    U0 = P.to_gpu(base, torch.float64)
    tgt = P.to_gpu(target, torch.float64)
    g = torch.Generator().manual_seed(9)
    eps = 1e-5
    for k in range(2):
        d = torch.randn(U0.shape, dtype=torch.float64, generator=g).cuda()
        if k == 0:
            d[4:] = 0.0     # the solution fields only
        jp = _loss(h.rollout_replay(U0 + eps * d, prob, tapes), tgt, base.dx, base.dy)
        jm = _loss(h.rollout_replay(U0 - eps * d, prob, tapes), tgt, base.dx, base.dy)
        fd = float((jp - jm) / (2 * eps))
        an = float((grads[torch.float64] * d).sum())
        print(f"[512^2 rollout] direction {k}: adjoint {an:.12e} central differences {fd:.12e}",
              flush=True)
        assert abs(an - fd) <= 1e-6 * abs(fd), (k, an, fd)
    prob = P.gpu_problem(base, torch.float32)
    X = P.to_gpu(base, torch.float32).requires_grad_(True)
    SN = h.Rollout.apply(X, prob, 200, 0, None)
    _loss(SN, P.to_gpu(target, torch.float32), base.dx, base.dy).backward()
    assert torch.equal(X.grad, grads[torch.float32])
