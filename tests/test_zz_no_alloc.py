"""The allocation-free step (hweno_rk3_step_static) against hweno_rk3_step.

The static variant runs the same kernels with its stage states in the
library's static device array instead of a caller workspace, so its states,
control blocks and tapes must equal the workspace entry point's bit for bit.
Two calls in a row, the second on a smaller grid, check that a call leaves
nothing in the array that the next one depends on; the largest grid that fits
(512 x 512 FP64 2D Euler fills the 64 MiB exactly) and the first one that does
not bound the size check.
"""
import ctypes

import pytest
import torch

import hweno_inputs as hi
import paper_2207_05258_amd as h
from paper_2207_05258_amd import hweno as hw

CTRL = h.CTRL_LEN


def _lib():
    return h.lib()


def _static(prob, S, ctrl, tape=None, dt=0.0, t_end=0.0, replay=None):
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return _lib().hweno_rk3_step_static(
        ctypes.byref(prob.c()), ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(ctrl.data_ptr()),
        float(dt), float(t_end), None if tape is None else ctypes.c_void_p(tape.data_ptr()),
        None if replay is None else ctypes.c_void_p(replay.data_ptr()), stream)


def _quadrants(n, m, dtype, seed, bc=h.OUTFLOW):
    w = hi.euler2d_quadrants(n, m, seed)
    prob = h.Problem(dim=2, nx=n, ny=m, physics="euler", dtype=dtype, dx=1.0 / n, dy=1.0 / m,
                     bc_x=bc, bc_y=bc)
    return prob, torch.as_tensor(w.S).to(dtype)


def _check_against_workspace(prob, S0, steps=2):
    """`steps` steps through both entry points from the same state; returns nothing,
    asserts bitwise equality of the states, control blocks and tapes."""
    A = S0.cuda().contiguous()
    B = A.clone()
    st = h.Stepper(prob)
    ctrl = torch.zeros(CTRL, dtype=torch.float64, device="cuda")
    tA = torch.zeros(steps, CTRL, dtype=torch.float64, device="cuda")
    tB = torch.zeros_like(tA)
    for k in range(steps):
        st.step(A, tape=tA[k])
        assert _static(prob, B, ctrl, tape=tB[k]) == 0, _lib().hweno_last_error().decode()
    torch.cuda.synchronize()
    print(f"static step {prob.nx}x{prob.ny} {prob.dtype}: t {float(ctrl[7]):.6e}", flush=True)
    assert torch.equal(A, B)
    assert torch.equal(st.ctrl, ctrl)
    assert torch.equal(tA, tB)
    assert int(ctrl[8:9].view(torch.int64).item()) == 0
    assert int(ctrl[9]) == steps


def test_static_step_rejects_grids_beyond_the_array():
    """Host checks, before any HIP call: the size limit, NULL pointers."""
    L = _lib()
    ctrl = ctypes.c_void_p(256)   # never dereferenced: the call returns before any HIP call
    S = ctypes.c_void_p(4096)
    big = h.Problem(dim=2, nx=513, ny=512, physics="euler", dtype=torch.float64, dx=1.0, dy=1.0)
    assert L.hweno_rk3_step_static(ctypes.byref(big.c()), S, ctrl, 0.0, 0.0, None, None, None) == 3
    assert "static scratch" in L.hweno_last_error().decode()
    big32 = h.Problem(dim=2, nx=725, ny=724, physics="euler", dtype=torch.float32, dx=1.0, dy=1.0)
    assert L.hweno_rk3_step_static(ctypes.byref(big32.c()), S, ctrl, 0.0, 0.0, None, None, None) == 3
    ok = h.Problem(dim=2, nx=64, ny=64, physics="euler", dtype=torch.float64, dx=1.0, dy=1.0)
    assert L.hweno_rk3_step_static(ctypes.byref(ok.c()), S, None, 0.0, 0.0, None, None, None) == 1
    assert L.hweno_rk3_step_static(ctypes.byref(ok.c()), None, ctrl, 0.0, 0.0, None, None, None) == 1
    odd = ctypes.c_void_p(4)
    assert L.hweno_rk3_step_static(ctypes.byref(ok.c()), S, odd, 0.0, 0.0, None, None, None) == 1
    assert L.hweno_rk3_step_static(ctypes.byref(ok.c()), S, ctrl, float("nan"), 0.0, None, None,
                                   None) == 1
    # an empty grid is a valid problem with nothing to do
    empty = h.Problem(dim=2, nx=0, ny=5, physics="euler", dtype=torch.float64, dx=1.0, dy=1.0)
    assert L.hweno_rk3_step_static(ctypes.byref(empty.c()), S, ctrl, 0.0, 0.0, None, None,
                                   None) == 0


@pytest.mark.gpu
def test_two_calls_in_a_row_the_second_smaller():
    """A 2D Euler FP64 step on 200 x 176, then a smaller FP32 one on 67 x 45 (and a
    1D Euler one), each bitwise equal to hweno_rk3_step on the same input."""
    prob, S = _quadrants(200, 176, torch.float64, 1)
    _check_against_workspace(prob, S)
    prob, S = _quadrants(67, 45, torch.float32, 2, bc=h.PERIODIC)
    _check_against_workspace(prob, S)
    w = hi.euler1d_piecewise(301, 3)
    prob = h.Problem(dim=1, nx=301, physics="euler", dtype=torch.float64, dx=w.dx, bc_x=w.bc_x)
    _check_against_workspace(prob, torch.as_tensor(w.S))


@pytest.mark.gpu
def test_largest_grid_that_fits_and_replay():
    """512 x 512 FP64 fills the array exactly; replayed speeds and dt give the same
    step as well; a fixed dt with t_end clipping goes through the same control."""
    prob, S = _quadrants(512, 512, torch.float64, 0)
    _check_against_workspace(prob, S, steps=1)
    A = S.cuda().contiguous()
    st = h.Stepper(prob)
    tape = torch.zeros(CTRL, dtype=torch.float64, device="cuda")
    ref = A.clone()
    st.step(ref, tape=tape)
    B = A.clone()
    ctrl = torch.zeros(CTRL, dtype=torch.float64, device="cuda")
    assert _static(prob, B, ctrl, replay=tape) == 0
    torch.cuda.synchronize()
    assert torch.equal(ref, B)
    # fixed dt, clipped by t_end on the second step
    prob2, S2 = _quadrants(96, 80, torch.float64, 4)
    A = S2.cuda().contiguous()
    B = A.clone()
    st = h.Stepper(prob2)
    ctrl = torch.zeros(CTRL, dtype=torch.float64, device="cuda")
    for _ in range(2):
        st.step(A, dt=1e-3, t_end=1.5e-3)
        assert _static(prob2, B, ctrl, dt=1e-3, t_end=1.5e-3) == 0
    torch.cuda.synchronize()
    assert torch.equal(A, B) and torch.equal(st.ctrl, ctrl)
    assert float(ctrl[7]) == pytest.approx(1.5e-3, rel=1e-15)
