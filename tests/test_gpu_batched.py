"""Batched uneven 2D Euler instances: the persistent batched kernels against
per-instance hweno_rk3_step (bitwise: same arithmetic) and against the oracle,
plus hipGraph capture and replay."""
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


def _batch(ws, dtype, **common_kw):
    states = [P.to_gpu(w, dtype) for w in ws]
    grids = [dict(dx=w.dx, dy=w.dy, bc_x=w.bc_x, bc_y=w.bc_y) for w in ws]
    common = h.Problem(dim=2, nx=1, ny=1, physics="euler", dtype=dtype, **common_kw)
    return states, grids, common


def _individual(ws, dtype, steps=1, **common_kw):
    outs, ctrls = [], []
    for w in ws:
        S = P.to_gpu(w, dtype)
        st = h.Stepper(P.gpu_problem(w, dtype, **common_kw))
        for _ in range(steps):
            st.step(S)
        outs.append(S)
        ctrls.append(st.ctrl.clone())
    return outs, ctrls


UNEVEN = [(37, 29), (16, 15), (5, 3), (64, 7), (1, 1), (33, 46), (100, 18)]


@pytest.mark.parametrize("blocks", [0, 5, 16], ids=["one_tile_per_wg", "persistent5", "banded16"])
@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_batched_equals_individual_bitwise(variant, dtype, blocks):
    """blocks=0 gives one workgroup per tile here (the batch has fewer tiles
    than resident workgroups); blocks=5 and 16 make every workgroup walk
    several tiles (plain striding below 8 workgroups, XCD bands from 8 on)."""
    ws = hi.batched_instances(len(UNEVEN), 3, sizes=UNEVEN)
    announce("batched == individual", variant, dtype, blocks)
    states, grids, common = _batch(ws, dtype)
    b = h.BatchedStepper(states, grids, common)
    for _ in range(2):
        b.step(variant=variant, blocks=blocks)
    ref, ctrls = _individual(ws, dtype, steps=2)
    for q in range(len(ws)):
        assert torch.equal(states[q], ref[q]), (q, ws[q].name)
        assert torch.equal(b.ctrl(q)[:10], ctrls[q][:10]), q


def test_batched_mixed_boundaries_equal_individual():
    """Instances with periodic, outflow and reflecting walls in one batch."""
    ws = hi.batched_instances(4, 21, sizes=[(30, 17), (17, 30), (24, 24), (9, 40)])
    bcs = [(hi.REFLECT, hi.REFLECT), (hi.REFLECT, hi.PERIODIC), (hi.OUTFLOW, hi.REFLECT),
           (hi.PERIODIC, hi.OUTFLOW)]
    for w, (bx, by) in zip(ws, bcs):
        w.bc_x, w.bc_y = bx, by
    announce("batched mixed walls")
    states, grids, common = _batch(ws, torch.float64)
    b = h.BatchedStepper(states, grids, common)
    b.step()
    ref, _ = _individual(ws, torch.float64)
    for q in range(len(ws)):
        assert torch.equal(states[q], ref[q]), q


@pytest.mark.parametrize("variant", [0, 1])
def test_batched_characteristic_limiter_equals_individual(variant):
    """The characteristic limiter variant, set on the common problem, in both tile variants."""
    ws = hi.batched_instances(3, 23, sizes=[(30, 17), (9, 40), (24, 24)])
    ws[1].bc_x = ws[1].bc_y = hi.REFLECT
    announce("batched characteristic limiter", variant)
    states, grids, common = _batch(ws, torch.float64, limiter_characteristic=True)
    b = h.BatchedStepper(states, grids, common)
    b.step(variant=variant, blocks=4)
    ref, _ = _individual(ws, torch.float64, limiter_characteristic=True)
    for q in range(len(ws)):
        assert torch.equal(states[q], ref[q]), q


def test_batched_against_oracle():
    ws = hi.batched_instances(4, 11, sizes=[(40, 23), (18, 35), (64, 16), (9, 9)])
    announce("batched vs oracle")
    states, grids, common = _batch(ws, torch.float64)
    S0 = [P.exact_input(S) for S in states]
    b = h.BatchedStepper(states, grids, common)
    b.step(variant=1, blocks=3)
    for q, w in enumerate(ws):
        ref, dt, _ = o.rk3_step(S0[q], P.oracle_problem(w))
        assert float(b.ctrl(q)[6]) == pytest.approx(dt, rel=1e-13)
        P.assert_within(P.step_errors(states[q], ref, w), 1e-12, f"batched {w.name}")


def test_batched_per_instance_time_control():
    ws = hi.batched_instances(3, 5, sizes=[(20, 20), (24, 16), (16, 24)])
    announce("batched dt/t_end")
    states, grids, common = _batch(ws, torch.float64)
    grids[0]["dt_fixed"] = 1e-4
    grids[1]["t_end"] = 1e-12       # reached after the first (tiny) step
    S0 = [S.clone() for S in states]
    b = h.BatchedStepper(states, grids, common)
    b.step()
    b.step()
    assert float(b.ctrl(0)[6]) == 1e-4 and float(b.ctrl(0)[7]) == pytest.approx(2e-4)
    assert float(b.ctrl(1)[7]) == pytest.approx(1e-12, rel=1e-9)
    assert b.statuses()[1] & h.hweno.ST_SKIPPED
    assert float(b.ctrl(1)[9]) == 1.0 and float(b.ctrl(2)[9]) == 2.0
    ref, _, _ = o.rk3_step(P.exact_input(S0[0]), P.oracle_problem(ws[0]), 1e-4)
    ref, _, _ = o.rk3_step(ref, P.oracle_problem(ws[0]), 1e-4)
    P.assert_within(P.step_errors(states[0], ref, ws[0]), 1e-12, "fixed dt instance")


def test_batched_graph_replays_match_eager():
    ws = hi.batched_instances(9, 2, side_lo=20, side_hi=70)
    announce("graph replay")
    states, grids, common = _batch(ws, torch.float32)
    eager_states = [S.clone() for S in states]
    b = h.BatchedStepper(states, grids, common)
    e = h.BatchedStepper(eager_states, grids, common)
    b.capture(steps=1)
    for r in range(4):
        b.replay()
        e.step()
        torch.cuda.synchronize()
        # eager work of the program between replays
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        for q in range(len(ws)):
            assert torch.equal(states[q], eager_states[q]), (r, q)
            assert torch.equal(b.ctrl(q)[:10], e.ctrl(q)[:10]), (r, q)
        del junk


def test_autotune_through_the_c_abi():
    """hweno_autotune times every (tile variant, grid) candidate on the instances it
    is given and returns the fastest: times are finite and positive, the choice is
    their minimum, the grid sizes are the documented candidates (resident capacity,
    2 and 4 workgroups per compute unit, one per tile), and the tuned instances have
    advanced by the steps it took (2 variants x 4 candidates x (1 + trials)).  The
    Python wrapper runs it on clones, leaving the batch untouched, and the stepper
    then steps with the chosen configuration exactly as per-instance steps do."""
    import ctypes
    ws = [hi.euler2d_quadrants(70, 41, 1), hi.euler2d_random_smooth(33, 90, 2),
          hi.euler2d_quadrants(128, 128, 3, bc=hi.PERIODIC)]
    announce("autotune C ABI")
    states, grids, common = _batch(ws, torch.float32)
    b = h.BatchedStepper(states, grids, common)
    before = [S.clone() for S in states]
    maps = (ctypes.c_void_p * 2)(*[m.data_ptr() for m in b.maps])
    totals = (ctypes.c_int32 * 2)(*b.total_tiles)
    times = (ctypes.c_double * 8)()
    sizes = (ctypes.c_int32 * 8)()
    v, blk = ctypes.c_int32(-1), ctypes.c_int32(-1)
    trials = 2
    rc = h.lib().hweno_autotune(ctypes.byref(b._c), b.desc.data_ptr(), maps, b.n, totals, trials,
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                ctypes.byref(v), ctypes.byref(blk), times, sizes)
    assert rc == 0, h.lib().hweno_last_error().decode()
    t = list(times)
    assert all(np.isfinite(x) and x > 0 for x in t)
    k = int(np.argmin(t))
    assert (v.value, blk.value) == (k // 4, sizes[k])
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for var in range(2):
        tot = b.total_tiles[var]
        got = [sizes[var * 4 + c] for c in range(4)]
        assert got[1:] == [min(2 * cus, tot), min(4 * cus, tot), tot]
        assert 1 <= got[0] <= tot
    # the instances it tuned on took 2 x 4 x (1 + trials) steps
    steps = [int(b.ctrl(q)[9]) for q in range(b.n)]
    assert steps == [2 * 4 * (1 + trials)] * b.n
    # the wrapper: clones only, cached, and the chosen configuration steps correctly
    states2 = [S.clone() for S in before]
    b2 = h.BatchedStepper(states2, grids, common)
    h.hweno._AUTOTUNE_CACHE.clear()
    best, res = h.autotune_batched(b2)
    assert best in res and (b2.variant, b2.blocks) == best
    assert all(torch.equal(x, y) for x, y in zip(states2, before))
    assert h.autotune_batched(b2) == (best, None)
    b2.step()
    ref, _ = _individual(ws, torch.float32)
    for q in range(len(ws)):
        assert torch.equal(states2[q], ref[q]), q


def test_batched_full_config_256_instances():
    """The configured batch: 256 instances, sides ~ U{64..512}, FP32, autotuned, for the
    configured 100 steps (each instance with its own time steps, the steps captured in a
    graph and replayed as the bench runs them): every instance admissible, and eight
    sampled instances bitwise equal to their own single-grid runs of 100 steps."""
    ws = hi.batched_instances(256, 0)
    announce("256 instances, 100 steps")
    states, grids, common = _batch(ws, torch.float32)
    b = h.BatchedStepper(states, grids, common)
    best, res = h.autotune_batched(b)
    assert best in res
    b.capture(steps=1)
    for _ in range(100):
        b.replay()
    torch.cuda.synchronize()
    assert all(s == 0 for s in b.statuses())
    rng = np.random.default_rng(1)
    for q in sorted(rng.choice(256, size=8, replace=False)):
        ref, ctrls = _individual([ws[q]], torch.float32, steps=100)
        assert torch.equal(states[q], ref[0]), q
        assert torch.equal(b.ctrl(q)[:10], ctrls[0][:10]), q
