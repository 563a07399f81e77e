#!/usr/bin/env python
"""Benchmark of the L-HWENO hot path on one MI355X: 2D Euler cell-stage updates/s.

Workload: 2D Euler (gamma 1.4) on [0,1]^2 at 4096 x 4096, seed-0 four-quadrant
piecewise-constant data (rho ~ U[0.1,2], u,v ~ U[-1,1], p ~ U[0.1,2]),
outflow boundaries, CFL 0.6, characteristic HWENO with the limiter, 12 fields
(U, U_x, U_y).  One "step" is one SSP-RK3 step (three fused stage kernels plus
the wave-speed reduction) with the time step computed on the device.

Prints ONE JSON line.  value = cells * 3 stages * steps / wall time of the
timed region (inputs resident in HBM).  The roofline object is for the
dominant kernel (the fused stage kernel), timed with HIP events around each of
its launches on the stream it runs on.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic floating-point work of one 2D Euler cell-stage (characteristic-wise
# with the limiter), counted per step of the method: pointwise physics
# ~85, per direction Roe average, eigenvectors and projections ~660, eight
# nonlinear reconstructions ~760, linear and mixed fluxes ~160, flux differences
# ~60, limiter ~510, Runge-Kutta combination ~36 -- about 3.8k.  This count sets
# `achieved` and `frac` of the roofline object.
FLOP_PER_CELL_STAGE = 3800.0
# The same work counted term by term on the formulation the kernel evaluates
# (+, -, *, /, sqrt, |.| each 1, fused multiply-add 2): two interfaces of ~1740,
# flux differences 72, limiter 8 x ~64, Runge-Kutta ~48, wave speeds ~15.
FLOP_PER_CELL_STAGE_DERIVED = 4130.0

# MI355X published peaks (dense vector FP64 / FP32, HBM3E)
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
PEAK_HBM_GBS = 8000.0

# Compulsory HBM bytes per cell-stage of the fused kernel (fields of 8 / 4 B):
# stage 1 reads S^n (12) and writes S1 (12) + limited base derivatives (8);
# stages 2, 3 read S_k (12), U^n (4), base (8) and write 12  -> 104 / 3 fields.
FIELDS_PER_CELL_STAGE = 104.0 / 3.0
# The compulsory count when the base derivatives are recomputed instead of
# stored: stage 1 reads 12 and writes 12, stages 2, 3 read 12 + 12 and write
# 12 -> 32 fields (256 B FP64, 128 B FP32).
FIELDS_PER_CELL_STAGE_SCOPE = 32.0

# HBM traffic of one stage-kernel launch from rocprofv3 --pmc FETCH_SIZE /
# WRITE_SIZE, scaled by a copy-kernel calibration, keyed by the hash of the 2D
# Euler stage kernels' machine code it was measured on (kernel_sha; other code
# reports null).
MEASURED_TRAFFIC = {
    # profiles/k_stage_euler2d_4096_f64_hbm_bytes.md, profiles/k_stage_euler2d_4096_f32_hbm_bytes.md
    ("cd5b3fb9f97aabc9", "f64", 4096): 5.0817e+09,
    ("cd5b3fb9f97aabc9", "f32", 4096): 2.6213e+09,
}

# VALU wave-instructions issued by one stage-kernel launch (rocprofv3 --pmc
# SQ_INSTS_VALU, average of the three stages), keyed like MEASURED_TRAFFIC.
MEASURED_VALU_WAVE_INSTR = {
    # profiles/k_stage_euler2d_4096_sq_counters.md
    ("cd5b3fb9f97aabc9", "f64", 4096): 8.950e8,
    ("cd5b3fb9f97aabc9", "f32", 4096): 8.624e8,
}
# Floating-point operations per FP64 cell-stage that the SQ counters of the same
# device code count (SQ_INSTS_VALU_{ADD,MUL,TRANS}_F64 + 2 x FMA over cells x
# stages), keyed like MEASURED_TRAFFIC.
MEASURED_FLOP_PER_CELL_STAGE = {
    # profiles/k_stage_euler2d_4096_sq_counters.md
    ("cd5b3fb9f97aabc9", "f64", 4096): 4393.0,
}
# VALU issue peak of the chip in lane-instructions/s: 256 CUs x 4 SIMDs x 2.4 GHz
# x 16 lanes per cycle for FP64, x 32 for FP32 (the FP32 vector peak of 157.3
# TFLOP/s is twice the FP64 one; the FP32 stage kernel, which has no packed
# instructions, issues above the 16-lane rate).
PEAK_VALU_LANE_INSTR = {"f64": 256 * 4 * 16 * 2.4e9, "f32": 256 * 4 * 32 * 2.4e9}


# FP32 flops (SQ_INSTS_VALU_FLOPS_FP32 x 64) and VALU wave-instructions per launch of the
# discrete-adjoint kernel at 512^2 (profiles/k_adjoint_euler2d_512_f32_sq_counters.md),
# keyed by the hash of the k_adjoint kernels' machine code
ADJOINT_PREFIX = "_ZN5hweno9k_adjointI"
MEASURED_ADJOINT = {
    ("2ec0cebfd3b86215", "f32", 512): {"flop": 5.712e7 * 64, "valu_wave_instr": 4.667e7},
}


# the fused stage kernels of 2D Euler, FP64 and FP32: the code the measured figures describe
STAGE_2D_EULER = ("_ZN5hweno7k_stageIdLi2ELi2E", "_ZN5hweno7k_stageIfLi2ELi2E")


def kernel_sha(prefix=STAGE_2D_EULER) -> str:
    """sha256[:16] of the machine code of the kernels whose mangled names start with
    `prefix` (a string or a tuple of them; default: the 2D Euler fused stage kernels
    k_stage in FP64 and FP32) in the gfx950 code object that libhweno.so embeds.  It
    changes with those kernels' code and with nothing else, so a traffic or counter
    figure measured for one build stays attached to exactly the code it was measured on,
    across changes to other kernels."""
    prefixes = (prefix,) if isinstance(prefix, str) else tuple(prefix)
    import struct
    from paper_2207_05258_amd import hweno as hw
    with open(hw.LIB_PATH, "rb") as fh:
        b = fh.read()

    def sections(elf):
        shoff = struct.unpack_from("<Q", elf, 0x28)[0]
        shentsize, shnum, shstrndx = struct.unpack_from("<HHH", elf, 0x3A)
        secs = [struct.unpack_from("<IIQQQQIIQQ", elf, shoff + i * shentsize) for i in range(shnum)]
        names = secs[shstrndx]
        strtab = elf[names[4]:names[4] + names[5]]
        return [(strtab[x[0]:strtab.index(b"\0", x[0])], x) for x in secs]

    fatbin = next((elf_sec for n, elf_sec in sections(b) if n == b".hip_fatbin"), None)
    if fatbin is None:
        return "unknown"
    fb = b[fatbin[4]:fatbin[4] + fatbin[5]]
    if not fb.startswith(b"__CLANG_OFFLOAD_BUNDLE__"):
        return "unknown"
    n, p = struct.unpack_from("<Q", fb, 24)[0], 32
    code = None
    for _ in range(n):
        off, size, tl = struct.unpack_from("<QQQ", fb, p)
        triple = fb[p + 24:p + 24 + tl]
        p += 24 + tl
        if triple.endswith(b"gfx950"):
            code = fb[off:off + size]
    if code is None or not code.startswith(b"\x7fELF"):
        return "unknown"
    secs = sections(code)
    symtab = next(x for nm, x in secs if nm == b".symtab")
    strtab = code[secs[symtab[6]][1][4]:][:secs[symtab[6]][1][5]]
    h = hashlib.sha256()
    found = []
    for i in range(symtab[5] // 24):
        st_name, st_info, _o, st_shndx, st_value, st_size = struct.unpack_from(
            "<IBBHQQ", code, symtab[4] + 24 * i)
        name = strtab[st_name:strtab.index(b"\0", st_name)]
        if (st_info & 0xF) == 2 and st_size > 0 and any(name.startswith(q.encode()) for q in prefixes):
            sec = secs[st_shndx][1]
            off = sec[4] + (st_value - sec[3])
            found.append((name, code[off:off + st_size]))
    for name, body in sorted(found):
        h.update(name)
        h.update(body)
    return h.hexdigest()[:16] if found else "unknown"


def cpu_baseline(n: int = 1024, strip: int = 1024, c2_steps: int = 1000):
    """The CPU oracle, as it stands (float64, torch CPU), timed on the host:
    one SSP-RK3 step of the n x n four-quadrant workload with all host threads;
    the same step on `strip` rows through the middle of that grid (the whole grid
    by default) with one thread; and the first `c2_steps` steps of the 1D Euler
    piecewise-constant run (N = 4000, T = 0.2) with one thread (the faster setting
    for 4000 cells: thread start-up dominates small tensors)."""
    import torch

    import hweno_inputs as hi
    from oracle import hweno_ref as o

    w = hi.euler2d_quadrants(n, n, 0)
    prob = o.problem_from_workload(w)
    S = o.as_tensor(w.S)
    cores = torch.get_num_threads()
    t0 = time.perf_counter()
    o.rk3_step(S, prob)
    dt_all = time.perf_counter() - t0
    j0 = (n - strip) // 2
    Ss = S[:, j0:j0 + strip, :].contiguous()
    torch.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        o.rk3_step(Ss, prob)
        dt_one = time.perf_counter() - t0
        w1 = hi.euler1d_piecewise(4000, 0)
        p1 = o.problem_from_workload(w1)
        S1 = o.as_tensor(w1.S)
        t = 0.0
        steps = 0
        t0 = time.perf_counter()
        while steps < c2_steps and t < 0.2:
            a0 = o.max_speeds(S1, p1)
            dt = min(o.cfl_dt(a0, p1), 0.2 - t)
            S1, _, _ = o.rk3_step(S1, p1, dt, [a0, None, None], t)
            t += dt
            steps += 1
        dt_c2 = time.perf_counter() - t0
    finally:
        torch.set_num_threads(cores)
    return {"value": n * n * 3 / dt_all, "unit": "cell-stage updates/s",
            "cores": cores, "kind": "oracle",
            "sample": f"one SSP-RK3 step (3 cell-stages per cell) of the four-quadrant 2D Euler "
                      f"workload at {n}x{n} in float64 (torch CPU, {cores} threads), {dt_all:.1f} s",
            "single_thread": {"value": n * strip * 3 / dt_one, "cores": 1,
                              "sample": f"the same step on rows {j0}..{j0 + strip - 1} of the "
                                        f"{n}x{n} grid ({n}x{strip} cells), {dt_one:.1f} s"},
            "euler1d_4000": {"value": 4000 * 3 * steps / dt_c2, "cores": 1,
                             "unit": "cell-stage updates/s",
                             "sample": f"first {steps} steps (t = {t:.3e} of 0.2) of the 1D Euler "
                                       f"piecewise-constant run, N = 4000, seed 0, "
                                       f"{dt_c2:.1f} s"}}


def run_gpu(n: int, dtype_name: str, steps: int, warmup: int, ny: int = 0):
    """The four-quadrant workload on an n x n grid (n x ny when ny is given)."""
    import torch

    import hweno_inputs as hi
    import paper_2207_05258_amd as h
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    ny = ny or n
    w = hi.euler2d_quadrants(n, ny, 0)
    S = torch.as_tensor(w.S).to(dtype).cuda().contiguous()
    del w
    prob = h.Problem(dim=2, nx=n, ny=ny, physics="euler", dtype=dtype, dx=1.0 / n, dy=1.0 / ny,
                     bc_x=h.OUTFLOW, bc_y=h.OUTFLOW)
    st = h.Stepper(prob)
    st.steps(S, warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    h.timing_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    st.steps(S, steps)      # one call: each step's stage-1 speeds come from the step before
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, stage_ms = h.timing_end()
    ev_ms = e0.elapsed_time(e1)
    status = st.status
    ok = status == 0 and bool(torch.isfinite(S).all())
    cells = n * ny
    rate = cells * 3 * steps / wall
    per_launch_s = stage_ms / 1e3 / max(launches, 1)
    flops = FLOP_PER_CELL_STAGE * cells
    achieved = flops / per_launch_s / 1e12
    achieved_derived = FLOP_PER_CELL_STAGE_DERIVED * cells / per_launch_s / 1e12
    byt = FIELDS_PER_CELL_STAGE * cells * (8 if dtype_name == "f64" else 4)
    return {
        "rate": rate, "wall_s": wall, "event_ms": ev_ms, "ms_per_step": wall * 1e3 / steps,
        "stage_launches": launches, "stage_ms_avg": per_launch_s * 1e3,
        "achieved_tflops": achieved, "achieved_tflops_derived": achieved_derived,
        "algorithmic_hbm_gbs": byt / per_launch_s / 1e9,
        "scope_hbm_gbs": FIELDS_PER_CELL_STAGE_SCOPE * cells * (8 if dtype_name == "f64" else 4)
        / per_launch_s / 1e9,
        "t": st.t, "status": status, "finite_ok": ok,
    }


def run_batched(steps: int, warmup: int, n_inst: int = 256, seed: int = 0):
    """256 uneven 2D Euler instances (sides ~ U{64..512}), FP32, autotuned tile
    variant and grid, one hipGraph per step replayed ``steps`` times."""
    import torch

    import hweno_inputs as hi
    import paper_2207_05258_amd as h
    ws = hi.batched_instances(n_inst, seed)
    states = [torch.as_tensor(w.S).to(torch.float32).cuda().contiguous() for w in ws]
    grids = [dict(dx=w.dx, dy=w.dy, bc_x=w.bc_x, bc_y=w.bc_y) for w in ws]
    del ws
    common = h.Problem(dim=2, nx=1, ny=1, physics="euler", dtype=torch.float32)
    b = h.BatchedStepper(states, grids, common)
    best, _ = h.autotune_batched(b)
    for _ in range(warmup):
        b.step()
    b.capture(steps=1)
    torch.cuda.synchronize()
    h.timing_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, stage_ms = h.timing_end()
    bad = sum(1 for st in b.statuses() if st)
    return {"value": b.cells * 3 * steps / wall, "unit": "cell-stage updates/s", "dtype": "f32",
            "instances": n_inst, "cells": b.cells, "variant": best[0], "blocks": best[1],
            "steps": steps, "ms_per_step": wall * 1e3 / steps, "failed_instances": bad,
            "graph": "one hipGraph per step (speeds, 3 persistent stages, time update)"}


def run_small(n: int = 4000, steps: int = 200):
    """A 1D Euler grid of n cells (piecewise-constant data, periodic, FP64), where a step
    is a few microseconds of GPU work: eager single-step calls, one multi-step call
    (no separate speed pass after the first step), and those single steps captured
    in one graph and replayed."""
    import torch

    import hweno_inputs as hi
    import paper_2207_05258_amd as h
    w = hi.euler1d_piecewise(n, 0)
    prob = h.Problem(dim=1, nx=n, ny=1, physics="euler", dtype=torch.float64, dx=w.dx,
                     bc_x=w.bc_x)
    S = torch.as_tensor(w.S).cuda().contiguous()
    st = h.Stepper(prob)
    for _ in range(5):
        st.step(S)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.step(S)
    torch.cuda.synchronize()
    eager = time.perf_counter() - t0
    t0 = time.perf_counter()
    st.steps(S, steps)
    torch.cuda.synchronize()
    multi = time.perf_counter() - t0
    st.capture(S, steps=steps)
    st.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.replay()
    torch.cuda.synchronize()
    graph = time.perf_counter() - t0
    return {"workload": f"1D Euler, {n} cells, FP64", "steps": steps,
            "eager_us_per_step": eager * 1e6 / steps, "multi_step_call_us_per_step": multi * 1e6 / steps,
            "graph_us_per_step": graph * 1e6 / steps,
            "graph_value": n * 3 * steps / graph, "unit": "cell-stage updates/s",
            "status": st.status}


def _time_to_solution(w, max_steps: int = 0, **kw):
    """Whole run of a 2D Euler workload with edge-described sides to its T in FP64:
    device-side time steps in multi-step calls of 256, the last one clipped to T.  A
    warm-up of a few steps on a copy first; the time covers the whole run.  With
    max_steps > 0 only that many steps are taken (for profiling runs)."""
    import torch

    import paper_2207_05258_amd as h
    nx, ny = w.nx, w.ny
    T = w.info["t_end"]
    edges = tuple(h.Edge(kind=tuple(e[0]), split=tuple(e[1]), state=(tuple(e[2][0]), tuple(e[2][1])))
                  for e in w.edges)
    prob = h.Problem(dim=2, nx=nx, ny=ny, physics="euler", dtype=torch.float64, dx=w.dx, dy=w.dy,
                     bc_x=w.bc_x, bc_y=w.bc_y, edges=edges,
                     obstacle=None if w.obstacle is None else tuple(w.obstacle), **kw)
    S = torch.as_tensor(w.S).cuda().contiguous()
    h.Stepper(prob).steps(S.clone(), 4)
    torch.cuda.synchronize()
    st = h.Stepper(prob)
    t0 = time.perf_counter()
    chunk = 256 if max_steps <= 0 else min(256, max_steps)
    taken = 0
    while st.t < T * (1 - 1e-13) and (max_steps <= 0 or taken < max_steps):
        st.steps(S, chunk, t_end=T)
        taken += chunk
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps = int(st.ctrl[9])
    return {"steps": steps, "seconds": wall, "value": 3.0 * steps * nx * ny / wall,
            "unit": "cell-stage updates/s", "t": st.t, "status": st.status & ~h.hweno.ST_SKIPPED}


def run_double_mach(nx: int = 1920, ny: int = 480, max_steps: int = 0):
    """Double Mach reflection (Example 3.11) on [0, 4] x [0, 1] to T = 0.2: post-shock
    inflow, a wall from x = 1/6 on the bottom, the exact shock motion on the top."""
    import hweno_inputs as hi
    r = _time_to_solution(hi.double_mach(nx, ny), max_steps)
    return {"workload": f"double Mach reflection (Example 3.11), {nx}x{ny}, T = 0.2, FP64", **r}


def run_forward_step(nx: int = 960, ny: int = 320, max_steps: int = 0):
    """Forward-facing step (Example 3.12) at the paper's 960 x 320 cells to T = 4, with the
    limiter on characteristic fields (with the component-wise limiter the pressure turns
    negative near t = 1.1)."""
    import hweno_inputs as hi
    r = _time_to_solution(hi.forward_step(nx, ny), max_steps, limiter_characteristic=True)
    return {"workload": f"forward-facing step (Example 3.12), {nx}x{ny}, T = 4, FP64, "
                        "characteristic limiter", **r}


def run_adjoint(n: int = 512, steps: int = 200, ckpt: int = 0, dtype_name: str = "f32"):
    """Differentiable rollout on a smooth periodic 2D Euler state, loss = 1/2 sum dx dy
    (rho_N - rho_target)^2.  ckpt = 0: the forward keeps every step's states in device
    memory and the backward runs the hand-written step adjoints only; ckpt > 0: a
    checkpoint every ckpt steps, segments recomputed (overlapped) in the backward."""
    import torch

    import hweno_inputs as hi
    import paper_2207_05258_amd as h
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    base, target = hi.adjoint_pair(n, 0)
    prob = h.Problem(dim=2, nx=n, ny=n, physics="euler", dtype=dtype, dx=base.dx, dy=base.dy)
    U0 = torch.as_tensor(base.S).to(dtype).cuda().contiguous()
    tgt = torch.as_tensor(target.S[0]).to(dtype).cuda()
    # warm-up: one whole rollout of the same size, so every kernel has run and the
    # caching allocator already holds the kept states (as in any training loop
    # after its first iteration)
    X = U0.clone().requires_grad_(True)
    S = h.Rollout.apply(X, prob, steps, ckpt, None)
    (0.5 * base.dx * base.dy * ((S[0] - tgt) ** 2).sum()).backward()
    del X, S
    torch.cuda.synchronize()
    X = U0.clone().requires_grad_(True)
    t0 = time.perf_counter()
    S = h.Rollout.apply(X, prob, steps, ckpt, None)
    loss = 0.5 * base.dx * base.dy * ((S[0] - tgt) ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd, bwd = t1 - t0, t2 - t1
    g = X.grad
    return {"grid": f"{n}x{n}", "dtype": dtype_name, "steps": steps,
            "checkpoint_every": ckpt if ckpt else "every step kept",
            "kept_bytes": h.rollout_bytes_kept(prob, steps) if ckpt == 0 else None,
            "forward_ms": fwd * 1e3, "backward_ms": bwd * 1e3, "backward_over_forward": bwd / fwd,
            "loss": float(loss.detach()),
            "grad_finite": bool(torch.isfinite(g).all()), "grad_norm_U": float(g[:4].norm())}


def adjoint_roofline(n: int = 512, steps: int = 20):
    """The discrete-adjoint kernel against the FP32 peaks: `steps` forward steps keeping
    their states, then their step adjoints newest first with the library's launch timer
    on (HIP events around every k_adjoint launch on its stream; the calls run on this
    thread, which the timer belongs to), and the counted flops and VALU instructions per
    launch of the same machine code (null for other code)."""
    import torch

    import hweno_inputs as hi
    import paper_2207_05258_amd as h
    base, _ = hi.adjoint_pair(n, 0)
    prob = h.Problem(dim=2, nx=n, ny=n, physics="euler", dtype=torch.float32, dx=base.dx, dy=base.dy)
    S = torch.as_tensor(base.S).float().cuda().contiguous()
    tapes = torch.zeros(steps, h.CTRL_LEN, dtype=torch.float64, device="cuda")
    inputs, steppers = [], []
    for q in range(steps):
        inputs.append(S.clone())
        steppers.append(h.Stepper(prob))
        steppers[-1].step(S, tape=tapes[q])
    lam = torch.randn(S.shape, generator=torch.Generator(device="cuda").manual_seed(0), device="cuda")
    ws = h.adjoint_workspace(prob)
    h.step_adjoint(prob, inputs[-1], steppers[-1], tapes[-1], lam.clone(), ws)   # warm-up
    torch.cuda.synchronize()
    h.timing_begin()
    for q in reversed(range(steps)):
        h.step_adjoint(prob, inputs[q], steppers[q], tapes[q], lam, ws)
    torch.cuda.synchronize()
    launches, ms = h.timing_end()
    sha = kernel_sha(ADJOINT_PREFIX)
    m = MEASURED_ADJOINT.get((sha, "f32", n))
    launch_ms = ms / launches if launches else None
    out = {"kernel": "k_adjoint (transposed stage operator and limiter)", "grid": f"{n}x{n}",
           "launches": launches, "launch_ms": None if launch_ms is None else round(launch_ms, 4),
           "bound": "alu", "peak": 157.3, "unit": "TFLOP/s", "achieved": None, "frac": None,
           "valu_issue": None, "kernel_sha": sha, "finite": bool(torch.isfinite(lam).all())}
    if m is not None and launch_ms:
        achieved = m["flop"] / (launch_ms * 1e-3) / 1e12
        out.update(achieved=round(achieved, 3), frac=round(achieved / 157.3, 4),
                   flop_per_launch=m["flop"],
                   valu_issue=round(m["valu_wave_instr"] * 64 / (launch_ms * 1e-3)
                                    / PEAK_VALU_LANE_INSTR["f32"], 4))
    return out


def summarize_pmc(root: str, match: str = "") -> str:
    """Markdown table of the mean value per dispatch of every rocprofv3 --pmc counter,
    per kernel, from the counter_collection.csv files under `root` (kernels whose
    name contains `match`).  Used to turn raw counter dumps into short summaries."""
    import csv
    import glob
    sums, counts, kernels, names = {}, {}, [], []
    for path in sorted(glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True)):
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                k, c = row.get("Kernel_Name", ""), row.get("Counter_Name", "")
                if match not in k:
                    continue
                key = (k, c)
                sums[key] = sums.get(key, 0.0) + float(row.get("Counter_Value", 0.0))
                counts[key] = counts.get(key, 0) + 1
                if k not in kernels:
                    kernels.append(k)
                if c not in names:
                    names.append(c)
    lines = ["| kernel | dispatches | " + " | ".join(names) + " |",
             "|---|---|" + "---|" * len(names)]
    for k in kernels:
        n = max(counts.get((k, c), 0) for c in names)
        vals = [f"{sums[(k, c)] / counts[(k, c)]:.4g}" if (k, c) in counts else "" for c in names]
        lines.append(f"| {k[:90]} | {n} | " + " | ".join(vals) + " |")
    return "\n".join(lines)


def summarize_trace(root: str, match: str = "k_stage<", last: int = 0) -> str:
    """Markdown summary of a rocprofv3 --kernel-trace --stats run under `root`: the
    kernel_stats.csv table, and from kernel_trace.csv the average duration of the last
    `last` dispatches whose name contains `match` (the timed region of a bench run:
    3 x steps stage launches), the GPU kernel time of every dispatch from the first of
    them on, and their launch shape."""
    import csv
    import glob
    out = []
    for path in sorted(glob.glob(os.path.join(root, "**", "*kernel_stats.csv"), recursive=True)):
        out += ["| kernel | calls | average ns | min ns | max ns | % of GPU time |",
                "|---|---|---|---|---|---|"]
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                out.append(f"| {row['Name'][:78]} | {row['Calls']} | {float(row['AverageNs']):.0f} | "
                           f"{float(row['MinNs']):.0f} | {float(row['MaxNs']):.0f} | "
                           f"{float(row['Percentage']):.2f} |")
    recs = []
    for path in sorted(glob.glob(os.path.join(root, "**", "*kernel_trace.csv"), recursive=True)):
        with open(path, newline="") as fh:
            recs += list(csv.DictReader(fh))
    recs.sort(key=lambda r: int(r["Start_Timestamp"]))
    sel = [i for i, r in enumerate(recs) if match in r["Kernel_Name"]]
    if last and len(sel) >= last:
        sel = sel[-last:]
        dur = [int(recs[i]["End_Timestamp"]) - int(recs[i]["Start_Timestamp"]) for i in sel]
        tail = recs[sel[0]:]
        busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in tail)
        span = max(int(r["End_Timestamp"]) for r in tail) - int(tail[0]["Start_Timestamp"])
        r0 = recs[sel[0]]

        def col(*names):
            return next((r0[n] for n in names if r0.get(n) not in (None, "")), "?")
        out += ["", f"Last {last} dispatches matching `{match}`: average duration "
                    f"{sum(dur) / len(dur) / 1e6:.4f} ms (min {min(dur) / 1e6:.4f}, max "
                    f"{max(dur) / 1e6:.4f}); GPU kernel time of all {len(tail)} dispatches from the "
                    f"first of them on: {busy / 1e6:.4f} ms, over a span of {span / 1e6:.4f} ms "
                    f"from the first start to the last end.",
                f"Launch shape: grid {col('Grid_Size', 'Grid_Size_X')} work-items in workgroups of "
                f"{col('Workgroup_Size', 'Workgroup_Size_X')}; LDS {col('LDS_Block_Size', 'Lds_Size')} B "
                f"per workgroup, scratch {col('Scratch_Size')} B per lane; the trace's VGPR "
                f"count field {col('VGPR_Count', 'Arch_VGPR_Count')}."]
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variant", action="store_true",
                    help="skip the secondary run in the other precision")
    ap.add_argument("--cpu-n", type=int, default=1024)
    ap.add_argument("--cpu-strip", type=int, default=1024,
                    help="rows of the one-thread oracle sample of the cpu-n grid")
    ap.add_argument("--cpu-c2-steps", type=int, default=1000,
                    help="steps of the 1D Euler N = 4000 run timed on one thread")
    ap.add_argument("--no-1024", action="store_true", help="skip the 1024^2 rows")
    ap.add_argument("--no-shard", action="store_true",
                    help="skip the 4096x512 rows (one GPU's share of 4096^2 in 8 slabs)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-instances run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint rollout run")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the small-grid eager-versus-graph run")
    ap.add_argument("--no-double-mach", action="store_true",
                    help="skip the double Mach reflection and forward-step runs")
    ap.add_argument("--only", choices=["batched", "adjoint", "double_mach", "forward_step", "small"],
                    default=None,
                    help="run only this part and print its JSON object (for profiling)")
    ap.add_argument("--adjoint-steps", type=int, default=200)
    ap.add_argument("--summarize-pmc", metavar="DIR", default=None,
                    help="print a markdown table of the rocprofv3 counters under DIR and exit")
    ap.add_argument("--match", default="", help="kernel-name filter of --summarize-pmc")
    ap.add_argument("--summarize-trace", metavar="DIR", default=None,
                    help="print a markdown summary of the rocprofv3 kernel trace under DIR and exit")
    ap.add_argument("--trace-last", type=int, default=0,
                    help="with --summarize-trace: average the last this many matching dispatches")
    ap.add_argument("--edge-steps", type=int, default=0,
                    help="run only this many steps of the double Mach and forward-step legs "
                         "(0 = to their end times)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of 1 GiB (for scaling HBM byte counters) and exit")
    args = ap.parse_args()

    if args.summarize_pmc:
        print(summarize_pmc(args.summarize_pmc, args.match))
        return
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace, args.match or "k_stage<", args.trace_last))
        return

    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8}))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the L-HWENO path runs on one GPU; multi-GPU runs are not supported "
              "(sharding a grid needs a halo exchange and a speed all-reduce per stage, which "
              "are not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU available", file=sys.stderr)
        sys.exit(2)
    import paper_2207_05258_amd as h
    h.lib()

    if args.only == "batched":
        print(json.dumps(run_batched(args.steps, max(args.warmup, 1))), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps(run_adjoint(steps=args.adjoint_steps)), flush=True)
        return
    if args.only == "small":
        print(json.dumps(run_small()), flush=True)
        return
    if args.only == "double_mach":
        print(json.dumps(run_double_mach(max_steps=args.edge_steps)), flush=True)
        return
    if args.only == "forward_step":
        print(json.dumps(run_forward_step(max_steps=args.edge_steps)), flush=True)
        return

    main_run = run_gpu(args.n, args.dtype, args.steps, args.warmup)
    print(f"# {args.dtype} {args.n}^2: {main_run['rate']:.4e} cell-stage/s, stage kernel "
          f"{main_run['stage_ms_avg']:.3f} ms, {main_run['achieved_tflops']:.2f} TFLOP/s",
          file=sys.stderr, flush=True)
    variant = None
    if not args.no_variant:
        other = "f32" if args.dtype == "f64" else "f64"
        v = run_gpu(args.n, other, max(args.steps // 2, 1), 1)
        variant = {"dtype": other, "value": v["rate"], "ms_per_step": v["ms_per_step"],
                   "stage_ms_avg": v["stage_ms_avg"],
                   "roofline_frac": v["achieved_tflops"] / PEAK_TFLOPS[other],
                   "status": v["status"]}

    rows_1024 = None
    if not args.no_1024 and args.n != 1024:
        rows_1024 = {}
        for dt_name in ("f64", "f32"):
            r = run_gpu(1024, dt_name, args.steps, args.warmup)
            rows_1024[dt_name] = {"value": r["rate"], "ms_per_step": r["ms_per_step"],
                                  "stage_ms_avg": r["stage_ms_avg"],
                                  "roofline_frac": r["achieved_tflops"] / PEAK_TFLOPS[dt_name],
                                  "status": r["status"]}
        print(f"# 1024^2: f64 {rows_1024['f64']['value']:.4e}, f32 {rows_1024['f32']['value']:.4e} "
              "cell-stage/s", file=sys.stderr, flush=True)

    # one GPU's share of the 4096^2 grid split into eight slabs (section "more than
    # one GPU" of the design notes): the stage kernel at the shard's own shape,
    # its halo rows read from the local buffer; the exchange it would add per
    # stage is 2 sides x 2 rows x 4096 x 12 fields, priced at one xGMI link
    shard = None
    if not args.no_shard and args.n == 4096:
        shard = {"shape": "4096x512", "of": "4096x4096 in 8 slabs",
                 "halo_bytes_per_stage": {}, "halo_us_per_stage_at_153GBps": {}}
        for dt_name in ("f64", "f32"):
            r = run_gpu(4096, dt_name, args.steps, args.warmup, ny=512)
            shard[dt_name] = {"value": r["rate"], "ms_per_step": r["ms_per_step"],
                              "stage_ms_avg": r["stage_ms_avg"], "status": r["status"]}
            hb = 2 * 2 * 4096 * 12 * (8 if dt_name == "f64" else 4)
            shard["halo_bytes_per_stage"][dt_name] = hb
            shard["halo_us_per_stage_at_153GBps"][dt_name] = round(hb / 153e9 * 1e6, 2)
        print(f"# 8-way shard 4096x512: f64 {shard['f64']['value']:.4e}, f32 "
              f"{shard['f32']['value']:.4e} cell-stage/s", file=sys.stderr, flush=True)

    batched = None
    if not args.no_batched:
        batched = run_batched(args.steps, max(args.warmup, 1))
        single_f32 = (variant["value"] if variant and variant["dtype"] == "f32"
                      else (main_run["rate"] if args.dtype == "f32" else None))
        batched["ratio_vs_single_grid_f32"] = (batched["value"] / single_f32) if single_f32 else None
        print(f"# batched: {batched['value']:.4e} cell-stage/s "
              f"(ratio {batched['ratio_vs_single_grid_f32']})", file=sys.stderr, flush=True)

    adjoint = None
    if not args.no_adjoint:
        # the configured rollout checkpoints every 20 steps; the target is a backward
        # of at most 3x the forward.  The rollout that keeps every step's states runs
        # first: its 9 GB of kept states come from the caching allocator's own
        # warm-up allocation only when no other rollout has fragmented the cache.
        kept = run_adjoint(steps=args.adjoint_steps, ckpt=0)
        adjoint = run_adjoint(steps=args.adjoint_steps, ckpt=20)
        adjoint["target_backward_over_forward"] = 3.0
        adjoint["meets_target"] = adjoint["backward_over_forward"] <= 3.0
        adjoint["every_step_kept"] = kept
        adjoint["roofline"] = adjoint_roofline()
        print(f"# adjoint: backward/forward {adjoint['backward_over_forward']:.2f} (checkpoint every "
              f"20), {adjoint['every_step_kept']['backward_over_forward']:.2f} (every step kept)",
              file=sys.stderr, flush=True)

    dmr = None if args.no_double_mach else run_double_mach()
    fstep = None if args.no_double_mach else run_forward_step()
    if dmr is not None:
        print(f"# double Mach 1920x480 to T = 0.2: {dmr['steps']} steps in {dmr['seconds']:.2f} s; "
              f"forward step 960x320 to T = 4: {fstep['steps']} steps in {fstep['seconds']:.2f} s",
              file=sys.stderr, flush=True)

    small = None if args.no_small else run_small()
    if small is not None:
        print(f"# small grid: {small['eager_us_per_step']:.1f} us/step eager, "
              f"{small['graph_us_per_step']:.1f} us/step as one graph", file=sys.stderr, flush=True)

    sha = kernel_sha()
    traffic = MEASURED_TRAFFIC.get((sha, args.dtype, args.n))
    wave_instr = MEASURED_VALU_WAVE_INSTR.get((sha, args.dtype, args.n))
    valu = None
    if wave_instr is not None:
        rate = wave_instr * 64 / (main_run["stage_ms_avg"] * 1e-3)
        peak_issue = PEAK_VALU_LANE_INSTR[args.dtype]
        valu = {"lane_instr_per_s": float(f"{rate:.4g}"), "peak": peak_issue,
                "frac": round(rate / peak_issue, 4),
                "source": "SQ_INSTS_VALU per launch (rocprofv3) over the live launch time"}
    cells = args.n * args.n
    esize = 8 if args.dtype == "f64" else 4
    counted = MEASURED_FLOP_PER_CELL_STAGE.get((sha, args.dtype, args.n))
    per_launch_s = main_run["stage_ms_avg"] * 1e-3
    roofline = {
        "bound": "alu",
        "achieved": round(main_run["achieved_tflops"], 3),
        "peak": PEAK_TFLOPS[args.dtype],
        "unit": "TFLOP/s",
        "frac": round(main_run["achieved_tflops"] / PEAK_TFLOPS[args.dtype], 4),
        "traffic": traffic,
        "kernel": "k_stage (fused SSP-RK3 stage)",
        "flop_per_cell_stage": FLOP_PER_CELL_STAGE,
        "derived": {"flop_per_cell_stage": FLOP_PER_CELL_STAGE_DERIVED,
                    "achieved": round(main_run["achieved_tflops_derived"], 3),
                    "frac": round(main_run["achieved_tflops_derived"] / PEAK_TFLOPS[args.dtype], 4)},
        "counted": None if counted is None else {
            "flop_per_cell_stage": counted,
            "achieved": round(counted * cells / per_launch_s / 1e12, 3),
            "frac": round(counted * cells / per_launch_s / 1e12 / PEAK_TFLOPS[args.dtype], 4),
            "source": "SQ_INSTS_VALU_*_F64 counters of the same device code"},
        "hbm_bytes_per_cell_stage": 32 * esize,
        "algorithmic_hbm_GBps": round(main_run["scope_hbm_gbs"], 1),
        "hbm_frac": round(main_run["scope_hbm_gbs"] / PEAK_HBM_GBS, 4),
        "stored_base_hbm_GBps": round(main_run["algorithmic_hbm_gbs"], 1),
        "traffic_over_algorithmic": None if traffic is None else
        round(traffic / (32 * esize * cells), 3),
        "stage_launch_ms": round(main_run["stage_ms_avg"], 4),
        "valu_issue": valu,
    }
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_n, args.cpu_strip,
                                                          args.cpu_c2_steps)
    out = {
        # value: the cell-stage rate; the %HBM roofline is roofline.hbm_frac, and the
        # adjoint/forward time is adjoint.backward_over_forward
        "metric": "2D Euler HWENO cell-stage updates/s + %HBM roofline; adjoint/forward time",
        "value": main_run["rate"],
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"2D Euler four-quadrant Riemann data, {args.n}x{args.n}, outflow, "
                               f"CFL 0.6, characteristic HWENO + limiter, SSP-RK3, seed 0",
                   "nx": args.n, "ny": args.n, "fields": 12, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper_timings": "none published: the paper shows efficiency only as error-versus-CPU-time "
                         "figures, without numbers or stated hardware",
        "variant": variant,
        "c3_1024": rows_1024,
        "shard_8way": shard,
        "batched": batched,
        "adjoint": adjoint,
        "small_grid": small,
        "double_mach": dmr,
        "forward_step": fstep,
        "status_word": main_run["status"],
        "kernel_sha": sha,
    }
    print(json.dumps(out), flush=True)
    if not main_run["finite_ok"]:
        sys.exit(1)


if __name__ == "__main__":
    main()
