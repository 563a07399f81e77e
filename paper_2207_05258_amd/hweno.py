"""Thin Python binding of the C ABI in include/hweno.h.

Argument marshalling only: every step of the hot path runs in the HIP
library.  Arrays are torch tensors on the GPU; the current torch stream is
passed to every call.  There is no CPU fallback: if the library is missing
the calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import Optional, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhweno.so")

HWENO_OK = 0
CTRL_LEN = 16
ST_NONFINITE, ST_RHO, ST_PRESSURE, ST_SKIPPED = 1, 2, 4, 8

PHYSICS = {"linadv": 0, "burgers": 1, "euler": 2}
DTYPES = {torch.float32: 0, torch.float64: 1}
PERIODIC, OUTFLOW, REFLECT, EDGES = 0, 1, 2, 3
SEG_OUTFLOW, SEG_REFLECT, SEG_STATE = 0, 1, 2


class HwenoError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {_status_name(code)}: {detail}")
        self.code = code


class _CEdge(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32 * 2), ("split", ctypes.c_double * 3),
        ("state", (ctypes.c_double * 4) * 2),
    ]


@dataclass(frozen=True)
class Edge:
    """One side under bc EDGES (mirrors hweno_edge): ghost cells before the split
    split[0] + split[1] t + split[2] d along the side take segment 0, the others
    segment 1; kinds SEG_OUTFLOW / SEG_REFLECT / SEG_STATE (the conserved state
    of that segment, derivatives zero)."""

    kind: Tuple[int, int] = (SEG_OUTFLOW, SEG_OUTFLOW)
    split: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    state: Tuple[Tuple[float, ...], Tuple[float, ...]] = ((0.0,) * 4, (0.0,) * 4)


class _CProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("physics", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("characteristic", ctypes.c_int32), ("limiter_on", ctypes.c_int32),
        ("limiter_characteristic", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("gamma_gas", ctypes.c_double), ("adv_speed", ctypes.c_double * 2),
        ("lin_w", ctypes.c_double * 3), ("lim_w", ctypes.c_double * 3),
        ("eps", ctypes.c_double), ("cfl", ctypes.c_double),
        ("edges", _CEdge * 4),
        ("obstacle", ctypes.c_int32 * 2),
    ]


class _CInstance(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_void_p), ("ws", ctypes.c_void_p),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("dt_fixed", ctypes.c_double), ("t_end", ctypes.c_double),
        ("ws_bytes", ctypes.c_int64),
        ("off_s1", ctypes.c_int64), ("off_s2", ctypes.c_int64), ("off_base", ctypes.c_int64),
        ("tile_begin", ctypes.c_int32 * 2), ("n_tiles", ctypes.c_int32 * 2),
    ]


BATCH_VARIANTS = 2
_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libhweno.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2207_05258_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(_CProblem)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        sig = {
            "hweno_validate": ([P], ctypes.c_int),
            "hweno_workspace_bytes": ([P], ctypes.c_size_t),
            "hweno_alpha": ([P, vp, vp, vp], ctypes.c_int),
            "hweno_rhs": ([P, vp, vp, vp, ctypes.c_int32, vp], ctypes.c_int),
            "hweno_limit": ([P, vp, vp, vp], ctypes.c_int),
            "hweno_rk3_step": ([P, vp, vp, ctypes.c_size_t, ctypes.c_double, ctypes.c_double,
                                vp, vp, vp], ctypes.c_int),
            "hweno_rk3_steps": ([P, vp, vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_double, vp, vp], ctypes.c_int),
            "hweno_rk3_step_static": ([P, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp],
                                      ctypes.c_int),
            "hweno_adjoint_workspace_bytes": ([P], ctypes.c_size_t),
            "hweno_rhs_adjoint": ([P, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
            "hweno_rk3_step_adjoint": ([P, vp, vp, ctypes.c_size_t, vp, vp, vp, ctypes.c_size_t,
                                        vp], ctypes.c_int),
            "hweno_batch_prepare": ([P, ctypes.POINTER(_CInstance), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "hweno_batch_tile_map": ([ctypes.POINTER(_CInstance), ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.c_int32], ctypes.c_int),
            "hweno_rk3_step_batched": ([P, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, vp], ctypes.c_int),
            "hweno_autotune": ([P, vp, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, vp,
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                dp, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "hweno_timing_begin": ([ctypes.c_int32], ctypes.c_int),
            "hweno_timing_end": ([ctypes.POINTER(ctypes.c_int64), dp], ctypes.c_int),
            "hweno_status_string": ([ctypes.c_int32], ctypes.c_char_p),
            "hweno_last_error": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _status_name(code: int) -> str:
    return lib().hweno_status_string(code).decode()


def _check(code: int, where: str):
    if code != HWENO_OK:
        raise HwenoError(code, where, lib().hweno_last_error().decode())


@dataclass
class Problem:
    """Parameters of a discretised problem (mirrors hweno_problem)."""

    dim: int
    nx: int
    ny: int = 1
    physics: str = "euler"
    dtype: torch.dtype = torch.float64
    dx: float = 1.0
    dy: float = 1.0
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    characteristic: bool = True
    limiter_on: bool = True
    limiter_characteristic: bool = False
    gamma_gas: float = 1.4
    adv_speed: Tuple[float, float] = (1.0, 1.0)
    lin_w: Tuple[float, float, float] = (0.98, 0.01, 0.01)
    lim_w: Tuple[float, float, float] = (0.98, 0.01, 0.01)
    eps: float = 1e-6
    cfl: float = 0.6
    # sides x_lo, x_hi, y_lo, y_hi, read where bc_x / bc_y is EDGES
    edges: Optional[Tuple[Edge, Edge, Edge, Edge]] = None
    # (i_s, j_s): cells i >= i_s, j < j_s are solid (a step against the bottom-right corner)
    obstacle: Optional[Tuple[int, int]] = None

    @property
    def m(self) -> int:
        if self.physics == "euler":
            return 3 if self.dim == 1 else 4
        return 1

    @property
    def nf(self) -> int:
        return self.m * (1 + self.dim)

    def shape(self) -> Tuple[int, int, int]:
        return (self.nf, self.ny if self.dim == 2 else 1, self.nx)

    def c(self) -> _CProblem:
        p = _CProblem()
        p.dim, p.nx, p.ny = self.dim, self.nx, (self.ny if self.dim == 2 else 1)
        p.physics = PHYSICS[self.physics]
        p.dtype = DTYPES[self.dtype]
        p.bc_x, p.bc_y = int(self.bc_x), int(self.bc_y)
        p.characteristic = int(bool(self.characteristic))
        p.limiter_on = int(bool(self.limiter_on))
        p.limiter_characteristic = int(bool(self.limiter_characteristic))
        p.dx, p.dy = float(self.dx), float(self.dy)
        p.gamma_gas = float(self.gamma_gas)
        p.adv_speed[:] = [float(x) for x in self.adv_speed]
        p.lin_w[:] = [float(x) for x in self.lin_w]
        p.lim_w[:] = [float(x) for x in self.lim_w]
        p.eps, p.cfl = float(self.eps), float(self.cfl)
        for e, edge in enumerate(self.edges or ()):
            p.edges[e].kind[:] = [int(x) for x in edge.kind]
            p.edges[e].split[:] = [float(x) for x in edge.split]
            for sgm in range(2):
                p.edges[e].state[sgm][:] = [float(x) for x in edge.state[sgm]]
        if self.obstacle is not None:
            p.obstacle[:] = [int(x) for x in self.obstacle]
        return p


def problem_for(S: torch.Tensor, dim: int, physics: str, dx: float, dy: float = 1.0,
                **kw) -> Problem:
    nf, ny, nx = S.shape
    return Problem(dim=dim, nx=nx, ny=ny, physics=physics, dtype=S.dtype, dx=dx, dy=dy, **kw)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _speeds(alpha_, device) -> torch.Tensor:
    """Wave speeds as a float64 device tensor; float32 input is refused (it would round them)."""
    if not torch.is_tensor(alpha_):
        alpha_ = torch.tensor([float(x) for x in alpha_], dtype=torch.float64)
    if alpha_.dtype != torch.float64:
        raise ValueError("wave speeds must be float64 (got %s)" % alpha_.dtype)
    return alpha_.to(device=device).contiguous()


def _require(t: torch.Tensor, prob: Problem, nfields: int, what: str):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a GPU tensor")
    if t.dtype != prob.dtype:
        raise ValueError(f"{what} dtype {t.dtype} does not match the problem's {prob.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    ny = prob.ny if prob.dim == 2 else 1
    if t.numel() != nfields * ny * prob.nx:
        raise ValueError(f"{what} has {t.numel()} values, expected {nfields}x{ny}x{prob.nx}")


def validate(prob: Problem):
    _check(lib().hweno_validate(ctypes.byref(prob.c())), "hweno_validate")


def workspace_bytes(prob: Problem) -> int:
    return int(lib().hweno_workspace_bytes(ctypes.byref(prob.c())))


def alpha(S: torch.Tensor, prob: Problem, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Global Lax-Friedrichs speeds (alpha_x, alpha_y) of the splitting in Section 2.1,
    as a float64 device tensor."""
    _require(S, prob, prob.nf, "state")
    a = out if out is not None else torch.zeros(2, dtype=torch.float64, device=S.device)
    _check(lib().hweno_alpha(ctypes.byref(prob.c()), _ptr(S), _ptr(a), _stream()), "hweno_alpha")
    return a


def rhs(S: torch.Tensor, prob: Problem, alpha_: Optional[torch.Tensor] = None,
        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Semi-discrete right-hand side L(S) of eqs. (odeH) / (ode2H): flux differences of the
    nonlinear HWENO flux (Section 2.1, characteristic-wise for Euler per Remarks 2.1-2.2)
    and of the linear derivative and mixed fluxes; speeds computed from S unless given."""
    _require(S, prob, prob.nf, "state")
    L = out if out is not None else torch.empty_like(S)
    if alpha_ is None:
        a = torch.zeros(2, dtype=torch.float64, device=S.device)
        compute = 1
    else:
        a = _speeds(alpha_, S.device)
        compute = 0
    _check(lib().hweno_rhs(ctypes.byref(prob.c()), _ptr(S), _ptr(L), _ptr(a), compute, _stream()),
           "hweno_rhs")
    return L


def limit(S: torch.Tensor, prob: Problem, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Limited derivatives of the HWENO limiter (Section 2.2): U_x along x [, U_y along y],
    m * dim fields."""
    _require(S, prob, prob.nf, "state")
    ny = prob.ny if prob.dim == 2 else 1
    D = out if out is not None else torch.empty((prob.m * prob.dim, ny, prob.nx),
                                                dtype=S.dtype, device=S.device)
    _check(lib().hweno_limit(ctypes.byref(prob.c()), _ptr(S), _ptr(D), _stream()), "hweno_limit")
    return D


class Stepper:
    """Owns the device workspace of hweno_rk3_step for one problem.

    ``ctrl`` (float64[16] on the device) is the step control block: stage
    speeds, last dt, simulated time t, status word, step count.
    """

    def __init__(self, prob: Problem, device="cuda", t0: float = 0.0):
        validate(prob)
        self.prob = prob
        self._c = prob.c()
        self.nbytes = max(workspace_bytes(prob), 256)
        # Only the control block must start at zero: every step writes the stage
        # states before reading them.
        self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.ws.data_ptr()) % 256
        self.ws = self.ws[off:off + self.nbytes]
        self.ctrl = self.ws[:CTRL_LEN * 8].view(torch.float64)
        self.ctrl.zero_()
        self.ctrl[7] = t0

    def step(self, S: torch.Tensor, dt: Optional[float] = None, t_end: Optional[float] = None,
             tape: Optional[torch.Tensor] = None, replay: Optional[torch.Tensor] = None):
        """One SSP-RK3 step of S in place (Section 2.2: the limited derivatives enter the
        stage combinations only); device-side CFL dt unless ``dt`` is given."""
        _require(S, self.prob, self.prob.nf, "state")
        for t, name in ((tape, "tape"), (replay, "replay")):
            if t is not None and (t.dtype != torch.float64 or t.numel() < CTRL_LEN or not t.is_cuda):
                raise ValueError(f"{name} must be a float64 GPU tensor of >= {CTRL_LEN} values")
        _check(lib().hweno_rk3_step(ctypes.byref(self._c), _ptr(S), _ptr(self.ws), self.nbytes,
                                    float(dt or 0.0), float(t_end or 0.0), _ptr(tape),
                                    _ptr(replay), _stream()), "hweno_rk3_step")
        return S

    def steps(self, S: torch.Tensor, n: int, dt: Optional[float] = None,
              t_end: Optional[float] = None, tapes: Optional[torch.Tensor] = None):
        """``n`` steps of S in place in one call (hweno_rk3_steps): each step's stage-1
        speeds are folded by the previous step's last stage; bitwise the same as ``n``
        calls of ``step``.  ``tapes``: float64 GPU tensor [n, CTRL_LEN] or None."""
        _require(S, self.prob, self.prob.nf, "state")
        if tapes is not None and (tapes.dtype != torch.float64 or not tapes.is_cuda or
                                  tapes.numel() < n * CTRL_LEN or not tapes.is_contiguous()):
            raise ValueError(f"tapes must be a contiguous float64 GPU tensor of >= {n} x {CTRL_LEN}")
        _check(lib().hweno_rk3_steps(ctypes.byref(self._c), _ptr(S), _ptr(self.ws), self.nbytes,
                                     int(n), float(dt or 0.0), float(t_end or 0.0), _ptr(tapes),
                                     _stream()), "hweno_rk3_steps")
        return S

    def capture(self, S: torch.Tensor, steps: int = 1, dt: Optional[float] = None,
                t_end: Optional[float] = None) -> "torch.cuda.CUDAGraph":
        """Capture ``steps`` steps of S (in place, device-side dt unless ``dt``) in one
        graph; ``replay()`` then advances S by that many steps with one launch from
        the host.  S and this stepper's workspace must stay alive while the graph is
        used.  For small grids, where a step is a few microseconds of GPU work, the
        per-step host launch cost is what the graph removes."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for _ in range(steps):
                    self.step(S, dt=dt, t_end=t_end)
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    @classmethod
    def _over(cls, prob: Problem, c: _CProblem, ws: torch.Tensor, nbytes: int) -> "Stepper":
        """A stepper over a caller-provided, 256-byte aligned workspace whose control
        block the caller has initialised (no checks, no allocation)."""
        self = cls.__new__(cls)
        self.prob, self._c, self.nbytes, self.ws = prob, c, nbytes, ws
        self.ctrl = ws[:CTRL_LEN * 8].view(torch.float64)
        return self

    @property
    def t(self) -> float:
        return float(self.ctrl[7])

    @property
    def status(self) -> int:
        return int(self.ctrl[8:9].view(torch.int64).item())

    @property
    def last_dt(self) -> float:
        return float(self.ctrl[6])


def timing_begin(enable: bool = True):
    """Start timing every Runge-Kutta stage-kernel launch (HIP events on its stream)."""
    _check(lib().hweno_timing_begin(1 if enable else 0), "hweno_timing_begin")


def timing_end() -> Tuple[int, float]:
    """Stop timing; returns (number of stage launches, their total milliseconds)."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(lib().hweno_timing_end(ctypes.byref(n), ctypes.byref(ms)), "hweno_timing_end")
    return int(n.value), float(ms.value)


STATIC_SCRATCH_BYTES = 64 * 1024 * 1024


def rk3_step_static(S: torch.Tensor, prob: Problem, ctrl: torch.Tensor, dt: Optional[float] = None,
                    t_end: Optional[float] = None, tape: Optional[torch.Tensor] = None,
                    replay: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One SSP-RK3 step of S in place through hweno_rk3_step_static: the stage states live
    in the library's static device array, so the call allocates nothing (for code under
    graph capture).  ``ctrl``: the caller's float64[16] control block on the device.
    Calls on one GPU share that array: do not overlap them."""
    _require(S, prob, prob.nf, "state")
    for t, name in ((ctrl, "ctrl"), (tape, "tape"), (replay, "replay")):
        if t is not None and (t.dtype != torch.float64 or t.numel() < CTRL_LEN or not t.is_cuda):
            raise ValueError(f"{name} must be a float64 GPU tensor of >= {CTRL_LEN} values")
    _check(lib().hweno_rk3_step_static(ctypes.byref(prob.c()), _ptr(S), _ptr(ctrl),
                                       float(dt or 0.0), float(t_end or 0.0), _ptr(tape),
                                       _ptr(replay), _stream()), "hweno_rk3_step_static")
    return S


def rk3_step_(S: torch.Tensor, prob: Problem, dt: Optional[float] = None) -> torch.Tensor:
    """One in-place step with a throw-away workspace (convenience)."""
    return Stepper(prob, device=S.device).step(S, dt=dt)


class BatchedStepper:
    """Many independent 2D Euler grids advanced together (hweno_rk3_step_batched).

    ``states``: list of GPU tensors [12, ny_k, nx_k] (advanced in place);
    ``grids``: list of dicts with dx, dy, bc_x, bc_y (and optional dt_fixed,
    t_end) per instance; ``common``: the shared Problem (weights, eps, cfl,
    dtype, ...).  All workspaces live in one caller-side buffer.
    """

    def __init__(self, states, grids, common: Problem):
        if common.dim != 2 or common.physics != "euler":
            raise ValueError("batched stepping is for 2D Euler")
        n = len(states)
        if n < 1 or len(grids) != n:
            raise ValueError("need one grid description per state")
        self.common = common
        self._c = common.c()
        self.states = states
        self.n = n
        arr = (_CInstance * n)()
        for q, (S, g) in enumerate(zip(states, grids)):
            _require(S, Problem(dim=2, nx=S.shape[2], ny=S.shape[1], dtype=common.dtype), 12, "state")
            I = arr[q]
            I.nx, I.ny = S.shape[2], S.shape[1]
            I.bc_x, I.bc_y = int(g.get("bc_x", PERIODIC)), int(g.get("bc_y", PERIODIC))
            I.dx, I.dy = float(g["dx"]), float(g["dy"])
            I.dt_fixed = float(g.get("dt_fixed", 0.0) or 0.0)
            I.t_end = float(g.get("t_end", 0.0) or 0.0)
        tot = (ctypes.c_int32 * BATCH_VARIANTS)()
        _check(lib().hweno_batch_prepare(ctypes.byref(self._c), arr, n, tot), "hweno_batch_prepare")
        self.total_tiles = [int(t) for t in tot]
        offs, total = [], 0
        for q in range(n):
            offs.append(total)
            total += (int(arr[q].ws_bytes) + 255) // 256 * 256
        device = states[0].device
        raw = torch.zeros(total + 256, dtype=torch.uint8, device=device)
        base = (-raw.data_ptr()) % 256
        self.ws = raw[base:base + total]
        for q in range(n):
            arr[q].state = states[q].data_ptr()
            arr[q].ws = self.ws.data_ptr() + offs[q]
        self._offs = offs
        self._host = arr
        blob = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
        self.desc = blob.to(device)
        self.maps = []
        for v in range(BATCH_VARIANTS):
            m = (ctypes.c_int32 * self.total_tiles[v])()
            _check(lib().hweno_batch_tile_map(arr, n, v, m, self.total_tiles[v]),
                   "hweno_batch_tile_map")
            self.maps.append(torch.frombuffer(bytearray(bytes(m)), dtype=torch.int32).to(device))
        self.cells = sum(int(S.shape[1]) * int(S.shape[2]) for S in states)
        self.variant = 0
        self.blocks = 0
        self.graph = None

    def ctrl(self, q: int) -> torch.Tensor:
        o = self._offs[q]
        return self.ws[o:o + CTRL_LEN * 8].view(torch.float64)

    def step(self, variant: Optional[int] = None, blocks: Optional[int] = None):
        v = self.variant if variant is None else int(variant)
        b = self.blocks if blocks is None else int(blocks)
        _check(lib().hweno_rk3_step_batched(ctypes.byref(self._c), self.desc.data_ptr(),
                                            self.maps[v].data_ptr(), self.n,
                                            self.total_tiles[v], v, b, _stream()),
               "hweno_rk3_step_batched")

    def statuses(self):
        return [int(self.ctrl(q)[8:9].view(torch.int64).item()) for q in range(self.n)]

    def capture(self, steps: int = 1):
        """Capture ``steps`` batched steps (speeds, 3 stages, time update each) in one graph."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for _ in range(steps):
                    self.step()
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()


_AUTOTUNE_CACHE = {}
AUTOTUNE_CANDIDATES = 4


def autotune_batched(stepper: BatchedStepper, trials: int = 2):
    """Tile variant and persistent grid size of ``stepper`` chosen by hweno_autotune.

    The library times every (variant, grid) candidate on clones of the states
    (the originals are untouched) with hipEvents and returns the fastest; this
    wrapper only prepares the clones, keeps the choice in ``stepper`` and caches it
    per process, keyed by the batch's dtype and its instances' shapes and boundary
    conditions.  Returns ((variant, blocks), {(variant, blocks): ms per step}), or
    the cached choice and None.
    """
    key = (stepper.common.dtype,
           tuple((int(I.nx), int(I.ny), int(I.bc_x), int(I.bc_y)) for I in stepper._host))
    if key in _AUTOTUNE_CACHE:
        stepper.variant, stepper.blocks = _AUTOTUNE_CACHE[key]
        return _AUTOTUNE_CACHE[key], None
    scratch_states = [S.clone() for S in stepper.states]
    grids = [dict(nx=int(stepper._host[q].nx), dx=stepper._host[q].dx, dy=stepper._host[q].dy,
                  bc_x=stepper._host[q].bc_x, bc_y=stepper._host[q].bc_y,
                  dt_fixed=stepper._host[q].dt_fixed, t_end=stepper._host[q].t_end)
             for q in range(stepper.n)]
    scratch = BatchedStepper(scratch_states, grids, stepper.common)
    maps = (ctypes.c_void_p * BATCH_VARIANTS)(*[m.data_ptr() for m in scratch.maps])
    totals = (ctypes.c_int32 * BATCH_VARIANTS)(*scratch.total_tiles)
    n_cand = BATCH_VARIANTS * AUTOTUNE_CANDIDATES
    times = (ctypes.c_double * n_cand)()
    sizes = (ctypes.c_int32 * n_cand)()
    v, b = ctypes.c_int32(-1), ctypes.c_int32(0)
    _check(lib().hweno_autotune(ctypes.byref(scratch._c), scratch.desc.data_ptr(), maps, scratch.n,
                                totals, int(trials), _stream(), ctypes.byref(v), ctypes.byref(b),
                                times, sizes), "hweno_autotune")
    results = {}
    for k in range(n_cand):
        results[(k // AUTOTUNE_CANDIDATES, int(sizes[k]))] = float(times[k])
    del scratch, scratch_states
    best = (int(v.value), int(b.value))
    stepper.variant, stepper.blocks = best
    _AUTOTUNE_CACHE[key] = best
    return best, results


def _aligned_buffer(nbytes: int, device) -> torch.Tensor:
    raw = torch.zeros(max(nbytes, 256) + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw[off:off + max(nbytes, 256)]


def adjoint_workspace(prob: Problem, device="cuda") -> torch.Tensor:
    """Device workspace for hweno_rhs_adjoint / hweno_rk3_step_adjoint."""
    n = int(lib().hweno_adjoint_workspace_bytes(ctypes.byref(prob.c())))
    if n == 0:
        validate(prob)
    return _aligned_buffer(n, device)


def rhs_adjoint(S: torch.Tensor, prob: Problem, alpha_: torch.Tensor, lam_rhs: torch.Tensor,
                lam_lim: Optional[torch.Tensor] = None, lam_state: Optional[torch.Tensor] = None,
                ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """lam_state += (dL/dS)^T lam_rhs + (dLim/dS)^T lam_lim with the speeds frozen: the
    transpose of the operator of eqs. (odeH) / (ode2H) and of the Section 2.2 limiter."""
    _require(S, prob, prob.nf, "state")
    _require(lam_rhs, prob, prob.nf, "lam_rhs")
    if lam_lim is not None:
        _require(lam_lim, prob, prob.m * prob.dim, "lam_lim")
    out = lam_state if lam_state is not None else torch.zeros_like(S)
    _require(out, prob, prob.nf, "lam_state")
    ws = ws if ws is not None else adjoint_workspace(prob, S.device)
    a = _speeds(alpha_, S.device)
    _check(lib().hweno_rhs_adjoint(ctypes.byref(prob.c()), _ptr(S), _ptr(a), _ptr(lam_rhs),
                                   _ptr(lam_lim), _ptr(out), _ptr(ws), ws.numel(), _stream()),
           "hweno_rhs_adjoint")
    return out


def step_adjoint(prob: Problem, state0: torch.Tensor, stepper: "Stepper", tape: torch.Tensor,
                 lam: torch.Tensor, ws: torch.Tensor) -> torch.Tensor:
    """lam <- (dS^{n+1}/dS^n)^T lam in place, for the step that ``stepper`` took from state0."""
    _require(state0, prob, prob.nf, "state0")
    _require(lam, prob, prob.nf, "lam")
    _check(lib().hweno_rk3_step_adjoint(ctypes.byref(prob.c()), _ptr(state0), _ptr(stepper.ws),
                                        stepper.nbytes, _ptr(tape), _ptr(lam), _ptr(ws),
                                        ws.numel(), _stream()), "hweno_rk3_step_adjoint")
    return lam


def rollout_replay(S0: torch.Tensor, prob: Problem, tapes: torch.Tensor) -> torch.Tensor:
    """Forward steps from S0 with the taped speeds and time steps (no autograd)."""
    S = S0.detach().clone().contiguous()
    st = Stepper(prob, device=S.device)
    for n in range(tapes.shape[0]):
        st.step(S, replay=tapes[n])
    return S


def _ws_stride(prob: Problem) -> int:
    return (max(workspace_bytes(prob), 256) + 255) // 256 * 256


def rollout_bytes_kept(prob: Problem, n_steps: int) -> int:
    """Device bytes that a rollout keeping every step's states holds until its backward
    (one step workspace, 256-byte aligned, and one input state per step)."""
    state = prob.nf * prob.shape()[1] * prob.nx * (8 if prob.dtype == torch.float64 else 4)
    return n_steps * (_ws_stride(prob) + state)


def _kept_steps(S: torch.Tensor, prob: Problem, n0: int, n1: int, dt: Optional[float],
                tapes: torch.Tensor):
    """Steps n0..n1-1 of S in place, each from its own workspace, keeping every step's
    input state and workspace (its stage states) for the backward: two allocations,
    control blocks zeroed by one fill.  Returns (inputs, steppers)."""
    validate(prob)
    n = n1 - n0
    stride = _ws_stride(prob)
    rows = max(n, 1)
    raw = torch.empty(rows * stride + 256, dtype=torch.uint8, device=S.device)
    off = (-raw.data_ptr()) % 256
    wsall = raw[off:off + rows * stride].view(rows, stride)
    wsall[:, :CTRL_LEN * 8].zero_()
    states = torch.empty((n,) + tuple(S.shape), dtype=S.dtype, device=S.device)
    c = prob.c()
    steppers = [Stepper._over(prob, c, wsall[q], stride) for q in range(n)]
    for q in range(n):
        states[q].copy_(S)
        steppers[q].step(S, dt=dt, tape=tapes[n0 + q])
    return [states[q] for q in range(n)], steppers


class Rollout(torch.autograd.Function):
    """n_steps SSP-RK3 steps as a differentiable function of the initial state.

    Forward: device-side CFL time steps (or ``dt``), one tape record per step
    (speeds of the three stages and dt).  What the backward needs of each step
    (its input state and its two intermediate stage states) is either kept in
    device memory for every step (``ckpt=0``), or kept as a checkpoint every
    ``ckpt`` steps and recomputed segment by segment, newest first, with the
    tape replayed; the replay of the next older segment runs on a side stream,
    overlapped with the adjoints of the current one.  The newest segment, whose
    adjoints come first, keeps its steps' states from the forward and is not
    replayed.  ``ckpt=None`` keeps every
    step when that takes at most half of the free device memory, else
    checkpoints every ~sqrt(n_steps) steps.  The backward applies the
    hand-written step adjoints in reverse.  Speeds and time steps are held
    fixed (replay semantics), so the gradient is that of the taped
    computation.  Returns the final state; ``Rollout.last_tapes`` keeps the
    tape of the most recent forward call.
    """

    last_tapes = None

    @staticmethod
    def forward(ctx, S0, prob: Problem, n_steps: int, ckpt: Optional[int] = None,
                dt: Optional[float] = None):
        # the step adjoint has no edge-described sides (whose splits also move
        # with the time each step reads): refuse before stepping
        if prob.bc_x == EDGES or (prob.dim == 2 and prob.bc_y == EDGES):
            raise HwenoError(2, "Rollout", "the adjoint has no edge-described sides")
        S = S0.detach().clone().contiguous()
        if ckpt is None:
            free, _ = torch.cuda.mem_get_info(S.device)
            if rollout_bytes_kept(prob, n_steps) <= free // 2:
                ckpt = 0
            else:
                ckpt = max(1, int(math.isqrt(max(n_steps, 1))))
        if ckpt < 0:
            raise ValueError("ckpt must be >= 0")
        tapes = torch.zeros(n_steps, CTRL_LEN, dtype=torch.float64, device=S.device)
        ckpts, kept = [], None
        if ckpt == 0:
            kept = _kept_steps(S, prob, 0, n_steps, dt, tapes)
        else:
            # one multi-step call per segment between checkpoints; the newest
            # segment, whose adjoints the backward takes first, keeps its steps'
            # states as the kept mode does, so it needs no replay
            st = Stepper(prob, device=S.device)
            last0 = ((n_steps - 1) // ckpt) * ckpt if n_steps > 0 else 0
            for n0 in range(0, last0, ckpt):
                n1 = min(n0 + ckpt, n_steps)
                ckpts.append(S.clone())
                st.steps(S, n1 - n0, dt=dt, tapes=tapes[n0:n1])
            kept = _kept_steps(S, prob, last0, n_steps, dt, tapes)
        ctx.prob, ctx.n_steps, ctx.ckpt = prob, n_steps, ckpt
        ctx.ckpts, ctx.tapes, ctx.kept = ckpts, tapes, kept
        Rollout.last_tapes = tapes
        return S

    @staticmethod
    def backward(ctx, g):
        prob, n_steps, ckpt = ctx.prob, ctx.n_steps, ctx.ckpt
        lam = g.detach().contiguous().clone()
        if n_steps == 0:
            ctx.kept = None
            return lam, None, None, None, None
        dev = lam.device
        ws = adjoint_workspace(prob, dev)
        if ckpt == 0:
            inputs, steppers = ctx.kept
            for n in reversed(range(n_steps)):
                step_adjoint(prob, inputs[n], steppers[n], ctx.tapes[n], lam, ws)
            # the kept states are two allocations, released together here (the
            # caching allocator reuses them in the next rollout of this size)
            ctx.kept = None
            return lam, None, None, None, None
        nseg = (n_steps + ckpt - 1) // ckpt
        per = min(ckpt, n_steps)
        # Two buffer sets of replayed segments: while the adjoints of one segment
        # run on the caller's stream, the next older segment is replayed on a
        # side stream (it depends only on its checkpoint), so the replay's
        # partly filled waves of workgroups overlap the adjoint kernels.  The
        # newest segment's states were kept by the forward.
        main = torch.cuda.current_stream(dev)
        side = torch.cuda.Stream(device=dev)
        steppers = [[Stepper(prob, device=dev) for _ in range(per)] for _ in range(2 if nseg > 1 else 0)]
        inputs = [[None] * per, [None] * per]
        free = [None, None]  # event: the adjoints that last read buffer set b are done
        side.wait_stream(main)

        def replay(seg, b):
            n0, n1 = seg * ckpt, min((seg + 1) * ckpt, n_steps)
            with torch.cuda.stream(side):
                if free[b] is not None:
                    side.wait_event(free[b])
                S = ctx.ckpts[seg].clone()
                for n in range(n0, n1):
                    x = S.clone()
                    x.record_stream(main)
                    inputs[b][n - n0] = x
                    steppers[b][n - n0].step(S, replay=ctx.tapes[n])
                done = torch.cuda.Event()
                done.record(side)
            return done

        ready = replay(nseg - 2, (nseg - 2) % 2) if nseg > 1 else None
        last0 = (nseg - 1) * ckpt
        kin, ksteppers = ctx.kept
        for n in reversed(range(last0, n_steps)):
            step_adjoint(prob, kin[n - last0], ksteppers[n - last0], ctx.tapes[n], lam, ws)
        ctx.kept = None
        for seg in reversed(range(nseg - 1)):
            b = seg % 2
            main.wait_event(ready)
            if seg > 0:
                ready = replay(seg - 1, (seg - 1) % 2)
            n0, n1 = seg * ckpt, min((seg + 1) * ckpt, n_steps)
            for n in reversed(range(n0, n1)):
                step_adjoint(prob, inputs[b][n - n0], steppers[b][n - n0], ctx.tapes[n], lam, ws)
            free[b] = torch.cuda.Event()
            free[b].record(main)
        return lam, None, None, None, None
