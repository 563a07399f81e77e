"""MI355X (gfx950) L-HWENO hot path: HIP kernels behind a C ABI, thin binding.

Zhang & Zhao, "A fifth-order finite difference HWENO scheme combined with
limiter for hyperbolic conservation laws" (arXiv 2207.05258).
"""
from .hweno import (BatchedStepper, Rollout, adjoint_workspace, autotune_batched, rhs_adjoint,
                    rollout_bytes_kept,
                    rollout_replay, step_adjoint, CTRL_LEN, EDGES, OUTFLOW, PERIODIC, REFLECT,  # noqa: F401
                    SEG_OUTFLOW, SEG_REFLECT, SEG_STATE, Edge, HwenoError, Problem, Stepper,
                    alpha, lib, limit, problem_for, rhs, rk3_step_, rk3_step_static, timing_begin, timing_end, validate,
                    workspace_bytes)
