"""The oracle against itself: how far one-ulp changes of the input move its
results, in the norms the GPU parity tests use.

A parity gate means something only above this floor.  The strict norm (per
conserved component, scaled by max |U_c|) is used everywhere except for the
operator of the blast-wave state at rest (Example 3.7), whose momentum vanishes
everywhere: there the strict norm divides the rounding of a pressure-carried
flux by 1, and the oracle perturbed by one ulp already lands above 1e-12.
These tests measure that floor, so that the relaxed scale (the larger of
max |U_c| and the reference increment max |dx L_U,c|) is used only where it has
to be, and check that the strict norm leaves a wide margin on the inputs the
whole-grid tests use.
"""
import torch

import hweno_inputs as hi
from oracle import hweno_ref as o
from tests import parity as P


def _ulp_perturbed(S, seed):
    """Every value times (1 + r 2^-52), r in {-1, 0, 1} seeded: one-ulp changes."""
    g = torch.Generator().manual_seed(seed)
    r = torch.randint(-1, 2, S.shape, generator=g).to(torch.float64)
    return S * (1.0 + r * 2.0 ** -52)


def test_blast_wave_operator_floor_needs_the_flux_scale():
    w = hi.blast_waves_1d(800)
    prob = o.problem_from_workload(w)
    S = o.as_tensor(w.S)
    alpha = o.max_speeds(S, prob)
    L = o.rhs(S, prob, alpha)
    strict, relaxed = 0.0, 0.0
    for seed in range(3):
        Lp = o.rhs(_ulp_perturbed(S, seed), prob, alpha)
        strict = max(strict, max(P.rhs_errors(Lp, L, S, w).values()))
        relaxed = max(relaxed, max(P.rhs_errors(Lp, L, S, w, flux_scale=True).values()))
    print(f"blast-wave operator floor: strict {strict:.2e}, flux-scaled {relaxed:.2e}")
    # the strict norm's floor reaches the FP64 gate: no implementation could pass it
    assert strict > 1e-12
    assert relaxed < 1e-13


def test_strict_norm_floor_of_the_other_workloads_is_far_below_the_gate():
    """One step of the inputs the parity tests use most (rough 2D data with walls,
    four quadrants, the 1D problems) moves by far less than 1e-12 under the
    strict norm when the input moves by one ulp."""
    cases = [hi.euler2d_quadrants(70, 45, 0), hi.euler2d_rough(47, 29, 8, bc=hi.REFLECT),
             hi.shu_osher_1d(400), hi.roughened(hi.forward_step(60, 20), 7)]
    for w in cases:
        kw = dict(limiter_characteristic=True) if w.obstacle is not None else {}
        prob = o.problem_from_workload(w, **kw)
        S = o.as_tensor(w.S)
        ref, dt, al = o.rk3_step(S, prob)
        out, _, _ = o.rk3_step(_ulp_perturbed(S, 1), prob, dt, al)
        worst = max(P.step_errors(out, ref, w).values())
        print(f"{w.name}: strict step floor {worst:.2e}")
        assert worst < 1e-13, (w.name, worst)
