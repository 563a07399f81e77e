"""Plants plausible mistakes in the oracle, one at a time, and runs the oracle's pins
(tests/test_oracle_*.py, CPU only) against each mutant: every mutant must make at least one
pin fail.  The mutants are dropped or swapped terms, wrong signs, indices, coefficients and
transposed operands in each part of the oracle: the Hermite values, the quintic's
coefficients, the smoothness indicators and nonlinear weights (Section 2.1), the mirrored
"-" reconstruction, the linear derivative fluxes, the limiter (Section 2.2) and its switch,
the Euler and scalar fluxes, their chain-rule products and speeds, the Roe average and
eigenvectors (Remarks 2.1/2.2), the splitting, the mixed flux (eq. mixed), the flux
differences (eqs. odeH/ode2H), the ghost cells and the obstacle, the time step, SSP-RK3 and
the clipped last step.  Each runs in a copy of the repository in a temporary
directory; nothing here touches the HIP path.

    python tests/oracle_mutants.py            # all mutants, four at a time
    python tests/oracle_mutants.py -j 2 tau_half swap_beta
"""
import argparse
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join("oracle", "hweno_ref.py")

# (name, text in the oracle, its replacement, which occurrence (1-based) to replace)
MUTANTS = [
    # Hermite values p0, p1, p2 and the quintic's coefficients
    ("p0_weight", "19.0 / 30.0 * f0", "19.0 / 31.0 * f0", 1),
    ("p0_derivative_sign", "(Hm + 10.0 * H0 - Hp) / 20.0", "(Hm + 10.0 * H0 + Hp) / 20.0", 1),
    ("p1_derivative_weight", "5.0 / 6.0 * f0 + 2.0 / 3.0 * H0", "5.0 / 6.0 * f0 + 1.0 / 3.0 * H0", 1),
    ("p2_derivative_sign", "fp / 6.0 + H0 / 3.0", "fp / 6.0 - H0 / 3.0", 1),
    ("a1_transposed", "27.0 / 64.0 * (fm - fp)", "27.0 / 64.0 * (fp - fm)", 1),
    ("a3_transposed", "15.0 / 8.0 * (fp - fm)", "15.0 / 8.0 * (fm - fp)", 1),
    ("a5_dropped_term", "a5 = 0.25 * Hm + H0 + 0.25 * Hp", "a5 = 0.25 * Hm + 0.25 * Hp", 1),
    # smoothness indicators and weights
    ("beta0_coefficient", "781.0 / 20.0 * (a3", "781.0 / 10.0 * (a3", 1),
    ("beta0_a4_coefficient", "1421461.0 / 2275.0 * a4 ** 2", "1421461.0 / 2000.0 * a4 ** 2", 1),
    ("beta0_a5_coefficient", "21520059541.0 / 1377684.0", "21520059541.0 / 1300000.0", 1),
    ("beta0_mixed_a3_a5", "8825.0 / 10934.0 * a5", "8825.0 / 10000.0 * a5", 1),
    ("beta0_cross_term", "(a1 + a3 / 4.0 + a5 / 16.0) ** 2", "(a1 + a3 / 4.0 - a5 / 16.0) ** 2", 1),
    ("beta1_index", "13.0 / 3.0 * (H0 - f0 + fm) ** 2", "13.0 / 3.0 * (H0 - f0 + fp) ** 2", 1),
    ("beta2_sign", "13.0 / 3.0 * (H0 + f0 - fp) ** 2", "13.0 / 3.0 * (H0 - f0 + fp) ** 2", 1),
    ("swap_beta", "w1 = lin[1] * (1.0 + tau / (b1 + eps))", "w1 = lin[1] * (1.0 + tau / (b2 + eps))", 1),
    ("tau_half", "tau = 0.25 * ((b0", "tau = 0.5 * ((b0", 1),
    ("tau_wrong_difference", "(b0 - b1).abs() + (b0 - b2).abs()", "(b0 - b1).abs() + (b1 - b2).abs()", 1),
    ("tau_no_square", "(b0 - b2).abs()) ** 2", "(b0 - b2).abs())", 1),
    ("weights_not_normalised", "return w0 / s, w1 / s, w2 / s", "return w0, w1, w2", 1),
    ("eps_scaled", "tau / (b0 + eps)", "tau / (b0 + 100.0 * eps)", 1),
    ("combination_sign", "p0 / g0 - g1 / g0 * p1", "p0 / g0 + g1 / g0 * p1", 1),
    ("swap_candidates", "+ w1 * p1 + w2 * p2", "+ w1 * p2 + w2 * p1", 1),
    # mirrored reconstruction and linear derivative fluxes
    ("minus_not_mirrored",
     "return hweno_plus(f_ip2, f_ip1, f_i, -H_ip2, -H_ip1, -H_i, lin, eps, linear)",
     "return hweno_plus(f_i, f_ip1, f_ip2, H_i, H_ip1, H_ip2, lin, eps, linear)", 1),
    ("minus_derivative_sign",
     "return hweno_plus(f_ip2, f_ip1, f_i, -H_ip2, -H_ip1, -H_i, lin, eps, linear)",
     "return hweno_plus(f_ip2, f_ip1, f_i, H_ip2, H_ip1, H_i, lin, eps, linear)", 1),
    ("hhat_scale", "(fm - 8.0 * f0 + 7.0 * fp) / (4.0 * dx)", "(fm - 8.0 * f0 + 7.0 * fp) / (2.0 * dx)", 1),
    ("hhat_derivative_sign", "(hm - 2.0 * h0 - 5.0 * hp) / 12.0", "(hm + 2.0 * h0 - 5.0 * hp) / 12.0", 1),
    ("hhat_minus_not_negated", "return -quintic_derivative(", "return quintic_derivative(", 1),
    # limiter
    ("limiter_q0_sign", "(up - um) - 0.25 * (vm + vp)", "(up - um) + 0.25 * (vm + vp)", 1),
    ("limiter_a2_transposed", "a2 = dx / 4.0 * (vm - vp)", "a2 = dx / 4.0 * (vp - vm)", 1),
    ("limiter_beta1_index", "b1 = (u0 - um) ** 2", "b1 = (u0 - up) ** 2", 1),
    ("limiter_beta0_coefficient", "781.0 / 20.0 * a3 ** 2", "781.0 / 10.0 * a3 ** 2", 1),
    ("limiter_beta0_a4_coefficient", "1421461.0 / 2275.0 * a4 ** 2", "1421461.0 / 2000.0 * a4 ** 2", 2),
    ("limiter_swap_candidates", "+ l1 * q1 + l2 * q2", "+ l1 * q2 + l2 * q1", 1),
    ("limiter_neighbours_swapped", "vm, vp = Dp.narrow(axis, 0, n), Dp.narrow(axis, 2, n)",
     "vm, vp = Dp.narrow(axis, 2, n), Dp.narrow(axis, 0, n)", 1),
    # Euler physics
    ("pressure_gamma", "p = (self.g - 1.0) * (E - 0.5 * rho", "p = self.g * (E - 0.5 * rho", 1),
    ("energy_flux_without_pressure",
     "torch.stack([rho * u, rho * u * u + p, rho * u * v, u * (E + p)], -1)",
     "torch.stack([rho * u, rho * u * u + p, rho * u * v, u * E], -1)", 1),
    ("y_flux_momenta_swapped", "torch.stack([rho * v, rho * u * v, rho * v * v + p, v * (E + p)], -1)",
     "torch.stack([rho * v, rho * v * v + p, rho * u * v, v * (E + p)], -1)", 1),
    ("jvp_pressure_sign", "+ 0.5 * (u * u + v * v) * r_s)", "- 0.5 * (u * u + v * v) * r_s)", 1),
    ("jvp_velocity_sign", "u_s = (m_s - u * r_s) / rho", "u_s = (m_s + u * r_s) / rho", 1),
    ("jvp_y_pressure_dropped", "n_s * v + n * v_s + p_s", "n_s * v + n * v_s", 1),
    ("sound_speed_without_gamma", "c = torch.sqrt(self.g * p / rho)", "c = torch.sqrt(p / rho)", 1),
    ("roe_weights_swapped", "u = (sL * uL + sR * uR) / (sL + sR)", "u = (sR * uL + sL * uR) / (sL + sR)", 1),
    ("roe_sound_speed", "(self.g - 1.0) * (H - 0.5 * (u * u + v * v))", "(self.g - 1.0) * (H - (u * u + v * v))", 1),
    ("eigenvector_enthalpy_sign", "torch.stack([one, u - c, v, H - u * c], -1)",
     "torch.stack([one, u - c, v, H + u * c], -1)", 1),
    ("eigenvector_y_shear", "torch.stack([zero, one, zero, u], -1)", "torch.stack([zero, one, zero, v], -1)", 1),
    # splitting, reconstruction inputs, mixed flux, differences
    ("split_derivative_field", "hP = [0.5 * (at(AD, k) + alpha * at(Dnp, k))",
     "hP = [0.5 * (at(AD, k) + alpha * at(Up, k))", 1),
    ("derivative_data_unscaled", "cHP = [dd * proj(x) for x in hP]", "cHP = [proj(x) for x in hP]", 1),
    ("minus_stencil_shifted", "hweno_minus(cfM[1], cfM[2], cfM[3], cHM[1], cHM[2], cHM[3]",
     "hweno_minus(cfM[0], cfM[1], cfM[2], cHM[0], cHM[1], cHM[2]", 1),
    ("mixed_scale", "- at(AT, 3)) / 12.0", "- at(AT, 3)) / 6.0", 1),
    ("difference_sign", "return -(Fh.narrow(axis, 1, n) - Fh.narrow(axis, 0, n)) / h",
     "return (Fh.narrow(axis, 1, n) - Fh.narrow(axis, 0, n)) / h", 1),
    ("mixed_x_divided_by_dy", "LW = _difference(eh, 2, prob.dx)", "LW = _difference(eh, 2, prob.dy)", 1),
    ("y_fluxes_exchanged", "LW = LW + _difference(th, 1, prob.dy)\n    LV = LV + _difference(xh, 1, prob.dy)",
     "LW = LW + _difference(xh, 1, prob.dy)\n    LV = LV + _difference(th, 1, prob.dy)", 1),
    # ghost cells, speeds, time step, Runge-Kutta
    ("periodic_shift", "return A.index_select(axis, k % n)", "return A.index_select(axis, (k + 1) % n)", 1),
    ("outflow_second_cell", "return A.index_select(axis, torch.clamp(k, 0, n - 1))",
     "return A.index_select(axis, torch.clamp(k, 1, n - 2))", 1),
    ("reflect_off_by_one", "mirror = torch.where(k < 0, -1 - k,", "mirror = torch.where(k < 0, -k,", 1),
    ("wall_parities_not_flipped", "return pu, [-q for q in pu], pu", "return pu, pu, pu", 1),
    ("wall_normal_momentum", "pu[1 + d] = -1.0", "pu[2 - d] = -1.0", 1),
    ("edge_split_depth_ignored", "split = e.split[0] + e.split[1] * t + e.split[2] * depth",
     "split = e.split[0] + e.split[1] * t", 1),
    ("edge_segments_exchanged", "seg1 = pos >= split", "seg1 = pos < split", 1),
    ("inflow_derivatives_kept", "val = torch.zeros(A.shape[0], 1, 1, dtype=A.dtype)",
     "val = torch.ones(A.shape[0], 1, 1, dtype=A.dtype)", 1),
    ("obstacle_front_mirror_off_by_one", "src_i = jj, (2 * i_s - 1 - ii)", "src_i = jj, (2 * i_s - ii)", 1),
    ("obstacle_solid_rows", "m[:j_s, i_s:] = True", "m[:j_s + 1, i_s:] = True", 1),
    ("char_limiter_not_projected_back", "return (R @ z.movedim(0, -1).unsqueeze(-1)).squeeze(-1).movedim(-1, 0)",
     "return z", 1),
    ("speed_without_sound", "return (u if d == 0 else v).abs() + c", "return (u if d == 0 else v).abs()", 1),
    ("cfl_2d_max", "return prob.cfl / (alpha[0] / prob.dx + alpha[1] / prob.dy)",
     "return prob.cfl / max(alpha[0] / prob.dx, alpha[1] / prob.dy)", 1),
    ("rk3_stage2_weights", "S2 = keep(0.75 * H0 + 0.25 * (", "S2 = keep(0.5 * H0 + 0.5 * (", 1),
    ("rk3_stage3_weights", "S3 = keep(H0 / 3.0 + 2.0 / 3.0 * (", "S3 = keep(H0 / 2.0 + 1.0 / 2.0 * (", 1),
    ("rk3_stage2_unlimited", "hat(S1, prob, t1)", "S1", 1),
    ("stage_times", "t1, t2 = t + dt, t + 0.5 * dt", "t1, t2 = t + dt, t + dt", 1),
    ("rk3_stage3_unlimited", "hat(S2, prob, t2) + dt", "S2 + dt", 1),
    ("cfl_1d_halved", "return prob.cfl * prob.dx / alpha[0]", "return 0.5 * prob.cfl * prob.dx / alpha[0]", 1),
    ("roe_enthalpy_unweighted", "H = (sL * HL + sR * HR) / (sL + sR)", "H = 0.5 * (HL + HR)", 1),
    ("mixed_first_sign", "mixed = (-at(AT, 0) + 7.0 * at(AT, 1)", "mixed = (at(AT, 0) + 7.0 * at(AT, 1)", 1),
    ("eps_in_tau", "tau = 0.25 * ((b0 - b1).abs() + (b0 - b2).abs()) ** 2",
     "tau = 0.25 * ((b0 - b1).abs() + (b0 - b2).abs()) ** 2 + eps", 1),
    # scalar laws, the limiter's driver, the obstacle, the run loop
    ("burgers_flux_not_halved", "return 0.5 * U * U", "return U * U", 1),
    ("burgers_jvp_without_u", "        return U * D\n", "        return D\n", 1),
    ("linadv_jvp_x_speed_only", "return self.prob.adv_speed[d] * D", "return self.prob.adv_speed[0] * D", 1),
    ("linadv_speed_signed", "abs(self.prob.adv_speed[d])", "self.prob.adv_speed[d]", 1),
    ("char_limiter_left_is_right", "Li = torch.linalg.inv(R)", "Li = R", 1),
    ("limiter_y_with_dx", "along(W, 1, prob.bc_y, prob.dy)", "along(W, 1, prob.bc_y, prob.dx)", 1),
    ("limiter_switch_ignored", "    if not prob.limiter_on:\n        return S\n", "", 1),
    ("obstacle_top_mirror_off_by_one", "(2 * j_s - 1 - jj)", "(2 * j_s - jj)", 1),
    ("obstacle_solid_columns", "m[:j_s, i_s:] = True", "m[:j_s, i_s + 1:] = True", 1),
    ("wall_tangential_derivative_flipped", "return pu, [-q for q in pu], pu",
     "return pu, [-q for q in pu], [-q for q in pu]", 1),
    ("solid_cells_not_kept", "return torch.where(solid, S, X) if prob.obstacle is not None else X",
     "return X", 1),
    ("last_step_not_clipped", "dt = min(dt, t_end - t)", "dt = dt", 1),
]

COPY = ["oracle", "tests", "hweno_inputs", "paper_2207_05258_amd", "pytest.ini"]


def mutate(src: str, find: str, repl: str, which: int) -> str:
    pos = -1
    for _ in range(which):
        pos = src.find(find, pos + 1)
        if pos < 0:
            raise ValueError(f"occurrence {which} of {find!r} not in the oracle")
    return src[:pos] + repl + src[pos + len(find):]


def run_one(m, threads):
    name, find, repl, which = m
    tmp = tempfile.mkdtemp(prefix=f"mut_{name}_")
    try:
        for p in COPY:
            s, d = os.path.join(ROOT, p), os.path.join(tmp, p)
            if os.path.isdir(s):
                shutil.copytree(s, d, ignore=shutil.ignore_patterns("__pycache__", "*.so"))
            else:
                shutil.copy(s, d)
        path = os.path.join(tmp, ORACLE)
        with open(path) as fh:
            src = fh.read()
        with open(path, "w") as fh:
            fh.write(mutate(src, find, repl, which))
        pins = sorted(f for f in os.listdir(os.path.join(tmp, "tests")) if f.startswith("test_oracle_"))
        env = dict(os.environ, OMP_NUM_THREADS=str(threads), PYTHONDONTWRITEBYTECODE="1")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p",
                            "no:cacheprovider"] + [os.path.join("tests", f) for f in pins],
                           cwd=tmp, env=env, capture_output=True, text=True, timeout=3600)
        lines = r.stdout.strip().splitlines()
        failed = next((ln.split()[1] for ln in lines if ln.startswith("FAILED")), "")
        return name, r.returncode != 0, failed or (lines[-1] if lines else r.stderr[-200:])
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=4, help="mutants run at once")
    ap.add_argument("names", nargs="*")
    args = ap.parse_args()
    with open(os.path.join(ROOT, ORACLE)) as fh:
        src = fh.read()
    todo = [m for m in MUTANTS if not args.names or m[0] in args.names]
    for m in todo:
        mutate(src, m[1], m[2], m[3])          # every mutation applies to the current oracle
    threads = max(1, (os.cpu_count() or 4) // args.j)
    survived = []
    with ThreadPoolExecutor(args.j) as ex:
        for name, caught, what in ex.map(lambda m: run_one(m, threads), todo):
            print(f"{name:32s} {'caught by ' + what if caught else 'SURVIVED: ' + what}", flush=True)
            if not caught:
                survived.append(name)
    print(f"{len(todo) - len(survived)} of {len(todo)} mutants caught"
          + (f"; survived: {', '.join(survived)}" if survived else ""), flush=True)
    sys.exit(1 if survived else 0)


if __name__ == "__main__":
    main()
