"""Writes the oracle's runs of the 1D Euler workload (N = 4000 cells, periodic
piecewise-constant data, seed 0) to T = 0.2 with its own CFL time steps and the last step
clipped at T (SSP-RK3 of Section 2.2, the scheme of Section 2.1): the number of steps and,
at every 8th cell from cell 3 on, the state and the derivative components.

    euler1d_4000_T0.2.txt        the limiter component by component (the default reading)
    euler1d_4000_char_T0.2.txt   the limiter in the cell's characteristic fields

Calls only the oracle and the seeded input generator; about four (component-wise) and
eight (characteristic) minutes on one thread.

    python tests/golden/make_euler1d_4000.py [--char]
"""
import os
import sys

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import hweno_inputs as hi  # noqa: E402
from oracle import hweno_ref as o  # noqa: E402

N, SEED, T, STRIDE, FIRST = 4000, 0, 0.2, 8, 3


def main(char: bool):
    torch.set_num_threads(1)
    out = os.path.join(HERE, "euler1d_4000_char_T0.2.txt" if char else "euler1d_4000_T0.2.txt")
    w = hi.euler1d_piecewise(N, SEED)
    prob = o.problem_from_workload(w, limiter_characteristic=char)
    S, steps = o.run(torch.as_tensor(w.S, dtype=torch.float64), prob, T)
    cells = list(range(FIRST, N, STRIDE))
    with open(out, "w") as fh:
        fh.write("# 1D Euler, N = 4000 periodic cells, piecewise-constant data (seed 0), gamma 1.4,\n")
        fh.write("# CFL time steps, SSP-RK3 (Section 2.2), last step clipped at T = 0.2, limiter "
                 + ("in characteristic fields" if char else "component by component") + ";\n")
        fh.write("# written by make_euler1d_4000.py from the oracle.  Rows: cell, U0 U1 U2, Ux0 Ux1 Ux2.\n")
        fh.write(f"steps {steps}\n")
        for i in cells:
            fh.write(f"{i} " + " ".join(f"{float(S[c, 0, i]):.17g}" for c in range(6)) + "\n")
    print(f"{steps} steps, {len(cells)} cells -> {out}")


if __name__ == "__main__":
    main("--char" in sys.argv)
