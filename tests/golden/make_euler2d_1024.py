"""Writes euler2d_1024_100steps.txt: the oracle's run of the 2D Euler four-quadrant workload
(1024 x 1024 cells on [0, 1]^2, seed 0, outflow sides) for 100 SSP-RK3 steps (Section 2.2),
each with its own CFL time step from the stage-1 speeds (global Lax-Friedrichs speeds of
Section 2.1): the time reached and, on six rows (0, 300, 511, 512, 700, 1023) at every 16th
column from column 5 on, all twelve fields.  Calls only the oracle and the seeded input
generator; about half an hour on eight threads.

    python tests/golden/make_euler2d_1024.py
"""
import os
import sys

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import hweno_inputs as hi  # noqa: E402
from oracle import hweno_ref as o  # noqa: E402

N, SEED, STEPS = 1024, 0, 100
ROWS = (0, 300, 511, 512, 700, 1023)
COLS = tuple(range(5, N, 16))
OUT = os.path.join(HERE, "euler2d_1024_100steps.txt")


def main():
    w = hi.euler2d_quadrants(N, N, SEED)
    prob = o.problem_from_workload(w)
    S = torch.as_tensor(w.S, dtype=torch.float64)
    t = 0.0
    for n in range(STEPS):
        S, dt, _ = o.rk3_step(S, prob)
        t += dt
        print(f"step {n + 1}: dt {dt:.17g}", flush=True)
    with open(OUT, "w") as fh:
        fh.write("# 2D Euler, 1024 x 1024 four-quadrant data (seed 0), outflow, gamma 1.4, CFL 0.6; 100\n")
        fh.write("# SSP-RK3 steps (Section 2.2) with the oracle's own time steps; written by\n")
        fh.write("# make_euler2d_1024.py from the oracle.  Rows: j i, then the 12 fields U, U_x, U_y.\n")
        fh.write(f"t {t:.17g}\n")
        for j in ROWS:
            for i in COLS:
                fh.write(f"{j} {i} " + " ".join(f"{float(S[f, j, i]):.17g}" for f in range(12)) + "\n")
    print(f"t = {t:.17g}, {len(ROWS) * len(COLS)} cells -> {OUT}")


if __name__ == "__main__":
    main()
