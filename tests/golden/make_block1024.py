"""Writes block1024_samples.txt: the FP64 oracle's state after 1000 steps of the
1024 x 1024 block workload, sampled at 4096 seeded nodes (plus the whole wall rows at
four columns).  Calls only the oracle; takes about an hour on one core.

Workload: velocity wall v = 0 on the left (half-way), traction-free walls elsewhere,
body force (0, -1e-5) ramped linearly over 500 steps, log-NH mu = 0.1, lam = 0.3,
F0 = I, v0 = 0, c = 10, omega = 2 - 1.6 / 1024.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lbm  # noqa: E402

N, STEPS, C = 1024, 1000, 10.0
OMEGA = 2.0 - 1.6 / N


def sample_nodes():
    rng = np.random.default_rng(2024)
    ys = rng.integers(0, N, 4096)
    xs = rng.integers(0, N, 4096)
    edge = np.arange(N)
    for col in (0, 1, N - 2, N - 1):
        ys = np.concatenate([ys, edge, np.full(N, col)])
        xs = np.concatenate([xs, np.full(N, col), edge])
    return ys, xs


def main():
    body = np.zeros((2, N, N))
    body[1] = -1e-5
    pb = lbm.Problem(nx=N, ny=N, c=C, omega=OMEGA, law="lognh", mu=0.1, lam=0.3, body=body,
                     ramp=lambda k: min(1.0, k / 500),
                     edges=[lbm.Edge("velocity"), lbm.Edge("traction"), lbm.Edge("traction"), lbm.Edge("traction")])
    st = lbm.initial_state(pb, np.zeros((2, N, N)))
    t0 = time.time()
    for k in range(STEPS):
        lbm.step(pb, st)
        if (k + 1) % 50 == 0:
            print(f"step {k + 1} {time.time() - t0:.0f} s", flush=True)
    U, u = lbm.observe(pb, st)
    ys, xs = sample_nodes()
    with open(os.path.join(HERE, "block1024_samples.txt"), "w") as fh:
        fh.write("# FP64 oracle, 1024x1024 block workload after 1000 steps (written by make_block1024.py)\n")
        fh.write("# y x v1 v2 F11-1 F12 F21 F22-1 u1 u2\n")
        for y, x in zip(ys, xs):
            vals = [U[0, y, x], U[1, y, x], U[2, y, x] - 1.0, U[3, y, x], U[4, y, x], U[5, y, x] - 1.0,
                    u[0, y, x], u[1, y, x]]
            fh.write(f"{y} {x} " + " ".join(f"{v:.17e}" for v in vals) + "\n")


if __name__ == "__main__":
    main()
