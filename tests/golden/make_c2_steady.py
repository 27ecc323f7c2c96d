"""Writes tests/golden/c2_steady_512.npz with the oracle only.

The 512 x 512 side-heated cavity at Ra 1e6, Pr 0.71 (U_char 0.1), seeded T0
perturbation (uniform +-1e-6, splitmix64 seed 1908083860), run by the FP64
oracle until the relative residual (K = 1000 steps) of u, v and T is <= 1e-8.
Stored: the step count S_o, the final residuals, the Nusselt numbers, the
full hot- and cold-wall temperature columns, u, v, T on every node rounded
to FP32 (for the FP32 comparison at 1e-4 of the field maxima; the rounding
is below 1e-7 of them), u, v, T in FP64 on every 4th node in each direction
(for the FP64 comparison at 1e-9), and the full-field maxima.

    python tests/golden/make_c2_steady.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth_inputs import SEED_C2, perturbation  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_steady_512.npz")


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    oracle.set_threads(threads)
    n = 512
    c = oracle.Case(n, n).set_physics(1e6, 0.71).set_cavity_walls()
    c.init(perturbation(n, n, SEED_C2))
    c.residual()
    t0 = time.time()
    tol, K = 1e-8, 1000
    while True:
        c.step(K)
        r = c.residual()
        if c.steps % 20000 == 0:
            print(f"{c.steps} steps, r = {r}, {time.time() - t0:.0f} s", flush=True)
        if r.max() <= tol or c.steps >= 6_000_000:
            break
    u, v, T = c.fetch("u"), c.fetch("v"), c.fetch("T")
    nu = c.nusselt()
    np.savez_compressed(
        OUT, steps=c.steps, residual=r, tol=tol, check_every=K,
        nusselt=np.array([nu[k] for k in ("nu_hot", "nu_cold", "nu_hot_max", "y_hot_max",
                                          "nu_cold_max", "y_cold_max", "nu_hot_o2",
                                          "nu_cold_o2")]),
        T_west=T[:, 0].copy(), T_east=T[:, -1].copy(),
        u_s=u[::4, ::4].copy(), v_s=v[::4, ::4].copy(), T_s=T[::4, ::4].copy(),
        u32=u.astype(np.float32), v32=v.astype(np.float32), T32=T.astype(np.float32),
        max_abs=np.array([np.abs(u).max(), np.abs(v).max(), np.abs(T).max()]))
    print(f"done: {c.steps} steps, r = {r}, Nu_hot = {nu['nu_hot']:.6f}, "
          f"{time.time() - t0:.0f} s -> {OUT}", flush=True)


if __name__ == "__main__":
    main()
