"""Writes tests/golden/sweep_steady_64.npz with the oracle only.

The three smallest-size classes of the 256-cavity sweep (splitmix64 seed
1908083864; the first cavity drawn with ny = 64 and aspect 1, 2 and 3:
draws 12, 39 and 3), seeded T0 perturbation (uniform +-1e-6, each cavity's
own seed), run by the FP64 oracle until the relative residual (K = 1000
steps) of u, v and T is <= 1e-8.  Stored per cavity: its draw index, the
step count, the final residuals, the Nusselt numbers and u, v, T rounded to
FP32 (a relative rounding of at most 6e-8 of each field's maximum, far
below the 1e-4 the FP32 path is held to).

    python tests/golden/make_sweep_steady.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth_inputs import cavity_sweep, perturbation  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep_steady_64.npz")
DRAWS = (12, 39, 3)


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    oracle.set_threads(threads)
    sweep = cavity_sweep(256)
    out = {"draws": np.array(DRAWS)}
    for k in DRAWS:
        c = sweep[k]
        assert c["ny"] == 64
        t0 = time.time()
        o = oracle.Case(c["nx"], c["ny"]).set_physics(c["Ra"], c["Pr"]).set_cavity_walls()
        o.init(perturbation(c["nx"], c["ny"], c["seed"]))
        steps, r = o.run_to_steady(tol=1e-8, check_every=1000, max_steps=5_000_000)
        nu = o.nusselt()
        out[f"steps_{k}"] = steps
        out[f"residual_{k}"] = r
        out[f"nu_{k}"] = np.array([nu["nu_hot"], nu["nu_cold"], nu["nu_hot_max"]])
        for f in ("u", "v", "T"):
            out[f"{f}_{k}"] = o.fetch(f).astype(np.float32)
        print(f"draw {k}: {c['nx']}x{c['ny']} Ra {c['Ra']:.4g} Pr {c['Pr']}: {steps} steps, "
              f"r = {r}, Nu {nu['nu_hot']:.8f}, {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, **out)
    print(f"-> {OUT}", flush=True)


if __name__ == "__main__":
    main()
