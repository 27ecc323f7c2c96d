"""Writes tests/golden/gs2_steady_64.npz with the oracle only.

Grid setting 2 (Sec. 5.1, Fig. 30): a 64 x 64 lattice under 32 x 32
temperature control volumes, Ra 1e4, Pr 0.71 (U_char 0.1), side-heated
cavity walls, from rest with T = 0, one energy step per 2NX = 64 lattice
steps, each energy step solved exactly (sparse direct solve of its implicit
system, not the line sweeps the library relaxes it with).  Run until the
relative change of u, v and T over 16 energy cycles is <= 1e-12.  Stored:
the step count, the last changes, the fields u, v, T on the lattice nodes
and the hot/cold wall Nusselt numbers.

    python tests/golden/make_gs2_steady.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.gs2 import GS2Case  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gs2_steady_64.npz")


def main():
    t0 = time.time()
    c = GS2Case(64, 64, solver="direct").set_physics(1e4, 0.71).init()
    steps, r = c.run_to_steady(1e-12, cycles=16, max_steps=2_000_000)
    nu = c.nusselt()
    np.savez_compressed(OUT, steps=steps, change=r, tol=1e-12, cycles=16,
                        u=c.fetch("u"), v=c.fetch("v"), T=c.fetch("T"),
                        nu_hot=nu["nu_hot"], nu_cold=nu["nu_cold"],
                        nu_hot_max=nu["nu_hot_max"], y_hot_max=nu["y_hot_max"])
    print(f"done: {steps} steps, change {r}, Nu_hot {nu['nu_hot']:.8f}, "
          f"{time.time() - t0:.0f} s -> {OUT}", flush=True)


if __name__ == "__main__":
    main()
