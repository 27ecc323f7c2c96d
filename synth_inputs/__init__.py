"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the method itself: it only draws numbers
(splitmix64, Steele, Lea & Flood 2014) and case descriptions.  Both the
oracle side and the GPU side receive the arrays it produces.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

SEED_C2 = 1908083860      # perturbation of the 512^2 Ra 1e6 cavity
SEED_C3 = 1908083860      # perturbation of the 4096^2 split cavity (same rule)
SEED_BATCH = 1908083864   # 256-cavity sweep
SEED_TRAIN = 1908083865   # warm-start training set
SEED_HELDOUT = 1908083866 # warm-start held-out set


def splitmix64(seed: int, n: int) -> np.ndarray:
    """First ``n`` outputs of splitmix64 started from ``seed`` (uint64)."""
    k = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int) -> np.ndarray:
    """``n`` doubles in [0, 1) from the top 53 bits of splitmix64."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def perturbation(nx: int, ny: int, seed: int, amp: float = 1e-6) -> np.ndarray:
    """T0 = amp * (2U - 1), U drawn in row-major order (j outer, i inner)."""
    u = uniform01(seed, nx * ny)
    return (amp * (2.0 * u - 1.0)).reshape(ny, nx)


class _Stream:
    """Sequential draws from one splitmix64 stream."""

    def __init__(self, seed: int):
        self.state = np.uint64(seed)

    def next_u64(self) -> int:
        with np.errstate(over="ignore"):
            self.state = self.state + _GAMMA
            z = self.state
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        return int(z)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (2.0 ** -53)

    def choice(self, items):
        return items[min(int(self.uniform() * len(items)), len(items) - 1)]


SWEEP_SIZES = (64, 96, 128, 192, 256, 384, 512)


def cavity_sweep(n: int, seed: int = SEED_BATCH, max_ny: int | None = None):
    """Heterogeneous side-heated cavities: per cavity, in draw order,
    ny from SWEEP_SIZES, aspect A in {1,2,3,4} (nx = A ny), log10 Ra ~ U[3, 6],
    Pr in {0.71, 7.0}.  ``max_ny`` caps ny after the draw (training sets)."""
    s = _Stream(seed)
    out = []
    for k in range(n):
        ny = s.choice(SWEEP_SIZES)
        A = s.choice((1, 2, 3, 4))
        lra = 3.0 + 3.0 * s.uniform()
        pr = s.choice((0.71, 7.0))
        if max_ny is not None:
            ny = min(ny, max_ny)
        out.append({"nx": A * ny, "ny": ny, "aspect": A, "Ra": 10.0 ** lra, "Pr": pr,
                    "seed": seed * 1000 + k})
    return out
