"""Plain FP64 reference of the Monte Carlo temperature solver and of the
coupled LBM-MCM method (Sec. 6, Eq 97-102, Fig. 39).

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle/``): it checks
the GPU library and is never called by it.

* Nodes are the lattice cell centres; the node temperature satisfies Eq 97,
  T_P = P_x+ T_E + P_x- T_W + P_y+ T_N + P_y- T_S, with the probabilities of
  Eq 99 (Delta x = Delta y = 1): link weights alpha - u (x+), alpha (x-),
  alpha - v (y+), alpha (y-), each P the weight over their sum D (Eq 100
  with alpha, which makes them sum to 1); u = v = 0 gives Eq 98.
* Walls lie on cell faces, half a spacing from the first node: a link
  through a wall with a fixed temperature is half as long, so its weight is
  doubled; a walker taking it is absorbed and records T_w.  A step into an
  adiabatic wall is refused and the walker stays (zero gradient).  The
  estimate is the mean of N recorded temperatures (Eq 102).
* Random numbers: splitmix64 (Steele, Lea and Flood, 2014; the constants
  of Vigna's published reference code), one counter-based stream per
  (node, walker): draw k is mix(s0 + (k + 1) * gamma) with
  s0 = mix(seed + (1 + node * N + walker) * gamma), and RN = (draw >> 11)
  * 2^-53.  Eq 101 picks x+, y+, x-, y- by the cumulative thresholds
  P_x+, P_x+ + P_y+, P_x+ + P_y+ + P_x-, all in FP64.
* The coupled method alternates lattice steps (D2Q9 BGK with the Eq 18 /
  Eq 81 buoyancy from the node temperatures) and MCM solves with the
  velocity of the last lattice step: one solve after every S lattice steps.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .gs2 import GS2Case

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def link_weights(u, v, al, fe=1.0, fn=1.0, fw=1.0, fs=1.0):
    """Eq 99's link weights (x+, y+, x-, y-); f* = 2 doubles a link through a
    fixed-temperature wall."""
    return fe * (al - u), fn * (al - v), fw * al, fs * al


def probabilities(u, v, al, fe=1.0, fn=1.0, fw=1.0, fs=1.0):
    """(P_x+, P_y+, P_x-, P_y-) of Eq 99 / Eq 100."""
    a, b, c, d = link_weights(u, v, al, fe, fn, fw, fs)
    D = ((a + b) + c) + d
    return a / D, b / D, c / D, d / D


def wall_factors(nx, ny, tfix):
    """Per-node doubling factors (east, north, west, south) of the links
    through fixed-temperature walls."""
    fe = np.ones((ny, nx)); fn = np.ones((ny, nx)); fw = np.ones((ny, nx)); fs = np.ones((ny, nx))
    if tfix[1]: fe[:, -1] = 2.0
    if tfix[3]: fn[-1, :] = 2.0
    if tfix[0]: fw[:, 0] = 2.0
    if tfix[2]: fs[0, :] = 2.0
    return fe, fn, fw, fs


def exact_expectation(u, v, al, tfix, Tw):
    """The field the estimator converges to: Eq 97 at every node with the
    wall rules above, solved directly.  u, v: [ny][nx]."""
    ny, nx = u.shape
    pxp, pyp, pxm, pym = probabilities(u, v, al, *wall_factors(nx, ny, tfix))
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    diag = np.ones((ny, nx))
    rhs = np.zeros((ny, nx))
    rows, cols, vals = [], [], []
    # (probability, neighbour offset, wall side when the neighbour is outside)
    for P, dj, di, side in ((pxp, 0, 1, 1), (pxm, 0, -1, 0), (pyp, 1, 0, 3), (pym, -1, 0, 2)):
        J, I = np.mgrid[0:ny, 0:nx]
        Jn, In = J + dj, I + di
        inside = (Jn >= 0) & (Jn < ny) & (In >= 0) & (In < nx)
        rows.append(idx[inside]); cols.append(idx[Jn[inside], In[inside]]); vals.append(-P[inside])
        out = ~inside
        if tfix[side]:
            rhs[out] += P[out] * Tw[side]
        else:  # refused step: the walker stays
            diag[out] -= P[out]
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(diag.ravel())
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), (n, n))
    return spla.spsolve(A.tocsc(), rhs.ravel()).reshape(ny, nx)


def walk(i, j, walker, N, seed, u, v, al, tfix, Tw, max_steps):
    """One walker from node (i, j): (recorded temperature or None, steps)."""
    ny, nx = u.shape
    node = j * nx + i
    s0 = mix64(seed + (1 + node * N + walker) * GAMMA)
    for k in range(max_steps):
        rn = (mix64(s0 + (k + 1) * GAMMA) >> 11) * (1.0 / 9007199254740992.0)
        f = (2.0 if tfix[1] and i == nx - 1 else 1.0, 2.0 if tfix[3] and j == ny - 1 else 1.0,
             2.0 if tfix[0] and i == 0 else 1.0, 2.0 if tfix[2] and j == 0 else 1.0)
        pxp, pyp, pxm, _ = probabilities(float(u[j, i]), float(v[j, i]), al, *f)
        c1 = pxp
        c2 = c1 + pyp
        c3 = c2 + pxm
        if rn < c1:
            ti, tj, side = i + 1, j, 1
        elif rn < c2:
            ti, tj, side = i, j + 1, 3
        elif rn < c3:
            ti, tj, side = i - 1, j, 0
        else:
            ti, tj, side = i, j - 1, 2
        if 0 <= ti < nx and 0 <= tj < ny:
            i, j = ti, tj
        elif tfix[side]:
            return Tw[side], k + 1
    return None, max_steps


class MCMCase(GS2Case):
    """Coupled LBM-MCM on one grid; the temperature solve is the estimator's
    expectation (N -> infinity), so the reference is deterministic."""

    def __init__(self, nx: int, ny: int, S: int = 100):
        super().__init__(nx if nx % 2 == 0 else nx + 1, ny if ny % 2 == 0 else ny + 1, S=S)
        self.nx, self.ny = nx, ny

    def init(self, T=None):
        super().init()
        self.f = self.f[:, :self.ny, :self.nx].copy()
        self.rho = np.ones((self.ny, self.nx))
        self.ux = np.zeros((self.ny, self.nx))
        self.uy = np.zeros((self.ny, self.nx))
        self.Tf = np.zeros((self.ny, self.nx)) if T is None else np.array(T, dtype=np.float64)
        self.steps = 0
        return self

    def energy_step(self):
        self.Tf = exact_expectation(self.ux, self.uy, self.alpha, self.tfix, self.Tw)

    def step(self, n: int):
        for _ in range(n):
            self.lbm_step()
            self.steps += 1
            if self.steps % self.S == 0:
                self.energy_step()
        return self

    def nusselt(self):
        """Half-cell wall flux, nu(j) = 2 ny (T_w - T_edge) / dT (Eq 90)."""
        dT = self.Tw[0] - self.Tw[1]
        dT = dT if dT != 0 else 1.0
        hot = 2.0 * self.ny * (self.Tw[0] - self.Tf[:, 0]) / dT
        cold = 2.0 * self.ny * (self.Tf[:, -1] - self.Tw[1]) / dT
        k = int(np.argmax(hot))
        return {"nu_hot": hot.mean(), "nu_cold": cold.mean(), "nu_hot_max": hot[k],
                "y_hot_max": (k + 0.5) / self.ny}
