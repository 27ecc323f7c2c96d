"""Plain FP64 numpy reference of the hybrid on grid setting 2 (Sec. 5.1).

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle/``): it checks
the GPU library and is never called by it.

What it computes (the readings are listed with the design notes):

* The velocity lives on a fine 2NX x 2NY lattice (nx = 2NX, ny = 2NY
  nodes at the fine cell centres), the temperature on a coarse NX x NY
  finite-volume grid whose cell (I, J) covers the fine cells
  {2I, 2I+1} x {2J, 2J+1} (cell size h = 2 lattice units, Fig. 30).
* Every lattice step is D2Q9 BGK with pull streaming, half-way bounce-back
  at walls at rest, and the buoyancy force of Eq 18 with G = (0, g beta
  (T - T_ref)) (Eq 81), T being the coarse field interpolated bilinearly to
  the fine node (wall ghosts: 2 T_w - T for a fixed wall, T for an
  adiabatic one).  T is held fixed between energy steps.
* After every S lattice steps (the paper: S = 2NX) one finite-volume energy
  step of length S advances T implicitly (backward Euler): upwind
  convection and central diffusion in the matrix, the QUICK minus upwind
  face-value difference taken from the old T as a deferred correction, the
  face velocities being the averages of the four fine-node velocities that
  straddle each coarse face (from the last lattice step).  The linear
  system is solved approximately by K alternating-direction line sweeps
  (x-lines, then y-lines, each line by the Thomas algorithm with the other
  direction's neighbours from the previous iterate), starting from the old
  T, or (solver="direct") exactly by a sparse direct solve.  A fixed point
  of the sweeps satisfies the whole system (a line relaxation that returns
  its start solves it), so the steady state does not depend on K and the
  direct solve is its K-free reference.
"""
from __future__ import annotations

import numpy as np

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WQ = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
SW, SE, SS, SN = 0, 1, 2, 3


def thomas(lo, di, up, rhs):
    """Solve the tridiagonal systems lo[k] x[k-1] + di[k] x[k] + up[k] x[k+1]
    = rhs[k] along the last axis (lo[0] and up[-1] unused), by forward
    elimination and back substitution."""
    n = di.shape[-1]
    cp = np.empty_like(di)
    rp = np.empty_like(di)
    cp[..., 0] = up[..., 0] / di[..., 0]
    rp[..., 0] = rhs[..., 0] / di[..., 0]
    for k in range(1, n):
        m = di[..., k] - lo[..., k] * cp[..., k - 1]
        cp[..., k] = up[..., k] / m
        rp[..., k] = (rhs[..., k] - lo[..., k] * rp[..., k - 1]) / m
    x = np.empty_like(di)
    x[..., n - 1] = rp[..., n - 1]
    for k in range(n - 2, -1, -1):
        x[..., k] = rp[..., k] - cp[..., k] * x[..., k + 1]
    return x


def quick_face(w, ll, l, r, rr):
    """Leonard's QUICK face value for a face between cells l and r."""
    return np.where(w >= 0.0, (6.0 * l + 3.0 * r - ll) / 8.0, (6.0 * r + 3.0 * l - rr) / 8.0)


class GS2Case:
    def __init__(self, nx: int, ny: int, S: int = 0, K: int = 4, solver: str = "adi"):
        if nx % 2 or ny % 2 or nx < 8 or ny < 8:
            raise ValueError("nx and ny must be even and >= 8")
        if solver not in ("adi", "direct"):
            raise ValueError("solver is 'adi' or 'direct'")
        self.solver = solver
        self.nx, self.ny = nx, ny
        self.NX, self.NY = nx // 2, ny // 2
        self.S = S if S > 0 else nx  # lattice steps per energy step (2NX)
        self.K = K
        self.tfix = [1, 1, 0, 0]
        self.Tw = [0.5, -0.5, 0.0, 0.0]
        self.steps = 0

    # ---- parameters ---------------------------------------------------
    def set_lattice(self, nu, alpha, gbeta, T_ref=0.0):
        self.nu, self.alpha, self.gbeta, self.T_ref = nu, alpha, gbeta, T_ref
        self.tau = 3.0 * nu + 0.5
        return self

    def set_physics(self, Ra, Pr, U_char=0.0):
        from . import physics_params
        p = physics_params(Ra, Pr, self.ny, U_char)
        self.params = p
        return self.set_lattice(p["nu"], p["alpha"], p["gbeta"], 0.0)

    def set_thermal(self, side, fixed: bool, T_wall=0.0):
        self.tfix[side] = 1 if fixed else 0
        self.Tw[side] = float(T_wall)
        return self

    def init(self, Tc=None):
        """Rest state, f = w; coarse temperature Tc [NY][NX] (default 0)."""
        self.f = np.broadcast_to(WQ[:, None, None], (9, self.ny, self.nx)).copy()
        self.T = np.zeros((self.NY, self.NX)) if Tc is None else np.array(Tc, dtype=np.float64)
        self.Tf = self.interp(self.T)
        self.rho = np.ones((self.ny, self.nx))
        self.ux = np.zeros((self.ny, self.nx))
        self.uy = np.zeros((self.ny, self.nx))
        self.steps = 0
        return self

    # ---- coarse field with one ghost layer ------------------------------
    def ghosted(self, T):
        """(NY+2, NX+2): x ghosts on every row first, then y ghosts on every
        column (corners take both rules in that order)."""
        g = np.empty((self.NY + 2, self.NX + 2))
        g[1:-1, 1:-1] = T
        g[1:-1, 0] = 2.0 * self.Tw[SW] - T[:, 0] if self.tfix[SW] else T[:, 0]
        g[1:-1, -1] = 2.0 * self.Tw[SE] - T[:, -1] if self.tfix[SE] else T[:, -1]
        g[0, :] = 2.0 * self.Tw[SS] - g[1, :] if self.tfix[SS] else g[1, :]
        g[-1, :] = 2.0 * self.Tw[SN] - g[-2, :] if self.tfix[SN] else g[-2, :]
        return g

    def interp(self, T):
        """Bilinear values at the fine cell centres from the coarse cell
        centres: fine i sits at coarse coordinate (2i - 1) / 4, i.e. between
        coarse cells (i - 1) // 2 and that + 1 with weight 3/4 (i even) or
        1/4 (i odd) on the second."""
        g = self.ghosted(T)
        i = np.arange(self.nx)
        j = np.arange(self.ny)
        I0 = (i - 1) // 2 + 1  # ghosted index of the left coarse cell
        J0 = (j - 1) // 2 + 1
        wx = np.where(i % 2 == 0, 0.75, 0.25)
        wy = np.where(j % 2 == 0, 0.75, 0.25)
        T00 = g[J0[:, None], I0[None, :]]
        T10 = g[J0[:, None], I0[None, :] + 1]
        T01 = g[J0[:, None] + 1, I0[None, :]]
        T11 = g[J0[:, None] + 1, I0[None, :] + 1]
        wxr, wyc = wx[None, :], wy[:, None]
        return (1.0 - wyc) * ((1.0 - wxr) * T00 + wxr * T10) + wyc * ((1.0 - wxr) * T01 + wxr * T11)

    # ---- one lattice step ----------------------------------------------
    def lbm_step(self):
        ny, nx = self.ny, self.nx
        fp = np.empty_like(self.f)
        for q in range(9):
            src = np.full((ny, nx), np.nan)
            # node (i, j) pulls from (i - ex, j - ey)
            ys = slice(max(0, EY[q]), ny + min(0, EY[q]))
            xs = slice(max(0, EX[q]), nx + min(0, EX[q]))
            ysrc = slice(max(0, -EY[q]), ny + min(0, -EY[q]))
            xsrc = slice(max(0, -EX[q]), nx + min(0, -EX[q]))
            src[ys, xs] = self.f[q][ysrc, xsrc]
            # links through a wall at rest: half-way bounce-back
            src = np.where(np.isnan(src), self.f[OPP[q]], src)
            fp[q] = src
        rho = np.zeros((ny, nx))
        mx = np.zeros((ny, nx))
        my = np.zeros((ny, nx))
        for q in range(9):
            rho += fp[q]
            mx += EX[q] * fp[q]
            my += EY[q] * fp[q]
        ux, uy = mx / rho, my / rho
        Gy = self.gbeta * (self.Tf - self.T_ref)
        usq = ux * ux + uy * uy
        for q in range(9):
            eu = EX[q] * ux + EY[q] * uy
            feq = rho * WQ[q] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq)
            F = 3.0 * ((EY[q] - uy) * Gy) * feq / rho  # G . (e - u) f_eq / (rho c_s^2)
            self.f[q] = fp[q] - (fp[q] - feq) / self.tau + F
        self.rho, self.ux, self.uy = rho, ux, uy

    # ---- one energy step -----------------------------------------------
    def face_velocities(self):
        NX, NY, ux, uy = self.NX, self.NY, self.ux, self.uy
        U = np.zeros((NY, NX + 1))
        V = np.zeros((NY + 1, NX))
        I = np.arange(1, NX)
        J = np.arange(NY)
        U[:, 1:NX] = 0.25 * ((ux[2 * J[:, None], 2 * I[None, :] - 1] + ux[2 * J[:, None], 2 * I[None, :]]) +
                             (ux[2 * J[:, None] + 1, 2 * I[None, :] - 1] + ux[2 * J[:, None] + 1, 2 * I[None, :]]))
        J = np.arange(1, NY)
        I = np.arange(NX)
        V[1:NY, :] = 0.25 * ((uy[2 * J[:, None] - 1, 2 * I[None, :]] + uy[2 * J[:, None], 2 * I[None, :]]) +
                             (uy[2 * J[:, None] - 1, 2 * I[None, :] + 1] + uy[2 * J[:, None], 2 * I[None, :] + 1]))
        return U, V

    def assemble(self, U, V, T):
        """Coefficients of a_P T_P - a_W T_W - a_E T_E - a_S T_S - a_N T_N = b."""
        NX, NY, al, h = self.NX, self.NY, self.alpha, 2.0
        dt = float(self.S)
        g = self.ghosted(T)
        # deferred correction h w (T_QUICK - T_upwind) on the interior faces
        DCx = np.zeros((NY, NX + 1))
        w = U[:, 1:NX]
        TL, TR = T[:, 0:NX - 1], T[:, 1:NX]
        TLL, TRR = g[1:-1, 0:NX - 1], g[1:-1, 3:NX + 2]
        DCx[:, 1:NX] = h * w * (quick_face(w, TLL, TL, TR, TRR) - np.where(w >= 0.0, TL, TR))
        DCy = np.zeros((NY + 1, NX))
        w = V[1:NY, :]
        TL, TR = T[0:NY - 1, :], T[1:NY, :]
        TLL, TRR = g[0:NY - 1, 1:-1], g[3:NY + 2, 1:-1]
        DCy[1:NY, :] = h * w * (quick_face(w, TLL, TL, TR, TRR) - np.where(w >= 0.0, TL, TR))
        aW = np.zeros((NY, NX)); aE = np.zeros((NY, NX))
        aS = np.zeros((NY, NX)); aN = np.zeros((NY, NX))
        cW = np.zeros((NY, NX)); cE = np.zeros((NY, NX))
        cS = np.zeros((NY, NX)); cN = np.zeros((NY, NX))
        sW = np.zeros((NY, NX)); sE = np.zeros((NY, NX))
        sS = np.zeros((NY, NX)); sN = np.zeros((NY, NX))
        # west faces (x-face I of cell I)
        uw = U[:, 0:NX]
        aW[:, 1:] = al + h * np.maximum(uw[:, 1:], 0.0)
        cW[:, 1:] = al + h * np.maximum(-uw[:, 1:], 0.0)
        sW[:, 1:] = DCx[:, 1:NX]
        if self.tfix[SW]:
            cW[:, 0] = 2.0 * al
            sW[:, 0] = 2.0 * al * self.Tw[SW]
        # east faces (x-face I+1)
        ue = U[:, 1:NX + 1]
        aE[:, :-1] = al + h * np.maximum(-ue[:, :-1], 0.0)
        cE[:, :-1] = al + h * np.maximum(ue[:, :-1], 0.0)
        sE[:, :-1] = -DCx[:, 1:NX]
        if self.tfix[SE]:
            cE[:, -1] = 2.0 * al
            sE[:, -1] = 2.0 * al * self.Tw[SE]
        # south faces (y-face J)
        vs = V[0:NY, :]
        aS[1:, :] = al + h * np.maximum(vs[1:, :], 0.0)
        cS[1:, :] = al + h * np.maximum(-vs[1:, :], 0.0)
        sS[1:, :] = DCy[1:NY, :]
        if self.tfix[SS]:
            cS[0, :] = 2.0 * al
            sS[0, :] = 2.0 * al * self.Tw[SS]
        # north faces (y-face J+1)
        vn = V[1:NY + 1, :]
        aN[:-1, :] = al + h * np.maximum(-vn[:-1, :], 0.0)
        cN[:-1, :] = al + h * np.maximum(vn[:-1, :], 0.0)
        sN[:-1, :] = -DCy[1:NY, :]
        if self.tfix[SN]:
            cN[-1, :] = 2.0 * al
            sN[-1, :] = 2.0 * al * self.Tw[SN]
        ct = h * h / dt
        aP = (((ct + cW) + cE) + cS) + cN
        b = ((((ct * T) + sW) + sE) + sS) + sN
        return aP, aW, aE, aS, aN, b

    def adi(self, coef, X, sweeps):
        aP, aW, aE, aS, aN, b = coef
        for _ in range(sweeps):
            Xs = np.zeros_like(X); Xs[1:, :] = X[:-1, :]
            Xn = np.zeros_like(X); Xn[:-1, :] = X[1:, :]
            X = thomas(-aW, aP, -aE, (b + aS * Xs) + aN * Xn)           # x-lines
            Xw = np.zeros_like(X); Xw[:, 1:] = X[:, :-1]
            Xe = np.zeros_like(X); Xe[:, :-1] = X[:, 1:]
            X = thomas((-aS).T, aP.T, (-aN).T, ((b + aW * Xw) + aE * Xe).T).T  # y-lines
        return X

    def matrix(self, coef):
        """The five-point system a_P T_P - sum a_nb T_nb = b as a sparse
        matrix (rows and columns in row-major cell order)."""
        import scipy.sparse as sp
        aP, aW, aE, aS, aN, _ = coef
        n = aP.size
        idx = np.arange(n).reshape(aP.shape)
        rows, cols, vals = [idx.ravel()], [idx.ravel()], [aP.ravel()]
        for a, dj, di in ((aW, 0, -1), (aE, 0, 1), (aS, -1, 0), (aN, 1, 0)):
            J, I = np.nonzero(a)
            rows.append(idx[J, I])
            cols.append(idx[J + dj, I + di])
            vals.append(-a[J, I])
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             (n, n))

    def direct(self, coef):
        """The implicit energy step solved exactly (sparse LU)."""
        import scipy.sparse.linalg as spla
        b = coef[5]
        return spla.spsolve(self.matrix(coef).tocsc(), b.ravel()).reshape(b.shape)

    def fv_step(self):
        U, V = self.face_velocities()
        coef = self.assemble(U, V, self.T)
        if self.solver == "direct":
            self.T = self.direct(coef)
        else:
            self.T = self.adi(coef, self.T.copy(), self.K)
        self.Tf = self.interp(self.T)

    def step(self, n: int):
        for _ in range(n):
            self.lbm_step()
            self.steps += 1
            if self.steps % self.S == 0:
                self.fv_step()
        return self

    def run_to_steady(self, tol, cycles=16, max_steps=10**7):
        """Step in blocks of `cycles` energy cycles until the relative
        change of u, v and T over a block, ||phi - phi_prev||_2 / ||phi||_2,
        is at most tol.  Returns the steps taken and the last changes."""
        K = cycles * self.S
        prev = [self.ux.copy(), self.uy.copy(), self.Tf.copy()]
        r = np.full(3, np.inf)
        while self.steps < max_steps:
            self.step(K)
            cur = [self.ux, self.uy, self.Tf]
            r = np.array([np.linalg.norm(a - b) / max(np.linalg.norm(a), 1e-300)
                          for a, b in zip(cur, prev)])
            prev = [a.copy() for a in cur]
            if r.max() <= tol:
                break
        return self.steps, r

    # ---- observables ---------------------------------------------------
    def fetch(self, field):
        return {"u": self.ux, "v": self.uy, "T": self.Tf, "rho": self.rho}[field].copy()

    def nusselt(self):
        """Wall-averaged Nusselt numbers from the half-cell wall flux of the
        fine field, nu(j) = 2 ny (T_w - T_edge) / dT (Eq 90 with X = x / ny)."""
        dT = self.Tw[SW] - self.Tw[SE]
        dT = dT if dT != 0 else 1.0
        hot = 2.0 * self.ny * (self.Tw[SW] - self.Tf[:, 0]) / dT
        cold = 2.0 * self.ny * (self.Tf[:, -1] - self.Tw[SE]) / dT
        k = int(np.argmax(hot))
        return {"nu_hot": hot.mean(), "nu_cold": cold.mean(), "nu_hot_max": hot[k],
                "y_hot_max": (k + 0.5) / self.ny}
