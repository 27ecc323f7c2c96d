"""Plain FP64 CPU oracle for the hybrid LBM-FVM method (arXiv:1908.08386).

TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP
library (``paper_1908_08386_amd``) and never imports it.

The arithmetic lives in ``lbmfvm_oracle.c`` (Mode H, Sec. 5) and
``dd_oracle.c`` (domain decomposition, Sec. 4); this module only marshals
numpy arrays through ctypes.  ``net.py`` is the numpy FP64 reference of the
learned initial guess (not part of the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbmfvm_oracle.so")
_SOURCES = ["lbmfvm_oracle.c", "dd_oracle.c"]

W, E, S, N = 0, 1, 2, 3
VEL_NOSLIP, VEL_PERIODIC = 0, 1
T_FIXED, T_ADIABATIC, T_PERIODIC = 0, 1, 2
CONV_QUICK, CONV_CENTRAL, CONV_UPWIND = 0, 1, 2
FIELD_U, FIELD_V, FIELD_T, FIELD_RHO = 0, 1, 2, 3
IFACE_NEQ, IFACE_FDGRAD = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    if not force and os.path.exists(_LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs)
        if os.path.getmtime(_LIB_PATH) >= newest:
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.oc_create.restype = vp
        L.oc_create.argtypes = [ctypes.c_int, ctypes.c_int]
        L.oc_destroy.argtypes = [vp]
        L.oc_set_lattice.argtypes = [vp] + [ctypes.c_double] * 6 + [ctypes.c_int]
        L.oc_set_wall.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_double]
        L.oc_init.argtypes = [vp, dp, dp, dp]
        L.oc_step.argtypes = [vp, ctypes.c_long]
        L.oc_steps.restype = ctypes.c_long
        L.oc_steps.argtypes = [vp]
        L.oc_fetch.argtypes = [vp, ctypes.c_int, dp]
        L.oc_fetch_f.argtypes = [vp, dp]
        L.oc_residual.argtypes = [vp, dp]
        L.oc_nusselt.argtypes = [vp, dp]
        L.oc_mass.argtypes = [vp, dp, dp]
        L.oc_physics_params.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_int, dp]
        L.oc_set_threads.argtypes = [ctypes.c_int]
        L.oc_feq.argtypes = [ctypes.c_double] * 3 + [dp]
        L.oc_force.argtypes = [ctypes.c_double] * 5 + [dp]
        L.oc_collide_node.argtypes = [dp] + [ctypes.c_double] * 6 + [dp]
        L.oc_geq5.argtypes = [ctypes.c_double] * 3 + [dp]
        if hasattr(L, "dd_create"):
            L.dd_create.restype = vp
            L.dd_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
            L.dd_destroy.argtypes = [vp]
            L.dd_set_wall.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_double]
            L.dd_set_lattice.argtypes = [vp] + [ctypes.c_double] * 5 + [ctypes.c_int]
            L.dd_init.argtypes = [vp, dp]
            L.dd_step.argtypes = [vp, ctypes.c_long]
            L.dd_fetch.argtypes = [vp, ctypes.c_int, dp]
            L.dd_nusselt.argtypes = [vp, dp]
            L.dd_residual.argtypes = [vp, dp]
            L.dd_reconstruct_node.argtypes = [ctypes.c_int, dp, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, dp]
            L.dd_boundary_density.restype = ctypes.c_double
            L.dd_boundary_density.argtypes = [ctypes.c_double] * 3
            L.dd_set_iface.argtypes = [vp, ctypes.c_int]
            L.dd_steps.restype = ctypes.c_long
            L.dd_steps.argtypes = [vp]
            L.dd_init_uniform_flow.argtypes = [vp, dp, ctypes.c_double, ctypes.c_double]
            L.dd_set_fv.argtypes = [vp, dp, dp, dp]
            L.dd_set_gdir.argtypes = [vp, ctypes.c_int]
            L.dd_set_lid.argtypes = [vp, ctypes.c_double]
            L.dd_set_level.argtypes = [vp, ctypes.c_double, ctypes.c_double]
            L.dd_zone_mass.restype = ctypes.c_double
            L.dd_zone_mass.argtypes = [vp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n: int) -> int:
    return lib().oc_set_threads(int(n))


def physics_params(Ra: float, Pr: float, H: int, U_char: float = 0.0, split: bool = False):
    """(U_c, nu, tau, alpha, tau_T, g*beta, T_ref, Ma) from Ra, Pr, H (Eq 82-89)."""
    out = np.zeros(8)
    rc = lib().oc_physics_params(float(Ra), float(Pr), int(H), float(U_char), int(split), _dp(out))
    if rc != 0:
        raise ValueError("invalid physical parameters")
    return dict(zip(["U_char", "nu", "tau", "alpha", "tau_T", "gbeta", "T_ref", "Ma"], out.tolist()))


def feq(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().oc_feq(rho, ux, uy, _dp(out))
    return out


def force(rho: float, ux: float, uy: float, Gx: float, Gy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().oc_force(rho, ux, uy, Gx, Gy, _dp(out))
    return out


def collide_node(f_pre, T, tau, gbeta, T_ref=0.0, gx=0.0, gy=0.0) -> np.ndarray:
    fp = np.ascontiguousarray(f_pre, dtype=np.float64)
    out = np.zeros(9)
    lib().oc_collide_node(_dp(fp), T, tau, gbeta, T_ref, gx, gy, _dp(out))
    return out


def geq5(T: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(5)
    lib().oc_geq5(T, ux, uy, _dp(out))
    return out


class Case:
    """Mode H cavity (whole-domain LBM velocity + FVM temperature)."""

    def __init__(self, nx: int, ny: int):
        self.nx, self.ny = int(nx), int(ny)
        self._h = lib().oc_create(self.nx, self.ny)
        if not self._h:
            raise MemoryError("oc_create failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oc_destroy(h)
            self._h = None

    def set_lattice(self, nu, alpha, gbeta=0.0, T_ref=0.0, gx=0.0, gy=0.0, conv=CONV_QUICK):
        if lib().oc_set_lattice(self._h, nu, alpha, gbeta, T_ref, gx, gy, int(conv)) != 0:
            raise ValueError("bad lattice parameters")
        return self

    def set_physics(self, Ra, Pr, U_char=0.0, T_ref=0.0):
        p = physics_params(Ra, Pr, self.ny, U_char)
        self.params = p
        return self.set_lattice(p["nu"], p["alpha"], p["gbeta"], T_ref)

    def set_wall(self, side, vel=VEL_NOSLIP, u_wall=0.0, thermal=T_ADIABATIC, T_wall=0.0):
        lib().oc_set_wall(self._h, int(side), int(vel), float(u_wall), int(thermal), float(T_wall))
        return self

    def set_cavity_walls(self, T_hot=0.5, T_cold=-0.5):
        """Side-heated cavity: hot west, cold east, adiabatic south/north, no slip."""
        self.set_wall(W, VEL_NOSLIP, 0.0, T_FIXED, T_hot)
        self.set_wall(E, VEL_NOSLIP, 0.0, T_FIXED, T_cold)
        self.set_wall(S, VEL_NOSLIP, 0.0, T_ADIABATIC, 0.0)
        self.set_wall(N, VEL_NOSLIP, 0.0, T_ADIABATIC, 0.0)
        return self

    def init(self, T0=None, u0=None, v0=None):
        shape = (self.ny, self.nx)
        arrs = []
        for a in (T0, u0, v0):
            if a is None:
                arrs.append(None)
            else:
                a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape))
                arrs.append(a)
        ptrs = [(_dp(a) if a is not None else None) for a in arrs]
        self._keep = arrs
        lib().oc_init(self._h, *ptrs)
        return self

    def step(self, n: int):
        lib().oc_step(self._h, int(n))
        return self

    @property
    def steps(self) -> int:
        return lib().oc_steps(self._h)

    def fetch(self, field) -> np.ndarray:
        idx = {"u": FIELD_U, "v": FIELD_V, "T": FIELD_T, "rho": FIELD_RHO}.get(field, field)
        out = np.empty((self.ny, self.nx))
        if lib().oc_fetch(self._h, int(idx), _dp(out)) != 0:
            raise ValueError(field)
        return out

    def fetch_f(self) -> np.ndarray:
        out = np.empty((9, self.ny, self.nx))
        lib().oc_fetch_f(self._h, _dp(out))
        return out

    def residual(self) -> np.ndarray:
        r = np.zeros(3)
        lib().oc_residual(self._h, _dp(r))
        return r

    def nusselt(self) -> dict:
        out = np.zeros(8)
        lib().oc_nusselt(self._h, _dp(out))
        keys = ["nu_hot", "nu_cold", "nu_hot_max", "y_hot_max", "nu_cold_max",
                "y_cold_max", "nu_hot_o2", "nu_cold_o2"]
        return dict(zip(keys, out.tolist()))

    def mass(self):
        a = ctypes.c_double()
        b = ctypes.c_double()
        lib().oc_mass(self._h, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def run_to_steady(self, tol=1e-8, check_every=1000, max_steps=10**7, fields=(0, 1, 2)):
        """Step in blocks of ``check_every`` until the largest residual of the
        chosen fields (0 u, 1 v, 2 T) is <= tol, or all of them are 0."""
        self.residual()  # snapshot the current state
        sel = list(fields)
        r = np.zeros(3)
        while self.steps < max_steps:
            self.step(check_every)
            r = self.residual()
            if r[sel].max() <= tol or not np.any(r[sel]):
                return self.steps, r
        return self.steps, r


SPLIT, PURE_FV, PURE_LBM = 0, 1, 2


def reconstruct_node(kind, f_f, rho_b, ub, vb, tau, dudx=0.0, dudy=0.0, dvdx=0.0):
    """Populations of the LBM artificial-boundary node (Eq 60 or Eq 70)."""
    ff = np.ascontiguousarray(f_f, dtype=np.float64)
    out = np.zeros(9)
    lib().dd_reconstruct_node(int(kind), _dp(ff), rho_b, ub, vb, tau, dudx, dudy, dvdx, _dp(out))
    return out


def boundary_density(rho0, pS, pbar):
    """Eq 93."""
    return lib().dd_boundary_density(float(rho0), float(pS), float(pbar))


class DDCase:
    """Domain-decomposed cavity (mode SPLIT: LBM west half, FV east half),
    or one of the single-method cavities (PURE_FV, PURE_LBM)."""

    def __init__(self, nx: int, ny: int, mode: int = SPLIT, iface: int = IFACE_NEQ):
        self.nx, self.ny, self.mode = int(nx), int(ny), int(mode)
        self._h = lib().dd_create(self.nx, self.ny, self.mode)
        if not self._h:
            raise ValueError("dd_create: bad size or mode")
        lib().dd_set_iface(self._h, int(iface))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().dd_destroy(h)
            self._h = None

    def set_lattice(self, nu, alpha, gbeta=0.0, T_ref=0.0, gx=0.0, conv=CONV_QUICK):
        if lib().dd_set_lattice(self._h, nu, alpha, gbeta, T_ref, gx, int(conv)) != 0:
            raise ValueError("bad lattice parameters")
        return self

    def set_physics(self, Ra, Pr, U_char=0.0, T_ref=0.0):
        p = physics_params(Ra, Pr, self.ny, U_char, split=True)
        self.params = p
        return self.set_lattice(p["nu"], p["alpha"], p["gbeta"], T_ref)

    def set_gravity_axis(self, axis: str):
        """'y' (default: gravity along -y) or 'x' (gravity along -x, buoyancy
        on the x-faces): the horizontally divided cavity stored transposed."""
        lib().dd_set_gdir(self._h, 1 if axis == "x" else 0)
        return self

    def set_thermal(self, side, fixed: bool, T_wall=0.0):
        lib().dd_set_wall(self._h, int(side), 0.0, 1 if fixed else 0, float(T_wall))
        return self

    def set_lid(self, u_wall: float):
        """The north wall slides along +x at u_wall (lattice units)."""
        if lib().dd_set_lid(self._h, float(u_wall)) != 0:
            raise ValueError("no sliding wall on a periodic axis")
        return self

    def set_level_gains(self, kp: float, ki: float):
        """Gains of the level of Eq 93 on the LBM zone's mass deficit and on
        its running sum (split mode)."""
        if lib().dd_set_level(self._h, float(kp), float(ki)) != 0:
            raise ValueError("dd_set_level: gains must be >= 0")
        return self

    def zone_mass(self) -> float:
        """Split mode: mass of the LBM nodes west of x_b (post-collision)."""
        return lib().dd_zone_mass(self._h)

    def set_periodic(self, axis: str):
        side = W if axis == "x" else S
        if lib().dd_set_wall(self._h, side, 0.0, 1 << 4, 0.0) != 0:
            raise ValueError("periodic sides only in the single-method modes")
        return self

    def set_cavity_walls(self, T_hot=0.5, T_cold=-0.5):
        self.set_thermal(W, True, T_hot).set_thermal(E, True, T_cold)
        return self.set_thermal(S, False).set_thermal(N, False)

    def init(self, T0=None, uniform_flow=None):
        T = None if T0 is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(T0, np.float64), (self.ny, self.nx)))
        self._keep = T
        if uniform_flow is None:
            lib().dd_init(self._h, _dp(T) if T is not None else None)
        else:
            lib().dd_init_uniform_flow(self._h, _dp(T) if T is not None else None,
                                       float(uniform_flow[0]), float(uniform_flow[1]))
        return self

    def set_fv(self, p=None, u=None, v=None):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (p, u, v)]
        self._keep_fv = arrs
        lib().dd_set_fv(self._h, *[(_dp(a) if a is not None else None) for a in arrs])
        return self

    def step(self, n: int):
        lib().dd_step(self._h, int(n))
        return self

    @property
    def steps(self) -> int:
        return lib().dd_steps(self._h)

    def fetch(self, field) -> np.ndarray:
        idx = {"u": 0, "v": 1, "T": 2, "rho": 3, "p": 4, "u_faces": 5, "v_faces": 6}[field]
        shape = {5: (self.ny, self.nx + 1), 6: (self.ny + 1, self.nx)}.get(idx, (self.ny, self.nx))
        out = np.empty(shape)
        if lib().dd_fetch(self._h, idx, _dp(out)) != 0:
            raise ValueError(field)
        return out

    def residual(self) -> np.ndarray:
        r = np.zeros(3)
        lib().dd_residual(self._h, _dp(r))
        return r

    def nusselt(self) -> dict:
        out = np.zeros(8)
        lib().dd_nusselt(self._h, _dp(out))
        keys = ["nu_hot", "nu_cold", "nu_hot_max", "y_hot_max", "nu_cold_max",
                "y_cold_max", "nu_hot_o2", "nu_cold_o2"]
        return dict(zip(keys, out.tolist()))

    def run_to_steady(self, tol=1e-8, check_every=1000, max_steps=10**7, fields=(0, 1, 2)):
        self.residual()
        sel = list(fields)
        r = np.zeros(3)
        while self.steps < max_steps:
            self.step(check_every)
            r = self.residual()
            if r[sel].max() <= tol or not np.any(r[sel]):
                break
        return self.steps, r
