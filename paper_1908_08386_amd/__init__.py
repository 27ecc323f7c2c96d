"""Python binding of liblbmfvm.so, the MI355X hybrid LBM-FVM library.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory (the workspace a case binds)
and the stream (torch's current stream on the chosen device).  Importing
this package fails loudly when the compiled library is absent; there is no
CPU fallback.

Entry points mirror include/lbmfvm.h:
    ctx = Context(device=0)
    c = Case(ctx, nx, ny, precision="f32")
    c.set_physics(Ra, Pr); c.set_cavity_walls(); c.init(T0)
    c.step(n); c.residual(); c.nusselt(); c.fetch("T")
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBMFVM_LIB") or os.path.join(_HERE, "liblbmfvm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_1908_08386_amd/build.py` "
        "(there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

# ---- constants (include/lbmfvm.h) -----------------------------------------
LF_OK, LF_EINVAL, LF_ENOMEM, LF_EWORKSPACE, LF_EDEVICE, LF_EUNSTABLE, LF_EDIVERGED, \
    LF_ENOTCONV, LF_ESTATE, LF_ENOTIMPL = range(10)
F32, F64 = 0, 1
MODE_HYBRID, MODE_SPLIT = 0, 1
IFACE_NEQ_EXTRAP, IFACE_FD_GRADIENT = 0, 1
CONV_QUICK, CONV_CENTRAL, CONV_UPWIND = 0, 1, 2
WALL_NOSLIP, WALL_PERIODIC = 0, 1
T_DIRICHLET, T_ADIABATIC, T_PERIODIC = 0, 1, 2
W, E, S, N = 0, 1, 2, 3
FIELD_U, FIELD_V, FIELD_T, FIELD_RHO = 0, 1, 2, 3
STOP_TOL, STOP_FLOOR = 1, 2
_FIELDS = {"u": FIELD_U, "v": FIELD_V, "T": FIELD_T, "rho": FIELD_RHO}
_STATUS = {0: "LF_OK", 1: "LF_EINVAL", 2: "LF_ENOMEM", 3: "LF_EWORKSPACE", 4: "LF_EDEVICE",
           5: "LF_EUNSTABLE", 6: "LF_EDIVERGED", 7: "LF_ENOTCONV", 8: "LF_ESTATE",
           9: "LF_ENOTIMPL"}


class lf_case_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("precision", ctypes.c_int),
                ("mode", ctypes.c_int), ("split_col", ctypes.c_int), ("overlap", ctypes.c_int),
                ("iface", ctypes.c_int)]


class lf_physics(ctypes.Structure):
    _fields_ = [("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("U_char", ctypes.c_double),
                ("T_ref", ctypes.c_double), ("conv", ctypes.c_int),
                ("body_gx", ctypes.c_double), ("body_gy", ctypes.c_double)]


class lf_wall(ctypes.Structure):
    _fields_ = [("vel", ctypes.c_int), ("u_wall", ctypes.c_double), ("thermal", ctypes.c_int),
                ("T_wall", ctypes.c_double)]


class lf_nusselt(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("nu_hot", "nu_cold", "nu_hot_max", "y_hot_max", "nu_cold_max", "y_cold_max",
                 "nu_hot_o2", "nu_cold_o2")]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64

_SIGS = {
    "lf_abi_version": (ctypes.c_int, []),
    "lf_last_error": (ctypes.c_char_p, []),
    "lf_ctx_create": (ctypes.c_int, [ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "lf_ctx_destroy": (ctypes.c_int, [_vp]),
    "lf_ctx_set_band": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lf_case_create": (ctypes.c_int, [_vp, ctypes.POINTER(lf_case_desc), ctypes.POINTER(_vp)]),
    "lf_case_destroy": (ctypes.c_int, [_vp]),
    "lf_case_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "lf_case_bind_workspace": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "lf_case_set_physics": (ctypes.c_int, [_vp, ctypes.POINTER(lf_physics)]),
    "lf_case_set_lattice": (ctypes.c_int, [_vp] + [ctypes.c_double] * 6 + [ctypes.c_int]),
    "lf_case_set_wall": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(lf_wall)]),
    "lf_case_get_params": (ctypes.c_int, [_vp, _dp]),
    "lf_case_init": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "lf_case_step": (ctypes.c_int, [_vp, _i64]),
    "lf_case_residual": (ctypes.c_int, [_vp, _dp]),
    "lf_case_run_to_steady": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int, _i64,
                                             ctypes.POINTER(_i64), _dp,
                                             ctypes.POINTER(ctypes.c_int)]),
    "lf_case_nusselt": (ctypes.c_int, [_vp, ctypes.POINTER(lf_nusselt)]),
    "lf_case_fetch": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_size_t, ctypes.c_int,
                                     ctypes.c_int]),
    "lf_case_mass": (ctypes.c_int, [_vp, _dp, _dp]),
    "lf_case_steps": (ctypes.c_int, [_vp, ctypes.POINTER(_i64)]),
    "lf_case_profile_steps": (ctypes.c_int, [_vp, _i64, _dp, _dp, _dp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def lib() -> ctypes.CDLL:
    return _lib


class LFError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.lf_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(st: int, where: str):
    if st != LF_OK:
        raise LFError(st, where)


def _dptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _torch_stream_ptr(device: int):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """A HIP device and stream (torch's current stream on that device)."""

    def __init__(self, device: int = 0, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm GPU visible: the library runs on MI355X only")
        self.device = int(device)
        s = _torch_stream_ptr(self.device) if stream is None else ctypes.c_void_p(int(stream))
        h = _vp()
        _check(_lib.lf_ctx_create(self.device, s, ctypes.byref(h)), "lf_ctx_create")
        self._h = h

    def set_band(self, rows: int):
        _check(_lib.lf_ctx_set_band(self._h, int(rows)), "lf_ctx_set_band")

    def close(self):
        if getattr(self, "_h", None):
            _lib.lf_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Case:
    """One cavity (Mode H).  Fields are numpy arrays of shape (ny, nx)."""

    def __init__(self, ctx: Context, nx: int, ny: int, precision: str = "f32",
                 mode: int = MODE_HYBRID, split_col: int = 0, iface: int = IFACE_NEQ_EXTRAP):
        self.ctx = ctx
        self.nx, self.ny = int(nx), int(ny)
        self.precision = F64 if precision in ("f64", F64, "fp64", "double") else F32
        d = lf_case_desc(self.nx, self.ny, self.precision, int(mode), int(split_col), 0, int(iface))
        h = _vp()
        _check(_lib.lf_case_create(ctx._h, ctypes.byref(d), ctypes.byref(h)), "lf_case_create")
        self._h = h
        nb = ctypes.c_size_t()
        _check(_lib.lf_case_workspace_bytes(h, ctypes.byref(nb)), "lf_case_workspace_bytes")
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8,
                                     device=f"cuda:{ctx.device}")
        _check(_lib.lf_case_bind_workspace(h, ctypes.c_void_p(self.workspace.data_ptr()),
                                           nb.value), "lf_case_bind_workspace")

    def close(self):
        if getattr(self, "_h", None):
            _lib.lf_case_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # ---- set-up ------------------------------------------------------------
    def set_physics(self, Ra, Pr, U_char=0.0, T_ref=float("nan"), conv=CONV_QUICK,
                    body_gx=0.0, body_gy=0.0):
        p = lf_physics(float(Ra), float(Pr), float(U_char), float(T_ref), int(conv),
                       float(body_gx), float(body_gy))
        _check(_lib.lf_case_set_physics(self._h, ctypes.byref(p)), "lf_case_set_physics")
        return self

    def set_lattice(self, nu, alpha, gbeta=0.0, T_ref=0.0, gx=0.0, gy=0.0, conv=CONV_QUICK):
        _check(_lib.lf_case_set_lattice(self._h, float(nu), float(alpha), float(gbeta),
                                        float(T_ref), float(gx), float(gy), int(conv)),
               "lf_case_set_lattice")
        return self

    def set_wall(self, side, vel=WALL_NOSLIP, u_wall=0.0, thermal=T_ADIABATIC, T_wall=0.0):
        w = lf_wall(int(vel), float(u_wall), int(thermal), float(T_wall))
        _check(_lib.lf_case_set_wall(self._h, int(side), ctypes.byref(w)), "lf_case_set_wall")
        return self

    def set_cavity_walls(self, T_hot=0.5, T_cold=-0.5):
        self.set_wall(W, WALL_NOSLIP, 0.0, T_DIRICHLET, T_hot)
        self.set_wall(E, WALL_NOSLIP, 0.0, T_DIRICHLET, T_cold)
        self.set_wall(S, WALL_NOSLIP, 0.0, T_ADIABATIC, 0.0)
        self.set_wall(N, WALL_NOSLIP, 0.0, T_ADIABATIC, 0.0)
        return self

    def params(self) -> dict:
        out = np.zeros(8)
        _check(_lib.lf_case_get_params(self._h, _dptr(out)), "lf_case_get_params")
        return dict(zip(["U_char", "nu", "tau", "alpha", "tau_T", "gbeta", "T_ref", "Ma"],
                        out.tolist()))

    def init(self, T0=None, u0=None, v0=None):
        shape = (self.ny, self.nx)
        arrs = [None if a is None else
                np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), shape))
                for a in (T0, u0, v0)]
        _check(_lib.lf_case_init(self._h, *[_dptr(a) for a in arrs]), "lf_case_init")
        return self

    # ---- stepping ----------------------------------------------------------
    def step(self, n: int = 1):
        _check(_lib.lf_case_step(self._h, int(n)), "lf_case_step")
        return self

    def profile_steps(self, n: int):
        """Run n steps timing every step kernel with HIP events: (avg, min, max) ms."""
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(_lib.lf_case_profile_steps(self._h, int(n), ctypes.byref(a), ctypes.byref(b),
                                          ctypes.byref(c)), "lf_case_profile_steps")
        return a.value, b.value, c.value

    @property
    def steps(self) -> int:
        v = _i64()
        _check(_lib.lf_case_steps(self._h, ctypes.byref(v)), "lf_case_steps")
        return v.value

    def residual(self) -> np.ndarray:
        r = np.zeros(3)
        _check(_lib.lf_case_residual(self._h, _dptr(r)), "lf_case_residual")
        return r

    def run_to_steady(self, tol=1e-8, check_every=1000, max_steps=10**7, raise_on_notconv=True):
        steps = _i64()
        r = np.zeros(3)
        rule = ctypes.c_int()
        st = _lib.lf_case_run_to_steady(self._h, float(tol), int(check_every), int(max_steps),
                                        ctypes.byref(steps), _dptr(r), ctypes.byref(rule))
        if st != LF_OK and not (st == LF_ENOTCONV and not raise_on_notconv):
            raise LFError(st, "lf_case_run_to_steady")
        return steps.value, r, rule.value

    # ---- observables -------------------------------------------------------
    def nusselt(self) -> dict:
        o = lf_nusselt()
        _check(_lib.lf_case_nusselt(self._h, ctypes.byref(o)), "lf_case_nusselt")
        return {k: getattr(o, k) for k, _ in lf_nusselt._fields_}

    def fetch(self, field) -> np.ndarray:
        out = np.empty((self.ny, self.nx), dtype=np.float64)
        _check(_lib.lf_case_fetch(self._h, _FIELDS.get(field, field),
                                  out.ctypes.data_as(_vp), out.nbytes, 0, 1), "lf_case_fetch")
        return out

    def fetch_device(self, field, out: torch.Tensor):
        """Copy a field into a device tensor (float64, or the case precision)."""
        as64 = 1 if out.dtype == torch.float64 else 0
        _check(_lib.lf_case_fetch(self._h, _FIELDS.get(field, field),
                                  ctypes.c_void_p(out.data_ptr()),
                                  out.numel() * out.element_size(), 1, as64), "lf_case_fetch")
        return out

    def mass(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(_lib.lf_case_mass(self._h, ctypes.byref(a), ctypes.byref(b)), "lf_case_mass")
        return a.value, b.value
