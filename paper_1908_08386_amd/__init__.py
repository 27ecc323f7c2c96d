"""Python binding of liblbmfvm.so, the MI355X hybrid LBM-FVM library.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory (the workspace a case binds)
and the stream (torch's current stream on the chosen device).  Importing
this package fails loudly when the compiled library is absent; there is no
CPU fallback.

Entry points mirror include/lbmfvm.h:
    ctx = Context(device=0)
    c = Case(ctx, nx, ny, precision="f32")          # lf_case_*
    c.set_physics(Ra, Pr); c.set_cavity_walls(); c.init(T0)
    c.step(n); c.residual(); c.nusselt(); c.fetch("T"); c.save() / c.load(blob)
    b = Batch(ctx, cases); b.init(T0s); b.run_to_steady()   # lf_batch_*
    net = Net(ctx); net.train_step(...); net.forward(...)    # lf_net_*
    resample(ctx, src, dst)                                   # lf_resample
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
MODE_HYBRID, MODE_SPLIT, MODE_PURE_FV, MODE_PURE_LBM, MODE_HYBRID_GS2, MODE_SPLIT_H, \
    MODE_LBM_MCM = range(7)
IFACE_NEQ_EXTRAP, IFACE_FD_GRADIENT = 0, 1
CONV_QUICK, CONV_CENTRAL, CONV_UPWIND = 0, 1, 2
WALL_NOSLIP, WALL_PERIODIC = 0, 1
T_DIRICHLET, T_ADIABATIC, T_PERIODIC = 0, 1, 2
W, E, S, N = 0, 1, 2, 3
FIELD_U, FIELD_V, FIELD_T, FIELD_RHO, FIELD_P = 0, 1, 2, 3, 4
STOP_TOL, STOP_FLOOR = 1, 2
_FIELDS = {"u": FIELD_U, "v": FIELD_V, "T": FIELD_T, "rho": FIELD_RHO, "p": FIELD_P}
_STATUS = {0: "LF_OK", 1: "LF_EINVAL", 2: "LF_ENOMEM", 3: "LF_EWORKSPACE", 4: "LF_EDEVICE",
           5: "LF_EUNSTABLE", 6: "LF_EDIVERGED", 7: "LF_ENOTCONV", 8: "LF_ESTATE",
           9: "LF_ENOTIMPL"}


class lf_case_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("precision", ctypes.c_int),
                ("mode", ctypes.c_int), ("split_col", ctypes.c_int), ("overlap", ctypes.c_int),
                ("iface", ctypes.c_int), ("tcomp", ctypes.c_int)]


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


class lf_net_desc(ctypes.Structure):
    _fields_ = [("res", ctypes.c_int), ("cin", ctypes.c_int), ("cout", ctypes.c_int),
                ("widths", ctypes.c_int * 5), ("max_batch", ctypes.c_int)]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
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
    "lf_case_set_subcycle": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "lf_case_set_mcm": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                       ctypes.c_int64]),
    "lf_case_mcm_capped": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint64)]),
    "lf_case_init": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "lf_case_step": (ctypes.c_int, [_vp, _i64]),
    "lf_case_residual": (ctypes.c_int, [_vp, _dp]),
    "lf_case_residual_noalloc": (ctypes.c_int, [_vp, _dp]),
    "lf_case_run_to_steady": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int, _i64,
                                             ctypes.POINTER(_i64), _dp,
                                             ctypes.POINTER(ctypes.c_int)]),
    "lf_case_nusselt": (ctypes.c_int, [_vp, ctypes.POINTER(lf_nusselt)]),
    "lf_case_fetch": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_size_t, ctypes.c_int,
                                     ctypes.c_int]),
    "lf_case_mass": (ctypes.c_int, [_vp, _dp, _dp]),
    "lf_case_steps": (ctypes.c_int, [_vp, ctypes.POINTER(_i64)]),
    "lf_case_profile_steps": (ctypes.c_int, [_vp, _i64, _dp, _dp, _dp]),
    "lf_batch_create": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(lf_case_desc),
                                       ctypes.POINTER(lf_physics), ctypes.POINTER(lf_wall),
                                       ctypes.POINTER(_vp)]),
    "lf_batch_destroy": (ctypes.c_int, [_vp]),
    "lf_batch_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "lf_batch_bind_workspace": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "lf_batch_set_band": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "lf_batch_init": (ctypes.c_int, [_vp, ctypes.POINTER(_dp), ctypes.POINTER(_dp),
                                     ctypes.POINTER(_dp)]),
    "lf_batch_step": (ctypes.c_int, [_vp, _i64]),
    "lf_batch_residual": (ctypes.c_int, [_vp, _dp]),
    "lf_batch_run_to_steady": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int, _i64,
                                              ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_int),
                                              _dp]),
    "lf_batch_reactivate": (ctypes.c_int, [_vp]),
    "lf_batch_get_params": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "lf_batch_steps": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_i64)]),
    "lf_batch_nusselt": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(lf_nusselt)]),
    "lf_batch_fetch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t,
                                      ctypes.c_int, ctypes.c_int]),
    "lf_batch_profile_steps": (ctypes.c_int, [_vp, _i64, _dp]),
    "lf_autotune": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_int, _vp, ctypes.c_size_t]),
    "lf_ctx_get_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int)]),
    "lf_case_save": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)]),
    "lf_case_load": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "lf_batch_init_device": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                            ctypes.POINTER(_vp)]),
    "lf_net_create": (ctypes.c_int, [_vp, ctypes.POINTER(lf_net_desc), ctypes.POINTER(_vp)]),
    "lf_net_destroy": (ctypes.c_int, [_vp]),
    "lf_net_param_count": (ctypes.c_int, [_vp, ctypes.POINTER(_i64)]),
    "lf_net_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "lf_net_bind_workspace": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "lf_net_set_weights": (ctypes.c_int, [_vp, _fp, _i64]),
    "lf_net_get_weights": (ctypes.c_int, [_vp, _fp, _i64]),
    "lf_net_get_grads": (ctypes.c_int, [_vp, _fp, _i64]),
    "lf_net_forward": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
    "lf_net_get_output": (ctypes.c_int, [_vp, _fp, ctypes.c_size_t]),
    "lf_net_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, _vp]),
    "lf_net_adam": (ctypes.c_int, [_vp, ctypes.c_float]),
    "lf_net_train_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_float, _vp]),
    "lf_net_flops": (ctypes.c_int, [_vp, _dp, _dp]),
    "lf_net_profile_train": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_float,
                                            ctypes.c_int, _dp]),
    "lf_resample": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64, _vp,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int]),
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



def _workspace(ctx, nbytes: int) -> torch.Tensor:
    """A device buffer for the library, allocated on the library's stream:
    the caching allocator then hands the block to other streams only after
    that stream's queued kernels are done with it."""
    with torch.cuda.stream(ctx.stream):
        return torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{ctx.device}")


def _release(obj, destroy):
    """Destroy a handle and drop its workspace once the library stream has
    finished the work queued on it (step and init are asynchronous)."""
    h = getattr(obj, "_h", None)
    if h:
        try:
            obj.ctx.stream.synchronize()
        except Exception:  # interpreter shutdown: torch may be gone already
            pass
        if destroy is not None:
            destroy(h)
        obj._h = None
    obj.workspace = None


class Context:
    """A HIP device and the stream the library enqueues on.  By default a
    dedicated torch stream (default priority) is created, so that batches can
    capture graphs on it; ``ctx.stream`` is that torch.cuda.Stream."""

    def __init__(self, device: int = 0, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm GPU visible: the library runs on MI355X only")
        self.device = int(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        s = ctypes.c_void_p(self.stream.cuda_stream)
        h = _vp()
        _check(_lib.lf_ctx_create(self.device, s, ctypes.byref(h)), "lf_ctx_create")
        self._h = h

    def enter(self):
        """Order the library stream after the work torch has queued on its
        current stream (inputs written by torch ops)."""
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def leave(self):
        """Order torch's current stream after the work queued on the library
        stream (outputs read by torch ops)."""
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def autotune(self, cache_path: str, budget_ms: int = 3000, scratch_bytes: int = 1 << 30):
        """Load or measure the batch band table (see lf_autotune)."""
        scratch = torch.empty(int(scratch_bytes), dtype=torch.uint8, device=f"cuda:{self.device}")
        _check(_lib.lf_autotune(self._h, cache_path.encode(), int(budget_ms),
                                ctypes.c_void_p(scratch.data_ptr()), scratch.numel()),
               "lf_autotune")
        torch.cuda.synchronize(self.device)
        del scratch
        return self.tuning()

    def tuning(self) -> dict:
        n = ctypes.c_int()
        ny = (ctypes.c_int * 16)()
        bd = (ctypes.c_int * 16)()
        _check(_lib.lf_ctx_get_tuning(self._h, ctypes.byref(n), ny, bd), "lf_ctx_get_tuning")
        return {int(ny[k]): int(bd[k]) for k in range(n.value)}

    def set_band(self, rows: int):
        _check(_lib.lf_ctx_set_band(self._h, int(rows)), "lf_ctx_set_band")

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lf_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals may be gone
            pass


class Case:
    """One cavity: Mode H (grid setting 1, or 2 with MODE_HYBRID_GS2), the split
    LBM|FV mode divided vertically (MODE_SPLIT) or horizontally (MODE_SPLIT_H),
    one of the single methods (MODE_PURE_FV, MODE_PURE_LBM), or LBM-MCM
    (MODE_LBM_MCM).
    Fields are numpy arrays of shape (ny, nx)."""

    def __init__(self, ctx: Context, nx: int, ny: int, precision: str = "f32",
                 mode: int = MODE_HYBRID, split_col: int = 0, iface: int = IFACE_NEQ_EXTRAP,
                 tcomp: bool = True):
        """tcomp: FP32 Mode H keeps T as a compensated hi + lo pair."""
        self.ctx = ctx
        self.nx, self.ny = int(nx), int(ny)
        self.precision = F64 if precision in ("f64", F64, "fp64", "double") else F32
        d = lf_case_desc(self.nx, self.ny, self.precision, int(mode), int(split_col), 0, int(iface),
                         int(bool(tcomp)))
        h = _vp()
        _check(_lib.lf_case_create(ctx._h, ctypes.byref(d), ctypes.byref(h)), "lf_case_create")
        self._h = h
        nb = ctypes.c_size_t()
        _check(_lib.lf_case_workspace_bytes(h, ctypes.byref(nb)), "lf_case_workspace_bytes")
        self.workspace = _workspace(ctx, int(nb.value))
        _check(_lib.lf_case_bind_workspace(h, ctypes.c_void_p(self.workspace.data_ptr()),
                                           nb.value), "lf_case_bind_workspace")

    def close(self):
        _release(self, _lib.lf_case_destroy if _lib is not None else None)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals may be gone
            pass

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
        """One side (W, E, S, N): no-slip wall sliding tangentially at u_wall
        (in the split, FV-only and LBM-only modes only the north wall, the
        lid of the lid-driven cavity), or periodic; fixed T_wall or
        adiabatic."""
        w = lf_wall(int(vel), float(u_wall), int(thermal), float(T_wall))
        _check(_lib.lf_case_set_wall(self._h, int(side), ctypes.byref(w)), "lf_case_set_wall")
        return self

    def set_subcycle(self, lattice_steps=0, sweeps=0):
        """Grid setting 2: lattice steps per energy step (0: nx) and line
        sweeps per energy step (0: 4)."""
        _check(_lib.lf_case_set_subcycle(self._h, int(lattice_steps), int(sweeps)),
               "lf_case_set_subcycle")
        return self

    def set_mcm(self, lattice_steps=100, walkers=256, seed=1908083868, max_steps=1 << 24):
        """LBM-MCM: lattice steps per Monte Carlo solve, walkers per node,
        stream seed and the step cap of a walk."""
        _check(_lib.lf_case_set_mcm(self._h, int(lattice_steps), int(walkers), int(seed),
                                    int(max_steps)), "lf_case_set_mcm")
        return self

    def mcm_capped(self) -> int:
        """Walkers of the last Monte Carlo solve stopped by the step cap."""
        n = ctypes.c_uint64()
        _check(_lib.lf_case_mcm_capped(self._h, ctypes.byref(n)), "lf_case_mcm_capped")
        return n.value

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

    def residual_noalloc(self) -> np.ndarray:
        """lf_case_residual_noalloc: the same residual with its partials in
        the library's per-GPU static scratch (for callers that cannot
        allocate); calls overlapping on one GPU race."""
        r = np.zeros(3)
        _check(_lib.lf_case_residual_noalloc(self._h, _dptr(r)), "lf_case_residual_noalloc")
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
        self.ctx.enter()
        _check(_lib.lf_case_fetch(self._h, _FIELDS.get(field, field),
                                  ctypes.c_void_p(out.data_ptr()),
                                  out.numel() * out.element_size(), 1, as64), "lf_case_fetch")
        self.ctx.leave()
        return out

    def save(self) -> bytes:
        """Checkpoint of the complete case state (see lf_case_save)."""
        n = ctypes.c_size_t()
        _check(_lib.lf_case_save(self._h, None, ctypes.byref(n)), "lf_case_save")
        buf = ctypes.create_string_buffer(n.value)
        _check(_lib.lf_case_save(self._h, buf, ctypes.byref(n)), "lf_case_save")
        return buf.raw[:n.value]

    def load(self, blob: bytes):
        """Restore a checkpoint taken from a case of the same geometry."""
        _check(_lib.lf_case_load(self._h, ctypes.c_char_p(blob), len(blob)), "lf_case_load")
        return self

    def mass(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(_lib.lf_case_mass(self._h, ctypes.byref(a), ctypes.byref(b)), "lf_case_mass")
        return a.value, b.value


class Batch:
    """Many Mode H cavities stepped together (see lf_batch_* in lbmfvm.h).

    ``cases`` is a list of dicts with keys nx, ny and Ra, Pr (optional:
    U_char, T_ref, walls = list of four (vel, u_wall, thermal, T_wall))."""

    def __init__(self, ctx: Context, cases, precision: str = "f32", tcomp: bool = True):
        self.ctx = ctx
        self.n = len(cases)
        prec = F64 if precision in ("f64", F64) else F32
        D = (lf_case_desc * self.n)()
        Ph = (lf_physics * self.n)()
        Wl = (lf_wall * (4 * self.n))()
        any_walls = False
        self.shapes = []
        for k, c in enumerate(cases):
            D[k] = lf_case_desc(int(c["nx"]), int(c["ny"]), prec, MODE_HYBRID, 0, 0, 0,
                                int(bool(tcomp)))
            Ph[k] = lf_physics(float(c["Ra"]), float(c["Pr"]), float(c.get("U_char", 0.0)),
                               float(c.get("T_ref", float("nan"))), CONV_QUICK, 0.0, 0.0)
            walls = c.get("walls")
            if walls is None:
                walls = [(WALL_NOSLIP, 0.0, T_DIRICHLET, 0.5), (WALL_NOSLIP, 0.0, T_DIRICHLET, -0.5),
                         (WALL_NOSLIP, 0.0, T_ADIABATIC, 0.0), (WALL_NOSLIP, 0.0, T_ADIABATIC, 0.0)]
            else:
                any_walls = True
            for sd in range(4):
                vel, uw, th, tw = walls[sd]
                Wl[4 * k + sd] = lf_wall(int(vel), float(uw), int(th), float(tw))
            self.shapes.append((int(c["ny"]), int(c["nx"])))
        h = _vp()
        _check(_lib.lf_batch_create(ctx._h, self.n, D, Ph, Wl if any_walls else None,
                                    ctypes.byref(h)), "lf_batch_create")
        self._h = h
        nb = ctypes.c_size_t()
        _check(_lib.lf_batch_workspace_bytes(h, ctypes.byref(nb)), "lf_batch_workspace_bytes")
        self.workspace = _workspace(ctx, int(nb.value))
        _check(_lib.lf_batch_bind_workspace(h, ctypes.c_void_p(self.workspace.data_ptr()),
                                            nb.value), "lf_batch_bind_workspace")

    def close(self):
        _release(self, _lib.lf_batch_destroy if _lib is not None else None)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals may be gone
            pass

    def set_band(self, rows: int, idx: int = -1):
        _check(_lib.lf_batch_set_band(self._h, int(idx), int(rows)), "lf_batch_set_band")
        return self

    def init(self, T0=None, u0=None, v0=None):
        keep = []

        def arr(lst):
            if lst is None:
                return None
            P = (_dp * self.n)()
            for k in range(self.n):
                a = lst[k]
                if a is None:
                    P[k] = None
                else:
                    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64),
                                                             self.shapes[k]))
                    keep.append(a)
                    P[k] = a.ctypes.data_as(_dp)
            return P
        _check(_lib.lf_batch_init(self._h, arr(T0), arr(u0), arr(v0)), "lf_batch_init")
        return self

    def init_device(self, T0=None, u0=None, v0=None):
        """Initial fields from lists of float64 CUDA tensors [ny][nx] (or
        None entries); read asynchronously on the context stream."""
        def arr(lst):
            if lst is None:
                return None
            P = (_vp * self.n)()
            for k in range(self.n):
                a = lst[k]
                if a is None:
                    P[k] = None
                    continue
                assert a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()
                assert tuple(a.shape) == self.shapes[k], (k, tuple(a.shape), self.shapes[k])
                P[k] = a.data_ptr()
            return P
        self.ctx.enter()
        _check(_lib.lf_batch_init_device(self._h, arr(T0), arr(u0), arr(v0)),
               "lf_batch_init_device")
        self.ctx.leave()
        return self

    def fetch_device(self, idx: int, field, out: torch.Tensor):
        """Copy a field into a contiguous float32 or float64 CUDA tensor
        [ny][nx] (asynchronous on the context stream)."""
        assert out.is_cuda and out.is_contiguous() and tuple(out.shape) == self.shapes[idx]
        as64 = 1 if out.dtype == torch.float64 else 0
        assert as64 or out.dtype == torch.float32
        self.ctx.enter()
        _check(_lib.lf_batch_fetch(self._h, int(idx), _FIELDS.get(field, field),
                                   ctypes.c_void_p(out.data_ptr()),
                                   out.numel() * out.element_size(), 1, as64),
               "lf_batch_fetch")
        self.ctx.leave()
        return out

    def step(self, n: int):
        _check(_lib.lf_batch_step(self._h, int(n)), "lf_batch_step")
        return self

    def residual(self) -> np.ndarray:
        r = np.zeros(3 * self.n)
        _check(_lib.lf_batch_residual(self._h, _dptr(r)), "lf_batch_residual")
        return r.reshape(self.n, 3)

    def run_to_steady(self, tol=1e-8, check_every=1000, max_steps=10**7, raise_on_notconv=True):
        steps = (_i64 * self.n)()
        rules = (ctypes.c_int * self.n)()
        r = np.zeros(3 * self.n)
        st = _lib.lf_batch_run_to_steady(self._h, float(tol), int(check_every), int(max_steps),
                                         steps, rules, _dptr(r))
        if st != LF_OK and not (st == LF_ENOTCONV and not raise_on_notconv):
            raise LFError(st, "lf_batch_run_to_steady")
        return np.array(steps[:]), np.array(rules[:]), r.reshape(self.n, 3)

    def reactivate(self):
        _check(_lib.lf_batch_reactivate(self._h), "lf_batch_reactivate")
        return self

    def params(self, idx: int) -> dict:
        out = np.zeros(8)
        _check(_lib.lf_batch_get_params(self._h, int(idx), _dptr(out)), "lf_batch_get_params")
        return dict(zip(["U_char", "nu", "tau", "alpha", "tau_T", "gbeta", "T_ref", "Ma"],
                        out.tolist()))

    def steps(self, idx: int) -> int:
        v = _i64()
        _check(_lib.lf_batch_steps(self._h, int(idx), ctypes.byref(v)), "lf_batch_steps")
        return v.value

    def nusselt(self, idx: int) -> dict:
        o = lf_nusselt()
        _check(_lib.lf_batch_nusselt(self._h, int(idx), ctypes.byref(o)), "lf_batch_nusselt")
        return {k: getattr(o, k) for k, _ in lf_nusselt._fields_}

    def fetch(self, idx: int, field) -> np.ndarray:
        out = np.empty(self.shapes[idx], dtype=np.float64)
        _check(_lib.lf_batch_fetch(self._h, int(idx), _FIELDS.get(field, field),
                                   out.ctypes.data_as(_vp), out.nbytes, 0, 1), "lf_batch_fetch")
        return out

    def profile_steps(self, n: int) -> float:
        a = ctypes.c_double()
        _check(_lib.lf_batch_profile_steps(self._h, int(n), ctypes.byref(a)),
               "lf_batch_profile_steps")
        return a.value


RESAMPLE_ANTISYM = 1


def resample(ctx: Context, src: torch.Tensor, dst: torch.Tensor, scale=1.0, offset=0.0,
             antisym=False):
    """Bilinear resampling of a cell-centred CUDA tensor src [sny][snx] (rows
    may be strided) into the contiguous CUDA tensor dst [dny][dnx]:
    dst = value * scale + offset, optionally reduced to its part that is odd
    under the 180-degree rotation (see lf_resample)."""
    assert src.is_cuda and dst.is_cuda and dst.is_contiguous() and src.stride(1) == 1
    assert src.dtype in (torch.float32, torch.float64) and dst.dtype in (torch.float32,
                                                                          torch.float64)
    sny, snx = src.shape
    dny, dnx = dst.shape
    ctx.enter()
    _check(_lib.lf_resample(ctx._h, ctypes.c_void_p(src.data_ptr()),
                            int(src.dtype == torch.float64), snx, sny, src.stride(0),
                            ctypes.c_void_p(dst.data_ptr()), int(dst.dtype == torch.float64),
                            dnx, dny, float(scale), float(offset),
                            RESAMPLE_ANTISYM if antisym else 0), "lf_resample")
    ctx.leave()
    return dst


class Net:
    """The learned initial guess (see lf_net_* in lbmfvm.h).  Device inputs
    are torch tensors: feat float32 [N][3] (log10 Ra, Pr, A), target float32
    [N][3][res][res], idx int32 [batch]."""

    def __init__(self, ctx: Context, res=128, widths=(32, 32, 64, 64, 128), cout=8,
                 max_batch=32):
        self.ctx = ctx
        self.res, self.widths, self.cout, self.max_batch = res, tuple(widths), cout, max_batch
        d = lf_net_desc(res, 8, cout, (ctypes.c_int * 5)(*widths), max_batch)
        h = _vp()
        _check(_lib.lf_net_create(ctx._h, ctypes.byref(d), ctypes.byref(h)), "lf_net_create")
        self._h = h
        n = _i64()
        _check(_lib.lf_net_param_count(h, ctypes.byref(n)), "lf_net_param_count")
        self.nparam = n.value
        nb = ctypes.c_size_t()
        _check(_lib.lf_net_workspace_bytes(h, ctypes.byref(nb)), "lf_net_workspace_bytes")
        self.workspace = _workspace(ctx, int(nb.value))
        _check(_lib.lf_net_bind_workspace(h, ctypes.c_void_p(self.workspace.data_ptr()),
                                          nb.value), "lf_net_bind_workspace")
        with torch.cuda.stream(ctx.stream):
            self.loss_dev = torch.zeros(1, dtype=torch.float32, device=f"cuda:{ctx.device}")

    def close(self):
        _release(self, _lib.lf_net_destroy if _lib is not None else None)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals may be gone
            pass

    def layer_shapes(self):
        """(Cout, Cin) of the ten convolutions, in the flat parameter order."""
        w0, w1, w2, w3, w4 = self.widths
        co = [w0, w1, w2, w3, w4, w3, w2, w1, w0, self.cout]
        ci = [8, w0, w1, w2, w3, w4, w3, w2, w1, w0]
        return list(zip(co, ci))

    def he_uniform(self, u: np.ndarray) -> np.ndarray:
        """Weights uniform in +-sqrt(6 / fan_in) from uniforms u in [0, 1)
        (one per parameter), biases zero; fan_in counts the 5 real input
        channels of the first layer."""
        u = np.asarray(u, np.float64)
        assert u.size == self.nparam
        out = np.zeros(self.nparam, np.float32)
        k = 0
        for li, (o, i) in enumerate(self.layer_shapes()):
            nw = o * 9 * i
            fan = 9 * (5 if li == 0 else i)
            b = math.sqrt(6.0 / fan) * (0.5 if li == len(self.layer_shapes()) - 1 else 1.0)
            out[k:k + nw] = ((2.0 * u[k:k + nw] - 1.0) * b).astype(np.float32)
            k += nw + o
        return out

    def set_weights(self, w):
        w = np.ascontiguousarray(w, np.float32)
        _check(_lib.lf_net_set_weights(self._h, w.ctypes.data_as(_fp), w.size),
               "lf_net_set_weights")
        return self

    def weights(self) -> np.ndarray:
        out = np.empty(self.nparam, np.float32)
        _check(_lib.lf_net_get_weights(self._h, out.ctypes.data_as(_fp), out.size),
               "lf_net_get_weights")
        return out

    def grads(self) -> np.ndarray:
        out = np.empty(self.nparam, np.float32)
        _check(_lib.lf_net_get_grads(self._h, out.ctypes.data_as(_fp), out.size),
               "lf_net_get_grads")
        return out

    @staticmethod
    def _p(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    def forward(self, feat, idx=None, batch=None, pred=None):
        batch = int(batch if batch is not None else (idx.numel() if idx is not None
                                                      else feat.shape[0]))
        self.ctx.enter()
        _check(_lib.lf_net_forward(self._h, self._p(feat), self._p(idx), batch, self._p(pred)),
               "lf_net_forward")
        self.ctx.leave()
        return pred

    def output(self, batch) -> np.ndarray:
        out = np.empty((batch, self.res, self.res, self.cout), np.float32)
        _check(_lib.lf_net_get_output(self._h, out.ctypes.data_as(_fp), out.size),
               "lf_net_get_output")
        return out

    def backward(self, feat, target, idx=None, batch=None):
        batch = int(batch if batch is not None else (idx.numel() if idx is not None
                                                      else feat.shape[0]))
        self.ctx.enter()
        _check(_lib.lf_net_backward(self._h, self._p(feat), self._p(target), self._p(idx), batch,
                                    self._p(self.loss_dev)), "lf_net_backward")
        self.ctx.leave()
        return self

    def adam(self, lr):
        _check(_lib.lf_net_adam(self._h, float(lr)), "lf_net_adam")
        return self

    def train_step(self, feat, target, idx, lr):
        self.ctx.enter()
        _check(_lib.lf_net_train_step(self._h, self._p(feat), self._p(target), self._p(idx),
                                      int(idx.numel()), float(lr), self._p(self.loss_dev)),
               "lf_net_train_step")
        self.ctx.leave()
        return self

    def loss(self) -> float:
        """Loss of the last backward / training step (synchronises)."""
        return float(self.loss_dev.item())

    def flops(self):
        f, t = ctypes.c_double(), ctypes.c_double()
        _check(_lib.lf_net_flops(self._h, ctypes.byref(f), ctypes.byref(t)), "lf_net_flops")
        return f.value, t.value

    def profile_train(self, feat, target, idx, lr, nsteps) -> float:
        a = ctypes.c_double()
        self.ctx.enter()
        _check(_lib.lf_net_profile_train(self._h, self._p(feat), self._p(target), self._p(idx),
                                         int(idx.numel()), float(lr), int(nsteps),
                                         ctypes.byref(a)), "lf_net_profile_train")
        return a.value
