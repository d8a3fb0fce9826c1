"""ctypes binding of libplace3d (include/place3d.h): argument marshalling only.

Every step of the hot path runs in the HIP library; this module allocates device memory with
PyTorch, passes raw pointers and the current stream, and reads results back.  There is no CPU
fallback: without the built library, or without a GPU, the calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libplace3d.so")

OK = 0
FP32, BF16X3 = 0, 1
DGRAD_FIELD, DGRAD_ADJOINT = 0, 1
PRECOND_MIXED, PRECOND_EPLACE, PRECOND_EPLACE3D = 0, 1, 2
OPT_MACRO_INSTANCE, OPT_FDA_VANILLA = 1, 2
KIND_MACRO, KIND_FIXED, KIND_FILLER, KIND_ZFIXED = 1, 2, 4, 8
NMETRICS, NSCALARS = 16, 32
M = dict(wa_bi=0, wa_z=1, hpwl=2, hpwl3d=3, ncut=4, norm_x=5, norm_y=6, norm_fda=7, fda_scale=8)
S = dict(a=0, lam=1, step=2, it=3, ovfl_bot=4, ovfl_top=5, energy=6, nonfinite=7, wl=8)
WLZ_FDA, WLZ_VALUE = 0, 1
STAGES = ("density", "gemm", "zmix", "dgrad", "wl_nets", "wl_nodes", "update", "bucket")
STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_SIZE", -3: "ERR_HIP", -4: "ERR_NONFINITE",
          -5: "ERR_UNSUPPORTED", -6: "ERR_NETLIST"}


class Place3dError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Problem_(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("n_pins", ctypes.c_int32), ("n_nets", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("die_x", ctypes.c_double), ("die_y", ctypes.c_double), ("gamma", ctypes.c_double),
                ("alpha", ctypes.c_double), ("target_density", ctypes.c_double),
                ("lambda_ramp", ctypes.c_double), ("precision", ctypes.c_int32), ("dgrad", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("options", ctypes.c_int32),
                ("size", ctypes.c_void_p), ("kind", ctypes.c_void_p), ("net_start", ctypes.c_void_p),
                ("pin2node", ctypes.c_void_p), ("pin_off", ctypes.c_void_p), ("fixed_xyz", ctypes.c_void_p)]


class FillerPlan_(ctypes.Structure):
    _fields_ = [("n_top", ctypes.c_int64), ("n_bot", ctypes.c_int64), ("n_free", ctypes.c_int64),
                ("side_top", ctypes.c_double), ("side_bot", ctypes.c_double), ("side_free", ctypes.c_double),
                ("vol_top", ctypes.c_double), ("vol_bot", ctypes.c_double), ("vol_free", ctypes.c_double),
                ("vol_a", ctypes.c_double)]


class State_(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("v", ctypes.c_void_p), ("v_prev", ctypes.c_void_p),
                ("g_prev", ctypes.c_void_p), ("scalars", ctypes.c_void_p)]


class MdProblem_(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_layer", ctypes.c_int32 * 3), ("n_pins", ctypes.c_int32),
                ("n_nets", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("die_x", ctypes.c_double), ("die_y", ctypes.c_double), ("gamma", ctypes.c_double),
                ("target_density", ctypes.c_double), ("lambda_ramp", ctypes.c_double), ("precision", ctypes.c_int32),
                ("size", ctypes.c_void_p), ("kind", ctypes.c_void_p), ("layer", ctypes.c_void_p),
                ("net_start", ctypes.c_void_p), ("pin2node", ctypes.c_void_p), ("pin_off", ctypes.c_void_p),
                ("fixed_xy", ctypes.c_void_p)]


LAYER_BOTTOM, LAYER_TOP, LAYER_HBT = 0, 1, 2
MD = dict(wa=0, hpwl=1, ovfl_bot=2, ovfl_top=3, ovfl_hbt=4, energy_bot=5, energy_top=6, energy_hbt=7)
MS = dict(a=0, lam_bot=1, lam_top=2, lam_hbt=3, step=4, it=5, metrics=8, nonfinite=16)

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2403_09070_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
        sig = {
            "place3d_abi_version": (i32, []),
            "place3d_last_error": (ctypes.c_char_p, [vp]),
            "place3d_workspace_size": (i32, [ctypes.POINTER(Problem_), ctypes.POINTER(ctypes.c_size_t)]),
            "place3d_create": (i32, [ctypes.POINTER(Problem_), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
            "place3d_destroy": (i32, [vp]),
            "place3d_density": (i32, [vp, vp, vp, vp]),
            "place3d_field": (i32, [vp, vp, vp, vp, vp, vp, vp, vp]),
            "place3d_field_force": (i32, [vp, vp, vp, vp, vp, f32, vp, i32, vp]),
            "place3d_density_vjp": (i32, [vp, vp, vp, f32, vp, vp, i32, vp]),
            "place3d_wl_grad": (i32, [vp, vp, vp, vp, i32, vp]),
            "place3d_wl_value": (i32, [vp, vp, vp, vp]),
            "place3d_wl_value_static": (i32, [vp, vp, vp, vp]),
            "place3d_wl_vjp": (i32, [vp, vp, vp, i32, vp, i32, vp]),
            "place3d_read_scalars": (i32, [vp, ctypes.POINTER(State_), vp, vp]),
            "place3d_gp_init": (i32, [vp, ctypes.POINTER(State_), vp, vp]),
            "place3d_step": (i32, [vp, ctypes.POINTER(State_), vp]),
            "place3d_profile_enable": (i32, [vp, i32]),
            "place3d_plan_fillers": (i32, [i32, vp, vp, vp, ctypes.c_double, ctypes.c_double, i32, i32, i32,
                                           ctypes.c_double, ctypes.c_double, ctypes.POINTER(FillerPlan_)]),
            "place3d_profile_read": (i32, [vp, i32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64), i32]),
            "place3d_md2d_workspace_size": (i32, [ctypes.POINTER(MdProblem_), ctypes.POINTER(ctypes.c_size_t)]),
            "place3d_md2d_create": (i32, [ctypes.POINTER(MdProblem_), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
            "place3d_md2d_destroy": (i32, [vp]),
            "place3d_md2d_last_error": (ctypes.c_char_p, [vp]),
            "place3d_md2d_eval": (i32, [vp, vp, vp, vp, vp, vp, vp]),
            "place3d_md2d_gp_init": (i32, [vp, ctypes.POINTER(State_), vp, vp]),
            "place3d_md2d_step": (i32, [vp, ctypes.POINTER(State_), vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.place3d_abi_version() != 2:
            raise ImportError("libplace3d ABI version mismatch")
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != OK:
        msg = lib().place3d_last_error(ctx)
        raise Place3dError(rc, msg.decode() if msg else "")


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("arrays passed to the library must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def hbt_alpha(die_x, dz, hbt_pitch, row_top, row_bot, beta, alpha0=3.5e-3):
    """Weight of the cut term, alpha = alpha0 (d_x eta^2 / d_z) ln(90 beta eta - 1),
    eta = 2 w' / (RH+ + RH-) (experimental setup, Sec. V-A)."""
    eta = 2.0 * hbt_pitch / (row_top + row_bot)
    return alpha0 * (die_x * eta * eta / dz) * math.log(90.0 * beta * eta - 1.0)


def plan_fillers(size, kind, z0, die_x, die_y, nx, ny, nz, u_top, u_bot):
    """place3d_plan_fillers on host arrays: a dict of the counts, sides and volumes."""
    size = np.ascontiguousarray(size, dtype=np.float32)
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    z0 = np.ascontiguousarray(z0, dtype=np.float32)
    n = int(kind.shape[0])
    if size.shape != (4, n) or z0.shape != (n,):
        raise ValueError("size must be [4][n] and z0 [n]")
    out = FillerPlan_()
    vp = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
    _check(lib().place3d_plan_fillers(n, vp(size), vp(kind), vp(z0), float(die_x), float(die_y), int(nx), int(ny),
                                      int(nz), float(u_top), float(u_bot), ctypes.byref(out)))
    return {k: getattr(out, k) for k, _ in FillerPlan_._fields_}


@dataclass
class State:
    u: torch.Tensor
    v: torch.Tensor
    v_prev: torch.Tensor
    g_prev: torch.Tensor
    scalars: torch.Tensor

    def cstruct(self):
        return State_(self.u.data_ptr(), self.v.data_ptr(), self.v_prev.data_ptr(), self.g_prev.data_ptr(),
                      self.scalars.data_ptr())

    def read(self):
        s = self.scalars.cpu().numpy()
        out = {k: float(s[v]) for k, v in S.items() if k != "wl"}
        for k, v in M.items():
            out[k] = float(s[S["wl"] + v])
        return out


class Problem:
    """A placement problem resident on the GPU with its library context.

    ``arrays`` holds numpy arrays in the C-ABI layouts (see synth.Case); they are copied to the
    device once.  ``gamma``, ``alpha`` etc. are plain parameters.
    """

    def __init__(self, *, size, kind, net_start, pin2node, pin_off, fixed_xyz, die_x, die_y, nx, ny, nz,
                 gamma, alpha, target_density=1.0, lambda_ramp=1.05, precision=FP32, dgrad=DGRAD_FIELD,
                 precond=PRECOND_MIXED, options=0, device="cuda"):
        L = lib()
        dev = torch.device(device)
        self.device = dev
        self.n = int(kind.shape[0])
        self.P = int(pin2node.shape[0])
        self.m = int(net_start.shape[0] - 1)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.die_x, self.die_y = float(die_x), float(die_y)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
        self.size = t(size, torch.float32)
        self.kind = t(kind, torch.uint8)
        self.net_start = t(net_start, torch.int32)
        self.pin2node = t(pin2node if self.P else np.zeros(1, np.int32), torch.int32)
        self.pin_off = t(pin_off if self.P else np.zeros((4, 1), np.float32), torch.float32)
        self.fixed_xyz = t(fixed_xyz, torch.float32)
        self.params = dict(gamma=float(gamma), alpha=float(alpha), target_density=float(target_density),
                           lambda_ramp=float(lambda_ramp), precision=int(precision), dgrad=int(dgrad),
                           precond=int(precond), options=int(options))
        self._p = Problem_(self.n, self.P, self.m, self.nx, self.ny, self.nz, self.die_x, self.die_y,
                           float(gamma), float(alpha), float(target_density), float(lambda_ramp),
                           int(precision), int(dgrad), int(precond), int(options),
                           self.size.data_ptr(), self.kind.data_ptr(), self.net_start.data_ptr(),
                           self.pin2node.data_ptr(), self.pin_off.data_ptr(), self.fixed_xyz.data_ptr())
        nbytes = ctypes.c_size_t()
        _check(L.place3d_workspace_size(ctypes.byref(self._p), ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self._ctx = ctypes.c_void_p()
        _check(L.place3d_create(ctypes.byref(self._p), ctypes.c_void_p(aligned), nbytes.value, _stream(),
                                ctypes.byref(self._ctx)))

    @staticmethod
    def case_params(case):
        """gamma, alpha, target density and lambda ramp of a synthetic case's configuration."""
        cfg = case.config
        wb = case.die_x / case.nx
        dz = case.nz * 0.5 * (wb + case.die_y / case.ny)
        return dict(gamma=cfg.gamma_bins * wb,
                    alpha=hbt_alpha(case.die_x, dz, cfg.hbt_pitch, cfg.row_top, cfg.row_bot, cfg.beta, cfg.alpha0),
                    target_density=cfg.target_density, lambda_ramp=cfg.lambda_ramp)

    @classmethod
    def from_case(cls, case, **kw):
        params = cls.case_params(case)
        params.update(kw)
        return cls(size=case.size, kind=case.kind, net_start=case.net_start, pin2node=case.pin2node,
                   pin_off=case.pin_off, fixed_xyz=case.xyz0, die_x=case.die_x, die_y=case.die_y,
                   nx=case.nx, ny=case.ny, nz=case.nz, **params)

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value and _lib is not None:
            _lib.place3d_destroy(ctx)
            self._ctx = None

    # ------------------------------------------------------------------ helpers
    def xyz(self, a):
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(self.device) \
            if not isinstance(a, torch.Tensor) else a.to(device=self.device, dtype=torch.float32).contiguous()

    def map_in(self, m):
        """A (nz, ny, nx) input map as a contiguous float32 device tensor."""
        t = torch.as_tensor(m).to(device=self.device, dtype=torch.float32).contiguous()
        if tuple(t.shape) != (self.nz, self.ny, self.nx):
            raise ValueError(f"map of shape {tuple(t.shape)}, expected {(self.nz, self.ny, self.nx)}")
        return t

    def new_map(self):
        return torch.empty((self.nz, self.ny, self.nx), dtype=torch.float32, device=self.device)

    def _grad(self, out):
        return torch.empty((3, self.n), dtype=torch.float32, device=self.device) if out is None else out

    # ------------------------------------------------------------------ calls
    def density(self, xyz, out=None):
        xyz = self.xyz(xyz)
        rho = self.new_map() if out is None else out
        _check(lib().place3d_density(self._ctx, _ptr(xyz), _ptr(rho), _stream()), self._ctx)
        return rho

    def field(self, rho, want=("phi", "ex", "ey", "ez"), energy=False):
        out = {k: self.new_map() for k in want}
        e = torch.zeros(1, dtype=torch.float64, device=self.device) if energy else None
        _check(lib().place3d_field(self._ctx, _ptr(self.map_in(rho)), _ptr(out.get("phi")), _ptr(out.get("ex")),
                                   _ptr(out.get("ey")), _ptr(out.get("ez")), _ptr(e), _stream()), self._ctx)
        if energy:
            out["energy"] = e
        return out

    def field_force(self, xyz, ex, ey, ez, lam=1.0, out=None, accumulate=False):
        xyz = self.xyz(xyz)
        g = self._grad(out)
        ex, ey, ez = self.map_in(ex), self.map_in(ey), self.map_in(ez)
        _check(lib().place3d_field_force(self._ctx, _ptr(xyz), _ptr(ex), _ptr(ey), _ptr(ez), float(lam), _ptr(g),
                                         int(accumulate), _stream()), self._ctx)
        return g

    def density_vjp(self, xyz, g_rho, out=None, accumulate=False, scale=1.0, d_scale=None):
        """grad (+)= scale * d_scale[0] * J^T g_rho; d_scale a one-element float64 device tensor or None."""
        xyz = self.xyz(xyz)
        g = self._grad(out)
        ds = None if d_scale is None else d_scale.to(device=self.device, dtype=torch.float64).contiguous()
        _check(lib().place3d_density_vjp(self._ctx, _ptr(xyz), _ptr(self.map_in(g_rho)), float(scale), _ptr(ds),
                                         _ptr(g), int(accumulate), _stream()), self._ctx)
        return g

    def wl_grad(self, xyz, out=None, accumulate=False):
        xyz = self.xyz(xyz)
        g = self._grad(out)
        met = torch.zeros(NMETRICS, dtype=torch.float64, device=self.device)
        _check(lib().place3d_wl_grad(self._ctx, _ptr(xyz), _ptr(g), _ptr(met), int(accumulate), _stream()),
               self._ctx)
        return g, met

    def wl_value(self, xyz):
        """The model's net totals at xyz (float64 [NMETRICS]; no gradient, nothing stored per pin)."""
        xyz = self.xyz(xyz)
        met = torch.empty(NMETRICS, dtype=torch.float64, device=self.device)
        _check(lib().place3d_wl_value(self._ctx, _ptr(xyz), _ptr(met), _stream()), self._ctx)
        return met

    def wl_value_static(self, xyz):
        """wl_value with the call's scratch in the library's static device array (no workspace scratch)."""
        xyz = self.xyz(xyz)
        met = torch.empty(NMETRICS, dtype=torch.float64, device=self.device)
        _check(lib().place3d_wl_value_static(self._ctx, _ptr(xyz), _ptr(met), _stream()), self._ctx)
        return met

    def wl_vjp(self, xyz, d_scale=None, z_mode=WLZ_FDA, out=None, accumulate=False):
        """Backward of the wirelength model, recomputed from xyz: grad (+)= d_scale[0] * dW/dxyz."""
        xyz = self.xyz(xyz)
        g = self._grad(out)
        ds = None if d_scale is None else d_scale.to(device=self.device, dtype=torch.float64).contiguous()
        _check(lib().place3d_wl_vjp(self._ctx, _ptr(xyz), _ptr(ds), int(z_mode), _ptr(g), int(accumulate),
                                    _stream()), self._ctx)
        return g

    def read_scalars(self, state):
        """The state's scalars on the host after waiting for the stream; raises Place3dError
        (ERR_NONFINITE) when an iteration met a NaN or infinity."""
        host = np.zeros(NSCALARS, dtype=np.float64)
        cs = state.cstruct()
        _check(lib().place3d_read_scalars(self._ctx, ctypes.byref(cs), ctypes.c_void_p(host.ctypes.data), _stream()),
               self._ctx)
        return host

    def new_state(self):
        z = lambda: torch.zeros((3, self.n), dtype=torch.float32, device=self.device)  # noqa: E731
        return State(z(), z(), z(), z(), torch.zeros(NSCALARS, dtype=torch.float64, device=self.device))

    def gp_init(self, xyz0, state=None):
        st = self.new_state() if state is None else state
        xyz0 = self.xyz(xyz0)
        cs = st.cstruct()
        _check(lib().place3d_gp_init(self._ctx, ctypes.byref(cs), _ptr(xyz0), _stream()), self._ctx)
        return st

    def profile(self, on=True, stages=None):
        """Bracket the launches of the named stages (all stages by default) with HIP events."""
        mask = 0
        if on:
            mask = 0xFF if stages is None else sum(1 << STAGES.index(k) for k in stages)
        _check(lib().place3d_profile_enable(self._ctx, int(mask)), self._ctx)

    def profile_read(self, reset=True):
        """{stage: (gpu milliseconds, launches)} since the last reset (waits for the events)."""
        out = {}
        for k, name in enumerate(STAGES):
            ms, cnt = ctypes.c_double(), ctypes.c_int64()
            last = reset and k == len(STAGES) - 1
            _check(lib().place3d_profile_read(self._ctx, k, ctypes.byref(ms), ctypes.byref(cnt), int(last)),
                   self._ctx)
            out[name] = (ms.value, cnt.value)
        return out

    def step(self, state):
        cs = state.cstruct()
        _check(lib().place3d_step(self._ctx, ctypes.byref(cs), _stream()), self._ctx)


def metrics_dict(met):
    m = met.cpu().numpy()
    return {k: float(m[v]) for k, v in M.items()}


def _check_md(rc, ctx=None):
    if rc != OK:
        msg = lib().place3d_md2d_last_error(ctx)
        raise Place3dError(rc, msg.decode() if msg else "")


@dataclass
class MdState:
    u: torch.Tensor
    v: torch.Tensor
    v_prev: torch.Tensor
    g_prev: torch.Tensor
    scalars: torch.Tensor

    def cstruct(self):
        return State_(self.u.data_ptr(), self.v.data_ptr(), self.v_prev.data_ptr(), self.g_prev.data_ptr(),
                      self.scalars.data_ptr())

    def read(self):
        s = self.scalars.cpu().numpy()
        out = {k: float(s[v]) for k, v in MS.items() if k != "metrics"}
        for k, v in MD.items():
            if v < 5:
                out[k] = float(s[MS["metrics"] + v])
        return out


class MultiDie2D:
    """A multi-die 2D placement problem (Sec. III-C, Eq. 2d-place) on the GPU with its context:
    nodes (instances at their die's size, HBTs, fillers) with a layer each, and the partial nets.
    ``size`` is [2][n] (w, h), ``pin_off`` [2][P]; the arrays are copied to the device once."""

    def __init__(self, *, size, kind, layer, net_start, pin2node, pin_off, fixed_xy, die_x, die_y, nx, ny, gamma,
                 target_density=1.0, lambda_ramp=1.05, precision=FP32, device="cuda"):
        L = lib()
        dev = torch.device(device)
        self.device = dev
        layer = np.asarray(layer, dtype=np.uint8)
        self.n = int(layer.shape[0])
        self.P = int(np.asarray(pin2node).shape[0])
        self.m = int(np.asarray(net_start).shape[0] - 1)
        self.nx, self.ny = int(nx), int(ny)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
        self.size = t(size, torch.float32)
        self.kind = t(kind, torch.uint8)
        self.layer = t(layer, torch.uint8)
        self.net_start = t(net_start, torch.int32)
        self.pin2node = t(pin2node if self.P else np.zeros(1, np.int32), torch.int32)
        self.pin_off = t(pin_off if self.P else np.zeros((2, 1), np.float32), torch.float32)
        self.fixed_xy = t(fixed_xy, torch.float32)
        counts = np.bincount(layer, minlength=3)[:3]
        self._p = MdProblem_(self.n, (ctypes.c_int32 * 3)(*[int(c) for c in counts]), self.P, self.m, self.nx,
                             self.ny, float(die_x), float(die_y), float(gamma), float(target_density),
                             float(lambda_ramp), int(precision), self.size.data_ptr(), self.kind.data_ptr(),
                             self.layer.data_ptr(), self.net_start.data_ptr(), self.pin2node.data_ptr(),
                             self.pin_off.data_ptr(), self.fixed_xy.data_ptr())
        nbytes = ctypes.c_size_t()
        _check_md(L.place3d_md2d_workspace_size(ctypes.byref(self._p), ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self._ctx = ctypes.c_void_p()
        _check_md(L.place3d_md2d_create(ctypes.byref(self._p), ctypes.c_void_p(aligned), nbytes.value, _stream(),
                                        ctypes.byref(self._ctx)))

    @classmethod
    def from_layered(cls, lay, **kw):
        """From a multi-die problem in the layout the multi-die oracle uses (w, h, kind, layer, partial
        nets, grid, gamma, ramp, target as attributes; fixed nodes take fixed_xy, default zeros)."""
        fixed_xy = kw.pop("fixed_xy", np.zeros((2, len(lay.w)), np.float32))
        g = lay.grid
        return cls(size=np.stack([lay.w, lay.h]).astype(np.float32), kind=lay.kind, layer=lay.layer,
                   net_start=np.asarray(lay.net_start, np.int32), pin2node=np.asarray(lay.pin2node, np.int32),
                   pin_off=np.asarray(lay.pin_off, np.float32), fixed_xy=fixed_xy, die_x=g.die_x, die_y=g.die_y,
                   nx=g.nx, ny=g.ny, gamma=lay.gamma, target_density=lay.target, lambda_ramp=lay.ramp, **kw)

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value and _lib is not None:
            _lib.place3d_md2d_destroy(ctx)
            self._ctx = None

    def xy(self, a):
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(self.device) \
            if not isinstance(a, torch.Tensor) else a.to(device=self.device, dtype=torch.float32).contiguous()

    def eval(self, xy, want_maps=True):
        """(grad_wl [2][n], grad_den [2][n], rho [3][ny][nx] or None, metrics float64 [NMETRICS])."""
        xy = self.xy(xy)
        gw = torch.empty((2, self.n), dtype=torch.float32, device=self.device)
        gd = torch.empty_like(gw)
        rho = torch.empty((3, self.ny, self.nx), dtype=torch.float32, device=self.device) if want_maps else None
        met = torch.empty(NMETRICS, dtype=torch.float64, device=self.device)
        _check_md(lib().place3d_md2d_eval(self._ctx, _ptr(xy), _ptr(gw), _ptr(gd), _ptr(rho), _ptr(met), _stream()),
                  self._ctx)
        return gw, gd, rho, met

    def new_state(self):
        z = lambda: torch.zeros((2, self.n), dtype=torch.float32, device=self.device)  # noqa: E731
        return MdState(z(), z(), z(), z(), torch.zeros(NSCALARS, dtype=torch.float64, device=self.device))

    def gp_init(self, xy0, state=None):
        st = self.new_state() if state is None else state
        xy0 = self.xy(xy0)
        cs = st.cstruct()
        _check_md(lib().place3d_md2d_gp_init(self._ctx, ctypes.byref(cs), _ptr(xy0), _stream()), self._ctx)
        return st

    def step(self, state):
        cs = state.cstruct()
        _check_md(lib().place3d_md2d_step(self._ctx, ctypes.byref(cs), _stream()), self._ctx)
