"""Python binding of ``lib/libswe_hip.so`` (ctypes).

Argument marshalling only: every step of the scheme runs in the library's HIP
kernels.  PyTorch provides the device workspace (one ``uint8`` tensor per
domain) and the HIP stream.  Importing this module without the built library
raises ImportError -- there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libswe_hip.so")

SWE_OK, SWE_E_ARG, SWE_E_NOMEM, SWE_E_HIP, SWE_E_UNSTABLE, SWE_E_STATE = 0, -1, -2, -3, -4, -5
BC_WALL, BC_PERIODIC, BC_NESTED = 0, 1, 2
FRICTION_NONE, FRICTION_LINEAR, FRICTION_QUADRATIC, FRICTION_MANNING = 0, 1, 2, 3
FORCING_WIND_STRESS, FORCING_BOUNDARY = 0, 1


class SweError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"swe error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("g", C.c_double),
        ("courant", C.c_double), ("theta", C.c_double), ("kappa", C.c_double),
        ("bc", C.c_int32 * 4), ("friction", C.c_int32), ("friction_coeff", C.c_double),
        ("rho_w", C.c_double), ("frs_width", C.c_int32), ("frs_d0", C.c_double),
        ("north_projection", C.c_int32), ("compensated_state", C.c_int32),
    ]


class Request(C.Structure):
    _fields_ = [
        ("id", C.c_int64), ("params", Params), ("horizon", C.c_double),
        ("Hc", C.POINTER(C.c_float)), ("land", C.POINTER(C.c_uint8)), ("f", C.POINTER(C.c_float)),
        ("theta", C.POINTER(C.c_float)), ("eta", C.POINTER(C.c_float)), ("hu", C.POINTER(C.c_float)),
        ("hv", C.POINTER(C.c_float)), ("n_wind", C.c_int32), ("n_bnd", C.c_int32),
        ("wind_t", C.POINTER(C.c_double)), ("wind_tau", C.POINTER(C.c_float)),
        ("bnd_t", C.POINTER(C.c_double)), ("bnd", C.POINTER(C.c_float)),
        ("out_eta", C.POINTER(C.c_float)), ("out_hu", C.POINTER(C.c_float)), ("out_hv", C.POINTER(C.c_float)),
    ]


class Completion(C.Structure):
    _fields_ = [("id", C.c_int64), ("t", C.c_double), ("steps", C.c_int64), ("tick", C.c_int64),
                ("status", C.c_int32), ("pad", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("ticks", C.c_int64), ("cell_steps", C.c_int64), ("arena_bytes", C.c_size_t),
                ("arena_used", C.c_size_t), ("arena_peak", C.c_size_t), ("active", C.c_int32),
                ("pending", C.c_int32), ("host_rebuild_s", C.c_double), ("host_launch_s", C.c_double),
                ("host_admit_s", C.c_double), ("host_wait_s", C.c_double), ("host_retire_s", C.c_double)]


# exported symbols of include/swe.h and their ctypes signatures
_VP, _F, _D, _U8 = C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_uint8)
SIGNATURES = {
    "swe_workspace_bytes": (C.c_int, [C.POINTER(Params), C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "swe_init_domain": (C.c_int, [C.POINTER(Params), _VP, C.c_size_t, _VP, C.c_int32, C.c_int32,
                                  _F, _U8, _F, _F, _F, _F, _F, C.POINTER(_VP)]),
    "swe_set_forcing": (C.c_int, [_VP, C.c_int32, C.c_int32, _D, _F]),
    "swe_set_boundary_field": (C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32, _D, _F]),
    "swe_wind_field_bytes": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "swe_set_wind_field": (C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32, _D, _F, C.c_double, _VP,
                                     C.c_size_t]),
    "swe_set_stress_field": (C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32, _D, _F, _VP, C.c_size_t]),
    "swe_step": (C.c_int, [_VP, C.c_int32]),
    "swe_step_dt": (C.c_int, [_VP, C.c_int32, _D]),
    "swe_set_dt_policy": (C.c_int, [_VP, C.c_double]),
    "swe_run_until": (C.c_int, [_VP, C.c_double, C.POINTER(C.c_int64)]),
    "swe_read_state": (C.c_int, [_VP, _VP, _VP, _VP, _D, _D]),
    "swe_set_state": (C.c_int, [_VP, _F, _F, _F, C.c_double]),
    "swe_diagnostics": (C.c_int, [_VP, _D, _D]),
    "swe_status": (C.c_int, [_VP]),
    "swe_set_tiling": (C.c_int, [_VP, C.c_int32, C.c_int32]),
    "swe_get_tiling": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)]),
    "swe_set_stage_tiling": (C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "swe_get_stage_tiling": (C.c_int, [_VP, C.c_int32] + [C.POINTER(C.c_int32)] * 5),
    "swe_list_tilings": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]),
    "swe_autotune_tiling": (C.c_int, [_VP, C.POINTER(C.c_int32)]),
    "swe_enable_timing": (C.c_int, [_VP, C.c_int32]),
    "swe_stage_times": (C.c_int, [_VP, _D, _D, C.POINTER(C.c_int64), C.c_int32]),
    "swe_destroy": (None, [_VP]),
    "swe_last_error": (C.c_char_p, []),
    "swe_ensemble_workspace_bytes": (C.c_int, [C.POINTER(_VP), C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "swe_ensemble_create": (C.c_int, [C.POINTER(_VP), C.c_int32, _VP, C.c_size_t, _VP, C.c_int32, C.c_int32,
                                      C.POINTER(_VP)]),
    "swe_ensemble_step": (C.c_int, [_VP, C.c_int32]),
    "swe_ensemble_info": (C.c_int, [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int32)]),
    "swe_ensemble_enable_timing": (C.c_int, [_VP, C.c_int32]),
    "swe_ensemble_stage_times": (C.c_int, [_VP, _D, _D, C.POINTER(C.c_int64), C.c_int32]),
    "swe_ensemble_use_graphs": (C.c_int, [_VP, C.c_int32]),
    "swe_ensemble_destroy": (None, [_VP]),
    "swe_server_create": (C.c_int, [_VP, C.c_size_t, _VP, _VP, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                    C.POINTER(_VP)]),
    "swe_server_submit": (C.c_int, [_VP, C.c_void_p]),
    "swe_server_tick": (C.c_int, [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "swe_server_poll": (C.c_int, [_VP, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "swe_server_get_stats": (C.c_int, [_VP, C.c_void_p]),
    "swe_server_destroy": (None, [_VP]),
    "swe_reconstruct_bathymetry": (C.c_int, [C.c_int32, C.c_int32, _VP, _VP, C.c_int32, C.c_float, _VP, _VP,
                                             _VP]),
    "swe_reconstruct_bathymetry_noalloc": (C.c_int, [C.c_int32, C.c_int32, _VP, _VP, C.c_int32, C.c_float, _VP,
                                                     _VP]),
    "swe_erode_land": (C.c_int, [C.c_int32, C.c_int32, _VP, _VP, _VP, _VP, _VP, C.c_float, _VP, _VP, _VP, _VP,
                                 _VP, _VP]),
    "swe_refine2": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, _VP, _VP, C.c_float, _VP, _VP, _VP, _VP, _VP]),
    "swe_coarsen2": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1912_02457_amd.build.build() "
                          "(hipcc, gfx950); there is no CPU fallback")
    L = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != SWE_OK:
        raise SweError(rc, load_library().swe_last_error().decode(errors="replace"))


def _f32(a, shape) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def _fp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_F)


def make_params(nx, ny, dx, dy, *, g=9.81, courant=0.45, theta=1.3, kappa=1e-3,
                bc: Sequence[int] = (BC_WALL,) * 4, friction=FRICTION_NONE, friction_coeff=0.0,
                rho_w=1025.0, frs_width=10, frs_d0=2.0, north_projection=False,
                compensated_state=True) -> Params:
    p = Params()
    p.nx, p.ny, p.dx, p.dy, p.g = int(nx), int(ny), float(dx), float(dy), float(g)
    p.courant, p.theta, p.kappa = float(courant), float(theta), float(kappa)
    for k in range(4):
        p.bc[k] = int(bc[k])
    p.friction, p.friction_coeff = int(friction), float(friction_coeff)
    p.rho_w, p.frs_width, p.frs_d0 = float(rho_w), int(frs_width), float(frs_d0)
    p.north_projection = 1 if north_projection else 0
    p.compensated_state = 1 if compensated_state else 0
    return p


def workspace_bytes(params: Params, max_wind_times: int = 1, max_bnd_times: int = 0) -> int:
    n = C.c_size_t()
    _check(load_library().swe_workspace_bytes(C.byref(params), max_wind_times, max_bnd_times, C.byref(n)))
    return n.value


class Domain:
    """One simulation domain resident on the GPU."""

    def __init__(self, params: Params, Hc, f, eta, hu, hv, land=None, north=None, *,
                 max_wind_times: int = 8, max_bnd_times: int = 0, device=None, stream=None):
        import torch
        L = load_library()
        self.params = params
        nx, ny = params.nx, params.ny
        self.nx, self.ny = nx, ny
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = workspace_bytes(params, max_wind_times, max_bnd_times)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise SweError(SWE_E_ARG, "workspace tensor is not 256-byte aligned")
        Hc = _f32(Hc, (ny + 1, nx + 1))
        f = _f32(f, (ny, nx))
        eta, hu, hv = (_f32(a, (ny, nx)) for a in (eta, hu, hv))
        north = None if north is None else _f32(north, (ny, nx))
        land_a = None if land is None else np.ascontiguousarray(np.asarray(land, dtype=np.uint8))
        if land_a is not None and land_a.shape != (ny, nx):
            raise ValueError("land mask shape")
        h = C.c_void_p()
        _check(L.swe_init_domain(
            C.byref(params), C.c_void_p(self.workspace.data_ptr()), nbytes,
            C.c_void_p(self.stream.cuda_stream), max_wind_times, max_bnd_times,
            _fp(Hc), None if land_a is None else land_a.ctypes.data_as(_U8), _fp(f), _fp(north),
            _fp(eta), _fp(hu), _fp(hv), C.byref(h)))
        self._h = h

    @classmethod
    def from_workload(cls, wl, *, north_projection=False, compensated_state=True, max_wind_times=None,
                      max_bnd_times=None,
                      device=None, stream=None) -> "Domain":
        p = make_params(wl.nx, wl.ny, wl.dx, wl.dy, g=wl.g, courant=wl.courant, theta=wl.theta,
                        kappa=wl.kappa, bc=wl.bc, friction=wl.friction,
                        friction_coeff=wl.friction_coeff, rho_w=wl.rho_w,
                        frs_width=wl.frs_width, frs_d0=wl.frs_d0,
                        north_projection=north_projection, compensated_state=compensated_state)
        nw = len(wl.wind_t)
        nb = 0 if wl.bnd is None else len(wl.bnd_t)
        dom = cls(p, wl.Hc, wl.f, wl.eta, wl.hu, wl.hv, land=wl.land, north=wl.north,
                  max_wind_times=max(nw, max_wind_times or 1),
                  max_bnd_times=max(nb, max_bnd_times or 0), device=device, stream=stream)
        dom.set_wind(wl.wind_t, wl.wind_tau)
        if wl.bnd is not None:
            if getattr(wl, "bnd_nx", 0) > 0:
                dom.set_boundary_field(wl.bnd_t, wl.bnd, wl.bnd_nx, wl.bnd_ny)
            else:
                dom.set_boundary(wl.bnd_t, wl.bnd)
        if getattr(wl, "w10", None) is not None:
            dom.set_wind_field(wl.w10_t, wl.w10, rho_air=getattr(wl, "rho_a", 1.225),
                               kind=getattr(wl, "w10_kind", 0))
        if getattr(wl, "dt_interval", 0.0) > 0.0:
            dom.set_dt_policy(wl.dt_interval)
        return dom

    # -- forcing -----------------------------------------------------------
    def set_wind(self, times, tau):
        t = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
        d = _f32(tau, (len(t), 2))
        _check(load_library().swe_set_forcing(self._h, FORCING_WIND_STRESS, len(t),
                                              t.ctypes.data_as(_D), _fp(d)))

    def set_boundary(self, times, data):
        t = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
        d = _f32(data, (len(t), 3, 2 * self.ny + 2 * self.nx))
        _check(load_library().swe_set_forcing(self._h, FORCING_BOUNDARY, len(t),
                                              t.ctypes.data_as(_D), _fp(d)))

    def set_boundary_field(self, times, data, n_x: int, n_y: int):
        """Boundary snapshots at their own spacing, [n_times][3][2 n_y + 2 n_x]
        (``swe_set_boundary_field``)."""
        t = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
        d = _f32(data, (len(t), 3, 2 * n_y + 2 * n_x))
        _check(load_library().swe_set_boundary_field(self._h, len(t), int(n_x), int(n_y),
                                                     t.ctypes.data_as(_D), _fp(d)))

    def set_wind_field(self, times, w10, rho_air: float = 1.225, kind: int = 0):
        """A field on its own grid, array [n_times][ny_w][nx_w][2]: wind at
        10 m in m/s (kind 0, Large and Pond stress per cell,
        ``swe_set_wind_field``) or wind stress in N/m^2 (kind 1,
        ``swe_set_stress_field``); trilinear interpolation; None removes it."""
        import torch
        L = load_library()
        if w10 is None:
            _check(L.swe_set_wind_field(self._h, 0, 0, 0, None, None, 1.0, None, 0))
            self.wind_field = None
            return
        t = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
        w = np.ascontiguousarray(np.asarray(w10, dtype=np.float32))
        if w.ndim != 4 or w.shape[0] != len(t) or w.shape[3] != 2:
            raise ValueError("w10 must be [n_times][ny_w][nx_w][2]")
        n = C.c_size_t()
        _check(L.swe_wind_field_bytes(len(t), w.shape[2], w.shape[1], C.byref(n)))
        buf = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        if kind == 1:
            _check(L.swe_set_stress_field(self._h, len(t), w.shape[2], w.shape[1], t.ctypes.data_as(_D), _fp(w),
                                          C.c_void_p(buf.data_ptr()), n.value))
        elif kind == 0:
            _check(L.swe_set_wind_field(self._h, len(t), w.shape[2], w.shape[1], t.ctypes.data_as(_D), _fp(w),
                                        float(rho_air), C.c_void_p(buf.data_ptr()), n.value))
        else:
            raise ValueError("kind must be 0 (wind at 10 m) or 1 (stress)")
        self.wind_field = buf  # borrowed by the library until replaced

    # -- time stepping -----------------------------------------------------
    def step(self, n: int = 1):
        _check(load_library().swe_step(self._h, int(n)))

    def set_dt_policy(self, interval: float = 0.0):
        """dt from the CFL condition every step (0) or only once every
        ``interval`` simulated seconds (``swe_set_dt_policy``)."""
        _check(load_library().swe_set_dt_policy(self._h, float(interval)))

    def step_dt(self, dts):
        d = np.ascontiguousarray(np.asarray(dts, dtype=np.float64))
        _check(load_library().swe_step_dt(self._h, len(d), d.ctypes.data_as(_D)))

    def run_until(self, t_end: float) -> int:
        n = C.c_int64()
        _check(load_library().swe_run_until(self._h, float(t_end), C.byref(n)))
        return n.value

    # -- state -------------------------------------------------------------
    def read_state(self):
        """Returns (eta, hu, hv, t, dt_next) with host float32 arrays."""
        e = np.empty((self.ny, self.nx), np.float32)
        u = np.empty_like(e)
        v = np.empty_like(e)
        t, dt = C.c_double(), C.c_double()
        _check(load_library().swe_read_state(self._h, e.ctypes.data, u.ctypes.data, v.ctypes.data,
                                             C.byref(t), C.byref(dt)))
        return e, u, v, t.value, dt.value

    def read_state_into(self, eta, hu, hv):
        """Copy the state into device tensors of shape (ny, nx), float32."""
        for a in (eta, hu, hv):
            if a.dtype.itemsize != 4 or tuple(a.shape) != (self.ny, self.nx) or not a.is_contiguous():
                raise ValueError("expected contiguous float32 (ny, nx) tensors")
        t, dt = C.c_double(), C.c_double()
        _check(load_library().swe_read_state(self._h, eta.data_ptr(), hu.data_ptr(), hv.data_ptr(),
                                             C.byref(t), C.byref(dt)))
        return t.value, dt.value

    def set_state(self, eta, hu, hv, t: float = 0.0):
        e, u, v = (_f32(a, (self.ny, self.nx)) for a in (eta, hu, hv))
        _check(load_library().swe_set_state(self._h, _fp(e), _fp(u), _fp(v), float(t)))

    def diagnostics(self):
        m, en = C.c_double(), C.c_double()
        _check(load_library().swe_diagnostics(self._h, C.byref(m), C.byref(en)))
        return m.value, en.value

    def status(self) -> int:
        return load_library().swe_status(self._h)

    def set_tiling(self, rows_per_wave: int = 0, order: int = -1):
        _check(load_library().swe_set_tiling(self._h, int(rows_per_wave), int(order)))

    def set_stage_tiling(self, stage: int, rows_per_wave: int, tail_rows_per_wave: int = 0, tail_rows: int = 0,
                         order: int = -1):
        """Tiling of one stage kernel: bands of rows_per_wave rows, and with
        tail_rows_per_wave > 0 the last rows (at least tail_rows) in bands of
        tail_rows_per_wave rows launched after the others."""
        _check(load_library().swe_set_stage_tiling(self._h, int(stage), int(rows_per_wave), int(tail_rows_per_wave),
                                                   int(tail_rows), int(order)))

    def stage_tiling(self, stage: int):
        """(rows per wave, tail rows per wave, tail rows, order, wavefronts per
        launch) of a stage kernel; the tail values are 0 for one band height."""
        v = [C.c_int32() for _ in range(5)]
        _check(load_library().swe_get_stage_tiling(self._h, int(stage), *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def list_tilings(self, stage: int):
        """Every (rows per wave, tail rows per wave, tail rows) the tuner may
        time for a stage kernel on this domain."""
        n = C.c_int32()
        lib = load_library()
        _check(lib.swe_list_tilings(self._h, int(stage), None, 0, C.byref(n)))
        buf = (C.c_int32 * (3 * n.value))()
        _check(lib.swe_list_tilings(self._h, int(stage), buf, n.value, C.byref(n)))
        return [tuple(buf[3 * k:3 * k + 3]) for k in range(n.value)]

    def autotune(self) -> int:
        """Time both stage kernels over candidate tilings (the simulation does
        not advance) and keep the fastest per stage; returns stage 1's rows per
        tile."""
        r = C.c_int32()
        _check(load_library().swe_autotune_tiling(self._h, C.byref(r)))
        return r.value

    def tiling(self, stage: int = 1):
        """(rows per wave, tile order, wavefronts per launch) of a stage kernel"""
        by, o, w = C.c_int32(), C.c_int32(), C.c_int32()
        _check(load_library().swe_get_tiling(self._h, int(stage), C.byref(by), C.byref(o), C.byref(w)))
        return by.value, o.value, w.value

    def enable_timing(self, on: bool = True):
        _check(load_library().swe_enable_timing(self._h, 1 if on else 0))

    def stage_times(self, reset: bool = True):
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        _check(load_library().swe_stage_times(self._h, C.byref(a), C.byref(b), C.byref(n), 1 if reset else 0))
        return a.value, b.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            load_library().swe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """Domains advanced together: one persistent launch per RK stage drains a
    device queue of (member, tile) items over all members.  Each member keeps
    its own time step; members stay usable for read_state / diagnostics and
    return to their own streams on close()."""

    def __init__(self, members: Sequence[Domain], *, rows_per_wave: int = 0, chunk: int = 0, stream=None):
        import torch
        L = load_library()
        if not members:
            raise ValueError("an ensemble needs at least one member")
        self.members = list(members)
        dev = self.members[0].device
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        n = len(self.members)
        arr = (_VP * n)(*[m._h for m in self.members])
        nb = C.c_size_t()
        _check(L.swe_ensemble_workspace_bytes(arr, n, int(rows_per_wave), C.byref(nb)))
        self.workspace = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=dev)
        h = C.c_void_p()
        _check(L.swe_ensemble_create(arr, n, C.c_void_p(self.workspace.data_ptr()), nb.value,
                                     C.c_void_p(self.stream.cuda_stream), int(rows_per_wave), int(chunk),
                                     C.byref(h)))
        self._h = h

    def step(self, n: int = 1):
        _check(load_library().swe_ensemble_step(self._h, int(n)))

    def use_graphs(self, on: bool = True):
        _check(load_library().swe_ensemble_use_graphs(self._h, 1 if on else 0))

    def info(self):
        """(rows per tile, items per atomic, work items per stage, blocks per launch)"""
        r, c, i, b = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int32()
        _check(load_library().swe_ensemble_info(self._h, C.byref(r), C.byref(c), C.byref(i), C.byref(b)))
        return r.value, c.value, i.value, b.value

    def enable_timing(self, on: bool = True):
        _check(load_library().swe_ensemble_enable_timing(self._h, 1 if on else 0))

    def stage_times(self, reset: bool = True):
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        _check(load_library().swe_ensemble_stage_times(self._h, C.byref(a), C.byref(b), C.byref(n),
                                                       1 if reset else 0))
        return a.value, b.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            load_library().swe_ensemble_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def params_of(wl, north_projection=False, compensated_state=True) -> Params:
    return make_params(wl.nx, wl.ny, wl.dx, wl.dy, g=wl.g, courant=wl.courant, theta=wl.theta,
                       kappa=wl.kappa, bc=wl.bc, friction=wl.friction, friction_coeff=wl.friction_coeff,
                       rho_w=wl.rho_w, frs_width=wl.frs_width, frs_d0=wl.frs_d0,
                       north_projection=north_projection, compensated_state=compensated_state)


class Server:
    """Continuous-batching serving loop over one device arena (a torch
    uint8 tensor of ``arena_bytes``): submit requests at any time, call
    tick() repeatedly, poll() the finished ones with their final state."""

    def __init__(self, arena_bytes: int, *, max_active: int = 64, steps_per_tick: int = 32,
                 rows_per_wave: int = 0, chunk: int = 0, device=None, stream=None, upload_stream=None):
        import torch
        L = load_library()
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.upload_stream = upload_stream if upload_stream is not None else torch.cuda.Stream(self.device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(L.swe_server_create(C.c_void_p(self.arena.data_ptr()), int(arena_bytes),
                                   C.c_void_p(self.stream.cuda_stream),
                                   C.c_void_p(self.upload_stream.cuda_stream), int(max_active),
                                   int(steps_per_tick), int(rows_per_wave), int(chunk), C.byref(h)))
        self._h = h
        self._out = {}  # id -> host result arrays, alive until polled

    def submit(self, wl, horizon: float, req_id: int, *, keep_result: bool = True, north_projection: bool = False,
               compensated_state: bool = True):
        """Queue workload ``wl`` to be advanced to simulated time ``horizon``."""
        ny, nx = wl.ny, wl.nx
        r = Request()
        r.id = int(req_id)
        r.params = params_of(wl, north_projection=north_projection, compensated_state=compensated_state)
        r.horizon = float(horizon)
        Hc = _f32(wl.Hc, (ny + 1, nx + 1))
        f = _f32(wl.f, (ny, nx))
        eta, hu, hv = (_f32(a, (ny, nx)) for a in (wl.eta, wl.hu, wl.hv))
        north = None if wl.north is None else _f32(wl.north, (ny, nx))
        land = None if wl.land is None else np.ascontiguousarray(np.asarray(wl.land, dtype=np.uint8))
        r.Hc, r.f, r.eta, r.hu, r.hv = _fp(Hc), _fp(f), _fp(eta), _fp(hu), _fp(hv)
        r.theta = _fp(north)
        if land is not None:
            r.land = land.ctypes.data_as(_U8)
        wt = np.ascontiguousarray(np.asarray(wl.wind_t, dtype=np.float64))
        wtau = _f32(wl.wind_tau, (len(wt), 2))
        r.n_wind = len(wt)
        r.wind_t, r.wind_tau = wt.ctypes.data_as(_D), _fp(wtau)
        if wl.bnd is not None:
            bt = np.ascontiguousarray(np.asarray(wl.bnd_t, dtype=np.float64))
            bd = _f32(wl.bnd, (len(bt), 3, 2 * ny + 2 * nx))
            r.n_bnd = len(bt)
            r.bnd_t, r.bnd = bt.ctypes.data_as(_D), _fp(bd)
        out = None
        if keep_result:
            out = tuple(np.empty((ny, nx), np.float32) for _ in range(3))
            r.out_eta, r.out_hu, r.out_hv = (_fp(a) for a in out)
        _check(load_library().swe_server_submit(self._h, C.addressof(r)))
        self._out[int(req_id)] = out

    def tick(self):
        """One tick; returns (active, waiting) request counts."""
        a, p = C.c_int32(), C.c_int32()
        _check(load_library().swe_server_tick(self._h, C.byref(a), C.byref(p)))
        return a.value, p.value

    def poll(self, max_n: int = 4096):
        """Finished requests: list of dicts with id, t, steps, tick, status
        and the final (eta, hu, hv) host arrays (or None)."""
        buf = (Completion * max_n)()
        n = C.c_int32()
        _check(load_library().swe_server_poll(self._h, C.addressof(buf), max_n, C.byref(n)))
        res = []
        for k in range(n.value):
            c = buf[k]
            res.append(dict(id=c.id, t=c.t, steps=c.steps, tick=c.tick, status=c.status,
                            state=self._out.pop(c.id, None)))
        return res

    def stats(self):
        st = ServerStats()
        _check(load_library().swe_server_get_stats(self._h, C.addressof(st)))
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load_library().swe_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- preprocessing of the input fields (device tensors in and out) --------

def _dev(t, dtype, shape, name):
    """Device pointer of a contiguous CUDA tensor of the given dtype/shape."""
    import torch
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _stream_of(t, stream):
    import torch
    return C.c_void_p((stream if stream is not None else torch.cuda.current_stream(t.device)).cuda_stream)


def reconstruct_bathymetry(Hm, land=None, *, iters: int = 10, smooth: float = 0.5, out=None, scratch=None,
                           stream=None):
    """Corner depths [ny+1, nx+1] from cell depths Hm [ny, nx] on the device
    (``swe_reconstruct_bathymetry``); returns ``out``."""
    import torch
    ny, nx = Hm.shape
    if out is None:
        out = torch.empty((ny + 1, nx + 1), dtype=torch.float32, device=Hm.device)
    if scratch is None and iters > 0:
        scratch = torch.empty((ny + 1, nx + 1), dtype=torch.float32, device=Hm.device)
    load_library()
    _check(_lib.swe_reconstruct_bathymetry(nx, ny, _dev(Hm, torch.float32, (ny, nx), "Hm"),
                                           _dev(land, torch.uint8, (ny, nx), "land"), int(iters), float(smooth),
                                           _dev(out, torch.float32, (ny + 1, nx + 1), "out"),
                                           _dev(scratch, torch.float32, (ny + 1, nx + 1), "scratch"),
                                           _stream_of(Hm, stream)))
    return out


def reconstruct_bathymetry_noalloc(Hm, land=None, *, iters: int = 10, smooth: float = 0.5, out=None,
                                   stream=None):
    """``swe_reconstruct_bathymetry_noalloc``: the same reconstruction with the
    library's own static scratch (no device allocation in the call; ``out``
    must then be given by a caller that cannot allocate).  Returns ``out``."""
    import torch
    ny, nx = Hm.shape
    if out is None:
        out = torch.empty((ny + 1, nx + 1), dtype=torch.float32, device=Hm.device)
    load_library()
    _check(_lib.swe_reconstruct_bathymetry_noalloc(nx, ny, _dev(Hm, torch.float32, (ny, nx), "Hm"),
                                                   _dev(land, torch.uint8, (ny, nx), "land"), int(iters),
                                                   float(smooth), _dev(out, torch.float32, (ny + 1, nx + 1), "out"),
                                                   _stream_of(Hm, stream)))
    return out


def erode_land(land, Hm, eta=None, hu=None, hv=None, *, land_depth: float = 5.0, stream=None):
    """One erosion of the land mask on the device (``swe_erode_land``).
    Returns (land, Hm, eta, hu, hv) as new tensors (None where not given)."""
    import torch
    ny, nx = land.shape
    outs = [torch.empty_like(land), torch.empty_like(Hm)] + [None if a is None else torch.empty_like(a)
                                                             for a in (eta, hu, hv)]
    f32 = torch.float32
    load_library()
    _check(_lib.swe_erode_land(nx, ny, _dev(land, torch.uint8, (ny, nx), "land"), _dev(Hm, f32, (ny, nx), "Hm"),
                               _dev(eta, f32, (ny, nx), "eta"), _dev(hu, f32, (ny, nx), "hu"),
                               _dev(hv, f32, (ny, nx), "hv"), float(land_depth),
                               *[_dev(o, torch.uint8 if k == 0 else f32, (ny, nx), "out")
                                 for k, o in enumerate(outs)], _stream_of(land, stream)))
    return tuple(outs)


def refine2(fields=None, land=None, Hc=None, *, theta: float = 1.0, stream=None):
    """Factor-two refinement on the device (``swe_refine2``).  fields is a
    [n, ny, nx] float32 tensor (or None); returns (fields, land, Hc) refined
    (None where not given)."""
    import torch
    ref = next(t for t in (fields, land, Hc) if t is not None)
    if fields is not None:
        nf, ny, nx = fields.shape
    elif land is not None:
        (ny, nx), nf = land.shape, 0
    else:
        ny, nx, nf = Hc.shape[0] - 1, Hc.shape[1] - 1, 0
    if land is not None and nf == 0:
        raise ValueError("refining the land mask needs at least one field")
    dev = ref.device
    fo = None if fields is None else torch.empty((nf, 2 * ny, 2 * nx), dtype=torch.float32, device=dev)
    lo = None if land is None else torch.empty((2 * ny, 2 * nx), dtype=torch.uint8, device=dev)
    ho = None if Hc is None else torch.empty((2 * ny + 1, 2 * nx + 1), dtype=torch.float32, device=dev)
    load_library()
    _check(_lib.swe_refine2(nx, ny, nf, _dev(fields, torch.float32, (nf, ny, nx), "fields"),
                            _dev(land, torch.uint8, (ny, nx), "land"), float(theta), _dev(fo, torch.float32,
                            (nf, 2 * ny, 2 * nx), "fields_out"), _dev(lo, torch.uint8, (2 * ny, 2 * nx), "land_out"),
                            _dev(Hc, torch.float32, (ny + 1, nx + 1), "Hc"),
                            _dev(ho, torch.float32, (2 * ny + 1, 2 * nx + 1), "Hc_out"), _stream_of(ref, stream)))
    return fo, lo, ho


def coarsen2(fields=None, land=None, Hc=None, *, stream=None):
    """Factor-two coarsening on the device (``swe_coarsen2``); nx, ny even.
    Returns (fields, land, Hc) coarsened (None where not given)."""
    import torch
    ref = next(t for t in (fields, land, Hc) if t is not None)
    if fields is not None:
        nf, ny, nx = fields.shape
    elif land is not None:
        (ny, nx), nf = land.shape, 0
    else:
        ny, nx, nf = Hc.shape[0] - 1, Hc.shape[1] - 1, 0
    if land is not None and nf == 0:
        raise ValueError("coarsening the land mask needs at least one field")
    dev = ref.device
    cy, cx = ny // 2, nx // 2
    fo = None if fields is None else torch.empty((nf, cy, cx), dtype=torch.float32, device=dev)
    lo = None if land is None else torch.empty((cy, cx), dtype=torch.uint8, device=dev)
    ho = None if Hc is None else torch.empty((cy + 1, cx + 1), dtype=torch.float32, device=dev)
    load_library()
    _check(_lib.swe_coarsen2(nx, ny, nf, _dev(fields, torch.float32, (nf, ny, nx), "fields"),
                             _dev(land, torch.uint8, (ny, nx), "land"), _dev(fo, torch.float32, (nf, cy, cx),
                             "fields_out"), _dev(lo, torch.uint8, (cy, cx), "land_out"),
                             _dev(Hc, torch.float32, (ny + 1, nx + 1), "Hc"),
                             _dev(ho, torch.float32, (cy + 1, cx + 1), "Hc_out"), _stream_of(ref, stream)))
    return fo, lo, ho
