"""ctypes front-end of the plain FP64 C oracle (``swe_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``; never by the product path.  It shares no
code with the HIP implementation; inputs come from the ``workloads`` package
(float32 arrays widened here to float64).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "swe_oracle.c")
# SWE_ORACLE_LIB lets the mutation test load a deliberately broken copy
LIB = os.environ.get("SWE_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None
_D = C.POINTER(C.c_double)


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("g", C.c_double),
        ("courant", C.c_double), ("theta", C.c_double), ("kappa", C.c_double),
        ("bc", C.c_int32 * 4), ("friction", C.c_int32), ("friction_coeff", C.c_double),
        ("rho_w", C.c_double), ("frs_width", C.c_int32), ("frs_d0", C.c_double),
        ("wind_n", C.c_int32), ("wind_t", _D), ("wind_tau", _D),
        ("bnd_n", C.c_int32), ("bnd_t", _D), ("bnd", _D),
        ("w10_n", C.c_int32), ("w10_nx", C.c_int32), ("w10_ny", C.c_int32),
        ("w10_t", _D), ("w10", _D), ("rho_a", C.c_double), ("dt_interval", C.c_double),
        ("w10_kind", C.c_int32),
    ]


class _Static(C.Structure):
    _fields_ = [("Hc", _D), ("land", C.POINTER(C.c_uint8)), ("f", _D), ("north", _D)]


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("SWE_ORACLE_LIB") and (
                not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build(force=True)
        L = C.CDLL(LIB)
        P, S = C.POINTER(_Params), C.POINTER(_Static)
        L.or_desing.restype = C.c_double
        L.or_desing.argtypes = [C.c_double, C.c_double]
        L.or_minmod3.restype = C.c_double
        L.or_minmod3.argtypes = [C.c_double] * 3
        L.or_limited_slope.restype = C.c_double
        L.or_limited_slope.argtypes = [C.c_double] * 3
        L.or_cu_flux.restype = None
        L.or_cu_flux.argtypes = [_D, _D, C.c_double, C.c_double, C.c_double, _D]
        L.or_rhs.restype = C.c_int
        L.or_rhs.argtypes = [P, S, _D, _D, _D, C.c_double, _D, _D, _D, _D]
        L.or_friction.restype = C.c_int
        L.or_friction.argtypes = [P, S, _D, _D, _D, _D]
        L.or_cfl_dt.restype = C.c_double
        L.or_cfl_dt.argtypes = [P, S, _D, _D, _D]
        L.or_step.restype = C.c_int
        L.or_step.argtypes = [P, S, _D, _D, _D, _D, C.c_double]
        L.or_run.restype = C.c_int64
        L.or_run.argtypes = [P, S, _D, _D, _D, _D, C.c_int64, C.c_double, C.c_double, _D, _D]
        L.or_diagnostics.restype = None
        L.or_diagnostics.argtypes = [P, S, _D, _D, _D, _D, _D]
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.restype = None
        L.or_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# elementary definitions -----------------------------------------------------

def desing(h: float, kappa: float) -> float:
    return lib().or_desing(float(h), float(kappa))


def minmod3(a, b, c) -> float:
    return lib().or_minmod3(float(a), float(b), float(c))


def limited_slope(dm, dp, theta) -> float:
    return lib().or_limited_slope(float(dm), float(dp), float(theta))


def cu_flux(L, R, Hf, g=9.81, kappa=1e-3) -> np.ndarray:
    Lb, Rb, out = _f64(L), _f64(R), np.zeros(3)
    lib().or_cu_flux(_dp(Lb), _dp(Rb), float(Hf), float(g), float(kappa), _dp(out))
    return out


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's loops over rows (results do not depend on it)."""
    lib().or_set_num_threads(int(n))


def resample_boundary(data, nx, ny, n_x, n_y):
    """Boundary snapshots given at their own spacing (section "Nesting the
    model": linear interpolation in space, like the wind) -> one value per
    boundary cell.  data [n][3][2 n_y + 2 n_x] holds the W and E sides (n_y
    samples each), then S and N (n_x); samples sit at the centres of equal
    parts of a side, values outside the first/last centre are held.
    Returns [n][3][2 ny + 2 nx]."""
    data = np.asarray(data, np.float64)
    out = np.empty(data.shape[:2] + (2 * ny + 2 * nx,))
    parts = [(0, n_y, 0, ny), (n_y, n_y, ny, ny), (2 * n_y, n_x, 2 * ny, nx), (2 * n_y + n_x, n_x, 2 * ny + nx, nx)]
    for a, n, b, m in parts:
        xp = (np.arange(n) + 0.5) / n        # sample centres along the side (unit length)
        x = (np.arange(m) + 0.5) / m          # cell centres
        for t in range(data.shape[0]):
            for f in range(3):
                out[t, f, b:b + m] = np.interp(x, xp, data[t, f, a:a + n])
    return out


class Oracle:
    """Oracle bound to one workload's static inputs and forcing."""

    def __init__(self, wl):
        self.wl = wl
        self.nx, self.ny = wl.nx, wl.ny
        self._keep = {}
        self.Hc = self._hold("Hc", _f64(wl.Hc))
        self.f = self._hold("f", _f64(wl.f))
        self.north = self._hold("north", _f64(wl.north))
        self.land = None if wl.land is None else self._hold(
            "land", np.ascontiguousarray(wl.land, dtype=np.uint8))
        wind_t = self._hold("wind_t", _f64(wl.wind_t))
        wind_tau = self._hold("wind_tau", _f64(wl.wind_tau).reshape(-1, 2))
        p = _Params()
        p.nx, p.ny = wl.nx, wl.ny
        p.dx, p.dy, p.g = wl.dx, wl.dy, wl.g
        p.courant, p.theta, p.kappa = wl.courant, wl.theta, wl.kappa
        for k in range(4):
            p.bc[k] = int(wl.bc[k])
        p.friction, p.friction_coeff = int(wl.friction), float(wl.friction_coeff)
        p.rho_w, p.frs_width, p.frs_d0 = wl.rho_w, int(wl.frs_width), wl.frs_d0
        p.wind_n, p.wind_t, p.wind_tau = len(wind_t), _dp(wind_t), _dp(wind_tau)
        if wl.bnd is not None:
            bt = self._hold("bnd_t", _f64(wl.bnd_t))
            raw = _f64(wl.bnd)
            if getattr(wl, "bnd_nx", 0) > 0:
                raw = resample_boundary(raw, wl.nx, wl.ny, wl.bnd_nx, wl.bnd_ny)
            bd = self._hold("bnd", raw)
            p.bnd_n, p.bnd_t, p.bnd = len(bt), _dp(bt), _dp(bd)
        else:
            p.bnd_n = 0
        w10 = getattr(wl, "w10", None)
        if w10 is not None:
            wt = self._hold("w10_t", _f64(wl.w10_t))
            wd = self._hold("w10", _f64(w10))
            p.w10_n, p.w10_ny, p.w10_nx = wd.shape[0], wd.shape[1], wd.shape[2]
            p.w10_t, p.w10 = _dp(wt), _dp(wd)
        p.rho_a = float(getattr(wl, "rho_a", 1.225))
        p.dt_interval = float(getattr(wl, "dt_interval", 0.0))
        p.w10_kind = int(getattr(wl, "w10_kind", 0))
        self.p = p
        s = _Static()
        s.Hc, s.f, s.north = _dp(self.Hc), _dp(self.f), _dp(self.north)
        s.land = None if self.land is None else self.land.ctypes.data_as(C.POINTER(C.c_uint8))
        self.s = s

    def _hold(self, k, a):
        self._keep[k] = a
        return a

    def initial_state(self):
        return tuple(_f64(a).copy() for a in (self.wl.eta, self.wl.hu, self.wl.hv))

    def rhs(self, state, t=0.0, faces=False):
        e, u, v = (_f64(a) for a in state)
        n = self.nx * self.ny
        M = [np.zeros((self.ny, self.nx)) for _ in range(3)]
        F = np.zeros((12, self.ny, self.nx)) if faces else None
        rc = lib().or_rhs(C.byref(self.p), C.byref(self.s), _dp(e), _dp(u), _dp(v), float(t),
                          _dp(M[0]), _dp(M[1]), _dp(M[2]), _dp(F))
        if rc:
            raise RuntimeError(f"or_rhs failed ({rc})")
        assert n == M[0].size
        return (tuple(M), F) if faces else tuple(M)

    def friction(self, state):
        e, u, v = (_f64(a) for a in state)
        S = np.zeros((self.ny, self.nx))
        rc = lib().or_friction(C.byref(self.p), C.byref(self.s), _dp(e), _dp(u), _dp(v), _dp(S))
        if rc:
            raise RuntimeError(f"or_friction failed ({rc})")
        return S

    def cfl_dt(self, state) -> float:
        e, u, v = (_f64(a) for a in state)
        return lib().or_cfl_dt(C.byref(self.p), C.byref(self.s), _dp(e), _dp(u), _dp(v))

    def step(self, state, t: float, dt: float):
        e, u, v = (_f64(a).copy() for a in state)
        tt = C.c_double(t)
        rc = lib().or_step(C.byref(self.p), C.byref(self.s), _dp(e), _dp(u), _dp(v), C.byref(tt), float(dt))
        if rc:
            raise RuntimeError(f"or_step failed ({rc})")
        return (e, u, v), tt.value

    def run(self, state=None, t: float = 0.0, nsteps: int = 1, t_end: float = 0.0,
            dt_fixed: float = 0.0, dts=None, record_dt: bool = True):
        """Returns (state, t, dts, steps_taken)."""
        if state is None:
            state = self.initial_state()
        e, u, v = (_f64(a).copy() for a in state)
        tt = C.c_double(t)
        dts_in = None if dts is None else _f64(dts)
        out = np.zeros(max(int(nsteps), 1)) if record_dt else None
        k = lib().or_run(C.byref(self.p), C.byref(self.s), _dp(e), _dp(u), _dp(v), C.byref(tt),
                         int(nsteps), float(t_end), float(dt_fixed), _dp(dts_in), _dp(out))
        if k < 0:
            raise RuntimeError(f"or_run failed ({k})")
        return (e, u, v), tt.value, (out[:k] if record_dt else None), int(k)

    def diagnostics(self, state):
        e, u, v = (_f64(a) for a in state)
        m, en = C.c_double(), C.c_double()
        lib().or_diagnostics(C.byref(self.p), C.byref(self.s), _dp(e), _dp(u), _dp(v),
                             C.byref(m), C.byref(en))
        return m.value, en.value
