"""Helpers for the oracle pin tests: float64 workload construction and the
textbook exact Riemann solution of the shallow-water dam break.  Nothing here
re-implements the finite-volume scheme."""

from __future__ import annotations

import numpy as np

from workloads import BC_WALL, Workload

G = 9.81


def make_wl(Hc, eta, hu=None, hv=None, f=0.0, north=0.0, land=None, dx=1000.0, dy=None,
            bc=(BC_WALL,) * 4, **kw) -> Workload:
    eta = np.asarray(eta, dtype=np.float64)
    ny, nx = eta.shape
    z = np.zeros((ny, nx))
    hu = z.copy() if hu is None else np.asarray(hu, np.float64)
    hv = z.copy() if hv is None else np.asarray(hv, np.float64)
    f = np.broadcast_to(np.asarray(f, np.float64), (ny, nx)).copy()
    north = np.broadcast_to(np.asarray(north, np.float64), (ny, nx)).copy()
    Hc = np.broadcast_to(np.asarray(Hc, np.float64), (ny + 1, nx + 1)).copy()
    return Workload(name="pin", nx=nx, ny=ny, dx=float(dx), dy=float(dx if dy is None else dy),
                    Hc=Hc, f=f, north=north, eta=eta, hu=hu, hv=hv,
                    land=None if land is None else np.asarray(land, np.uint8), bc=tuple(bc), **kw)


def hbar(Hc):
    return 0.25 * (Hc[:-1, :-1] + Hc[:-1, 1:] + Hc[1:, :-1] + Hc[1:, 1:])


# --- exact Riemann solution for two fluid states at rest on a flat bed ----------

def _fk(h, hk):
    if h > hk:  # shock
        return (h - hk) * np.sqrt(0.5 * G * (h + hk) / (h * hk))
    return 2.0 * (np.sqrt(G * h) - np.sqrt(G * hk))  # rarefaction


def dam_break_depth(hL: float, hR: float, xi: np.ndarray) -> np.ndarray:
    """Depth of the self-similar dam-break solution at xi = x/t (dam at x=0,
    both sides initially at rest, hL > hR >= 0).  hR > 0 is Stoker's wet-bed
    solution, hR = 0 Ritter's dry-bed solution."""
    cL = np.sqrt(G * hL)
    xi = np.asarray(xi, dtype=np.float64)
    if hR <= 0.0:
        h = np.where(xi <= -cL, hL, np.where(xi >= 2.0 * cL, 0.0, (2.0 * cL - xi) ** 2 / (9.0 * G)))
        return h
    # Newton / bisection on f_L(h) + f_R(h) = 0 (uL = uR = 0)
    lo, hi = hR, hL
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _fk(mid, hL) + _fk(mid, hR) > 0.0:
            hi = mid
        else:
            lo = mid
    hs = 0.5 * (lo + hi)
    us = 0.5 * (_fk(hs, hR) - _fk(hs, hL))
    cs = np.sqrt(G * hs)
    cR = np.sqrt(G * hR)
    sR = cR * np.sqrt(0.5 * (hs + hR) * hs / (hR * hR))  # right shock speed
    fan = ((2.0 * cL - xi) / 3.0) ** 2 / G
    h = np.where(xi <= -cL, hL,
                 np.where(xi <= us - cs, fan, np.where(xi < sR, hs, hR)))
    return h


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    n = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (n if n > 0 else 1.0)
