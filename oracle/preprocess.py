"""FP64 reference of the input preprocessing the paper applies before the
hot path (sections "Bathymetry" and "Refinement and coarsening of grid").
Plain numpy, step by step in the paper's order; test infrastructure only
(imported by tests/, never by the product path).  It shares no code with
the HIP path or with the input generators.

* reconstruct_bathymetry: intersection depths of a piecewise bilinear
  surface from cell-centre depths -- planar slopes per cell, corner
  estimates averaged over the cells meeting at a corner, then repeated
  correction by the reconstructed midpoint misfit and smoothing.
* erode_land: one row of land cells turned into water; their surface by
  gray dilation (maximum over water neighbours), their depth set to the
  land value.
* refine2 / coarsen2: factor-two change of resolution of cell fields (slope
  limited reconstruction evaluated at the sub-cell centres / averages of the
  water children), of the land mask, and of the corner depths (the bilinear
  surface at the refined intersections / sampled at the coarse ones).

Readings (where the paper is not specific): slopes are minmod-limited
one-sided differences in cell units, a difference towards land or outside
the domain counts as 0; a corner touched only by land cells keeps the mean
of the four (land) cell values around it; smoothing is H <- (1 - w) H +
(w/4)(sum of the 4 neighbours) with edge values repeated, w = 1/2 by
default; the correction adds the
reconstructed misfit (the printed update adds it); land cells carry no
misfit; erosion uses the 4-neighbourhood and a cell outside the domain
counts as land; an eroded cell's momenta are 0.  Refinement uses the
scheme's generalized minmod (theta = 1 is plain minmod) with the same rule
toward land and the domain edge; coarsening averages the water children and
makes a coarse cell land only when all four children are land.
"""

from __future__ import annotations

import numpy as np


def _minmod(a, b):
    return np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def _slopes(v, wet):
    """Limited x and y slopes (cell units) of a cell field; differences to a
    non-wet or missing neighbour are 0."""
    ny, nx = v.shape
    sx = np.zeros((ny, nx))
    sy = np.zeros((ny, nx))
    for j in range(ny):
        for i in range(nx):
            if not wet[j, i]:
                continue
            dl = v[j, i] - v[j, i - 1] if i > 0 and wet[j, i - 1] else 0.0
            dr = v[j, i + 1] - v[j, i] if i + 1 < nx and wet[j, i + 1] else 0.0
            ds = v[j, i] - v[j - 1, i] if j > 0 and wet[j - 1, i] else 0.0
            dn = v[j + 1, i] - v[j, i] if j + 1 < ny and wet[j + 1, i] else 0.0
            sx[j, i] = _minmod(dl, dr)
            sy[j, i] = _minmod(ds, dn)
    return sx, sy


def _corner_average(v, wet):
    """Equations recon_1-3: evaluate each wet cell's plane at its four
    corners and average the estimates that meet at each intersection.
    Returns (corner values, number of wet cells at each corner)."""
    ny, nx = v.shape
    sx, sy = _slopes(v, wet)
    acc = np.zeros((ny + 1, nx + 1))
    cnt = np.zeros((ny + 1, nx + 1))
    for j in range(ny):
        for i in range(nx):
            if not wet[j, i]:
                continue
            for dj in (0, 1):
                for di in (0, 1):
                    acc[j + dj, i + di] += v[j, i] + (di - 0.5) * sx[j, i] + (dj - 0.5) * sy[j, i]
                    cnt[j + dj, i + di] += 1.0
    out = np.zeros((ny + 1, nx + 1))
    m = cnt > 0
    out[m] = acc[m] / cnt[m]
    return out, cnt


def _midpoints(Hc):
    return 0.25 * (Hc[:-1, :-1] + Hc[:-1, 1:] + Hc[1:, :-1] + Hc[1:, 1:])


def _smooth(Hc, w):
    """H <- (1 - w) H + (w/4) (sum of the 4 neighbours); a neighbour outside
    the domain is replaced by the corner itself."""
    ny1, nx1 = Hc.shape
    out = np.empty_like(Hc)
    for j in range(ny1):
        for i in range(nx1):
            s = (Hc[j, max(i - 1, 0)] + Hc[j, min(i + 1, nx1 - 1)] +
                 Hc[max(j - 1, 0), i] + Hc[min(j + 1, ny1 - 1), i])
            out[j, i] = (1.0 - w) * Hc[j, i] + 0.25 * w * s
    return out


def reconstruct_bathymetry(Hm, land=None, iters=10, smooth=0.5):
    """Corner depths [ny+1][nx+1] from cell-centre depths [ny][nx] (section
    "Bathymetry"): the initial guess of eqs. recon_1-3, then `iters` rounds
    of (a) misfit dH = Hm - (mean of the cell's 4 corners) on water cells,
    (b) its corner estimate by eqs. recon_1-3, added to the corners, and
    (c) smoothing with weight `smooth` (1/2 gives H/2 + sum of 4 / 8).
    Corners touching no water cell hold the mean of the four cell values
    around them (edge cells repeated) throughout."""
    Hm = np.asarray(Hm, np.float64)
    ny, nx = Hm.shape
    wet = np.ones((ny, nx), bool) if land is None else (np.asarray(land) == 0)
    Hs, cnt = _corner_average(Hm, wet)
    pad = np.pad(Hm, 1, mode="edge")
    fill = 0.25 * (pad[:-1, :-1] + pad[:-1, 1:] + pad[1:, :-1] + pad[1:, 1:])
    keep = cnt > 0
    Hs = np.where(keep, Hs, fill)
    for _ in range(iters):
        dH = np.where(wet, Hm - _midpoints(Hs), 0.0)
        dHc, c2 = _corner_average(dH, wet)
        Hs = Hs + np.where(c2 > 0, dHc, 0.0)
        Hs = np.where(keep, _smooth(Hs, smooth), fill)
    return Hs


def erode_land(land, Hm, eta, hu, hv, land_depth=5.0):
    """One erosion of the land mask: land cells with a water 4-neighbour
    become water with depth land_depth, surface = max over their water
    neighbours (gray dilation), momenta 0.  Returns (land, Hm, eta, hu, hv)."""
    land = np.asarray(land).astype(bool)
    ny, nx = land.shape
    L2, H2 = land.copy(), np.asarray(Hm, np.float64).copy()
    e2, u2, v2 = (np.asarray(a, np.float64).copy() for a in (eta, hu, hv))
    for j in range(ny):
        for i in range(nx):
            if not land[j, i]:
                continue
            nb = [(j, i - 1), (j, i + 1), (j - 1, i), (j + 1, i)]
            vals = [eta[b] for b in nb if 0 <= b[0] < ny and 0 <= b[1] < nx and not land[b]]
            if vals:
                L2[j, i] = False
                H2[j, i] = land_depth
                e2[j, i] = max(vals)
                u2[j, i] = v2[j, i] = 0.0
    return L2.astype(np.uint8), H2, e2, u2, v2


def _minmod3(a, b, c):
    if a > 0.0 and b > 0.0 and c > 0.0:
        return min(a, b, c)
    if a < 0.0 and b < 0.0 and c < 0.0:
        return max(a, b, c)
    return 0.0


def refine2(fields, land=None, Hc=None, theta=1.0):
    """Factor-two refinement (section "Refinement and coarsening of grid").
    Each cell field is reconstructed linearly per cell with the scheme's
    generalized minmod, minmod(theta D-, (D- + D+)/2, theta D+), and evaluated
    at the four sub-cell centres (+-1/4 cell); a difference toward land or
    outside the domain is 0, so such cells, and land cells, stay constant.
    Every sub-cell inherits its parent's land flag.  The corner depths are
    the bilinear surface evaluated at the refined intersections.
    Returns (list of [2ny][2nx] fields, land [2ny][2nx] or None,
    Hc [2ny+1][2nx+1] or None)."""
    outs = []
    for v in fields:
        v = np.asarray(v, np.float64)
        ny, nx = v.shape
        wet = np.ones((ny, nx), bool) if land is None else (np.asarray(land) == 0)
        r = np.empty((2 * ny, 2 * nx))
        for j in range(ny):
            for i in range(nx):
                sx = sy = 0.0
                if wet[j, i]:
                    dl = v[j, i] - v[j, i - 1] if i > 0 and wet[j, i - 1] else 0.0
                    dr = v[j, i + 1] - v[j, i] if i + 1 < nx and wet[j, i + 1] else 0.0
                    ds = v[j, i] - v[j - 1, i] if j > 0 and wet[j - 1, i] else 0.0
                    dn = v[j + 1, i] - v[j, i] if j + 1 < ny and wet[j + 1, i] else 0.0
                    sx = _minmod3(theta * dl, 0.5 * (dl + dr), theta * dr)
                    sy = _minmod3(theta * ds, 0.5 * (ds + dn), theta * dn)
                for dj in (0, 1):
                    for di in (0, 1):
                        r[2 * j + dj, 2 * i + di] = v[j, i] + (0.5 * di - 0.25) * sx + (0.5 * dj - 0.25) * sy
        outs.append(r)
    land2 = None
    if land is not None:
        land2 = np.repeat(np.repeat(np.asarray(land, np.uint8), 2, axis=0), 2, axis=1)
    Hc2 = None
    if Hc is not None:
        Hc = np.asarray(Hc, np.float64)
        ny1, nx1 = Hc.shape
        Hc2 = np.empty((2 * ny1 - 1, 2 * nx1 - 1))
        for J in range(2 * ny1 - 1):
            for I in range(2 * nx1 - 1):
                j, i = J // 2, I // 2
                wy, wx = 0.5 * (J % 2), 0.5 * (I % 2)
                j1, i1 = min(j + 1, ny1 - 1), min(i + 1, nx1 - 1)
                Hc2[J, I] = ((1 - wy) * ((1 - wx) * Hc[j, i] + wx * Hc[j, i1]) +
                             wy * ((1 - wx) * Hc[j1, i] + wx * Hc[j1, i1]))
    return outs, land2, Hc2


def coarsen2(fields, land=None, Hc=None):
    """Factor-two coarsening (same section): a coarse cell is the average of
    its four children, over the water children only when some of them are
    land; it is land when all four are.  Corner depths are sampled at the
    coarse intersections.  nx and ny must be even.
    Returns (list of [ny/2][nx/2] fields, land or None, Hc or None)."""
    outs = []
    for v in fields:
        v = np.asarray(v, np.float64)
        ny, nx = v.shape
        r = np.empty((ny // 2, nx // 2))
        for j in range(ny // 2):
            for i in range(nx // 2):
                kids = [(2 * j + a, 2 * i + b) for a in (0, 1) for b in (0, 1)]
                if land is not None:
                    water = [k for k in kids if not land[k]]
                    if water:
                        kids = water
                r[j, i] = sum(v[k] for k in kids) / len(kids)
        outs.append(r)
    land2 = None
    if land is not None:
        L = np.asarray(land) != 0
        land2 = (L[0::2, 0::2] & L[0::2, 1::2] & L[1::2, 0::2] & L[1::2, 1::2]).astype(np.uint8)
    Hc2 = None if Hc is None else np.asarray(Hc, np.float64)[::2, ::2].copy()
    return outs, land2, Hc2
