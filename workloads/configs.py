"""Seeded input generators for the five benchmark configurations, the
grid-convergence case and small randomized test domains.

Every generator works in float64 numpy with a fixed seed and rounds to float32
exactly once, so the FP64 oracle (which widens the float32 arrays back to
float64) and the FP32 HIP path start from bit-identical inputs.

Array conventions (shared by both implementations):

* cell fields are ``[ny][nx]`` row-major with x fastest;
* the bathymetry ``Hc`` is the equilibrium depth (metres, positive downwards)
  at cell intersections, ``[ny+1][nx+1]`` (the piecewise bilinear surface of
  the paper's Figure 1b);
* ``land`` is an optional ``uint8`` ``[ny][nx]`` static land mask;
* ``north`` is the angle theta between the grid y-axis and the local north
  vector, so north = (sin theta, cos theta) (section "Coriolis force");
* boundary snapshots are ``[n_times][3][perimeter]`` for (eta, hu, hv) where the
  perimeter is the West strip (ny values, by row), East strip (ny), South strip
  (nx values, by column) and North strip (nx);
* wind snapshots are uniform stresses ``[n_times][2]`` in N/m^2.
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np
from scipy.ndimage import gaussian_filter

G = 9.81
OMEGA = 7.2921e-5  # rad/s, section "Coriolis force"

BC_WALL, BC_PERIODIC, BC_NESTED = 0, 1, 2
FRIC_NONE, FRIC_LINEAR, FRIC_QUADRATIC, FRIC_MANNING = 0, 1, 2, 3


def perimeter_len(nx: int, ny: int) -> int:
    return 2 * ny + 2 * nx


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    Hc: np.ndarray
    f: np.ndarray
    north: np.ndarray
    eta: np.ndarray
    hu: np.ndarray
    hv: np.ndarray
    land: Optional[np.ndarray] = None
    g: float = G
    courant: float = 0.45
    theta: float = 1.3  # generalized-minmod parameter
    kappa: float = 1e-3  # desingularisation / dry tolerance (m)
    bc: tuple = (BC_WALL, BC_WALL, BC_WALL, BC_WALL)  # W, E, S, N
    friction: int = FRIC_NONE
    friction_coeff: float = 0.0
    rho_w: float = 1025.0
    frs_width: int = 10
    frs_d0: float = 2.0
    wind_t: np.ndarray = field(default_factory=lambda: np.zeros(1))
    wind_tau: np.ndarray = field(default_factory=lambda: np.zeros((1, 2), np.float32))
    bnd_t: Optional[np.ndarray] = None
    bnd: Optional[np.ndarray] = None
    # > 0: bnd holds bnd_ny samples along the W/E sides and bnd_nx along S/N
    # (boundary data at its own spacing); 0: one value per boundary cell
    bnd_nx: int = 0
    bnd_ny: int = 0
    # wind at 10 m on its own grid: [n][ny_w][nx_w][2] m/s at times w10_t
    w10_t: Optional[np.ndarray] = None
    w10: Optional[np.ndarray] = None
    rho_a: float = 1.225
    # 0: w10 holds wind at 10 m (m/s); 1: it holds wind stress (N/m^2)
    w10_kind: int = 0
    # > 0: dt from the CFL condition only once every dt_interval seconds
    # (the real-world runs' policy); 0: every step
    dt_interval: float = 0.0
    steps: int = 1
    dt_fixed: Optional[float] = None
    t_end: Optional[float] = None

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def copy(self, **kw) -> "Workload":
        return replace(self, **kw)


# ---------------------------------------------------------------------------
# helpers (input construction only)
# ---------------------------------------------------------------------------

def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _smooth_noise(rng, shape, sigma, mode="reflect"):
    z = gaussian_filter(rng.standard_normal(shape), sigma=sigma, mode=mode)
    return (z - z.mean()) / z.std()


def _minmod2(a, b):
    return np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def _corner_estimates(Hm, wet):
    """Piecewise-planar corner estimates averaged over the wet cells that meet
    at each intersection (initial guess of the section "Bathymetry").
    Returns (corner values, number of wet contributors)."""
    ny, nx = Hm.shape
    Hw = np.where(wet, Hm, 0.0)
    # one-sided differences; a difference toward a dry/land or missing cell is 0
    dxm = np.zeros_like(Hm)
    dxp = np.zeros_like(Hm)
    ok = wet[:, 1:] & wet[:, :-1]
    d = np.where(ok, Hw[:, 1:] - Hw[:, :-1], 0.0)
    dxm[:, 1:] = d
    dxp[:, :-1] = d
    dym = np.zeros_like(Hm)
    dyp = np.zeros_like(Hm)
    ok = wet[1:, :] & wet[:-1, :]
    d = np.where(ok, Hw[1:, :] - Hw[:-1, :], 0.0)
    dym[1:, :] = d
    dyp[:-1, :] = d
    sx = _minmod2(dxm, dxp)
    sy = _minmod2(dym, dyp)
    acc = np.zeros((ny + 1, nx + 1))
    cnt = np.zeros((ny + 1, nx + 1))
    w = wet.astype(np.float64)
    for oy, ox, ssx, ssy in ((0, 0, -1, -1), (0, 1, 1, -1), (1, 0, -1, 1), (1, 1, 1, 1)):
        val = Hw + 0.5 * ssx * sx + 0.5 * ssy * sy
        acc[oy:oy + ny, ox:ox + nx] += val * w
        cnt[oy:oy + ny, ox:ox + nx] += w
    est = np.where(cnt > 0, acc / np.maximum(cnt, 1.0), 0.0)
    return est, cnt


def _smooth_corners(Hc):
    p = np.pad(Hc, 1, mode="edge")
    return 0.5 * Hc + 0.125 * (p[:-2, 1:-1] + p[2:, 1:-1] + p[1:-1, :-2] + p[1:-1, 2:])


def reconstruct_corners(Hm, wet, iters=10, land_value=None):
    """Bilinear bathymetry at intersections from cell values (the iterative
    procedure of the section "Bathymetry": planar slopes -> corner averages,
    then repeated midpoint correction and smoothing).  Corners that touch no
    wet cell take the mean of the (land) cell values around them."""
    ny, nx = Hm.shape
    Hs, cnt = _corner_estimates(Hm, wet)
    if land_value is None:
        # mean of all surrounding cell values for corners with no wet neighbour
        p = np.pad(Hm, 1, mode="edge")
        fill = 0.25 * (p[:-1, :-1] + p[:-1, 1:] + p[1:, :-1] + p[1:, 1:])
    else:
        fill = np.full((ny + 1, nx + 1), float(land_value))
    Hs = np.where(cnt > 0, Hs, fill)
    for _ in range(iters):
        mid = 0.25 * (Hs[:-1, :-1] + Hs[:-1, 1:] + Hs[1:, :-1] + Hs[1:, 1:])
        dH = np.where(wet, Hm - mid, 0.0)
        dHc, c2 = _corner_estimates(dH, wet)
        Hs = Hs + np.where(c2 > 0, dHc, 0.0)
        Hs = np.where(cnt > 0, _smooth_corners(Hs), fill)
    return Hs, cnt


def _cell_centres(nx, ny, dx, dy):
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    return np.meshgrid(x, y)


def _pole_fields(nx, ny, dx, dy, pole, lat_of_dist):
    """Latitude and north angle from a pole position (metres, grid frame)."""
    X, Y = _cell_centres(nx, ny, dx, dy)
    px, py = pole
    d = np.hypot(px - X, py - Y)
    lat = lat_of_dist(d)
    north = np.arctan2(px - X, py - Y)
    f = 2.0 * OMEGA * np.sin(np.deg2rad(lat))
    return f, north, lat


def _gauss_bump(nx, ny, amp, sigma_cells):
    """Gaussian bump centred in the domain; r in cells from the centre."""
    i = np.arange(nx) + 0.5 - nx / 2.0
    j = np.arange(ny) + 0.5 - ny / 2.0
    I, J = np.meshgrid(i, j)
    return amp * np.exp(-(I * I + J * J) / (2.0 * sigma_cells * sigma_cells))


def _boundary_uniform(nx, ny, times, eta_of_t, hu_of_t=None):
    P = perimeter_len(nx, ny)
    out = np.zeros((len(times), 3, P))
    for k, t in enumerate(times):
        out[k, 0, :] = eta_of_t(t)
        if hu_of_t is not None:
            out[k, 1, :] = hu_of_t(t)
    return out


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

def config1() -> Workload:
    """128x128, 1 km cells, flat 100 m, walls, f = 1.2e-4, 1 m Gaussian bump
    (sigma = 10 cells) at the centre, fluid at rest, C = 0.45, 200 steps."""
    nx = ny = 128
    Hc = np.full((ny + 1, nx + 1), 100.0)
    return Workload(
        name="config1_bump_128x128",
        nx=nx, ny=ny, dx=1000.0, dy=1000.0,
        Hc=_f32(Hc),
        f=_f32(np.full((ny, nx), 1.2e-4)),
        north=_f32(np.zeros((ny, nx))),
        eta=_f32(_gauss_bump(nx, ny, 1.0, 10.0)),
        hu=_f32(np.zeros((ny, nx))), hv=_f32(np.zeros((ny, nx))),
        courant=0.45, steps=200,
    )


def coastal_cells(nx, ny, seed_bathy, seed_land, land_frac=0.35):
    """Cell-centre depths and land mask of the coastal generator, before the
    corners are built: log-normal depths (median 150 m, 5..3000 m) from
    Gaussian-smoothed noise (sigma 8 cells), land where an independent smooth
    field (sigma 16 cells) is below its land_frac quantile, land cells at
    -5 m (above the datum).  Returns (Hm float64 [ny][nx], land bool)."""
    rng = np.random.default_rng(seed_bathy)
    Z = _smooth_noise(rng, (ny, nx), 8.0)
    Hm = np.clip(150.0 * np.exp(1.0 * Z), 5.0, 3000.0)
    rng2 = np.random.default_rng(seed_land)
    L = _smooth_noise(rng2, (ny, nx), 16.0)
    land = L < np.percentile(L, 100.0 * land_frac)
    return np.where(land, -5.0, Hm), land


def _coastal(nx, ny, dx, seed_bathy, seed_land, land_frac=0.35, recon_iters=10):
    Hm, land = coastal_cells(nx, ny, seed_bathy, seed_land, land_frac)
    wet = ~land
    Hc, cnt = reconstruct_corners(Hm, wet, iters=recon_iters, land_value=-5.0)
    # every intersection touching a wet cell stays at least 1 m deep
    Hc = np.where(cnt > 0, np.maximum(Hc, 1.0), Hc)
    return Hc, land


def config2(seed: int = 2, nx: int = 2600, ny: int = 900, hours: float = 1.0) -> Workload:
    """NorKyst-shaped synthetic coastal domain: 2600x900 at 800 m, log-normal
    bathymetry (median 150 m, 5..3000 m) reconstructed at intersections, ~35 %
    land from thresholded smooth noise, latitude 58..71 N along the long axis
    with the matching north angle, linear drag r = 3e-3 m/s, uniform wind
    stress 0.1 N/m^2, all sides nested to a 1 m M2 tide (hourly snapshots)."""
    dx = dy = 800.0
    Hc, land = _coastal(nx, ny, dx, seed, seed + 1)
    Lx, Ly = nx * dx, ny * dy
    D = 19.0 * Lx / 13.0  # pole east of the domain: lat 71 N at the east edge, 58 N at the west
    f, north, _ = _pole_fields(nx, ny, dx, dy, (Lx + D, 0.5 * Ly), lambda d: 90.0 - 19.0 * d / D)
    T = 3600.0 * hours
    times = np.arange(0.0, T + 3600.0 + 1e-9, 3600.0)
    m2 = 44712.0  # 12.42 h
    bnd = _boundary_uniform(nx, ny, times, lambda t: 1.0 * np.sin(2.0 * np.pi * t / m2))
    z = np.zeros((ny, nx))
    return Workload(
        name=f"config2_norkyst_{nx}x{ny}",
        nx=nx, ny=ny, dx=dx, dy=dy,
        Hc=_f32(Hc), land=land.astype(np.uint8), f=_f32(f), north=_f32(north),
        eta=_f32(z), hu=_f32(z), hv=_f32(z),
        courant=0.45, bc=(BC_NESTED,) * 4,
        friction=FRIC_LINEAR, friction_coeff=3e-3,
        wind_t=np.array([0.0]), wind_tau=_f32([[0.1, 0.0]]),
        bnd_t=times, bnd=_f32(bnd),
        steps=0, t_end=T,
    )


def config3(nx: int = 1024, ny: int = 1024, steps: int = 5000) -> Workload:
    """Moving wet-dry front: 50 m cells, 20 m deep flat half, then a 1:50 beach
    from the mid-line (dry from x = L/2 + 1 km) up to the far wall; incoming
    0.5 m, 10 min sine wave nested on the West side, walls elsewhere, Manning
    n = 0.03, dry tolerance 1e-3 m, f = 0."""
    dx = dy = 50.0
    L = nx * dx
    xc = np.arange(nx + 1) * dx
    Hx = np.where(xc <= 0.5 * L, 20.0, 20.0 - (xc - 0.5 * L) / 50.0)
    Hc = np.tile(Hx, (ny + 1, 1))
    Hbar = 0.25 * (Hc[:-1, :-1] + Hc[:-1, 1:] + Hc[1:, :-1] + Hc[1:, 1:])
    eta = np.maximum(0.0, -Hbar)
    times = np.arange(0.0, 2400.0 + 1e-9, 15.0)
    c0 = np.sqrt(G * 20.0)
    amp = lambda t: 0.5 * np.sin(2.0 * np.pi * t / 600.0)  # noqa: E731
    bnd = _boundary_uniform(nx, ny, times, amp, lambda t: c0 * amp(t))
    z = np.zeros((ny, nx))
    return Workload(
        name=f"config3_beach_{nx}x{ny}",
        nx=nx, ny=ny, dx=dx, dy=dy,
        Hc=_f32(Hc), f=_f32(z), north=_f32(z),
        eta=_f32(eta), hu=_f32(z), hv=_f32(z),
        courant=0.45, kappa=1e-3,
        bc=(BC_NESTED, BC_WALL, BC_WALL, BC_WALL),
        friction=FRIC_MANNING, friction_coeff=0.03,
        bnd_t=times, bnd=_f32(bnd),
        steps=steps,
    )


def config4_sizes(seed: int = 4, n: int = 256):
    rng = np.random.default_rng(seed)
    nx = rng.integers(200, 1001, size=n)
    ny = rng.integers(200, 601, size=n)
    return [(int(a), int(b)) for a, b in zip(nx, ny)]


def config4_member(k: int, seed: int = 4, n: int = 256, steps: int = 500) -> Workload:
    """Ensemble member k: coastal generator at 1 km cells, walls, f = 1.2e-4,
    wind stress tau_x ~ N(0.1, 0.03) N/m^2, eta = 1 m Gaussian bump plus
    smooth noise of standard deviation 0.05 m."""
    nx, ny = config4_sizes(seed, n)[k]
    rng = np.random.default_rng([seed, k])
    sb, sl = (int(v) for v in rng.integers(0, 2**31 - 1, size=2))
    Hc, land = _coastal(nx, ny, 1000.0, sb, sl)
    tau = float(rng.normal(0.1, 0.03))
    noise = 0.05 * _smooth_noise(rng, (ny, nx), 5.0)
    eta = np.where(land, 0.0, _gauss_bump(nx, ny, 1.0, 10.0) + noise)
    z = np.zeros((ny, nx))
    return Workload(
        name=f"config4_member{k}_{nx}x{ny}",
        nx=nx, ny=ny, dx=1000.0, dy=1000.0,
        Hc=_f32(Hc), land=land.astype(np.uint8),
        f=_f32(np.full((ny, nx), 1.2e-4)), north=_f32(z),
        eta=_f32(eta), hu=_f32(z), hv=_f32(z),
        courant=0.45,
        wind_t=np.array([0.0]), wind_tau=_f32([[tau, 0.0]]),
        steps=steps,
    )


def config5_requests(seed: int = 5, n: int = 2000, rate: float = 20.0):
    """Poisson arrivals (rate per second), sizes nx~U{100..2000},
    ny~U{100..800}, horizons U[1, 24] simulated hours."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    nx = rng.integers(100, 2001, size=n)
    ny = rng.integers(100, 801, size=n)
    horizon = rng.uniform(1.0, 24.0, size=n) * 3600.0
    return [dict(arrival=float(a), nx=int(x), ny=int(y), horizon=float(h))
            for a, x, y, h in zip(arrivals, nx, ny, horizon)]


def config5_member(nx: int, ny: int, horizon: float) -> Workload:
    """Config-1-style forecast request: 1 km cells, 100 m flat, walls,
    f = 1.2e-4, 1 m Gaussian bump (sigma = 10 cells) at the centre."""
    z = np.zeros((ny, nx))
    return Workload(
        name=f"config5_request_{nx}x{ny}",
        nx=nx, ny=ny, dx=1000.0, dy=1000.0,
        Hc=_f32(np.full((ny + 1, nx + 1), 100.0)),
        f=_f32(np.full((ny, nx), 1.2e-4)), north=_f32(z),
        eta=_f32(_gauss_bump(nx, ny, 1.0, 10.0)), hu=_f32(z), hv=_f32(z),
        courant=0.45, steps=0, t_end=float(horizon),
    )


def _peaks(s, t):
    return (3.0 * (1 - s) ** 2 * np.exp(-s ** 2 - (t + 1) ** 2)
            - 10.0 * (s / 5.0 - s ** 3 - t ** 5) * np.exp(-s ** 2 - t ** 2)
            - 1.0 / 3.0 * np.exp(-(s + 1) ** 2 - t ** 2))


def convergence_case(N: int, L_km: float = 500.0, c_km: float = 300.0,
                     pole_km=(1500.0, 1500.0)) -> Workload:
    """Grid-convergence benchmark (section "Convergence of the numerical
    scheme"): peaks bathymetry 100 + 10 peaks(6x/500-3, 6y/500-3) at the
    intersections, cosine bump of radius 300 km in the centre, latitude and
    north angle from a pole at (1500, 1500) km (which reproduces the printed
    33.7..56.3 degree north angles and 56.0..67.4 degree latitudes), walls,
    fixed dt = 1600/N s, end time 800 s."""
    dx = L_km * 1000.0 / N
    xc = np.arange(N + 1) * dx / 1000.0  # km
    XC, YC = np.meshgrid(xc, xc)
    Hc = 100.0 + 10.0 * _peaks(6.0 * XC / L_km - 3.0, 6.0 * YC / L_km - 3.0)
    X, Y = _cell_centres(N, N, dx / 1000.0, dx / 1000.0)
    r = np.hypot(X - 0.5 * L_km, Y - 0.5 * L_km)
    eta = np.where(r <= c_km, 0.5 * (1.0 + np.cos(np.pi * r / c_km)), 0.0)
    px, py = pole_km
    dmin = np.hypot(px - L_km, py - L_km)
    f, north, _ = _pole_fields(N, N, dx, dx, (px * 1000.0, py * 1000.0),
                               lambda d: 90.0 - 22.6 * d / (dmin * 1000.0))
    z = np.zeros((N, N))
    dt = 1600.0 / N
    return Workload(
        name=f"convergence_{N}",
        nx=N, ny=N, dx=dx, dy=dx,
        Hc=_f32(Hc), f=_f32(f), north=_f32(north),
        eta=_f32(eta), hu=_f32(z), hv=_f32(z),
        courant=0.45, steps=int(round(800.0 / dt)), dt_fixed=dt,
    )


def rossby_case(N: int = 350, theta_deg: float = 0.0, dx: float = 20e3, H: float = 50.0,
                f_ref: float = 8e-5, beta: float = 2e-11, amp: float = 0.5, sigma_cells: float = 15.0,
                steps: int = 300) -> Workload:
    """Planetary Rossby waves on a beta plane (section "Coriolis force", eq.
    betaplane): N x N cells of dx, flat depth H, walls, north vector
    n = (sin theta, cos theta) the same in every cell, f = f_ref + beta n.(x -
    x_ref) with x_ref the domain centre, and a Gaussian bump in geostrophic
    balance with the local f at the centre (f v = g d(eta)/dx, f u =
    -g d(eta)/dy, momenta H u, H v).  f_ref = 8e-5 reads the printed 8e-4 as
    2 omega sin 33 deg."""
    X, Y = _cell_centres(N, N, dx, dx)
    xr = yr = 0.5 * N * dx
    th = np.deg2rad(theta_deg)
    nxv, nyv = np.sin(th), np.cos(th)
    f = f_ref + beta * (nxv * (X - xr) + nyv * (Y - yr))
    s2 = (sigma_cells * dx) ** 2
    rx, ry = X - xr, Y - yr
    eta = amp * np.exp(-(rx * rx + ry * ry) / (2.0 * s2))
    detadx = -rx / s2 * eta
    detady = -ry / s2 * eta
    u = -G * detady / f
    v = G * detadx / f
    return Workload(
        name=f"rossby_{N}_theta{theta_deg:g}",
        nx=N, ny=N, dx=dx, dy=dx,
        Hc=_f32(np.full((N + 1, N + 1), H)), f=_f32(f), north=_f32(np.full((N, N), th)),
        eta=_f32(eta), hu=_f32(H * u), hv=_f32(H * v),
        courant=0.45, steps=steps,
    )


def add_wind_field(wl: Workload, nx_w: int, ny_w: int, times, mean=(8.0, 3.0), amp: float = 7.0,
                   seed: int = 0) -> Workload:
    """The workload with a smooth random wind at 10 m on an nx_w x ny_w grid
    (one snapshot per entry of times), speeds around |mean| +- amp m/s."""
    rng = np.random.default_rng(seed)
    n = len(times)
    w = np.empty((n, ny_w, nx_w, 2))
    for k in range(n):
        for c in range(2):
            z = _smooth_noise(rng, (ny_w, nx_w), 1.0) if min(nx_w, ny_w) > 2 else rng.standard_normal((ny_w, nx_w))
            w[k, :, :, c] = mean[c] + amp * z
    return wl.copy(w10_t=np.asarray(times, np.float64), w10=_f32(w))


def rotate_ccw(wl: Workload) -> Workload:
    """The same problem turned a quarter turn counter-clockwise: the cell at
    (x, y) moves to (Ly - y, x), momenta (hu, hv) -> (-hv, hu), north angles
    minus 90 degrees, sides W, E, S, N -> S, N, E, W.  Input arrays only."""
    def r(a):
        return None if a is None else np.ascontiguousarray(np.asarray(a).T[:, ::-1])
    if wl.bnd is not None:
        raise ValueError("rotate_ccw: nested boundary data is not rotated")
    W, E, S, Nn = wl.bc
    tau = np.asarray(wl.wind_tau)
    return wl.copy(
        name=wl.name + "_rot",
        nx=wl.ny, ny=wl.nx, dx=wl.dy, dy=wl.dx,
        Hc=r(wl.Hc), f=r(wl.f), north=None if wl.north is None else _f32(r(wl.north) - np.pi / 2),
        eta=r(wl.eta), hu=_f32(-r(wl.hv)), hv=r(wl.hu),
        land=r(wl.land), bc=(S, Nn, E, W),
        wind_tau=_f32(np.stack([-tau[:, 1], tau[:, 0]], axis=1)),
    )


def unrotate_ccw(a: np.ndarray) -> np.ndarray:
    """Inverse of the array map of rotate_ccw for a scalar field."""
    return np.ascontiguousarray(np.asarray(a)[:, ::-1].T)


def random_small(nx: int, ny: int, seed: int, bc=(BC_WALL,) * 4, friction=FRIC_NONE,
                 friction_coeff=0.0, land_frac: float = 0.0, wet_dry: bool = False,
                 wind=(0.0, 0.0), north_random: bool = True, depth=(20.0, 400.0),
                 amp: float = 0.3, momentum: float = 1.0, dx: float = 500.0,
                 dy: Optional[float] = None, steps: int = 10) -> Workload:
    """Small randomized domain exercising every term: smooth random bathymetry
    (optionally with a dry shoal or a land mask), random smooth eta/hu/hv,
    spatially varying f and north angle, wind snapshots and, for nested sides,
    time-varying boundary strips."""
    dy = dx if dy is None else dy
    rng = np.random.default_rng(seed)
    lo, hi = depth
    Hc = lo + (hi - lo) * 0.5 * (1.0 + np.tanh(_smooth_noise(rng, (ny + 1, nx + 1), 3.0)))
    if bc[0] == BC_PERIODIC:
        Hc[:, nx] = Hc[:, 0]
    if bc[2] == BC_PERIODIC:
        Hc[ny, :] = Hc[0, :]
    if wet_dry:
        # a shoal rising above the datum in one corner region
        xc = np.linspace(0.0, 1.0, nx + 1)[None, :]
        yc = np.linspace(0.0, 1.0, ny + 1)[:, None]
        Hc = Hc - (lo + 8.0) * np.exp(-((xc - 0.7) ** 2 + (yc - 0.6) ** 2) / 0.03)
    land = None
    if land_frac > 0.0:
        Lf = _smooth_noise(rng, (ny, nx), 2.0)
        land = (Lf < np.percentile(Lf, 100.0 * land_frac)).astype(np.uint8)
    Hbar = 0.25 * (Hc[:-1, :-1] + Hc[:-1, 1:] + Hc[1:, :-1] + Hc[1:, 1:])
    eta = amp * _smooth_noise(rng, (ny, nx), 2.0)
    if wet_dry:
        eta = np.where(Hbar + eta < 0.0, -Hbar, eta)  # dry cells start with h = 0
    hdepth = np.maximum(Hbar + eta, 0.0)
    hu = momentum * _smooth_noise(rng, (ny, nx), 2.0) * np.minimum(hdepth, 1.0)
    hv = momentum * _smooth_noise(rng, (ny, nx), 2.0) * np.minimum(hdepth, 1.0)
    f = 1e-4 * (1.0 + 0.3 * _smooth_noise(rng, (ny, nx), 4.0))
    north = (rng.uniform(-np.pi, np.pi) + 0.3 * _smooth_noise(rng, (ny, nx), 4.0)) if north_random \
        else np.zeros((ny, nx))
    wind_t = np.array([0.0, 600.0])
    wind_tau = np.array([[wind[0], wind[1]], [0.5 * wind[0] - 0.02, 1.5 * wind[1] + 0.03]])
    times = np.array([0.0, 300.0, 900.0])
    P = perimeter_len(nx, ny)
    bnd = np.stack([np.stack([0.2 * _smooth_noise(rng, (P,), 2.0) * (k + 1) / 3.0,
                              0.5 * _smooth_noise(rng, (P,), 2.0),
                              0.5 * _smooth_noise(rng, (P,), 2.0)]) for k in range(len(times))])
    if land is not None:
        eta = np.where(land > 0, 0.0, eta)
    return Workload(
        name=f"random_{nx}x{ny}_s{seed}",
        nx=nx, ny=ny, dx=dx, dy=dy,
        Hc=_f32(Hc), land=land, f=_f32(f), north=_f32(north),
        eta=_f32(eta), hu=_f32(hu), hv=_f32(hv),
        courant=0.45, bc=tuple(bc), friction=friction, friction_coeff=friction_coeff,
        wind_t=wind_t, wind_tau=_f32(wind_tau), bnd_t=times, bnd=_f32(bnd),
        frs_width=min(10, max(1, min(nx, ny) // 4)),
        steps=steps,
    )
