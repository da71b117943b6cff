"""GPU parity of the device preprocessing (sections "Bathymetry" and
"Refinement and coarsening of grid") against the FP64 oracle in
oracle/preprocess.py, through the C ABI.

Tolerances.  Land masks, erosion (copies and maxima of float32 values) and
sampled corners are bit-exact.  The bathymetry rounds hold values of size up
to M = max|Hm| in float32 through about 8 roundings each (corner update,
neighbour sum, smoothing), about 16 u M per round with u = 2^-24; the
update shrinks from round to round, so after 11 rounds the error stays below
176 u M ~ 1.05e-5 M: the bar is 2e-5 M.  Refinement and coarsening take 2-4
float32 roundings of values of size max|v|: the bar is 1e-6 max|v|."""

import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import preprocess as P  # noqa: E402
from workloads import coastal_cells  # noqa: E402

pytestmark = pytest.mark.gpu

RECON_TOL = 2e-5
FIELD_TOL = 1e-6


@pytest.fixture(scope="module")
def swe():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_02457_amd import swe as S
    S.load_library()
    return S


def _cuda(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _coastal(nx, ny, seed):
    Hm, land = coastal_cells(nx, ny, seed, seed + 1)
    return Hm.astype(np.float32), land.astype(np.uint8)


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("nx,ny,land_on,iters,smooth", [
    (150, 40, True, 10, 0.5),     # 3 x 3 tiles with ragged edges, land
    (150, 40, False, 10, 0.5),
    (150, 40, True, 7, 0.0),      # odd round count, no smoothing
    (70, 33, True, 0, 0.5),       # initial guess only
    (129, 17, True, 1, 0.5),
    (1, 1, False, 3, 0.5),        # one cell
    (5, 3, True, 4, 0.5),         # tiny, part land
])
def test_reconstruct_matches_oracle(swe, nx, ny, land_on, iters, smooth):
    _say(f"reconstruct nx={nx} ny={ny} land={land_on} iters={iters} smooth={smooth}")
    if nx >= 8:
        Hm, land = _coastal(nx, ny, 11)
    else:
        rng = np.random.default_rng(3)
        Hm = rng.uniform(5.0, 80.0, (ny, nx)).astype(np.float32)
        land = (rng.uniform(size=(ny, nx)) < 0.3).astype(np.uint8)
        Hm = np.where(land != 0, np.float32(-5.0), Hm)
    if not land_on:
        land = None
    ref = P.reconstruct_bathymetry(Hm, land, iters=iters, smooth=smooth)
    out = swe.reconstruct_bathymetry(_cuda(Hm), None if land is None else _cuda(land), iters=iters,
                                     smooth=smooth)
    got = _host(out).astype(np.float64)
    M = np.abs(Hm).max()
    err = np.abs(got - ref).max() / M
    _say(f"  max |gpu - oracle| / max|Hm| = {err:.3e}")
    assert got.shape == ref.shape
    assert err <= RECON_TOL
    if land is not None:
        # corners touching no water cell: the fill, within one float32 rounding
        pad = np.pad(land, 1, mode="edge") != 0
        dry = pad[:-1, :-1] & pad[:-1, 1:] & pad[1:, :-1] & pad[1:, 1:]
        assert np.abs(got - ref)[dry].max(initial=0.0) <= 2.0 ** -23 * M


def test_reconstruct_all_land(swe):
    rng = np.random.default_rng(4)
    Hm = -rng.uniform(1.0, 9.0, (20, 70)).astype(np.float32)
    land = np.ones(Hm.shape, np.uint8)
    ref = P.reconstruct_bathymetry(Hm, land, iters=3)
    got = _host(swe.reconstruct_bathymetry(_cuda(Hm), _cuda(land), iters=3)).astype(np.float64)
    assert np.abs(got - ref).max() <= 2.0 ** -23 * np.abs(Hm).max()


def test_reconstruct_full_size_sampled(swe):
    """A 2600 x 900 coastal field (the NorKyst-800 grid shape), 10 rounds, on
    the device; the oracle recomputes windows around sample points with a
    margin of 3 k + 3 cells (a cell influences corners at most 3 k + 2 away
    after k rounds), which reproduces those corners of the full grid."""
    nx, ny, k = 2600, 900, 10
    Hm, land = _coastal(nx, ny, 2)
    _say("reconstruct 2600x900 full size")
    got = _host(swe.reconstruct_bathymetry(_cuda(Hm), _cuda(land), iters=k)).astype(np.float64)
    margin, half = 3 * k + 3, 12
    M = np.abs(Hm).max()
    worst = 0.0
    for (j, i) in [(0, 0), (ny - 1, nx - 1), (0, nx // 2), (ny // 2, 0), (450, 1300), (300, 2000), (777, 555),
                   (ny - 1, 17)]:
        j0, j1 = max(0, j - half - margin), min(ny, j + half + margin)
        i0, i1 = max(0, i - half - margin), min(nx, i + half + margin)
        ref = P.reconstruct_bathymetry(Hm[j0:j1, i0:i1], land[j0:j1, i0:i1], iters=k)
        # corners of the window that no artificial window edge can reach
        a0 = 0 if j0 == 0 else margin
        b0 = 0 if i0 == 0 else margin
        a1 = ref.shape[0] if j1 == ny else ref.shape[0] - margin
        b1 = ref.shape[1] if i1 == nx else ref.shape[1] - margin
        assert a1 - a0 > half and b1 - b0 > half
        g = got[j0 + a0:j0 + a1, i0 + b0:i0 + b1]
        worst = max(worst, np.abs(g - ref[a0:a1, b0:b1]).max() / M)
    _say(f"  sampled max |gpu - oracle| / max|Hm| = {worst:.3e}")
    assert worst <= RECON_TOL


def test_reconstruct_output_buffers(swe):
    """Even and odd round counts end in the caller's output buffer; the
    scratch buffer is only workspace."""
    import torch
    Hm, land = _coastal(90, 30, 5)
    for k in (1, 2, 5):
        out = torch.full((31, 91), -1.0, device="cuda")
        scratch = torch.full((31, 91), -2.0, device="cuda")
        swe.reconstruct_bathymetry(_cuda(Hm), _cuda(land), iters=k, out=out, scratch=scratch)
        ref = P.reconstruct_bathymetry(Hm, land, iters=k)
        assert np.abs(_host(out) - ref).max() <= RECON_TOL * np.abs(Hm).max()


@pytest.mark.parametrize("nx,ny", [(300, 70), (1, 1), (2600, 900)])
def test_erode_bitexact(swe, nx, ny):
    _say(f"erode nx={nx} ny={ny}")
    rng = np.random.default_rng(nx + ny)
    if nx > 2:
        Hm, land = _coastal(nx, ny, 7)
    else:
        Hm = np.full((ny, nx), -5.0, np.float32)
        land = np.ones((ny, nx), np.uint8)
    eta, hu, hv = (rng.standard_normal((ny, nx)).astype(np.float32) for _ in range(3))
    ref = P.erode_land(land, Hm, eta, hu, hv, land_depth=5.0)
    got = swe.erode_land(_cuda(land), _cuda(Hm), _cuda(eta), _cuda(hu), _cuda(hv), land_depth=5.0)
    for r, g in zip(ref, got):
        g = _host(g)
        assert np.array_equal(g.astype(np.float64), np.asarray(r, np.float64))
    # without the optional state fields
    L2, H2, e2, u2, v2 = swe.erode_land(_cuda(land), _cuda(Hm))
    assert e2 is None and u2 is None and v2 is None
    assert np.array_equal(_host(L2), ref[0]) and np.array_equal(_host(H2).astype(np.float64), ref[1])


def test_erode_twice_matches_oracle(swe):
    Hm, land = _coastal(200, 60, 9)
    z = np.zeros(Hm.shape, np.float32)
    r1 = P.erode_land(land, Hm, z, z, z)
    r2 = P.erode_land(*r1)
    g = swe.erode_land(_cuda(land), _cuda(Hm), _cuda(z), _cuda(z), _cuda(z))
    g = swe.erode_land(*g)
    assert np.array_equal(_host(g[0]), r2[0])
    assert np.array_equal(_host(g[1]).astype(np.float64), r2[1])


def _fields(nf, ny, nx, seed):
    rng = np.random.default_rng(seed)
    from scipy.ndimage import gaussian_filter
    return np.stack([gaussian_filter(rng.standard_normal((ny, nx)), 2.0) * (k + 1) for k in range(nf)]
                    ).astype(np.float32)


@pytest.mark.parametrize("nx,ny,theta,land_on", [(300, 70, 1.0, True), (300, 70, 1.3, False), (1, 1, 1.0, True),
                                                 (37, 23, 2.0, True)])
def test_refine_matches_oracle(swe, nx, ny, theta, land_on):
    _say(f"refine nx={nx} ny={ny} theta={theta} land={land_on}")
    F = _fields(3, ny, nx, 21)
    rng = np.random.default_rng(22)
    land = (rng.uniform(size=(ny, nx)) < 0.15).astype(np.uint8) if land_on else None
    Hc = rng.uniform(1.0, 200.0, (ny + 1, nx + 1)).astype(np.float32)
    ref_f, ref_l, ref_h = P.refine2(list(F), land, Hc, theta=theta)
    fo, lo, ho = swe.refine2(_cuda(F), None if land is None else _cuda(land), _cuda(Hc), theta=theta)
    fo = _host(fo).astype(np.float64)
    for k in range(3):
        assert np.abs(fo[k] - ref_f[k]).max() <= FIELD_TOL * np.abs(F[k]).max()
    if land_on:
        assert np.array_equal(_host(lo), ref_l)
    else:
        assert lo is None
    assert np.abs(_host(ho) - ref_h).max() <= FIELD_TOL * np.abs(Hc).max()


@pytest.mark.parametrize("nx,ny,land_on", [(300, 70, True), (2, 2, True), (64, 46, False)])
def test_coarsen_matches_oracle(swe, nx, ny, land_on):
    _say(f"coarsen nx={nx} ny={ny} land={land_on}")
    F = _fields(2, ny, nx, 31)
    rng = np.random.default_rng(32)
    land = (rng.uniform(size=(ny, nx)) < 0.4).astype(np.uint8) if land_on else None
    Hc = rng.uniform(1.0, 200.0, (ny + 1, nx + 1)).astype(np.float32)
    ref_f, ref_l, ref_h = P.coarsen2(list(F), land, Hc)
    fo, lo, ho = swe.coarsen2(_cuda(F), None if land is None else _cuda(land), _cuda(Hc))
    fo = _host(fo).astype(np.float64)
    for k in range(2):
        assert np.abs(fo[k] - ref_f[k]).max() <= FIELD_TOL * np.abs(F[k]).max()
    if land_on:
        assert np.array_equal(_host(lo), ref_l)
    assert np.array_equal(_host(ho).astype(np.float64), ref_h)


def test_refine_coarsen_full_size(swe):
    """NorKyst-shaped 2600 x 900 fields: refinement checked against the oracle
    on bands of rows (it reads one row either side), coarsening of the result
    gives the input back, and corners round-trip exactly."""
    nx, ny = 2600, 900
    _say("refine/coarsen 2600x900 full size")
    F = _fields(3, ny, nx, 41)
    Hm, land = _coastal(nx, ny, 2)
    Hc = np.abs(np.random.default_rng(42).standard_normal((ny + 1, nx + 1))).astype(np.float32) * 100.0
    fo, lo, ho = swe.refine2(_cuda(F), _cuda(land), _cuda(Hc), theta=1.3)
    fh = _host(fo)
    for a, b in ((0, 6), (447, 453), (894, 900)):
        a0, b0 = max(0, a - 1), min(ny, b + 1)
        rf, rl, _ = P.refine2([F[k][a0:b0] for k in range(3)], land[a0:b0], None, theta=1.3)
        for k in range(3):
            g = fh[k][2 * a:2 * b]
            r = rf[k][2 * (a - a0):2 * (b - a0)]
            assert np.abs(g - r).max() <= FIELD_TOL * np.abs(F[k]).max()
    c_f, c_l, c_h = swe.coarsen2(fo, lo, ho)
    assert np.abs(_host(c_f) - F).max() <= FIELD_TOL * np.abs(F).max()
    assert np.array_equal(_host(c_l), land)
    assert np.array_equal(_host(c_h), Hc)


def test_preprocessed_domain_steps(swe):
    """The chain the paper applies to model data -- erode once, reconstruct
    the corners, refine by two -- feeds a domain that then steps: walls and
    land keep the mass to float32 accuracy."""
    import torch
    from paper_1912_02457_amd import Domain, make_params
    nx, ny = 160, 96
    Hm, land = _coastal(nx, ny, 13)
    z = np.zeros((ny, nx), np.float32)
    eta = z.copy()
    j, i = np.mgrid[0:ny, 0:nx]
    eta += 0.3 * np.exp(-((i - 80.0) ** 2 + (j - 48.0) ** 2) / 50.0).astype(np.float32)
    L, H, e, u, v = swe.erode_land(_cuda(land), _cuda(Hm), _cuda(eta), _cuda(z), _cuda(z))
    Hc = swe.reconstruct_bathymetry(H, L, iters=10)
    fo, L2, Hc2 = swe.refine2(torch.stack([e, u, v]), L, Hc)
    Hc2 = torch.clamp(Hc2, min=-5.0)
    p = make_params(2 * nx, 2 * ny, 400.0, 400.0)
    f = np.full((2 * ny, 2 * nx), 1.2e-4, np.float32)
    fh = _host(fo)
    dom = Domain(p, _host(Hc2), f, fh[0], fh[1], fh[2], land=_host(L2))
    m0, _ = dom.diagnostics()
    dom.step(50)
    m1, _ = dom.diagnostics()
    eta1, hu1, hv1, t, dt = dom.read_state()
    assert np.isfinite(eta1).all() and t > 0
    assert abs(m1 - m0) <= 1e-6 * abs(m0)
