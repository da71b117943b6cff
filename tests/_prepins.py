"""Pins of the preprocessing oracle (sections "Bathymetry" and "Refinement
and coarsening of grid").  Each check takes the oracle module as an argument
so that the mutation test can run the same checks on planted mistakes.
Every check raises AssertionError when its property fails."""

import numpy as np
from scipy.ndimage import binary_erosion, gaussian_filter, grey_dilation

CROSS = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]], bool)


def _rough(seed, ny, nx, sigma=3.0, land_frac=0.0):
    rng = np.random.default_rng(seed)
    z = gaussian_filter(rng.standard_normal((ny, nx)), sigma)
    Hm = np.clip(150.0 * np.exp(z / z.std()), 5.0, 3000.0)
    land = None
    if land_frac > 0.0:
        L = gaussian_filter(rng.standard_normal((ny, nx)), 4.0)
        land = (L < np.quantile(L, land_frac)).astype(np.uint8)
        Hm = np.where(land != 0, -5.0, Hm)
    return Hm, land


def _mid(H):
    return 0.25 * (H[:-1, :-1] + H[:-1, 1:] + H[1:, :-1] + H[1:, 1:])


def recon_constant(P):
    """A constant bottom is reproduced exactly, with and without smoothing."""
    Hm = np.full((9, 11), 37.25)
    for it, w in ((0, 0.5), (6, 0.5), (6, 0.0)):
        H = P.reconstruct_bathymetry(Hm, iters=it, smooth=w)
        assert H.shape == (10, 12)
        assert np.abs(H - 37.25).max() <= 1e-12


def recon_plane(P):
    """Planar cell values (the average of a plane over a cell is its centre
    value): eqs. recon_1-3 give the plane's corner values exactly wherever
    all four cells at a corner have both neighbours in each direction, and
    each round of correction + smoothing leaves a plane unchanged, so the
    error made at the edges moves inward at most two corners a round."""
    ny, nx = 36, 40
    j, i = np.mgrid[0:ny, 0:nx]
    Hm = 50.0 + 1.7 * (i + 0.5) - 0.9 * (j + 0.5)
    J, I = np.mgrid[0:ny + 1, 0:nx + 1]
    exact = 50.0 + 1.7 * I - 0.9 * J
    d = np.minimum.reduce([I, J, nx - I, ny - J])
    for k in (0, 1, 4):
        H = P.reconstruct_bathymetry(Hm, iters=k)
        inner = d >= 2 * k + 2
        assert np.abs(H - exact)[inner].max() <= 1e-11, k
        # the edges do differ (slopes toward the outside count as 0)
        assert np.abs(H - exact)[d == 0].max() > 1e-3


def recon_correction_reduces_misfit(P):
    """Without smoothing each correction round brings the midpoints of the
    bilinear surface closer to the target cell values (the purpose of the
    first stage of the iteration)."""
    for seed, frac in ((0, 0.0), (1, 0.2)):
        Hm, land = _rough(seed, 40, 48, land_frac=frac)
        wet = np.ones(Hm.shape, bool) if land is None else land == 0
        prev = np.inf
        for k in range(0, 7):
            H = P.reconstruct_bathymetry(Hm, land, iters=k, smooth=0.0)
            m = np.sqrt(np.mean((Hm - _mid(H))[wet] ** 2))
            assert m < prev, (seed, k, m, prev)
            prev = m
        m0 = np.sqrt(np.mean((Hm - _mid(P.reconstruct_bathymetry(Hm, land, iters=0)))[wet] ** 2))
        assert prev < 0.5 * m0


def recon_iteration_converges(P):
    """With the default smoothing the update between two rounds shrinks
    geometrically (the stopping rule of the section relies on it)."""
    Hm, land = _rough(2, 40, 48, land_frac=0.2)
    Hs = [P.reconstruct_bathymetry(Hm, land, iters=k) for k in range(0, 11)]
    upd = [np.abs(Hs[k + 1] - Hs[k]).max() for k in range(10)]
    for a, b in zip(upd, upd[1:]):
        assert b < 0.8 * a, upd
    assert upd[-1] < 0.01 * upd[0]


def recon_smoother_modes(P):
    """The smoother keeps planes and, at weight 1/2, removes the corner
    checkerboard (the mode invisible to the midpoint misfit) in one pass."""
    J, I = np.mgrid[0:12, 0:14]
    plane = 3.0 + 0.25 * I - 0.5 * J
    cb = np.where((I + J) % 2 == 0, 1.0, -1.0)
    inner = (I > 0) & (I < 13) & (J > 0) & (J < 11)
    assert np.abs(P._smooth(plane, 0.5) - plane)[inner].max() <= 1e-13
    assert np.abs(P._smooth(plane + cb, 0.5) - plane)[inner].max() <= 1e-13
    assert np.abs(P._smooth(plane + cb, 0.0) - plane - cb).max() <= 1e-13


def recon_land(P):
    """Corners touching only land cells hold the mean of the four cell values
    around them; a lone water cell in land gives its own value at its four
    corners in the initial guess (no water neighbour, so zero slopes)."""
    ny, nx = 7, 8
    rng = np.random.default_rng(5)
    Hm = -rng.uniform(1.0, 9.0, (ny, nx))
    land = np.ones((ny, nx), np.uint8)
    land[3, 4] = 0
    Hm[3, 4] = 42.0
    H = P.reconstruct_bathymetry(Hm, land, iters=0)
    pad = np.pad(Hm, 1, mode="edge")
    fill = 0.25 * (pad[:-1, :-1] + pad[:-1, 1:] + pad[1:, :-1] + pad[1:, 1:])
    own = np.zeros((ny + 1, nx + 1), bool)
    own[3:5, 4:6] = True
    assert np.all(H[own] == 42.0)
    assert np.abs(H[~own] - fill[~own]).max() <= 1e-14
    H10 = P.reconstruct_bathymetry(Hm, land, iters=10)
    assert np.abs(H10[~own] - fill[~own]).max() <= 1e-14


def recon_symmetry(P):
    """Mirror in x, mirror in y and transposition commute with the whole
    reconstruction (land included)."""
    Hm, land = _rough(3, 17, 21, land_frac=0.25)
    H = P.reconstruct_bathymetry(Hm, land, iters=5)
    for f in (lambda a: a[:, ::-1], lambda a: a[::-1, :], lambda a: a.T):
        Hf = P.reconstruct_bathymetry(f(Hm), f(land), iters=5)
        assert np.abs(Hf - f(H)).max() <= 1e-10 * np.abs(H).max()


def recon_affine(P):
    """reconstruct(a Hm + b) = a reconstruct(Hm) + b for a > 0 (only
    differences are limited; the fill is a mean)."""
    Hm, land = _rough(4, 15, 19, land_frac=0.2)
    H = P.reconstruct_bathymetry(Hm, land, iters=4)
    H2 = P.reconstruct_bathymetry(2.5 * Hm - 7.0, land, iters=4)
    assert np.abs(H2 - (2.5 * H - 7.0)).max() <= 1e-10 * np.abs(H2).max()


def recon_locality(P):
    """A change of one cell value reaches only corners within 3 k + 2 cells
    after k rounds (each round reads corners up to three away), so a window
    with that margin reproduces the full grid."""
    Hm, land = _rough(6, 44, 44)
    k = 5
    H = P.reconstruct_bathymetry(Hm, land, iters=k)
    Hm2 = Hm.copy()
    Hm2[22, 21] += 40.0
    H2 = P.reconstruct_bathymetry(Hm2, land, iters=k)
    J, I = np.mgrid[0:45, 0:45]
    far = np.maximum(np.maximum(I - 22, 21 - I), np.maximum(J - 23, 22 - J)) > 3 * k + 2
    assert np.all(H2[far] == H[far])
    assert np.abs(H2 - H).max() > 1.0


def erosion_textbook(P):
    """One round equals binary erosion of the land mask with the 4-connected
    structuring element (outside = land) and gray dilation of eta over the
    water cells; eroded cells get the land depth and zero momenta."""
    rng = np.random.default_rng(7)
    land = (gaussian_filter(rng.standard_normal((23, 31)), 2.0) < 0.1).astype(np.uint8)
    Hm = np.where(land != 0, -3.0, rng.uniform(5.0, 90.0, land.shape))
    eta, hu, hv = (rng.standard_normal(land.shape) for _ in range(3))
    L2, H2, e2, u2, v2 = P.erode_land(land, Hm, eta, hu, hv, land_depth=5.0)
    want = binary_erosion(land != 0, structure=CROSS, border_value=1)
    assert np.array_equal(L2 != 0, want)
    eroded = (land != 0) & ~want
    assert eroded.sum() > 20
    dil = grey_dilation(np.where(land != 0, -np.inf, eta), footprint=CROSS, mode="constant", cval=-np.inf)
    assert np.array_equal(e2[eroded], dil[eroded])
    assert np.all(H2[eroded] == 5.0) and np.all(u2[eroded] == 0.0) and np.all(v2[eroded] == 0.0)
    keep = ~eroded
    for a, b in ((H2, Hm), (e2, eta), (u2, hu), (v2, hv)):
        assert np.array_equal(a[keep], b[keep])


def erosion_strait(P):
    """A one-cell strait through a land bar is three cells wide after one
    round and five after two."""
    land = np.zeros((15, 20), np.uint8)
    land[:, 8:13] = 1
    land[7, :] = 0
    Hm = np.where(land != 0, -5.0, 30.0)
    z = np.zeros(land.shape)
    a = P.erode_land(land, Hm, z, z, z)
    assert np.array_equal(np.flatnonzero(a[0][:, 10] == 0), [6, 7, 8])
    b = P.erode_land(*a)
    assert np.array_equal(np.flatnonzero(b[0][:, 10] == 0), [5, 6, 7, 8, 9])


def _linear(ny, nx, a=2.0, b=0.7, c=-1.3):
    j, i = np.mgrid[0:ny, 0:nx]
    return a + b * (i + 0.5) + c * (j + 0.5)


def refine_conserves_and_inverts(P):
    """The four children average to the parent (each field, land or not),
    coarsening undoes refinement for cells, land and corners, and the
    children stay within the range of the parent and its neighbours."""
    rng = np.random.default_rng(8)
    ny, nx = 13, 17
    v = rng.standard_normal((ny, nx))
    land = (rng.uniform(size=(ny, nx)) < 0.2).astype(np.uint8)
    Hc = rng.uniform(1.0, 50.0, (ny + 1, nx + 1))
    for th in (1.0, 1.3, 2.0):
        (r,), L2, H2 = P.refine2([v], land, Hc, theta=th)
        kids = 0.25 * (r[0::2, 0::2] + r[0::2, 1::2] + r[1::2, 0::2] + r[1::2, 1::2])
        assert np.abs(kids - v).max() <= 1e-14
        (c,), L3, H3 = P.coarsen2([r], L2, H2)
        assert np.abs(c - v).max() <= 1e-14
        assert np.array_equal(L3, land) and np.array_equal(H3, Hc)
        pad = np.pad(v, 1, mode="edge")
        lo = np.minimum.reduce([pad[1:-1, 1:-1], pad[:-2, 1:-1], pad[2:, 1:-1], pad[1:-1, :-2], pad[1:-1, 2:]])
        hi = np.maximum.reduce([pad[1:-1, 1:-1], pad[:-2, 1:-1], pad[2:, 1:-1], pad[1:-1, :-2], pad[1:-1, 2:]])
        for a in (0, 1):
            for b in (0, 1):
                assert np.all(r[a::2, b::2] >= lo - 1e-14) and np.all(r[a::2, b::2] <= hi + 1e-14)


def refine_linear_exact(P):
    """A linear field is refined exactly (children = the field at the
    sub-cell centres) away from the edges, for any theta in [1, 2]; cells at
    the edge and next to land keep a constant value (first order)."""
    ny, nx = 9, 12
    v = _linear(ny, nx)
    vf = _linear(2 * ny, 2 * nx, 2.0, 0.35, -0.65)
    for th in (1.0, 1.3, 2.0):
        (r,), _, _ = P.refine2([v], None, None, theta=th)
        assert np.abs(r - vf)[2:-2, 2:-2].max() <= 1e-13
        assert np.abs(r[0::2, 0] - r[0::2, 1]).max() == 0.0
    land = np.zeros((ny, nx), np.uint8)
    land[4, 6] = 1
    (r,), L2, _ = P.refine2([v], land, None)
    for (j, i) in ((4, 5), (4, 6), (4, 7)):
        blk = r[2 * j:2 * j + 2, 2 * i:2 * i + 2]
        assert np.abs(blk[:, 0] - blk[:, 1]).max() == 0.0
    assert L2[8:10, 12:14].all() and L2.sum() == 4


def refine_bilinear_corners(P):
    """The refined corners are the bilinear surface: a global bilinear
    function is reproduced exactly, and the mean depth of the four children
    (each the mean of its corners) equals the parent's."""
    J, I = np.mgrid[0:8, 0:11]
    f = lambda x, y: 4.0 + 0.5 * x - 0.25 * y + 0.125 * x * y
    _, _, R = P.refine2([], None, f(I, J).astype(np.float64))
    J2, I2 = np.mgrid[0:15, 0:21]
    assert np.abs(R - f(I2 / 2.0, J2 / 2.0)).max() <= 1e-12
    rng = np.random.default_rng(9)
    Hc = rng.uniform(1.0, 50.0, (8, 11))
    _, _, R = P.refine2([], None, Hc)
    m = _mid(R)
    kids = 0.25 * (m[0::2, 0::2] + m[0::2, 1::2] + m[1::2, 0::2] + m[1::2, 1::2])
    assert np.abs(kids - _mid(Hc)).max() <= 1e-13


def coarsen_land(P):
    """A coarse cell averages its water children only; it is land when all
    four children are, and then holds their plain average."""
    v = np.arange(16.0).reshape(4, 4)
    land = np.zeros((4, 4), np.uint8)
    land[0, 0] = 1
    land[2:4, 2:4] = 1
    v[0, 0] = 1e6
    (c,), L, _ = P.coarsen2([v], land, None)
    assert c[0, 0] == (1.0 + 4.0 + 5.0) / 3.0
    assert c[1, 1] == (10.0 + 11.0 + 14.0 + 15.0) / 4.0
    assert np.array_equal(L, [[0, 0], [0, 1]])
    assert c[0, 1] == (2.0 + 3.0 + 6.0 + 7.0) / 4.0


ALL = [recon_constant, recon_plane, recon_correction_reduces_misfit, recon_iteration_converges,
       recon_smoother_modes, recon_land, recon_symmetry, recon_affine, recon_locality,
       erosion_textbook, erosion_strait, refine_conserves_and_inverts, refine_linear_exact,
       refine_bilinear_corners, coarsen_land]
