"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded float32 inputs, element by element, to 1e-4 relative L2 and
5e-4 relative Linf per field (eta by its own norm, hu and hv by the momentum
magnitude), plus self-consistency checks of the GPU path."""

import sys
import zlib

import numpy as np
import pytest

from oracle import oracle as O
from tests._parity import assert_parity, parity
from workloads import (BC_NESTED, BC_PERIODIC, BC_WALL, FRIC_LINEAR, FRIC_MANNING, FRIC_NONE, add_wind_field,
                       FRIC_QUADRATIC, config1, config2, config3, random_small, rossby_case, rotate_ccw,
                       unrotate_ccw)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    from paper_1912_02457_amd import load_library
    load_library()
    return torch


def _dom(wl, comp=False, **kw):
    """A domain with the float32 state of the paper unless comp is set (the
    compensated state has tests of its own in test_gpu_compensated.py)."""
    from paper_1912_02457_amd import Domain
    return Domain.from_workload(wl, device="cuda:0", compensated_state=comp, **kw)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_both(wl, nsteps, proj=False, comp=False):
    """Oracle with its own CFL dt; GPU once replaying the oracle's dt sequence
    and once with its own on-device dt."""
    ref, t_ref, dts, k = O.Oracle(wl).run(nsteps=nsteps)
    assert k == nsteps
    d = _dom(wl, comp=comp, north_projection=proj)
    d.step_dt(dts)
    rep = d.read_state()
    d.close()
    d = _dom(wl, comp=comp, north_projection=proj)
    d.step(nsteps)
    own = d.read_state()
    d.close()
    return ref, t_ref, rep, own


def test_config1_plain_method():
    """128x128 bump, walls, constant f, 200 steps (the plain-method case)."""
    wl = config1()
    _say("config1 200 steps")
    ref, t_ref, rep, own = run_both(wl, 200)
    p1 = assert_parity(rep, ref, label="config1 dt-replay")
    p2 = assert_parity(own, ref, label="config1 own-dt")
    assert abs(own[3] - t_ref) <= 1e-5 * t_ref
    _say("config1", p1, p2)


CASES = [
    # name, nx, ny, kwargs
    ("walls_land", 133, 71, dict(land_frac=0.2, friction=FRIC_LINEAR, friction_coeff=3e-3, wind=(0.1, 0.05))),
    ("periodic", 64, 48, dict(bc=(BC_PERIODIC,) * 4, friction=FRIC_QUADRATIC, friction_coeff=2e-3)),
    ("nested_all", 97, 83, dict(bc=(BC_NESTED,) * 4, land_frac=0.1, wind=(-0.05, 0.1))),
    ("nested_mixed", 61, 130, dict(bc=(BC_NESTED, BC_WALL, BC_PERIODIC, BC_PERIODIC))),
    ("wet_dry_manning", 120, 90, dict(wet_dry=True, friction=FRIC_MANNING, friction_coeff=0.03, amp=0.5)),
    ("ragged_small", 5, 3, dict()),
    ("tiny_2x2", 2, 2, dict(bc=(BC_NESTED, BC_WALL, BC_NESTED, BC_WALL))),
    ("one_strip_edge", 60, 17, dict(land_frac=0.3)),
    ("strip_plus_one", 61, 16, dict(bc=(BC_WALL, BC_NESTED, BC_WALL, BC_WALL))),
    ("tall", 7, 301, dict(bc=(BC_PERIODIC, BC_PERIODIC, BC_NESTED, BC_NESTED), friction=FRIC_LINEAR,
                          friction_coeff=1e-3)),
    ("anisotropic", 150, 40, dict(dx=300.0, dy=900.0, land_frac=0.15, wind=(0.2, -0.1))),
    # mostly land: a few lakes and channels, many rows and tiles without water
    ("mostly_land", 90, 70, dict(land_frac=0.85, bc=(BC_NESTED, BC_WALL, BC_WALL, BC_NESTED), wind=(0.1, -0.05))),
    # a dry shoal and a land mask together (wet-dry fix next to land faces)
    ("wet_dry_land", 110, 80, dict(wet_dry=True, land_frac=0.3, friction=FRIC_QUADRATIC, friction_coeff=2e-3,
                                   amp=0.5)),
]


@pytest.mark.parametrize("comp", [False, True], ids=["f32state", "compensated"])
@pytest.mark.parametrize("name,nx,ny,kw", CASES, ids=[c[0] for c in CASES])
def test_random_cases(name, nx, ny, kw, comp):
    wl = random_small(nx, ny, seed=zlib.crc32(name.encode()) % 1000, steps=30, **kw)
    _say("case", name, nx, ny, "compensated" if comp else "float32 state")
    ref, t_ref, rep, own = run_both(wl, 30, comp=comp)
    assert_parity(rep, ref, wl.land, label=f"{name} dt-replay")
    assert_parity(own, ref, wl.land, label=f"{name} own-dt")
    if wl.land is not None:
        lm = wl.land > 0
        assert np.array_equal(own[0][lm], wl.eta[lm]) and np.array_equal(own[1][lm], wl.hu[lm])


def test_north_projection_variant():
    """The literal north-vector projection kernel agrees with the oracle (which
    always evaluates the projection) for random north angles."""
    wl = random_small(90, 70, seed=17, north_random=True, land_frac=0.1, steps=30,
                      bc=(BC_NESTED, BC_WALL, BC_WALL, BC_NESTED))
    _say("north projection")
    ref, t_ref, rep, own = run_both(wl, 30, proj=True)
    assert_parity(rep, ref, wl.land, label="proj dt-replay")
    assert_parity(own, ref, wl.land, label="proj own-dt")


@pytest.mark.parametrize("case", ["walls", "nested_land"])
def test_gridded_wind_matches_oracle(case):
    """Wind at 10 m on a coarse grid of its own (bilinear in space, linear in
    time between snapshots, Large and Pond stress with speeds on both sides of
    the 11 m/s break), 60 steps against the oracle."""
    if case == "walls":
        wl = random_small(97, 83, seed=31, friction=FRIC_LINEAR, friction_coeff=2e-3)
        wl = add_wind_field(wl, 7, 5, [0.0, 60.0], seed=3)
    else:
        wl = random_small(120, 70, seed=32, bc=(BC_NESTED, BC_WALL, BC_NESTED, BC_WALL), land_frac=0.15)
        wl = add_wind_field(wl, 4, 9, [0.0, 30.0, 90.0], mean=(-6.0, 9.0), seed=4)
    sp = np.hypot(wl.w10[..., 0], wl.w10[..., 1])
    assert sp.min() < 11.0 < sp.max()
    _say(f"gridded wind {case}")
    ref, t_ref, rep, own = run_both(wl, 60)
    assert_parity(rep, ref, label=f"w10 {case} dt-replay")
    assert_parity(own, ref, label=f"w10 {case} own-dt")
    # the field does act: without it the run differs well beyond the tolerance
    base = wl.copy(w10=None, w10_t=None)
    d = _dom(base)
    d.step_dt(O.Oracle(wl).run(nsteps=60)[2])
    off = d.read_state()
    d.close()
    assert parity(off, ref)["hu_l2"] > 5e-4


def test_stress_field_matches_oracle():
    """A gridded wind-stress field (N/m^2 at the samples, interpolated as it
    is) on walls + land, 60 steps against the oracle; the same numbers read as
    wind at 10 m give a different run."""
    wl = add_wind_field(random_small(97, 83, seed=34, land_frac=0.15), 6, 5, [0.0, 40.0, 80.0], seed=6)
    W = wl.w10.astype(np.float64)
    sp = np.hypot(W[..., 0], W[..., 1])[..., None]
    wl = wl.copy(w10=(1.5e-3 * 1.225 * sp * W).astype(np.float32), w10_kind=1)
    _say("stress field")
    ref, t_ref, rep, own = run_both(wl, 60)
    assert_parity(rep, ref, label="stress field dt-replay")
    assert_parity(own, ref, label="stress field own-dt")
    d = _dom(wl.copy(w10_kind=0))
    d.step_dt(O.Oracle(wl).run(nsteps=60)[2])
    other = d.read_state()
    d.close()
    assert parity(other, ref)["hu_l2"] > 5e-4


def test_boundary_field_matches_oracle():
    """Nested sides fed with boundary snapshots at their own spacing (5
    samples along W/E, 8 along S/N, three snapshots), 80 steps against the
    oracle, and equal to the same run given the per-cell strips the oracle
    resampled."""
    base = random_small(97, 83, seed=35, bc=(BC_NESTED,) * 4, land_frac=0.1)
    rng = np.random.default_rng(36)
    n_x, n_y = 8, 5
    coarse = np.stack([np.stack([0.2 * rng.standard_normal(2 * n_y + 2 * n_x) * (k + 1) / 3.0,
                                 0.4 * rng.standard_normal(2 * n_y + 2 * n_x),
                                 0.4 * rng.standard_normal(2 * n_y + 2 * n_x)]) for k in range(3)])
    times = np.array([0.0, 50.0, 120.0])
    wl = base.copy(bnd_t=times, bnd=coarse.astype(np.float32), bnd_nx=n_x, bnd_ny=n_y)
    _say("boundary field")
    ref, t_ref, rep, own = run_both(wl, 80)
    assert_parity(rep, ref, label="boundary field dt-replay")
    assert_parity(own, ref, label="boundary field own-dt")
    cells = O.resample_boundary(coarse.astype(np.float32), wl.nx, wl.ny, n_x, n_y).astype(np.float32)
    d = _dom(base.copy(bnd_t=times, bnd=cells))
    d.step(80)
    same = d.read_state()
    d.close()
    p = parity(same, own[:3])
    assert max(p.values()) <= 1e-6, p


def test_forcing_changes_reach_replayed_graphs():
    """Step graphs captured with a wind field are dropped when the field is
    removed or the dt policy set: graph replay (16-step chunks) equals
    one-by-one launches bitwise after each change."""
    wl = add_wind_field(random_small(97, 83, seed=33), 5, 4, [0.0, 60.0], seed=5).copy(w10=None, w10_t=None)
    field = add_wind_field(random_small(97, 83, seed=33), 5, 4, [0.0, 60.0], seed=5)
    out = []
    for eager in (False, True):
        d = _dom(wl)
        d.enable_timing(eager)  # timing mode launches every step eagerly
        d.set_wind_field(field.w10_t, field.w10)
        d.step(32)
        d.set_wind_field(None, None)
        d.step(32)
        d.set_dt_policy(20.0)
        d.step(32)
        out.append(d.read_state())
        d.close()
    for x, y in zip(out[0][:4], out[1][:4]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("comp", [False, True], ids=["f32state", "compensated"])
def test_new_boundary_data_mid_run_matches_oracle(comp):
    """New boundary snapshots handed over between steps reach the nested
    ghost cells of the very next stage (the state's ghost frame is rebuilt
    from them): 15 steps with one set of snapshots, then 15 with another
    (0.5 m higher, momenta reversed), against the oracle restarted from its
    state after the first 15 steps with the second set.  dt replay and own
    dt."""
    wl = random_small(97, 83, seed=41, steps=30, bc=(BC_NESTED,) * 4, land_frac=0.1)
    b2 = np.array(wl.bnd, dtype=np.float32).copy()
    b2[:, 0] += 0.5
    b2[:, 1:] *= -1.0
    wl2 = wl.copy(bnd=b2)
    _say("new boundary data mid-run", "compensated" if comp else "float32 state")
    s1, t1, dts1, k1 = O.Oracle(wl).run(nsteps=15)
    ref, t_ref, dts2, k2 = O.Oracle(wl2).run(state=s1, t=t1, nsteps=15)
    assert k1 == 15 and k2 == 15
    for mode in ("replay", "own"):
        d = _dom(wl, comp=comp)
        if mode == "replay":
            d.step_dt(dts1)
        else:
            d.step(15)
        d.set_boundary(wl2.bnd_t, b2)
        if mode == "replay":
            d.step_dt(dts2)
        else:
            d.step(15)
        got = d.read_state()
        d.close()
        assert_parity(got, ref, wl.land, label=f"new boundary data, {mode}")


@pytest.mark.parametrize("proj", [False, True])
def test_rossby_beta_plane_matches_oracle(proj):
    """The beta-plane Rossby-wave case of section "Coriolis force" (350 x 350
    cells of 20 km, H = 50 m, f = 8e-5 + 2e-11 n.(x - x_c), north at 30
    degrees, geostrophic eddy), 300 steps (8.4 h), both Coriolis variants."""
    wl = rossby_case(N=350, theta_deg=30.0, steps=300)
    _say(f"rossby proj={proj}")
    ref, t_ref, rep, own = run_both(wl, 300, proj=proj)
    p1 = assert_parity(rep, ref, label="rossby dt-replay")
    p2 = assert_parity(own, ref, label="rossby own-dt")
    _say(p1, p2)


def test_rossby_quarter_turn_on_gpu():
    """The quarter-turned beta-plane problem (north, f gradient and momenta
    turned with the grid) gives the quarter-turned GPU solution; the x and y
    directions take different code paths (lane shifts vs. the row window), so
    the agreement is to float32 rounding, not bitwise."""
    wl = rossby_case(N=350, theta_deg=0.0, steps=300)
    dts = np.full(300, 100.0)
    a = _dom(wl, north_projection=True)
    a.step_dt(dts)
    ea, ua, va, _, _ = a.read_state()
    a.close()
    b = _dom(rotate_ccw(wl), north_projection=True)
    b.step_dt(dts)
    eb, ub, vb, _, _ = b.read_state()
    b.close()
    back = (unrotate_ccw(eb), unrotate_ccw(vb), -unrotate_ccw(ub))
    p = assert_parity(back, (ea, ua, va), l2=1e-5, linf=5e-5, label="quarter turn")
    _say(p)


@pytest.mark.parametrize("which", ["config2", "config3"])
def test_full_size_first_steps(which):
    """Full-size NorKyst-shaped and wet-dry domains: 3 steps, the launch
    configuration the benchmark times, every cell compared."""
    wl = config2() if which == "config2" else config3()
    _say("full size", which, wl.nx, wl.ny)
    ref, t_ref, dts, k = O.Oracle(wl).run(nsteps=3)
    d = _dom(wl)
    d.step_dt(dts)
    rep = d.read_state()
    d.close()
    d = _dom(wl)
    d.autotune()  # the tilings bench.py times (tails, tile order) as the tuner picks them
    _say("tuned tilings", d.stage_tiling(1), d.stage_tiling(2))
    d.step(3)
    own = d.read_state()
    d.close()
    p1 = assert_parity(rep, ref, wl.land, label=f"{which} dt-replay")
    p2 = assert_parity(own, ref, wl.land, label=f"{which} own-dt")
    _say(which, p1, p2)


def test_denormal_momenta_at_dry_front():
    """Denormal momenta in the last wet cells before the beach's dry front
    (the state a long run reaches as numerical diffusion creeps ahead of
    the wave): the face between the last wet cell and the first dry one has
    a denormal a+ - a-, whose FP32 reciprocal must not turn the flux into
    inf * 0.  Stays finite and matches the oracle."""
    wl = config3(nx=128, ny=16, steps=30)
    hu = wl.hu.copy()
    hu[:, 81:85] = np.float32(2.8e-45) * np.arange(1, 5, dtype=np.float32)
    wl = wl.copy(hu=hu)
    assert np.count_nonzero(hu) == 64 and hu.max() < 1e-43
    _say("denormal dry front")
    ref, t_ref, rep, own = run_both(wl, 30)
    for a in own[:3]:
        assert np.isfinite(a).all()
    assert_parity(rep, ref, label="denormal front dt-replay")
    assert_parity(own, ref, label="denormal front own-dt")


def test_config3_runs_dry_front_stays_sane():
    """500 steps of the wet-dry beach: no NaN, depth non-negative up to the
    dry tolerance scale, incoming wave entered."""
    wl = config3()
    d = _dom(wl)
    d.step(500)
    e, u, v, t, dt = d.read_state()
    d.close()
    Hc = wl.Hc.astype(np.float64)
    hb = e + 0.25 * (Hc[:-1, :-1] + Hc[:-1, 1:] + Hc[1:, :-1] + Hc[1:, 1:])
    assert np.all(np.isfinite(e)) and hb.min() > -1e-2
    assert np.abs(e[:, :50]).max() > 0.05


def test_repeatable_and_graph_equals_direct():
    """Bitwise repeatability, and the HIP-graph path (chunks of 16 steps)
    equals direct launches bit for bit."""
    wl = random_small(200, 150, seed=4, land_frac=0.2, bc=(BC_NESTED, BC_WALL, BC_NESTED, BC_WALL),
                      friction=FRIC_MANNING, friction_coeff=0.03)
    outs = []
    for timing in (False, False, True):
        d = _dom(wl)
        if timing:
            d.enable_timing(True)  # timing mode launches kernels one by one
        d.step(40)
        outs.append(d.read_state())
        d.close()
    for k in range(3):
        assert np.array_equal(outs[0][k], outs[1][k])
        assert np.array_equal(outs[0][k], outs[2][k])
    assert outs[0][3] == outs[1][3] == outs[2][3]


def test_checkpoint_resume_bitwise():
    wl = random_small(100, 70, seed=8, land_frac=0.1, friction=FRIC_LINEAR, friction_coeff=2e-3,
                      wind=(0.1, 0.0))
    d = _dom(wl)
    d.step(25)
    full = d.read_state()
    d.close()
    d = _dom(wl)
    d.step(10)
    e, u, v, t, _ = d.read_state()
    d.close()
    d2 = _dom(wl)
    d2.set_state(e, u, v, t)
    d2.step(15)
    res = d2.read_state()
    d2.close()
    for k in range(3):
        assert np.array_equal(full[k], res[k])
    assert full[3] == res[3]


def test_run_until_hits_t_end_and_matches_oracle():
    wl = random_small(80, 64, seed=12, bc=(BC_NESTED, BC_NESTED, BC_WALL, BC_WALL))
    t_end = 157.25
    ref, t_ref, dts, k = O.Oracle(wl).run(nsteps=100000, t_end=t_end)
    d = _dom(wl)
    n = d.run_until(t_end)
    st = d.read_state()
    d.close()
    assert st[3] == t_end and t_ref == t_end
    assert n == k
    assert_parity(st, ref, wl.land, label="run_until")


def test_diagnostics_match_oracle():
    wl = random_small(90, 77, seed=6, land_frac=0.25)
    o = O.Oracle(wl)
    m0, e0 = o.diagnostics(o.initial_state())
    d = _dom(wl)
    m, e = d.diagnostics()
    assert m == pytest.approx(m0, rel=1e-12)
    assert e == pytest.approx(e0, rel=1e-10)
    d.step(50)
    m1, e1 = d.diagnostics()
    d.close()
    assert abs(m1 - m0) / m0 < 1e-6  # closed basin: mass conserved to float32 state rounding


def test_unstable_flag_raised():
    """An overflowing momentum field (finite input) makes the state non-finite;
    the device flag turns into SWE_E_UNSTABLE on the next synchronising call."""
    from paper_1912_02457_amd import SweError
    wl = random_small(64, 32, seed=3)
    wl = wl.copy(hu=np.full_like(wl.hu, 3e38))
    d = _dom(wl)
    d.step(3)
    with pytest.raises(SweError) as ei:
        d.read_state()
    assert ei.value.code == -4
    d.close()


def test_negative_depth_flag_raised():
    """A water depth below -kappa in a wet cell (here handed in through
    set_state; the scheme itself keeps h >= 0 under its CFL bound) raises the
    device flag: SWE_E_UNSTABLE naming the depth, not a non-finite value; a
    valid state handed in afterwards clears it."""
    from paper_1912_02457_amd import SweError
    wl = random_small(64, 32, seed=3)
    d = _dom(wl)
    Hbar = 0.25 * (wl.Hc[:-1, :-1] + wl.Hc[1:, :-1] + wl.Hc[:-1, 1:] + wl.Hc[1:, 1:])
    eta = wl.eta.copy()
    eta[10, 20] = -Hbar[10, 20] - 0.5
    d.set_state(eta, wl.hu, wl.hv)
    assert d.status() == -4
    with pytest.raises(SweError) as ei:
        d.read_state()
    assert ei.value.code == -4 and "depth" in str(ei.value), str(ei.value)
    d.set_state(wl.eta, wl.hu, wl.hv)
    assert d.status() == 0
    d.step(5)
    d.read_state()
    d.close()


def test_lake_at_rest_gpu():
    """Float32 GPU: a lake at rest over random bathymetry with land, f and
    nested sides holding the rest state stays at rest to float32 rounding."""
    wl = random_small(150, 100, seed=2, land_frac=0.2, bc=(BC_NESTED, BC_WALL, BC_WALL, BC_NESTED),
                      depth=(20.0, 3000.0))
    wl = wl.copy(eta=np.zeros_like(wl.eta), hu=np.zeros_like(wl.hu), hv=np.zeros_like(wl.hv),
                 bnd=np.zeros_like(wl.bnd), wind_tau=np.zeros_like(wl.wind_tau))
    d = _dom(wl)
    d.step(200)
    e, u, v, t, _ = d.read_state()
    d.close()
    assert np.abs(e).max() == 0.0
    assert np.abs(u).max() == 0.0 and np.abs(v).max() == 0.0


@pytest.mark.parametrize("which", ["walls_land", "nested_all"])
def test_autotune_leaves_the_simulation_alone(which):
    """The tiling sweep runs stage 1 repeatedly but restores the control
    block: the state, time and next dt are unchanged, and the following
    steps equal those of an untuned twin bitwise."""
    name, nx, ny, kw = next(c for c in CASES if c[0] == which)
    wl = random_small(nx, ny, seed=77, **kw)
    a, b = _dom(wl), _dom(wl)
    a.step(3)
    b.step(3)
    before = a.read_state()
    by = a.autotune()
    assert by >= 2 and a.tiling()[0] == by
    for st in (1, 2):  # the listing covers whatever the tuner settled on
        lst = a.list_tilings(st)
        assert a.stage_tiling(st)[:3] in lst and len(set(lst)) == len(lst)
        assert all(t[1] == 0 for t in lst[:5])  # one-height tilings first (tails only where they fit)
    after = a.read_state()
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    a.step(37)
    b.step(37)
    for x, y in zip(a.read_state(), b.read_state()):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_tiling_does_not_change_results():
    """Rows per wave only changes the work decomposition: results are bitwise
    identical for tile heights that split the domain differently (interior
    and edge tiles, ragged last tile)."""
    wl = random_small(190, 97, seed=21, land_frac=0.15, bc=(BC_NESTED, BC_WALL, BC_PERIODIC, BC_PERIODIC),
                      friction=FRIC_MANNING, friction_coeff=0.03, wind=(0.1, -0.1))
    outs = []
    for by, order in ((0, -1), (3, 0), (7, 1), (16, 2), (64, 3), (200, 1)):
        d = _dom(wl)
        d.set_tiling(by, order)
        d.step(20)
        outs.append((d.tiling(), d.read_state()))
        d.close()
    _say("tilings", [o[0] for o in outs])
    for (_, st) in outs[1:]:
        for k in range(3):
            assert np.array_equal(st[k], outs[0][1][k])


def test_two_band_heights_do_not_change_results():
    """A tiling whose last rows are split into shorter bands launched after
    the others (per stage kernel) gives bitwise the results of one band
    height, for tails that are ragged, a single band, or most of the domain,
    in every tile order; bad arguments are refused."""
    from paper_1912_02457_amd import SweError
    wl = random_small(190, 97, seed=21, land_frac=0.15, bc=(BC_NESTED, BC_WALL, BC_PERIODIC, BC_PERIODIC),
                      friction=FRIC_MANNING, friction_coeff=0.03, wind=(0.1, -0.1))
    d = _dom(wl)
    d.set_tiling(8, 0)
    d.step(20)
    ref = d.read_state()
    d.close()
    for s1, s2, order in (((8, 2, 20), (5, 3, 9), 0), ((16, 4, 40), (12, 2, 1), 1), ((3, 2, 90), (64, 4, 33), 2),
                          ((10, 3, 30), (7, 2, 50), 3)):
        d = _dom(wl)
        d.set_stage_tiling(1, *s1, order=order)
        d.set_stage_tiling(2, *s2, order=order)
        t1, t2 = d.stage_tiling(1), d.stage_tiling(2)
        assert t1[0] == s1[0] and t1[1] == s1[1] and t1[2] >= s1[2] and t1[3] == order
        assert t2[0] == s2[0] and t2[1] == s2[1] and t2[2] >= s2[2]
        d.step(20)
        got = d.read_state()
        d.close()
        _say("two band heights", s1, s2, order, t1, t2)
        for k in range(4):
            assert np.array_equal(got[k], ref[k]), (s1, s2, order, k)
    d = _dom(wl)
    d.set_stage_tiling(2, 8, 8, 30)  # tail not shorter: one band height
    assert d.stage_tiling(2)[:3] == (8, 0, 0)
    for bad in ((3, 8, 0, 0), (1, 0, 0, 0), (1, 8, -1, 0), (1, 8, 2, -5)):
        with pytest.raises(SweError):
            d.set_stage_tiling(*bad)
    d.close()


def test_max_size_domain_tiling_invariant_and_conserving():
    """A 16384 x 16384 domain (268 M cells, 1 GiB per state plane, the
    32-bit byte offsets near their range): finite, mass conserved by the
    float64 diagnostic to float32 rounding, the CFL step of the initial state,
    and bitwise the same under three tilings (one with row-band-major tile
    numbering and tails of short bands, as the tuner picks at this size)."""
    import torch
    N = 16384
    z = np.zeros((N, N), np.float32)
    i = np.arange(N, dtype=np.float32) + 0.5 - N / 2
    bump = np.exp(-(i[None, :] ** 2 + i[:, None] ** 2) / (2 * 40.0 ** 2)).astype(np.float32)
    from workloads import Workload
    wl = Workload(name="max", nx=N, ny=N, dx=1000.0, dy=1000.0, Hc=np.full((N + 1, N + 1), 100.0, np.float32),
                  f=np.full((N, N), 1.2e-4, np.float32), north=z, eta=bump, hu=z, hv=z)
    del z
    _say("max size init")
    outs = []
    for by in (5, 16, (48, 3, 500, 1, 24, 2, 300)):
        d = _dom(wl)
        m0, _ = d.diagnostics()
        e = torch.empty((N, N), dtype=torch.float32, device="cuda:0")
        u, v = torch.empty_like(e), torch.empty_like(e)
        _, dt0 = d.read_state_into(e, u, v)
        assert dt0 == pytest.approx(0.45 * 0.25 * 1000.0 / np.sqrt(9.81 * (100.0 + float(bump.max()))), rel=1e-5)
        if isinstance(by, tuple):
            d.set_stage_tiling(1, *by[0:3], order=by[3])
            d.set_stage_tiling(2, *by[4:7], order=by[3])
        else:
            d.set_tiling(by)
        d.step(6)
        m1, _ = d.diagnostics()
        d.read_state_into(e, u, v)
        assert abs(m1 - m0) <= 1e-6 * m0
        assert bool(torch.isfinite(e).all()) and bool(torch.isfinite(u).all())
        outs.append((e, u, v))
        d.close()
        _say(f"max size by={by} mass drift {abs(m1 - m0) / m0:.2e}")
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert bool(torch.equal(a, b))
