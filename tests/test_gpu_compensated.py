"""GPU tests of the compensated state (each stored float32 value of Q^n and
Q* keeps its rounding error in a second plane, updated by an error-free
sum): parity with the FP64 oracle on random cases, the error after a long
run against the plain float32 state, bitwise agreement with the ensemble
launch, and the tiling sweep and set_state leaving it alone."""

import sys
import zlib

import numpy as np
import pytest

from oracle import oracle as O
from tests._parity import assert_parity, parity
from workloads import (BC_NESTED, BC_PERIODIC, BC_WALL, FRIC_LINEAR, FRIC_MANNING, FRIC_QUADRATIC,
                       random_small)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    from paper_1912_02457_amd import load_library
    load_library()
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dom(wl, comp=True, **kw):
    from paper_1912_02457_amd import Domain
    return Domain.from_workload(wl, device="cuda:0", compensated_state=comp, **kw)


CASES = [
    ("walls_land", 133, 71, dict(land_frac=0.2, friction=FRIC_LINEAR, friction_coeff=3e-3, wind=(0.1, 0.05))),
    ("periodic", 64, 48, dict(bc=(BC_PERIODIC,) * 4, friction=FRIC_QUADRATIC, friction_coeff=2e-3)),
    ("nested_all", 97, 83, dict(bc=(BC_NESTED,) * 4, land_frac=0.1, wind=(-0.05, 0.1))),
    ("wet_dry_manning", 120, 90, dict(wet_dry=True, friction=FRIC_MANNING, friction_coeff=0.03, amp=0.5)),
    ("strip_plus_one", 61, 16, dict(bc=(BC_WALL, BC_NESTED, BC_WALL, BC_WALL))),
]


@pytest.mark.parametrize("name,nx,ny,kw", CASES, ids=[c[0] for c in CASES])
def test_compensated_matches_oracle(name, nx, ny, kw):
    wl = random_small(nx, ny, seed=zlib.crc32(name.encode()) % 1000, steps=30, **kw)
    _say("compensated case", name, nx, ny)
    ref, t_ref, dts, k = O.Oracle(wl).run(nsteps=60)
    d = _dom(wl)
    d.step(60)
    got = d.read_state()
    d.close()
    assert_parity(got, ref, wl.land, label=f"compensated {name}")
    assert abs(got[3] - t_ref) <= 1e-5 * t_ref
    if wl.land is not None:
        lm = wl.land > 0
        assert np.array_equal(got[0][lm], wl.eta[lm]) and np.array_equal(got[1][lm], wl.hu[lm])


def test_compensated_long_run_closer_to_oracle():
    """Over 3000 steps of a deep basin with land, the error of the plain
    float32 state grows with the number of stored roundings; the compensated
    state stays closer to the FP64 oracle (same dt sequence on all sides)."""
    wl = random_small(96, 80, seed=5, land_frac=0.1, depth=(200.0, 3000.0), amp=0.5,
                      friction=FRIC_LINEAR, friction_coeff=1e-3, wind=(0.05, 0.02))
    n = 3000
    _say("long run oracle", n)
    ref, t_ref, dts, k = O.Oracle(wl).run(nsteps=n)
    out = {}
    for comp in (False, True):
        d = _dom(wl, comp=comp)
        d.step_dt(dts)
        out[comp] = parity(d.read_state(), ref, wl.land)
        d.close()
    _say("plain", out[False])
    _say("compensated", out[True])
    for key in ("eta_linf", "hu_linf", "hv_linf", "eta_l2", "hu_l2", "hv_l2"):
        assert out[True][key] <= out[False][key] * 1.05, key
    assert out[True]["eta_linf"] < 0.5 * out[False]["eta_linf"]


def test_compensated_ensemble_bitwise():
    """Compensated members inside the persistent ensemble launch equal their
    standalone twins bit for bit; an ensemble cannot mix the two state kinds."""
    from paper_1912_02457_amd import Ensemble, SweError
    wls = [random_small(97, 83, seed=21, bc=(BC_NESTED,) * 4, land_frac=0.1),
           random_small(64, 48, seed=22, bc=(BC_PERIODIC,) * 4, friction=FRIC_QUADRATIC, friction_coeff=2e-3),
           random_small(40, 30, seed=23, wind=(0.1, 0.0))]
    alone = []
    for wl in wls:
        d = _dom(wl)
        d.step(41)
        alone.append(d.read_state())
        d.close()
    doms = [_dom(wl) for wl in wls]
    with Ensemble(doms) as e:
        e.step(16)
        e.step(25)
        got = [d.read_state() for d in doms]
    for d in doms:
        d.close()
    for g, a in zip(got, alone):
        for x, y in zip(g[:5], a[:5]):
            assert np.array_equal(x, y)
    mixed = [_dom(wls[0]), _dom(wls[1], comp=False)]
    with pytest.raises(SweError):
        Ensemble(mixed)
    for d in mixed:
        d.close()


def test_compensated_autotune_and_tiling_leave_it_alone():
    """The tiling sweep saves and restores the error planes with the state;
    tile heights do not change compensated results."""
    name, nx, ny, kw = CASES[2]
    wl = random_small(nx, ny, seed=77, **kw)
    a, b = _dom(wl), _dom(wl)
    a.step(3)
    b.step(3)
    by = a.autotune()
    assert by >= 2
    a.step(37)
    b.step(37)
    for x, y in zip(a.read_state(), b.read_state()):
        assert np.array_equal(x, y)
    a.close()
    b.close()
    outs = []
    for by in (0, 3, 16, 200):
        d = _dom(wl)
        d.set_tiling(by)
        d.step(20)
        outs.append(d.read_state())
        d.close()
    for st in outs[1:]:
        for k in range(3):
            assert np.array_equal(st[k], outs[0][k])


def test_compensated_set_state_restarts_errors():
    """set_state hands in float32 values with no rounding error: a domain
    that ran and was then reset to a state continues exactly like a fresh
    domain created from that state."""
    wl = random_small(70, 50, seed=31, land_frac=0.1)
    d = _dom(wl)
    d.step(25)
    st = d.read_state()
    d.set_state(wl.eta, wl.hu, wl.hv, 0.0)
    d.step(25)
    again = d.read_state()
    d.close()
    for x, y in zip(st[:4], again[:4]):
        assert np.array_equal(x, y)
