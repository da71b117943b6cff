"""GPU tests of the time-step update policy of section "Real-world
simulations" (dt from the CFL condition only once per update interval; the
paper's runs use 20 simulated minutes): parity with the oracle under the
same policy, the held dt between updates, run-to-time, graphs and the
ensemble launch."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from tests._parity import assert_parity
from workloads import BC_NESTED, FRIC_LINEAR, config1, random_small

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


def _dom(wl, **kw):
    from paper_1912_02457_amd import Domain
    return Domain.from_workload(wl, device="cuda:0", **kw)


@pytest.mark.parametrize("name,nx,ny,kw", [
    ("walls_land", 133, 71, dict(land_frac=0.2, friction=FRIC_LINEAR, friction_coeff=3e-3, wind=(0.1, 0.05))),
    ("nested_all", 97, 83, dict(bc=(BC_NESTED,) * 4, land_frac=0.1, wind=(-0.05, 0.1))),
])
def test_dt_policy_matches_oracle(name, nx, ny, kw):
    """Both sides hold dt between updates every 5 simulated seconds; 300
    steps (several updates, through the 16-step graph chunks)."""
    wl = random_small(nx, ny, seed=7, **kw).copy(dt_interval=5.0)
    _say(f"dt policy parity {name}")
    ref, t_ref, dts, k = O.Oracle(wl).run(nsteps=300)
    nup = 1 + int(np.sum(np.diff(dts) != 0))
    assert nup >= 4
    d = _dom(wl)
    d.step(300)
    got = d.read_state()
    d.close()
    assert_parity(got, ref, land=wl.land, label=f"dt policy {name}")
    assert abs(got[3] - t_ref) <= 1e-5 * t_ref


def test_dt_policy_holds_dt_on_gpu():
    """Step by step: the dt the next step takes (reported by read_state) stays
    the same between updates and changes at the first step starting at or
    after each update time; with the policy off it changes every step."""
    wl = config1()
    d = _dom(wl)
    d.set_dt_policy(40.0)
    nxt, seq = 0.0, []
    for n in range(70):
        _, _, _, t, dt_next = d.read_state()
        up = n == 0 or t >= nxt
        if up:
            nxt = nxt + 40.0 if nxt + 40.0 > t else t + 40.0
        seq.append((up, dt_next))
        d.step(1)
    d.close()
    ups = [u for u, _ in seq]
    assert 5 <= sum(ups) <= 8
    for (u, dt), (_, prev) in zip(seq[1:], seq[:-1]):
        if not u:
            assert dt == prev
    held = [dt for u, dt in seq if u]
    assert len(set(held)) == len(held)
    d = _dom(wl)
    vals = []
    for n in range(10):
        vals.append(d.read_state()[4])
        d.step(1)
    d.close()
    assert len(set(vals)) == 10


def test_dt_policy_run_until_and_reset():
    """run_until ends exactly at its time under the policy and takes the
    oracle's number of steps; set_dt_policy(0) goes back to every-step dt
    (bitwise the never-held run from the same state).  Float32 state: a
    restart from a state handed in starts the compensated state's error
    planes at zero, so only the float32 state restarts bitwise."""
    wl = random_small(64, 48, seed=9).copy(dt_interval=7.0)
    ref, t_ref, dts, k = O.Oracle(wl).run(nsteps=100000, t_end=61.0)
    d = _dom(wl, compensated_state=False)
    n = d.run_until(61.0)
    got = d.read_state()
    assert got[3] == 61.0 and n == k
    assert_parity(got, ref, land=wl.land, label="dt policy run_until")
    d.set_dt_policy(0.0)
    d.step(5)
    a = d.read_state()
    d.close()
    d2 = _dom(wl.copy(dt_interval=0.0), compensated_state=False)
    d2.set_state(got[0], got[1], got[2], 61.0)
    d2.step(5)
    b = d2.read_state()
    d2.close()
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)


def test_dt_policy_in_ensemble_bitwise():
    """Members with the policy inside the persistent ensemble launch equal
    their standalone twins bit for bit."""
    from paper_1912_02457_amd import Ensemble
    wls = [random_small(97, 83, seed=11, bc=(BC_NESTED,) * 4).copy(dt_interval=3.0),
           random_small(64, 48, seed=12).copy(dt_interval=11.0), random_small(40, 30, seed=13)]
    alone = []
    for wl in wls:
        d = _dom(wl)
        d.step(53)
        alone.append(d.read_state())
        d.close()
    doms = [_dom(wl) for wl in wls]
    with Ensemble(doms) as e:
        e.step(16)
        e.step(37)
        got = [d.read_state() for d in doms]
    for d in doms:
        d.close()
    for g, a in zip(got, alone):
        for x, y in zip(g[:5], a[:5]):
            assert np.array_equal(x, y)
