"""GPU tests of the batched ensemble: every member advanced inside the
persistent ensemble launch must equal, bitwise, the same domain stepped on its
own (the per-member arithmetic does not depend on the batch, and the dt
reduction is a max), and ensemble members of the many-domain workload must
meet the oracle parity bar."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from tests._parity import assert_parity
from workloads import (BC_NESTED, BC_PERIODIC, BC_WALL, FRIC_LINEAR, FRIC_MANNING, FRIC_QUADRATIC,
                       config4_member, random_small)

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


MIX = [
    (133, 71, dict(land_frac=0.2, friction=FRIC_LINEAR, friction_coeff=3e-3, wind=(0.1, 0.05))),
    (64, 48, dict(bc=(BC_PERIODIC,) * 4, friction=FRIC_QUADRATIC, friction_coeff=2e-3)),
    (97, 83, dict(bc=(BC_NESTED,) * 4, land_frac=0.1, wind=(-0.05, 0.1))),
    (5, 3, dict()),
    (120, 90, dict(wet_dry=True, friction=FRIC_MANNING, friction_coeff=0.03, amp=0.5)),
    (61, 130, dict(bc=(BC_NESTED, BC_WALL, BC_PERIODIC, BC_PERIODIC))),
    (300, 7, dict(land_frac=0.3)),
    (2, 2, dict(bc=(BC_NESTED, BC_WALL, BC_NESTED, BC_WALL))),
]


def _mix_workloads():
    return [random_small(nx, ny, seed=100 + k, **kw) for k, (nx, ny, kw) in enumerate(MIX)]


def _same(a, b, label):
    for name, x, y in zip(("eta", "hu", "hv"), a[:3], b[:3]):
        assert np.array_equal(x, y), f"{label}: {name} differs (max |diff| {np.abs(x - y).max():.3e})"
    assert a[3] == b[3], f"{label}: t {a[3]} != {b[3]}"
    assert a[4] == b[4], f"{label}: dt_next {a[4]} != {b[4]}"


@pytest.mark.parametrize("rows,chunk", [(0, 0), (1, 1), (7, 3), (64, 16)])
def test_members_equal_standalone_bitwise(rows, chunk):
    """37 steps (two 16-step graph chunks plus 5 direct steps) of a mix of
    sizes, boundary kinds, frictions, land and wet-dry: each member equals its
    standalone twin bit for bit."""
    from paper_1912_02457_amd import Ensemble
    wls = _mix_workloads()
    n = 37
    _say(f"ensemble mix rows={rows} chunk={chunk}")
    alone = []
    for wl in wls:
        d = _dom(wl)
        d.step(n)
        alone.append(d.read_state())
        d.close()
    doms = [_dom(wl) for wl in wls]
    with Ensemble(doms, rows_per_wave=rows, chunk=chunk) as e:
        by, ch, items, blocks = e.info()
        assert by == (rows or by) and ch == (chunk or ch) and items >= len(wls) and blocks % 8 == 0
        e.step(16)
        e.step(n - 16)
        got = [d.read_state() for d in doms]
    for k, (g, a) in enumerate(zip(got, alone)):
        _same(g, a, f"member {k} {wls[k].name}")
    for d in doms:
        d.close()


def test_members_joining_at_different_parities_and_leaving():
    """Members that already took an odd or even number of steps join one
    ensemble; after the ensemble is released they step on their own again:
    every member still equals its twin that was never batched."""
    from paper_1912_02457_amd import Ensemble
    wls = _mix_workloads()[:5]
    pre = [0, 1, 2, 3, 5]
    doms, twins = [], []
    for wl, p in zip(wls, pre):
        d = _dom(wl)
        if p:
            d.step(p)
        doms.append(d)
        twins.append(_dom(wl))
    e = Ensemble(doms)
    e.step(21)
    e.close()
    for d in doms:
        d.step(4)
    for d, tw, p in zip(doms, twins, pre):
        tw.step(p + 25)
        _same(d.read_state(), tw.read_state(), f"pre={p}")
    for d in doms + twins:
        d.close()


def test_ensemble_stage_timing_path_equals_graph_path():
    """Event-timed direct launches give the same result as the graph path."""
    from paper_1912_02457_amd import Ensemble
    wls = _mix_workloads()[:4]
    a = [_dom(wl) for wl in wls]
    b = [_dom(wl) for wl in wls]
    ea, eb = Ensemble(a), Ensemble(b)
    ea.step(32)
    eb.enable_timing(True)
    eb.step(32)
    ms1, ms2, nl = eb.stage_times()
    assert nl == 32 and ms1 > 0 and ms2 > 0
    ea.close()
    eb.close()
    for x, y in zip(a, b):
        _same(x.read_state(), y.read_state(), "timed vs graph")
        x.close()
        y.close()


def test_member_calls_rejected_while_batched():
    from paper_1912_02457_amd import Ensemble, SweError
    wl = random_small(40, 30, seed=7)
    d = _dom(wl)
    e = Ensemble([d])
    for call in (lambda: d.step(1), lambda: d.run_until(10.0), lambda: d.set_tiling(4),
                 lambda: d.set_state(wl.eta, wl.hu, wl.hv), lambda: Ensemble([d])):
        with pytest.raises(SweError) as ei:
            call()
        assert ei.value.code == -5
    # reading and diagnostics stay available
    d.read_state()
    d.diagnostics()
    e.close()
    d.step(1)
    d.close()


def test_destroyed_member_breaks_ensemble_cleanly():
    from paper_1912_02457_amd import Ensemble, SweError
    a, b = _dom(random_small(30, 20, seed=8)), _dom(random_small(20, 30, seed=9))
    e = Ensemble([a, b])
    e.step(2)
    a.close()
    with pytest.raises(SweError) as ei:
        e.step(1)
    assert ei.value.code == -5
    e.close()
    b.step(1)
    b.close()


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_config4_members_match_oracle(k):
    """Members of the 256-member ensemble (coastal 1 km domains with land,
    walls, f = 1.2e-4, per-member wind) inside one ensemble of 8 members,
    60 steps each with its own dt, against the FP64 oracle."""
    from paper_1912_02457_amd import Ensemble
    n = 60
    wl = config4_member(k)
    others = [config4_member(j) for j in range(8) if j != k][:7]
    _say(f"config4 member {k} {wl.nx}x{wl.ny}")
    ref, t_ref, dts, kk = O.Oracle(wl).run(nsteps=n)
    assert kk == n
    doms = [_dom(wl)] + [_dom(o) for o in others]
    with Ensemble(doms) as e:
        e.step(n)
        got = doms[0].read_state()
    p = assert_parity(got, ref, label=f"config4 member {k}")
    assert abs(got[3] - t_ref) <= 1e-5 * t_ref
    _say(p)
    for d in doms:
        d.close()
