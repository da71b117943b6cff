"""GPU tests of the continuous-batching serving loop: requests of different
sizes and horizons join and leave the batch at tick boundaries; each result
equals, bitwise, the same request run alone to its horizon, admission
respects the arena, and a served request meets the oracle parity bar."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from tests._parity import assert_parity
from workloads import FRIC_LINEAR, config5_member, random_small

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


def _alone(wl, horizon):
    from paper_1912_02457_amd import Domain
    d = Domain.from_workload(wl, device="cuda:0")
    k = d.run_until(horizon)
    st = d.read_state()
    d.close()
    return st, k


def _drain(srv, max_ticks=100000):
    done = []
    for _ in range(max_ticks):
        a, p = srv.tick()
        done += srv.poll()
        if a == 0 and p == 0:
            return done
    raise AssertionError("server did not drain")


REQS = [
    # (workload, horizon s)
    (lambda: config5_member(150, 100, 0), 900.0),
    (lambda: config5_member(300, 120, 0), 200.0),
    (lambda: random_small(97, 83, seed=41, land_frac=0.15, friction=FRIC_LINEAR, friction_coeff=2e-3,
                          wind=(0.1, -0.05)), 600.0),
    (lambda: config5_member(100, 100, 0), 0.0),
    (lambda: config5_member(611, 37, 0), 1500.0),
    (lambda: random_small(64, 200, seed=42, wet_dry=True, amp=0.4), 120.0),
    (lambda: config5_member(120, 260, 0), 333.3),
]


@pytest.mark.parametrize("steps_per_tick,max_active", [(8, 64), (5, 2), (32, 3)])
def test_served_results_equal_standalone_bitwise(steps_per_tick, max_active):
    from paper_1912_02457_amd import Server
    wls = [(mk(), h) for mk, h in REQS]
    _say(f"server K={steps_per_tick} slots={max_active}")
    with Server(1 << 30, max_active=max_active, steps_per_tick=steps_per_tick, device="cuda:0") as srv:
        for k, (wl, h) in enumerate(wls):
            srv.submit(wl, h, req_id=100 + k)
        # a few ticks, then a late arrival
        srv.tick()
        late = config5_member(90, 140, 0)
        srv.submit(late, 450.0, req_id=999)
        done = _drain(srv)
        st = srv.stats()
    wls.append((late, 450.0))
    ids = [100 + k for k in range(len(REQS))] + [999]
    assert sorted(c["id"] for c in done) == sorted(ids)
    assert st["completed"] == len(ids) and st["active"] == 0 and st["pending"] == 0
    assert st["arena_used"] == 0 and st["arena_peak"] > 0
    by_id = {c["id"]: c for c in done}
    for rid, (wl, h) in zip(ids, wls):
        c = by_id[rid]
        assert c["status"] == 0
        (e, u, v, t, _), k = _alone(wl, h)
        assert c["t"] == t, (rid, c["t"], t)
        assert c["steps"] == k
        for name, a, b in zip(("eta", "hu", "hv"), c["state"], (e, u, v)):
            assert np.array_equal(a, b), f"request {rid}: {name} differs from the standalone run"


def test_admission_respects_arena_and_slots():
    """An arena that holds about two of the requests at a time: never more
    than that is resident, everything still completes in arrival order of
    admission, and a request larger than the arena is refused at submit."""
    from paper_1912_02457_amd import Server, SweError, workspace_bytes
    from paper_1912_02457_amd.swe import params_of
    wls = [config5_member(200, 150, 0) for _ in range(6)]
    one = workspace_bytes(params_of(wls[0]), 1, 0)
    arena = int(2.5 * one)
    with Server(arena, max_active=8, steps_per_tick=16, device="cuda:0") as srv:
        for k, wl in enumerate(wls):
            srv.submit(wl, 300.0 + 50.0 * k, req_id=k)
        big = config5_member(1200, 800, 0)
        with pytest.raises(SweError) as ei:
            srv.submit(big, 10.0, req_id=77)
        assert ei.value.code == -2
        peak_active = 0
        done = []
        for _ in range(10000):
            a, p = srv.tick()
            peak_active = max(peak_active, a)
            done += srv.poll()
            if a == 0 and p == 0:
                break
        st = srv.stats()
    assert peak_active <= 2
    assert st["arena_peak"] <= arena
    assert sorted(c["id"] for c in done) == list(range(6))


def test_served_request_matches_oracle():
    """A served forecast request (flat 100 m, walls, f = 1.2e-4, Gaussian
    bump) run to a 2000 s horizon inside a mix, against the FP64 oracle run
    to the same time."""
    from paper_1912_02457_amd import Server
    wl = config5_member(160, 120, 2000.0)
    ref, t_ref, dts, k = O.Oracle(wl).run(nsteps=10 ** 6, t_end=2000.0)
    assert abs(t_ref - 2000.0) < 1e-9
    with Server(1 << 30, max_active=8, steps_per_tick=16, device="cuda:0") as srv:
        srv.submit(config5_member(300, 200, 0), 3000.0, req_id=1)
        srv.submit(wl, 2000.0, req_id=2)
        srv.submit(config5_member(50, 400, 0), 700.0, req_id=3)
        done = {c["id"]: c for c in _drain(srv)}
    got = done[2]
    assert got["t"] == 2000.0 and abs(got["steps"] - k) <= 1
    p = assert_parity(got["state"] + (got["t"], 0.0), ref, label="served request")
    _say(p)


def test_refused_request_is_reported_and_others_complete():
    """A request whose inputs are refused when it is started (a NaN in the
    initial state) completes at once with SWE_E_ARG; the rest of the stream
    is served as usual."""
    from paper_1912_02457_amd import Server
    good = config5_member(80, 60, 0)
    bad_eta = good.eta.copy()
    bad_eta[10, 10] = np.nan
    bad = good.copy(eta=bad_eta)
    with Server(1 << 28, max_active=4, steps_per_tick=8, device="cuda:0") as srv:
        srv.submit(good, 200.0, req_id=1)
        srv.submit(bad, 200.0, req_id=2)
        srv.submit(good, 100.0, req_id=3)
        done = {c["id"]: c for c in _drain(srv)}
    assert done[2]["status"] == -1 and done[2]["steps"] == 0
    assert done[1]["status"] == 0 and done[1]["t"] == 200.0
    assert done[3]["status"] == 0 and done[3]["t"] == 100.0


def test_mixed_kinds_are_served_in_turn():
    """Requests with the compensated state or the literal north projection
    run other kernel variants than the plain ones, so one batch holds one
    kind: a stream that alternates kinds still completes every request,
    each bitwise equal to its standalone run of the same kind, and never
    mixes kinds in the active set."""
    from paper_1912_02457_amd import Domain, Server
    f32 = dict(compensated_state=False)
    kinds = [f32, dict(compensated_state=True), f32, dict(north_projection=True), dict(compensated_state=True),
             f32]
    wls = [(config5_member(120 + 30 * k, 90 + 10 * k, 0), 300.0 + 40.0 * k) for k in range(len(kinds))]
    with Server(1 << 30, max_active=8, steps_per_tick=16, device="cuda:0") as srv:
        for k, ((wl, h), kw) in enumerate(zip(wls, kinds)):
            srv.submit(wl, h, req_id=k, **kw)
        done = _drain(srv)
        st = srv.stats()
    assert sorted(c["id"] for c in done) == list(range(len(kinds)))
    assert st["completed"] == len(kinds) and st["arena_used"] == 0
    by_id = {c["id"]: c for c in done}
    for k, ((wl, h), kw) in enumerate(zip(wls, kinds)):
        c = by_id[k]
        assert c["status"] == 0
        d = Domain.from_workload(wl, device="cuda:0", **kw)
        n = d.run_until(h)
        e, u, v, t, _ = d.read_state()
        d.close()
        assert c["t"] == t and c["steps"] == n
        for a, b in zip(c["state"], (e, u, v)):
            assert np.array_equal(a, b), f"request {k} ({kw}) differs from its standalone run"
