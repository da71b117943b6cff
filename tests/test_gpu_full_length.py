"""Parity at each configuration's full step count: the HIP path against the
FP64 oracle's stored final state (tests/golden/, written by
tests/golden/make_golden.py from oracle/ alone), element by element, to
1e-4 relative L2 and 5e-4 relative Linf per field (eta by its own norm, hu
and hv by the momentum magnitude; land excluded).

Two time-step modes: own dt (each side its CFL dt, eq. cfl, every step; the
gated result) and dt replay (the GPU takes the oracle's dt sequence, which
isolates the spatial operator).  The default state (compensated: each
stored float32 value keeps its rounding error) must meet the bar on every
configuration.  The paper's plain float32 state is run too: it meets the bar
where the run is short enough, and where its storage rounding alone exceeds
the Linf bar (the NorKyst-sized hour and the served requests; see
test_oracle_float32_state.py) its numbers are recorded and only the L2 bar
is asserted.

Set FULL_LENGTH_REPORT=path to append one JSON line per case there."""

import json
import os
import sys
import time

import numpy as np
import pytest

from tests._parity import L2_TOL, LINF_TOL, parity

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
sys.path.insert(0, GOLDEN)
import make_golden as MG  # noqa: E402

# configurations whose float32-state result is expected inside the Linf bar
FLOAT32_LINF_OK = {"config1", "config3"} | {f"config4_m{k}" for k in range(8)}

CASES = ["config1", "config2", "config3"] + [f"config4_m{k}" for k in range(8)] + [f"config5_r{k}" for k in range(6)]


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


def golden(name):
    """Decoded oracle result: (eta, hu, hv) on the full grid (land cells 0),
    the dt sequence, the final time, the steps taken."""
    path = os.path.join(GOLDEN, f"{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"fixture {name}.npz not generated")
    z = np.load(path)
    wl = MG.workload(name)
    wet = np.ones((wl.ny, wl.nx), bool) if wl.land is None else (np.asarray(wl.land) == 0)
    out = []
    for f in ("eta", "hu", "hv"):
        a = np.zeros((wl.ny, wl.nx))
        a[wet] = MG.decode_field(z[f"{f}_z"], float(z[f"{f}_q"]), int(z["count"]))
        out.append(a)
    return wl, tuple(out), np.asarray(z["dts"]), float(z["t"]), int(z["steps"])


def _report(rec):
    path = os.environ.get("FULL_LENGTH_REPORT")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(rec) + "\n")


def _run(wl, comp, dts=None):
    from paper_1912_02457_amd import Domain
    d = Domain.from_workload(wl, device="cuda:0", compensated_state=comp)
    if dts is not None:
        d.step_dt(dts)
        k = len(dts)
    elif wl.t_end:
        k = d.run_until(wl.t_end)
    else:
        d.step(wl.steps)
        k = wl.steps
    st = d.read_state()
    d.close()
    return st, k


@pytest.mark.parametrize("name", CASES)
def test_full_length_parity(name):
    wl, ref, dts, t_ref, k_ref = golden(name)
    _say("full length", name, wl.nx, wl.ny, k_ref, "steps")
    for comp in (True, False):
        for mode in ("own", "replay"):
            t0 = time.time()
            st, k = _run(wl, comp, dts if mode == "replay" else None)
            p = {a: float(b) for a, b in parity(st, ref, wl.land).items()}
            rec = {"config": name, "state": "compensated" if comp else "float32", "dt": mode, "steps": int(k),
                   "oracle_steps": k_ref, "t": float(st[3]), "t_oracle": t_ref, **p,
                   "seconds": round(time.time() - t0, 2)}
            _say(json.dumps(rec))
            _report(rec)
            # the run covers the oracle's simulated time (own dt: same end time
            # and, in practice, the same number of steps)
            assert abs(st[3] - t_ref) <= 1e-9 * max(t_ref, 1.0) + (0.0 if wl.t_end else 1e-5 * t_ref), (st[3], t_ref)
            l2 = max(p["eta_l2"], p["hu_l2"], p["hv_l2"])
            linf = max(p["eta_linf"], p["hu_linf"], p["hv_linf"])
            assert l2 <= L2_TOL, f"{name} {rec['state']} {mode}: relative L2 {l2:.3e}"
            if comp or name in FLOAT32_LINF_OK:
                assert linf <= LINF_TOL, f"{name} {rec['state']} {mode}: relative Linf {linf:.3e}"
