"""What storing the state in float32 (as the paper does) costs by itself,
with no float32 arithmetic anywhere: the FP64 oracle whose state is rounded
to float32 after every step, against the plain FP64 oracle, both over the
full step count (fixtures written by tests/golden/make_golden.py from the
oracle alone).

On the NorKyst-sized hour (config 2) this rounding alone exceeds the 5e-4
relative Linf bar while staying inside the 1e-4 L2 bar -- the pattern the
GPU's float32 state shows there (tests/test_gpu_full_length.py), and the
reason the benchmarked path keeps each stored value's rounding error."""

import os
import sys

import numpy as np
import pytest

from tests._parity import L2_TOL, LINF_TOL, parity

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
sys.path.insert(0, GOLDEN)
import make_golden as MG  # noqa: E402


def _decoded(name):
    path = os.path.join(GOLDEN, f"{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"fixture {name}.npz not generated")
    z = np.load(path)
    base = name[: -len("_f32state")] if name.endswith("_f32state") else name
    wl = MG.workload(base)
    wet = np.ones((wl.ny, wl.nx), bool) if wl.land is None else (np.asarray(wl.land) == 0)
    out = []
    for f in ("eta", "hu", "hv"):
        a = np.zeros((wl.ny, wl.nx))
        a[wet] = MG.decode_field(z[f"{f}_z"], float(z[f"{f}_q"]), int(z["count"]))
        out.append(a)
    return wl, tuple(out), float(z["t"]), int(z["steps"])


def test_float32_storage_alone_exceeds_linf_on_config2():
    wl, exact, t, k = _decoded("config2")
    _, rounded, t32, k32 = _decoded("config2_f32state")
    assert t == t32 == 3600.0
    assert abs(k - k32) <= 2
    p = parity(rounded, exact, wl.land)
    l2 = max(p["eta_l2"], p["hu_l2"], p["hv_l2"])
    linf = max(p["eta_linf"], p["hu_linf"], p["hv_linf"])
    print(f"config 2, float32 storage alone: L2 {l2:.2e}, Linf {linf:.2e}", {a: f"{b:.2e}" for a, b in p.items()})
    assert l2 <= L2_TOL
    assert linf > LINF_TOL


def test_float32_storage_on_a_served_request():
    wl, exact, t, k = _decoded("config5_r0")
    _, rounded, t32, k32 = _decoded("config5_r0_f32state")
    assert t == t32 == 7200.0
    p = parity(rounded, exact, wl.land)
    l2 = max(p["eta_l2"], p["hu_l2"], p["hv_l2"])
    linf = max(p["eta_linf"], p["hu_linf"], p["hv_linf"])
    print(f"request 0 (2 h), float32 storage alone: L2 {l2:.2e}, Linf {linf:.2e}")
    # inside the L2 bar; the Linf deviation is of the size the GPU's float32
    # state shows on this request (1.9e-4 with the oracle's dt sequence)
    assert l2 <= L2_TOL
    assert 1e-5 < linf < 5e-3
