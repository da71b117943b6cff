"""Benchmark: SSP-RK2 steps of the eta-based central-upwind shallow-water
scheme on the NorKyst-shaped synthetic domain (2600 x 900 cells at 800 m,
~35 % land, nested M2-tide boundaries, linear drag, uniform wind stress,
latitude-dependent f), one MI355X.

One "step" = both stage kernels of one SSP-RK2 step over the whole domain,
with the time step computed on the device from the CFL condition.  Inputs are
resident in HBM before the timed region starts.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# Algorithmic bytes per cell and stage (float32 state; Coriolis-field plane
# f carries the land mask; corner depths count one float per cell):
#   stage 1, wet cell : read eta,hu,hv (12) + Hc (4) + f (4), write Q* (12)      = 32
#   stage 2, wet cell : read Q* (12) + Q^n (12) + Hc (4) + f (4), write Q^n+1 (12) = 44
#   land cell, either stage: read its Q (12) + Hc (4) + f (4) for the neighbours,
#   nothing written (land is frozen)                                            = 20
BYTES = {1: (32, 20), 2: (44, 20)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the oracle sample")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run warmup + this many steps (for rocprofv3 runs), no JSON")
    return ap.parse_args()


def cpu_baseline(wl, target_s):
    """The FP64 oracle as it is, on this host's cores, over a bounded number
    of steps of the same workload."""
    from oracle import oracle as orc
    o = orc.Oracle(wl)
    st = o.initial_state()
    t = 0.0
    steps = 0
    t0 = time.perf_counter()
    while True:
        st, t, _, k = o.run(st, t, nsteps=1, record_dt=False)
        steps += k
        el = time.perf_counter() - t0
        if el >= target_s or steps >= 2000:
            break
    return {
        "value": wl.nx * wl.ny * steps / el,
        "unit": "cell-updates/s",
        "cores": orc.num_threads(),
        "kind": "oracle",
        "sample": f"first {steps} steps of the same {wl.nx}x{wl.ny} workload, FP64 C oracle, "
                  f"{el:.1f} s wall",
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}); the shallow-water path here is a "
              "single-GPU build and no multi-GPU figure is produced", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1912_02457_amd import Domain
    from workloads import config2

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    wl = config2()
    cells = wl.nx * wl.ny
    land_cells = int(np.count_nonzero(wl.land)) if wl.land is not None else 0
    wet_cells = cells - land_cells
    dom = Domain.from_workload(wl, device="cuda:0")
    rows_per_wave, tile_order, waves = dom.tiling()

    dom.step(a.warmup)
    torch.cuda.synchronize()
    if a.profile_steps:
        dom.step(a.profile_steps)
        torch.cuda.synchronize()
        print(f"profiled {a.profile_steps} steps", flush=True)
        return

    # timed region: K steps through the captured HIP graphs of the stage
    # kernels (the production path), wall clock with a device sync on both sides
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dom.step(a.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    # the same K steps with every stage launch bracketed by HIP events
    # (hipExtLaunchKernelGGL start/stop events on the domain's stream): the
    # per-kernel durations behind the roofline figure
    dom.enable_timing(True)
    dom.stage_times(reset=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom.step(a.steps)
    torch.cuda.synchronize()
    el_events = time.perf_counter() - t1
    ms1, ms2, nl = dom.stage_times(reset=True)
    dom.enable_timing(False)

    e, u, v, t_sim, dt_next = dom.read_state()
    finite = bool(np.isfinite(e).all() and np.isfinite(u).all() and np.isfinite(v).all())
    dom.close()

    b1 = BYTES[1][0] * wet_cells + BYTES[1][1] * land_cells
    b2 = BYTES[2][0] * wet_cells + BYTES[2][1] * land_cells
    dominant = 2 if ms2 >= ms1 else 1
    ms_dom = ms2 if dominant == 2 else ms1
    bytes_dom = b2 if dominant == 2 else b1
    achieved = bytes_dom / (ms_dom * 1e-3) / 1e9

    value = cells * a.steps / el
    out = {
        "metric": "cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": el / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "norkyst_2600x900_800m_nested_m2_tide",
            "nx": wl.nx, "ny": wl.ny, "dx_m": wl.dx, "cells": cells, "land_fraction": land_cells / cells,
            "boundaries": "nested (M2 tide, hourly snapshots) on all sides", "friction": "linear r=3e-3 m/s",
            "wind_stress_Nm2": 0.1, "courant": wl.courant, "dt_s": dt_next,
            "rows_per_wave": rows_per_wave, "tile_order": tile_order, "waves_per_stage": waves,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"stage_kernel<{dominant}>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes_per_launch": bytes_dom,
            "avg_launch_ms": ms_dom,
            "stage1_ms": ms1, "stage2_ms": ms2, "timed_launches": nl,
            "timing": "HIP start/stop events around every stage launch over K steps",
        },
        "event_timed_pass": {"value": cells * a.steps / el_events, "ms_per_step": el_events / a.steps * 1e3,
                             "note": "same K steps launched one by one with start/stop events per stage kernel"},
        "sim_time_s": t_sim,
        "state_finite": finite,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
