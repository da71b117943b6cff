"""Benchmark: SSP-RK2 steps of the eta-based central-upwind shallow-water
scheme on the NorKyst-shaped synthetic domain (2600 x 900 cells at 800 m,
~35 % land, nested M2-tide boundaries, linear drag, uniform wind stress,
latitude-dependent f), one MI355X.

One "step" = both stage kernels of one SSP-RK2 step over the whole domain,
with the time step computed on the device from the CFL condition.  Inputs are
resident in HBM before the timed region starts.  Prints ONE JSON line; beside
the headline figure it carries
  "ensemble": 256 coastal members (200..1000 x 200..600 cells) advanced by
              the persistent ensemble launch, against a per-domain loop;
  "serving":  the continuous-batching server on Poisson arrivals of forecast
              requests (time-scaled: horizons and inter-arrival times x0.1),
              with p50/p99 latency next to throughput;
  "preprocess": the device preprocessing of the same grid's cell depths
              (bathymetry reconstruction, land erosion, refinement).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-ensemble] [--no-serving]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# Algorithmic bytes per cell and stage launch: the per-cell figure of the
# scheme's two sweeps (state, corner depth and the Coriolis plane f that also
# carries the land mask; the north-angle plane is not read, the projection
# being an identity), counted for every cell of the domain:
#   float32 state (the paper's):
#     stage 1: read eta,hu,hv (12) + Hc (4) + f (4), write Q* (12)            = 32
#     stage 2: read Q* (12) + Q^n (12) + Hc (4) + f (4), write Q^n+1 (12)     = 44
#   compensated state (each stored value with its rounding error in 16 bits,
#   i.e. 18 B of state per cell):
#     stage 1: the above + read 3 error planes of Q^n (6), write 3 of Q* (6)  = 44
#     stage 2: the above + read 3 of Q* and 3 of Q^n (12), write 3 (6)        = 62
BYTES = {False: {1: 32, 2: 44}, True: {1: 44, 2: 62}}
# Secondary: the VALU issue rate.  Without packed FP32 (excluded by the build
# flags) the issue rate is 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12
# lane-instructions/s.
VALU_PEAK_TLANE = 256 * 4 * 16 * 2.4e9 / 1e12
TRAFFIC_FILES = {
    False: os.path.join(ROOT, "profiles", "traffic_stage_kernels_norkyst_2600x900.md"),
    True: os.path.join(ROOT, "profiles", "traffic_stage_kernels_compensated_norkyst_2600x900.md"),
}
KERNEL_SOURCE = os.path.join(ROOT, "paper_1912_02457_amd", "csrc", "swe_kernels.hip")
GRAPH_CHUNK = 16  # steps per captured graph (swe_step)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the oracle sample")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--ensemble-members", type=int, default=256)
    ap.add_argument("--ensemble-steps", type=int, default=500)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-max-active", type=int, default=128)
    ap.add_argument("--serve-steps-per-tick", type=int, default=24)
    ap.add_argument("--serve-rows", type=int, default=0, help="rows per tile of the server's ensemble (0 = default)")
    ap.add_argument("--serve-chunk", type=int, default=0, help="tiles per queue pop of the server's ensemble (0 = default)")
    ap.add_argument("--serve-unloaded-requests", type=int, default=150,
                    help="requests of the unloaded stream (0 = skip it)")
    ap.add_argument("--serve-unloaded-spread", type=float, default=8.0,
                    help="factor on the inter-arrival times of the unloaded stream")
    ap.add_argument("--serve-baseline-requests", type=int, default=60,
                    help="requests of the stream run one by one for the unbatched comparison")
    ap.add_argument("--serve-time-scale", type=float, default=0.1,
                    help="factor on horizons and inter-arrival times of the stand-in request stream")
    ap.add_argument("--serve-full", action="store_true",
                    help="serve the request stream as specified (2000 requests, 20/s, horizons 1-24 h) and a "
                         "second stream at --serve-rate-low requests/s")
    ap.add_argument("--serve-rate", type=float, default=20.0,
                    help="with --serve-full: arrival rate of the specified stream (requests/s)")
    ap.add_argument("--serve-rate-low", type=float, default=5.0)
    ap.add_argument("--serve-only", action="store_true", help="only the serving section (JSON with it alone)")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run warmup + this many steps (for rocprofv3 runs), no JSON")
    ap.add_argument("--no-preprocess", action="store_true")
    ap.add_argument("--no-full-length", action="store_true",
                    help="skip the full-step-count parity of configs 2 and 3 against the stored oracle results")
    ap.add_argument("--no-strip", action="store_true", help="skip the one-strip-of-8 measurement")
    ap.add_argument("--no-sweep", action="store_true", help="skip the domain-size sweep")
    ap.add_argument("--sweep-max", type=int, default=8192,
                    help="largest N of the N x N size sweep (powers of two from 512; 16384 needs ~30 GB of host memory)")
    ap.add_argument("--sweep-steps", type=int, default=100)
    ap.add_argument("--no-float32-state", action="store_true",
                    help="skip the measurement of the float32-state kernels")
    ap.add_argument("--count-tilings", action="store_true",
                    help="profiler run: 3 steps at every tiling the tuner may choose (no tuning, no timing)")
    ap.add_argument("--profile-workload", default="config2",
                    help="with --profile-steps / --count-tilings: config2 (default) or convN, the grid-convergence "
                         "case at N x N")
    ap.add_argument("--float32-state", action="store_true",
                    help="with --profile-steps / --count-tilings: the float32-state kernels instead of the "
                         "compensated ones")
    ap.add_argument("--preprocess-only", action="store_true",
                    help="only the device preprocessing section (for profiler runs)")
    ap.add_argument("--preprocess-reps", type=int, default=50)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="with --profile-steps: also run a plain 256 MiB device copy (counter calibration)")
    return ap.parse_args()


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_sample(o, st0, target_s, max_steps):
    """Steps of the oracle from st0 until target_s of wall time has passed
    (one step at a least); returns (steps, seconds, state, t)."""
    st, t, steps = st0, 0.0, 0
    t0 = time.perf_counter()
    while True:
        st, t, _, k = o.run(st, t, nsteps=1, record_dt=False)
        steps += k
        el = time.perf_counter() - t0
        if el >= target_s or steps >= max_steps:
            return steps, el, st, t


def cpu_baseline(wl, target_s):
    """The FP64 oracle as it is, on this host's cores, over a bounded number
    of steps of the same workload: once with every thread the OpenMP runtime
    offers and once with one thread."""
    from oracle import oracle as orc
    o = orc.Oracle(wl)
    st0 = o.initial_state()
    threads = orc.num_threads()
    steps, el, st, t = _oracle_sample(o, st0, target_s, 2000)
    orc.set_num_threads(1)
    steps1, el1, _, _ = _oracle_sample(o, st0, target_s / 2, 2000)
    orc.set_num_threads(threads)
    cells = wl.nx * wl.ny
    return {
        "value": cells * steps / el,
        "unit": "cell-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {steps} steps of the same {wl.nx}x{wl.ny} workload, FP64 C oracle, {threads} "
                  f"threads, {el:.1f} s wall; 1 thread: first {steps1} steps, {el1:.1f} s",
        "value_1thread": cells * steps1 / el1,
        "nproc": os.cpu_count(),
        "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
        "cpu_model": _cpu_model(),
    }, st, t, steps


def error_vs_oracle(wl, ref, t_ref, steps, np, compensated=False):
    """The HIP path over the oracle sample's steps (its own CFL dt), compared
    element by element with the FP64 oracle: relative L2 and Linf per field,
    eta by its own norm, hu and hv by the norm of the momentum magnitude,
    land cells excluded."""
    from paper_1912_02457_amd import Domain
    dom = Domain.from_workload(wl, device="cuda:0", compensated_state=compensated)
    dom.autotune()  # the tilings the timed region uses
    dom.step(steps)
    e, u, v, t, _ = dom.read_state()
    dom.close()
    m = np.ones((wl.ny, wl.nx), bool) if wl.land is None else (np.asarray(wl.land) == 0)
    re, ru, rv = (np.asarray(x, np.float64)[m] for x in ref)
    ge, gu, gv = (np.asarray(x, np.float64)[m] for x in (e, u, v))
    mom = np.sqrt(ru ** 2 + rv ** 2)
    out = {"steps": steps, "t_s": t, "t_oracle_s": t_ref}
    for name, g, r, n2, ni in (("eta", ge, re, np.linalg.norm(re), np.abs(re).max()),
                               ("hu", gu, ru, np.linalg.norm(mom), mom.max()),
                               ("hv", gv, rv, np.linalg.norm(mom), mom.max())):
        out[f"{name}_rel_l2"] = float(np.linalg.norm(g - r) / max(n2, 1e-30))
        out[f"{name}_rel_linf"] = float(np.abs(g - r).max() / max(ni, 1e-30))
    out["note"] = ("same steps as the cpu_baseline sample; each configuration's full step count is "
                   "compared with stored oracle results in tests/test_gpu_full_length.py")
    return out


def measured_traffic(comp: bool, kernel: str, rows: int, tail_rpw: int = 0, tail_rows: int = 0, order: int = 0):
    """HBM bytes per launch of ``kernel`` (stage1 / stage2, of the float32 or
    the compensated state) under a tiling (rows per tile, the tail's rows
    per tile and rows, tile order) from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (scaled by the copy-kernel calibration), or None when
    that tiling was not counted or the kernel source changed since."""
    path = TRAFFIC_FILES[comp]
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    src = hashlib.sha1(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if vals.get("kernel_source_sha1") != src:
        return None
    # "- stage2_rows7_order1: one 122.8; 1x74 120.8; ..." (MB per launch)
    want = f"{tail_rpw}x{tail_rows}" if tail_rpw else "one"
    for item in vals.get(f"{kernel}_rows{rows}_order{order}", "").split(";"):
        parts = item.split()
        if len(parts) == 2 and parts[0] == want:
            return float(parts[1]) * 1e6
    return None


def _copy_calibration(a, torch):
    """Three device-to-device copies of 256 MiB: the reference a profiler's
    HBM byte counters are scaled by."""
    if not a.copy_calibration:
        return
    x = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()


def warm_graphs(dom, warmup, k):
    """Untimed: `warmup` steps, then the timed step count once at the parity
    the timed region starts at (twice when k is odd: the second call runs at
    the other parity and returns to the first), so that every graph the timed
    call replays -- the 16-step chunks and the k mod 16 remainder -- is
    captured and instantiated before the clock starts."""
    dom.step(warmup)
    dom.step(k)
    if k % 2:
        dom.step(k)


def valu_counted(comp: bool, kernel: str):
    """VALU lane-instructions per cell of one launch (SQ_INSTS_VALU x 64 /
    cells) from the committed counter run, or None if the kernels changed."""
    path = TRAFFIC_FILES[comp]
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha1") != hashlib.sha1(open(KERNEL_SOURCE, "rb").read()).hexdigest():
        return None
    v = vals.get(f"{kernel}_valu_lane_instr_per_cell")
    return None if v is None else float(v)


def time_domain(a, np, torch, wl, comp):
    """Tiling measured first (swe_autotune_tiling), graphs warmed, then the
    timed region: exactly a.steps SSP-RK2 steps through the captured graphs
    between device synchronisations (HIP events on the domain's stream around
    it as well); then a second pass launched step by step with HIP start/stop
    events around every stage kernel, the per-kernel durations."""
    from paper_1912_02457_amd import Domain
    dom = Domain.from_workload(wl, device="cuda:0", compensated_state=comp)
    dom.autotune()  # measured tiling (does not advance the simulation)
    til = [dom.stage_tiling(1), dom.stage_tiling(2)]
    warm_graphs(dom, a.warmup, a.steps)
    st = dom.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(st)
    dom.step(a.steps)
    ev1.record(st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    n_ev = max(a.steps, 100)
    dom.enable_timing(True)
    dom.stage_times(reset=True)
    dom.step(n_ev)
    ms1, ms2, nl = dom.stage_times(reset=True)
    dom.enable_timing(False)
    e, u, v, t_sim, dt_next = dom.read_state()
    finite = bool(np.isfinite(e).all() and np.isfinite(u).all() and np.isfinite(v).all())
    dom.close()
    return {"el": el, "gpu_ms": gpu_ms, "ms1": ms1, "ms2": ms2, "launches": nl, "tiling": til,
            "t_sim": t_sim, "dt_next": dt_next, "finite": finite}


def roofline_of(wl, comp, r):
    """HBM roofline of the dominant stage kernel of one timed domain."""
    cells = wl.nx * wl.ny
    dominant = 2 if r["ms2"] >= r["ms1"] else 1
    ms = r["ms2"] if dominant == 2 else r["ms1"]
    til = r["tiling"][dominant - 1]
    bpl = BYTES[comp][dominant] * cells
    gbs = bpl / (ms * 1e-3) / 1e9
    traffic = measured_traffic(comp, f"stage{dominant}", *til[:4])
    vpc = valu_counted(comp, f"stage{dominant}")
    out = {
        "bound": "hbm",
        "kernel": f"stage_kernel<{dominant}>" + (" (compensated state)" if comp else " (float32 state)"),
        "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
        "traffic": traffic,
        "bytes_per_cell": BYTES[comp][dominant], "cells": cells, "algorithmic_bytes_per_launch": bpl,
        "avg_launch_ms": ms, "stage1_ms": r["ms1"], "stage2_ms": r["ms2"], "timed_launches": r["launches"],
        "timing": "HIP start/stop events around every stage launch (hipExtLaunchKernelGGL on the domain's stream)",
        "traffic_frac": None if traffic is None else traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "valu": None if vpc is None else {
            "lane_instr_per_cell": vpc, "peak_T_lane_instr_per_s": VALU_PEAK_TLANE,
            "frac": vpc * cells / (ms * 1e-3) / 1e12 / VALU_PEAK_TLANE,
            "source": "SQ_INSTS_VALU x 64 / cells of a counter run of the same kernels (profiles/)"},
    }
    if comp:
        # the same duration against the float32-state bytes (the paper's state)
        out["frac_at_float32_state_bytes"] = BYTES[False][dominant] * cells / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    return out


def bench_single(a, np, torch):
    from paper_1912_02457_amd import Domain
    from workloads import config2

    if a.count_tilings or a.profile_steps:
        if a.profile_workload.startswith("conv"):
            from workloads import convergence_case
            wl = convergence_case(int(a.profile_workload[4:]))
        else:
            wl = config2()
        comp = not a.float32_state
        dom = Domain.from_workload(wl, device="cuda:0", compensated_state=comp)
        if a.count_tilings:
            # every tiling the tuner may settle on, in each of the four tile
            # orders, 3 steps each: order o, list entry i ran as stage k's
            # dispatches 3 (o n + i) .. +2, with n the longer list (the
            # shorter one repeats its last entry)
            l1, l2 = dom.list_tilings(1), dom.list_tilings(2)
            n = max(len(l1), len(l2))
            for order in range(4):
                for i in range(n):
                    dom.set_stage_tiling(1, *l1[min(i, len(l1) - 1)], order)
                    dom.set_stage_tiling(2, *l2[min(i, len(l2) - 1)], order)
                    dom.step(3)
            torch.cuda.synchronize()
            _copy_calibration(a, torch)
            dom.close()
            print(json.dumps({"counted_tilings": [l1, l2], "orders": 4, "steps_per_tiling": 3, "compensated": comp}),
                  flush=True)
            return None, wl
        dom.autotune()
        warm_graphs(dom, a.warmup, a.profile_steps)
        torch.cuda.synchronize()
        dom.step(a.profile_steps)
        torch.cuda.synchronize()
        _copy_calibration(a, torch)
        print(json.dumps({"profiled_steps": a.profile_steps, "compensated": comp, "workload": a.profile_workload,
                          "stage_tiling": [dom.stage_tiling(1), dom.stage_tiling(2)]}), flush=True)
        dom.close()
        return None, wl

    wl = config2()
    cells = wl.nx * wl.ny
    land_cells = int(np.count_nonzero(wl.land)) if wl.land is not None else 0
    r = time_domain(a, np, torch, wl, True)
    value = cells * a.steps / r["el"]
    (rw1, trw1, tr1, ord1, wv1), (rw2, trw2, tr2, ord2, wv2) = r["tiling"]
    out = {
        "metric": "cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["el"] / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "norkyst_2600x900_800m_nested_m2_tide",
            "nx": wl.nx, "ny": wl.ny, "dx_m": wl.dx, "cells": cells, "land_fraction": land_cells / cells,
            "boundaries": "nested (M2 tide, hourly snapshots) on all sides", "friction": "linear r=3e-3 m/s",
            "wind_stress_Nm2": 0.1, "courant": wl.courant, "dt_s": r["dt_next"],
            "state": "compensated (float32 value + its rounding error kept to 16 bits, per field); float32 arithmetic",
            "rows_per_wave": [rw1, rw2], "tail_rows_per_wave": [trw1, trw2], "tail_rows": [tr1, tr2],
            "tile_order": [ord1, ord2], "waves_per_stage": [wv1, wv2],
            "tiling": "measured per stage kernel before the timed region (swe_autotune_tiling)",
            "timed_region": f"{a.steps} steps through captured HIP graphs, every graph captured in the "
                            f"untimed warm-up; device synchronisation on both sides",
        },
        "roofline": roofline_of(wl, True, r),
        "gpu_ms_per_step": r["gpu_ms"] / a.steps,
        "stage_kernels_ms_per_step": r["ms1"] + r["ms2"],
        "sim_time_s": r["t_sim"],
        "state_finite": r["finite"],
    }
    return out, wl


def bench_float32_state(a, np, torch, wl, full_value):
    """The same workload and timed region with the paper's float32 state:
    faster, but over this configuration's hour of simulated time its storage
    rounding alone moves the result past the 5e-4 relative Linf bar, so it is
    not the headline."""
    r = time_domain(a, np, torch, wl, False)
    cells = wl.nx * wl.ny
    v = cells * a.steps / r["el"]
    return {"value": v, "unit": "cell-updates/s", "ms_per_step": r["el"] / a.steps * 1e3, "steps": a.steps,
            "gpu_ms_per_step": r["gpu_ms"] / a.steps, "stage1_ms": r["ms1"], "stage2_ms": r["ms2"],
            "rows_per_wave": [t[:3] for t in r["tiling"]], "tile_order": [t[3] for t in r["tiling"]],
            "rate_vs_headline": v / full_value,
            "roofline": roofline_of(wl, False, r),
            "note": "same workload and timed region as the headline, compensated_state=0"}


def bench_strip(a, np, torch, wl, full_value):
    """One GPU's share of the headline domain if it were split into 8 row
    strips: 2600 x 117 cells (900/8 rows plus the 4 halo rows a stage reads),
    cut from the same fields, walls on all sides (the exchange with the
    neighbouring strips is not modelled).  Shows how far below the whole
    domain's rate a strip runs on its own."""
    from paper_1912_02457_amd import Domain
    from workloads import BC_WALL
    ny = 900 // 8 + 4
    sw = wl.copy(ny=ny, Hc=wl.Hc[:ny + 1], land=None if wl.land is None else wl.land[:ny], f=wl.f[:ny],
                 north=None if wl.north is None else wl.north[:ny], eta=wl.eta[:ny], hu=wl.hu[:ny],
                 hv=wl.hv[:ny], bc=(BC_WALL,) * 4, bnd=None, bnd_t=None)
    dom = Domain.from_workload(sw, device="cuda:0")
    dom.autotune()
    n = 2000
    warm_graphs(dom, 100, n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dom.step(n)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dom.enable_timing(True)
    dom.stage_times(reset=True)
    dom.step(500)
    ms1, ms2, _ = dom.stage_times(reset=True)
    dom.close()
    v = sw.nx * sw.ny * n / el
    return {"shape": [sw.nx, sw.ny], "value": v, "unit": "cell-updates/s", "ms_per_step": el / n * 1e3,
            "stage1_ms": ms1, "stage2_ms": ms2, "rate_vs_whole_domain": v / full_value,
            "note": "one of 8 row strips of the headline domain with its halo rows, walls, no exchange"}


# Total simulation times of the grid-convergence benchmark on a Tesla P100,
# from the appendix table of timings (N x N cells, 1600 simulated seconds at
# dt = 1600/N s, i.e. N steps): context for the size sweep, other hardware.
PAPER_P100_TOTAL_S = {512: 0.169710, 1024: 1.170814, 2048: 9.133564, 4096: 72.832028,
                      8192: 582.599290, 16384: 4695.904546}
# ... and the time to download the state (eta, hu, hv) to the host, same table
PAPER_P100_DOWNLOAD_S = {512: 0.000929, 1024: 0.002773, 2048: 0.019642, 4096: 0.077541,
                         8192: 0.305405, 16384: 1.218880}


def bench_sweep(a, np, torch):
    """The paper's own benchmark shape: the grid-convergence case (peaks
    bathymetry, cosine bump, latitude and north angle from a pole, walls) at
    N x N for N = 512 .. sweep_max, for each state kind: tiling measured,
    graphs warmed, sweep_steps timed steps through the captured graphs, then
    the stage kernels event-timed.  Per size: cell-updates/s, stage kernel
    durations, algorithmic HBM fraction of each, and the time the paper's run
    (N steps) would take at this rate next to the P100's."""
    from paper_1912_02457_amd import Domain
    from workloads import convergence_case
    out = []
    N = 512
    while N <= a.sweep_max:
        t_gen = time.perf_counter()
        wl = convergence_case(N)
        t_gen = time.perf_counter() - t_gen
        cells = N * N
        row = {"n": N, "cells": cells, "input_generation_s": t_gen}
        for comp in (True, False):
            dom = Domain.from_workload(wl, device="cuda:0", compensated_state=comp)
            dom.autotune()
            warm_graphs(dom, 20, a.sweep_steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dom.step(a.sweep_steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            dom.enable_timing(True)
            dom.stage_times(reset=True)
            dom.step(a.sweep_steps)
            ms1, ms2, _ = dom.stage_times(reset=True)
            rows = [dom.stage_tiling(1)[:4], dom.stage_tiling(2)[:4]]
            rec = {}
            if comp:
                # state download into pinned host memory (the paper's download time)
                host = [torch.empty((N, N), dtype=torch.float32, pin_memory=True) for _ in range(3)]
                dl = []
                for _ in range(3):
                    t1 = time.perf_counter()
                    dom.read_state_into(*host)
                    dl.append(time.perf_counter() - t1)
                rec["state_finite"] = bool(torch.isfinite(host[0]).all())
                rec.update({"download_s": min(dl), "download_gb_s": 12.0 * cells / min(dl) / 1e9,
                            "paper_p100_download_s": PAPER_P100_DOWNLOAD_S.get(N)})
                del host
            dom.close()
            v = cells * a.sweep_steps / el
            b1, b2 = BYTES[comp][1] * cells, BYTES[comp][2] * cells
            rec.update({"value": v, "ms_per_step": el / a.sweep_steps * 1e3, "stage1_ms": ms1, "stage2_ms": ms2,
                        "rows_per_wave": rows,
                        "hbm_frac_stage1": b1 / (ms1 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "hbm_frac_stage2": b2 / (ms2 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "hbm_frac_step": (b1 + b2) / ((ms1 + ms2) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "paper_run_s": N * el / a.sweep_steps})
            row["compensated" if comp else "float32_state"] = rec
        row["paper_p100_total_s"] = PAPER_P100_TOTAL_S.get(N)
        del wl
        out.append(row)
        _progress(f"sweep {N}^2: {row['compensated']['value']:.3e} (compensated), "
                  f"{row['float32_state']['value']:.3e} (float32 state) cell-updates/s")
        N *= 2
    return {"workload": "grid-convergence case (peaks bathymetry, cosine bump, pole latitude/north, walls), N x N",
            "steps": a.sweep_steps, "sizes": out,
            "bytes_per_cell": {"compensated": [BYTES[True][1], BYTES[True][2]],
                               "float32_state": [BYTES[False][1], BYTES[False][2]]},
            "note": "paper_run_s = N steps (1600 s at dt = 1600/N) at the measured rate; "
                    "paper_p100_total_s is the paper's Tesla P100 total (context, other hardware); "
                    "download_s = best of 3 copies of eta, hu, hv into pinned host memory (swe_read_state)"}


def full_length_parity(torch):
    """The benchmarked path over a configuration's full step count, each side
    with its own CFL dt every step, against the oracle's stored final state
    (tests/golden): config 2 (the NorKyst-sized hour, both state kinds) and
    config 3 (the wet-dry beach, 5000 steps).  The bar: 1e-4 relative L2 and
    5e-4 relative Linf per field; tests/test_gpu_full_length.py runs every
    configuration, also with the oracle's dt sequence."""
    from paper_1912_02457_amd import Domain
    gdir = os.path.join(ROOT, "tests", "golden")
    if gdir not in sys.path:
        sys.path.insert(0, gdir)
    import make_golden as MG
    out = {}
    for name, kinds in (("config2", (True, False)), ("config3", (True,))):
        g = golden_state(name)
        if g is None:
            continue
        ref, land = g
        wl = MG.workload(name)
        for comp in kinds:
            d = Domain.from_workload(wl, device="cuda:0", compensated_state=comp)
            if wl.t_end:
                k = d.run_until(wl.t_end)
            else:
                d.step(wl.steps)
                k = wl.steps
            st = d.read_state()
            d.close()
            w = worst([rel_errors(st, ref, land)])
            out[f"{name}_{'compensated' if comp else 'float32_state'}"] = {
                "steps": int(k), "t_s": float(st[3]), "l2": w["l2"], "linf": w["linf"],
                "meets_bar": bool(w["l2"] <= 1e-4 and w["linf"] <= 5e-4)}
    return out


def _member(k):
    from workloads import config4_member
    return config4_member(k)


def golden_state(name):
    """Final state of the FP64 oracle after a configuration's full step count,
    stored by tests/golden/make_golden.py (which calls only the oracle):
    (eta, hu, hv) on the full grid, or None without the fixture."""
    import numpy as np
    gdir = os.path.join(ROOT, "tests", "golden")
    path = os.path.join(gdir, f"{name}.npz")
    if not os.path.exists(path):
        return None
    if gdir not in sys.path:
        sys.path.insert(0, gdir)
    import make_golden as MG
    z = np.load(path)
    wl = MG.workload(name)
    wet = np.ones((wl.ny, wl.nx), bool) if wl.land is None else (np.asarray(wl.land) == 0)
    out = []
    for f in ("eta", "hu", "hv"):
        arr = np.zeros((wl.ny, wl.nx))
        arr[wet] = MG.decode_field(z[f"{f}_z"], float(z[f"{f}_q"]), int(z["count"]))
        out.append(arr)
    return tuple(out), wl.land


def rel_errors(got, ref, land):
    """Relative L2 and Linf per field (eta by its own norm, hu and hv by the
    momentum magnitude; land excluded), as in the tests."""
    import numpy as np
    from tests._parity import parity
    return {k: float(v) for k, v in parity(got, ref, land).items()}


def worst(errs):
    return {"l2": max(max(e[k] for k in e if k.endswith("_l2")) for e in errs),
            "linf": max(max(e[k] for k in e if k.endswith("_linf")) for e in errs)}


def _member(k):
    from workloads import config4_member
    return config4_member(k)


def _ensemble_leg(wls, comp, S, torch):
    """One persistent ensemble of the members: tile shape from a short sweep,
    S steps from the initial state (the untimed warm-up, capturing every
    graph the timed call replays) after which members 0-7 are compared with
    the oracle's state at the same step, then S timed steps."""
    from paper_1912_02457_amd import Domain, Ensemble
    from paper_1912_02457_amd.tune import autotune_ensemble
    cells = sum(w.nx * w.ny for w in wls)
    probe = [Domain.from_workload(w, device="cuda:0", compensated_state=comp) for w in wls]
    rows, chunk, rep = autotune_ensemble(probe, steps=16)
    for d in probe:
        d.close()
    del probe
    doms = [Domain.from_workload(w, device="cuda:0", compensated_state=comp) for w in wls]
    torch.cuda.synchronize()
    ens = Ensemble(doms, rows_per_wave=rows, chunk=chunk)
    info = ens.info()
    ens.step(S)  # untimed: S steps from the initial state, graphs captured
    errs = []
    for k in range(min(8, len(doms))):
        g = golden_state(f"config4_m{k}") if S == 500 else None
        if g is not None:
            e, u, v, t, _ = doms[k].read_state()
            errs.append(rel_errors((e, u, v), g[0], g[1]))
    if S % 2:
        ens.step(S)  # the graphs of the other step parity, where the timed call starts
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(S)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ens.enable_timing(True)
    ens.stage_times()
    ens.step(32)
    ms1, ms2, _ = ens.stage_times()
    ens.close()
    # the plain alternative: the same members stepped one domain at a time
    # (each through its own captured graphs)
    L = 64
    for d in doms:
        d.step(16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in doms:
        d.step(L)
    torch.cuda.synchronize()
    el_loop = time.perf_counter() - t0
    for d in doms:
        d.close()
    value, loop = cells * S / el, cells * L / el_loop
    return {"value": value, "unit": "cell-updates/s", "ms_per_step": el / S * 1e3, "rows_per_wave": rows,
            "chunk": chunk, "work_items": info[2], "blocks": info[3], "stage1_ms": ms1, "stage2_ms": ms2,
            "per_domain_loop_value": loop, "speedup_vs_loop": value / loop,
            "error_vs_fp64": {"members": len(errs), "steps": S, "worst": worst(errs) if errs else None,
                              "per_member": errs},
            "autotune": {k: v for k, v in rep.items() if k != "trials"}}


def bench_ensemble(a, torch):
    """256-member ensemble (coastal 1 km domains, walls, per-member wind),
    each member with its own dt: aggregate cell-updates/s of the persistent
    ensemble launch (autotuned tiles, graph replay) against stepping the same
    domains one after the other, for the float32 state (inside the parity
    bar over the 500 steps: members 0-7 are compared with the oracle) and
    the compensated state."""
    from concurrent.futures import ProcessPoolExecutor
    n = a.ensemble_members
    with ProcessPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        wls = list(ex.map(_member, range(n), chunksize=4))
    cells = sum(w.nx * w.ny for w in wls)
    S = a.ensemble_steps
    f32 = _ensemble_leg(wls, False, S, torch)
    comp = _ensemble_leg(wls, True, S, torch)
    out = {"metric": "ensemble aggregate cell-updates/s", "state": "float32 (meets the parity bar at 500 steps)",
           "workload": f"{n} coastal members 200..1000 x 200..600 cells at 1 km, walls, f=1.2e-4, "
                       "per-member wind, own dt each",
           "members": n, "cells": cells, "steps": S}
    out.update(f32)
    out["compensated_state"] = comp
    return out


def bench_serving(a, torch):
    """Continuous batching of forecast requests (flat 100 m, walls,
    f = 1.2e-4, Gaussian bump; sizes 100..2000 x 100..800) arriving as a
    Poisson stream, compensated state.  By default a stand-in that fits the
    benchmark's time: horizons and inter-arrival times scaled by
    ``serve_time_scale`` (same offered load, 1000 requests); --serve-full
    runs the stream as specified (2000 requests, 20/s, horizons 1-24 h) and
    a second stream at --serve-rate-low requests/s.  Latency = completion
    minus arrival, wall clock.  Error vs FP64: the first six requests with
    their horizon capped at 2 h, served in a mix of 24 such requests,
    against the oracle's results."""
    import numpy as np
    from workloads import config5_requests

    out = {}
    if a.serve_full:
        reqs = config5_requests(rate=a.serve_rate)
        arrivals = np.array([r["arrival"] for r in reqs])
        horizons = [r["horizon"] for r in reqs]
        out = _serve_stream(a, torch, reqs, arrivals, horizons, scale=1.0)
        out["stream"] = f"as specified: 2000 requests, Poisson {a.serve_rate:g}/s, horizons U[1, 24] h"
        if a.serve_baseline_requests > 0:
            out["one_by_one"] = serve_one_by_one(reqs[:a.serve_baseline_requests], horizons, torch)
        if a.serve_rate_low > 0:
            low = config5_requests(rate=a.serve_rate_low)
            arr_low = np.array([r["arrival"] for r in low])
            u = _serve_stream(a, torch, low, arr_low, [r["horizon"] for r in low], scale=1.0)
            out["low_rate"] = {k: u[k] for k in ("workload", "requests", "completed_ok", "latency_s",
                                                 "offered_cell_steps_per_s", "value", "mean_active", "span_s")}
    else:
        sc = a.serve_time_scale
        reqs = config5_requests()[: a.serve_requests]
        arrivals = np.array([r["arrival"] for r in reqs]) * sc
        horizons = [r["horizon"] * sc for r in reqs]
        out = _serve_stream(a, torch, reqs, arrivals, horizons, scale=sc)
        out["stream"] = (f"stand-in for the specified stream: {len(reqs)} requests, horizons and inter-arrival "
                         f"times x {sc} (same offered load), so that it fits the benchmark's run time")
        if a.serve_baseline_requests > 0:
            out["one_by_one"] = serve_one_by_one(reqs[:a.serve_baseline_requests], horizons, torch)
        if a.serve_unloaded_requests > 0:
            n = a.serve_unloaded_requests
            u = _serve_stream(a, torch, reqs[:n], arrivals[:n] * a.serve_unloaded_spread, horizons[:n], scale=sc)
            out["unloaded"] = {k: u[k] for k in ("workload", "requests", "completed_ok", "latency_s",
                                                 "offered_cell_steps_per_s", "value", "mean_active")}
    out["error_vs_fp64"] = serve_error_vs_fp64(a, torch)
    return out


def serve_error_vs_fp64(a, torch):
    """The first six requests of the stream, horizon capped at 2 h, served
    together with 18 more capped requests through one server; each result
    against the oracle's (tests/golden/config5_r<k>)."""
    from paper_1912_02457_amd import Server
    from workloads import config5_requests
    from workloads.configs import config5_member
    reqs = config5_requests()[:24]
    cap = 7200.0
    errs = []
    with Server(16 << 30, max_active=a.serve_max_active, steps_per_tick=a.serve_steps_per_tick,
                device="cuda:0") as srv:
        for k, r in enumerate(reqs):
            srv.submit(config5_member(r["nx"], r["ny"], 0.0), min(r["horizon"], cap), req_id=k, keep_result=k < 6)
        done = {}
        while len(done) < len(reqs):
            srv.tick()
            for c in srv.poll():
                done[c["id"]] = c
    for k in range(6):
        g = golden_state(f"config5_r{k}")
        c = done[k]
        if g is not None and c["status"] == 0:
            e = rel_errors(c["state"], g[0], g[1])
            e["steps"] = int(c["steps"])
            errs.append(e)
    return {"requests": len(errs), "horizon_s": cap, "mix": len(reqs), "worst": worst(errs) if errs else None,
            "per_request": errs}


def _serve_stream(a, torch, reqs, arrivals, horizons, scale):
    """One request stream through a fresh server; throughput, latency and
    server counters."""
    from collections import deque
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    from paper_1912_02457_amd import Server
    from workloads.configs import config5_member

    sc = scale
    srv = Server(48 << 30, max_active=a.serve_max_active, steps_per_tick=a.serve_steps_per_tick,
                 rows_per_wave=a.serve_rows, chunk=a.serve_chunk, device="cuda:0")
    done_at = {}
    submitted = threading.Event()
    errors = []

    def feeder():
        try:
            with ThreadPoolExecutor(6) as ex:
                window = deque()
                nxt = 0
                for k in range(len(reqs)):
                    while nxt < len(reqs) and len(window) < 24:
                        r = reqs[nxt]
                        window.append(ex.submit(config5_member, r["nx"], r["ny"], 0.0))
                        nxt += 1
                    wl = window.popleft().result()
                    wait = t0 + arrivals[k] - time.perf_counter()
                    if wait > 0:
                        time.sleep(wait)
                    srv.submit(wl, horizons[k], req_id=k, keep_result=False)
        except Exception as exc:  # surfaced by the main thread
            errors.append(exc)
        finally:
            submitted.set()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = threading.Thread(target=feeder, daemon=True)
    th.start()
    busy_s = 0.0  # wall time of ticks that had requests resident
    active_time = 0.0  # integral of the active count over time
    sat_s, sat_cells = 0.0, 0  # ticks that ran with requests still waiting
    last = t0
    last_note = t0
    last_cells = 0
    while True:
        act, pend = srv.tick()
        now = time.perf_counter()
        cells_now = srv.stats()["cell_steps"]
        if act:
            busy_s += now - last
            active_time += act * (now - last)
        if pend:
            sat_s += now - last
            sat_cells += cells_now - last_cells
        last, last_cells = now, cells_now
        for c in srv.poll():
            done_at[c["id"]] = (now, c["status"], c["steps"])
        if now - last_note > 30.0:
            last_note = now
            _progress(f"serving: {len(done_at)}/{len(reqs)} requests done, {act} active, {pend} waiting")
        if submitted.is_set() and act == 0 and pend == 0:
            break
        if act == 0 and pend == 0:
            time.sleep(2e-4)
            last = time.perf_counter()
    th.join()
    if errors:
        raise errors[0]
    t_end = time.perf_counter()
    st = srv.stats()
    srv.close()
    lat = np.array([done_at[k][0] - (t0 + arrivals[k]) for k in range(len(reqs))])
    ok = sum(1 for v in done_at.values() if v[1] == 0)
    cell_steps = st["cell_steps"]
    span = t_end - t0
    offered = sum(r["nx"] * r["ny"] * np.ceil(h / 3.59) for r, h in zip(reqs, horizons))
    return {
        "metric": "served cell-updates/s",
        "value": cell_steps / span,
        "unit": "cell-updates/s",
        "workload": f"{len(reqs)} forecast requests, Poisson arrivals at "
                    f"{(len(reqs) - 1) / max(arrivals[-1] - arrivals[0], 1e-9):.0f}/s, "
                    f"nx 100..2000 x ny 100..800 at 1 km, horizons U[1,24] h x {sc}",
        "requests": len(reqs), "completed_ok": ok, "time_scale": sc,
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max()), "mean": float(lat.mean())},
        "offered_cell_steps_per_s": float(offered / (arrivals[-1] - arrivals[0] + 1e-9)),
        "saturated_value": sat_cells / sat_s if sat_s > 0 else None,
        "saturated_s": sat_s,
        "span_s": span, "busy_s": busy_s, "mean_active": active_time / max(busy_s, 1e-9),
        "ticks": st["ticks"], "steps_per_tick": a.serve_steps_per_tick, "max_active": a.serve_max_active,
        "rows_per_wave": a.serve_rows, "chunk": a.serve_chunk,
        "arena_peak_GiB": st["arena_peak"] / 2**30,
        "host_s": {k[5:-2]: round(st[k], 3) for k in st if k.startswith("host_")},
    }


def serve_one_by_one(reqs, horizons, torch):
    """The plain alternative to batching: the same requests run one after the
    other, each alone on the GPU (its own domain, run_until its horizon).
    Inputs are built before the clock starts; cell-updates/s over the run."""
    from paper_1912_02457_amd import Domain
    from workloads.configs import config5_member
    wls = [config5_member(r["nx"], r["ny"], 0.0) for r in reqs]
    cells = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for wl, h in zip(wls, horizons):
        d = Domain.from_workload(wl, device="cuda:0")
        k = d.run_until(h)
        cells += wl.nx * wl.ny * k
        d.close()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"requests": len(wls), "value": cells / el, "unit": "cell-updates/s",
            "note": "first requests of the same stream, each run alone in arrival order (init and run_until)"}


PRE_SOURCE = os.path.join(ROOT, "paper_1912_02457_amd", "csrc", "swe_preprocess.hip")
PRE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_recon_round_kernel_norkyst_2600x900.md")


def measured_pre_traffic():
    """HBM bytes per launch of the reconstruction round kernel from the
    committed FETCH_SIZE / WRITE_SIZE runs, or None if the source changed."""
    if not os.path.exists(PRE_TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(PRE_TRAFFIC_FILE):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha1") != hashlib.sha1(open(PRE_SOURCE, "rb").read()).hexdigest():
        return None
    v = vals.get("recon_round_hbm_bytes_per_launch")
    return None if v is None else float(v)


def bench_preprocess(a, np, torch):
    """Device preprocessing of the 2600 x 900 coastal grid (the cell depths
    and land mask behind the headline domain): bathymetry reconstruction
    (10 rounds), one land erosion, factor-two refinement of (eta, hu, hv),
    land and corners.  Each operation is captured once in a HIP graph and
    replayed; HIP events on the replay stream time the replays.  The round
    kernel's average duration = (time of 10-round calls - time of 0-round
    calls) / 10."""
    from paper_1912_02457_amd import swe
    from workloads import coastal_cells

    nx, ny = 2600, 900
    Hm_np, land_np = coastal_cells(nx, ny, 2, 3)
    dev = torch.device("cuda:0")
    Hm = torch.from_numpy(Hm_np.astype(np.float32)).to(dev)
    land = torch.from_numpy(land_np.astype(np.uint8)).to(dev)
    state = torch.zeros((3, ny, nx), dtype=torch.float32, device=dev)
    Hc = torch.empty((ny + 1, nx + 1), dtype=torch.float32, device=dev)
    scratch = torch.empty_like(Hc)
    side = torch.cuda.Stream(dev)

    ops = {
        "recon10": lambda: swe.reconstruct_bathymetry(Hm, land, iters=10, out=Hc, scratch=scratch),
        "recon0": lambda: swe.reconstruct_bathymetry(Hm, land, iters=0, out=Hc, scratch=scratch),
        "erode": lambda: swe.erode_land(land, Hm, state[0], state[1], state[2]),
        "refine": lambda: swe.refine2(state, land, Hc),
    }
    if a.preprocess_only and a.copy_calibration:
        x = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    reps = a.preprocess_reps
    ms = {}
    for name, fn in ops.items():
        with torch.cuda.stream(side):
            for _ in range(3):
                fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            fn()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            g.replay()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(side)
            for _ in range(reps):
                g.replay()
            e1.record(side)
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1) / reps
        del g
    # the same round kernel on an 8192 x 8192 grid (a smooth analytic
    # bottom with a land band; timing only), where the launch holds about
    # four times as many waves as are resident at once
    L_ = 8192
    yy, xx = torch.meshgrid(torch.arange(L_, device=dev, dtype=torch.float32),
                            torch.arange(L_, device=dev, dtype=torch.float32), indexing="ij")
    Hm_l = 200.0 + 150.0 * torch.sin(xx / 97.0) * torch.cos(yy / 131.0)
    land_l = ((torch.sin(xx / 611.0) + torch.cos(yy / 389.0)) > 1.2).to(torch.uint8)
    Hm_l = torch.where(land_l > 0, torch.full_like(Hm_l, -5.0), Hm_l).contiguous()
    del yy, xx
    Hc_l = torch.empty((L_ + 1, L_ + 1), dtype=torch.float32, device=dev)
    scratch_l = torch.empty_like(Hc_l)
    for name, it in (("large10", 10), ("large0", 0)):
        fn = (lambda it=it: swe.reconstruct_bathymetry(Hm_l, land_l, iters=it, out=Hc_l, scratch=scratch_l))
        with torch.cuda.stream(side):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(side)
            for _ in range(5):
                fn()
            e1.record(side)
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1) / 5
    del Hm_l, land_l, Hc_l, scratch_l
    CL, NL = (L_ + 1) ** 2, L_ * L_
    large_round_ms = (ms["large10"] - ms["large0"]) / 10.0
    large_gbs = (8 * CL + 5 * NL) / (large_round_ms * 1e-3) / 1e9

    C_, N_ = (ny + 1) * (nx + 1), nx * ny
    round_ms = (ms["recon10"] - ms["recon0"]) / 10.0
    round_bytes = 8 * C_ + 5 * N_          # corners in and out, cell depths, land flags
    gbs = round_bytes / (round_ms * 1e-3) / 1e9
    traffic = measured_pre_traffic()
    erode_bytes = 34 * N_
    refine_bytes = 13 * N_ + 4 * C_ + 52 * N_ + 4 * (2 * ny + 1) * (2 * nx + 1)
    return {
        "workload": "norkyst_2600x900 coastal cell depths + land (seeds 2, 3)",
        "reconstruct": {"ms_per_call": ms["recon10"], "rounds": 10, "init_ms": ms["recon0"],
                        "corner_rounds_per_s": C_ * 11 / (ms["recon10"] * 1e-3),
                        "roofline": {"bound": "hbm", "kernel": "recon_round_kernel<false>", "achieved": gbs,
                                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                                     "traffic": traffic, "avg_launch_ms": round_ms,
                                     "algorithmic_bytes_per_launch": round_bytes}},
        "reconstruct_8192x8192": {"ms_per_call": ms["large10"], "avg_round_ms": large_round_ms,
                                  "GBs": large_gbs, "frac": large_gbs / HBM_PEAK_GBS,
                                  "timing": "5 eager calls between HIP events"},
        "erode": {"ms_per_call": ms["erode"], "GBs": erode_bytes / (ms["erode"] * 1e-3) / 1e9},
        "refine": {"ms_per_call": ms["refine"], "fields": 3,
                   "GBs": refine_bytes / (ms["refine"] * 1e-3) / 1e9},
        "timing": f"HIP graph of each call replayed {reps}x between HIP events on the replay stream",
    }


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}); the shallow-water path here is a "
              "single-GPU build and no multi-GPU figure is produced", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if a.preprocess_only:
        print(json.dumps({"preprocess": bench_preprocess(a, np, torch)}), flush=True)
        return
    if a.serve_only:
        print(json.dumps({"serving": bench_serving(a, torch)}), flush=True)
        return
    out, wl = bench_single(a, np, torch)
    if out is None:
        return
    _progress(f"single domain: {out['value']:.3e} cell-updates/s")
    if not a.no_strip:
        out["strip_of_8"] = bench_strip(a, np, torch, wl, out["value"])
        _progress(f"strip: {out['strip_of_8']['value']:.3e} cell-updates/s")
    if not a.no_sweep:
        out["size_sweep"] = bench_sweep(a, np, torch)
    if not a.no_float32_state:
        out["float32_state"] = bench_float32_state(a, np, torch, wl, out["value"])
        _progress(f"float32 state: {out['float32_state']['value']:.3e} cell-updates/s")
    if not a.no_full_length:
        out["full_length_parity"] = full_length_parity(torch)
        _progress("full-length parity: " + ", ".join(f"{k} Linf {v['linf']:.1e}"
                                                      for k, v in out["full_length_parity"].items()))
    if not a.no_ensemble:
        out["ensemble"] = bench_ensemble(a, torch)
        _progress(f"ensemble: {out['ensemble']['value']:.3e} cell-updates/s")
    if not a.no_serving:
        out["serving"] = bench_serving(a, torch)
        _progress(f"serving: p50 {out['serving']['latency_s']['p50']:.3f} s")
    if not a.no_preprocess:
        out["preprocess"] = bench_preprocess(a, np, torch)
        _progress(f"preprocess: reconstruction {out['preprocess']['reconstruct']['ms_per_call']:.3f} ms")
    if not a.no_cpu_baseline:
        out["cpu_baseline"], ref, t_ref, steps = cpu_baseline(wl, a.cpu_seconds)
        _progress("cpu baseline done")
        out["error_vs_oracle"] = error_vs_oracle(wl, ref, t_ref, steps, np, compensated=True)
        out["error_vs_oracle_float32_state"] = error_vs_oracle(wl, ref, t_ref, steps, np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
