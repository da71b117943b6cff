"""Full-length parity report: the HIP path against the FP64 oracle after each
configuration's whole step count (not collected by pytest: too long for the
test suite).

    python tests/parity_report.py oracle CONFIG DIR   # CPU: FP64 oracle, own dt
    python tests/parity_report.py gpu CONFIG DIR      # GPU: own dt, and dt replay
                                                      #      if DIR has the oracle's dts
    python tests/parity_report.py gpucomp CONFIG DIR  # the same with the compensated state
    python tests/parity_report.py compare CONFIG DIR  # per-field relative L2 / Linf
    python tests/parity_report.py fp32state CONFIG DIR
        # the FP64 oracle with its state rounded to float32 after every step,
        # against DIR/CONFIG_oracle.npz: the deviation that storing the state
        # in float32 alone produces (a floor for any float32-state solver)

CONFIG is one of config1, config2, config3, config4_m<k> (ensemble member k),
config5_r<k> (served request k, horizon capped at 2 h).  The oracle writes
DIR/CONFIG_oracle.npz (final state in float64, the dt sequence, t); the GPU
run writes DIR/CONFIG_gpu_own.npz and DIR/CONFIG_gpu_replay.npz (float32).
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def workload(name):
    import workloads as W
    from workloads.configs import config5_member
    if name == "config1":
        return W.config1()
    if name == "config2":
        return W.config2()
    if name == "config3":
        return W.config3()
    if name.startswith("config4_m"):
        return W.config4_member(int(name[len("config4_m"):]))
    if name.startswith("config5_r"):
        k = int(name[len("config5_r"):])
        r = W.config5_requests()[k]
        return config5_member(r["nx"], r["ny"], min(r["horizon"], 7200.0))
    raise SystemExit(f"unknown config {name}")


def run_oracle(name, out):
    from oracle import oracle as orc
    wl = workload(name)
    o = orc.Oracle(wl)
    t0 = time.time()
    if wl.t_end:
        st, t, dts, k = o.run(nsteps=10 ** 7, t_end=wl.t_end)
    else:
        st, t, dts, k = o.run(nsteps=wl.steps)
    el = time.time() - t0
    np.savez(os.path.join(out, f"{name}_oracle.npz"), eta=st[0], hu=st[1], hv=st[2], dts=dts, t=t)
    print(json.dumps({"config": name, "oracle_steps": k, "t": t, "seconds": el,
                      "cell_updates_per_s": wl.nx * wl.ny * k / el, "threads": orc.num_threads()}), flush=True)


def run_gpu(name, out, comp=False):
    import torch
    from paper_1912_02457_amd import Domain
    torch.cuda.set_device(0)
    wl = workload(name)
    tag = "comp_" if comp else ""
    d = Domain.from_workload(wl, device="cuda:0", compensated_state=comp)
    t0 = time.time()
    if wl.t_end:
        k = d.run_until(wl.t_end)
    else:
        d.step(wl.steps)
        k = wl.steps
    e, u, v, t, _ = d.read_state()
    el = time.time() - t0
    d.close()
    np.savez_compressed(os.path.join(out, f"{name}_gpu_{tag}own.npz"), eta=e, hu=u, hv=v, t=t, steps=k)
    info = {"config": name, "gpu_steps": k, "t": t, "seconds": el}
    ref = os.path.join(out, f"{name}_oracle.npz")
    if os.path.exists(ref):
        dts = np.load(ref)["dts"]
        d = Domain.from_workload(wl, device="cuda:0", compensated_state=comp)
        d.step_dt(dts)
        e, u, v, t, _ = d.read_state()
        d.close()
        np.savez_compressed(os.path.join(out, f"{name}_gpu_{tag}replay.npz"), eta=e, hu=u, hv=v, t=t)
        info["replay_steps"] = len(dts)
    print(json.dumps(info), flush=True)


def compare(name, out):
    from tests._parity import parity
    wl = workload(name)
    ref = np.load(os.path.join(out, f"{name}_oracle.npz"))
    refst = (ref["eta"], ref["hu"], ref["hv"])
    res = {"config": name, "oracle_t": float(ref["t"]), "steps": int(len(ref["dts"]))}
    for mode in ("own", "replay", "comp_own", "comp_replay"):
        p = os.path.join(out, f"{name}_gpu_{mode}.npz")
        if os.path.exists(p):
            g = np.load(p)
            res[mode] = {k: float(v) for k, v in parity((g["eta"], g["hu"], g["hv"]), refst, wl.land).items()}
            res[mode]["t"] = float(g["t"])
    print(json.dumps(res), flush=True)
    return res


def run_fp32state(name, out):
    from oracle import oracle as orc
    from tests._parity import parity
    wl = workload(name)
    o = orc.Oracle(wl)
    st = o.initial_state()
    t, k = 0.0, 0
    t0 = time.time()
    while (t < wl.t_end) if wl.t_end else (k < wl.steps):
        st, t, _, n = o.run(st, t, nsteps=1, t_end=wl.t_end or 0.0, record_dt=False)
        st = tuple(np.asarray(a, np.float32).astype(np.float64) for a in st)
        k += n
    ref = np.load(os.path.join(out, f"{name}_oracle.npz"))
    np.savez_compressed(os.path.join(out, f"{name}_fp32state.npz"), eta=st[0], hu=st[1], hv=st[2], t=t)
    p = parity(st, (ref["eta"], ref["hu"], ref["hv"]), wl.land)
    print(json.dumps({"config": name, "steps": k, "t": t, "fp32_state_vs_fp64": {a: float(b) for a, b in p.items()},
                      "seconds": time.time() - t0}), flush=True)


if __name__ == "__main__":
    mode, name, out = sys.argv[1], sys.argv[2], sys.argv[3]
    os.makedirs(out, exist_ok=True)
    {"oracle": run_oracle, "gpu": run_gpu, "gpucomp": lambda n, o: run_gpu(n, o, comp=True), "compare": compare,
     "fp32state": run_fp32state}[mode](name, out)
