"""Writes the full-length parity fixtures of tests/golden/ from the FP64 oracle.

Every stored value here comes from ``oracle/`` alone (the inputs from the
seeded generators of ``workloads/``); nothing is taken from the HIP path.

For each configuration the oracle runs the whole step count of the
configuration (own CFL dt, eq. cfl, every step) and the fixture keeps:
  * the final state (eta, hu, hv) over the water cells, encoded losslessly
    after quantisation to a step q (a power of two) no larger than 1e-6 of
    the field's root-mean-square over the water cells (so quantisation moves
    a relative L2 error by at most 1e-6 and a relative Linf error by less);
  * the dt sequence (float64, exact) and the final time (float64);
  * the steps taken.
``float32state`` fixtures hold the same for the oracle whose state is
rounded to float32 after every step (what storing the state in float32, as
the paper does, does to the FP64 result; section "Accuracy, precision and
GPUs").

    python tests/golden/make_golden.py run NAME [NAME ...] --raw DIR
        runs the oracle and keeps the float64 results in DIR
    python tests/golden/make_golden.py encode NAME [NAME ...] --raw DIR
        writes tests/golden/NAME.npz from DIR

NAME is config1, config2, config3, config4_m<k> (ensemble member k, 500
steps), config5_r<k> (served request k, horizon capped at 2 simulated
hours), or any of these with the suffix _f32state.
"""

from __future__ import annotations

import argparse
import json
import lzma
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CONFIG5_CAP_S = 7200.0


def workload(name: str):
    import workloads as W
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
        return W.config5_member(r["nx"], r["ny"], min(r["horizon"], CONFIG5_CAP_S))
    raise SystemExit(f"unknown configuration {name}")


def run(name: str, raw: str) -> None:
    from oracle import oracle as orc
    f32 = name.endswith("_f32state")
    base = name[: -len("_f32state")] if f32 else name
    wl = workload(base)
    o = orc.Oracle(wl)
    t0 = time.time()
    if not f32:
        if wl.t_end:
            st, t, dts, k = o.run(nsteps=10 ** 7, t_end=wl.t_end)
        else:
            st, t, dts, k = o.run(nsteps=wl.steps)
    else:
        st = o.initial_state()
        t, k, dl = 0.0, 0, []
        while (t < wl.t_end) if wl.t_end else (k < wl.steps):
            st, t, d1, n = o.run(st, t, nsteps=1, t_end=wl.t_end or 0.0)
            st = tuple(np.asarray(a, np.float32).astype(np.float64) for a in st)
            dl.extend(d1.tolist())
            k += n
        dts = np.asarray(dl)
    el = time.time() - t0
    np.savez(os.path.join(raw, f"{name}.npz"), eta=st[0], hu=st[1], hv=st[2], dts=np.asarray(dts), t=t, steps=k)
    print(json.dumps({"config": name, "steps": int(k), "t": float(t), "seconds": round(el, 1),
                      "threads": orc.num_threads()}), flush=True)


# ---- lossless coding of a quantised field --------------------------------

def quantum(v: np.ndarray) -> float:
    """Largest power of two not above 1e-6 of the root-mean-square of v."""
    rms = float(np.sqrt(np.mean(v * v))) if v.size else 0.0
    if rms == 0.0:
        return 1.0
    return float(2.0 ** np.floor(np.log2(1e-6 * rms)))


def encode_field(v: np.ndarray, q: float) -> np.ndarray:
    n = np.rint(v / q).astype(np.int64)
    d = np.diff(n, prepend=np.int64(0))
    if np.abs(d).max(initial=0) < 2 ** 31:
        raw = d.astype("<i4").tobytes()
        tag = b"4"
    else:
        raw = d.astype("<i8").tobytes()
        tag = b"8"
    return np.frombuffer(tag + lzma.compress(raw, preset=9 | lzma.PRESET_EXTREME), dtype=np.uint8)


def decode_field(blob: np.ndarray, q: float, count: int) -> np.ndarray:
    b = blob.tobytes()
    dt = "<i4" if b[:1] == b"4" else "<i8"
    d = np.frombuffer(lzma.decompress(b[1:]), dtype=dt).astype(np.int64)
    assert d.size == count
    return np.cumsum(d).astype(np.float64) * q


def encode(name: str, raw: str) -> str:
    base = name[: -len("_f32state")] if name.endswith("_f32state") else name
    wl = workload(base)
    r = np.load(os.path.join(raw, f"{name}.npz"))
    wet = np.ones((wl.ny, wl.nx), bool) if wl.land is None else (np.asarray(wl.land) == 0)
    out = {"nx": wl.nx, "ny": wl.ny, "t": float(r["t"]), "steps": int(r["steps"]), "dts": np.asarray(r["dts"]),
           "count": int(wet.sum())}
    for f in ("eta", "hu", "hv"):
        v = np.asarray(r[f], np.float64)[wet]
        q = quantum(v)
        out[f"{f}_q"] = q
        out[f"{f}_z"] = encode_field(v, q)
    path = os.path.join(HERE, f"{name}.npz")
    np.savez(path, **out)
    return path


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["run", "encode"])
    ap.add_argument("names", nargs="+")
    ap.add_argument("--raw", required=True)
    a = ap.parse_args()
    os.makedirs(a.raw, exist_ok=True)
    for n in a.names:
        if a.mode == "run":
            run(n, a.raw)
        else:
            p = encode(n, a.raw)
            print(p, os.path.getsize(p), flush=True)


if __name__ == "__main__":
    main()
