"""Measured choice of the ensemble's work decomposition.

The persistent ensemble kernel takes two knobs: rows per tile (the strip
height one wavefront sweeps; taller tiles amortise the 4-row halo of the
two-row stencil, shorter ones balance the tail of the queue) and the number
of work items a wavefront claims per atomic.  ``autotune_ensemble`` times a
few steps of every candidate on the real members and keeps the fastest; the
result is cached on disk under a key made of the member shapes, so a
repeated ensemble of the same shapes skips the sweep.
"""

from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Iterable, Optional, Sequence, Tuple

DEFAULT_ROWS = (4, 8, 16, 32, 64)
DEFAULT_CHUNKS = (1, 2, 4)


def _key(members, device_name: str) -> str:
    shapes = sorted((m.nx, m.ny) for m in members)
    proj = bool(members[0].params.north_projection)
    h = hashlib.sha1(json.dumps([device_name, proj, shapes]).encode()).hexdigest()
    return h[:20]


def _load(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: Optional[str], table: dict):
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune_ensemble(members: Sequence, *, rows: Iterable[int] = DEFAULT_ROWS,
                      chunks: Iterable[int] = DEFAULT_CHUNKS, steps: int = 32,
                      cache: Optional[str] = None) -> Tuple[int, int, dict]:
    """Returns (rows_per_wave, chunk, report).  The members' states advance
    by ``steps + 2`` steps per candidate tried (the sweep runs the real
    workload); use fresh or throw-away domains when that matters."""
    import torch
    from .swe import Ensemble
    dev = members[0].device
    name = torch.cuda.get_device_name(dev)
    key = _key(members, name)
    table = _load(cache)
    if key in table:
        e = table[key]
        return int(e["rows"]), int(e["chunk"]), dict(e, cached=True)
    cells = sum(m.nx * m.ny for m in members)
    trials = []
    for r in rows:
        for c in chunks:
            ens = Ensemble(members, rows_per_wave=r, chunk=c)
            ens.use_graphs(False)
            ens.step(2)
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            ens.step(steps)
            torch.cuda.synchronize(dev)
            el = time.perf_counter() - t0
            ens.close()
            trials.append({"rows": r, "chunk": c, "cell_updates_per_s": cells * steps / el})
    best = max(trials, key=lambda t: t["cell_updates_per_s"])
    entry = {"rows": best["rows"], "chunk": best["chunk"], "cell_updates_per_s": best["cell_updates_per_s"],
             "members": len(members), "cells": cells, "device": name}
    table[key] = entry
    _store(cache, table)
    return best["rows"], best["chunk"], dict(entry, cached=False, trials=trials)
