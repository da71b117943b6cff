"""Element-wise comparison of a float32 GPU state with the FP64 oracle.

eta is normalised by its own norm; hu and hv by the norm of the momentum
magnitude sqrt(hu^2 + hv^2) of the reference (so a field that is nearly zero,
e.g. hv in a 1-D flow, is not divided by ~0).  Land cells are excluded.
"""

import numpy as np

L2_TOL = 1e-4
LINF_TOL = 5e-4


def parity(gpu, ref, land=None):
    e, u, v = (np.asarray(a, np.float64) for a in gpu[:3])
    re, ru, rv = (np.asarray(a, np.float64) for a in ref[:3])
    m = np.ones(re.shape, bool) if land is None else (np.asarray(land) == 0)
    mom = np.sqrt(ru ** 2 + rv ** 2)[m]
    n_e2 = max(np.linalg.norm(re[m]), 1e-30)
    n_m2 = max(np.linalg.norm(mom), 1e-30)
    n_ei = max(np.abs(re[m]).max(initial=0.0), 1e-30)
    n_mi = max(mom.max(initial=0.0), 1e-30)
    out = {
        "eta_l2": np.linalg.norm((e - re)[m]) / n_e2,
        "eta_linf": np.abs((e - re)[m]).max(initial=0.0) / n_ei,
        "hu_l2": np.linalg.norm((u - ru)[m]) / n_m2,
        "hu_linf": np.abs((u - ru)[m]).max(initial=0.0) / n_mi,
        "hv_l2": np.linalg.norm((v - rv)[m]) / n_m2,
        "hv_linf": np.abs((v - rv)[m]).max(initial=0.0) / n_mi,
    }
    return out


def assert_parity(gpu, ref, land=None, l2=L2_TOL, linf=LINF_TOL, label=""):
    p = parity(gpu, ref, land)
    bad = {k: v for k, v in p.items() if v > (l2 if k.endswith("l2") else linf)}
    assert not bad, f"{label} parity failed: {bad} (all: {p})"
    return p
