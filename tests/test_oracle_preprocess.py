"""CPU pins of the preprocessing oracle (sections "Bathymetry" and
"Refinement and coarsening of grid"), and a mutation check: each planted
mistake in a copy of the oracle must fail at least one pin."""

import importlib.util
import os
import sys
import tempfile

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import _prepins as PINS  # noqa: E402
from oracle import preprocess as P  # noqa: E402


@pytest.mark.parametrize("pin", PINS.ALL, ids=[f.__name__ for f in PINS.ALL])
def test_preprocess_pin(pin):
    pin(P)


MUTANTS = {
    "corner_plane_sign": ("acc[j + dj, i + di] += v[j, i] + (di - 0.5) * sx[j, i] + (dj - 0.5) * sy[j, i]",
                          "acc[j + dj, i + di] += v[j, i] - (di - 0.5) * sx[j, i] + (dj - 0.5) * sy[j, i]"),
    "corner_plane_full_slope": ("acc[j + dj, i + di] += v[j, i] + (di - 0.5) * sx[j, i] + (dj - 0.5) * sy[j, i]",
                                "acc[j + dj, i + di] += v[j, i] + (2 * di - 1) * sx[j, i] + (dj - 0.5) * sy[j, i]"),
    "correction_subtracted": ("Hs = Hs + np.where(c2 > 0, dHc, 0.0)", "Hs = Hs - np.where(c2 > 0, dHc, 0.0)"),
    "misfit_on_one_corner": ("return 0.25 * (Hc[:-1, :-1] + Hc[:-1, 1:] + Hc[1:, :-1] + Hc[1:, 1:])",
                             "return 0.25 * (Hc[:-1, :-1] + Hc[:-1, 1:] + Hc[1:, :-1] + Hc[:-1, :-1])"),
    "smoother_weights": ("out[j, i] = (1.0 - w) * Hc[j, i] + 0.25 * w * s", "out[j, i] = (1.0 - w) * Hc[j, i] + 0.125 * w * s"),
    "slope_through_land": ("dl = v[j, i] - v[j, i - 1] if i > 0 and wet[j, i - 1] else 0.0\n            dr",
                           "dl = v[j, i] - v[j, i - 1] if i > 0 else 0.0\n            dr"),
    "slope_unlimited": ("sx[j, i] = _minmod(dl, dr)", "sx[j, i] = 0.5 * (dl + dr)"),
    "fill_from_land_estimate": ("Hs = np.where(keep, _smooth(Hs, smooth), fill)", "Hs = _smooth(Hs, smooth)"),
    "erosion_8_neighbours": ("nb = [(j, i - 1), (j, i + 1), (j - 1, i), (j + 1, i)]",
                             "nb = [(j, i - 1), (j, i + 1), (j - 1, i), (j + 1, i), (j - 1, i - 1), (j + 1, i + 1)]"),
    "erosion_min_not_max": ("e2[j, i] = max(vals)", "e2[j, i] = min(vals)"),
    "erosion_in_place": ("vals = [eta[b] for b in nb if 0 <= b[0] < ny and 0 <= b[1] < nx and not land[b]]",
                         "vals = [eta[b] for b in nb if 0 <= b[0] < ny and 0 <= b[1] < nx and not L2[b]]"),
    "refine_half_cell_offset": ("r[2 * j + dj, 2 * i + di] = v[j, i] + (0.5 * di - 0.25) * sx + (0.5 * dj - 0.25) * sy",
                                "r[2 * j + dj, 2 * i + di] = v[j, i] + (di - 0.5) * sx + (0.5 * dj - 0.25) * sy"),
    "refine_unhalved_central": ("sx = _minmod3(theta * dl, 0.5 * (dl + dr), theta * dr)",
                                "sx = _minmod3(theta * dl, dl + dr, theta * dr)"),
    "refine_corner_weights_swapped": ("Hc2[J, I] = ((1 - wy) * ((1 - wx) * Hc[j, i] + wx * Hc[j, i1]) +",
                                      "Hc2[J, I] = ((1 - wy) * (wx * Hc[j, i] + (1 - wx) * Hc[j, i1]) +"),
    "coarsen_counts_land": ("                    if water:\n                        kids = water\n", ""),
    "coarsen_land_any": ("land2 = (L[0::2, 0::2] & L[0::2, 1::2] & L[1::2, 0::2] & L[1::2, 1::2])",
                         "land2 = (L[0::2, 0::2] | L[0::2, 1::2] | L[1::2, 0::2] | L[1::2, 1::2])"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_preprocess_pins_catch_mutant(name):
    old, new = MUTANTS[name]
    src = open(P.__file__).read()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {name}"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mutant_preprocess.py")
        with open(path, "w") as fh:
            fh.write(src.replace(old, new))
        spec = importlib.util.spec_from_file_location("mutant_preprocess", path)
        M = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(M)
        for pin in PINS.ALL:
            try:
                pin(M)
            except (AssertionError, ValueError, IndexError, ZeroDivisionError):
                return
        pytest.fail(f"no pin caught mutant {name}")
