"""The allocation-free reconstruction entry point against the one that takes
a caller's scratch plane: the same kernels, so the corner depths must agree
bitwise, on two calls in a row (the second on a smaller grid, after the
first has filled the library's static scratch), and sizes beyond the static
scratch are refused before any device work."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_reconstruction_matches_scratch_entry_point():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    from paper_1912_02457_amd import swe
    from workloads import coastal_cells

    dev = torch.device("cuda:0")
    for nx, ny, iters, seed in ((1400, 900, 10, 2), (233, 157, 7, 5)):
        _say("noalloc reconstruction", nx, ny, iters)
        Hm_np, land_np = coastal_cells(nx, ny, seed, seed + 1)
        Hm = torch.from_numpy(Hm_np.astype(np.float32)).to(dev)
        land = torch.from_numpy(land_np.astype(np.uint8)).to(dev)
        ref = swe.reconstruct_bathymetry(Hm, land, iters=iters)
        out = torch.full((ny + 1, nx + 1), float("nan"), dtype=torch.float32, device=dev)
        swe.reconstruct_bathymetry_noalloc(Hm, land, iters=iters, out=out)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
        assert torch.equal(out, ref), f"{nx}x{ny}: differs from the scratch entry point"
        # no land mask, an odd and an even number of rounds (the last round
        # writes Hc either way)
        for it in (iters + 1, 0):
            ref = swe.reconstruct_bathymetry(Hm, None, iters=it)
            out = swe.reconstruct_bathymetry_noalloc(Hm, None, iters=it)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), f"{nx}x{ny}, {it} rounds, no land"


def test_noalloc_rejects_sizes_beyond_the_static_scratch():
    import torch
    from paper_1912_02457_amd import swe
    from paper_1912_02457_amd.swe import SweError
    swe.load_library()
    L = swe._lib
    # (2048 + 1) * (2048 + 1) > 4194304 corners: refused before any device work
    rc = L.swe_reconstruct_bathymetry_noalloc(2048, 2048, None, None, 10, 0.5, None, None)
    assert rc == -1 and b"static scratch" in L.swe_last_error()
    rc = L.swe_reconstruct_bathymetry_noalloc(0, 5, None, None, 10, 0.5, None, None)
    assert rc == -1
    dev = torch.device("cuda:0")
    Hm = torch.ones((2048, 2048), dtype=torch.float32, device=dev)
    with pytest.raises(SweError):
        swe.reconstruct_bathymetry_noalloc(Hm, None, iters=3)
