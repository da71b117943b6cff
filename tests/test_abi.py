"""C-ABI checks that need no GPU: the HIP library loads, exports every entry
point that include/swe.h declares, and rejects invalid arguments before any
device work."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "swe.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(swe_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1912_02457_amd import swe
    if not os.path.exists(swe.LIB_PATH):
        from paper_1912_02457_amd import build
        build.build()
    return swe.load_library()


def test_exports_every_declared_symbol(lib):
    syms = header_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in include/swe.h but not exported"
    from paper_1912_02457_amd import swe
    assert set(swe.SIGNATURES) == set(syms), "binding signatures out of sync with the header"


def test_params_struct_layout_matches_header():
    """The ctypes mirror of swe_params has the C layout (checked against a
    tiny C translation unit compiled here)."""
    import subprocess
    import tempfile
    from paper_1912_02457_amd import swe
    src = ('#include <stddef.h>\n#include <stdio.h>\n#include "swe.h"\nint main(){printf("%zu %zu %zu %zu\\n",'
           'sizeof(swe_params), offsetof(swe_params, bc), offsetof(swe_params, frs_d0),'
           'offsetof(swe_params, north_projection));return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    P = swe.Params
    assert [int(x) for x in out] == [C.sizeof(P), P.bc.offset, P.frs_d0.offset, P.north_projection.offset]


def _params(**kw):
    from paper_1912_02457_amd import swe
    base = dict(nx=16, ny=12, dx=100.0, dy=100.0)
    base.update(kw)
    return swe.make_params(base.pop("nx"), base.pop("ny"), base.pop("dx"), base.pop("dy"), **base)


@pytest.mark.parametrize("kw", [dict(nx=1), dict(ny=0), dict(dx=-1.0), dict(courant=0.0), dict(courant=1.5),
                                dict(theta=0.5), dict(kappa=0.0), dict(bc=(1, 0, 0, 0)), dict(bc=(0, 0, 3, 0)),
                                dict(friction=7), dict(frs_width=0), dict(frs_width=33), dict(frs_d0=0.0)])
def test_invalid_params_rejected(lib, kw):
    from paper_1912_02457_amd import swe
    n = C.c_size_t()
    rc = lib.swe_workspace_bytes(C.byref(_params(**kw)), 1, 0, C.byref(n))
    assert rc == swe.SWE_E_ARG
    assert lib.swe_last_error().decode()


def test_workspace_size_grows_with_domain(lib):
    from paper_1912_02457_amd import swe
    a = swe.workspace_bytes(_params(nx=100, ny=100))
    b = swe.workspace_bytes(_params(nx=200, ny=100))
    c = swe.workspace_bytes(_params(nx=200, ny=100), 1, 10)
    assert 0 < a < b < c
    # 6 state planes + f + corners, 256-byte rows
    assert b >= 8 * 100 * 256 * 4


def test_init_rejects_bad_inputs_before_device_work(lib):
    """Validation happens on the host: a NaN input or a mismatched periodic
    seam is refused without touching the workspace pointer."""
    from paper_1912_02457_amd import swe
    p = _params()
    ny, nx = 12, 16
    z = np.zeros((ny, nx), np.float32)
    Hc = np.full((ny + 1, nx + 1), 10.0, np.float32)
    f = np.zeros((ny, nx), np.float32)
    bad = z.copy()
    bad[3, 4] = np.nan
    F = C.POINTER(C.c_float)
    h = C.c_void_p()
    fake_ws = C.c_void_p(256 * 1024)  # never dereferenced: validation fails first
    rc = lib.swe_init_domain(C.byref(p), fake_ws, 1 << 30, None, 1, 0, Hc.ctypes.data_as(F), None,
                             f.ctypes.data_as(F), None, bad.ctypes.data_as(F), z.ctypes.data_as(F),
                             z.ctypes.data_as(F), C.byref(h))
    assert rc == swe.SWE_E_ARG and "non-finite" in lib.swe_last_error().decode()
    pp = _params(bc=(1, 1, 0, 0))
    Hc2 = Hc.copy()
    Hc2[5, 0] = 11.0
    rc = lib.swe_init_domain(C.byref(pp), fake_ws, 1 << 30, None, 1, 0, Hc2.ctypes.data_as(F), None,
                             f.ctypes.data_as(F), None, z.ctypes.data_as(F), z.ctypes.data_as(F),
                             z.ctypes.data_as(F), C.byref(h))
    assert rc == swe.SWE_E_ARG and "periodic" in lib.swe_last_error().decode()
    rc = lib.swe_init_domain(C.byref(p), C.c_void_p(256 * 1024 + 8), 1 << 30, None, 1, 0, Hc.ctypes.data_as(F),
                             None, f.ctypes.data_as(F), None, z.ctypes.data_as(F), z.ctypes.data_as(F),
                             z.ctypes.data_as(F), C.byref(h))
    assert rc == swe.SWE_E_ARG and "aligned" in lib.swe_last_error().decode()
    rc = lib.swe_init_domain(C.byref(p), fake_ws, 16, None, 1, 0, Hc.ctypes.data_as(F),
                             None, f.ctypes.data_as(F), None, z.ctypes.data_as(F), z.ctypes.data_as(F),
                             z.ctypes.data_as(F), C.byref(h))
    assert rc == swe.SWE_E_NOMEM


def test_null_handles_rejected(lib):
    from paper_1912_02457_amd import swe
    assert lib.swe_step(None, 1) == swe.SWE_E_ARG
    assert lib.swe_status(None) == swe.SWE_E_ARG
    assert lib.swe_autotune_tiling(None, None) == swe.SWE_E_ARG
    lib.swe_destroy(None)


def test_ensemble_arguments_rejected_without_gpu(lib):
    import ctypes as C
    from paper_1912_02457_amd import swe
    n = C.c_size_t()
    assert lib.swe_ensemble_workspace_bytes(None, 1, 0, C.byref(n)) == swe.SWE_E_ARG
    empty = (C.c_void_p * 1)(None)
    assert lib.swe_ensemble_workspace_bytes(empty, 1, 0, C.byref(n)) == swe.SWE_E_ARG
    assert lib.swe_ensemble_workspace_bytes(empty, 0, 0, C.byref(n)) == swe.SWE_E_ARG
    h = C.c_void_p()
    assert lib.swe_ensemble_create(empty, 1, None, 0, None, 0, 0, C.byref(h)) == swe.SWE_E_ARG
    assert lib.swe_ensemble_create(None, 0, None, 0, None, 0, 0, C.byref(h)) == swe.SWE_E_ARG
    assert lib.swe_ensemble_step(None, 1) == swe.SWE_E_ARG
    assert lib.swe_ensemble_info(None, None, None, None, None) == swe.SWE_E_ARG
    assert lib.swe_ensemble_stage_times(None, None, None, None, 0) == swe.SWE_E_ARG
    lib.swe_ensemble_destroy(None)


def test_server_arguments_rejected_without_gpu(lib):
    import ctypes as C
    from paper_1912_02457_amd import swe
    h = C.c_void_p()
    fake = C.c_void_p(1 << 20)  # never dereferenced: validation fails first
    assert lib.swe_server_create(None, 1 << 20, None, None, 4, 8, 0, 0, C.byref(h)) == swe.SWE_E_ARG
    assert lib.swe_server_create(fake, 1 << 20, None, None, 0, 8, 0, 0, C.byref(h)) == swe.SWE_E_ARG
    assert lib.swe_server_create(fake, 1 << 20, None, None, 4, 0, 0, 0, C.byref(h)) == swe.SWE_E_ARG
    assert lib.swe_server_create(C.c_void_p((1 << 20) + 8), 1 << 20, None, None, 4, 8, 0, 0,
                                 C.byref(h)) == swe.SWE_E_ARG
    assert lib.swe_server_submit(None, None) == swe.SWE_E_ARG
    assert lib.swe_server_tick(None, None, None) == swe.SWE_E_ARG
    n = C.c_int32()
    assert lib.swe_server_poll(None, None, 0, C.byref(n)) == swe.SWE_E_ARG
    assert lib.swe_server_get_stats(None, None) == swe.SWE_E_ARG
    lib.swe_server_destroy(None)


def test_request_struct_layout_matches_header():
    import subprocess
    import tempfile
    from paper_1912_02457_amd import swe
    src = ('#include <stddef.h>\n#include <stdio.h>\n#include "swe.h"\nint main(){printf("%zu %zu %zu %zu %zu %zu\\n",'
           'sizeof(swe_request), offsetof(swe_request, horizon), offsetof(swe_request, n_wind),'
           'offsetof(swe_request, out_hv), sizeof(swe_completion), sizeof(swe_server_stats));return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = [int(x) for x in subprocess.check_output([exe]).decode().split()]
    R = swe.Request
    assert out == [C.sizeof(R), R.horizon.offset, R.n_wind.offset, R.out_hv.offset,
                   C.sizeof(swe.Completion), C.sizeof(swe.ServerStats)]


def test_product_path_has_no_oracle_or_cpu_fallback():
    """The package never imports the oracle and has no numpy time stepping."""
    pkg = os.path.join(ROOT, "paper_1912_02457_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in txt.lower().replace("oracle_", ""), fn


def test_preprocess_rejects_invalid_arguments(lib):
    """The preprocessing entry points refuse bad sizes, pointers and
    parameters before enqueueing anything (the pointers here are never
    dereferenced: each call fails its argument checks first)."""
    from paper_1912_02457_amd import swe
    p = C.c_void_p(0x1000)  # never dereferenced
    E = swe.SWE_E_ARG
    rb = lib.swe_reconstruct_bathymetry
    assert rb(0, 5, p, None, 0, 0.5, p, p, None) == E
    assert rb(5, 5, None, None, 0, 0.5, p, p, None) == E
    assert rb(5, 5, p, None, 0, 0.5, None, p, None) == E
    assert rb(5, 5, p, None, 3, 0.5, p, None, None) == E      # scratch needed
    assert rb(5, 5, p, None, -1, 0.5, p, p, None) == E
    assert rb(5, 5, p, None, 2, 1.5, p, p, None) == E
    assert rb(5, 5, p, None, 2, float("nan"), p, p, None) == E
    assert b"smooth" in lib.swe_last_error()
    assert rb(40000, 40000, p, None, 2, 0.5, p, p, None) == E  # 6.4 GB corner plane
    el = lib.swe_erode_land
    assert el(0, 4, p, p, None, None, None, 5.0, p, p, None, None, None, None) == E
    assert el(4, 4, None, p, None, None, None, 5.0, p, p, None, None, None, None) == E
    assert el(4, 4, p, p, p, None, None, 5.0, p, p, None, None, None, None) == E   # eta without output
    assert el(4, 4, p, p, None, None, None, float("inf"), p, p, None, None, None, None) == E
    rf = lib.swe_refine2
    assert rf(4, 4, 1, p, None, 0.5, p, None, None, None, None) == E     # theta < 1
    assert rf(4, 4, 1, None, None, 1.0, p, None, None, None, None) == E
    assert rf(4, 4, 0, None, p, 1.0, None, p, None, None, None) == E     # land_out with no field
    assert rf(4, 4, 1, p, None, 1.0, p, p, None, None, None) == E        # land_out without land
    assert rf(4, 4, 0, None, None, 1.0, None, None, p, None, None) == E  # Hc without Hc_out
    assert rf(30000, 30000, 0, None, None, 1.0, None, None, p, p, None) == E
    cs = lib.swe_coarsen2
    assert cs(5, 4, 1, p, None, p, None, None, None, None) == E          # odd nx
    assert cs(4, 0, 1, p, None, p, None, None, None, None) == E
    assert cs(4, 4, 1, p, None, p, p, None, None, None) == E             # land_out without land
    assert cs(4, 4, 0, None, None, None, None, p, None, None) == E


def test_dt_policy_rejects_null_domain(lib):
    from paper_1912_02457_amd import swe
    assert lib.swe_set_dt_policy(None, 1200.0) == swe.SWE_E_ARG


def test_stress_field_rejects_invalid_arguments(lib):
    from paper_1912_02457_amd import swe
    assert lib.swe_set_stress_field(None, 1, 2, 2, None, None, None, 0) == swe.SWE_E_ARG


def test_boundary_field_rejects_invalid_arguments(lib):
    from paper_1912_02457_amd import swe
    t = (C.c_double * 1)(0.0)
    assert lib.swe_set_boundary_field(None, 1, 4, 4, t, None) == swe.SWE_E_ARG
