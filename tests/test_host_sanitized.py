"""Host-side builds with AddressSanitizer and UndefinedBehaviorSanitizer (no
GPU needed):

* the stage kernels' index maps (swe_maps.h), tile maps (swe_device.h) and
  the serving loop's arena allocator (swe_arena.h), checked for in-bounds
  access and allocator invariants over many shapes by tests/host_check.cpp;
* the FP64 oracle over every boundary kind, friction law, forcing and the
  dt policy (tests/oracle_sanitize_driver.c);
* the library's C ABI on its host-only paths -- size queries and the
  refusal of invalid arguments and inputs before any device work
  (tests/abi_sanitize_driver.cpp) -- with the library's host code built
  with the sanitizers (device code is not built with them)."""

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1912_02457_amd", "csrc")
ROCM = "/opt/rocm"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...:\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(f"{ROCM}/include"),
                    reason="needs g++ and the HIP headers")
def test_index_maps_and_arena_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_check")
    _run(["g++", "-O1", "-g", "-std=c++17", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{CSRC}", *SAN,
          os.path.join(HERE, "host_check.cpp"), "-o", exe])
    r = _run([exe], timeout=600, env=ENV)
    assert "bad 0" in r.stdout and "runtime error" not in r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", f"-I{os.path.join(ROOT, 'oracle')}", *SAN,
          os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "swe_oracle.c"), "-lm",
          "-o", exe])
    r = _run([exe], timeout=300, env=ENV)
    assert "bad 0" in r.stdout and "runtime error" not in r.stderr


@pytest.mark.skipif(shutil.which("hipcc") is None or not os.path.exists(f"{ROCM}/lib/llvm/bin/clang++"),
                    reason="needs hipcc and ROCm's clang++")
def test_abi_host_paths_under_sanitizers(tmp_path):
    d = str(tmp_path)
    # host code with the sanitizers (each flag behind -Xarch_host: no
    # sanitizer in device code); the stage-kernel source is replaced by
    # launch stubs, the preprocessing source keeps its device code
    host = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
            "-fno-omit-frame-pointer"]
    jobs = []
    for src in ("swe_api.hip", "swe_ensemble.hip", "swe_server.hip"):
        jobs.append(["hipcc", "--offload-host-only", "-O1", "-g", "-std=c++17", "-fPIC", *host, "-c",
                     os.path.join(CSRC, src), "-o", os.path.join(d, src + ".o")])
    jobs.append(["hipcc", "--offload-host-only", "-O1", "-g", "-std=c++17", "-fPIC", f"-I{CSRC}", *host, "-c",
                 os.path.join(HERE, "abi_sanitize_stubs.hip"), "-o", os.path.join(d, "stubs.o")])
    jobs.append(["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", *host, "-c",
                 os.path.join(CSRC, "swe_preprocess.hip"), "-o", os.path.join(d, "swe_preprocess.hip.o")])
    clang = f"{ROCM}/lib/llvm/bin/clang++"
    jobs.append([clang, "-O1", "-g", "-std=c++17", f"-I{os.path.join(ROOT, 'include')}", *SAN, "-c",
                 os.path.join(HERE, "abi_sanitize_driver.cpp"), "-o", os.path.join(d, "driver.o")])
    with ThreadPoolExecutor(len(jobs)) as ex:
        list(ex.map(_run, jobs))
    exe = os.path.join(d, "abi_san")
    objs = [os.path.join(d, f) for f in ("driver.o", "swe_api.hip.o", "swe_ensemble.hip.o", "swe_server.hip.o",
                                         "swe_preprocess.hip.o", "stubs.o")]
    _run([clang, "-fsanitize=address,undefined", *objs, f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib",
          "-o", exe])
    r = _run([exe], timeout=300, env=ENV)
    assert "bad 0" in r.stdout and "runtime error" not in r.stderr
