"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

`host_sanitize.cpp` drives the host-only entry points (grid validation, the
rectilinear axis tables, the well and indicator partition builders,
footprint estimates, the early error paths of set-up) over seeded random
grids and malformed inputs.  The C-ABI translation unit is compiled with the
sanitizers on its host code (`-Xarch_host` before each sanitizer flag, so no
device code is instrumented) and linked with the library's other objects; the
program runs on the CPU, no GPU is touched.  The set-up-time stage builders
(fault-cut pieces and supports, graph supports) need a device and are
covered by the GPU parity tests instead."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = "-Xarch_host -fsanitize=address,undefined -Xarch_host -fno-sanitize-recover=all".split()


@pytest.mark.timeout(900)
def test_host_code_under_sanitizers(tmp_path):
    from paper_2001_01624_amd import build as B

    hipcc = B.hipcc()
    if not shutil.which(hipcc) and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    objs = [os.path.join(B.BUILD, s.replace(".hip", ".o")) for s in B.SOURCES]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    inc = os.path.join(ROOT, "include")
    capi_o = str(tmp_path / "capi_san.o")
    drv_o = str(tmp_path / "host_sanitize.o")
    exe = str(tmp_path / "host_sanitize")
    base = [hipcc, "-O1", "-g", "-std=c++17", *SAN, "-Xarch_host", "-fno-omit-frame-pointer"]
    steps = [
        base + ["-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-I", inc, "-c", os.path.join(B.CSRC, "capi.hip"), "-o", capi_o],
        base + ["-I", inc, "-c", os.path.join(HERE, "host_sanitize.cpp"), "-o", drv_o],
        [hipcc, *SAN, "--offload-arch=gfx950", drv_o, capi_o]
        + [o for o in objs if not o.endswith(os.sep + "capi.o")] + ["-o", exe],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "host sanitize ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
