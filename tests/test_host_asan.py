"""The library's host code under the address sanitizer, on the CPU.

pool.cpp and capi.cpp are compiled for the host only with AddressSanitizer
and linked against tests/host/fake_hip.cpp, an emulation of the HIP calls
they make (device memory is host memory, graph launches run the pool's
bookkeeping transitions with scripted decisions, sweeps touch every plane
they would read or write).  tests/host/host_driver.cpp then drives random
sequences through the C ABI: pool admission, advances, polls, promotions,
early and late retirement and re-creation; the single-solve API (create,
step, solve with its polling loop, field access, checkpoints); and the
allocation-free solve.  Every buffer handed over has exactly the documented
size, so any host access outside an allocation fails the test."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
SRC = [os.path.join(ROOT, "paper_2004_11227_amd", "csrc", f) for f in ("pool.cpp", "capi.cpp")] + \
      [os.path.join(ROOT, "tests", "host", f) for f in ("fake_hip.cpp", "host_driver.cpp")]


@pytest.fixture(scope="module")
def driver():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp(prefix="mf_asan_")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "--cuda-host-only",
             "-Xarch_host", "-fsanitize=address", "-fno-omit-frame-pointer",
             "-I", os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument"]
    procs, objs = [], []
    for s in SRC:
        o = os.path.join(d, os.path.basename(s) + ".o")
        objs.append(o)
        procs.append(subprocess.Popen([HIPCC, *flags, "-c", s, "-o", o], stdout=subprocess.PIPE,
                                      stderr=subprocess.PIPE, text=True))
    for p in procs:
        out, err = p.communicate(timeout=600)
        assert p.returncode == 0, err[-4000:]
    # the host-only object of capi.cpp refers to the device code object of
    # its static array: give it a stand-in
    nm = subprocess.run(["nm", "--undefined-only", objs[1]], capture_output=True, text=True, check=True).stdout
    fat = re.findall(r"__hip_fatbin_[0-9a-f]+", nm)
    stub = os.path.join(d, "fatbin.c")
    with open(stub, "w") as f:
        for name in sorted(set(fat)):
            f.write(f"char {name}[64];\n")
    subprocess.run(["gcc", "-c", stub, "-o", stub + ".o"], check=True)
    exe = os.path.join(d, "host_driver")
    subprocess.run([HIPCC, "-Xarch_host", "-fsanitize=address", "-o", exe, *objs, stub + ".o"], check=True,
                   capture_output=True, timeout=600)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_host_code_is_clean_under_asan(driver, seed):
    r = subprocess.run([driver, "3", str(seed)], capture_output=True, text=True, timeout=600,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0"})
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "host_driver ok" in r.stdout
