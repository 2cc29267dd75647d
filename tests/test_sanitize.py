"""Sanitizer runs on the CPU: the oracle, and the host side of the C-ABI
(layouts, bounds, workspace sizes, stream headers, batch descriptor tables
and every argument check that returns before device work), each built with
AddressSanitizer and UndefinedBehaviorSanitizer and driven through its
valid and error paths by a small driver in tests/sanitize/.  Any invalid
access or undefined operation aborts the driver.  For the library only the
host pass is instrumented (each -fsanitize= follows -Xarch_host); no code
built here runs on a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1503_00638_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["bsg_api", "bsg_round", "bsg_shuffle", "bsg_lz4", "bsg_batch", "bsg_fullcov"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])}...: rc {r.returncode}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = tmp_path / "oracle_driver"
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
          os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-lm",
          "-o", str(exe)])
    r = _run([str(exe)], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1", "OMP_NUM_THREADS": "4"},
             timeout=600)
    assert "oracle sanitizer driver ok" in r.stdout


def test_abi_host_side_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("no hipcc")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-fno-omit-frame-pointer",
             "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    procs, objs = [], []
    for s in SOURCES:
        o = str(tmp_path / f"{s}.o")
        procs.append(subprocess.Popen([HIPCC, *flags, *host_san, "-c", os.path.join(CSRC, s + ".hip"),
                                       "-o", o], stdout=subprocess.PIPE, stderr=subprocess.PIPE))
        objs.append(o)
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err.decode()[-3000:]
    drv = str(tmp_path / "driver.o")
    _run([HIPCC, "-O1", "-g", "-std=c++17", *host_san, "-fno-omit-frame-pointer", "-I",
          os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "abi_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "abi_driver")
    _run([HIPCC, *host_san, *objs, drv, "-o", exe])
    r = _run([exe], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0"}, timeout=600)
    assert "abi sanitizer driver ok" in r.stdout
