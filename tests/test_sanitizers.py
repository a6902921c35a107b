"""Sanitizer builds of the host code, on the CPU: the oracle's C sources under gcc's AddressSanitizer
and UndefinedBehaviorSanitizer, running the oracle pin tests in a child process; and the library
compiled with the same sanitizers on its host side, driven by tests/san_host_driver.c (rank
controllers, MPO builder, autotuner table files, argument checks that must fail before any HIP
call).  No GPU is used; the child processes stop at the first error a sanitizer reports."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}
ORACLE_TESTS = ["test_oracle_pid.py", "test_oracle_heff.py", "test_oracle_svd.py", "test_oracle_models.py",
                "test_oracle_circuit.py", "test_oracle_mlp.py", "test_oracle_sched.py", "test_oracle_dmrg.py"]


def test_oracle_pins_under_asan_ubsan():
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=libasan, TNA_ORACLE_LIB_SUFFIX="_san",
               TNA_ORACLE_EXTRA_CFLAGS="-O1 -g -fno-omit-frame-pointer -fsanitize=address,undefined "
                                       "-fno-sanitize-recover=all")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu and not slow", "-p", "no:cacheprovider",
           *[os.path.join("tests", t) for t in ORACLE_TESTS]]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, out


def test_library_host_code_under_asan_ubsan(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not found")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    flags = ["--offload-arch=gfx950", "-x", "hip", "-O1", "-g", "-fPIC", "-std=c++17", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san, "-I", os.path.join(ROOT, "include")]
    sys.path.insert(0, os.path.join(ROOT, "paper_2604_03960_amd"))
    from build import SOURCES
    srcs = [os.path.join(ROOT, "paper_2604_03960_amd", "csrc", f) for f in SOURCES]
    srcs.append(os.path.join(ROOT, "tests", "san_host_driver.c"))

    def cc(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run(["hipcc", *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(cc, srcs))
    exe = str(tmp_path / "san_host_driver")
    r = subprocess.run(["hipcc", "--offload-arch=gfx950", *san, *objs, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe, str(tmp_path)], env=dict(os.environ, **SAN_ENV), capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "all checks passed" in r.stdout
