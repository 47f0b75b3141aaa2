"""Host-side memory and undefined-behaviour checks (CPU only, no GPU needed).

* The C oracle (kfrts.c, hmm.c) built with AddressSanitizer and
  UndefinedBehaviorSanitizer (gcc), driven through small and edge-case inputs
  (empty sequences, T = 0/1, failing factorisations, impossible HMM data) by
  tests/sanitize/oracle_driver.c.
* The host side of libpks (argument validation, workspace sizing, the
  tuning-cache parser, error reporting) built with the same sanitizers on the
  host (hipcc, -Xarch_host; device code is compiled unchanged and never runs)
  and driven through every rejection path by tests/sanitize/abi_driver.cpp.
Either driver exits non-zero on a failed check or a sanitizer report."""
import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1905_13002_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def test_oracle_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not found")
    srcs = [os.path.join(ROOT, "oracle", f) for f in ("kfrts.c", "hmm.c")]
    srcs.append(os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"))
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call([gcc, "-std=c99"] + SAN + srcs + ["-o", exe, "-lm", "-pthread"])
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


def _host_sources():
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))
    return [os.path.join(CSRC, f) for f in names]


def test_host_abi_under_asan_ubsan(tmp_path):
    hipcc = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    srcs = _host_sources()
    driver = os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp")
    headers = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith((".h", ".hpp"))]
    tag = _digest(srcs + headers + [driver, os.path.join(ROOT, "include", "pks.h")])
    exe = os.path.join(OUT, "abi_driver_" + tag)
    if not os.path.exists(exe):
        os.makedirs(OUT, exist_ok=True)
        common = ["-std=c++17", "--offload-arch=gfx950", "-I" + os.path.join(ROOT, "include"),
                  "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        host_san = []
        for flag in SAN:
            host_san += ["-Xarch_host", flag]

        def compile_one(src):
            obj = os.path.join(OUT, os.path.basename(src) + "." + tag + ".o")
            lang = ["-x", "hip"] if src.endswith(".hip") else []
            subprocess.check_call([hipcc] + common + host_san + lang + ["-c", src, "-o", obj],
                                  stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
            return obj

        with cf.ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 1))) as ex:
            objs = list(ex.map(compile_one, srcs + [driver]))
        tmp = exe + ".tmp%d" % os.getpid()
        subprocess.check_call([hipcc, "--offload-arch=gfx950"] + host_san + objs + ["-o", tmp])
        os.replace(tmp, exe)
    env = dict(ENV, PKS_DRIVER_CACHE=str(tmp_path / "cache.json"), HIP_VISIBLE_DEVICES="")
    # the driver must not reach a GPU: hide any device from the HIP runtime
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
