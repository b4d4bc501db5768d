"""Host AddressSanitizer / UndefinedBehaviorSanitizer runs, on the CPU.

Two drivers under tests/sanitize/ are built with the sanitizers and run:
  - oracle_check.c with the oracle's C code (gcc), on ragged and degenerate
    grids, with checks of what the operator's definition fixes;
  - abi_check.cpp with the HIP library's host code: every source is compiled
    with the sanitizers on its host side only (device code is built as usual
    and never runs), and the driver calls each entry point's argument checks,
    the creation calls without a device and the host-only sliced-ELLPACK
    layout builder.
Reports are fatal (no recovery) and LeakSanitizer checks the heap at exit.
The library objects are cached in the package's build folder, keyed by the
hash of the source, the headers and the flags, so only a changed source is
rebuilt (a build from nothing takes about two minutes on 8 cores).
"""
import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_DIR = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2603_23343_amd", "csrc")
INC = os.path.join(ROOT, "include")
CACHE = os.path.join(ROOT, "paper_2603_23343_amd", "_build", "sanitize")
ROCM = "/opt/rocm"
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANGXX = os.path.join(ROCM, "lib", "llvm", "bin", "clang++")

# sanitizer flags of the host compilation (each behind -Xarch_host for hipcc)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
HOST_SAN = [a for f in SAN + ["-O1", "-g"] for a in ("-Xarch_host", f)]
HIP_FLAGS = ["-std=c++20", "-O3", "--offload-arch=gfx950", "-I", INC, "-I", CSRC,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN]
RUN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _run(exe):
    env = dict(os.environ, **RUN_ENV)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "Sanitizer" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_check")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", *SAN, "-static-libasan", "-static-libubsan",
           os.path.join(SAN_DIR, "oracle_check.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    assert "oracle_check: ok" in _run(exe)


def _headers_hash():
    h = hashlib.sha256(" ".join(HIP_FLAGS).encode())
    for d in (CSRC, INC):
        for f in sorted(os.listdir(d)):
            if f.endswith((".hpp", ".h")):
                with open(os.path.join(d, f), "rb") as fh:
                    h.update(f.encode() + fh.read())
    return h.hexdigest()


def _object(src, hh):
    with open(src, "rb") as fh:
        key = hashlib.sha256(hh.encode() + fh.read()).hexdigest()[:20]
    base = os.path.basename(src)
    obj = os.path.join(CACHE, f"{base}.{key}.o")
    if os.path.exists(obj):
        return obj
    for old in os.listdir(CACHE):  # the same source's stale objects
        if old.startswith(base + ".") and old.endswith(".o"):
            os.remove(os.path.join(CACHE, old))
    tmp = obj + ".tmp"
    r = subprocess.run([HIPCC, *HIP_FLAGS, "-c", src, "-o", tmp], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    os.replace(tmp, obj)
    return obj


@pytest.mark.timeout(900)
def test_abi_host_code_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)):
        pytest.skip("ROCm compilers not found")
    os.makedirs(CACHE, exist_ok=True)
    hh = _headers_hash()
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with cf.ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 4))) as ex:
        objs = list(ex.map(lambda s: _object(s, hh), srcs))
    exe = str(tmp_path / "abi_check")
    lib = os.path.join(ROCM, "lib")
    cmd = [CLANGXX, "-std=c++20", "-O1", "-g", *SAN, "-D__HIP_PLATFORM_AMD__", "-I", INC,
           "-I", os.path.join(ROCM, "include"), os.path.join(SAN_DIR, "abi_check.cpp"), *objs, "-o", exe,
           "-L", lib, "-lamdhip64", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{lib}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "abi_check: ok" in _run(exe)
