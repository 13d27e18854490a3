"""CPU builds with AddressSanitizer and UndefinedBehaviorSanitizer.

- the oracle: a C driver through all its paths, and the oracle's own test
  suite against a sanitized build of the library (gcc's runtime preloaded);
- the host side of libfmm (validation, workspace sizing and carving of every
  entry point): a C++ driver, and the host-side ABI tests against a build
  whose host code is sanitized (the device code is the normal build; no
  kernel runs on the CPU).
Sanitizers apply to host code only (every hipcc use puts -Xarch_host before
-fsanitize).  Any sanitizer report fails the run (no recovery)."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

from conftest import ROOT

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CSRC = os.path.join(ROOT, "paper_1502_07303_amd", "csrc")
SAN_C = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
SAN_HIP = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
HIP_FLAGS = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-ffp-contract=off", "-Xclang",
             "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include")]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")


def _need(tool):
    if shutil.which(tool) is None and not os.path.exists(tool):
        pytest.skip(f"{tool} not available")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-2000:], r.stderr[-4000:])
    return r


def test_oracle_driver_sanitized(tmp_path):
    _need("gcc")
    exe = tmp_path / "san_oracle"
    _run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off"] + SAN_C +
         [os.path.join(ROOT, "tests", "sanitize_oracle.c"), os.path.join(ROOT, "oracle", "fmm_oracle.c"), "-lm",
          "-o", str(exe)])
    r = _run([str(exe)], env=ENV)
    assert r.stdout.strip() == "ok"


def test_oracle_suite_under_sanitizers(tmp_path):
    _need("gcc")
    lib = tmp_path / "liboracle_san.so"
    _run(["gcc", "-std=c11", "-O1", "-g", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"] + SAN_C +
         [os.path.join(ROOT, "oracle", "fmm_oracle.c"), "-lm", "-o", str(lib)])
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(ENV, FMM_ORACLE_LIB=str(lib), LD_PRELOAD=asan)
    _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
          os.path.join(ROOT, "tests", "test_oracle.py"), os.path.join(ROOT, "tests", "test_oracle_adjoint.py")],
         env=env, cwd=ROOT)


def _device_objects(tmp_path):
    """The kernels' objects (normal build), compiled here if build() has not."""
    objs = []
    for src in ("fmm_kernels.hip", "fmm_adjoint.hip"):
        o = os.path.join(ROOT, "paper_1502_07303_amd", "_build", os.path.splitext(src)[0] + ".o")
        if not os.path.exists(o):
            o = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
            _run([HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-ffp-contract=off", "-Xclang",
                  "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-c",
                  os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    return objs


def test_host_driver_sanitized(tmp_path):
    _need(HIPCC)
    api = tmp_path / "api_san.o"
    drv = tmp_path / "drv_san.o"
    exe = tmp_path / "san_host"
    _run([HIPCC] + HIP_FLAGS + SAN_HIP + ["-x", "hip", "-c", os.path.join(CSRC, "fmm_api.cpp"), "-o", str(api)])
    _run([HIPCC] + HIP_FLAGS + SAN_HIP + ["-x", "hip", "-c", os.path.join(ROOT, "tests", "sanitize_host.cpp"),
                                          "-o", str(drv)])
    _run([HIPCC, "--offload-arch=gfx950"] + SAN_HIP[:4] + [str(drv), str(api)] + _device_objects(tmp_path) +
         ["-o", str(exe)])
    r = _run([str(exe)], env=ENV)
    assert r.stdout.strip() == "ok"


def test_abi_suite_under_sanitizers(tmp_path):
    _need(HIPCC)
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts:
        pytest.skip("clang AddressSanitizer runtime not found")
    api = tmp_path / "api_san.o"
    lib = tmp_path / "libfmm_san.so"
    _run([HIPCC] + HIP_FLAGS + SAN_HIP + ["-x", "hip", "-c", os.path.join(CSRC, "fmm_api.cpp"), "-o", str(api)])
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + SAN_HIP[:4] + ["-Xarch_host", "-shared-libsan",
                                                                              str(api)] +
         _device_objects(tmp_path) + ["-o", str(lib)])
    env = dict(ENV, FMM_LIB=str(lib), LD_PRELOAD=rts[0])
    _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
          os.path.join(ROOT, "tests", "test_abi.py")], env=env, cwd=ROOT)
