"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The library's host sources (argument checks, plans, schedules, the tune-cache
  reader, the no-allocation entry point) are compiled with both sanitizers on
  their host side and linked with the already built kernel objects into a small
  driver that walks every validation path of the C-ABI that needs no GPU
  (tests/sanitize/abi_checks.c).
* The FP64 oracle is compiled with both sanitizers into a driver that runs each
  of its entry points on small and degenerate shapes (tests/sanitize/oracle_checks.c).

A sanitizer report aborts the driver, so a zero exit status means no memory or
undefined-behaviour error was seen on these paths.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_cs_0103001_amd", "csrc")
KOBJ = os.path.join(ROOT, "paper_cs_0103001_amd", "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
# host-side instrumentation only: device code of the .hip sources is built as usual
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
# every library source but the two kernel files, whose built objects are reused
KERNEL_SOURCES = ("kernels.hip", "ragged_kernels.hip")
KERNEL_OBJECTS = [k + ".o" for k in KERNEL_SOURCES]


def _host_sources():
    from paper_cs_0103001_amd.build import SOURCES
    return [s for s in SOURCES if s not in KERNEL_SOURCES]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_checks")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", "-o", exe, os.path.join(HERE, "sanitize", "oracle_checks.c"),
          os.path.join(ROOT, "oracle", "oracle_fft.c"), "-lm", "-lpthread"])
    r = _run([exe], env=SAN_ENV, timeout=120)
    assert "0 failure(s)" in r.stdout


def _have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(_have_gpu(), reason="walks the no-device paths")
def test_abi_validation_under_asan_ubsan(tmp_path):
    if not (os.path.exists(CLANGXX) and os.path.exists(HIPCC)):
        pytest.skip("ROCm clang++/hipcc not found")
    kobjs = [os.path.join(KOBJ, o) for o in KERNEL_OBJECTS]
    if not all(os.path.exists(o) for o in kobjs):
        pytest.skip("kernel objects not built (run __graft_entry__.build())")
    objs = []
    for src in _host_sources():
        obj = str(tmp_path / (src + ".o"))
        _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN,
              "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    drv = str(tmp_path / "abi_checks.o")
    _run([CLANGXX, "-x", "c", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-c", os.path.join(HERE, "sanitize", "abi_checks.c"), "-o", drv])
    exe = str(tmp_path / "abi_checks")
    _run([CLANGXX, "-fsanitize=address,undefined", "-o", exe, drv, *objs, *kobjs,
          "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lrocprofiler-sdk-roctx",
          "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    # no GPU: plan creation past the argument checks reports FFT_ERR_HIP
    r = _run([exe], env=SAN_ENV, timeout=120)
    assert "0 failure(s)" in r.stdout
