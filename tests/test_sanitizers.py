"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the CPU oracle and of
the C ABI's host code, run on the CPU.

- oracle: every entry point on small, ragged and degenerate inputs
  (tests/native/oracle_sanitize.c, gcc);
- C ABI: parameter validation, scratch layout arithmetic up to the largest
  sizes, every argument error of every entry point, and (without a GPU) the
  cleanup paths of the create calls after a failed device allocation, with the
  kernel launchers replaced by counting stubs (tests/native/abi_host_check.cpp,
  hipcc with the sanitizers on the host side only).

A finding (out-of-bounds access, leak, signed overflow, bad shift) fails the run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2201_11924_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    run(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-ffp-contract=off", "-Wall", "-Wno-unused-function", "-o", exe,
         os.path.join(NATIVE, "oracle_sanitize.c"), "-lm"])
    out = run([exe], env=SAN_ENV)
    assert "clean" in out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_c_abi_host_code_under_asan_ubsan(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", *san, "-fno-omit-frame-pointer",
              "-ffp-contract=off", "-I", os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument"]
    jobs = [(os.path.join(CSRC, f + ".hip"), str(tmp_path / (f + ".o")))
            for f in ("api", "noalloc", "aggregate", "batch_api", "net_api", "noise_gen", "geometry")]
    jobs += [(os.path.join(NATIVE, f + ".cpp"), str(tmp_path / (f + ".o")))
             for f in ("abi_host_stubs", "abi_host_check")]
    procs = [subprocess.Popen([HIPCC, *common, "-x", "hip", "-c", src, "-o", obj], stdout=subprocess.PIPE,
                              stderr=subprocess.PIPE, text=True) for src, obj in jobs]
    for p, (src, _) in zip(procs, jobs):
        out, err = p.communicate()
        assert p.returncode == 0, f"{src}\n{err[-4000:]}"
    exe = str(tmp_path / "abi_check")
    run([HIPCC, "--offload-arch=gfx950", *san, "-o", exe, *[obj for _, obj in jobs], "-L/opt/rocm/lib",
         "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"])
    out = run([exe], env=SAN_ENV)
    assert "clean" in out
    shutil.rmtree(tmp_path, ignore_errors=True)
