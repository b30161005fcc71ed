"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The schedule-cache file of fit_plan_tune (csrc/tune_cache.hpp): a small C++
  program (tests/host/tune_cache_check.cpp) built with both sanitizers.
* The plain-C oracle: lse_oracle.c built with both sanitizers (gcc), and the
  oracle's CPU tests run against that build (LSE_ORACLE_LIB) in a child
  process with gcc's ASan runtime preloaded.
* The host side of the C ABI (argument validation, workspace layout,
  schedules, plans, timing, the tune cache): csrc/api.hip rebuilt with the
  sanitizers on its host code only (the GPU code is left as it is) and linked
  with the other objects of the last library build, and the CPU ABI tests run
  against it (LSEFIT_LIB) in a child process with clang's ASan runtime
  preloaded.

Leak detection is off in the Python children (the interpreter itself keeps
memory until exit); every other report fails the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1512_08017_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build", "obj")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _run(cmd, env=None, timeout=600):
    res = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    if res.returncode != 0:
        raise AssertionError(f"{' '.join(cmd)}\nexit {res.returncode}\n{res.stdout[-4000:]}\n{res.stderr[-4000:]}")
    return res


def _runtime(compiler, name):
    path = subprocess.run([compiler, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not path or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not found by {compiler}")
    return path


def test_tune_cache_under_sanitizers(tmp_path):
    exe = tmp_path / "tune_cache_check"
    _run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-I" + INCLUDE, "-I" + CSRC,
          os.path.join(ROOT, "tests", "host", "tune_cache_check.cpp"), "-o", str(exe)])
    out = _run([str(exe), str(tmp_path)])
    assert "tune cache checks passed" in out.stdout


def test_oracle_under_sanitizers(tmp_path):
    lib = tmp_path / "liblse_oracle_san.so"
    _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
          "-o", str(lib), os.path.join(ROOT, "oracle", "csrc", "lse_oracle.c"), "-lm"])
    env = dict(os.environ, **SAN_ENV, LSE_ORACLE_LIB=str(lib), LD_PRELOAD=_runtime("gcc", "libasan.so"),
               OMP_NUM_THREADS="4")
    # the torch autograd pins do not touch the C oracle and are left out (torch under ASan is slow)
    out = _run([sys.executable, "-m", "pytest", "-q", "-s", "-x", "-p", "no:cacheprovider", "-p", "no:xdist",
                "-k", "not autograd", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                os.path.join(ROOT, "tests", "test_oracle_mutations.py"),
                os.path.join(ROOT, "tests", "test_oracle_cheb.py")], env=env, timeout=900)
    assert " passed" in out.stdout and "failed" not in out.stdout


def test_abi_host_code_under_sanitizers(tmp_path):
    objs = [os.path.join(OBJDIR, f) for f in sorted(os.listdir(OBJDIR))] if os.path.isdir(OBJDIR) else []
    objs = [o for o in objs if o.endswith(".hip.o") and not o.endswith("api.hip.o")]
    if not objs:
        pytest.skip("no objects of a library build under _build/obj (run the build first)")
    api_o = tmp_path / "api.hip.o"
    lib = tmp_path / "liblsefit_san.so"
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++20", "-fPIC", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
          "-I" + INCLUDE, "-I" + CSRC, "-c", os.path.join(CSRC, "api.hip"), "-o", str(api_o)], timeout=900)
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", str(lib), str(api_o), *objs,
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-shared-libsan"], timeout=900)
    env = dict(os.environ, **SAN_ENV, LSEFIT_LIB=str(lib),
               LD_PRELOAD=_runtime("/opt/rocm/llvm/bin/clang", "libclang_rt.asan-x86_64.so"))
    out = _run([sys.executable, "-m", "pytest", "-q", "-s", "-x", "-p", "no:cacheprovider", "-p", "no:xdist",
                "-m", "not gpu", os.path.join(ROOT, "tests", "test_abi.py")], env=env, timeout=900)
    assert " passed" in out.stdout and "failed" not in out.stdout
