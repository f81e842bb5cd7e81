"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* oracle.c, built by gcc with -fsanitize=address,undefined, runs the oracle's
  pin battery (tests/test_oracle_pins.py, test_oracle_adjoint_slab.py,
  test_oracle_pencil.py) in a child Python that preloads gcc's ASan runtime.
* The library's host code (argument checks, plan bookkeeping, status
  strings), built by hipcc with the same sanitizers on the host side only,
  runs the C-ABI checks of
  tests/test_abi_cpu.py in a child that preloads clang's ASan runtime (which
  carries the UBSan handlers).

UBSan findings abort (-fno-sanitize-recover); leak checking is off because
the Python interpreter itself is not instrumented.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


def _child_env(preload: str, **extra) -> dict:
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env.update(extra)
    return env


def _run_pytest(files, env, timeout=900):
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu",
           "-p", "no:cacheprovider", *[os.path.join(ROOT, "tests", f) for f in files]]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_pins_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's ASan runtime not installed")
    lib = tmp_path / "liboracle_san.so"
    subprocess.run([gcc, "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "oracle.c"),
                    "-o", str(lib), "-lm"], check=True)
    out = _run_pytest(["test_oracle_pins.py", "test_oracle_adjoint_slab.py",
                       "test_oracle_pencil.py"],
                      _child_env(asan, ORACLE_LIB=str(lib), OMP_NUM_THREADS="4"))
    assert " passed" in out


def test_abi_host_checks_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts:
        pytest.skip("clang's ASan runtime not installed")
    lib = tmp_path / "libgfft_san.so"
    csrc = os.path.join(ROOT, "paper_2202_12756_amd", "csrc")
    # the device code is built as usual (never run here); the sanitizers and
    # their shared runtime apply to the host code only
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-shared-libsan",
                    f"-Wl,-rpath,{os.path.dirname(rts[-1])}",
                    os.path.join(csrc, "kernels.hip"), os.path.join(csrc, "gfft.hip"),
                    "-o", str(lib)], check=True, capture_output=True)
    out = _run_pytest(["test_abi_cpu.py"], _child_env(rts[-1], GFFT_LIB=str(lib)))
    assert " passed" in out
