"""The oracle and the host builds of the kernels' per-state code under AddressSanitizer and UBSan (CPU only).

Builds oracle/oracle_capi.cpp with clang and -fsanitize=address,undefined,
then re-runs the CPU tests that exercise it and the host builds of
sweeps.hpp, team.hpp, jsiia.hpp, hessian.hpp, abi_scan.hpp and fd_scan.hpp (compiled with the same sanitizers on the
host pass only) in a child process with the sanitizer runtime preloaded. Any
out-of-bounds access, use after free or undefined behaviour (signed overflow,
misaligned or null access, invalid shift, ...) aborts the child.
"""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-shared-libasan"]
TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_grad.py", "tests/test_kernel_math_cpu.py",
         "tests/test_team_cpu.py", "tests/test_jsiia_cpu.py", "tests/test_oracle_hessian.py",
         "tests/test_hessian_cpu.py", "tests/test_abi_scan_cpu.py", "tests/test_fd_scan_cpu.py"]


def _runtime():
    hits = glob.glob(os.path.join(ROCM, "llvm", "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so"))
    return hits[0] if hits else None


@pytest.mark.skipif(_runtime() is None, reason="no clang sanitizer runtime in this ROCm installation")
def test_oracle_and_kernel_host_builds_under_asan_ubsan(tmp_path):
    oracle_so = str(tmp_path / "liboracle_asan.so")
    subprocess.run([os.path.join(ROCM, "llvm", "bin", "clang++"), "-std=c++17", "-O1", "-g", "-fPIC", "-shared",
                    "-ffp-contract=off", *SAN, "-o", oracle_so, os.path.join(ROOT, "oracle", "oracle_capi.cpp")],
                   check=True)
    host_flags = " ".join(f"-Xarch_host {f}" for f in SAN) + " -g"  # host pass only: no GPU code is built
    preload = _runtime() + (":" + os.environ["LD_PRELOAD"] if os.environ.get("LD_PRELOAD") else "")
    env = dict(os.environ, PDYN_ORACLE_LIB=oracle_so, PDYN_HOST_BUILD_FLAGS=host_flags, LD_PRELOAD=preload,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    try:  # the modules build their host libraries independently: run them side by side
        import xdist  # noqa: F401
        par = ["-n", str(min(4, len(TESTS), os.cpu_count() or 1))]
    except ImportError:
        par = []
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *par, "-m", "not gpu",
                        *TESTS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
