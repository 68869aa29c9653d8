"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds the oracle (g++) and the library's host code (hipcc; the device code
is built as usual, only the host pass is instrumented) with
-fsanitize=address,undefined into a temporary directory, then runs, in
subprocesses with the sanitizer runtimes preloaded into the interpreter:
  * oracle checks: the hand example, brute force on random small graphs with
    the row membership test, sorting and fingerprints;
  * the library's CPU tests (symbols, structure layouts, the host-side planner,
    host-side argument checks) through its ctypes binding.
Any sanitizer report fails the run (halt_on_error; leaks are not checked, the
interpreter itself holds memory until exit).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _clang_asan():
    base = "/opt/rocm/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for ver in sorted(os.listdir(base), reverse=True):
        path = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(path):
            return path
    return None


ORACLE_CHECKS = r"""
import sys
sys.path.insert(0, %(root)r)
import numpy as np
import oracle
from tests import pins
from tests.cases import load_hand_example, random_small_graph, random_small_pattern
from synth.patterns import ISO, MONO
assert oracle._LIB == %(lib)r, oracle._LIB
g, cases = load_hand_example()
for name, p, mode, rows in cases:
    r = oracle.match(g, p, mode)
    assert r.count == rows.shape[0], name
for seed in range(40):
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(2, 8))
    g = random_small_graph(rng, n, float(rng.uniform(0.2, 0.8)), int(rng.integers(1, 3)),
                           int(rng.integers(1, 3)))
    k = int(rng.integers(1, min(n, 4) + 1))
    p = random_small_pattern(rng, k, len(g.vcols), len(g.ecols), connected=seed %% 4 != 0)
    for mode in (ISO, MONO):
        want = pins.brute(g, p, mode)
        got = oracle.match(g, p, mode, threads=1 + seed %% 3)
        assert got.count == want.shape[0]
        assert (got.rows == want).all()
        assert (oracle.check_rows(g, p, mode, want, threads=2) == 1).all()
        assert oracle.fingerprint(oracle.sort_rows(got.rows)) == got.fingerprint
        oracle.match(g, p, mode, threads=2, rows=False, max_tested=3)
print("oracle checks passed")
"""


def _run(cmd, env, timeout):
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=timeout, cwd=ROOT)
    report = [l for l in (r.stdout + r.stderr).splitlines()
              if "ERROR: AddressSanitizer" in l or "runtime error:" in l or "SUMMARY:" in l]
    assert r.returncode == 0 and not report, (r.returncode, report[:10], r.stderr[-3000:])
    return r.stdout


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
                    "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-o", lib,
                    os.path.join(ROOT, "oracle", "hpm_oracle.cpp")], check=True)
    env = dict(os.environ, HPM_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    script = tmp_path / "checks.py"
    script.write_text(ORACLE_CHECKS % {"root": ROOT, "lib": lib})
    assert "oracle checks passed" in _run([sys.executable, str(script)], env, 600)


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    asan = _clang_asan()
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not asan or not os.path.exists(hipcc):
        pytest.skip("hipcc or the clang sanitizer runtime not installed")
    from paper_2507_04130_amd import build as hb
    lib = str(tmp_path / "libhpm_san.so")
    cmd = [hipcc, f"--offload-arch={hb.ARCH}", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"),
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan",
           "-o", lib] + [os.path.join(hb.CSRC, s) for s in hb.SOURCES]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, HPM_LIBRARY=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:protect_shadow_gap=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                os.path.join(ROOT, "tests", "test_lib_cpu.py"),
                os.path.join(ROOT, "tests", "test_sanitizers_probe.py")], env, 900)
    assert " passed" in out and "skipped" not in out, out[-500:]
    shutil.rmtree(tmp_path, ignore_errors=True)
