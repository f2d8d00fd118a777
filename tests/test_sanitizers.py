"""AddressSanitizer and UBSan over the host code: the C oracle (gcc) and the
library's host side (hipcc, sanitizers on host code only).  No GPU."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GCC_SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer"]
ASAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:detect_odr_violation=0:alloc_dealloc_mismatch=0:abort_on_error=1",
            "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

ORACLE_DRIVE = r'''
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle
from qaa_inputs import planted_unique_3sat
for n, seed in ((3, 0), (6, 1), (9, 2), (12, 3)):
    inst = planted_unique_3sat(n, seed)
    e = oracle.energy(n, inst.clauses)
    z = np.array([0, (1 << n) - 1, 5 % (1 << n)], np.uint64)
    assert np.array_equal(oracle.energy_at(n, inst.clauses, z), e[z.astype(np.int64)])
    psi = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, psi, 3.0, 12)
    oracle.evolve(n, inst.clauses, psi, 3.0, 12, 3, 9, knots=[0.0, 0.4, 1.0])
    oracle.observables(n, inst.clauses, psi)
    oracle.levels(n, inst.clauses, 0.5, 2)
oracle.energy(4, [])
print("oracle drive: done")
'''


def _gcc_asan():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if p.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def _run_sanitized(code, lib_env, preload, args):
    env = dict(os.environ)
    env.update(ASAN_ENV)
    env.update(lib_env)
    env["LD_PRELOAD"] = preload
    env["OMP_NUM_THREADS"] = "2"
    return subprocess.run([sys.executable, "-c", code] + args, env=env, capture_output=True, text=True,
                          timeout=600)


def test_oracle_clean_under_asan_and_ubsan():
    asan = _gcc_asan()
    if not asan:
        pytest.skip("gcc's ASan runtime is not installed")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "liboracle_san.so")
        subprocess.check_call(["gcc"] + GCC_SAN + ["-fopenmp", "-fPIC", "-shared", "-fcx-limited-range", "-std=c11",
                               "-o", lib, os.path.join(ROOT, "oracle", "qaa_oracle.c"), "-lm"])
        p = _run_sanitized(ORACLE_DRIVE, {"QAA_ORACLE_LIB": lib}, asan, [ROOT])
    out = p.stdout + p.stderr
    assert p.returncode == 0 and "oracle drive: done" in out, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-3000:]


def test_the_sanitizer_harness_reports_an_overflow():
    """The same build flags and runtime catch a heap overflow (a CPU-side
    check that the two tests here are not vacuous)."""
    asan = _gcc_asan()
    if not asan:
        pytest.skip("gcc's ASan runtime is not installed")
    src = "#include <stdlib.h>\nint poke(int i) { int *a = malloc(4 * sizeof(int)); a[i] = 1; int r = a[0]; " \
          "free(a); return r; }\n"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "poke.c")
        lib = os.path.join(d, "libpoke.so")
        with open(c, "w") as f:
            f.write(src)
        subprocess.check_call(["gcc"] + GCC_SAN + ["-fPIC", "-shared", "-o", lib, c])
        code = "import ctypes, sys; ctypes.CDLL(sys.argv[1]).poke(4)"
        p = _run_sanitized(code, {}, asan, [lib])
    assert p.returncode != 0
    assert "heap-buffer-overflow" in p.stderr or "insufficient space" in p.stderr, p.stderr[-2000:]


def test_library_host_code_clean_under_asan_and_ubsan():
    """Builds libqaa with sanitized host code (about a minute) and drives
    every entry point that needs no GPU (paper_1103_1399_amd/sanitize_check.py)."""
    p = subprocess.run([sys.executable, os.path.join(ROOT, "paper_1103_1399_amd", "sanitize_check.py")],
                       capture_output=True, text=True, timeout=1200)
    out = p.stdout + p.stderr
    if p.returncode == 2:
        pytest.skip("no clang ASan runtime under /opt/rocm/llvm")
    assert p.returncode == 0 and "sanitizer check: clean" in out, out[-3000:]
