"""Run the library's host code under AddressSanitizer and UBSan.

Builds libqaa with the sanitizers on its host code only (the GPU code is
compiled as usual, not instrumented) into a temporary directory, then, in
a child process with the sanitizer runtime preloaded, drives every entry
point that works without a GPU: clause-list validation and encoding,
instance info, the pass planner over n = 14..34 for both amplitude types
and several plan choices (including step ranges, schedule tables and the
smaller-tile replays), plan files, the bit-sliced energy model and the
tridiagonal eigenvalue solver.  Exit status 0 when the drive finishes with
no sanitizer report.

    python paper_1103_1399_amd/sanitize_check.py
"""
import concurrent.futures
import glob
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, HERE)
import build as qaa_build  # noqa: E402

SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_sanitized(out_dir):
    flags = [f for f in qaa_build.HIP_FLAGS if f not in ("-O3", "-shared")] + ["-O1", "-g"]
    objs = []

    def compile_one(src):
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        subprocess.check_call([qaa_build.hipcc()] + flags + SANITIZE + ["-c", "-I", os.path.join(ROOT, "include"),
                              "-I", qaa_build.CSRC, os.path.join(qaa_build.CSRC, src), "-o", obj])
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=len(qaa_build.SOURCES)) as ex:
        objs = list(ex.map(compile_one, qaa_build.SOURCES))
    lib = os.path.join(out_dir, "libqaa_sanitized.so")
    subprocess.check_call([qaa_build.hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + SANITIZE + objs +
                          qaa_build.LINK_FLAGS + ["-o", lib])
    return lib


DRIVE = r'''
import json, os, sys, tempfile
sys.path.insert(0, sys.argv[1])
import numpy as np
import paper_1103_1399_amd as qaa
from qaa_inputs import planted_unique_3sat
assert qaa.LIB_PATH == os.environ["QAA_LIBRARY"]
for n in (1, 3, 10, 20, 28, 34):
    h = qaa.qaa_instance_create(n, planted_unique_3sat(min(n, 18), 1).literals() if n >= 3 else [])
    qaa.qaa_instance_info(h)
    qaa.qaa_instance_destroy(h)
for n, bad in ((5, [0, 1, 2]), (5, [1, 1, 2]), (5, [1, 2, 99]), (0, [1, 2, 3]), (99, [1, 2, 3])):
    try:
        qaa.qaa_instance_create(n, np.asarray(bad, np.int32))
        raise SystemExit("accepted a bad instance")
    except qaa.QaaError:
        pass
for n in range(14, 35):
    for dt in (qaa.QAA_C64, qaa.QAA_C128):
        qaa.qaa_plan_info(n, dt)
        qaa.qaa_debug_pass_descs(n, dt, 20, 5.0, 7, 0, 7)
        qaa.qaa_debug_pass_descs(n, dt, 300, 5.0, 9, 2, 5, knots=[0.0, 0.3, 1.0])
for n in (22, 24, 28, 30):
    for ch in ({"balance": 1, "passengers": 0, "tiles": 0}, {"balance": 0, "passengers": 1, "tiles": 1},
               {"balance": 0, "passengers": 1, "tiles": 2}):
        qaa.qaa_plan_set(n, qaa.QAA_C64, ch)
        qaa.qaa_debug_pass_descs(n, qaa.QAA_C64, 20, 5.0, 5, 0, 5)
    qaa.qaa_plan_set(n, qaa.QAA_C64, None)
for n, tb in ((16, 10), (18, 9), (20, 10), (21, 11)):
    qaa.qaa_debug_pass_descs(n, qaa.QAA_C64, 20, 5.0, 3, 0, 3, tile_bits=tb)
with tempfile.TemporaryDirectory() as d:
    path = os.path.join(d, "plans.txt")
    qaa.qaa_plan_set(24, qaa.QAA_C64, {"balance": 1, "passengers": 0, "tiles": 1})
    qaa.qaa_plan_save(path)
    qaa.qaa_plan_set(24, qaa.QAA_C64, None)
    qaa.qaa_plan_load(path)
    qaa.qaa_plan_set(24, qaa.QAA_C64, None)
    with open(path, "w") as f:
        f.write("garbage line\n24 0 x 1 1\n")
    try:
        qaa.qaa_plan_load(path)
    except qaa.QaaError:
        pass
inst = planted_unique_3sat(16, 2)
h = qaa.qaa_instance_create(16, inst.literals())
for z0 in (0, 32, 65504):
    qaa.qaa_debug_energy_block(h, z0)
qaa.qaa_instance_destroy(h)
rng = np.random.default_rng(0)
for m in (1, 2, 5, 40):
    a = rng.standard_normal(m)
    b = np.abs(rng.standard_normal(m)) + 0.1
    qaa.qaa_debug_tridiag_levels(a, b, min(3, m))
print("sanitized drive: done")
'''


def main():
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt:
        print("no clang ASan runtime found", file=sys.stderr)
        return 2
    with tempfile.TemporaryDirectory() as d:
        lib = build_sanitized(d)
        env = dict(os.environ)
        env.update({"QAA_LIBRARY": lib, "LD_PRELOAD": rt[0],
                    "ASAN_OPTIONS": "detect_leaks=0:detect_odr_violation=0:alloc_dealloc_mismatch=0:abort_on_error=1",
                    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
        p = subprocess.run([sys.executable, "-c", DRIVE, ROOT], env=env, capture_output=True, text=True,
                           timeout=900)
    out = p.stdout + p.stderr
    bad = p.returncode != 0 or "AddressSanitizer" in out or "runtime error:" in out
    sys.stdout.write(out[-4000:])
    print("sanitizer check: %s" % ("FAILED" if bad else "clean"))
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main())
