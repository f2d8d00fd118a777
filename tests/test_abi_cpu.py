"""C-ABI checks that need no GPU: the library loads, exports every function
include/qaa.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT

import paper_1103_1399_amd as qaa


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "qaa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(qaa_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ["qaa_instance_create", "qaa_instance_destroy", "qaa_instance_info", "qaa_energy_table",
                 "qaa_state_init_uniform", "qaa_evolve", "qaa_evolve_range", "qaa_evolve_batch",
                 "qaa_observables", "qaa_status_str", "qaa_last_error"]:
        assert must in names


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(qaa.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name
    # and the binding wraps each of them under the same name
    for name in _declared_functions():
        assert hasattr(qaa, name), name


def test_status_strings():
    assert qaa.qaa_status_str(qaa.QAA_OK) == "ok"
    assert qaa.qaa_status_str(qaa.QAA_ERR_INVALID_ARG) == "invalid argument"
    assert qaa.qaa_status_str(99) == "unknown status"
    assert qaa.qaa_version() >= 100


@pytest.mark.parametrize("n,lits,msg", [
    (0, [], "n=0"),
    (35, [], "n=35"),
    (4, [1, 2, 5], "out of range"),
    (4, [1, 0, 2], "out of range"),
    (4, [1, -1, 2], "repeats a variable"),
    (4, [3, 2, 3], "repeats a variable"),
])
def test_instance_create_rejects(n, lits, msg):
    with pytest.raises(qaa.QaaError) as ei:
        qaa.qaa_instance_create(n, lits)
    assert ei.value.status == qaa.QAA_ERR_INVALID_ARG
    assert msg in str(ei.value)


def test_instance_create_and_info_without_table():
    lits = [1, -2, 3, -1, 2, 4, 2, 3, 4, 2, 3, 4]   # duplicate clause allowed
    h = qaa.qaa_instance_create(4, lits)
    try:
        info = qaa.qaa_instance_info(h)
        assert info == {"n": 4, "m": 4, "e_min": -1, "e_max": -1, "degeneracy": -1}
    finally:
        qaa.qaa_instance_destroy(h)
    qaa.qaa_instance_destroy(None)   # NULL is ignored


def test_zero_clause_instance():
    h = qaa.qaa_instance_create(1, [])
    assert qaa.qaa_instance_info(h)["m"] == 0
    qaa.qaa_instance_destroy(h)


def test_evolve_rejects_before_any_device_call():
    h = qaa.qaa_instance_create(5, [1, 2, 3])
    try:
        st = qaa.qaa_state(h, 0x1000, qaa.QAA_C64, 0x2000, qaa.QAA_E_U8)
        sched = qaa.qaa_schedule(qaa.QAA_SCHED_LINEAR)
        lib = qaa._lib
        # energy table not computed yet -> NOT_READY
        rc = lib.qaa_evolve(ctypes.byref(st), ctypes.byref(sched), 1.0, 10, None)
        assert rc == qaa.QAA_ERR_NOT_READY
        assert "qaa_energy_table" in qaa.qaa_last_error()
        # the allocation-free variant validates the same way, before it
        # looks up its device scratch
        rc = lib.qaa_evolve_range_noalloc(ctypes.byref(st), ctypes.byref(sched), 1.0, 10, 0, 10, None)
        assert rc == qaa.QAA_ERR_NOT_READY
        assert "qaa_evolve_range_noalloc" in qaa.qaa_last_error()
        assert lib.qaa_evolve_range_noalloc(None, None, 1.0, 10, 0, 10, None) == qaa.QAA_ERR_INVALID_ARG
        # NULL state / missing buffers
        assert lib.qaa_evolve(None, None, 1.0, 10, None) == qaa.QAA_ERR_INVALID_ARG
        bad = qaa.qaa_state(h, None, qaa.QAA_C64, 0x2000, qaa.QAA_E_U8)
        assert lib.qaa_evolve(ctypes.byref(bad), None, 1.0, 10, None) == qaa.QAA_ERR_INVALID_ARG
        bad = qaa.qaa_state(h, 0x1000, 7, 0x2000, qaa.QAA_E_U8)
        assert lib.qaa_evolve(ctypes.byref(bad), None, 1.0, 10, None) == qaa.QAA_ERR_INVALID_ARG
        assert lib.qaa_observables(ctypes.byref(st), None, None) == qaa.QAA_ERR_INVALID_ARG
        out = qaa.qaa_obs()
        assert lib.qaa_observables(ctypes.byref(st), ctypes.byref(out), None) == qaa.QAA_ERR_NOT_READY
        assert lib.qaa_energy_table(h, None, 0, None) == qaa.QAA_ERR_INVALID_ARG
        assert lib.qaa_energy_table(h, 0x1000, 5, None) == qaa.QAA_ERR_INVALID_ARG
        assert lib.qaa_evolve_batch(-1, None, None, None, None, None) == qaa.QAA_ERR_INVALID_ARG
        assert lib.qaa_evolve_batch(0, None, None, None, None, None) == qaa.QAA_OK
    finally:
        qaa.qaa_instance_destroy(h)


@pytest.mark.parametrize("sched,msg", [
    (dict(kind=7), "unknown schedule kind"),
    (dict(kind=1, count=1, values=[0.0]), "2..256 knots"),
    (dict(kind=1, count=257, values=[0.5] * 257), "2..256 knots"),
    (dict(kind=1, count=3, values=None), "values is NULL"),
    (dict(kind=1, count=3, values=[0.0, float("nan"), 1.0]), "knot 1"),
    (dict(kind=1, count=3, values=[0.0, 0.5, 1.5]), "knot 2"),
    (dict(kind=1, count=2, values=[-0.25, 1.0]), "knot 0"),
])
def test_bad_schedules_are_rejected(sched, msg):
    """Schedule tables are checked before anything touches the device, in
    every call that takes one."""
    vals = sched.get("values")
    arr = None if vals is None else (ctypes.c_double * len(vals))(*vals)
    sc = qaa.qaa_schedule(sched["kind"], sched.get("count", 0),
                          None if arr is None else ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)))
    h = qaa.qaa_instance_create(5, [1, 2, 3])
    try:
        st = qaa.qaa_state(h, 0x1000, qaa.QAA_C64, 0x2000, qaa.QAA_E_U8)
        lib = qaa._lib
        assert lib.qaa_evolve(ctypes.byref(st), ctypes.byref(sc), 1.0, 10, None) == qaa.QAA_ERR_INVALID_ARG
        assert msg in qaa.qaa_last_error()
        assert lib.qaa_evolve_range(ctypes.byref(st), ctypes.byref(sc), 1.0, 10, 0, 5, None) == \
            qaa.QAA_ERR_INVALID_ARG
        states = (qaa.qaa_state * 1)(st)
        scheds = (qaa.qaa_schedule * 1)(sc)
        t_arr = (ctypes.c_double * 1)(1.0)
        n_arr = (ctypes.c_int64 * 1)(10)
        assert lib.qaa_evolve_batch(1, states, scheds, t_arr, n_arr, None) == qaa.QAA_ERR_INVALID_ARG
        assert msg in qaa.qaa_last_error()
        cnt, size = ctypes.c_int32(), ctypes.c_int32()
        assert lib.qaa_debug_pass_descs(20, 0, 10, ctypes.byref(sc), 1.0, 10, 0, 10, 0, None, 0, ctypes.byref(cnt),
                                        ctypes.byref(size)) == qaa.QAA_ERR_INVALID_ARG
    finally:
        qaa.qaa_instance_destroy(h)


def test_good_schedule_passes_to_the_state_checks():
    """A valid table gets past the schedule check (the missing energy table
    is what stops it), and the linear kind ignores count and values."""
    h = qaa.qaa_instance_create(5, [1, 2, 3])
    try:
        st = qaa.qaa_state(h, 0x1000, qaa.QAA_C64, 0x2000, qaa.QAA_E_U8)
        lib = qaa._lib
        for sc in (qaa.make_schedule([0.0, 0.3, 1.0]), qaa.make_schedule([1.0] * 256),
                   qaa.qaa_schedule(qaa.QAA_SCHED_LINEAR, 99, None)):
            assert lib.qaa_evolve(ctypes.byref(st), ctypes.byref(sc), 1.0, 10, None) == qaa.QAA_ERR_NOT_READY
    finally:
        qaa.qaa_instance_destroy(h)


@pytest.mark.parametrize("n,dtype,expect", [
    (6, 0, (0, 1, 0)),
    (13, 0, (0, 1, 0)),
    (14, 0, (13, 2, 1)),
    (21, 0, (13, 2, 1)),
    (22, 0, (13, 2, 1)),        # the top set in a 2^14 tile holds the 9 high qubits
    (23, 0, (14, 2, 1)),        # 14 + 9: every set in 2^14 tiles, two sets
    (24, 0, (13, 3, 2)),
    (28, 0, (13, 3, 2)),
    (29, 0, (13, 3, 2)),
    (30, 0, (13, 3, 2)),        # 13 + 8 + 9: the top set in a 2^14 tile
    (31, 0, (14, 3, 2)),        # 14 + 9 + 8: every set in 2^14 tiles
    (33, 0, (13, 4, 3)),
    (34, 0, (13, 4, 3)),
    (12, 1, (0, 1, 0)),
    (13, 1, (12, 2, 1)),
    (28, 1, (12, 3, 2)),
    (29, 1, (12, 4, 3)),
])
def test_plan_info(n, dtype, expect):
    p = qaa.qaa_plan_info(n, dtype)
    assert (p["tile_bits"], p["sets"], p["passes_per_step"]) == expect


def test_plan_info_rejects():
    with pytest.raises(qaa.QaaError):
        qaa.qaa_plan_info(0)
    with pytest.raises(qaa.QaaError):
        qaa.qaa_plan_info(10, 3)


def test_server_create_rejects_bad_config():
    lib = qaa._lib
    out = ctypes.c_void_p()
    assert lib.qaa_server_create(None, ctypes.byref(out)) == qaa.QAA_ERR_INVALID_ARG
    for slots, budget in [(0, 1 << 30), (65, 1 << 30), (2, 0)]:
        cfg = qaa.qaa_server_config(budget, slots, 0)
        assert lib.qaa_server_create(ctypes.byref(cfg), ctypes.byref(out)) == qaa.QAA_ERR_INVALID_ARG
        assert out.value is None
    cfg = qaa.qaa_server_config(1 << 30, 2, 0)
    assert lib.qaa_server_create(ctypes.byref(cfg), None) == qaa.QAA_ERR_INVALID_ARG
    # calls on a NULL server are rejected, destroy ignores it
    t = ctypes.c_int64()
    lits = (ctypes.c_int32 * 3)(1, 2, 3)
    assert lib.qaa_server_submit(None, 3, 1, lits, None, 1.0, 10, ctypes.byref(t)) == qaa.QAA_ERR_INVALID_ARG
    r = qaa.qaa_server_result()
    assert lib.qaa_server_poll(None, 1, ctypes.byref(r)) == qaa.QAA_ERR_INVALID_ARG
    assert lib.qaa_server_wait(None, 1, ctypes.byref(r)) == qaa.QAA_ERR_INVALID_ARG
    assert lib.qaa_server_stats(None, None, None, None) == qaa.QAA_ERR_INVALID_ARG
    lib.qaa_server_destroy(None)


def test_one_hip_runtime_in_process():
    # the binding loads torch first, so libqaa shares torch's HIP runtime
    # instead of mapping a second copy that would compete for the device
    pytest.importorskip("torch")
    maps = open("/proc/self/maps").read().splitlines()
    hip = {line.split()[-1] for line in maps if "libamdhip64" in line}
    assert len(hip) == 1, hip


def test_library_carries_roctx_ranges():
    # API calls and pass launches are named for rocprofv3 --marker-trace
    maps = open("/proc/self/maps").read()
    assert "librocprofiler-sdk-roctx" in maps


def _bp(choice):
    return {"balance": choice["balance"], "passengers": choice["passengers"]}


def test_plan_choice_defaults_set_and_reset():
    assert _bp(qaa.qaa_plan_get(16)) == {"balance": 1, "passengers": 0}      # two sets
    assert qaa.qaa_plan_get(16)["tiles"] == 0                                # below n = 22: base tiles only
    assert _bp(qaa.qaa_plan_get(28)) == {"balance": 0, "passengers": 1}      # three sets
    default28 = qaa.qaa_plan_get(28)
    try:
        qaa.qaa_plan_set(28, qaa.QAA_C64, {"balance": 1, "passengers": 0, "tiles": 2})
        assert qaa.qaa_plan_get(28) == {"balance": 1, "passengers": 0, "tiles": 2}
        assert qaa.qaa_plan_info(28)["tile_bits"] == 14
        assert qaa.qaa_plan_get(28, qaa.QAA_C128)["tiles"] == 0          # per dtype; complex128: base tiles
        qaa.qaa_plan_set(28, qaa.QAA_C128, {"balance": 0, "passengers": 1, "tiles": 2})
        assert qaa.qaa_plan_get(28, qaa.QAA_C128)["tiles"] == 0          # recorded but not applicable
        assert qaa.qaa_plan_info(28, qaa.QAA_C128)["tile_bits"] == 12
    finally:
        qaa.qaa_plan_set(28, qaa.QAA_C64, None)
        qaa.qaa_plan_set(28, qaa.QAA_C128, None)
    assert qaa.qaa_plan_get(28) == default28
    lib = qaa._lib
    for bad in (qaa.qaa_plan_choice(2, 0, 0), qaa.qaa_plan_choice(0, 0, 3), qaa.qaa_plan_choice(0, 0, -1)):
        assert lib.qaa_plan_set(28, 0, ctypes.byref(bad)) == qaa.QAA_ERR_INVALID_ARG
    assert lib.qaa_plan_set(35, 0, None) == qaa.QAA_ERR_INVALID_ARG
    assert lib.qaa_plan_get(28, 0, None) == qaa.QAA_ERR_INVALID_ARG
    assert lib.qaa_autotune(None, 10, None, None, None) == qaa.QAA_ERR_INVALID_ARG


def test_spectrum_rejects_before_any_device_call():
    h = qaa.qaa_instance_create(5, [1, 2, 3])
    lib = qaa._lib
    s_ok = (ctypes.c_double * 2)(0.2, 0.8)
    out = (ctypes.c_double * 8)()
    try:
        def call(inst=h, table=0x1000, etype=0, count=2, svals=s_ok, v0=0x2000, iters=10, k=2, ev=out):
            return lib.qaa_spectrum(inst, table, etype, count, svals, v0, iters, k, ev, None, None)
        assert call(inst=None) == qaa.QAA_ERR_INVALID_ARG
        assert call(table=None) == qaa.QAA_ERR_INVALID_ARG
        assert call(v0=None) == qaa.QAA_ERR_INVALID_ARG
        assert call(etype=4) == qaa.QAA_ERR_INVALID_ARG
        assert call(count=-1) == qaa.QAA_ERR_INVALID_ARG
        assert call(svals=None) == qaa.QAA_ERR_INVALID_ARG
        assert call(iters=0) == qaa.QAA_ERR_INVALID_ARG
        assert call(iters=qaa.QAA_SPECTRUM_MAX_ITERS + 1) == qaa.QAA_ERR_INVALID_ARG
        assert call(k=0) == qaa.QAA_ERR_INVALID_ARG
        assert call(k=11) == qaa.QAA_ERR_INVALID_ARG
        bad = (ctypes.c_double * 2)(0.2, 1.5)
        assert call(svals=bad) == qaa.QAA_ERR_INVALID_ARG
        assert "s_values[1]" in qaa.qaa_last_error()
        assert call(v0=0x2004) == qaa.QAA_ERR_INVALID_ARG
        # everything valid but no energy table yet
        assert call() == qaa.QAA_ERR_NOT_READY
        assert call(count=0) == qaa.QAA_ERR_NOT_READY
    finally:
        qaa.qaa_instance_destroy(h)


def test_binding_checks_buffers_before_handing_pointers_over():
    """The C ABI sees bare pointers; the binding refuses host tensors and
    buffers too small for 2^n elements instead of passing them on."""
    import torch
    h = qaa.qaa_instance_create(6, [1, 2, 3])
    try:
        with pytest.raises(TypeError, match="device tensor"):
            qaa.make_state(h, torch.zeros(64, dtype=torch.complex64))
        with pytest.raises(TypeError, match="device tensor"):
            qaa.qaa_energy_table(h, torch.zeros(64, dtype=torch.uint8), qaa.QAA_E_U8)
        with pytest.raises(TypeError, match="device tensor"):
            qaa.qaa_spectrum(h, torch.zeros(64, dtype=torch.uint8), qaa.QAA_E_U8, [0.5],
                             torch.zeros(64, dtype=torch.float64), 10, 1)
        with pytest.raises(TypeError, match="float64"):
            qaa.qaa_spectrum(h, torch.zeros(64, dtype=torch.uint8), qaa.QAA_E_U8, [0.5],
                             torch.zeros(64, dtype=torch.float32), 10, 1)
    finally:
        qaa.qaa_instance_destroy(h)


def test_plan_choices_save_and_load(tmp_path):
    """Plan choices round-trip through a file; malformed lines are skipped."""
    path = str(tmp_path / "plans.txt")
    try:
        qaa.qaa_plan_set(27, qaa.QAA_C64, {"balance": 1, "passengers": 0, "tiles": 1})
        qaa.qaa_plan_set(20, qaa.QAA_C128, {"balance": 0, "passengers": 0, "tiles": 0})
        qaa.qaa_plan_save(path)
        text = open(path).read()
        assert "27 0 1 0 1" in text and "20 1 0 0 0" in text
        qaa.qaa_plan_set(27, qaa.QAA_C64, None)
        qaa.qaa_plan_set(20, qaa.QAA_C128, None)
        with open(path, "a") as f:
            f.write("garbage line\n99 0 1 1 1\n26 0 0 1 7\n")
        assert qaa.qaa_plan_load(path) == 2
        assert qaa.qaa_plan_get(27) == {"balance": 1, "passengers": 0, "tiles": 1}
    finally:
        qaa.qaa_plan_set(27, qaa.QAA_C64, None)
        qaa.qaa_plan_set(20, qaa.QAA_C128, None)
    with pytest.raises(qaa.QaaError):
        qaa.qaa_plan_load(str(tmp_path / "missing.txt"))


def test_autotune_cache_is_read_before_the_first_plan(tmp_path):
    """A process started with QAA_AUTOTUNE_CACHE naming a plan file uses its
    choices from the first plan lookup on (no GPU needed to plan)."""
    import subprocess
    import sys
    path = tmp_path / "cache.txt"
    path.write_text("# tuned\n28 0 1 0 2\n")
    code = ("import paper_1103_1399_amd as q; p = q.qaa_plan_get(28); i = q.qaa_plan_info(28); "
            "print(p['balance'], p['passengers'], p['tiles'], i['tile_bits'])")
    env = dict(os.environ, QAA_AUTOTUNE_CACHE=str(path))
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["1", "0", "2", "14"]
