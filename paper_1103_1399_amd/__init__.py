"""Python binding of libqaa (include/qaa.h): argument marshalling only.

Every step of the evolution runs in the library's gfx950 kernels; this module
converts arguments (PyTorch tensors give device pointers and streams) and
raises on non-OK status codes.  Importing it without the built library
raises ImportError: there is no fallback path.

The C-ABI names are exported unchanged (``qaa_instance_create``,
``qaa_energy_table``, ``qaa_state_init_uniform``, ``qaa_evolve``,
``qaa_evolve_range``, ``qaa_evolve_batch``, ``qaa_observables``, ...), plus
small conveniences (``Instance``, ``State``) built only from those calls.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# QAA_LIBRARY: load another build of the library (the sanitizer build of the
# host code, paper_1103_1399_amd/sanitize_check.py) instead of the in-tree one.
LIB_PATH = os.environ.get("QAA_LIBRARY") or os.path.join(_HERE, "libqaa.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libqaa is not built (expected at %s); run `python paper_1103_1399_amd/build.py`" % LIB_PATH)

# One HIP runtime per process.  PyTorch's ROCm wheels carry their own copies
# of the HIP and HSA runtimes; when torch is loaded first, libqaa's runtime
# dependency resolves to the copy already in the process.  Loaded the other
# way round, the process holds two runtimes and the second one to start
# finds no usable device.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = ctypes.CDLL(LIB_PATH)

# status codes (qaa_status)
QAA_OK = 0
QAA_ERR_INVALID_ARG = 1
QAA_ERR_UNSUPPORTED = 2
QAA_ERR_OUT_OF_MEMORY = 3
QAA_ERR_DEVICE = 4
QAA_ERR_NOT_READY = 5
QAA_ERR_INTERNAL = 6
QAA_ERR_CANCELLED = 7
# dtypes / table element types
QAA_C64 = 0
QAA_C128 = 1
QAA_E_U8 = 0
QAA_E_U16 = 1
QAA_SCHED_LINEAR = 0
QAA_SCHED_TABLE = 1
QAA_SCHED_MAX_KNOTS = 256
QAA_SPECTRUM_MAX_ITERS = 1024
QAA_MAX_QUBITS = 34


class QaaError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s: %s (%s)" % (where, msg, _lib.qaa_status_str(status).decode()))
        self.status = status


class qaa_state(ctypes.Structure):
    _fields_ = [("inst", ctypes.c_void_p), ("amp", ctypes.c_void_p), ("dtype", ctypes.c_int),
                ("table", ctypes.c_void_p), ("etype", ctypes.c_int)]


class qaa_schedule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("count", ctypes.c_int32), ("values", ctypes.POINTER(ctypes.c_double))]


def make_schedule(knots=None):
    """A qaa_schedule for `knots` (None: the linear schedule s = t/T).

    knots are the values of s at u = j/(len(knots) - 1), u = t/T; the
    returned structure keeps the knot array alive as an attribute.
    """
    if knots is None:
        return qaa_schedule(QAA_SCHED_LINEAR, 0, None)
    vals = [float(v) for v in knots]
    arr = (ctypes.c_double * max(1, len(vals)))(*vals)
    sched = qaa_schedule(QAA_SCHED_TABLE, len(vals), ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)))
    sched._keep = arr
    return sched


class qaa_obs(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double), ("energy", ctypes.c_double), ("p_success", ctypes.c_double),
                ("e_min", ctypes.c_int32), ("degeneracy", ctypes.c_int64)]


class qaa_plan_choice(ctypes.Structure):
    _fields_ = [("balance", ctypes.c_int32), ("passengers", ctypes.c_int32), ("tiles", ctypes.c_int32)]


class qaa_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("slots", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class qaa_server_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("done", ctypes.c_int32), ("obs", qaa_obs),
                ("queued_s", ctypes.c_double), ("latency_s", ctypes.c_double),
                ("steps", ctypes.c_int64), ("steps_done", ctypes.c_int64)]


_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_st = ctypes.c_int

_SIGS = {
    "qaa_instance_create": (_st, [ctypes.c_int32, ctypes.c_int32, _i32p, ctypes.POINTER(_vp)]),
    "qaa_instance_destroy": (None, [_vp]),
    "qaa_instance_info": (_st, [_vp, _i32p, _i32p, _i32p, _i32p, _i64p]),
    "qaa_energy_table": (_st, [_vp, _vp, ctypes.c_int, _vp]),
    "qaa_energy_stats": (_st, [_vp, _vp]),
    "qaa_debug_energy_block": (_st, [_vp, ctypes.c_uint64, _i32p]),
    "qaa_state_init_uniform": (_st, [ctypes.POINTER(qaa_state), _vp]),
    "qaa_state_init_basis": (_st, [ctypes.POINTER(qaa_state), ctypes.c_uint64, _vp]),
    "qaa_evolve": (_st, [ctypes.POINTER(qaa_state), ctypes.POINTER(qaa_schedule), ctypes.c_double,
                         ctypes.c_int64, _vp]),
    "qaa_evolve_range": (_st, [ctypes.POINTER(qaa_state), ctypes.POINTER(qaa_schedule), ctypes.c_double,
                               ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _vp]),
    "qaa_evolve_range_noalloc": (_st, [ctypes.POINTER(qaa_state), ctypes.POINTER(qaa_schedule), ctypes.c_double,
                                       ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _vp]),
    "qaa_evolve_batch": (_st, [ctypes.c_int32, ctypes.POINTER(qaa_state), ctypes.POINTER(qaa_schedule), _f64p,
                               _i64p, _vp]),
    "qaa_observables": (_st, [ctypes.POINTER(qaa_state), ctypes.POINTER(qaa_obs), _vp]),
    "qaa_spectrum": (_st, [_vp, _vp, ctypes.c_int, ctypes.c_int32, _f64p, _vp, ctypes.c_int32, ctypes.c_int32,
                           _f64p, _f64p, _vp]),
    "qaa_debug_tridiag_levels": (_st, [_f64p, _f64p, ctypes.c_int32, ctypes.c_int32, _f64p, _f64p]),
    "qaa_plan_info": (_st, [ctypes.c_int32, ctypes.c_int, _i32p, _i32p, _i32p]),
    "qaa_debug_pass_descs": (_st, [ctypes.c_int32, ctypes.c_int, ctypes.c_int32, ctypes.POINTER(qaa_schedule),
                                   ctypes.c_double, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                   _vp, ctypes.c_int32, _i32p, _i32p]),
    "qaa_profile_enable": (_st, [ctypes.c_int32]),
    "qaa_profile_read": (_st, [ctypes.c_void_p, ctypes.c_int32]),
    "qaa_server_footprint": (ctypes.c_uint64, [ctypes.c_int32, ctypes.c_int32]),
    "qaa_server_create": (_st, [ctypes.POINTER(qaa_server_config), ctypes.POINTER(_vp)]),
    "qaa_server_submit": (_st, [_vp, ctypes.c_int32, ctypes.c_int32, _i32p, ctypes.POINTER(qaa_schedule),
                                ctypes.c_double, ctypes.c_int64, _i64p]),
    "qaa_server_poll": (_st, [_vp, ctypes.c_int64, ctypes.POINTER(qaa_server_result)]),
    "qaa_server_wait": (_st, [_vp, ctypes.c_int64, ctypes.POINTER(qaa_server_result)]),
    "qaa_server_cancel": (_st, [_vp, ctypes.c_int64]),
    "qaa_server_stats": (_st, [_vp, _i64p, _i64p, ctypes.POINTER(ctypes.c_uint64)]),
    "qaa_server_destroy": (None, [_vp]),
    "qaa_plan_get": (_st, [ctypes.c_int32, ctypes.c_int, ctypes.POINTER(qaa_plan_choice)]),
    "qaa_plan_set": (_st, [ctypes.c_int32, ctypes.c_int, ctypes.POINTER(qaa_plan_choice)]),
    "qaa_autotune": (_st, [ctypes.POINTER(qaa_state), ctypes.c_int64, ctypes.POINTER(qaa_plan_choice),
                           ctypes.POINTER(ctypes.c_double), _vp]),
    "qaa_plan_save": (_st, [ctypes.c_char_p]),
    "qaa_plan_load": (_st, [ctypes.c_char_p, _i32p]),
    "qaa_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "qaa_last_error": (ctypes.c_char_p, []),
    "qaa_version": (ctypes.c_int32, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


def _check(status: int, where: str) -> None:
    if status != QAA_OK:
        raise QaaError(status, where, _lib.qaa_last_error().decode())


def _stream_ptr(stream) -> int | None:
    """hipStream_t of a torch stream (None -> torch's current stream)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) or None


# ---------------------------------------------------------------------------
# C-ABI calls, same names
# ---------------------------------------------------------------------------

def qaa_instance_create(n: int, lits) -> int:
    import numpy as np
    arr = np.ascontiguousarray(np.asarray(lits, dtype=np.int32).reshape(-1))
    if arr.size % 3:
        raise ValueError("literal count must be a multiple of 3")
    out = _vp()
    _check(_lib.qaa_instance_create(int(n), arr.size // 3, arr.ctypes.data_as(_i32p), ctypes.byref(out)),
           "qaa_instance_create")
    return out.value


def qaa_instance_destroy(handle: int) -> None:
    _lib.qaa_instance_destroy(handle)


def qaa_instance_info(handle: int) -> dict:
    n, m, emin, emax = (ctypes.c_int32() for _ in range(4))
    deg = ctypes.c_int64()
    _check(_lib.qaa_instance_info(handle, ctypes.byref(n), ctypes.byref(m), ctypes.byref(emin),
                                  ctypes.byref(emax), ctypes.byref(deg)), "qaa_instance_info")
    return {"n": n.value, "m": m.value, "e_min": emin.value, "e_max": emax.value, "degeneracy": deg.value}


def _check_buffer(t, n: int, elem_bytes: int, what: str) -> None:
    """The C ABI takes bare device pointers and cannot see buffer sizes: a
    tensor handed to it must be a contiguous device tensor holding at least
    2^n elements of the expected width."""
    if not getattr(t, "is_cuda", False):
        raise TypeError("%s must be a device tensor" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if t.element_size() != elem_bytes:
        raise TypeError("%s must have %d-byte elements" % (what, elem_bytes))
    if t.numel() < (1 << n):
        raise ValueError("%s holds %d elements, needs 2^%d" % (what, t.numel(), n))


def qaa_energy_table(handle: int, table, etype: int, stream=None) -> None:
    _check_buffer(table, qaa_instance_info(handle)["n"], 1 if int(etype) == QAA_E_U8 else 2, "energy table")
    _check(_lib.qaa_energy_table(handle, table.data_ptr(), int(etype), _stream_ptr(stream)), "qaa_energy_table")


def qaa_debug_energy_block(handle: int, z0: int):
    """E(z0 .. z0 + 31) by the energy kernel's arithmetic, on the host."""
    out = (ctypes.c_int32 * 32)()
    _check(_lib.qaa_debug_energy_block(handle, int(z0), out), "qaa_debug_energy_block")
    return list(out)


def qaa_energy_stats(handle: int, stream=None) -> None:
    """E_min, E_max and the ground-manifold size without building a table."""
    _check(_lib.qaa_energy_stats(handle, _stream_ptr(stream)), "qaa_energy_stats")


def make_state(handle: int, amp, table=None, etype: int | None = None) -> qaa_state:
    import torch
    if amp.dtype == torch.complex64:
        dt = QAA_C64
    elif amp.dtype == torch.complex128:
        dt = QAA_C128
    else:
        raise TypeError("amplitudes must be complex64 or complex128")
    n = qaa_instance_info(handle)["n"]
    _check_buffer(amp, n, amp.element_size(), "amplitudes")
    if table is not None:
        if etype is None:
            etype = QAA_E_U8 if table.dtype == torch.uint8 else QAA_E_U16
        _check_buffer(table, n, 1 if etype == QAA_E_U8 else 2, "energy table")
        tp = table.data_ptr()
    else:
        # no table: recompute mode (energies scored from the clause records;
        # etype is the width they are held in, uint8 unless given)
        tp, etype = None, QAA_E_U8 if etype is None else etype
    return qaa_state(handle, amp.data_ptr(), dt, tp, int(etype))


def qaa_state_init_uniform(state: qaa_state, stream=None) -> None:
    _check(_lib.qaa_state_init_uniform(ctypes.byref(state), _stream_ptr(stream)), "qaa_state_init_uniform")


def qaa_state_init_basis(state: qaa_state, z0: int, stream=None) -> None:
    _check(_lib.qaa_state_init_basis(ctypes.byref(state), int(z0), _stream_ptr(stream)), "qaa_state_init_basis")


def qaa_evolve(state: qaa_state, T: float, steps: int, stream=None, knots=None) -> None:
    """Evolve in place; knots: None (linear schedule) or a schedule table."""
    sched = make_schedule(knots)
    _check(_lib.qaa_evolve(ctypes.byref(state), ctypes.byref(sched), float(T), int(steps), _stream_ptr(stream)),
           "qaa_evolve")


def qaa_evolve_range(state: qaa_state, T: float, steps: int, k0: int, k1: int, stream=None, knots=None) -> None:
    sched = make_schedule(knots)
    _check(_lib.qaa_evolve_range(ctypes.byref(state), ctypes.byref(sched), float(T), int(steps), int(k0), int(k1),
                                 _stream_ptr(stream)), "qaa_evolve_range")


def qaa_evolve_range_noalloc(state: qaa_state, T: float, steps: int, k0: int, k1: int, stream=None,
                             knots=None) -> None:
    """qaa_evolve_range without any device allocation (library-owned static
    scratch; overlapping calls on one device race)."""
    sched = make_schedule(knots)
    _check(_lib.qaa_evolve_range_noalloc(ctypes.byref(state), ctypes.byref(sched), float(T), int(steps), int(k0),
                                         int(k1), _stream_ptr(stream)), "qaa_evolve_range_noalloc")


def qaa_evolve_batch(states, Ts, steps, stream=None, knots=None) -> None:
    """Evolve states together; knots: None (all linear) or one entry per
    state, each None (linear) or a schedule table."""
    cnt = len(states)
    arr = (qaa_state * cnt)(*states)
    t_arr = (ctypes.c_double * cnt)(*[float(t) for t in Ts])
    s_arr = (ctypes.c_int64 * cnt)(*[int(s) for s in steps])
    scheds = None
    if knots is not None:
        if len(knots) != cnt:
            raise ValueError("qaa_evolve_batch: one schedule per state")
        held = [make_schedule(k) for k in knots]
        scheds = (qaa_schedule * cnt)(*held)
    _check(_lib.qaa_evolve_batch(cnt, arr, scheds, t_arr, s_arr, _stream_ptr(stream)), "qaa_evolve_batch")


def qaa_observables(state: qaa_state, stream=None) -> dict:
    out = qaa_obs()
    _check(_lib.qaa_observables(ctypes.byref(state), ctypes.byref(out), _stream_ptr(stream)), "qaa_observables")
    return {"norm": out.norm, "energy": out.energy, "p_success": out.p_success, "e_min": out.e_min,
            "degeneracy": out.degeneracy}


def qaa_spectrum(handle: int, table, etype: int, s_values, v0, iters: int, k: int, stream=None, bounds=False):
    """The k lowest levels of H(s) at each s (Lanczos from the device
    vector v0, float64 of length 2^n): a numpy array [len(s), k], or with
    bounds=True the pair (levels, residual norms)."""
    import numpy as np
    import torch
    if v0.dtype != torch.float64:
        raise TypeError("v0 must be a float64 device tensor")
    n = qaa_instance_info(handle)["n"]
    _check_buffer(v0, n, 8, "v0")
    _check_buffer(table, n, 1 if int(etype) == QAA_E_U8 else 2, "energy table")
    sv = [float(x) for x in s_values]
    cnt = len(sv)
    s_arr = (ctypes.c_double * max(1, cnt))(*sv)
    out = (ctypes.c_double * max(1, cnt * int(k)))()
    bnd = (ctypes.c_double * max(1, cnt * int(k)))() if bounds else None
    _check(_lib.qaa_spectrum(handle, table.data_ptr(), int(etype), cnt, s_arr, v0.data_ptr(), int(iters), int(k),
                             out, bnd, _stream_ptr(stream)), "qaa_spectrum")
    ev = np.frombuffer(out, dtype=np.float64, count=cnt * int(k)).reshape(cnt, int(k)).copy()
    if not bounds:
        return ev
    return ev, np.frombuffer(bnd, dtype=np.float64, count=cnt * int(k)).reshape(cnt, int(k)).copy()


def qaa_debug_tridiag_levels(alpha, beta, k: int):
    """Levels and residual norms qaa_spectrum would report for the
    tridiagonal matrix (alpha, beta); host only."""
    import numpy as np
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    if a.shape != b.shape:
        raise ValueError("alpha and beta must have the same length (beta[m-1] is the last residual)")
    ev = np.empty(int(k))
    bd = np.empty(int(k))
    _check(_lib.qaa_debug_tridiag_levels(a.ctypes.data_as(_f64p), b.ctypes.data_as(_f64p), a.size, int(k),
                                         ev.ctypes.data_as(_f64p), bd.ctypes.data_as(_f64p)),
           "qaa_debug_tridiag_levels")
    return ev, bd


def qaa_plan_info(n: int, dtype: int = QAA_C64) -> dict:
    tb, sets, pps = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.qaa_plan_info(int(n), int(dtype), ctypes.byref(tb), ctypes.byref(sets), ctypes.byref(pps)),
           "qaa_plan_info")
    return {"tile_bits": tb.value, "sets": sets.value, "passes_per_step": pps.value}


class PassDesc(ctypes.Structure):
    """Mirror of the library's internal pass descriptor (diagnostics only)."""
    _fields_ = [("n", ctypes.c_int32), ("n_rest", ctypes.c_int32), ("n_res", ctypes.c_int32),
                ("phase_at", ctypes.c_int32), ("emax", ctypes.c_int32), ("set_id", ctypes.c_int32),
                ("reverse", ctypes.c_int32), ("persist", ctypes.c_int32),
                ("tA", ctypes.c_double), ("sA", ctypes.c_double), ("tB", ctypes.c_double),
                ("sB", ctypes.c_double),
                ("phi", ctypes.c_double), ("gphase", ctypes.c_double),
                ("tile_begin", ctypes.c_uint64), ("tile_count", ctypes.c_uint64),
                ("acc_in", ctypes.c_void_p), ("acc_out", ctypes.c_void_p), ("acc_zero", ctypes.c_void_p),
                ("red_src", ctypes.c_void_p), ("red_dst", ctypes.c_void_p),
                ("clauses", ctypes.c_void_p), ("m", ctypes.c_int32), ("xcd_map", ctypes.c_int32),
                ("reg_bits", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("goff_first", ctypes.c_uint64 * 32), ("goff_last", ctypes.c_uint64 * 32),
                ("ljp", (ctypes.c_uint16 * 32) * 12), ("lj", (ctypes.c_uint16 * 32) * 12),
                ("rest_mask", ctypes.c_uint64),
                ("tile_pos", ctypes.c_uint8 * 16), ("rest_pos", ctypes.c_uint8 * 40),
                ("tpos", (ctypes.c_uint8 * 16) * 12), ("gpos_first", ctypes.c_uint8 * 16),
                ("gpos_last", ctypes.c_uint8 * 16), ("masks", ctypes.c_uint32 * 12)]


def qaa_debug_pass_descs(n: int, dtype: int, emax: int, T: float, steps: int, k0: int, k1: int, knots=None,
                         tile_bits: int = 0):
    """Pass descriptors of the plan (tile_bits 0) or of the same planner's
    plan for smaller tiles (host-side replay only)."""
    count, size = ctypes.c_int32(), ctypes.c_int32()
    sched = make_schedule(knots)
    _check(_lib.qaa_debug_pass_descs(n, dtype, emax, ctypes.byref(sched), T, steps, k0, k1, int(tile_bits), None, 0,
                                     ctypes.byref(count), ctypes.byref(size)), "qaa_debug_pass_descs")
    if size.value != ctypes.sizeof(PassDesc):
        raise RuntimeError("pass descriptor layout mismatch (%d vs %d bytes)" % (size.value, ctypes.sizeof(PassDesc)))
    arr = (PassDesc * max(1, count.value))()
    _check(_lib.qaa_debug_pass_descs(n, dtype, emax, ctypes.byref(sched), T, steps, k0, k1, int(tile_bits), arr,
                                     count.value, ctypes.byref(count), ctypes.byref(size)), "qaa_debug_pass_descs")
    return list(arr)[:count.value]


class qaa_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("kernel_ms", ctypes.c_double), ("min_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double)]


def qaa_profile_enable(on: bool = True) -> None:
    _check(_lib.qaa_profile_enable(1 if on else 0), "qaa_profile_enable")


def qaa_profile_read(reset: bool = True) -> dict:
    out = qaa_profile()
    _check(_lib.qaa_profile_read(ctypes.byref(out), 1 if reset else 0), "qaa_profile_read")
    return {"launches": out.launches, "kernel_ms": out.kernel_ms, "min_ms": out.min_ms, "max_ms": out.max_ms,
            "alg_bytes": out.alg_bytes}


def qaa_plan_get(n: int, dtype: int = QAA_C64) -> dict:
    c = qaa_plan_choice()
    _check(_lib.qaa_plan_get(int(n), int(dtype), ctypes.byref(c)), "qaa_plan_get")
    return {"balance": c.balance, "passengers": c.passengers, "tiles": c.tiles}


def qaa_plan_set(n: int, dtype: int = QAA_C64, choice: dict | None = None) -> None:
    """Record a plan choice for (n, dtype); None restores the default."""
    if choice is None:
        _check(_lib.qaa_plan_set(int(n), int(dtype), None), "qaa_plan_set")
        return
    c = qaa_plan_choice(int(choice["balance"]), int(choice["passengers"]), int(choice.get("tiles", 0)))
    _check(_lib.qaa_plan_set(int(n), int(dtype), ctypes.byref(c)), "qaa_plan_set")


def qaa_plan_save(path: str) -> None:
    _check(_lib.qaa_plan_save(os.fsencode(path)), "qaa_plan_save")


def qaa_plan_load(path: str) -> int:
    count = ctypes.c_int32()
    _check(_lib.qaa_plan_load(os.fsencode(path), ctypes.byref(count)), "qaa_plan_load")
    return count.value


def qaa_autotune(state: qaa_state, steps: int = 20, stream=None) -> dict:
    best = qaa_plan_choice()
    ms = ctypes.c_double()
    _check(_lib.qaa_autotune(ctypes.byref(state), int(steps), ctypes.byref(best), ctypes.byref(ms),
                             _stream_ptr(stream)), "qaa_autotune")
    return {"balance": best.balance, "passengers": best.passengers, "tiles": best.tiles, "ms_per_step": ms.value}


def _result_dict(r: qaa_server_result) -> dict:
    o = r.obs
    return {"status": r.status, "done": bool(r.done), "queued_s": r.queued_s, "latency_s": r.latency_s,
            "steps": r.steps, "steps_done": r.steps_done,
            "norm": o.norm, "energy": o.energy, "p_success": o.p_success, "e_min": o.e_min,
            "degeneracy": o.degeneracy}


def qaa_server_footprint(n: int, m: int) -> int:
    """Device bytes a request is charged at admission (0: out of range)."""
    return int(_lib.qaa_server_footprint(int(n), int(m)))


def qaa_server_create(hbm_budget_bytes: int, slots: int) -> int:
    cfg = qaa_server_config(int(hbm_budget_bytes), int(slots), 0)
    out = _vp()
    _check(_lib.qaa_server_create(ctypes.byref(cfg), ctypes.byref(out)), "qaa_server_create")
    return out.value


def qaa_server_submit(server: int, n: int, lits, T: float, steps: int, knots=None) -> int:
    import numpy as np
    arr = np.ascontiguousarray(np.asarray(lits, dtype=np.int32).reshape(-1))
    sched = make_schedule(knots)
    t = ctypes.c_int64()
    _check(_lib.qaa_server_submit(server, int(n), arr.size // 3, arr.ctypes.data_as(_i32p), ctypes.byref(sched),
                                  float(T), int(steps), ctypes.byref(t)), "qaa_server_submit")
    return t.value


def qaa_server_poll(server: int, ticket: int) -> dict:
    r = qaa_server_result()
    _check(_lib.qaa_server_poll(server, int(ticket), ctypes.byref(r)), "qaa_server_poll")
    return _result_dict(r)


def qaa_server_cancel(server: int, ticket: int) -> None:
    """Cancel a queued or running request (see qaa.h)."""
    _check(_lib.qaa_server_cancel(server, int(ticket)), "qaa_server_cancel")


def qaa_server_wait(server: int, ticket: int) -> dict:
    r = qaa_server_result()
    _check(_lib.qaa_server_wait(server, int(ticket), ctypes.byref(r)), "qaa_server_wait")
    return _result_dict(r)


def qaa_server_stats(server: int) -> dict:
    q, rn, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint64()
    _check(_lib.qaa_server_stats(server, ctypes.byref(q), ctypes.byref(rn), ctypes.byref(b)), "qaa_server_stats")
    return {"queued": q.value, "running": rn.value, "bytes_in_use": b.value}


def qaa_server_destroy(server: int) -> None:
    _lib.qaa_server_destroy(server)


def qaa_status_str(status: int) -> str:
    return _lib.qaa_status_str(int(status)).decode()


def qaa_last_error() -> str:
    return _lib.qaa_last_error().decode()


def qaa_version() -> int:
    return int(_lib.qaa_version())


# ---------------------------------------------------------------------------
# Conveniences built from the calls above
# ---------------------------------------------------------------------------

class Instance:
    """Owns a qaa_instance handle."""

    def __init__(self, n: int, clauses):
        self.n = int(n)
        self.handle = qaa_instance_create(n, clauses)

    def info(self) -> dict:
        return qaa_instance_info(self.handle)

    def energy_stats(self, stream=None) -> dict:
        qaa_energy_stats(self.handle, stream)
        return self.info()

    def energy_table(self, device="cuda", etype: int = QAA_E_U8, stream=None):
        import torch
        dt = torch.uint8 if etype == QAA_E_U8 else torch.int16
        table = torch.empty(1 << self.n, dtype=dt, device=device)
        qaa_energy_table(self.handle, table, etype, stream)
        return table

    def spectrum(self, table, s_values, v0, iters: int, k: int, stream=None, bounds=False):
        """Lowest k levels of H(s) per s (see qaa_spectrum)."""
        import torch
        etype = QAA_E_U8 if table.dtype == torch.uint8 else QAA_E_U16
        return qaa_spectrum(self.handle, table, etype, s_values, v0, iters, k, stream, bounds)

    def close(self):
        if self.handle:
            qaa_instance_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class State:
    """A device state vector bound to an instance and its energy table."""

    def __init__(self, inst: Instance, table, dtype=None, device="cuda", amp=None, etype=None):
        """table None: recompute mode (qaa_energy_stats must have run)."""
        import torch
        self.inst = inst
        self.table = table
        if amp is None:
            amp = torch.empty(1 << inst.n, dtype=dtype or torch.complex64, device=device)
        self.amp = amp
        if table is not None:
            etype = QAA_E_U8 if table.dtype == torch.uint8 else QAA_E_U16
        elif etype is None:
            e_max = inst.info()["e_max"]
            etype = QAA_E_U8 if 0 <= e_max <= 255 else QAA_E_U16
        self.c = make_state(inst.handle, amp, table, etype)

    def init_uniform(self, stream=None):
        qaa_state_init_uniform(self.c, stream)
        return self

    def init_basis(self, z0: int, stream=None):
        qaa_state_init_basis(self.c, z0, stream)
        return self

    def evolve(self, T: float, steps: int, stream=None, knots=None):
        qaa_evolve(self.c, T, steps, stream, knots)
        return self

    def evolve_range(self, T: float, steps: int, k0: int, k1: int, stream=None, knots=None):
        qaa_evolve_range(self.c, T, steps, k0, k1, stream, knots)
        return self

    def observables(self, stream=None) -> dict:
        return qaa_observables(self.c, stream)
