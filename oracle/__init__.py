"""CPU oracle for the adiabatic 3-SAT evolution -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library (``paper_1103_1399_amd``) never
imports it and shares no code with it.

The arithmetic lives in ``qaa_oracle.c`` (plain C, complex128, OpenMP over
basis states); this module is ctypes marshalling plus two numpy helpers that
build dense matrices for the small-n pins.  Every function states which part
of the paper it follows:

* energy, energy_at -- Sec. 4.3: E(z) = number of clauses the assignment z
                      leaves unsatisfied; literals as in Sec. 2.2; x_i is bit
                      (i-1) of z (basis order |q_n ... q_1> of Sec. 2.1).
* init_uniform     -- Sec. 2.1: uniform superposition, the ground state of
                      H_B = sum_i (1 - sigma^x_i)/2.
* evolve           -- eq. 1 of Sec. 2.1, H(s) = (1-s) H_B + s H_P with s = t/T
                      (or s(t/T) from a piecewise-linear schedule table),
                      integrated by N second-order (Strang) steps with the
                      schedule evaluated at step midpoints (the paper is silent
                      on the integrator; this reading is the documented one).
* observables      -- norm, <H_P>, and the success probability: the weight on
                      the ground manifold of H_P (Sec. 2.1), i.e. on all z with
                      E(z) = E_min.
* levels           -- the lowest distinct eigenvalues of H(s) = (1-s) H_B + s H_P
                      (eq. 1): the spectrum whose lowest gap sets how slowly
                      the sweep must go (Sec. 2.1).  Dense ``eigvalsh`` for
                      n <= 11, else scipy ``eigsh`` on a matrix-free H(s).
* dense_h_b / dense_strang_step -- small-n dense matrices used only to pin
                      the oracle (scipy ``expm``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qaa_oracle.c")
# QAA_ORACLE_LIB: load another build of the C oracle (the sanitizer build of
# tests/test_sanitizers.py) instead of oracle/liboracle.so.
_LIB = os.environ.get("QAA_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fcx-limited-range",
               "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            lib = ctypes.CDLL(_LIB)
            i32p = ctypes.POINTER(ctypes.c_int32)
            f64p = ctypes.POINTER(ctypes.c_double)
            i64p = ctypes.POINTER(ctypes.c_int64)
            lib.oracle_energy.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p]
            lib.oracle_energy.restype = ctypes.c_int
            lib.oracle_energy_at.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.c_int64, i32p]
            lib.oracle_energy_at.restype = ctypes.c_int
            lib.oracle_init_uniform.argtypes = [ctypes.c_int, f64p]
            lib.oracle_init_uniform.restype = None
            lib.oracle_evolve.argtypes = [ctypes.c_int, ctypes.c_int, i32p, f64p, ctypes.c_double,
                                          ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, f64p, ctypes.c_int]
            lib.oracle_evolve.restype = ctypes.c_int
            lib.oracle_observables.argtypes = [ctypes.c_int, ctypes.c_int, i32p, f64p, f64p, i32p, i64p]
            lib.oracle_observables.restype = ctypes.c_int
            lib.oracle_num_threads.argtypes = []
            lib.oracle_num_threads.restype = ctypes.c_int
            lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
            lib.oracle_set_num_threads.restype = None
            _lib = lib
    return _lib


def _lits(clauses) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(clauses, dtype=np.int32).reshape(-1, 3))
    return a


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(t: int) -> None:
    """Threads the oracle's OpenMP loops use from now on (timing only)."""
    _load().oracle_set_num_threads(int(t))


def energy(n: int, clauses) -> np.ndarray:
    """E(z) for z = 0 .. 2^n - 1 (int32), Sec. 4.3 energy function."""
    lits = _lits(clauses)
    out = np.empty(1 << n, dtype=np.int32)
    rc = _load().oracle_energy(n, lits.shape[0], _ptr(lits, ctypes.c_int32), _ptr(out, ctypes.c_int32))
    if rc != 0:
        raise ValueError("literal out of range")
    return out


def energy_at(n: int, clauses, zs) -> np.ndarray:
    """E(z) for the given basis states only (Sec. 4.3 energy function)."""
    lits = _lits(clauses)
    z = np.ascontiguousarray(np.asarray(zs, dtype=np.uint64))
    out = np.empty(z.size, dtype=np.int32)
    rc = _load().oracle_energy_at(n, lits.shape[0], _ptr(lits, ctypes.c_int32), _ptr(z, ctypes.c_uint64),
                                  z.size, _ptr(out, ctypes.c_int32))
    if rc != 0:
        raise ValueError("literal out of range")
    return out


def init_uniform(n: int) -> np.ndarray:
    """Uniform superposition 2^{-n/2} sum_z |z> (Sec. 2.1), complex128."""
    psi = np.empty(1 << n, dtype=np.complex128)
    _load().oracle_init_uniform(n, _ptr(psi.view(np.float64), ctypes.c_double))
    return psi


def evolve(n: int, clauses, psi: np.ndarray, T: float, N: int, k0: int = 0, k1: int | None = None,
           knots=None) -> np.ndarray:
    """Apply steps k0 .. k1-1 of the N-step second-order evolution (in place).

    psi must be a C-contiguous complex128 array of length 2^n.  knots: None
    (linear schedule s = t/T) or the values of s at u = j/(len - 1).
    """
    if k1 is None:
        k1 = N
    if psi.dtype != np.complex128 or not psi.flags.c_contiguous or psi.shape != (1 << n,):
        raise ValueError("psi must be contiguous complex128 of length 2^n")
    lits = _lits(clauses)
    kn = np.ascontiguousarray(np.asarray([] if knots is None else knots, dtype=np.float64))
    kn_ptr = _ptr(kn, ctypes.c_double) if kn.size else None
    rc = _load().oracle_evolve(n, lits.shape[0], _ptr(lits, ctypes.c_int32),
                               _ptr(psi.view(np.float64), ctypes.c_double), float(T), int(N), int(k0), int(k1),
                               kn_ptr, int(kn.size))
    if rc != 0:
        raise ValueError("oracle_evolve: bad arguments")
    return psi


def observables(n: int, clauses, psi: np.ndarray) -> dict:
    """norm, <H_P>, success probability on the E_min manifold, E_min, degeneracy."""
    lits = _lits(clauses)
    out = np.zeros(3, dtype=np.float64)
    emin = ctypes.c_int32(0)
    deg = ctypes.c_int64(0)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    rc = _load().oracle_observables(n, lits.shape[0], _ptr(lits, ctypes.c_int32),
                                    _ptr(psi.view(np.float64), ctypes.c_double), _ptr(out, ctypes.c_double),
                                    ctypes.byref(emin), ctypes.byref(deg))
    if rc != 0:
        raise ValueError("oracle_observables: bad arguments")
    return {"norm": float(out[0]), "energy": float(out[1]), "p_success": float(out[2]),
            "e_min": int(emin.value), "degeneracy": int(deg.value)}


# ---------------------------------------------------------------------------
# Dense small-n helpers (pins only).  H_B is assembled from Kronecker
# products, independently of the pairwise loop in qaa_oracle.c.
# ---------------------------------------------------------------------------

def dense_h_b(n: int) -> np.ndarray:
    """H_B = sum_i (1 - sigma^x_i)/2 as a dense 2^n x 2^n matrix.

    Kronecker order follows |q_n ... q_1>: the right-most factor acts on q_1,
    i.e. on bit 0 of z.
    """
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    one = np.eye(2)
    h = np.zeros((1 << n, 1 << n))
    for i in range(1, n + 1):            # qubit q_i
        ops = [one] * n                  # ops[0] is q_n ... ops[n-1] is q_1
        ops[n - i] = (one - sx) / 2.0
        m = ops[0]
        for o in ops[1:]:
            m = np.kron(m, o)
        h += m
    return h


def dense_strang_step(n: int, e_diag: np.ndarray, T: float, N: int, k: int) -> np.ndarray:
    """Dense propagator of step k: expm of each factor, multiplied in time order."""
    from scipy.linalg import expm
    dt = T / N
    s = (k + 0.5) / N
    hp = np.diag(e_diag.astype(np.float64))
    half = expm(-1j * (dt / 2.0) * s * hp)
    drive = expm(-1j * dt * (1.0 - s) * dense_h_b(n))
    return half @ drive @ half


def _flip(x: np.ndarray, q: int) -> np.ndarray:
    """x(z xor 2^q) for all z: swap the halves of every block of 2^(q+1)."""
    return x.reshape(-1, 2, 1 << q)[:, ::-1, :].reshape(-1)


def levels(n: int, clauses, s: float, k: int, merge: float = 1e-8) -> np.ndarray:
    """The k lowest distinct eigenvalues of H(s) = (1-s) H_B + s H_P (eq. 1).

    Eigenvalues closer than `merge` count as one level.  n <= 11: dense
    matrix (H_B from Kronecker products) and numpy ``eigvalsh``, any s and
    any clause list.  Larger n: scipy ``eigsh`` (ARPACK) with H(s) applied
    matrix-free, (H x)(z) = ((1-s) n/2 + s E(z)) x(z) - (1-s)/2 sum_q x(z xor 2^q),
    for 0 < s < 1 and at least one clause only: at s = 0, s = 1 or without
    clauses the start vector's Krylov space has only as many dimensions as
    H(s) has levels (n + 1, or the number of distinct energies), which
    ARPACK's restarted iteration does not handle (those cases have closed
    forms instead).
    """
    E = energy(n, clauses).astype(np.float64)
    if n <= 11:
        h = (1.0 - s) * dense_h_b(n) + s * np.diag(E)
        w = np.linalg.eigvalsh(h)
    else:
        if not (0.0 < s < 1.0) or len(_lits(clauses)) == 0:
            raise ValueError("levels: n > 11 needs 0 < s < 1 and at least one clause")
        from scipy.sparse.linalg import LinearOperator, eigsh
        dim = 1 << n
        diag = (1.0 - s) * 0.5 * n + s * E

        def mv(x):
            x = np.asarray(x, dtype=np.float64).reshape(-1)
            y = diag * x
            for q in range(n):
                y -= 0.5 * (1.0 - s) * _flip(x, q)
            return y

        op = LinearOperator((dim, dim), matvec=mv, dtype=np.float64)
        start = np.cos(np.arange(dim) * 0.7071) + 1.5      # fixed, not an eigenvector
        w = np.sort(eigsh(op, k=k + 2, which="SA", tol=1e-14, v0=start, return_eigenvectors=False))
    out = []
    for x in w:
        if not out or x - out[-1] > merge:
            out.append(float(x))
        if len(out) == k:
            break
    return np.asarray(out)
