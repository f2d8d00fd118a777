"""GPU parity of the spectrum of H(s) = (1 - s) H_B + s H_P (eq. 1):
qaa_spectrum (Lanczos on the device, through the C ABI) against the CPU
oracle (dense eigvalsh for n <= 11, ARPACK for larger n at 0 < s < 1) and,
at any size, against closed forms (s = 0, s = 1, no clauses) and the
variational bounds 0 < E0(s) < s m/8.

Bar: FP64 eigenvalues within 1e-9 (absolute; the levels are O(1..m)) once
the Lanczos run is long enough for them to converge.
"""
import numpy as np
import pytest

import oracle
from qaa_inputs import planted_unique_3sat

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def qaa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1103_1399_amd as m
    return m


def _v0(n, seed):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.standard_normal(1 << n)).cuda()


def _setup(qaa, n, seed, clauses=None):
    inst_in = planted_unique_3sat(n, seed) if clauses is None else None
    cl = inst_in.clauses if clauses is None else np.asarray(clauses, np.int32).reshape(-1, 3)
    inst = qaa.Instance(n, cl.reshape(-1))
    table = inst.energy_table()
    return cl, inst, table


@pytest.mark.parametrize("n", [4, 8, 10])
def test_small_spectrum_vs_dense_oracle(qaa, n):
    """Krylov space of full dimension: every requested level is exact."""
    cl, inst, table = _setup(qaa, n, 1100 + n)
    svals = [0.0, 0.25, 0.5, 0.75, 1.0]
    print("spectrum n", n, flush=True)
    got = inst.spectrum(table, svals, _v0(n, n), iters=min(1 << n, 400), k=3)
    for i, s in enumerate(svals):
        ref = oracle.levels(n, cl, s, 3)
        assert np.allclose(got[i, :len(ref)], ref, atol=TOL, rtol=0), (s, got[i], ref)


@pytest.mark.parametrize("n,iters", [(12, 300), (14, 300), (16, 400)])
def test_spectrum_vs_arpack(qaa, n, iters):
    cl, inst, table = _setup(qaa, n, 1200 + n)
    svals = [0.3, 0.5, 0.7]
    print("spectrum n", n, "iters", iters, flush=True)
    got = inst.spectrum(table, svals, _v0(n, n + 1), iters=iters, k=2)
    for i, s in enumerate(svals):
        ref = oracle.levels(n, cl, s, 2)
        assert np.allclose(got[i], ref, atol=TOL, rtol=0), (s, got[i], ref)


def test_closed_forms_at_n20(qaa):
    """s = 0: the driver's levels 0, 1, 2; s = 1: the three lowest energies;
    no clauses: (1 - s) times 0, 1, 2.  In each case the Krylov space closes
    after as many steps as there are levels, and the values are exact."""
    n = 20
    cl, inst, table = _setup(qaa, n, 1300)
    v0 = _v0(n, 3)
    got = inst.spectrum(table, [0.0, 1.0], v0, iters=80, k=3)
    assert np.allclose(got[0], [0.0, 1.0, 2.0], atol=TOL, rtol=0)
    E = np.unique(oracle.energy(n, cl))
    assert np.allclose(got[1], E[:3], atol=TOL, rtol=0)
    _, free, ftable = _setup(qaa, n, 0, clauses=np.zeros((0, 3), np.int32))
    got = free.spectrum(ftable, [0.4], v0, iters=40, k=3)
    assert np.allclose(got[0], 0.6 * np.arange(3), atol=TOL, rtol=0)


def test_ground_level_bounds_at_n20(qaa):
    n = 20
    cl, inst, table = _setup(qaa, n, 1301)
    m = cl.shape[0]
    svals = [0.2, 0.5, 0.8]
    got = inst.spectrum(table, svals, _v0(n, 4), iters=200, k=2)
    for i, s in enumerate(svals):
        assert 0.0 < got[i, 0] < s * m / 8.0
        assert got[i, 1] > got[i, 0]


def test_spectrum_is_deterministic_and_per_s(qaa):
    n = 14
    cl, inst, table = _setup(qaa, n, 1302)
    v0 = _v0(n, 5)
    a = inst.spectrum(table, [0.35, 0.65], v0, iters=120, k=2)
    b = inst.spectrum(table, [0.35, 0.65], v0, iters=120, k=2)
    c = inst.spectrum(table, [0.65], v0, iters=120, k=2)
    assert np.array_equal(a, b)
    assert np.array_equal(a[1], c[0])


def test_zero_start_vector_is_reported(qaa):
    n = 10
    cl, inst, table = _setup(qaa, n, 1303)
    with pytest.raises(qaa.QaaError) as ei:
        inst.spectrum(table, [0.5], torch.zeros(1 << n, dtype=torch.float64, device="cuda"), iters=10, k=1)
    assert ei.value.status == qaa.QAA_ERR_INVALID_ARG


def test_uint16_table_gives_the_same_levels(qaa):
    n = 13
    cl, inst, table = _setup(qaa, n, 1304)
    t16 = inst.energy_table(etype=qaa.QAA_E_U16)
    v0 = _v0(n, 6)
    a = inst.spectrum(table, [0.45], v0, iters=100, k=2)
    b = inst.spectrum(t16, [0.45], v0, iters=100, k=2)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("iters", [6, 12, 40])
def test_residual_bounds_hold(qaa, iters):
    """Each returned Ritz value has an eigenvalue of H(s) within its bound
    (all eigenvalues from dense eigvalsh at n = 8), also far from
    convergence."""
    n = 8
    cl, inst, table = _setup(qaa, n, 1305)
    E = oracle.energy(n, cl).astype(float)
    svals = [0.3, 0.6]
    ev, bd = inst.spectrum(table, svals, _v0(n, 7), iters=iters, k=3, bounds=True)
    for i, s in enumerate(svals):
        w = np.linalg.eigvalsh((1 - s) * oracle.dense_h_b(n) + s * np.diag(E))
        for x, b in zip(ev[i], bd[i]):
            assert np.min(np.abs(w - x)) <= b * (1 + 1e-9) + 1e-12, (s, x, b)


def test_residual_bounds_are_small_once_converged(qaa):
    n = 14
    cl, inst, table = _setup(qaa, n, 1214)
    ev, bd = inst.spectrum(table, [0.3, 0.5, 0.7], _v0(n, n + 1), iters=300, k=2, bounds=True)
    assert np.all(bd < 1e-8), bd
    assert np.allclose(ev, inst.spectrum(table, [0.3, 0.5, 0.7], _v0(n, n + 1), iters=300, k=2), atol=0, rtol=0)


def test_workspace_too_large_is_reported(qaa):
    """n = 30 with 1024 Lanczos steps needs ~8.8 TB of workspace: refused
    with QAA_ERR_OUT_OF_MEMORY before any kernel runs (v0 and the table
    are full size, so nothing could read past them either way)."""
    n = 30
    inst = qaa.Instance(n, [])
    table = inst.energy_table()
    v0 = torch.ones(1 << n, dtype=torch.float64, device="cuda")
    with pytest.raises(qaa.QaaError) as ei:
        inst.spectrum(table, [0.5], v0, iters=1024, k=2)
    assert ei.value.status == qaa.QAA_ERR_OUT_OF_MEMORY
    del v0, table
    torch.cuda.empty_cache()
