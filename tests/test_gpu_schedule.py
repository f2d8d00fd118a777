"""GPU parity of schedule tables (s(u) piecewise linear through equally
spaced knots, u = t/T): the HIP path through the C ABI against the CPU
oracle, on every execution path (one-workgroup states, two- and three-set
pass plans, complex64 and complex128, step ranges, batched calls, n = 28).

Bars as for the linear schedule: complex64 L2 <= 1e-4 and |dP| <= 1e-5
against the complex128 oracle; complex128 within 1e-10.
"""
import numpy as np
import pytest

import oracle
from qaa_inputs import SplitMix64, planted_unique_3sat

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L2_TOL_C64 = 1e-4
P_TOL_C64 = 1e-5
L2_TOL_C128 = 1e-10

TABLES = {
    "slow middle": [0.0, 0.35, 0.45, 0.5, 0.55, 0.65, 1.0],
    "non-monotone": [0.0, 0.9, 0.2, 1.0],
    "256 knots": list(np.linspace(0.0, 1.0, 256) ** 1.5),
}


@pytest.fixture(scope="module")
def qaa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1103_1399_amd as m
    return m


def _states(qaa, n, seed, dtype):
    inst_in = planted_unique_3sat(n, seed)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    return inst_in, inst, table


def _check(st, psi, clauses, n, l2_tol, p_tol):
    got = st.amp.cpu().numpy().astype(np.complex128)
    obs = st.observables()
    ref = oracle.observables(n, clauses, psi)
    l2 = float(np.linalg.norm(got - psi))
    dp = abs(obs["p_success"] - ref["p_success"])
    assert l2 <= l2_tol, "L2 %.3g" % l2
    assert dp <= p_tol, "dP %.3g" % dp
    assert abs(obs["norm"] - 1.0) <= 10 * l2_tol


@pytest.mark.parametrize("name", list(TABLES))
@pytest.mark.parametrize("n,T,N", [(10, 10.0, 1000), (13, 10.0, 300), (16, 10.0, 200), (22, 5.0, 24)])
def test_table_schedule_c64_vs_oracle(qaa, name, n, T, N):
    knots = TABLES[name]
    print("table", name, "n", n, "T", T, "N", N, flush=True)
    inst_in, inst, table = _states(qaa, n, 900 + n, torch.complex64)
    st = qaa.State(inst, table).init_uniform().evolve(T, N, knots=knots)
    psi = oracle.init_uniform(n)
    oracle.evolve(n, inst_in.clauses, psi, T, N, knots=knots)
    _check(st, psi, inst_in.clauses, n, L2_TOL_C64, P_TOL_C64)


@pytest.mark.parametrize("n,T,N", [(12, 10.0, 300), (15, 8.0, 60), (20, 5.0, 12)])
def test_table_schedule_c128_vs_oracle(qaa, n, T, N):
    knots = TABLES["slow middle"]
    inst_in, inst, table = _states(qaa, n, 950 + n, torch.complex128)
    st = qaa.State(inst, table, dtype=torch.complex128).init_uniform().evolve(T, N, knots=knots)
    psi = oracle.init_uniform(n)
    oracle.evolve(n, inst_in.clauses, psi, T, N, knots=knots)
    _check(st, psi, inst_in.clauses, n, L2_TOL_C128, L2_TOL_C128)


@pytest.mark.parametrize("n", [11, 18])
def test_two_knot_table_is_the_linear_schedule_to_the_bit(qaa, n):
    inst_in, inst, table = _states(qaa, n, 970 + n, torch.complex64)
    a = qaa.State(inst, table).init_uniform().evolve(7.0, 90)
    b = qaa.State(inst, table).init_uniform().evolve(7.0, 90, knots=[0.0, 1.0])
    torch.cuda.synchronize()
    assert torch.equal(a.amp, b.amp)


@pytest.mark.parametrize("n", [12, 17])
def test_table_schedule_step_ranges(qaa, n):
    """evolve_range(0, K) then (K, N) under a table equals the oracle's run."""
    knots = TABLES["non-monotone"]
    T, N, K = 6.0, 50, 23
    inst_in, inst, table = _states(qaa, n, 980 + n, torch.complex64)
    st = qaa.State(inst, table).init_uniform()
    st.evolve_range(T, N, 0, K, knots=knots)
    st.evolve_range(T, N, K, N, knots=knots)
    psi = oracle.init_uniform(n)
    oracle.evolve(n, inst_in.clauses, psi, T, N, knots=knots)
    _check(st, psi, inst_in.clauses, n, L2_TOL_C64, P_TOL_C64)


def test_batch_with_mixed_schedules_equals_individual(qaa):
    """A batched call where each state has its own schedule (linear or a
    table), on both the one-workgroup and the lock-step pass path."""
    ns = [8, 12, 13, 14, 16, 21, 22, 15]
    Ts = [3.0, 4.0, 5.0, 6.0, 3.0, 4.5, 3.5, 5.0]
    Ns = [40, 50, 30, 20, 15, 7, 5, 11]
    tabs = [TABLES["slow middle"], None, TABLES["256 knots"], TABLES["non-monotone"], None,
            TABLES["slow middle"], TABLES["256 knots"], [0.2, 0.2]]
    singles, batch, ins = [], [], []
    for i, n in enumerate(ns):
        inst_in, inst, table = _states(qaa, n, 1000 + i, torch.complex64)
        singles.append(qaa.State(inst, table).init_uniform().evolve(Ts[i], Ns[i], knots=tabs[i]))
        batch.append(qaa.State(inst, table).init_uniform())
        ins.append(inst_in)
    qaa.qaa_evolve_batch([b.c for b in batch], Ts, Ns, knots=tabs)
    torch.cuda.synchronize()
    for i, (n, sgl, b) in enumerate(zip(ns, singles, batch)):
        diff = float(torch.linalg.vector_norm((sgl.amp - b.amp).to(torch.complex128)).item())
        assert diff < 2e-6, (n, diff)
        if n <= 16:
            psi = oracle.init_uniform(n)
            oracle.evolve(n, ins[i].clauses, psi, Ts[i], Ns[i], knots=tabs[i])
            _check(b, psi, ins[i].clauses, n, L2_TOL_C64, P_TOL_C64)


def test_full_size_table_driver_only_closed_form(qaa):
    """n = 28, m = 0 from |z0> under a 3-knot table with N a multiple of the
    segment count: Theta = T (1 - mean of the segment averages) exactly, and
    psi(z) = a^{n-d} b^d; checked on a sample and by the norm."""
    n, T, N, z0 = 28, 50.0, 6, 0x3C3C3C3
    knots = [0.0, 0.8, 1.0]
    inst = qaa.Instance(n, [])
    table = inst.energy_table()
    st = qaa.State(inst, table).init_basis(z0).evolve(T, N, knots=knots)
    obs = st.observables()
    v = np.asarray(knots)
    th = T * (1.0 - np.mean((v[:-1] + v[1:]) / 2.0))
    a = (1 + np.exp(-1j * th)) / 2
    b = (1 - np.exp(-1j * th)) / 2
    rng = SplitMix64(6)
    zs = np.asarray([rng.below(1 << n) for _ in range(4096)] + [z0, z0 ^ 1, z0 ^ (1 << 27)], dtype=np.int64)
    got = st.amp[torch.from_numpy(zs).cuda()].cpu().numpy().astype(np.complex128)
    d = np.array([bin(int(z) ^ z0).count("1") for z in zs])
    expect = a ** (n - d) * b ** d
    assert np.max(np.abs(got - expect)) < 2e-6
    assert abs(obs["norm"] - 1.0) < 1e-6


def test_batch_mixed_dtypes_and_table_types_vs_oracle(qaa):
    """One batched call over complex64 and complex128 states with uint8 and
    uint16 energy tables, one-workgroup and pass-plan sizes, linear and
    table schedules: every launch group of the batch against the oracle."""
    cases = [(9, torch.complex128, qaa.QAA_E_U8, None), (12, torch.complex128, qaa.QAA_E_U16, TABLES["slow middle"]),
             (14, torch.complex128, qaa.QAA_E_U8, TABLES["non-monotone"]), (15, torch.complex128, qaa.QAA_E_U16, None),
             (10, torch.complex64, qaa.QAA_E_U16, TABLES["256 knots"]), (16, torch.complex64, qaa.QAA_E_U16,
                                                                        TABLES["slow middle"])]
    states, ins, Ts, Ns, knots = [], [], [], [], []
    for i, (n, dt, et, kn) in enumerate(cases):
        inst_in = planted_unique_3sat(n, 1100 + i)
        inst = qaa.Instance(n, inst_in.literals())
        table = inst.energy_table(etype=et)
        states.append(qaa.State(inst, table, dtype=dt).init_uniform())
        ins.append(inst_in)
        Ts.append(4.0 + i)
        Ns.append(20 + 5 * i)
        knots.append(kn)
    qaa.qaa_evolve_batch([st.c for st in states], Ts, Ns, knots=knots)
    torch.cuda.synchronize()
    for (n, dt, et, kn), st, inst_in, T, N in zip(cases, states, ins, Ts, Ns):
        psi = oracle.init_uniform(n)
        oracle.evolve(n, inst_in.clauses, psi, T, N, knots=kn)
        tol = L2_TOL_C128 if dt == torch.complex128 else L2_TOL_C64
        _check(st, psi, inst_in.clauses, n, tol, tol if dt == torch.complex128 else P_TOL_C64)
