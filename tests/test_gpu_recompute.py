"""Recompute mode (a state with no energy table): the violated-clause count of
Sec. 4.3 is scored from the clause records inside the phase passes, the
single-workgroup kernel and the observables reduction.  Checked against the
oracle, and against the table mode on the same inputs."""

import numpy as np
import pytest
import torch

import oracle
from qaa_inputs import planted_unique_3sat

pytestmark = pytest.mark.gpu

L2_TOL_C64 = 1e-4
P_TOL_C64 = 1e-5
L2_TOL_C128 = 1e-10


@pytest.fixture(scope="module")
def qaa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1103_1399_amd as m
    return m


def _oracle_run(n, clauses, T, N):
    psi = oracle.init_uniform(n)
    oracle.evolve(n, clauses, psi, T, N)
    return psi, oracle.observables(n, clauses, psi)


def _check(st, obs, psi, ref, l2_tol, p_tol):
    got = st.amp.cpu().numpy().astype(np.complex128)
    l2 = float(np.linalg.norm(got - psi))
    assert l2 <= l2_tol, "L2 %.3g" % l2
    assert abs(obs["p_success"] - ref["p_success"]) <= p_tol
    assert abs(obs["energy"] - ref["energy"]) <= 10 * l2_tol * max(1.0, ref["energy"])
    assert obs["e_min"] == ref["e_min"] and obs["degeneracy"] == ref["degeneracy"]


def _pair(qaa, n, clauses, T, N, dtype=torch.complex64, etype=None):
    """The same job with a table and without one: (table state, its
    observables, recompute state, its observables)."""
    lits = np.asarray(clauses, np.int32).reshape(-1)
    a_inst = qaa.Instance(n, lits)
    et = qaa.QAA_E_U8 if etype is None else etype
    table = a_inst.energy_table(etype=et)
    a = qaa.State(a_inst, table, dtype=dtype).init_uniform()
    a.evolve(T, N)
    oa = a.observables()
    b_inst = qaa.Instance(n, lits)
    b_inst.energy_stats()
    b = qaa.State(b_inst, None, dtype=dtype, etype=et).init_uniform()
    b.evolve(T, N)
    ob = b.observables()
    return a, oa, b, ob


@pytest.mark.parametrize("n,seed", [(3, 0), (10, 1), (13, 2), (16, 3), (22, 4), (24, 5)])
def test_energy_stats_equal_the_table_statistics(qaa, n, seed):
    inst_in = planted_unique_3sat(n, 300 + seed)
    lits = inst_in.literals()
    a = qaa.Instance(n, lits)
    a.energy_table()
    b = qaa.Instance(n, lits)
    ib = b.energy_stats()
    ia = a.info()
    e = oracle.energy(n, inst_in.clauses)
    assert (ib["e_min"], ib["e_max"], ib["degeneracy"]) == (ia["e_min"], ia["e_max"], ia["degeneracy"])
    assert (ib["e_min"], ib["e_max"], ib["degeneracy"]) == (int(e.min()), int(e.max()), int((e == e.min()).sum()))


def test_energy_stats_past_255(qaa):
    """Counts above 255 take the 16-plane counter (the u8 overflow rerun)."""
    n = 14
    cl = [[1, 2, 3]] * 300 + planted_unique_3sat(n, 7).clauses.tolist()
    inst = qaa.Instance(n, np.asarray(cl, np.int32).reshape(-1))
    info = inst.energy_stats()
    e = oracle.energy(n, cl)
    assert (info["e_min"], info["e_max"], info["degeneracy"]) == (int(e.min()), int(e.max()),
                                                                   int((e == e.min()).sum()))


@pytest.mark.parametrize("n,T,N", [(10, 10.0, 200),    # one workgroup holds the state
                                   (13, 5.0, 40),
                                   (16, 6.0, 30),      # m > 128: clause records in chunks
                                   (20, 5.0, 10),
                                   (22, 5.0, 8),       # 2^14 tiles (default plan at this n)
                                   (24, 4.0, 6)])      # three sets
def test_recompute_vs_oracle_and_table_mode(qaa, n, T, N):
    inst_in = planted_unique_3sat(n, 400 + n)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    a, oa, b, ob = _pair(qaa, n, inst_in.clauses, T, N)
    _check(b, ob, psi, ref, L2_TOL_C64, P_TOL_C64)
    # the same integer energies feed the same arithmetic: identical states
    assert torch.equal(a.amp, b.amp)
    for k in ("norm", "energy", "p_success"):
        assert abs(oa[k] - ob[k]) <= 1e-12 * max(1.0, abs(oa[k])), k


@pytest.mark.parametrize("n", [22, 24])
def test_recompute_with_base_tiles(qaa, n):
    """Recompute mode on the 2^13-amplitude tile plan as well."""
    T, N = 4.0, 5
    inst_in = planted_unique_3sat(n, 410 + n)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    try:
        qaa.qaa_plan_set(n, qaa.QAA_C64, {"balance": 0, "passengers": 1, "tiles": 0})
        a, oa, b, ob = _pair(qaa, n, inst_in.clauses, T, N)
    finally:
        qaa.qaa_plan_set(n, qaa.QAA_C64, None)
    _check(b, ob, psi, ref, L2_TOL_C64, P_TOL_C64)
    assert torch.equal(a.amp, b.amp)


@pytest.mark.parametrize("n,T,N", [(9, 5.0, 60), (15, 6.0, 20)])
def test_recompute_complex128_vs_oracle(qaa, n, T, N):
    inst_in = planted_unique_3sat(n, 420 + n)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    a, oa, b, ob = _pair(qaa, n, inst_in.clauses, T, N, dtype=torch.complex128)
    _check(b, ob, psi, ref, L2_TOL_C128, 1e-12)
    assert torch.equal(a.amp, b.amp)


@pytest.mark.parametrize("n,N", [(11, 30), (16, 8)])
def test_recompute_uint16_width_past_255(qaa, n, N):
    """Energies above 255 held at 16 bits: the resident kernel and the
    passes against the oracle and the uint16 table."""
    T = 0.05                      # E up to ~300: a short T keeps the phases tame
    cl = [[1, 2, 3]] * 300 + planted_unique_3sat(n, 430 + n).clauses.tolist()
    psi, ref = _oracle_run(n, cl, T, N)
    a, oa, b, ob = _pair(qaa, n, cl, T, N, etype=qaa.QAA_E_U16)
    assert b.c.etype == qaa.QAA_E_U16
    _check(b, ob, psi, ref, L2_TOL_C64, P_TOL_C64)
    assert torch.equal(a.amp, b.amp)


def test_recompute_observables_on_the_same_state(qaa):
    """qaa_observables with no table on a state the table mode evolved."""
    n, T, N = 17, 5.0, 20
    inst_in = planted_unique_3sat(n, 81)
    lits = inst_in.literals()
    a_inst = qaa.Instance(n, lits)
    table = a_inst.energy_table()
    a = qaa.State(a_inst, table).init_uniform()
    a.evolve(T, N)
    oa = a.observables()
    b_inst = qaa.Instance(n, lits)
    b_inst.energy_stats()
    b = qaa.State(b_inst, None, amp=a.amp)
    ob = b.observables()
    ref = oracle.observables(n, inst_in.clauses, a.amp.cpu().numpy().astype(np.complex128))
    for k in ("norm", "energy", "p_success"):
        assert abs(ob[k] - oa[k]) <= 1e-12 * max(1.0, abs(oa[k])), k
        assert abs(ob[k] - ref[k]) <= 1e-12 * max(1.0, abs(ref[k])), k


def test_recompute_needs_the_statistics(qaa):
    n = 12
    inst = qaa.Instance(n, planted_unique_3sat(n, 3).literals())
    st = qaa.State(inst, None, etype=qaa.QAA_E_U8).init_uniform()
    with pytest.raises(qaa.QaaError) as ei:
        st.evolve(1.0, 2)
    assert ei.value.status == qaa.QAA_ERR_NOT_READY


def test_recompute_u8_width_rejects_counts_past_255(qaa):
    n = 14
    cl = [[1, 2, 3]] * 300
    inst = qaa.Instance(n, np.asarray(cl, np.int32).reshape(-1))
    inst.energy_stats()
    st = qaa.State(inst, None, etype=qaa.QAA_E_U8).init_uniform()
    with pytest.raises(qaa.QaaError) as ei:
        st.evolve(1.0, 2)
    assert ei.value.status == qaa.QAA_ERR_UNSUPPORTED


def test_batch_refuses_a_state_without_a_table(qaa):
    n = 14
    inst = qaa.Instance(n, planted_unique_3sat(n, 4).literals())
    inst.energy_stats()
    st = qaa.State(inst, None).init_uniform()
    with pytest.raises(qaa.QaaError) as ei:
        qaa.qaa_evolve_batch([st.c], [1.0], [2])
    assert ei.value.status == qaa.QAA_ERR_UNSUPPORTED


def test_full_size_recompute_first_steps(qaa):
    """n = 28, T = 50, steps 0..3 of 5000 (the benchmark's job) with no
    table: identical to the table mode's state."""
    n, T, N, K = 28, 50.0, 5000, 3
    inst_in = planted_unique_3sat(n, 0)
    lits = inst_in.literals()
    a_inst = qaa.Instance(n, lits)
    table = a_inst.energy_table()
    a = qaa.State(a_inst, table).init_uniform()
    a.evolve_range(T, N, 0, K)
    oa = a.observables()
    del table
    b_inst = qaa.Instance(n, lits)
    b_inst.energy_stats()
    b = qaa.State(b_inst, None).init_uniform()
    b.evolve_range(T, N, 0, K)
    ob = b.observables()
    assert torch.equal(a.amp, b.amp)
    for k in ("norm", "energy", "p_success"):
        assert abs(oa[k] - ob[k]) <= 1e-12 * max(1.0, abs(oa[k])), k
