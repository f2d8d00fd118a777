"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars: energy tables bit-exact; complex64 final state L2 <= 1e-4 and
|dP_success| <= 1e-5 against the complex128 oracle; complex128 GPU runs
within 1e-10.  Every input is seeded and synthetic.
"""
import json
import os

import numpy as np
import pytest

import oracle
from conftest import GOLDEN
from qaa_inputs import SplitMix64, planted_unique_3sat

torch = pytest.importorskip("torch")
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


def _run_gpu(qaa, n, clauses, T, N, dtype=None, etype=None, basis=None):
    inst = qaa.Instance(n, np.asarray(clauses, np.int32).reshape(-1))
    et = qaa.QAA_E_U8 if etype is None else etype
    table = inst.energy_table(etype=et)
    st = qaa.State(inst, table, dtype=dtype or torch.complex64)
    if basis is None:
        st.init_uniform()
    else:
        st.init_basis(basis)
    st.evolve(T, N)
    obs = st.observables()
    return inst, table, st, obs


def _oracle_run(n, clauses, T, N, basis=None):
    if basis is None:
        psi = oracle.init_uniform(n)
    else:
        psi = np.zeros(1 << n, np.complex128)
        psi[basis] = 1.0
    oracle.evolve(n, clauses, psi, T, N)
    return psi, oracle.observables(n, clauses, psi)


def _compare(st, obs, psi, ref, l2_tol, p_tol):
    got = st.amp.cpu().numpy().astype(np.complex128)
    l2 = float(np.linalg.norm(got - psi))
    dp = abs(obs["p_success"] - ref["p_success"])
    de = abs(obs["energy"] - ref["energy"])
    assert l2 <= l2_tol, "L2 %.3g" % l2
    assert dp <= p_tol, "dP %.3g" % dp
    assert de <= 10 * l2_tol * max(1.0, ref["energy"]), "d<H_P> %.3g" % de
    assert abs(obs["norm"] - 1.0) <= 10 * l2_tol
    return l2, dp


# --------------------------------------------------------------------------
# Energy table
# --------------------------------------------------------------------------

def test_energy_table_worked_example(qaa, worked_example):
    n, cl = worked_example["n"], worked_example["clauses"]
    inst = qaa.Instance(n, np.asarray(cl, np.int32).reshape(-1))
    table = inst.energy_table()
    assert np.array_equal(table.cpu().numpy().astype(np.int32), oracle.energy(n, cl))
    info = inst.info()
    assert info["e_min"] == 0 and info["degeneracy"] == 1
    assert table.cpu().numpy()[10] == 0


@pytest.mark.parametrize("n,seed", [(3, 0), (4, 1), (7, 2), (10, 3), (13, 4), (16, 5), (20, 6), (22, 7)])
@pytest.mark.parametrize("etype", [0, 1])
def test_energy_table_bit_exact(qaa, n, seed, etype):
    inst_in = planted_unique_3sat(n, seed)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table(etype=etype)
    got = table.cpu().numpy()
    if etype == 1:
        got = got.view(np.uint16)
    E = oracle.energy(n, inst_in.clauses)
    assert np.array_equal(got.astype(np.int32), E)
    info = inst.info()
    assert info["e_min"] == E.min() and info["e_max"] == E.max()
    assert info["degeneracy"] == np.count_nonzero(E == E.min())


def test_energy_table_small_n_without_clauses(qaa):
    for n in (1, 2, 3):
        inst = qaa.Instance(n, [])
        table = inst.energy_table()
        assert table.cpu().numpy().tolist() == [0] * (1 << n)
        assert inst.info()["degeneracy"] == 1 << n


def test_energy_table_u8_overflow_is_rejected(qaa):
    n = 5
    cl = [[1, 2, 3]] * 300          # E = 300 on the 4 states with x1=x2=x3=0
    inst = qaa.Instance(n, np.asarray(cl, np.int32).reshape(-1))
    with pytest.raises(qaa.QaaError) as ei:
        inst.energy_table(etype=qaa.QAA_E_U8)
    assert ei.value.status == qaa.QAA_ERR_UNSUPPORTED
    table = inst.energy_table(etype=qaa.QAA_E_U16)
    assert np.array_equal(table.cpu().numpy().view(np.uint16).astype(np.int32), oracle.energy(n, cl))
    assert inst.info()["e_max"] == 300


def test_energy_table_full_size_n28_sampled(qaa):
    """n = 28 (the headline size): bit-exact on a sample computed by the
    oracle one state at a time, plus the exact counting identity
    sum_z E(z) = m 2^{n-3} and the unique planted zero."""
    n = 28
    inst_in = planted_unique_3sat(n, 0)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    rng = SplitMix64(28)
    zs = [rng.below(1 << n) for _ in range(20000)]
    zs += list(range(4096)) + list(range((1 << n) - 4096, 1 << n)) + [inst_in.planted]
    zs = np.asarray(zs, dtype=np.int64)
    got = table[torch.from_numpy(zs).cuda()].cpu().numpy().astype(np.int32)
    assert np.array_equal(got, oracle.energy_at(n, inst_in.clauses, zs.astype(np.uint64)))
    total = int(table.to(torch.int64).sum().item())
    assert total == inst_in.m * (1 << (n - 3))
    info = inst.info()
    assert info["e_min"] == 0 and info["degeneracy"] == 1
    assert int(table[inst_in.planted].item()) == 0


# --------------------------------------------------------------------------
# Evolution parity
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(10))
def test_evolve_n10_T10_1000_steps(qaa, seed):
    """n = 10, T = 10, 1000 steps: complex64 GPU vs complex128 oracle."""
    n, T, N = 10, 10.0, 1000
    inst_in = planted_unique_3sat(n, seed)
    _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    _compare(st, obs, psi, ref, L2_TOL_C64, P_TOL_C64)


@pytest.mark.parametrize("n,T,N,etype", [(8, 5.0, 77, 0), (9, 6.0, 65, 0), (9, 6.0, 65, 1), (10, 4.0, 33, 0),
                                         (11, 7.0, 101, 0), (11, 7.0, 101, 1), (12, 5.0, 45, 0), (12, 5.0, 45, 1)])
def test_register_resident_sizes_vs_oracle(qaa, n, T, N, etype):
    """n = 8..12 (one state in registers, lane qubits rotated across lanes,
    the wave qubits after an exchange that alternates the layout): odd step
    counts past one 32-step chunk, so runs end in either layout."""
    inst_in = planted_unique_3sat(n, 120 + n)
    _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N, etype=etype)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    _compare(st, obs, psi, ref, L2_TOL_C64, P_TOL_C64)


@pytest.mark.parametrize("n", [9, 10, 11, 12])
def test_register_resident_ranges_compose(qaa, n):
    """Ranges that stop after an odd number of steps (the state is stored
    from the other layout) and resume: equal to the uninterrupted run to
    rounding, and to the oracle."""
    T, N, K = 6.0, 90, 37
    inst_in = planted_unique_3sat(n, 130 + n)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    a = qaa.State(inst, table).init_uniform().evolve(T, N)
    b = qaa.State(inst, table).init_uniform()
    b.evolve_range(T, N, 0, K)
    b.evolve_range(T, N, K, N)
    torch.cuda.synchronize()
    diff = float(torch.linalg.vector_norm((a.amp - b.amp).to(torch.complex128)).item())
    assert diff < 1e-5
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    _compare(b, b.observables(), psi, ref, L2_TOL_C64, P_TOL_C64)


@pytest.mark.parametrize("n,T,N", [(5, 3.0, 40), (13, 5.0, 60), (14, 5.0, 60), (15, 8.0, 80), (17, 5.0, 50),
                                   (21, 5.0, 30), (22, 5.0, 12), (23, 4.0, 8)])
def test_evolve_multipass_parity(qaa, n, T, N):
    """Sizes around every plan boundary: resident (n <= 13), two qubit sets
    (14..21), three sets (22..), including ragged last sets."""
    inst_in = planted_unique_3sat(n, 100 + n)
    _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    _compare(st, obs, psi, ref, L2_TOL_C64, P_TOL_C64)


@pytest.mark.parametrize("n,T,N", [(6, 4.0, 50), (12, 5.0, 40), (13, 5.0, 40), (16, 6.0, 30), (20, 5.0, 10)])
def test_evolve_complex128_parity(qaa, n, T, N):
    inst_in = planted_unique_3sat(n, 200 + n)
    _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N, dtype=torch.complex128)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    _compare(st, obs, psi, ref, L2_TOL_C128, 1e-12)


def test_evolve_u16_table_path(qaa):
    n, T, N = 15, 6.0, 40
    inst_in = planted_unique_3sat(n, 31)
    _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N, etype=qaa.QAA_E_U16)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    _compare(st, obs, psi, ref, L2_TOL_C64, P_TOL_C64)


def test_evolve_from_basis_state(qaa):
    n, T, N = 16, 5.0, 40
    inst_in = planted_unique_3sat(n, 41)
    _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N, basis=12345)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N, basis=12345)
    _compare(st, obs, psi, ref, L2_TOL_C64, P_TOL_C64)


def test_evolve_n24_three_sets_vs_oracle(qaa):
    """n = 24 runs the same three-set pass structure as n = 28."""
    n, T, N = 24, 50.0, 6
    inst_in = planted_unique_3sat(n, 0)
    _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    _compare(st, obs, psi, ref, L2_TOL_C64, P_TOL_C64)


def test_evolve_range_composes(qaa):
    n, T, N, K = 16, 8.0, 60, 23
    inst_in = planted_unique_3sat(n, 51)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    a = qaa.State(inst, table).init_uniform().evolve(T, N)
    b = qaa.State(inst, table).init_uniform()
    b.evolve_range(T, N, 0, K)
    b.evolve_range(T, N, K, N)
    torch.cuda.synchronize()
    diff = float(torch.linalg.vector_norm((a.amp - b.amp).to(torch.complex128)).item())
    assert diff < 1e-5
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    _compare(b, b.observables(), psi, ref, L2_TOL_C64, P_TOL_C64)


def test_zero_steps_and_zero_time_are_identity(qaa):
    n = 15
    inst_in = planted_unique_3sat(n, 61)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    st = qaa.State(inst, table).init_uniform()
    ref = st.amp.clone()
    st.evolve(5.0, 0)
    assert torch.equal(st.amp, ref)
    st.evolve(0.0, 7)
    assert torch.equal(st.amp, ref)
    obs = st.observables()
    # 2^{-n/2} is rounded once to FP32 for odd n
    assert abs(obs["p_success"] - 2.0 ** -n) < 2.0 ** -n * 1e-6
    assert abs(obs["energy"] - inst_in.m / 8.0) < inst_in.m / 8.0 * 1e-6


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_evolve_tiny_states(qaa, n):
    """The smallest states (a single clause when n >= 3, none below) through
    the resident path, against the oracle, complex64 and complex128."""
    clauses = np.asarray([[1, -2, 3]] if n >= 3 else np.zeros((0, 3)), np.int32).reshape(-1, 3)
    T, N = 3.0, 25
    psi, ref = _oracle_run(n, clauses, T, N)
    for dtype, l2_tol in ((torch.complex64, L2_TOL_C64), (torch.complex128, L2_TOL_C128)):
        inst = qaa.Instance(n, clauses.reshape(-1))
        table = inst.energy_table()
        st = qaa.State(inst, table, dtype=dtype).init_uniform()
        st.evolve(T, N)
        obs = st.observables()
        got = st.amp.cpu().numpy().astype(np.complex128)
        assert np.linalg.norm(got - psi) <= l2_tol
        assert abs(obs["p_success"] - ref["p_success"]) <= max(l2_tol, 1e-12)
        inst.close()


@pytest.mark.parametrize("seed", range(8))
def test_random_configurations_vs_oracle(qaa, seed):
    """Seeded random draws of n (5..23), T, step count, dtype and the table
    type against the oracle: resident, two-set and three-set plans, both
    energy widths, any step size (angles reduced by pi included)."""
    rng = SplitMix64(9000 + seed)
    n = 5 + rng.below(19)
    T = rng.uniform(0.5, 40.0)
    N = 1 + rng.below(60)
    dtype = torch.complex128 if rng.below(3) == 0 else torch.complex64
    et = qaa.QAA_E_U16 if rng.below(2) else qaa.QAA_E_U8
    inst_in = planted_unique_3sat(n, 9100 + seed)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N, dtype=dtype, etype=et)
    tol = L2_TOL_C128 if dtype == torch.complex128 else L2_TOL_C64
    _compare(st, obs, psi, ref, tol, max(tol, 1e-12) if dtype == torch.complex128 else P_TOL_C64)


@pytest.mark.parametrize("choice", [{"balance": 0, "passengers": 0, "tiles": 0},
                                    {"balance": 1, "passengers": 0, "tiles": 0},
                                    {"balance": 0, "passengers": 1, "tiles": 0},
                                    {"balance": 1, "passengers": 1, "tiles": 0}])
def test_plan_choices_vs_oracle(qaa, choice):
    """Every qubit assignment of a three-set plan (n = 22, 2^13 tiles) on
    the GPU."""
    n, T, N = 22, 5.0, 12
    inst_in = planted_unique_3sat(n, 77)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    try:
        qaa.qaa_plan_set(n, qaa.QAA_C64, choice)
        _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N)
    finally:
        qaa.qaa_plan_set(n, qaa.QAA_C64, None)
    _compare(st, obs, psi, ref, L2_TOL_C64, P_TOL_C64)


@pytest.mark.parametrize("n,tiles,passengers", [(22, 1, 1), (22, 2, 1), (23, 1, 0), (24, 1, 1), (24, 2, 1),
                                                (24, 2, 0)])
def test_wide_tile_plans_vs_oracle(qaa, n, tiles, passengers):
    """2^14-amplitude tiles on the GPU (the top set only, or every set):
    two- and three-set plans against the oracle."""
    T, N = 5.0, 6
    inst_in = planted_unique_3sat(n, 90 + n)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    try:
        qaa.qaa_plan_set(n, qaa.QAA_C64, {"balance": 0, "passengers": passengers, "tiles": tiles})
        assert qaa.qaa_plan_get(n)["tiles"] == tiles
        _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N)
    finally:
        qaa.qaa_plan_set(n, qaa.QAA_C64, None)
    _compare(st, obs, psi, ref, L2_TOL_C64, P_TOL_C64)


def test_wide_tiles_fall_back_with_a_uint16_table(qaa):
    """A uint16 table does not fit the 2^14 tile's LDS: the recorded choice
    is ignored for it and the base tile runs (same result)."""
    n, T, N = 22, 4.0, 5
    inst_in = planted_unique_3sat(n, 95)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    try:
        qaa.qaa_plan_set(n, qaa.QAA_C64, {"balance": 0, "passengers": 1, "tiles": 2})
        _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N, etype=qaa.QAA_E_U16)
    finally:
        qaa.qaa_plan_set(n, qaa.QAA_C64, None)
    _compare(st, obs, psi, ref, L2_TOL_C64, P_TOL_C64)


def test_cache_blocked_schedule_vs_oracle(qaa, monkeypatch):
    """The cache-blocking switch (passes between two top-set passes run group
    by group over the top index bits) on the GPU: same result."""
    monkeypatch.setenv("QAA_CHUNK_LOG2_BYTES", "22")
    n, T, N = 23, 4.0, 5
    inst_in = planted_unique_3sat(n, 41)
    psi, ref = _oracle_run(n, inst_in.clauses, T, N)
    try:    # three sets of 2^13 tiles: chunking needs a top set above set 1
        qaa.qaa_plan_set(n, qaa.QAA_C64, {"balance": 0, "passengers": 1, "tiles": 0})
        _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N)
    finally:
        qaa.qaa_plan_set(n, qaa.QAA_C64, None)
    _compare(st, obs, psi, ref, L2_TOL_C64, P_TOL_C64)


def test_autotune_records_a_choice(qaa):
    n = 23
    inst_in = planted_unique_3sat(n, 5)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    st = qaa.State(inst, table)
    try:
        best = qaa.qaa_autotune(st.c, steps=10)
        assert best["balance"] in (0, 1) and best["passengers"] in (0, 1) and best["tiles"] in (0, 1, 2)
        assert best["ms_per_step"] > 0
        assert qaa.qaa_plan_get(n) == {"balance": best["balance"], "passengers": best["passengers"],
                                       "tiles": best["tiles"]}
        # the tuned plan evolves correctly
        T, N = 4.0, 6
        psi, ref = _oracle_run(n, inst_in.clauses, T, N)
        st.init_uniform().evolve(T, N)
        _compare(st, st.observables(), psi, ref, L2_TOL_C64, P_TOL_C64)
    finally:
        qaa.qaa_plan_set(n, qaa.QAA_C64, None)


def test_deterministic(qaa):
    n, T, N = 18, 5.0, 20
    inst_in = planted_unique_3sat(n, 71)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    a = qaa.State(inst, table).init_uniform().evolve(T, N)
    b = qaa.State(inst, table).init_uniform().evolve(T, N)
    torch.cuda.synchronize()
    assert torch.equal(a.amp, b.amp)
    assert a.observables() == b.observables()


def test_observables_match_oracle_on_same_state(qaa):
    n, T, N = 17, 5.0, 30
    inst_in = planted_unique_3sat(n, 81)
    _, _, st, obs = _run_gpu(qaa, n, inst_in.clauses, T, N)
    ref = oracle.observables(n, inst_in.clauses, st.amp.cpu().numpy().astype(np.complex128))
    for k in ("norm", "energy", "p_success"):
        assert abs(obs[k] - ref[k]) <= 1e-12 * max(1.0, abs(ref[k])), k
    assert obs["e_min"] == ref["e_min"] and obs["degeneracy"] == ref["degeneracy"]


def test_batch_equals_individual(qaa):
    """One batched call over uneven n (resident and multi-pass states) gives
    each state what qaa_evolve gives it alone (same plan; the batched passes
    compute their coefficients on the device, so agreement is to rounding)."""
    ns = [6, 10, 13, 14, 15, 17, 21, 22, 14]
    Ts = [3.0, 4.0, 5.0, 6.0, 7.0, 2.5, 4.5, 3.5, 0.0]
    Ns = [30, 40, 50, 20, 9, 10, 7, 5, 0]
    insts, singles, batch = [], [], []
    for i, n in enumerate(ns):
        inst_in = planted_unique_3sat(n, 300 + i)
        inst = qaa.Instance(n, inst_in.literals())
        table = inst.energy_table()
        insts.append((inst, inst_in))
        singles.append(qaa.State(inst, table).init_uniform().evolve(Ts[i], Ns[i]))
        batch.append(qaa.State(inst, table).init_uniform())
    qaa.qaa_evolve_batch([b.c for b in batch], Ts, Ns)
    torch.cuda.synchronize()
    for (inst, inst_in), n, T, N, sgl, b in zip(insts, ns, Ts, Ns, singles, batch):
        diff = float(torch.linalg.vector_norm((sgl.amp - b.amp).to(torch.complex128)).item())
        assert diff < 2e-6, (n, diff)
        if n <= 17:
            psi, ref = _oracle_run(n, inst_in.clauses, T, N)
            _compare(b, b.observables(), psi, ref, L2_TOL_C64, P_TOL_C64)


def test_batch_groups_join_the_callers_stream(qaa):
    """Launch groups after the first run on library streams that are joined
    back into the caller's stream: work queued on that stream right after
    the call (no device synchronisation) sees every state finished."""
    ns, Ts, Ns = [20, 22], [1.0, 4.0], [4, 300]      # the n = 22 group runs long
    insts, batch, tables = [], [], []
    for i, n in enumerate(ns):
        inst = qaa.Instance(n, planted_unique_3sat(n, 500 + i).literals())
        table = inst.energy_table()
        insts.append(inst)
        tables.append(table)
        batch.append(qaa.State(inst, table).init_uniform())
    solo = qaa.State(insts[1], tables[1]).init_uniform().evolve(Ts[1], Ns[1])
    torch.cuda.synchronize()
    caller = torch.cuda.Stream()
    caller.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(caller):
        qaa.qaa_evolve_batch([b.c for b in batch], Ts, Ns, stream=caller)
        snaps = [b.amp.clone() for b in batch]
    torch.cuda.synchronize()
    for snap, b in zip(snaps, batch):
        assert torch.equal(snap, b.amp)
    diff = float(torch.linalg.vector_norm((solo.amp - batch[1].amp).to(torch.complex128)).item())
    assert diff < 2e-6, diff


def test_batch_many_uneven_states_vs_oracle(qaa):
    """A batch drawn like the batched workload (n uniform, T uniform,
    steps = round(T/dt)), shortened: 40 states, n in 12..17, T in [1, 3)."""
    from qaa_inputs import batch_workload
    wl = batch_workload(40, seed=99, n_lo=12, n_hi=17, t_lo=1.0, t_hi=3.0, dt=0.01)
    states, Ts, Ns, ins = [], [], [], []
    for n, T, N, iseed in wl:
        inst_in = planted_unique_3sat(n, iseed)
        inst = qaa.Instance(n, inst_in.literals())
        st = qaa.State(inst, inst.energy_table()).init_uniform()
        states.append(st)
        Ts.append(T)
        Ns.append(N)
        ins.append(inst_in)
    qaa.qaa_evolve_batch([st.c for st in states], Ts, Ns)
    torch.cuda.synchronize()
    for st, inst_in, (n, T, N, _) in list(zip(states, ins, wl))[::5]:
        psi, ref = _oracle_run(n, inst_in.clauses, T, N)
        _compare(st, st.observables(), psi, ref, L2_TOL_C64, P_TOL_C64)


# --------------------------------------------------------------------------
# Full size (n = 28), the launch configuration the benchmark times
# --------------------------------------------------------------------------

def test_full_size_driver_only_closed_form(qaa):
    """m = 0 from |z0> at n = 28: psi(z) = a^{n-d} b^d with Theta = T/2
    (holds for any step count); checked on a sample and by the norm."""
    n, T, N, z0 = 28, 50.0, 6, 0x5A5A5A5
    inst = qaa.Instance(n, [])
    table = inst.energy_table()
    st = qaa.State(inst, table).init_basis(z0).evolve(T, N)
    obs = st.observables()
    th = T / 2.0
    a = (1 + np.exp(-1j * th)) / 2
    b = (1 - np.exp(-1j * th)) / 2
    rng = SplitMix64(5)
    zs = np.asarray([rng.below(1 << n) for _ in range(4096)] + [z0, z0 ^ 1, z0 ^ (1 << 27)], dtype=np.int64)
    got = st.amp[torch.from_numpy(zs).cuda()].cpu().numpy().astype(np.complex128)
    d = np.array([bin(int(z) ^ z0).count("1") for z in zs])
    expect = a ** (n - d) * b ** d
    # FP32 rounding of ~n rotations per step, each step: well under 1e-5
    # relative to the largest amplitude
    assert np.max(np.abs(got - expect)) < 2e-6
    assert abs(obs["norm"] - 1.0) < 1e-6


def test_full_size_c64_vs_c128_first_steps(qaa):
    """n = 28, T = 50, steps 0..4 of 5000: complex64 against the complex128
    GPU path (itself pinned to the oracle at smaller n)."""
    n, T, N, K = 28, 50.0, 5000, 4
    inst_in = planted_unique_3sat(n, 0)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    a = qaa.State(inst, table, dtype=torch.complex64).init_uniform()
    a.evolve_range(T, N, 0, K)
    oa = a.observables()
    b = qaa.State(inst, table, dtype=torch.complex128).init_uniform()
    b.evolve_range(T, N, 0, K)
    ob = b.observables()
    diff = float(torch.linalg.vector_norm(a.amp.to(torch.complex128) - b.amp).item())
    assert diff < 1e-5
    assert abs(oa["p_success"] - ob["p_success"]) < 1e-9
    assert abs(ob["norm"] - 1.0) < 1e-12
    assert abs(oa["norm"] - 1.0) < 1e-5


def test_full_size_first_steps_vs_oracle(qaa):
    """n = 28 seed 0, T = 50, steps 0..9 of 5000 in the benchmark's launch
    configuration (complex64, uint8 table, the three-set pass plan), against
    the complex128 CPU oracle over the whole state vector."""
    n, T, N, K = 28, 50.0, 5000, 10
    inst_in = planted_unique_3sat(n, 0)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    a = qaa.State(inst, table, dtype=torch.complex64).init_uniform()
    a.evolve_range(T, N, 0, K)
    oa = a.observables()
    got = a.amp.cpu().numpy()
    del a, table
    torch.cuda.empty_cache()
    psi = oracle.init_uniform(n)
    oracle.evolve(n, inst_in.clauses, psi, T, N, 0, K)
    ref = oracle.observables(n, inst_in.clauses, psi)
    l2 = float(np.sqrt(np.sum(np.abs(got.astype(np.complex128) - psi) ** 2)))
    assert l2 <= L2_TOL_C64, l2
    assert abs(oa["p_success"] - ref["p_success"]) <= P_TOL_C64
    assert abs(oa["energy"] - ref["energy"]) <= 1e-4 * max(1.0, ref["energy"])
    del psi, got


def test_full_size_full_job_c64_vs_c128(qaa):
    """The benchmark's job in full (n = 28 seed 0, T = 50, 5000 steps):
    complex64 against the complex128 GPU path at the workload's tolerances
    (final-state L2 <= 1e-4, |dP_success| <= 1e-5)."""
    n, T, N = 28, 50.0, 5000
    inst_in = planted_unique_3sat(n, 0)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    a = qaa.State(inst, table, dtype=torch.complex64).init_uniform().evolve(T, N)
    oa = a.observables()
    b = qaa.State(inst, table, dtype=torch.complex128).init_uniform().evolve(T, N)
    ob = b.observables()
    l2 = float(torch.linalg.vector_norm(a.amp.to(torch.complex128) - b.amp).item())
    assert l2 <= L2_TOL_C64, l2
    assert abs(oa["p_success"] - ob["p_success"]) <= P_TOL_C64
    assert abs(oa["energy"] - ob["energy"]) <= 1e-4 * max(1.0, ob["energy"])
    assert abs(ob["norm"] - 1.0) < 1e-10
    assert ob["p_success"] > 0.5          # T = 50 is slow enough to find the planted solution
    del a, b, table
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,N,sets", [(29, 5, 3), (30, 5, 3), (31, 5, 3), (33, 3, 4), (34, 2, 4)])
def test_large_n_driver_only_closed_form(qaa, n, N, sets):
    """n = 29 (3 sets), 30 (3 sets, the top one in 2^14 tiles), 31 (3 sets,
    all in 2^14 tiles; a 16 GiB state), 33 (4 sets, 3 passes per step) and
    the largest n the library accepts, 34 (128 GiB state + 16 GiB table):
    the m = 0 closed form from a basis state, sampled."""
    assert n <= qaa.QAA_MAX_QUBITS
    free, _ = torch.cuda.mem_get_info()
    if free < (9 << n) + (4 << 30):
        pytest.skip("needs %d GiB of free device memory" % (((9 << n) >> 30) + 4))
    T, z0 = 20.0, (0x2B6D5A93 & ((1 << n) - 1))
    assert qaa.qaa_plan_info(n)["sets"] == sets
    inst = qaa.Instance(n, [])
    table = inst.energy_table()
    st = qaa.State(inst, table).init_basis(z0).evolve(T, N)
    obs = st.observables()
    th = T / 2.0
    a = (1 + np.exp(-1j * th)) / 2
    b = (1 - np.exp(-1j * th)) / 2
    rng = SplitMix64(n)
    zs = np.asarray([rng.below(1 << n) for _ in range(4096)] + [z0, z0 ^ 1, z0 ^ (1 << (n - 1))], dtype=np.int64)
    got = st.amp[torch.from_numpy(zs).cuda()].cpu().numpy().astype(np.complex128)
    d = np.array([bin(int(z) ^ z0).count("1") for z in zs])
    expect = a ** (n - d) * b ** d
    assert np.max(np.abs(got - expect)) < 2e-6
    assert abs(obs["norm"] - 1.0) < 1e-6
    del st, table
    torch.cuda.empty_cache()


def test_n29_complex128_four_sets_vs_oracle(qaa):
    """A planted instance at n = 29 in complex128 runs four qubit sets
    (12 + 8 + 8 + 1, three passes per step): against the oracle over the
    whole 2^29-amplitude state, with clauses."""
    n, T, N, K = 29, 50.0, 5000, 3
    free, _ = torch.cuda.mem_get_info()
    if free < (18 << n) + (4 << 30):
        pytest.skip("needs %d GiB of free device memory" % (((18 << n) >> 30) + 4))
    assert qaa.qaa_plan_info(n, qaa.QAA_C128)["sets"] == 4
    inst_in = planted_unique_3sat(n, 0)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    a = qaa.State(inst, table, dtype=torch.complex128).init_uniform()
    a.evolve_range(T, N, 0, K)
    oa = a.observables()
    got = a.amp.cpu().numpy()
    del a, table
    torch.cuda.empty_cache()
    psi = oracle.init_uniform(n)
    oracle.evolve(n, inst_in.clauses, psi, T, N, 0, K)
    ref = oracle.observables(n, inst_in.clauses, psi)
    l2 = float(np.sqrt(np.sum(np.abs(got - psi) ** 2)))
    assert l2 <= L2_TOL_C128, l2
    assert abs(oa["p_success"] - ref["p_success"]) <= 1e-12
    assert abs(oa["energy"] - ref["energy"]) <= 1e-9 * ref["energy"]
    del psi, got


@pytest.mark.parametrize("tiles,sets", [(1, 3), (0, 4)])
def test_n30_c64_vs_c128_first_steps(qaa, tiles, sets):
    """A planted instance at n = 30: complex64 against the complex128 GPU
    path over the first steps of a T = 50, 5000-step run, with the default
    plan (three sets, the top one in 2^14 tiles) and with four sets of
    2^13 tiles (three passes per step)."""
    n, T, N, K = 30, 50.0, 5000, 3
    inst_in = planted_unique_3sat(n, 0)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    info = inst.info()
    assert info["e_min"] == 0 and info["degeneracy"] == 1
    try:
        qaa.qaa_plan_set(n, qaa.QAA_C64, {"balance": 0, "passengers": 1, "tiles": tiles})
        assert qaa.qaa_plan_info(n)["sets"] == sets
        a = qaa.State(inst, table, dtype=torch.complex64).init_uniform()
        a.evolve_range(T, N, 0, K)
        oa = a.observables()
    finally:
        qaa.qaa_plan_set(n, qaa.QAA_C64, None)
    b = qaa.State(inst, table, dtype=torch.complex128).init_uniform()
    b.evolve_range(T, N, 0, K)
    ob = b.observables()
    diff = float(torch.linalg.vector_norm(a.amp.to(torch.complex128) - b.amp).item())
    assert diff < 1e-5
    assert abs(oa["p_success"] - ob["p_success"]) < 1e-10
    assert abs(oa["energy"] - ob["energy"]) < 1e-5 * ob["energy"]
    assert abs(ob["norm"] - 1.0) < 1e-12
    del a, b, table
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# n = 20, T = 100, 10^4 steps against stored oracle results
# --------------------------------------------------------------------------

def _golden_c2():
    path = os.path.join(GOLDEN, "c2_n20_oracle.json")
    if not os.path.exists(path):
        return []
    with open(path) as f:
        return json.load(f)["records"]


def sampled_l2(got, exp, n):
    """Whole-state L2 error estimated from stored samples: entry 0 is the
    planted solution (counted once), entries 1.. are distinct basis states
    drawn uniformly from the other 2^n - 1, so their mean squared error
    scales to the rest of the state."""
    d2 = np.abs(got - exp) ** 2
    rest = float(np.mean(d2[1:])) * ((1 << n) - 1) if d2.size > 1 else 0.0
    return float(np.sqrt(d2[0] + rest))


@pytest.mark.parametrize("rec", _golden_c2(), ids=lambda r: "seed%d" % r["seed"])
def test_n20_T100_10k_steps_vs_stored_oracle(qaa, rec):
    """n = 20, T = 100, 10^4 steps (the workload's full length) against the
    stored oracle run: complex64 P_success within 1e-5, and the final-state
    L2 <= 1e-4 twice over -- estimated from the oracle's stored samples, and
    exactly over all 2^20 amplitudes against a complex128 GPU run of the same
    job whose own samples match the oracle's to 1e-9."""
    n = rec["n"]
    inst_in = planted_unique_3sat(n, rec["seed"])
    assert inst_in.m == rec["m"] and inst_in.planted == rec["planted"]
    inst, table, st, obs = _run_gpu(qaa, n, inst_in.clauses, rec["T"], rec["steps"])
    ref = rec["observables"]
    assert abs(obs["p_success"] - ref["p_success"]) <= P_TOL_C64
    assert abs(obs["energy"] - ref["energy"]) <= 1e-4
    assert abs(obs["norm"] - 1.0) <= 1e-4
    zs = torch.tensor(rec["sample_z"], dtype=torch.int64, device="cuda")
    exp = np.array([complex(a, b) for a, b in rec["sample_amp"]])
    got = st.amp[zs].cpu().numpy().astype(np.complex128)
    assert sampled_l2(got, exp, n) <= L2_TOL_C64
    # the complex128 path over the same job: pinned to the stored samples,
    # then the whole complex64 state against it
    wide = qaa.State(inst, table, dtype=torch.complex128).init_uniform().evolve(rec["T"], rec["steps"])
    ow = wide.observables()
    assert abs(ow["p_success"] - ref["p_success"]) <= 1e-9
    got_w = wide.amp[zs].cpu().numpy()
    assert np.max(np.abs(got_w - exp)) <= 1e-9
    l2 = float(torch.linalg.vector_norm(st.amp.to(torch.complex128) - wide.amp).item())
    assert l2 <= L2_TOL_C64, l2


def _golden_c4():
    with open(os.path.join(GOLDEN, "c4_mix_oracle.json")) as f:
        return json.load(f)["records"]


def test_batch_at_full_length_vs_stored_oracle(qaa):
    """One qaa_evolve_batch call at the batched workload's own lengths: the
    five n = 20, T = 100, 10^4-step states and twelve states of the batched
    mix (n = 13..22, up to 9926 steps; resident, two- and three-set plans,
    coefficients computed on the device), each against its stored oracle
    run: |dP_success| <= 1e-5 and the sampled whole-state L2 <= 1e-4."""
    recs = _golden_c2() + _golden_c4()
    assert len(recs) == 17
    states, keep = [], []
    for rec in recs:
        inst_in = planted_unique_3sat(rec["n"], rec["seed"])
        assert inst_in.m == rec["m"] and inst_in.planted == rec["planted"]
        inst = qaa.Instance(rec["n"], inst_in.literals())
        st = qaa.State(inst, inst.energy_table()).init_uniform()
        states.append(st)
        keep.append(inst)
    qaa.qaa_evolve_batch([st.c for st in states], [r["T"] for r in recs], [r["steps"] for r in recs])
    torch.cuda.synchronize()
    for rec, st in zip(recs, states):
        obs = st.observables()
        ref = rec["observables"]
        zs = torch.tensor(rec["sample_z"], dtype=torch.int64, device="cuda")
        got = st.amp[zs].cpu().numpy().astype(np.complex128)
        exp = np.array([complex(a, b) for a, b in rec["sample_amp"]])
        what = "n=%d T=%.2f steps=%d" % (rec["n"], rec["T"], rec["steps"])
        assert abs(obs["p_success"] - ref["p_success"]) <= P_TOL_C64, what
        assert abs(obs["energy"] - ref["energy"]) <= 1e-4 * max(1.0, ref["energy"]), what
        assert sampled_l2(got, exp, rec["n"]) <= L2_TOL_C64, what


def test_binding_refuses_undersized_device_buffers(qaa):
    inst = qaa.Instance(12, planted_unique_3sat(12, 5).literals())
    small = torch.zeros(1 << 11, dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError, match="needs 2\\^12"):
        qaa.make_state(inst.handle, small)
    with pytest.raises(ValueError, match="needs 2\\^12"):
        qaa.qaa_energy_table(inst.handle, torch.zeros(1 << 11, dtype=torch.uint8, device="cuda"), qaa.QAA_E_U8)
    with pytest.raises(TypeError, match="2-byte"):
        qaa.qaa_energy_table(inst.handle, torch.zeros(1 << 12, dtype=torch.uint8, device="cuda"), qaa.QAA_E_U16)
