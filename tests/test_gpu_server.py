"""GPU tests of the solve-request server (qaa_server_*): every result equals
the same solve run alone through qaa_evolve, admission never exceeds the HBM
budget, and oversize or malformed requests are reported."""
import time

import numpy as np
import pytest

import oracle
from qaa_inputs import planted_unique_3sat

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qaa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1103_1399_amd as m
    return m


def _solo(qaa, n, lits, T, steps, knots=None):
    inst = qaa.Instance(n, lits)
    table = inst.energy_table()
    st = qaa.State(inst, table)
    st.init_uniform()
    st.evolve(T, steps, knots=knots)
    obs = st.observables()
    torch.cuda.synchronize()
    inst.close()
    return obs


def _mix():
    reqs = []
    for i, (n, T, steps) in enumerate([(8, 4.0, 40), (11, 5.0, 50), (14, 5.0, 30), (16, 6.0, 30), (9, 3.0, 25),
                                       (18, 5.0, 12), (13, 6.0, 60), (15, 4.0, 20), (20, 5.0, 6), (12, 2.0, 17)]):
        inst = planted_unique_3sat(n, 100 + i)
        reqs.append((n, inst.literals(), T, steps))
    return reqs


def test_server_results_equal_solo_runs(qaa):
    reqs = _mix()
    sv = qaa.qaa_server_create(hbm_budget_bytes=1 << 30, slots=4)
    try:
        tickets = [qaa.qaa_server_submit(sv, n, lits, T, steps) for n, lits, T, steps in reqs]
        results = [qaa.qaa_server_wait(sv, t) for t in tickets]
    finally:
        qaa.qaa_server_destroy(sv)
    for (n, lits, T, steps), r in zip(reqs, results):
        assert r["done"] and r["status"] == qaa.QAA_OK, (n, r)
        assert 0.0 <= r["queued_s"] <= r["latency_s"]
        solo = _solo(qaa, n, lits, T, steps)
        # same kernels, same plan, deterministic reductions: identical numbers
        for key in ("norm", "energy", "p_success", "e_min", "degeneracy"):
            assert r[key] == solo[key], (n, key, r[key], solo[key])


def test_server_result_matches_oracle(qaa):
    n, T, steps = 12, 6.0, 80
    inst = planted_unique_3sat(n, 7)
    sv = qaa.qaa_server_create(hbm_budget_bytes=1 << 28, slots=1)
    try:
        r = qaa.qaa_server_wait(sv, qaa.qaa_server_submit(sv, n, inst.literals(), T, steps))
    finally:
        qaa.qaa_server_destroy(sv)
    psi = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, psi, T, steps)
    ref = oracle.observables(n, inst.clauses, psi)
    assert abs(r["p_success"] - ref["p_success"]) <= 1e-5
    assert abs(r["energy"] - ref["energy"]) <= 1e-4
    assert abs(r["norm"] - 1.0) <= 1e-5


def test_server_admission_respects_budget(qaa):
    n = 18
    insts = [planted_unique_3sat(n, 200 + i) for i in range(6)]
    fp = max(qaa.qaa_server_footprint(n, inst.m) for inst in insts)
    assert fp >= (1 << n) * 9
    sv = qaa.qaa_server_create(hbm_budget_bytes=2 * fp, slots=4)
    try:
        tickets = [qaa.qaa_server_submit(sv, n, inst.literals(), 5.0, 40) for inst in insts]
        peak = 0
        while True:
            s = qaa.qaa_server_stats(sv)
            peak = max(peak, s["bytes_in_use"])
            assert s["running"] <= 2 and s["bytes_in_use"] <= 2 * fp
            if s["queued"] == 0 and s["running"] == 0:
                break
        res = [qaa.qaa_server_wait(sv, t) for t in tickets]
        assert all(r["done"] and r["status"] == qaa.QAA_OK for r in res)
        assert qaa.qaa_server_stats(sv)["bytes_in_use"] == 0
        # too large for the whole budget: refused at submit
        with pytest.raises(qaa.QaaError) as e:
            qaa.qaa_server_submit(sv, n + 2, planted_unique_3sat(n + 2, 1).literals(), 1.0, 1)
        assert e.value.status == qaa.QAA_ERR_OUT_OF_MEMORY
        # malformed clauses: reported through the result
        t = qaa.qaa_server_submit(sv, 5, [1, 2, 9], 1.0, 1)
        r = qaa.qaa_server_wait(sv, t)
        assert r["done"] and r["status"] == qaa.QAA_ERR_INVALID_ARG
    finally:
        qaa.qaa_server_destroy(sv)


def test_server_requests_with_schedule_tables(qaa):
    """Each request may carry its own schedule; results equal the solo runs
    with the same table, and a bad table is refused at submit."""
    tabs = [[0.0, 0.4, 0.5, 0.6, 1.0], None, [0.0, 0.9, 0.2, 1.0], list(np.linspace(0, 1, 256) ** 2)]
    reqs = [(n, planted_unique_3sat(n, 400 + n).literals(), 5.0, 30) for n in (10, 14, 17, 12)]
    sv = qaa.qaa_server_create(hbm_budget_bytes=1 << 30, slots=2)
    try:
        with pytest.raises(qaa.QaaError) as ei:
            qaa.qaa_server_submit(sv, 10, reqs[0][1], 5.0, 30, knots=[0.0, 1.5])
        assert ei.value.status == qaa.QAA_ERR_INVALID_ARG
        tickets = [qaa.qaa_server_submit(sv, n, lits, T, steps, knots=k) for (n, lits, T, steps), k in zip(reqs, tabs)]
        results = [qaa.qaa_server_wait(sv, t) for t in tickets]
    finally:
        qaa.qaa_server_destroy(sv)
    for (n, lits, T, steps), k, r in zip(reqs, tabs, results):
        assert r["done"] and r["status"] == qaa.QAA_OK, (n, r)
        solo = _solo(qaa, n, lits, T, steps, knots=k)
        for key in ("norm", "energy", "p_success"):
            assert r[key] == solo[key], (n, key, r[key], solo[key])
    # the tables took effect: the first request differs from its linear run
    lin = _solo(qaa, *reqs[0])
    assert lin["p_success"] != results[0]["p_success"]


def test_server_footprint_charges_what_a_solve_can_hold(qaa):
    n = 20
    assert qaa.qaa_server_footprint(n, 200) == (1 << n) * 9 + 16 * 200 + (64 << 10)
    # more than 255 clauses: the table may widen to uint16
    assert qaa.qaa_server_footprint(n, 300) == (1 << n) * 10 + 16 * 300 + (64 << 10)
    assert qaa.qaa_server_footprint(0, 10) == 0 and qaa.qaa_server_footprint(n, -1) == 0


def test_server_overlaps_solves(qaa):
    """Continuous batching: a short request submitted while a long one runs
    is admitted into the free slot and finishes first; the long one is
    still running when the short one is done, so both were on the device
    at once (nothing in the library serialises them)."""
    long_inst = planted_unique_3sat(22, 11)
    short_inst = planted_unique_3sat(12, 12)
    sv = qaa.qaa_server_create(hbm_budget_bytes=1 << 32, slots=2)
    try:
        t_long = qaa.qaa_server_submit(sv, 22, long_inst.literals(), 100.0, 10000)
        t0 = time.perf_counter()
        while qaa.qaa_server_stats(sv)["running"] < 1:
            assert time.perf_counter() - t0 < 30
        t_short = qaa.qaa_server_submit(sv, 12, short_inst.literals(), 2.0, 200)
        r_short = qaa.qaa_server_wait(sv, t_short)
        r_long = qaa.qaa_server_poll(sv, t_long)
        assert r_short["done"] and r_short["status"] == qaa.QAA_OK
        assert not r_long["done"], "the short solve waited for the long one"
        assert r_short["queued_s"] < 0.1
        r_long = qaa.qaa_server_wait(sv, t_long)
        assert r_long["done"] and r_long["status"] == qaa.QAA_OK
        assert r_long["latency_s"] > r_short["latency_s"]
    finally:
        qaa.qaa_server_destroy(sv)


def test_server_reports_progress_of_chunked_solves(qaa):
    """A solve longer than one chunk of steps (2^13 steps at n = 22) runs as
    several qaa_evolve_range calls: poll reports the steps finished, and the
    result matches the same solve in one qaa_evolve call (a chunk boundary
    applies two half-phases where one call merges them)."""
    n, T, steps = 22, 90.0, 9000
    lits = planted_unique_3sat(n, 140).literals()
    sv = qaa.qaa_server_create(hbm_budget_bytes=1 << 30, slots=1)
    seen = set()
    try:
        t = qaa.qaa_server_submit(sv, n, lits, T, steps)
        while True:
            r = qaa.qaa_server_poll(sv, t)
            assert r["steps"] == steps and 0 <= r["steps_done"] <= steps
            seen.add(r["steps_done"])
            if r["done"]:
                break
            time.sleep(0.001)
    finally:
        qaa.qaa_server_destroy(sv)
    assert r["status"] == qaa.QAA_OK and r["steps_done"] == steps
    assert seen <= {0, 8192, steps}
    solo = _solo(qaa, n, lits, T, steps)
    for key in ("norm", "energy", "p_success"):
        assert abs(r[key] - solo[key]) <= 1e-6 * max(1.0, abs(solo[key])), key
    assert r["e_min"] == solo["e_min"] and r["degeneracy"] == solo["degeneracy"]


def test_server_cancels_queued_and_running_requests(qaa):
    """One slot: a long solve runs, two more wait.  Cancelling a queued one
    takes it out at once; cancelling the running one stops it at a chunk
    boundary (2^11 steps at n = 24); the last one then runs to the end with
    the same result as alone."""
    long_lits = planted_unique_3sat(24, 150).literals()
    small = planted_unique_3sat(14, 151)
    sv = qaa.qaa_server_create(hbm_budget_bytes=1 << 30, slots=1)
    try:
        t_long = qaa.qaa_server_submit(sv, 24, long_lits, 3000.0, 300000)
        t_q1 = qaa.qaa_server_submit(sv, 14, small.literals(), 4.0, 40)
        t_q2 = qaa.qaa_server_submit(sv, 14, small.literals(), 4.0, 40)
        while qaa.qaa_server_poll(sv, t_long)["steps_done"] == 0:
            time.sleep(0.01)
        qaa.qaa_server_cancel(sv, t_q1)
        r1 = qaa.qaa_server_poll(sv, t_q1)
        assert r1["done"] and r1["status"] == qaa.QAA_ERR_CANCELLED and r1["steps_done"] == 0
        qaa.qaa_server_cancel(sv, t_long)
        rl = qaa.qaa_server_wait(sv, t_long)
        assert rl["status"] == qaa.QAA_ERR_CANCELLED
        assert 0 < rl["steps_done"] < 300000 and rl["steps_done"] % 2048 == 0
        r2 = qaa.qaa_server_wait(sv, t_q2)
        assert r2["status"] == qaa.QAA_OK and r2["steps_done"] == 40
        qaa.qaa_server_cancel(sv, t_q2)            # finished: unchanged
        assert qaa.qaa_server_poll(sv, t_q2)["status"] == qaa.QAA_OK
        with pytest.raises(qaa.QaaError) as ei:
            qaa.qaa_server_cancel(sv, 10 ** 9)
        assert ei.value.status == qaa.QAA_ERR_INVALID_ARG
    finally:
        qaa.qaa_server_destroy(sv)
    solo = _solo(qaa, 14, small.literals(), 4.0, 40)
    for key in ("norm", "energy", "p_success"):
        assert r2[key] == solo[key], key
