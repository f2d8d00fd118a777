"""The allocation-free evolution entry point (qaa_evolve_range_noalloc)
against qaa_evolve_range, through the C ABI: two calls in a row (the second
on a smaller state), bit-identical results, and the oracle's bar.  Named to
be collected last: it must pass both alone and after every other test."""
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


def _pair(qaa, n, seed):
    inst_in = planted_unique_3sat(n, seed)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    a = qaa.State(inst, table).init_uniform()
    b = qaa.State(inst, table).init_uniform()
    return inst_in, inst, a, b


# a three-set plan, then a smaller two-set plan, then a state held in one
# workgroup (no scratch at all), then the three-set plan again
CASES = [(22, 5.0, 12, 0, 12), (16, 6.0, 40, 5, 31), (10, 3.0, 30, 0, 30), (23, 4.0, 9, 2, 9)]


def test_noalloc_equals_evolve_range_in_a_row(qaa):
    for n, T, N, k0, k1 in CASES:
        print("case n=%d T=%g N=%d range %d..%d" % (n, T, N, k0, k1), flush=True)
        inst_in, inst, a, b = _pair(qaa, n, 600 + n)
        qaa.qaa_evolve_range(a.c, T, N, k0, k1)
        qaa.qaa_evolve_range_noalloc(b.c, T, N, k0, k1)
        torch.cuda.synchronize()
        assert torch.equal(a.amp, b.amp), n
        # and the oracle's bar on the same range
        psi = oracle.init_uniform(n)
        oracle.evolve(n, inst_in.clauses, psi, T, N, k0, k1)
        got = b.amp.cpu().numpy().astype(np.complex128)
        assert np.linalg.norm(got - psi) <= 1e-4
        ob, ref = b.observables(), oracle.observables(n, inst_in.clauses, psi)
        assert abs(ob["p_success"] - ref["p_success"]) <= 1e-5
        inst.close()


def test_noalloc_on_a_side_stream_and_schedule_table(qaa):
    """The caller's stream and a schedule table pass through unchanged."""
    n, T, N = 18, 4.0, 20
    knots = [0.0, 0.2, 0.7, 1.0]
    _, inst, a, b = _pair(qaa, n, 640)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    qaa.qaa_evolve_range(a.c, T, N, 0, N, knots=knots)
    qaa.qaa_evolve_range_noalloc(b.c, T, N, 0, N, stream=s, knots=knots)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(a.amp, b.amp)
    inst.close()


def test_noalloc_rejects_like_evolve_range(qaa):
    _, inst, a, b = _pair(qaa, 15, 650)
    with pytest.raises(qaa.QaaError) as ei:
        qaa.qaa_evolve_range_noalloc(b.c, 1.0, 10, 5, 11)
    assert ei.value.status == qaa.QAA_ERR_INVALID_ARG
    with pytest.raises(qaa.QaaError):
        qaa.qaa_evolve_range_noalloc(b.c, float("nan"), 10, 0, 10)
    inst.close()
