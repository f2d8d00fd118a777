"""Seeded input generator: published RNG values, planting and uniqueness."""
import numpy as np
import pytest

import oracle
from qaa_inputs import SplitMix64, batch_workload, planted_unique_3sat, serving_workload


def test_splitmix64_published_values():
    """First outputs for seed 0 as published with the SplitMix64 reference code."""
    r = SplitMix64(0)
    assert [r.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_below_is_in_range_and_covers():
    r = SplitMix64(123)
    xs = [r.below(7) for _ in range(2000)]
    assert min(xs) == 0 and max(xs) == 6
    counts = np.bincount(xs, minlength=7)
    assert counts.min() > 200


@pytest.mark.parametrize("n", [3, 4, 6, 7, 10, 12, 15])
def test_instance_is_unique_and_first_unique(n):
    inst = planted_unique_3sat(n, 100 + n)
    E = oracle.energy(n, inst.clauses)
    assert np.count_nonzero(E == 0) == 1 and E[inst.planted] == 0
    # stopping rule: without the last clause there is more than one solution
    E2 = oracle.energy(n, inst.clauses[:-1])
    assert np.count_nonzero(E2 == 0) > 1


def test_clauses_have_distinct_variables_and_valid_literals():
    inst = planted_unique_3sat(16, 5)
    v = np.abs(inst.clauses)
    assert v.min() >= 1 and v.max() <= 16
    assert all(len(set(row)) == 3 for row in v.tolist())


def test_deterministic():
    a = planted_unique_3sat(11, 77)
    b = planted_unique_3sat(11, 77)
    assert np.array_equal(a.clauses, b.clauses) and a.planted == b.planted


def test_large_n_bitset_path_agrees_with_candidates():
    """n = 18 runs through the bitset and then the candidate list; the
    oracle's exhaustive energy confirms the planted state is the only zero."""
    inst = planted_unique_3sat(18, 3)
    E = oracle.energy(18, inst.clauses)
    assert np.count_nonzero(E == 0) == 1 and E[inst.planted] == 0


def test_workload_recipes():
    w = batch_workload(64, seed=1)
    assert len(w) == 64
    for n, T, steps, s in w:
        assert 12 <= n <= 22 and 10 <= T < 100 and steps == round(T / 0.01)
    reqs = serving_workload(50, rate=0.5, seed=2)
    arr = [r["arrival"] for r in reqs]
    assert all(b > a for a, b in zip(arr, arr[1:]))
    assert all(16 <= r["n"] <= 31 for r in reqs)
