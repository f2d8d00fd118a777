"""The energy kernel's bit-sliced counting (carry-save planes over 32 basis
states per thread), run on the host through qaa_debug_energy_block, against
the oracle's clause-by-clause E(z) (Sec. 4.3).  No GPU."""
import numpy as np
import pytest

import oracle
import paper_1103_1399_amd as qaa
from qaa_inputs import SplitMix64, planted_unique_3sat


def _blocks(n, clauses, z0s):
    h = qaa.qaa_instance_create(n, np.asarray(clauses, np.int32).reshape(-1))
    try:
        return {z0: qaa.qaa_debug_energy_block(h, z0) for z0 in z0s}
    finally:
        qaa.qaa_instance_destroy(h)


def _random_clauses(n, m, seed):
    rng = SplitMix64(seed)
    out = []
    for _ in range(m):
        vs = []
        while len(vs) < 3:
            v = 1 + rng.below(n)
            if v not in vs:
                vs.append(v)
        out.append([v if rng.below(2) else -v for v in vs])
    return np.asarray(out, np.int32).reshape(-1, 3)


@pytest.mark.parametrize("n,m,seed", [(5, 0, 1), (5, 7, 2), (8, 8, 3), (10, 41, 4), (12, 255, 5), (12, 256, 6),
                                      (14, 300, 7), (16, 97, 8), (9, 1000, 9)])
def test_block_counts_match_the_oracle(n, m, seed):
    """Every 32-state block of small instances (eight-clause tree, ripple
    tail, 8 and 16 counter planes), and sampled blocks of larger ones."""
    cl = _random_clauses(n, m, seed)
    E = oracle.energy(n, cl)
    z0s = list(range(0, 1 << n, 32))
    if len(z0s) > 64:
        rng = SplitMix64(seed)
        z0s = sorted({32 * rng.below((1 << n) // 32) for _ in range(64)} | {0, (1 << n) - 32})
    for z0, got in _blocks(n, cl, z0s).items():
        assert got == E[z0:z0 + 32].tolist(), z0


def test_planted_instance_at_high_bits():
    """Clauses on bits >= 5 only and mixed ones, on a planted instance with
    n = 20: the planted block has its zero, sampled blocks match."""
    inst = planted_unique_3sat(20, 3)
    zs = [inst.planted & ~31] + [32 * k for k in (0, 1, 777, 32767)]
    got = _blocks(20, inst.clauses, zs)
    for z0, e in got.items():
        ref = oracle.energy_at(20, inst.clauses, np.arange(z0, z0 + 32, dtype=np.uint64))
        assert e == ref.tolist()
    assert got[inst.planted & ~31][inst.planted & 31] == 0


def test_tiny_n_and_overflow_width():
    """n < 5 (one partial block) and counts above 255 (16 planes)."""
    for n in (3, 4):
        cl = [[1, -2, 3]] * 5
        E = oracle.energy(n, cl)
        got = _blocks(n, cl, [0])[0]
        assert got[:1 << n] == E.tolist()
    cl = [[1, 2, 3]] * 300
    E = oracle.energy(5, cl)
    assert _blocks(5, cl, [0])[0] == E.tolist()
    assert max(E) == 300


def test_rejects_misaligned_block():
    h = qaa.qaa_instance_create(8, [1, 2, 3])
    try:
        with pytest.raises(qaa.QaaError):
            qaa.qaa_debug_energy_block(h, 16)
        with pytest.raises(qaa.QaaError):
            qaa.qaa_debug_energy_block(h, 256)
    finally:
        qaa.qaa_instance_destroy(h)
