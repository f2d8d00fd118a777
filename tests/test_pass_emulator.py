"""Host-side replay of the pass plan (no GPU).

The library exports the exact pass descriptors it would launch
(qaa_debug_pass_descs).  This test replays them in numpy, complex128:
  * every pass's (workgroup, thread, register) -> basis-state map is a
    bijection onto [0, 2^n) (no element skipped, none touched twice);
  * every residency's (thread, register) -> tile-slot map is a bijection
    onto the 2^TB slots, and the LDS swizzle is a permutation;
  * applying the descriptors' operations (rotations with their
    coefficients, the diagonal phase with its LUT angle and global phase)
    reproduces the CPU oracle's evolution to 1e-12.
The kernels' device code itself is covered by the GPU parity tests.
"""
import numpy as np
import pytest

import oracle
import paper_1103_1399_amd as qaa
from qaa_inputs import planted_unique_3sat


def _pdep(x, positions):
    """Place bit k of x at positions[k] (vectorised over x)."""
    out = np.zeros_like(x)
    for k, p in enumerate(positions):
        out |= ((x >> k) & 1) << p
    return out


def _pad(l, dtype):
    return l + (2 * (l >> 5) if dtype == 0 else (l >> 4))


def _replay(n, dtype, E, psi, T, N, k0, k1, knots=None, tile_bits=0, any_tile=False):
    descs = qaa.qaa_debug_pass_descs(n, dtype, int(E.max()), T, N, k0, k1, knots, tile_bits=tile_bits)
    if not descs:
        return psi, descs
    for d in descs:
        # register bits per thread the pass was planned for (complex64
        # two-set plans in 2^13 tiles use 4, other complex64 plans 5)
        RB = d.reg_bits
        assert RB == (5 if dtype == qaa.QAA_C64 else 4) or (dtype == qaa.QAA_C64 and RB == 4)
        R = 1 << RB
        # each pass's tile size (sets may differ: 2^14-amplitude top sets)
        TB = n - d.n_rest
        if tile_bits and not any_tile:
            assert TB == tile_bits
        assert TB in ((9, 10, 11, 12, 13, 14) if dtype == qaa.QAA_C64 else (8, 9, 10, 11, 12))
        WB = TB - RB
        WG = 1 << WB
        TSP = _pad(1 << TB, dtype)
        tid = np.arange(WG, dtype=np.int64)
        tile_pos = list(d.tile_pos[:TB])
        rest_pos = list(d.rest_pos[:d.n_rest])
        assert sorted(tile_pos + rest_pos) == list(range(n))
        assert d.rest_mask == sum(1 << b for b in rest_pos)
        assert tile_pos[:4] == [0, 1, 2, 3]             # 16-byte energy chunks are contiguous
        assert d.tile_begin + d.tile_count <= (1 << d.n_rest)
        blocks = np.arange(d.tile_begin, d.tile_begin + d.tile_count, dtype=np.int64)
        base = _pdep(blocks, rest_pos)                                  # [B]
        last = d.n_res - 1
        lts, ljs = [], []
        for r in range(d.n_res):
            tp = list(d.tpos[r][:WB])
            lj = np.array(list(d.lj[r][:R]), dtype=np.int64)
            ljp = np.array(list(d.ljp[r][:R]), dtype=np.int64)
            assert np.array_equal(ljp, _pad(lj, dtype))
            lt = _pdep(tid, tp)
            l = lt[:, None] | lj[None, :]                                # [WG, R]
            assert np.array_equal(np.sort(l.reshape(-1)), np.arange(1 << TB))
            # padded LDS slots: in range and distinct
            lp = _pad(lt, dtype)[:, None] + ljp[None, :]
            assert lp.max() < TSP and np.unique(lp).size == lp.size
            if dtype == 0:                                              # register pairs adjacent
                assert np.all(lj[1::2] == lj[0::2] + 1)
            lts.append(lt)
            ljs.append(lj)
        # global maps of the first and last residency agree with the tile map
        for r, gpos, goff in ((0, d.gpos_first, d.goff_first), (last, d.gpos_last, d.goff_last)):
            tg = _pdep(tid, list(gpos[:WB]))
            gof = np.array(list(goff[:R]), dtype=np.int64)
            g_direct = tg[:, None] | gof[None, :]
            g_tile = _pdep(lts[r][:, None] | ljs[r][None, :], tile_pos)
            assert np.array_equal(g_direct, g_tile)
            if dtype == 0:                                              # lanes cover contiguous 256 B
                assert list(gpos[:4]) == [1, 2, 3, 4]
            else:
                assert list(gpos[:4]) == [0, 1, 2, 3]
        l_all = np.arange(1 << TB, dtype=np.int64)
        g = base[:, None] | _pdep(l_all, tile_pos)[None, :]             # [B, TS]
        assert np.unique(g).size == g.size
        tiles = psi[g]
        etile = E[g]
        for t, sn in ((d.tA, d.sA), (d.tB, d.sB)):
            if t or sn:
                # three shears by (t, s, t) compose to the rotation with
                # cos = 1 - t s: t = tan(theta/4) and s = sin(theta/2)
                c = 1.0 - t * sn
                assert abs(c * c + sn * sn - 1.0) < 1e-15
                assert abs(2.0 * t / (1.0 + t * t) - sn) < 1e-15
        lut = np.exp(-1j * (d.phi * np.arange(int(E.max()) + 1) + d.gphase))
        for r in range(d.n_res):
            l = lts[r][:, None] | ljs[r][None, :]
            v = tiles[:, l]                                             # [B, WG, R]

            def rot(v, mask, t, s):
                for b in range(RB):
                    if (mask >> b) & 1:
                        lo = [j for j in range(R) if not (j >> b) & 1]
                        hi = [j | (1 << b) for j in lo]
                        x0, x1 = v[..., lo].copy(), v[..., hi].copy()
                        c = 1.0 - t * s
                        v[..., lo] = c * x0 + 1j * s * x1
                        v[..., hi] = c * x1 + 1j * s * x0
                return v

            v = rot(v, d.masks[r] & 0xFF, d.tA, d.sA)
            if r == d.phase_at:
                v = v * lut[etile[:, l]]
            v = rot(v, (d.masks[r] >> 8) & 0xFF, d.tB, d.sB)
            tiles[:, l] = v
        psi[g] = tiles
    return psi, descs


@pytest.mark.parametrize("n,dtype,T,N", [(14, 0, 5.0, 4), (16, 0, 6.0, 3), (21, 0, 5.0, 2), (22, 0, 5.0, 1),
                                         (13, 1, 5.0, 4), (17, 1, 5.0, 3),
                                         # large steps: rotation angles reduced by pi (odd and even n)
                                         (15, 0, 50.0, 5), (14, 0, 40.0, 3)])
def test_pass_plan_replays_the_oracle(n, dtype, T, N):
    inst = planted_unique_3sat(n, 500 + n)
    E = oracle.energy(n, inst.clauses).astype(np.int64)
    psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
    got, descs = _replay(n, dtype, E, psi, T, N, 0, N)
    sets = qaa.qaa_plan_info(n, dtype)["sets"]
    full = [d for d in descs if d.tile_count == (1 << d.n_rest)]
    if len(full) == len(descs):
        assert len(descs) == (sets - 1) * N + 1
    ref = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, ref, T, N)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("n,dtype,tile_bits,sets,T,N", [
    (16, 0, 10, 3, 6.0, 3),     # 10 + 5 + 1: a ragged top set
    (20, 0, 10, 3, 5.0, 2),     # 10 + 5 + 5: three full sets, as n = 28 runs
    (18, 0, 9, 4, 5.0, 2),      # 9 + 4 + 4 + 1: four sets, as n = 30..34 run
    (19, 0, 9, 4, 4.0, 2),      # 9 + 4 + 4 + 2
    (17, 1, 9, 3, 5.0, 3),      # complex128: 9 + 5 + 3
    (17, 1, 8, 4, 5.0, 2),      # complex128: 8 + 4 + 4 + 1
    (21, 1, 8, 5, 5.0, 1),      # complex128: 8 + 4 + 4 + 4 + 1
])
def test_smaller_tile_plans_replay_the_oracle(n, dtype, tile_bits, sets, T, N):
    """The planner's plans for smaller tiles: three, four and five qubit
    sets (the shapes n = 28..34 run with the library's tiles) at sizes the
    oracle handles, with clauses, replayed against the oracle.  Covers the
    zig-zag set order, the passenger-qubit move and the turn passes of
    every plan depth."""
    inst = planted_unique_3sat(n, 700 + n)
    E = oracle.energy(n, inst.clauses).astype(np.int64)
    psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
    got, descs = _replay(n, dtype, E, psi, T, N, 0, N, tile_bits=tile_bits)
    n_sets = len({d.set_id for d in descs})
    assert n_sets == sets
    assert len(descs) == (n_sets - 1) * N + 1
    ref = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, ref, T, N)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("n,dtype,tile_bits,spread,T,N", [
    (20, 0, 10, 2, 5.0, 2),     # 10 + (3 + 2) + 5: set 1 takes the 2 highest qubits
    (20, 0, 10, 4, 4.0, 2),     # 10 + (1 + 4) + 5
    (18, 0, 10, 1, 5.0, 3),     # 10 + (4 + 1) + 3 (ragged top set)
    (17, 1, 9, 2, 5.0, 2),      # complex128: 9 + (3 + 2) + 3
])
def test_spread_plans_replay_the_oracle(n, dtype, tile_bits, spread, T, N, monkeypatch):
    """Three-set plans whose set 1 takes the highest qubits and whose top set
    takes the run between (the library's layout from n = 30 on), replayed
    against the oracle."""
    monkeypatch.setenv("QAA_PLAN_SPREAD", str(spread))
    inst = planted_unique_3sat(n, 720 + n)
    E = oracle.energy(n, inst.clauses).astype(np.int64)
    psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
    got, descs = _replay(n, dtype, E, psi, T, N, 0, N, tile_bits=tile_bits)
    assert len({d.set_id for d in descs}) == 3
    s1 = [d for d in descs if d.set_id == 1][0]
    assert n - 1 in [s1.tile_pos[j] for j in range(s1.n - s1.n_rest)]     # set 1 holds the top qubit
    ref = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, ref, T, N)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("n,tile_bits,tiles,sets,T,N,passengers", [
    (22, 0, 1, 2, 5.0, 1, (0,)),        # the library's n = 22: 13 + 9, the top set in a 2^14 tile
    (18, 9, 1, 3, 5.0, 2, (0, 1)),      # 9 + 4 + 5: three sets, the top one wide (as n = 30)
    (19, 9, 1, 4, 4.0, 2, (1,)),        # 9 + 4 + 4 + 2: four sets, the top one wide
    (19, 9, 2, 3, 4.0, 2, (0, 1)),      # 10 + 5 + 4: every set wide, the high qubits split evenly
    (20, 9, 2, 3, 4.0, 2, (1,)),        # 10 + 5 + 5 (as n = 31, 32)
])
def test_wide_tile_plans_replay_the_oracle(n, tile_bits, tiles, sets, T, N, passengers):
    """Plans with wide tiles (the top set only, or every set with the high
    qubits split evenly) replayed against the oracle, with clauses and both
    choices of the passenger move where three sets allow it: the library's
    2^14 tiles at n = 22, and the same shapes at smaller n with base tiles
    of 2^9 amplitudes and wide ones of 2^10."""
    inst = planted_unique_3sat(n, 800 + n)
    E = oracle.energy(n, inst.clauses).astype(np.int64)
    ref = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, ref, T, N)
    wide = tile_bits + 1 if tile_bits else 14
    for pas in passengers:
        try:
            qaa.qaa_plan_set(n, qaa.QAA_C64, {"balance": 0, "passengers": pas, "tiles": tiles})
            psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
            got, descs = _replay(n, 0, E, psi, T, N, 0, N, tile_bits=tile_bits, any_tile=True)
        finally:
            qaa.qaa_plan_set(n, qaa.QAA_C64, None)
        tbs = sorted({n - d.n_rest for d in descs})
        assert wide in tbs
        n_sets = len({d.set_id for d in descs})
        assert n_sets == sets
        assert len(descs) == (n_sets - 1) * N + 1
        assert np.max(np.abs(got - ref)) < 1e-12


def test_smaller_tile_override_is_checked():
    with pytest.raises(qaa.QaaError):
        qaa.qaa_debug_pass_descs(20, 0, 10, 5.0, 10, 0, 10, tile_bits=8)
    with pytest.raises(qaa.QaaError):
        qaa.qaa_debug_pass_descs(20, 0, 10, 5.0, 10, 0, 10, tile_bits=14)
    # the library's own tile size gives the library's own plan
    a = qaa.qaa_debug_pass_descs(20, 0, 10, 5.0, 10, 0, 10, tile_bits=13)
    b = qaa.qaa_debug_pass_descs(20, 0, 10, 5.0, 10, 0, 10)
    assert [bytes(x) for x in a] == [bytes(x) for x in b]


@pytest.mark.parametrize("n,T,N,chunk_log2", [(22, 5.0, 2, 19), (22, 4.0, 2, 20)])
def test_chunked_schedule_replays_the_oracle(n, T, N, chunk_log2, monkeypatch):
    """Passes between two passes over the top qubit set run chunk group by
    chunk group; the reordered launches still give the oracle's result."""
    monkeypatch.setenv("QAA_CHUNK_LOG2_BYTES", str(chunk_log2))
    inst = planted_unique_3sat(n, 600 + n)
    E = oracle.energy(n, inst.clauses).astype(np.int64)
    psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
    try:    # three sets of 2^13 tiles (chunking needs a top set above set 1)
        qaa.qaa_plan_set(n, qaa.QAA_C64, {"balance": 0, "passengers": 1, "tiles": 0})
        got, descs = _replay(n, 0, E, psi, T, N, 0, N)
    finally:
        qaa.qaa_plan_set(n, qaa.QAA_C64, None)
    cbits = min(n + 3 - chunk_log2, n - 21)        # the top qubit set starts at bit 21
    assert any(d.tile_count < (1 << d.n_rest) for d in descs)
    assert all(d.tile_count in ((1 << d.n_rest), (1 << (d.n_rest - cbits))) for d in descs)
    ref = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, ref, T, N)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("n,tile_bits,choice", [
    (16, 0, {"balance": 0, "passengers": 0, "tiles": 0}), (16, 0, {"balance": 1, "passengers": 0, "tiles": 0}),
    # three sets (10 + 5 + 3 with 10-bit tiles, the shape of n = 22..29)
    (18, 10, {"balance": 0, "passengers": 0, "tiles": 0}), (18, 10, {"balance": 1, "passengers": 0, "tiles": 0}),
    (18, 10, {"balance": 0, "passengers": 1, "tiles": 0}), (18, 10, {"balance": 1, "passengers": 1, "tiles": 0})])
def test_every_plan_choice_replays_the_oracle(n, tile_bits, choice):
    """Which set rotates which qubit is a free choice (qaa_plan_set); every
    choice must still rotate each qubit exactly once per step."""
    T, N = 5.0, 2          # two steps: first, middle, both turns and last passes
    inst = planted_unique_3sat(n, 700 + n)
    E = oracle.energy(n, inst.clauses).astype(np.int64)
    psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
    try:
        qaa.qaa_plan_set(n, 0, choice)
        got, _ = _replay(n, 0, E, psi, T, N, 0, N, tile_bits=tile_bits)
    finally:
        qaa.qaa_plan_set(n, 0, None)
    ref = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, ref, T, N)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_pass_plan_range_replay():
    n, T, N = 17, 5.0, 9
    inst = planted_unique_3sat(n, 7)
    E = oracle.energy(n, inst.clauses).astype(np.int64)
    psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
    psi, _ = _replay(n, 0, E, psi, T, N, 0, 4)
    psi, _ = _replay(n, 0, E, psi, T, N, 4, N)
    ref = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, ref, T, N)
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_pass_descs_for_whole_tile_states_are_empty():
    assert qaa.qaa_debug_pass_descs(13, 0, 10, 5.0, 10, 0, 10) == []
    assert qaa.qaa_debug_pass_descs(20, 0, 10, 5.0, 10, 3, 3) == []


def _tables():
    rng = np.random.default_rng(11)
    return {
        "3 knots": [0.0, 0.7, 1.0],
        "17 knots, slow middle": list(0.5 + 0.5 * np.sin(np.linspace(-np.pi / 2, np.pi / 2, 17)) ** 3),
        "256 random knots": list(np.sort(rng.random(256))),
        "non-monotone": [0.0, 0.9, 0.2, 1.0],
    }


@pytest.mark.parametrize("name,n,dtype,T,N",
                         [(name, n, dt, T, N) for name in _tables() for (n, dt, T, N) in ((16, 0, 6.0, 5),
                                                                                          (15, 1, 7.0, 4))]
                         + [("256 random knots", 18, 0, 5.0, 3)])      # three qubit sets (10-bit tiles)
def test_table_schedule_replays_the_oracle(name, n, dtype, T, N):
    """The host planner's coefficients for a schedule table (every pass kind,
    merged phases between steps of different s) give the oracle's result."""
    knots = _tables()[name]
    inst = planted_unique_3sat(n, 800 + n)
    E = oracle.energy(n, inst.clauses).astype(np.int64)
    psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
    got, _ = _replay(n, dtype, E, psi, T, N, 0, N, knots, tile_bits=10 if n == 18 else 0)
    ref = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, ref, T, N, knots=knots)
    assert np.max(np.abs(got - ref)) < 1e-12
    # and the table really changes the result
    lin = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, lin, T, N)
    assert np.max(np.abs(lin - ref)) > 1e-4


def test_table_schedule_range_replay():
    n, T, N = 17, 5.0, 9
    knots = [0.0, 0.2, 0.25, 0.3, 1.0]
    inst = planted_unique_3sat(n, 9)
    E = oracle.energy(n, inst.clauses).astype(np.int64)
    psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
    psi, _ = _replay(n, 0, E, psi, T, N, 0, 5, knots)
    psi, _ = _replay(n, 0, E, psi, T, N, 5, N, knots)
    ref = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, ref, T, N, knots=knots)
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_two_knot_table_is_the_linear_schedule_to_the_bit():
    a = qaa.qaa_debug_pass_descs(20, 0, 30, 9.0, 7, 0, 7)
    b = qaa.qaa_debug_pass_descs(20, 0, 30, 9.0, 7, 0, 7, [0.0, 1.0])
    assert len(a) == len(b) > 0
    for x, y in zip(a, b):
        assert bytes(x) == bytes(y)
