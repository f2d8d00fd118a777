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


def _swz_c64(l):
    return l ^ (((l >> 5) ^ (l >> 10)) & 31)


def _replay(n, dtype, E, psi, T, N, k0, k1):
    plan = qaa.qaa_plan_info(n, dtype)
    TB = plan["tile_bits"]
    RB = 5 if dtype == qaa.QAA_C64 else 4
    WB = TB - RB
    R, WG = 1 << RB, 1 << WB
    descs = qaa.qaa_debug_pass_descs(n, dtype, int(E.max()), T, N, k0, k1)
    tid = np.arange(WG, dtype=np.int64)
    reg = np.arange(R, dtype=np.int64)
    for d in descs:
        tile_pos = list(d.tile_pos[:TB])
        rest_pos = list(d.rest_pos[:d.n_rest])
        assert sorted(tile_pos + rest_pos) == list(range(n))
        blocks = np.arange(1 << d.n_rest, dtype=np.int64)
        base = _pdep(blocks, rest_pos)                                  # [B]
        # load layout: l = tid + i * WG
        l_load = (tid[:, None] + reg[None, :] * WG)                     # [WG, R]
        off = _pdep(l_load, tile_pos)                                   # [WG, R]
        g = base[:, None, None] | off[None]                             # [B, WG, R]
        flat = g.reshape(-1)
        assert np.array_equal(np.sort(flat), np.arange(1 << n))
        tiles = np.empty((blocks.size, 1 << TB), np.complex128)
        tiles[:, l_load.reshape(-1)] = psi[g.reshape(blocks.size, -1)]
        etile = np.empty((blocks.size, 1 << TB), np.int64)
        etile[:, l_load.reshape(-1)] = E[g.reshape(blocks.size, -1)]
        assert np.array_equal(np.sort(_swz_c64(np.arange(1 << TB))), np.arange(1 << TB))
        lut = np.exp(-1j * (d.phi * np.arange(int(E.max()) + 1) + d.gphase))
        for r in range(d.n_res):
            gb = list(d.gbits[r][:RB])
            tp = list(d.tpos[r][:WB])
            assert sorted(gb + tp) == list(range(TB))
            lt = _pdep(tid, tp)
            lj = _pdep(reg, gb)
            l = lt[:, None] | lj[None, :]                               # [WG, R]
            assert np.array_equal(np.sort(l.reshape(-1)), np.arange(1 << TB))
            v = tiles[:, l]                                             # [B, WG, R]

            def rot(v, mask, cm1, s):
                for b in range(RB):
                    if (mask >> b) & 1:
                        lo = [j for j in range(R) if not (j >> b) & 1]
                        hi = [j | (1 << b) for j in lo]
                        x0, x1 = v[..., lo].copy(), v[..., hi].copy()
                        c = 1.0 + cm1
                        v[..., lo] = c * x0 + 1j * s * x1
                        v[..., hi] = c * x1 + 1j * s * x0
                return v

            v = rot(v, d.maskA[r], d.cm1A, d.sA)
            if r == d.phase_at:
                v = v * lut[etile[:, l]]
            v = rot(v, d.maskB[r], d.cm1B, d.sB)
            tiles[:, l] = v
        psi[g.reshape(blocks.size, -1)] = tiles[:, l_load.reshape(-1)]
    return psi, descs


@pytest.mark.parametrize("n,dtype,T,N", [(14, 0, 5.0, 4), (16, 0, 6.0, 3), (21, 0, 5.0, 2), (22, 0, 5.0, 2),
                                         (13, 1, 5.0, 4), (17, 1, 5.0, 3)])
def test_pass_plan_replays_the_oracle(n, dtype, T, N):
    inst = planted_unique_3sat(n, 500 + n)
    E = oracle.energy(n, inst.clauses).astype(np.int64)
    psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
    got, descs = _replay(n, dtype, E, psi, T, N, 0, N)
    sets = qaa.qaa_plan_info(n, dtype)["sets"]
    assert len(descs) == (sets - 1) * N + 1
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
