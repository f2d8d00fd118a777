"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these re-derive the oracle's own formulas: they use the paper's
worked example and its stated uniqueness (Sec. 2.2), counting identities,
closed-form evolutions, dense matrix exponentials built from Kronecker
products (scipy), convergence order, and symmetries.
"""
import itertools

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from qaa_inputs import planted_unique_3sat


def _satisfies_all(clauses, x):
    """Proposition P of Sec. 2.2 on assignment x = (x_1..x_n): AND of ORs."""
    def lit(l):
        v = abs(l)
        return x[v - 1] == 1 if l > 0 else x[v - 1] == 0
    return all(any(lit(l) for l in c) for c in clauses)


# --------------------------------------------------------------------------
# Energy function (Sec. 4.3) and the worked example (Sec. 2.2)
# --------------------------------------------------------------------------

def test_worked_example_has_exactly_one_solution(worked_example):
    """The paper states the example formula has only one solution."""
    n, cl = worked_example["n"], worked_example["clauses"]
    sols = [x for x in itertools.product((0, 1), repeat=n) if _satisfies_all(cl, x)]
    assert len(sols) == 1
    E = oracle.energy(n, cl)
    zeros = np.nonzero(E == 0)[0]
    assert zeros.size == 1
    # x_i is bit (i-1) of z (basis order |q_n ... q_1>)
    z = int(zeros[0])
    assert tuple((z >> (i - 1)) & 1 for i in range(1, n + 1)) == sols[0]
    assert sols[0] == (0, 1, 0, 1, 0, 0) and z == 10


def test_worked_example_stated_solution_is_off_by_x1(worked_example):
    """Reading of the printed solution: it leaves one clause unsatisfied.

    (not x1 or not x2 or not x4) -- the 11th clause -- is false at the
    printed x = (1,1,0,1,0,0); flipping x1 gives the unique solution.
    """
    n, cl = worked_example["n"], worked_example["clauses"]
    x = worked_example["stated_solution_x1_to_x6"]
    unsat = [i for i, c in enumerate(cl) if not _satisfies_all([c], x)]
    assert unsat == [10]
    z = sum(b << i for i, b in enumerate(x))
    assert oracle.energy(n, cl)[z] == 1


def test_worked_example_has_two_duplicate_clauses(worked_example):
    """Duplicated clauses are counted once per copy (the example has two)."""
    cl = [tuple(c) for c in worked_example["clauses"]]
    dups = len(cl) - len(set(cl))
    assert dups == 2
    E = oracle.energy(worked_example["n"], cl)
    # each copy contributes: sum over z of E is m * 2^{n-3} with m = 27
    assert int(E.sum()) == 27 * 2 ** (6 - 3) == 216


@pytest.mark.parametrize("n,seed", [(6, 1), (9, 2), (12, 3), (14, 4)])
def test_energy_sum_identity(n, seed):
    """A clause over 3 distinct variables is false for exactly 2^{n-3} of the
    2^n assignments, so sum_z E(z) = m 2^{n-3} (and <H_P> of the uniform
    state is m/8)."""
    inst = planted_unique_3sat(n, seed)
    E = oracle.energy(n, inst.clauses)
    assert int(E.sum()) == inst.m * 2 ** (n - 3)
    assert E.min() >= 0 and E.max() <= inst.m


@pytest.mark.parametrize("n,seed", [(5, 0), (8, 11), (11, 12), (13, 13)])
def test_planted_solution_is_the_unique_ground_state(n, seed):
    inst = planted_unique_3sat(n, seed)
    E = oracle.energy(n, inst.clauses)
    assert np.count_nonzero(E == 0) == 1
    assert E[inst.planted] == 0


def test_energy_per_clause_indicator():
    """One clause: E is 1 exactly on the 2^{n-3} assignments falsifying all
    three literals (enumerated here by building them bit by bit)."""
    n = 7
    cl = [[3, -5, 7]]
    E = oracle.energy(n, cl)
    falsifying = set()
    for rest in range(1 << (n - 3)):
        # place the 4 free bits into positions {0,1,3,5} and fix x3=0, x5=1, x7=0
        free = [0, 1, 3, 5]
        z = 0
        for j, p in enumerate(free):
            z |= ((rest >> j) & 1) << p
        z |= 1 << 4          # x5 = 1 makes "-5" false
        falsifying.add(z)
    assert set(np.nonzero(E)[0].tolist()) == falsifying
    assert set(np.unique(E).tolist()) == {0, 1}


def _energy_by_proposition(clauses, z):
    """Count the clauses the assignment z falsifies, reading each literal
    from the bits of z directly (Sec. 2.2: x_i is bit i-1 of z)."""
    x = [(z >> i) & 1 for i in range(64)]
    return sum(0 if _satisfies_all([c], x) else 1 for c in clauses)


@pytest.mark.parametrize("n,seed", [(5, 31), (12, 32), (17, 33)])
def test_energy_at_matches_the_full_table(n, seed):
    """energy_at (the sampled checker used at full size) agrees with the
    whole table on random z and on both corners z = 0 and z = 2^n - 1."""
    inst = planted_unique_3sat(n, seed)
    E = oracle.energy(n, inst.clauses)
    rng = np.random.default_rng(seed)
    zs = np.concatenate([[0, (1 << n) - 1, inst.planted], rng.integers(0, 1 << n, 500)]).astype(np.uint64)
    got = oracle.energy_at(n, inst.clauses, zs)
    assert np.array_equal(got, E[zs.astype(np.int64)])


@pytest.mark.parametrize("n", [28, 34])
def test_energy_at_matches_the_proposition_at_large_n(n):
    """Above what a full table allows, energy_at is checked against a count
    written from the clause definition, z by z, including z with the top
    bits set (a truncated index would lose them)."""
    rng = np.random.default_rng(n)
    cl = []
    for _ in range(60):
        v = rng.choice(n, size=3, replace=False) + 1
        v[0] = n if len(cl) % 5 == 0 else v[0]       # some clauses on the top variable
        if len(set(v.tolist())) < 3:
            continue
        cl.append([int(a) * (1 if rng.random() < 0.5 else -1) for a in v])
    zs = np.concatenate([[0, (1 << n) - 1, 1 << (n - 1)], rng.integers(0, 1 << n, 40, dtype=np.int64)])
    got = oracle.energy_at(n, cl, zs.astype(np.uint64))
    want = [_energy_by_proposition(cl, int(z)) for z in zs]
    assert got.tolist() == want


def test_energy_rejects_out_of_range_literal():
    with pytest.raises(ValueError):
        oracle.energy(4, [[1, 2, 5]])


# --------------------------------------------------------------------------
# Evolution pins
# --------------------------------------------------------------------------

def _basis(n, z0):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[z0] = 1.0
    return psi


def test_uniform_state_is_stationary_without_clauses():
    """m = 0: H(s) = (1-s) H_B and the uniform state has H_B eigenvalue 0,
    so it is left exactly unchanged (the s = 0 ground-state check)."""
    n = 5
    psi = oracle.init_uniform(n)
    ref = psi.copy()
    oracle.evolve(n, np.zeros((0, 3), np.int32), psi, T=3.7, N=17)
    assert np.max(np.abs(psi - ref)) < 1e-14


@pytest.mark.parametrize("n,z0", [(4, 0), (5, 0b10110), (6, 0b111111)])
def test_driver_only_closed_form(n, z0):
    """m = 0 from |z0>: each qubit sees exp(-i Theta (1 - sigma^x)/2) with
    Theta = sum_k dt (1 - s_k) = T/2, so psi(z) = a^{n-d} b^d, d the Hamming
    distance to z0, a = (1 + e^{-i Theta})/2, b = (1 - e^{-i Theta})/2."""
    T, N = 2.9, 23
    psi = _basis(n, z0)
    oracle.evolve(n, np.zeros((0, 3), np.int32), psi, T=T, N=N)
    th = T / 2.0
    a = (1 + np.exp(-1j * th)) / 2
    b = (1 - np.exp(-1j * th)) / 2
    d = np.array([bin(z ^ z0).count("1") for z in range(1 << n)])
    expect = a ** (n - d) * b ** d
    assert np.max(np.abs(psi - expect)) < 1e-13


@pytest.mark.parametrize("n,seed,k", [(4, 5, 0), (6, 6, 7), (8, 7, 19)])
def test_one_step_matches_dense_expm(n, seed, k):
    """Step k equals expm(-i dt/2 s H_P) expm(-i dt (1-s) H_B) expm(-i dt/2 s H_P)
    with H_B assembled from Kronecker products."""
    inst = planted_unique_3sat(n, seed)
    T, N = 10.0, 20
    rng = np.random.default_rng(seed)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    U = oracle.dense_strang_step(n, oracle.energy(n, inst.clauses), T, N, k)
    expect = U @ psi
    got = psi.copy()
    oracle.evolve(n, inst.clauses, got, T=T, N=N, k0=k, k1=k + 1)
    assert np.max(np.abs(got - expect)) < 1e-13


def test_dense_h_b_spectrum():
    """H_B = sum (1 - sigma^x)/2 has eigenvalue j with multiplicity C(n, j)."""
    n = 5
    w = np.linalg.eigvalsh(oracle.dense_h_b(n))
    vals, counts = np.unique(np.round(w).astype(int), return_counts=True)
    from math import comb
    assert vals.tolist() == list(range(n + 1))
    assert counts.tolist() == [comb(n, j) for j in range(n + 1)]
    assert np.max(np.abs(w - np.round(w))) < 1e-12


def test_worked_example_full_evolution_matches_dense_product(worked_example):
    n, cl = worked_example["n"], worked_example["clauses"]
    T, N = 10.0, 60
    E = oracle.energy(n, cl)
    psi = oracle.init_uniform(n)
    expect = psi.copy()
    for k in range(N):
        expect = oracle.dense_strang_step(n, E, T, N, k) @ expect
    oracle.evolve(n, cl, psi, T=T, N=N)
    assert np.max(np.abs(psi - expect)) < 1e-12


def _exact_reference(n, E, T, nsub):
    """Time-ordered propagator from nsub exponential-midpoint substeps."""
    hb = oracle.dense_h_b(n)
    hp = np.diag(E.astype(float))
    psi = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    h = T / nsub
    for j in range(nsub):
        s = (j + 0.5) / nsub
        psi = expm(-1j * h * ((1 - s) * hb + s * hp)) @ psi
    return psi


def test_second_order_convergence():
    """Global error of the Strang steps falls as dt^2: halving dt divides it by ~4."""
    n = 5
    inst = planted_unique_3sat(n, 21)
    E = oracle.energy(n, inst.clauses)
    T = 4.0
    ref = _exact_reference(n, E, T, 4096)
    errs = []
    for N in (8, 16, 32):
        psi = oracle.init_uniform(n)
        oracle.evolve(n, inst.clauses, psi, T=T, N=N)
        errs.append(np.linalg.norm(psi - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, (errs, r1, r2)


def test_norm_is_conserved():
    n = 10
    inst = planted_unique_3sat(n, 3)
    psi = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, psi, T=10.0, N=1000)
    obs = oracle.observables(n, inst.clauses, psi)
    assert abs(obs["norm"] - 1.0) < 1e-12


def test_zero_steps_gives_uniform_observables():
    """No evolution: P_success = degeneracy / 2^n and <H_P> = m/8 exactly."""
    n = 9
    inst = planted_unique_3sat(n, 4)
    psi = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, psi, T=5.0, N=0)
    obs = oracle.observables(n, inst.clauses, psi)
    assert obs["degeneracy"] == 1 and obs["e_min"] == 0
    assert abs(obs["p_success"] - 2.0 ** -n) < 1e-15
    assert abs(obs["energy"] - inst.m / 8.0) < 1e-12


def _random_state(n, seed):
    rng = np.random.default_rng(seed)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return psi / np.linalg.norm(psi)


def test_success_probability_without_clauses_is_the_norm():
    """m = 0: every z has E = 0, so the ground manifold is all 2^n states
    and P_success is the whole norm (Sec. 2.1, degeneracy 2^n)."""
    n = 6
    psi = _random_state(n, 1)
    obs = oracle.observables(n, np.zeros((0, 3), np.int32), psi)
    assert obs["e_min"] == 0 and obs["degeneracy"] == 1 << n
    assert abs(obs["p_success"] - 1.0) < 1e-13 and abs(obs["energy"]) == 0.0


def test_success_probability_sums_every_solution():
    """A formula with several solutions: P_success is the weight on all of
    them (found here by brute force over the assignments), not on one."""
    n = 7
    # x1 = 1 is forced by the four clauses over (1, 2, 3) without the pattern
    # x1 = 1 falsifies; the clauses over (4, 5, 6) and (5, 6, 7) prune the rest
    cl = [[1, 2, 3], [1, -2, 3], [1, 2, -3], [1, -2, -3],
          [4, 5, 6], [-4, 5, 6], [4, -5, 6], [4, 5, -6], [-4, -5, 6], [-4, 5, -6], [4, -5, -6],
          [5, 6, 7], [-5, 6, 7], [5, -6, 7], [5, 6, -7], [-5, -6, 7], [5, -6, -7]]
    sols = [z for z in range(1 << n) if _satisfies_all(cl, [(z >> i) & 1 for i in range(n)])]
    assert 2 <= len(sols) <= 8
    psi = _random_state(n, 2)
    obs = oracle.observables(n, cl, psi)
    assert obs["e_min"] == 0 and obs["degeneracy"] == len(sols)
    want = sum(abs(psi[z]) ** 2 for z in sols)
    assert abs(obs["p_success"] - want) < 1e-14
    # the largest single weight is not the answer
    assert abs(obs["p_success"] - max(abs(psi[z]) ** 2 for z in sols)) > 1e-3


def test_success_probability_on_an_unsatisfiable_formula():
    """All eight sign patterns over (x1, x2, x3): every assignment falsifies
    exactly one of them, so E_min = 1; one more clause over (x4, x5, x6)
    lifts 1/8 of the states to E = 2.  The ground manifold is the other 7/8."""
    n = 6
    cl = [[a * 1, b * 2, c * 3] for a in (1, -1) for b in (1, -1) for c in (1, -1)] + [[4, -5, 6]]
    psi = _random_state(n, 3)
    obs = oracle.observables(n, cl, psi)
    assert obs["e_min"] == 1 and obs["degeneracy"] == (1 << n) - (1 << (n - 3))
    lifted = [z for z in range(1 << n) if ((z >> 3) & 1) == 0 and ((z >> 4) & 1) == 1 and ((z >> 5) & 1) == 0]
    assert len(lifted) == 1 << (n - 3)
    want = 1.0 - sum(abs(psi[z]) ** 2 for z in lifted)
    assert abs(obs["p_success"] - want) < 1e-13
    assert abs(obs["energy"] - (1.0 + (1.0 - want))) < 1e-13


def test_step_ranges_compose():
    n = 7
    inst = planted_unique_3sat(n, 8)
    a = oracle.init_uniform(n)
    b = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, a, T=6.0, N=40)
    oracle.evolve(n, inst.clauses, b, T=6.0, N=40, k0=0, k1=13)
    oracle.evolve(n, inst.clauses, b, T=6.0, N=40, k0=13, k1=40)
    assert np.array_equal(a, b)


def test_gauge_flip_of_one_variable():
    """Negating variable v in every clause and relabelling z -> z xor 2^{v-1}
    is a symmetry: H_B is invariant under X_v and the start is uniform."""
    n, v = 8, 3
    inst = planted_unique_3sat(n, 9)
    flipped = inst.clauses.copy()
    mask = np.abs(flipped) == v
    flipped[mask] = -flipped[mask]
    a = oracle.init_uniform(n)
    b = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, a, T=7.0, N=70)
    oracle.evolve(n, flipped, b, T=7.0, N=70)
    z = np.arange(1 << n)
    assert np.max(np.abs(b - a[z ^ (1 << (v - 1))])) < 1e-13
    oa = oracle.observables(n, inst.clauses, a)
    ob = oracle.observables(n, flipped, b)
    assert abs(oa["p_success"] - ob["p_success"]) < 1e-13
    assert abs(oa["energy"] - ob["energy"]) < 1e-12


def test_variable_relabelling():
    """Permuting variable labels permutes the bits of z."""
    n = 7
    inst = planted_unique_3sat(n, 10)
    perm = [3, 0, 6, 1, 5, 2, 4]            # old variable i (0-based) -> new perm[i]
    relab = np.sign(inst.clauses) * (np.array(perm)[np.abs(inst.clauses) - 1] + 1)
    a = oracle.init_uniform(n)
    b = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, a, T=5.0, N=50)
    oracle.evolve(n, relab, b, T=5.0, N=50)
    z = np.arange(1 << n)
    znew = np.zeros_like(z)
    for i, p in enumerate(perm):
        znew |= ((z >> i) & 1) << p
    assert np.max(np.abs(b[znew] - a)) < 1e-13


def test_slow_sweep_reaches_the_solution(worked_example):
    """Slow enough evolution ends near the ground state of H_P (Sec. 2.1)."""
    n, cl = worked_example["n"], worked_example["clauses"]
    psi = oracle.init_uniform(n)
    oracle.evolve(n, cl, psi, T=100.0, N=10000)
    obs = oracle.observables(n, cl, psi)
    fast = oracle.init_uniform(n)
    oracle.evolve(n, cl, fast, T=1.0, N=100)
    assert obs["p_success"] > 0.9
    assert oracle.observables(n, cl, fast)["p_success"] < obs["p_success"]


# --------------------------------------------------------------------------
# Schedule tables: s(u) piecewise linear through equally spaced knots
# (u = t/T).  The paper's schedule is s = u (Sec. 2.1, eq. 1); the table
# is checked against numpy's own piecewise-linear interpolation, dense
# exponentials, exact decompositions and closed forms.
# --------------------------------------------------------------------------

def _dense_step_at(n, E, dt, s):
    """expm(-i dt/2 s H_P) expm(-i dt (1-s) H_B) expm(-i dt/2 s H_P)."""
    hp = np.diag(E.astype(np.float64))
    half = expm(-1j * (dt / 2.0) * s * hp)
    return half @ expm(-1j * dt * (1.0 - s) * oracle.dense_h_b(n)) @ half


def test_two_knot_table_is_the_linear_schedule():
    n = 7
    inst = planted_unique_3sat(n, 31)
    a = oracle.init_uniform(n)
    b = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, a, T=6.0, N=40)
    oracle.evolve(n, inst.clauses, b, T=6.0, N=40, knots=[0.0, 1.0])
    assert np.array_equal(a, b)


@pytest.mark.parametrize("count", [3, 5, 33, 256])
def test_knots_on_the_line_give_the_linear_schedule(count):
    """Interpolating knots that lie on s = u reproduces s = u."""
    n = 7
    inst = planted_unique_3sat(n, 32)
    a = oracle.init_uniform(n)
    b = oracle.init_uniform(n)
    oracle.evolve(n, inst.clauses, a, T=6.0, N=45)
    oracle.evolve(n, inst.clauses, b, T=6.0, N=45, knots=np.linspace(0.0, 1.0, count))
    assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("knots", [[0.0, 0.9, 0.2, 1.0], [0.3, 0.3], list(np.linspace(0, 1, 11) ** 2)])
def test_table_steps_match_dense_expm_with_numpy_interp(knots):
    """Every step equals the dense Strang product at s = numpy.interp(u_k)."""
    n, N, T = 6, 13, 8.0
    inst = planted_unique_3sat(n, 33)
    E = oracle.energy(n, inst.clauses)
    grid = np.linspace(0.0, 1.0, len(knots))
    rng = np.random.default_rng(34)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    for k in range(N):
        s = float(np.interp((k + 0.5) / N, grid, knots))
        expect = _dense_step_at(n, E, T / N, s) @ psi
        got = psi.copy()
        oracle.evolve(n, inst.clauses, got, T=T, N=N, k0=k, k1=k + 1, knots=knots)
        assert np.max(np.abs(got - expect)) < 1e-13, k
        psi = expect


def test_ramp_table_decomposes_into_driver_linear_sweep_and_phase():
    """Knots {0, 0, 1, 1} with N = 3q: the first third has s = 0 (pure
    driver, exp(-i T/3 H_B) exactly), the middle third is the linear sweep
    over time T/3 in q steps, the last third has s = 1 (pure phase
    exp(-i T/3 H_P) exactly).  From a basis state the driver part is the
    closed form a^{n-d} b^d."""
    n, q, T, z0 = 6, 11, 9.0, 0b101101
    inst = planted_unique_3sat(n, 35)
    E = oracle.energy(n, inst.clauses)
    th = T / 3.0
    a = (1 + np.exp(-1j * th)) / 2
    b = (1 - np.exp(-1j * th)) / 2
    d = np.array([bin(z ^ z0).count("1") for z in range(1 << n)])
    expect = a ** (n - d) * b ** d
    oracle.evolve(n, inst.clauses, expect, T=T / 3.0, N=q)
    expect = expect * np.exp(-1j * th * E)
    got = _basis(n, z0)
    oracle.evolve(n, inst.clauses, got, T=T, N=3 * q, knots=[0.0, 0.0, 1.0, 1.0])
    assert np.max(np.abs(got - expect)) < 1e-13


@pytest.mark.parametrize("knots", [[0.0, 0.8, 1.0], [0.1, 0.6, 0.2, 0.9, 1.0]])
def test_table_driver_only_closed_form(knots):
    """m = 0 from |z0>: the driver angles add up to Theta = sum_k dt (1 - s_k).
    With N a multiple of the segment count, the midpoints of each segment are
    placed symmetrically in it, so the sum of s over them is exact:
    Theta = T (1 - mean over segments of (v_j + v_{j+1})/2)."""
    n, z0, T = 5, 0b01101, 3.3
    segs = len(knots) - 1
    N = 7 * segs
    v = np.asarray(knots)
    th = T * (1.0 - np.mean((v[:-1] + v[1:]) / 2.0))
    a = (1 + np.exp(-1j * th)) / 2
    b = (1 - np.exp(-1j * th)) / 2
    d = np.array([bin(z ^ z0).count("1") for z in range(1 << n)])
    psi = _basis(n, z0)
    oracle.evolve(n, np.zeros((0, 3), np.int32), psi, T=T, N=N, knots=knots)
    assert np.max(np.abs(psi - a ** (n - d) * b ** d)) < 1e-13


def test_table_second_order_convergence():
    """With steps that never straddle a knot, a table schedule keeps the
    dt^2 global error (reference: fine exponential-midpoint substeps of
    H(s(t)) with s from numpy.interp)."""
    n = 5
    inst = planted_unique_3sat(n, 36)
    E = oracle.energy(n, inst.clauses)
    knots = [0.0, 0.5, 0.6, 0.7, 1.0]
    grid = np.linspace(0.0, 1.0, len(knots))
    T, nsub = 4.0, 4096
    hb, hp = oracle.dense_h_b(n), np.diag(E.astype(float))
    ref = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    for j in range(nsub):
        s = float(np.interp((j + 0.5) / nsub, grid, knots))
        ref = expm(-1j * (T / nsub) * ((1 - s) * hb + s * hp)) @ ref
    errs = []
    for N in (8, 16, 32):
        psi = oracle.init_uniform(n)
        oracle.evolve(n, inst.clauses, psi, T=T, N=N, knots=knots)
        errs.append(np.linalg.norm(psi - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, (errs, r1, r2)


@pytest.mark.parametrize("knots", [[0.5], [0.0, 1.2], [0.0, float("nan"), 1.0]])
def test_oracle_rejects_bad_tables(knots):
    psi = oracle.init_uniform(4)
    with pytest.raises(ValueError):
        oracle.evolve(4, [[1, 2, 3]], psi, T=1.0, N=3, knots=knots)


# --------------------------------------------------------------------------
# Spectrum of H(s) (eq. 1): closed forms at the ends, the two independent
# constructions (dense Kronecker products / matrix-free flips) against each
# other, variational bounds and first-order perturbation theory.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [6, 11])
def test_levels_at_s0_are_the_driver_spectrum(n):
    """H(0) = H_B has levels 0, 1, 2, ... (Hamming weight of the X basis)."""
    inst = planted_unique_3sat(n, 41)
    assert np.allclose(oracle.levels(n, inst.clauses, 0.0, 3), [0.0, 1.0, 2.0], atol=1e-9)


@pytest.mark.parametrize("n", [7, 11])
def test_levels_at_s1_are_the_sorted_energies(n):
    inst = planted_unique_3sat(n, 42)
    E = np.unique(oracle.energy(n, inst.clauses))
    assert np.allclose(oracle.levels(n, inst.clauses, 1.0, 3), E[:3], atol=1e-9)


@pytest.mark.parametrize("n,s", [(6, 0.3), (10, 0.55)])
def test_levels_without_clauses_scale_with_one_minus_s(n, s):
    assert np.allclose(oracle.levels(n, np.zeros((0, 3), np.int32), s, 3), (1 - s) * np.arange(3), atol=1e-9)


def test_dense_and_matrix_free_levels_agree():
    """The dense construction (n <= 11) against ARPACK on the matrix-free
    flips written out again here, at n = 11."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    n = 11
    inst = planted_unique_3sat(n, 43)
    for s in (0.2, 0.5, 0.8):
        dense = oracle.levels(n, inst.clauses, s, 3)
        E = oracle.energy(n, inst.clauses).astype(float)
        diag = (1 - s) * n / 2 + s * E
        op = LinearOperator((1 << n, 1 << n), dtype=float,
                            matvec=lambda x: diag * x.ravel() - 0.5 * (1 - s) * sum(
                                oracle._flip(x.ravel(), q) for q in range(n)))
        w = np.sort(eigsh(op, k=3, which="SA", tol=1e-13, return_eigenvectors=False))
        assert np.allclose(dense, w, atol=1e-9)


@pytest.mark.parametrize("n", [10, 13])
def test_ground_level_bounds(n):
    """0 < E0(s) < <uniform|H(s)|uniform> = s m/8 for 0 < s < 1: both terms are
    positive semidefinite with different kernels (uniform state, planted z*),
    and the uniform state is a trial vector."""
    inst = planted_unique_3sat(n, 44)
    for s in (0.1, 0.4, 0.7, 0.95):
        e0 = oracle.levels(n, inst.clauses, s, 1)[0]
        assert 0.0 < e0 < s * inst.m / 8.0


def test_ground_level_first_order_at_both_ends():
    """E0(h) = h m/8 + O(h^2) (perturbing the uniform ground state of H_B by
    H_P - H_B) and E0(1-h) = h n/2 + O(h^2) (perturbing |z*> by H_B - H_P)."""
    n, h = 9, 1e-5
    inst = planted_unique_3sat(n, 45)
    assert abs(oracle.levels(n, inst.clauses, h, 1)[0] / h - inst.m / 8.0) < 1e-2 * inst.m / 8.0
    assert abs(oracle.levels(n, inst.clauses, 1 - h, 1)[0] / h - n / 2.0) < 1e-2 * n / 2.0


@pytest.mark.parametrize("s", [0.3, 0.6])
def test_matrix_free_levels_continue_the_dense_ones(s):
    """n = 12 (ARPACK path) against dense eigvalsh of the same matrix."""
    n = 12
    inst = planted_unique_3sat(n, 46)
    E = oracle.energy(n, inst.clauses).astype(float)
    w = np.linalg.eigvalsh((1 - s) * oracle.dense_h_b(n) + s * np.diag(E))
    assert np.allclose(oracle.levels(n, inst.clauses, s, 3), w[:3], atol=1e-9)


def test_matrix_free_levels_refuse_degenerate_cases():
    inst = planted_unique_3sat(12, 47)
    for s in (0.0, 1.0):
        with pytest.raises(ValueError):
            oracle.levels(12, inst.clauses, s, 2)
    with pytest.raises(ValueError):
        oracle.levels(12, np.zeros((0, 3), np.int32), 0.5, 2)
