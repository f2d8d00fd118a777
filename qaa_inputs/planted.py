"""Planted unique-solution 3-SAT generator and workload recipes.

See the package docstring for the recipe.  All randomness comes from one
SplitMix64 stream per instance, so an instance is a pure function of
(n, seed).
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field

import numpy as np

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (Steele, Lea & Flood, OOPSLA 2014)."""

    GOLDEN = 0x9E3779B97F4A7C15

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + self.GOLDEN) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def below(self, k: int) -> int:
        """Uniform integer in [0, k) by rejection (no modulo bias)."""
        if k <= 0:
            raise ValueError("k must be positive")
        limit = (1 << 64) - ((1 << 64) % k)
        while True:
            r = self.next_u64()
            if r < limit:
                return r % k

    def uniform(self, lo: float, hi: float) -> float:
        """Uniform double in [lo, hi) from the top 53 bits."""
        u = (self.next_u64() >> 11) * (1.0 / (1 << 53))
        return lo + (hi - lo) * u


@dataclass
class Instance:
    """A 3-SAT formula: n variables, clauses as signed 1-based literal triples."""

    n: int
    clauses: np.ndarray            # int32 [m, 3]
    planted: int | None = None     # z* (bit i-1 of z is x_i)
    seed: int | None = None
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.clauses.shape[0])

    def literals(self) -> np.ndarray:
        """Flat int32 array of 3m literals (the C-ABI input format)."""
        return np.ascontiguousarray(self.clauses.reshape(-1), dtype=np.int32)


def _clear_violators(words: np.ndarray, n: int, var_idx, neg_bits) -> None:
    """Clear, in the alive bitset, every z that violates the clause.

    The clause over variables (0-based) var_idx with negation flags neg_bits
    is violated iff each variable takes the value that makes its literal
    false: 0 for a positive literal, 1 for a negated one.  z is stored as bit
    (z & 63) of word z >> 6; the bitset is viewed as an array with one axis of
    length 2 per high bit of z so that the violating words are a slice.
    """
    nw = n - 6
    low_sel = [(v, b) for v, b in zip(var_idx, neg_bits) if v < 6]
    high_sel = [(v - 6, b) for v, b in zip(var_idx, neg_bits) if v >= 6]
    # which of the 64 low positions violate the low part of the clause
    lm = 0
    for j in range(64):
        if all(((j >> v) & 1) == b for v, b in low_sel):
            lm |= 1 << j
    keep = np.uint64(~lm & 0xFFFFFFFFFFFFFFFF)
    if nw == 0:
        words &= keep
        return
    view = words.reshape((2,) * nw)   # axis 0 is the highest word bit
    index = [slice(None)] * nw
    for hv, b in high_sel:
        index[nw - 1 - hv] = b
    view[tuple(index)] &= keep


def planted_unique_3sat(n: int, seed: int, max_clauses: int = 100000) -> Instance:
    """Draw a planted 3-SAT instance whose only solution is the planted z*."""
    if n < 3:
        raise ValueError("3-SAT over distinct variables needs n >= 3")
    if n > 34:
        raise ValueError("n > 34 not supported")
    rng = SplitMix64(seed)
    zstar = rng.next_u64() & ((1 << n) - 1)
    clauses: list[tuple[int, int, int]] = []

    # alive set: bitset while large, candidate list once small
    use_bits = n >= 6
    if use_bits:
        words = np.full(1 << (n - 6), np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
        alive_count = 1 << n
        cand = None
    else:
        cand = np.arange(1 << n, dtype=np.int64)
        alive_count = cand.size
    switch_at = 1 << 16

    while alive_count > 1:
        if len(clauses) >= max_clauses:
            raise RuntimeError("planted generator did not reach uniqueness")
        v1 = rng.below(n)
        v2 = rng.below(n)
        while v2 == v1:
            v2 = rng.below(n)
        v3 = rng.below(n)
        while v3 == v1 or v3 == v2:
            v3 = rng.below(n)
        vs = (v1, v2, v3)
        zbits = tuple((zstar >> v) & 1 for v in vs)
        while True:
            pat = rng.below(8)
            neg = tuple((pat >> j) & 1 for j in range(3))
            # literal j is false under z* iff z*_v == neg_j; all three false
            # means z* violates the clause, which is the one pattern rejected
            if neg != zbits:
                break
        clauses.append(tuple((-(v + 1) if b else (v + 1)) for v, b in zip(vs, neg)))
        if cand is None:
            _clear_violators(words, n, vs, neg)
            alive_count = int(np.bitwise_count(words).sum())
            if alive_count <= switch_at:
                nz = np.nonzero(words)[0]
                bits = np.unpackbits(words[nz].view(np.uint8), bitorder="little").reshape(-1, 64)
                w_idx, b_idx = np.nonzero(bits)
                cand = (nz[w_idx].astype(np.int64) << 6) | b_idx.astype(np.int64)
                del words
        else:
            viol = np.ones(cand.size, dtype=bool)
            for v, b in zip(vs, neg):
                viol &= ((cand >> v) & 1) == b
            cand = cand[~viol]
            alive_count = int(cand.size)
    assert alive_count == 1
    if cand is not None:
        assert int(cand[0]) == zstar
    arr = np.asarray(clauses, dtype=np.int32).reshape(-1, 3)
    return Instance(n=n, clauses=arr, planted=int(zstar), seed=seed)


def batch_workload(count: int = 512, seed: int = 2024, n_lo: int = 12, n_hi: int = 22,
                   t_lo: float = 10.0, t_hi: float = 100.0, dt: float = 0.01):
    """The batched workload: ``count`` instances drawn from one master seed.

    For each instance the master stream draws n ~ U{n_lo..n_hi}, T ~ U[t_lo, t_hi)
    and the instance seed.  steps = round(T/dt), so the schedule ends at s = 1
    with dt' = T/steps close to dt.
    Returns a list of (n, T, steps, instance_seed) tuples.
    """
    master = SplitMix64(seed)
    out = []
    for _ in range(count):
        n = n_lo + master.below(n_hi - n_lo + 1)
        T = master.uniform(t_lo, t_hi)
        iseed = master.next_u64()
        steps = max(1, int(round(T / dt)))
        out.append((n, T, steps, iseed))
    return out


def serving_workload(count: int, rate: float, seed: int = 7, n_lo: int = 16, n_hi: int = 31,
                     t_lo: float = 10.0, t_hi: float = 200.0, dt: float = 0.01):
    """Poisson arrivals of solve requests.

    Returns a list of dicts {arrival, n, T, steps, seed}; inter-arrival times
    are exponential with the given rate (requests per second), by inversion of
    a uniform draw.
    """
    master = SplitMix64(seed)
    t = 0.0
    out = []
    for _ in range(count):
        u = master.uniform(0.0, 1.0)
        t += -math.log1p(-u) / rate
        n = n_lo + master.below(n_hi - n_lo + 1)
        T = master.uniform(t_lo, t_hi)
        iseed = master.next_u64()
        out.append({"arrival": t, "n": n, "T": T, "steps": max(1, int(round(T / dt))), "seed": iseed})
    return out


def save_instance(inst: Instance, path: str) -> None:
    with open(path, "w") as f:
        json.dump({"n": inst.n, "seed": inst.seed, "planted": inst.planted,
                   "clauses": inst.clauses.tolist(), "meta": inst.meta}, f)


def load_instance(path: str) -> Instance:
    with open(path) as f:
        d = json.load(f)
    return Instance(n=int(d["n"]), clauses=np.asarray(d["clauses"], dtype=np.int32).reshape(-1, 3),
                    planted=d.get("planted"), seed=d.get("seed"), meta=d.get("meta", {}))
