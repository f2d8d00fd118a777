"""Write the oracle's results for the n = 20 workload (stored expected values).

Workload: planted unique-solution 3-SAT, n = 20, seeds 0..4, linear
schedule, T = 100, 10^4 second-order steps (dt = 0.01), uniform start.
For each seed the CPU oracle (complex128) is run in full; the file keeps
its observables and the final amplitudes at 512 sampled basis states
(the planted solution first, then indices drawn with SplitMix64 from seed
0xC2).  Only ``oracle`` and the input generator are called.

Usage: python tests/golden/make_golden_c2.py  (about 5 CPU-minutes per seed
on 8 cores).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from qaa_inputs import SplitMix64, planted_unique_3sat  # noqa: E402

N_QUBITS, T, STEPS, SEEDS, SAMPLES = 20, 100.0, 10000, (0, 1, 2, 3, 4), 512
OUT = os.path.join(HERE, "c2_n20_oracle.json")


def sample_indices(n, first):
    rng = SplitMix64(0xC2)
    idx = [int(first)]
    seen = {int(first)}
    while len(idx) < SAMPLES:
        z = rng.below(1 << n)
        if z not in seen:
            seen.add(z)
            idx.append(z)
    return idx


def main():
    records = []
    for seed in SEEDS:
        t0 = time.time()
        inst = planted_unique_3sat(N_QUBITS, seed)
        psi = oracle.init_uniform(N_QUBITS)
        oracle.evolve(N_QUBITS, inst.clauses, psi, T, STEPS)
        obs = oracle.observables(N_QUBITS, inst.clauses, psi)
        idx = sample_indices(N_QUBITS, inst.planted)
        amps = [[float(psi[z].real), float(psi[z].imag)] for z in idx]
        records.append({"seed": seed, "n": N_QUBITS, "m": inst.m, "planted": inst.planted, "T": T,
                        "steps": STEPS, "observables": obs, "sample_z": idx, "sample_amp": amps})
        print("seed %d m=%d P=%.8f <H>=%.8f norm-1=%.2e (%.0f s)" % (
            seed, inst.m, obs["p_success"], obs["energy"], obs["norm"] - 1, time.time() - t0), flush=True)
    with open(OUT, "w") as f:
        json.dump({"workload": "planted 3-SAT n=20, T=100, 10^4 steps, uniform start",
                   "oracle_threads": oracle.num_threads(), "records": records}, f)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
