"""Write the oracle's results for states of the batched workload (stored
expected values).

Workload: the first 12 draws of the batched benchmark's mix (master seed
2024: n ~ U{12..22}, T ~ U[10, 100), steps = round(T/0.01)), each a planted
unique-solution 3-SAT instance evolved from the uniform start under the
linear schedule.  They span every plan kind: whole state in one workgroup
(n = 13), two qubit sets (n = 14..21) and three (n = 22), and up to 9926
steps.  For each state the CPU oracle (complex128) runs in full; the file
keeps its observables, the final amplitude at the planted solution, and the
final amplitudes at 511 further basis states drawn uniformly with SplitMix64
(seed 0xC4 + index) -- enough to estimate the whole-state L2 error.  Only
``oracle`` and the input generator are called.

Usage: python tests/golden/make_golden_c4.py  (about 10 CPU-minutes on 8
cores).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from qaa_inputs import SplitMix64, batch_workload, planted_unique_3sat  # noqa: E402

COUNT, MASTER_SEED, SAMPLES = 12, 2024, 512
OUT = os.path.join(HERE, "c4_mix_oracle.json")


def sample_indices(n, planted, stream_seed):
    """The planted solution, then SAMPLES - 1 distinct other basis states
    drawn uniformly (so they estimate the sum over the remaining 2^n - 1)."""
    rng = SplitMix64(stream_seed)
    idx = [int(planted)]
    seen = {int(planted)}
    want = min(SAMPLES, 1 << n)
    while len(idx) < want:
        z = rng.below(1 << n)
        if z not in seen:
            seen.add(z)
            idx.append(z)
    return idx


def main():
    records = []
    for i, (n, T, steps, iseed) in enumerate(batch_workload(512, MASTER_SEED)[:COUNT]):
        t0 = time.time()
        inst = planted_unique_3sat(n, iseed)
        psi = oracle.init_uniform(n)
        oracle.evolve(n, inst.clauses, psi, T, steps)
        obs = oracle.observables(n, inst.clauses, psi)
        idx = sample_indices(n, inst.planted, 0xC4 + i)
        amps = [[float(psi[z].real), float(psi[z].imag)] for z in idx]
        records.append({"index": i, "n": n, "T": T, "steps": steps, "seed": iseed, "m": inst.m,
                        "planted": inst.planted, "observables": obs, "sample_z": idx, "sample_amp": amps})
        print("state %d n=%d T=%.2f steps=%d m=%d P=%.8f (%.0f s)" % (i, n, T, steps, inst.m, obs["p_success"],
                                                                     time.time() - t0), flush=True)
    with open(OUT, "w") as f:
        json.dump({"workload": "first %d draws of the batched mix (master seed %d), linear schedule, uniform "
                               "start" % (COUNT, MASTER_SEED),
                   "oracle_threads": oracle.num_threads(), "records": records}, f)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
