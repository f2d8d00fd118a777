#!/usr/bin/env python
"""Benchmark of the adiabatic 3-SAT evolution on one MI355X.

Workload (the headline configuration): planted unique-solution 3-SAT with
n = 28 variables (seed 0), linear schedule s = t/T with T = 50 and 5000
second-order steps (dt = 0.01), complex64 state (2 GiB) with a uint8 energy
table (256 MiB), uniform start.

One benchmark "step" is one second-order step of the whole path.  The
timed region is exactly K steps (steps 0..K-1 of the 5000-step schedule,
with the closing half phase) on a state and energy table already resident
in HBM; HIP events on the launch stream bracket them.  The one-off parts of
the job -- energy table from the clause list, uniform initial state, FP64
observables -- are timed on their own right before and after, and charged
to the job's N steps:

    ms_per_step = steps_region / K + (table + init + observables) / N
    value       = 2^n / ms_per_step          (amplitude-steps per second)

which is the same costing cpu_baseline uses, so gpu_over_cpu compares like
with like.  `region` reports the raw K-step figures (steps_region / K).

Also reported on the same JSON line:
  roofline     -- HBM roofline of the dominant kernel (the fused pass):
                  algorithmic bytes per launch / event-measured launch time.
  cpu_baseline -- the CPU oracle timed on a bounded sample of the same job.
  batch        -- 512 planted instances (n ~ U{12..22}, T ~ U[10,100)) in one
                  qaa_evolve_batch call: solves/s and amplitude-steps/s, against
                  one qaa_evolve call per instance on a sample.
  serving      -- Poisson request streams through the request server: p50/p99
                  latency and solves/s per arrival rate.
  spectrum     -- the two lowest levels of H(s) on a grid of s for one
                  planted instance (qaa_spectrum): minimum gap and time.
(--no-extras skips the last three; they run after the timed region.
--schedule-knots K runs the headline job under a K-knot schedule table.)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2^n amplitude-steps/s at n=28 (% HBM roofline); batched solves/s; p50/p99"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published peak

# HBM traffic of the pass kernel measured with rocprofv3 --pmc (FETCH_SIZE and
# WRITE_SIZE runs, scaled by the same counters' reading for a plain copy of
# known size), per launch of the timed region's mix.  Valid only for the
# sources it was taken on (the pass kernels, their shared device helpers,
# the descriptor layout and the planner that decides the passes' tiles,
# grids and order).
PASS_KERNEL_SOURCES = ("paper_1103_1399_amd/csrc/pass_kernels.hip", "paper_1103_1399_amd/csrc/kernel_common.h",
                       "paper_1103_1399_amd/csrc/qaa_internal.h", "paper_1103_1399_amd/csrc/qaa_api.hip")
MEASURED_TRAFFIC = {
    "kernel_source_sha256": "81d5340307927aa18a92062671b2ba3a10ff7c97386d95326dfdce0d42849321",
    "bytes_per_launch": 4.4343e+09,
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for rel in PASS_KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def schedule_table(count):
    """None for the linear schedule, else `count` knots of
    s(u) = u + 0.9 sin(2 pi u) / (2 pi) (monotone, slowest at u = 1/2)."""
    if count == 0:
        return None
    u = [j / (count - 1) for j in range(count)]
    return [min(1.0, max(0.0, x + 0.9 * math.sin(2 * math.pi * x) / (2 * math.pi))) for x in u]


def _host_cpus():
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = None
    return os.cpu_count(), aff


def _oracle_job_rate(oracle, n, clauses, T, N, sample_steps, knots):
    """Energy table once, then the first `sample_steps` steps; returns
    (table s, s/step, amplitude-steps/s with the table charged to N steps)."""
    t0 = time.perf_counter()
    oracle.energy(n, clauses)
    t_e = time.perf_counter() - t0
    psi = oracle.init_uniform(n)
    t0 = time.perf_counter()
    oracle.evolve(n, clauses, psi, T, N, 0, sample_steps, knots=knots)    # recomputes E inside
    t_ev = time.perf_counter() - t0
    t_step = max(1e-9, (t_ev - t_e) / sample_steps)
    return t_e, t_step, (2.0 ** n) / (t_step + t_e / N)


def cpu_baseline(inst, n, T, N, sample_steps, knots=None, single_n=22):
    """Oracle on the host cores: energy table once, then `sample_steps` steps;
    the per-step rate is extrapolated to the full N-step job (table charged
    to N steps, as for the GPU figure).  Also the same costing on one thread,
    on the n = single_n instance of the same generator (one step), so the
    1-thread sample stays within seconds."""
    import oracle
    from qaa_inputs import planted_unique_3sat
    oracle.build()
    threads = oracle.num_threads()
    t_e, t_step, rate = _oracle_job_rate(oracle, n, inst.clauses, T, N, sample_steps, knots)
    one = None
    if single_n:
        small = planted_unique_3sat(single_n, 0)
        oracle.set_num_threads(1)
        try:
            e1, s1, r1 = _oracle_job_rate(oracle, single_n, small.clauses, T, N, 1, knots)
        finally:
            oracle.set_num_threads(threads)
        one = {"n": single_n, "m": small.m, "threads": 1, "table_s": e1, "s_per_step": s1,
               "value": r1, "unit": "amplitude-steps/s"}
    host, aff = _host_cpus()
    return {
        "value": rate,
        "unit": "amplitude-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "n=%d seed 0: energy table %.1f s, then %d of the %d steps (%.2f s/step) on %d threads; "
                  "rate = 2^n / (s/step + table/%d), complex128 C oracle with OpenMP"
                  % (n, t_e, sample_steps, N, t_step, threads, N),
        "host_cpus": host,
        "affinity_cpus": aff,
        "table_s": t_e,
        "s_per_step": t_step,
        "single_thread": one,
    }


def device_copy_gbs(torch, nbytes, reps=8):
    """Read + write bandwidth of a plain device-to-device copy of nbytes
    (torch copy_ of two fresh buffers), HIP events over `reps` copies: the
    practical ceiling an HBM-bound pass is compared with."""
    src = torch.ones(nbytes // 8, dtype=torch.complex64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    secs = a.elapsed_time(b) * 1e-3
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes * reps / secs / 1e9


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[i]


def run_batch(qaa, torch, count, seed, loop_sample):
    """Batched solves: `count` instances (n ~ U{12..22}, T ~ U[10, 100),
    steps = round(T/0.01)) evolved together by qaa_evolve_batch; compared
    with one qaa_evolve call per instance on the first `loop_sample` of them."""
    from qaa_inputs import batch_workload, planted_unique_3sat
    wl = batch_workload(count, seed)
    dev = torch.device("cuda:0")
    insts, states, keep = [], [], []
    for n, T, steps, iseed in wl:
        inst = qaa.Instance(n, planted_unique_3sat(n, iseed).literals())
        table = inst.energy_table()
        amp = torch.empty(1 << n, dtype=torch.complex64, device=dev)
        st = qaa.make_state(inst.handle, amp, table, qaa.QAA_E_U8)
        insts.append(inst)
        states.append(st)
        keep.append((amp, table))
    Ts = [w[1] for w in wl]
    Ns = [w[2] for w in wl]
    amp_steps = sum((1 << w[0]) * w[2] for w in wl)
    for st in states:
        qaa.qaa_state_init_uniform(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qaa.qaa_evolve_batch(states, Ts, Ns)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    p_batch = [qaa.qaa_observables(st)["p_success"] for st in states[:loop_sample]]
    # per-instance launches on the same states, same accuracy (same kernels)
    for st in states[:loop_sample]:
        qaa.qaa_state_init_uniform(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st, T, N in zip(states[:loop_sample], Ts, Ns):
        qaa.qaa_evolve(st, T, N)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    p_loop = [qaa.qaa_observables(st)["p_success"] for st in states[:loop_sample]]
    loop_amp_steps = sum((1 << w[0]) * w[2] for w in wl[:loop_sample])
    for inst in insts:
        inst.close()
    plans = {}
    for n in sorted({w[0] for w in wl}):
        info = qaa.qaa_plan_info(n)
        plans[str(n)] = {"sets": info["sets"], "tile_bits": info["tile_bits"], **qaa.qaa_plan_get(n)}
    return {
        "workload": "%d planted 3-SAT instances, n ~ U{12..22}, T ~ U[10,100), dt ~ 0.01 (seed %d)" % (count, seed),
        "plan_per_n": plans,
        "solves_per_s": count / t_batch,
        "amp_steps_per_s": amp_steps / t_batch,
        "seconds": t_batch,
        "amp_steps": amp_steps,
        "loop": {"instances": loop_sample, "amp_steps_per_s": loop_amp_steps / t_loop, "seconds": t_loop,
                 "max_abs_dp_vs_batch": max(abs(a - b) for a, b in zip(p_batch, p_loop)) if loop_sample else None},
    }


def run_spectrum(qaa, torch, n, points, iters, seed):
    """Lowest two levels of H(s) on an even grid of `points` values of s in
    [0, 1] for one planted instance (qaa_spectrum, Lanczos on the device):
    the minimum gap along the path and the time it takes."""
    import numpy as np
    from qaa_inputs import planted_unique_3sat
    inst_in = planted_unique_3sat(n, seed)
    inst = qaa.Instance(n, inst_in.literals())
    table = inst.energy_table()
    v0 = torch.from_numpy(np.random.default_rng(seed).standard_normal(1 << n)).cuda()
    svals = [i / (points - 1) for i in range(points)]
    inst.spectrum(table, svals[:1], v0, iters=min(iters, 20), k=2)     # warm-up (allocator, code objects)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, bd = inst.spectrum(table, svals, v0, iters=iters, k=2, bounds=True)
    secs = time.perf_counter() - t0
    gaps = ev[:, 1] - ev[:, 0]
    i = int(np.argmin(gaps))
    inst.close()
    return {"n": n, "m": inst_in.m, "seed": seed, "points": points, "lanczos_steps": iters, "seconds": secs,
            "ms_per_point": secs / points * 1e3, "lanczos_steps_per_s": points * iters / secs,
            "min_gap": float(gaps[i]), "s_at_min_gap": svals[i], "e0_at_min_gap": float(ev[i, 0]),
            "max_residual_bound": float(np.nanmax(bd))}


def run_serving(qaa, count, rates, n_lo, n_hi, t_lo, t_hi, slots, budget):
    """Open-loop serving: Poisson arrivals at each rate (requests/s), each a
    planted 3-SAT solve; reports latency percentiles and completed solves/s."""
    from qaa_inputs import serving_workload
    out = []
    for rate in rates:
        wl = serving_workload(count, rate, n_lo=n_lo, n_hi=n_hi, t_lo=t_lo, t_hi=t_hi)
        res, secs = _serve_stream(qaa, wl, slots, budget, verbose=False)
        lat = [r["latency_s"] for r in res]
        out.append({"rate_per_s": rate, "requests": count, "p50_s": _percentile(lat, 50),
                    "p99_s": _percentile(lat, 99), "mean_queued_s": sum(r["queued_s"] for r in res) / count,
                    "solves_per_s": count / secs,
                    "amp_steps_per_s": sum((1 << w["n"]) * w["steps"] for w in wl) / secs})
        log("serving rate %.2f/s: p50 %.3f s p99 %.3f s, %.2f solves/s"
            % (rate, out[-1]["p50_s"], out[-1]["p99_s"], out[-1]["solves_per_s"]))
    return {"workload": "Poisson arrivals, n ~ U{%d..%d}, T ~ U[%g,%g), dt ~ 0.01, %d slots, %.1f GiB budget"
                        % (n_lo, n_hi, t_lo, t_hi, slots, budget / 2.0 ** 30), "points": out}


def _bootstrap_ci(xs, q, reps=2000, seed=1):
    """95 % bootstrap interval of the q-th percentile of xs."""
    import random
    rng = random.Random(seed)
    est = sorted(_percentile([xs[rng.randrange(len(xs))] for _ in xs], q) for _ in range(reps))
    return [est[int(0.025 * reps)], est[int(0.975 * reps) - 1]]


def _serve_stream(qaa, wl, slots, budget, verbose=True):
    """Submit the requests of wl at their arrival times (open loop) and poll
    them; returns the results in request order and the wall time from the
    first arrival to the last completion.  verbose: log each completion, and
    each quarter of a running request's steps as the server reports them."""
    from qaa_inputs import planted_unique_3sat
    lits = [planted_unique_3sat(w["n"], w["seed"]).literals() for w in wl]
    count = len(wl)
    res = [None] * count
    tickets = []
    quarter = [0] * count
    done = 0
    sv = qaa.qaa_server_create(budget, slots)
    try:
        t0 = time.perf_counter()
        while done < count:
            now = time.perf_counter() - t0
            while len(tickets) < count and wl[len(tickets)]["arrival"] <= now:
                w = wl[len(tickets)]
                tickets.append(qaa.qaa_server_submit(sv, w["n"], lits[len(tickets)], w["T"], w["steps"]))
            for j, t in enumerate(tickets):
                if res[j] is not None:
                    continue
                r = qaa.qaa_server_poll(sv, t)
                if r["done"]:
                    res[j] = r
                    done += 1
                    if verbose:
                        log("  request %d/%d n=%d T=%.1f done (%d finished): latency %.2f s, queued %.2f s"
                            % (j + 1, count, wl[j]["n"], wl[j]["T"], done, r["latency_s"], r["queued_s"]))
                elif verbose and r["steps"] and 4 * r["steps_done"] // r["steps"] > quarter[j]:
                    quarter[j] = 4 * r["steps_done"] // r["steps"]
                    log("  request %d/%d n=%d: %d of %d steps" % (j + 1, count, wl[j]["n"], r["steps_done"],
                                                                r["steps"]))
            nxt = wl[len(tickets)]["arrival"] - (time.perf_counter() - t0) if len(tickets) < count else 0.002
            time.sleep(min(0.002, max(0.0, nxt)))
        t_end = time.perf_counter()
    finally:
        qaa.qaa_server_destroy(sv)
    bad = [r for r in res if r["status"] != qaa.QAA_OK]
    if bad:
        raise RuntimeError("serving: %d requests failed (status %d)" % (len(bad), bad[0]["status"]))
    return res, t_end - t0


def _exclusive_step_ms(qaa, torch, n_lo, n_hi, seed=77, steps=10, warm=2):
    """Step time of one request running alone, per n (complex64, uint8
    table), and its one-off set-up (table, initial state, observables)."""
    from qaa_inputs import planted_unique_3sat
    out = {}
    for n in range(n_lo, n_hi + 1):
        li = planted_unique_3sat(n, seed + n).literals()
        amp = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
        table = torch.empty(1 << n, dtype=torch.uint8, device="cuda")
        h = qaa.Instance(n, li)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qaa.qaa_energy_table(h.handle, table, qaa.QAA_E_U8)
        st = qaa.make_state(h.handle, amp, table, qaa.QAA_E_U8)
        qaa.qaa_state_init_uniform(st)
        qaa.qaa_observables(st)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        qaa.qaa_evolve_range(st, 100.0, 10000, 0, warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qaa.qaa_evolve_range(st, 100.0, 10000, warm, warm + steps)
        torch.cuda.synchronize()
        out[n] = {"step_ms": (time.perf_counter() - t0) / steps * 1e3, "setup_s": setup}
        h.close()
        del amp, table
        log("  alone: n=%d %.4f ms/step, set-up %.3f s" % (n, out[n]["step_ms"], setup))
    torch.cuda.empty_cache()          # the server allocates on its own
    return out


def run_serving_c5(qaa, torch, fractions, count, n_lo, n_hi, capacity_sample, one_slot, slots, budget,
                   t_lo=10.0, t_hi=200.0):
    """The serving workload: n ~ U{n_lo..n_hi}, T ~ U[t_lo, t_hi), dt = 0.01,
    Poisson arrivals at fractions of capacity; latency p50/p99 with 95 %
    bootstrap intervals and completed solves/s per arrival rate.

    Capacity (solves/s): the exclusive-service model 1 / E[service] from
    each n's measured step time alone (E over the n and T distributions),
    and, when capacity_sample > 0, a closed-loop measurement (that many
    requests submitted at once, completed requests over the makespan) which
    also counts the overlap of small solves; the arrival rates use the
    closed-loop figure when there is one.  one_slot > 0: the same arrival
    stream at that fraction once more through a one-slot server (one solve
    at a time), the plain path the slots are compared with."""
    from qaa_inputs import serving_workload
    dt = 0.01
    out = {"workload": "Poisson arrivals, n ~ U{%d..%d}, T ~ U[%g,%g), dt = %g, %d slots, %.0f GiB budget"
                       % (n_lo, n_hi, t_lo, t_hi, dt, slots, budget / 2.0 ** 30)}
    log("serving: exclusive step times for n = %d..%d" % (n_lo, n_hi))
    alone = _exclusive_step_ms(qaa, torch, n_lo, n_hi)
    mean_steps = (t_lo + t_hi) / 2.0 / dt
    service = sum(a["setup_s"] + mean_steps * a["step_ms"] * 1e-3 for a in alone.values()) / len(alone)
    out["alone"] = {str(k): v for k, v in alone.items()}
    out["capacity_model"] = {"mean_service_s": service, "solves_per_s": 1.0 / service,
                             "basis": "1 / E[set-up + steps x step time alone], n and T uniform"}
    capacity = 1.0 / service
    log("serving: exclusive-service capacity %.4f solves/s (mean service %.2f s)" % (capacity, service))
    if capacity_sample > 0:
        wl = serving_workload(capacity_sample, 1e9, seed=55, n_lo=n_lo, n_hi=n_hi, t_lo=t_lo, t_hi=t_hi, dt=dt)
        log("serving capacity: %d requests at once" % capacity_sample)
        res, secs = _serve_stream(qaa, wl, slots, budget, verbose=False)
        capacity = capacity_sample / secs
        out["capacity"] = {"requests": capacity_sample, "seconds": secs, "solves_per_s": capacity,
                           "amp_steps": sum((1 << w["n"]) * w["steps"] for w in wl)}
        log("serving capacity (closed loop): %.4f solves/s" % capacity)
    points = []

    def point(f, nslots):
        rate = f * capacity
        wl = serving_workload(count, rate, seed=int(1000 * f) + 7, n_lo=n_lo, n_hi=n_hi, t_lo=t_lo, t_hi=t_hi,
                              dt=dt)
        log("serving at %.2f of capacity: %.4f requests/s, %d requests, %d slots" % (f, rate, count, nslots))
        res, secs = _serve_stream(qaa, wl, nslots, budget)
        lat = [r["latency_s"] for r in res]
        p = {"fraction": f, "slots": nslots, "rate_per_s": rate, "requests": count, "seconds": secs,
             "p50_s": _percentile(lat, 50), "p50_ci95": _bootstrap_ci(lat, 50),
             "p99_s": _percentile(lat, 99), "p99_ci95": _bootstrap_ci(lat, 99),
             "mean_queued_s": sum(r["queued_s"] for r in res) / count, "solves_per_s": count / secs,
             "n": [w["n"] for w in wl], "latency_s": [round(x, 4) for x in lat]}
        log("serving %.2f (%d slots): p50 %.3f s p99 %.3f s, %.3f solves/s"
            % (f, nslots, p["p50_s"], p["p99_s"], p["solves_per_s"]))
        return p

    for f in fractions:
        points.append(point(f, slots))
    if one_slot > 0:
        points.append(point(one_slot, 1))
    out["points"] = points
    return out


def run_recompute(qaa, torch, n, lits, T, N, K, knots, table_amp):
    """The timed job's K steps again on a state with no energy table (the
    phase passes score the clauses themselves): energy statistics, initial
    state and the steps timed apart; the final state compared with the
    table mode's bit for bit."""
    amp = torch.empty(1 << n, dtype=torch.complex64, device=table_amp.device)
    h = qaa.Instance(n, lits)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qaa.qaa_energy_stats(h.handle)
    t_stats = time.perf_counter() - t0
    st = qaa.make_state(h.handle, amp, None, qaa.QAA_E_U8)
    qaa.qaa_state_init_uniform(st)
    torch.cuda.synchronize()
    qaa.qaa_profile_read(reset=True)
    qaa.qaa_profile_enable(True)
    t0 = time.perf_counter()
    qaa.qaa_evolve_range(st, T, N, 0, K, knots=knots)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    qaa.qaa_profile_enable(False)
    prof = qaa.qaa_profile_read(reset=True)
    obs = qaa.qaa_observables(st)
    same = bool(torch.equal(amp, table_amp))
    h.close()
    del amp
    avg_ms = prof["kernel_ms"] / max(1, prof["launches"])
    return {"steps": K, "ms_per_step_steps": secs / K * 1e3, "energy_stats_s": t_stats,
            "amp_steps_per_s": (1 << n) * K / secs, "pass_launches": prof["launches"],
            "avg_launch_ms": avg_ms,
            "achieved_gbs": prof["alg_bytes"] / max(1, prof["launches"]) / (avg_ms * 1e-3) / 1e9
            if prof["launches"] else 0.0,
            "identical_state": same, "p_success": obs["p_success"], "norm": obs["norm"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--record", type=str, default="", metavar="PATH",
                    help="also append the result line, with the host and library versions, to this JSONL file")
    ap.add_argument("--steps", type=int, default=5000, help="second-order steps timed (default: the full job)")
    ap.add_argument("--warmup", type=int, default=20, help="untimed warm-up steps")
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--T", type=float, default=50.0, help="total evolution time of the schedule")
    ap.add_argument("--schedule-steps", type=int, default=5000, help="second-order steps of the whole schedule")
    ap.add_argument("--schedule-knots", type=int, default=0, metavar="K",
                    help="0: the linear schedule s = t/T; K >= 2: a K-knot schedule table sampling "
                         "s(u) = u + 0.9 sin(2 pi u)/(2 pi), which slows the sweep around s = 1/2")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=2)
    ap.add_argument("--no-pass-events", action="store_true",
                    help="time the region without the per-pass events (no roofline object): at small n the "
                         "events' host cost per launch exceeds a pass and the profiled run becomes launch-bound")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 2 GiB device copy (torch copy_), the reference dispatch for "
                         "scaling HBM counter readings")
    ap.add_argument("--batch", type=int, default=512, metavar="COUNT",
                    help="batched workload size (512 is the full one; 0 skips it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the recompute-mode, batched, serving and spectrum workloads")
    ap.add_argument("--no-recompute", dest="recompute", action="store_false",
                    help="skip the recompute-mode run (the same steps with no energy table)")
    ap.add_argument("--batch-loop-sample", type=int, default=64)
    ap.add_argument("--serve", type=str, default="4,8", metavar="RATES",
                    help="open-loop serving at these comma-separated arrival rates (requests/s); '' skips it")
    ap.add_argument("--serve-requests", type=int, default=60)
    ap.add_argument("--serve-n", type=str, default="16,24", help="n range lo,hi of served requests")
    ap.add_argument("--serve-t", type=str, default="10,50", help="T range lo,hi of served requests")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-c5", type=str, default="", metavar="FRACTIONS",
                    help="the serving workload (n ~ U{16..31} by default, T ~ U[10,200)) at these "
                         "comma-separated fractions of capacity; minutes to hours, off by default")
    ap.add_argument("--serve-c5-requests", type=int, default=200, help="requests per arrival rate")
    ap.add_argument("--serve-c5-n", type=str, default="16,31", help="n range lo,hi of the served requests")
    ap.add_argument("--serve-c5-t", type=str, default="10,200", help="T range lo,hi of the served requests")
    ap.add_argument("--serve-c5-capacity-sample", type=int, default=0, metavar="COUNT",
                    help="closed-loop capacity from COUNT requests submitted at once (0: the exclusive-service "
                         "model alone)")
    ap.add_argument("--serve-c5-one-slot", type=float, default=0.0, metavar="FRACTION",
                    help="also run that fraction's arrival stream through a one-slot server")
    ap.add_argument("--spectrum", type=str, default="20,21,150", metavar="N,POINTS,ITERS",
                    help="lowest two levels of H(s) for an n-qubit instance on POINTS values of s with ITERS "
                         "Lanczos steps each (qaa_spectrum); empty: skip")
    ap.add_argument("--autotune", action="store_true",
                    help="run the plan autotuner for this n before the timed region (qaa_autotune)")
    ap.add_argument("--precision", action="store_true",
                    help="also run the same job with a complex128 state and report the complex64 error")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library evolves each state on a single MI355X and has no "
              "multi-GPU path (asked for --gpus %d, WORLD_SIZE=%d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1103_1399_amd as qaa
    from qaa_inputs import planted_unique_3sat

    n, T, N = args.n, args.T, args.schedule_steps
    if args.schedule_knots == 1 or args.schedule_knots > 256:
        print("--schedule-knots must be 0 or in [2, 256]", file=sys.stderr)
        sys.exit(2)
    knots = schedule_table(args.schedule_knots)
    K, W = args.steps, args.warmup
    if not (1 <= K <= N) or not (0 <= W <= N):
        print("--steps must be in [1, %d] and --warmup in [0, %d]" % (N, N), file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    log("generating instance n=%d seed=%d" % (n, args.seed))
    inst_in = planted_unique_3sat(n, args.seed)
    lits = inst_in.literals()
    plan = qaa.qaa_plan_info(n, qaa.QAA_C64)

    # device buffers (allocated before timing)
    table = torch.empty(1 << n, dtype=torch.uint8, device=dev)
    amp = torch.empty(1 << n, dtype=torch.complex64, device=dev)

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.complex64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (src.numel() * 8, dst.numel() * 8))
        del src, dst

    copy_gbs = device_copy_gbs(torch, 8 << n)
    log("device copy of %d bytes: %.0f GB/s (read + write)" % (8 << n, copy_gbs))

    # warm-up: full path on the same buffers, W steps
    log("warm-up (%d steps)" % W)
    h = qaa.Instance(n, lits)
    qaa.qaa_energy_table(h.handle, table, qaa.QAA_E_U8)
    st = qaa.make_state(h.handle, amp, table, qaa.QAA_E_U8)
    if args.autotune:
        tuned = qaa.qaa_autotune(st, steps=10)
        log("autotune: %s" % tuned)
    qaa.qaa_state_init_uniform(st)
    if W:
        qaa.qaa_evolve_range(st, T, N, 0, W, knots=knots)
    qaa.qaa_observables(st)
    torch.cuda.synchronize()
    h.close()

    # one-off parts of the job, timed on their own: the energy table from
    # the clause list (synchronous call) and the uniform initial state
    log("job set-up: energy table and initial state")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = qaa.Instance(n, lits)
    qaa.qaa_energy_table(h.handle, table, qaa.QAA_E_U8)
    torch.cuda.synchronize()
    t_table = time.perf_counter() - t0
    st = qaa.make_state(h.handle, amp, table, qaa.QAA_E_U8)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    ev[0].record()
    qaa.qaa_state_init_uniform(st)
    ev[1].record()
    torch.cuda.synchronize()
    t_init = ev[0].elapsed_time(ev[1]) * 1e-3

    # the timed region: exactly K steps, synchronized on both sides
    log("timed: %d steps" % K)
    qaa.qaa_profile_read(reset=True)
    qaa.qaa_profile_enable(not args.no_pass_events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[2].record()
    qaa.qaa_evolve_range(st, T, N, 0, K, knots=knots)
    ev[3].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    qaa.qaa_profile_enable(False)
    prof = qaa.qaa_profile_read(reset=True)
    secs = t1 - t0
    t_steps_events = ev[2].elapsed_time(ev[3]) * 1e-3

    ev[4].record()
    obs = qaa.qaa_observables(st)
    ev[5].record()
    torch.cuda.synchronize()
    t_obs = ev[4].elapsed_time(ev[5]) * 1e-3
    log("timed region %.4f s for %d steps (events %.4f s); table %.4f s, init %.5f s, observables %.5f s; "
        "P_success=%.6f norm=%.9f" % (secs, K, t_steps_events, t_table, t_init, t_obs, obs["p_success"],
                                     obs["norm"]))
    # whole-job costing: steady steps plus the one-off parts charged to N steps
    s_per_step = secs / K + (t_table + t_init + t_obs) / N

    avg_ms = prof["kernel_ms"] / max(1, prof["launches"])
    bytes_per_launch = prof["alg_bytes"] / max(1, prof["launches"])
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if prof["launches"] else 0.0
    traffic = None
    if MEASURED_TRAFFIC["kernel_source_sha256"] == kernel_source_sha():
        traffic = MEASURED_TRAFFIC["bytes_per_launch"]
    roofline = None if args.no_pass_events else {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "copy_gbs": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4),
        "kernel": "qaa pass_kernel (complex64, uint8 table, 2^%d-amplitude tiles)" % plan["tile_bits"],
        "launches": prof["launches"],
        "avg_launch_ms": round(avg_ms, 4),
        "alg_bytes_per_launch": bytes_per_launch,
    }

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, %d steps sample)" % args.cpu_sample_steps)
        cpu = cpu_baseline(inst_in, n, T, N, args.cpu_sample_steps, knots)

    extras = {}
    if args.no_extras:
        args.batch, args.serve, args.spectrum, args.recompute = 0, "", "", False
    if args.precision:
        log("precision study: complex128 run of the same %d steps" % K)
        ref = torch.empty(1 << n, dtype=torch.complex128, device=dev)
        h2 = qaa.Instance(n, lits)
        qaa.qaa_energy_table(h2.handle, table, qaa.QAA_E_U8)
        st2 = qaa.make_state(h2.handle, ref, table, qaa.QAA_E_U8)
        qaa.qaa_state_init_uniform(st2)
        qaa.qaa_evolve_range(st2, T, N, 0, K, knots=knots)
        obs2 = qaa.qaa_observables(st2)
        l2 = float(torch.linalg.vector_norm(amp.to(torch.complex128) - ref).item())
        extras["precision"] = {
            "reference": "complex128 state on the GPU, same kernels' FP64 variant",
            "l2_state": l2,
            "abs_dp_success": abs(obs["p_success"] - obs2["p_success"]),
            "abs_d_energy": abs(obs["energy"] - obs2["energy"]),
            "norm_c64_minus_1": obs["norm"] - 1.0,
            "p_success_c128": obs2["p_success"],
        }
        h2.close()
        del ref
    if args.recompute:
        log("recompute mode: the same %d steps with no energy table" % K)
        extras["recompute"] = run_recompute(qaa, torch, n, lits, T, N, K, knots, amp)
        log("recompute: %.4f ms/step (table mode %.4f), identical state: %s" % (
            extras["recompute"]["ms_per_step_steps"], secs / K * 1e3, extras["recompute"]["identical_state"]))
    if args.batch:
        log("batched workload (%d instances)" % args.batch)
        extras["batch"] = run_batch(qaa, torch, args.batch, 2024, min(args.batch, args.batch_loop_sample))
        log("batch: %.2f solves/s, %.3e amp-steps/s (loop %.3e)" % (
            extras["batch"]["solves_per_s"], extras["batch"]["amp_steps_per_s"],
            extras["batch"]["loop"]["amp_steps_per_s"]))
    if args.spectrum:
        sn, sp, si = (int(x) for x in args.spectrum.split(","))
        log("spectrum: n=%d, %d values of s, %d Lanczos steps each" % (sn, sp, si))
        extras["spectrum"] = run_spectrum(qaa, torch, sn, sp, si, 7)
        log("spectrum: %.3f s, min gap %.4f at s=%.2f" % (extras["spectrum"]["seconds"], extras["spectrum"]["min_gap"],
                                                       extras["spectrum"]["s_at_min_gap"]))
    if args.serve:
        rates = [float(x) for x in args.serve.split(",") if x]
        nlo, nhi = (int(x) for x in args.serve_n.split(","))
        tlo, thi = (float(x) for x in args.serve_t.split(","))
        extras["serving"] = run_serving(qaa, args.serve_requests, rates, nlo, nhi, tlo, thi, args.serve_slots,
                                        int(args.serve_budget_gib * 2 ** 30))

    if args.serve_c5:
        fr = [float(x) for x in args.serve_c5.split(",") if x]
        lo, hi = (int(x) for x in args.serve_c5_n.split(","))
        tlo, thi = (float(x) for x in args.serve_c5_t.split(","))
        extras["serving_c5"] = run_serving_c5(qaa, torch, fr, args.serve_c5_requests, lo, hi,
                                              args.serve_c5_capacity_sample, args.serve_c5_one_slot,
                                              args.serve_slots, 256 << 30, tlo, thi)

    value = (2.0 ** n) / s_per_step
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "amplitude-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": s_per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "planted unique-solution 3-SAT, n=%d qubits (m=%d clauses, seed %d), %s schedule "
                        "T=%g with %d second-order steps, complex64 state + uint8 energy table, uniform start"
                        % (n, inst_in.m, args.seed,
                           "linear" if knots is None else "%d-knot table" % len(knots), T, N),
            "n": n, "m": inst_in.m, "T": T, "schedule_steps": N,
            "schedule": "linear" if knots is None else {"knots": len(knots)},
            "plan": plan,
            "plan_choice": qaa.qaa_plan_get(n, qaa.QAA_C64),
        },
        "region": {"steps": K, "seconds": secs, "ms_per_step": secs / K * 1e3,
                   "amp_steps_per_s": (2.0 ** n) * K / secs, "events_seconds": t_steps_events,
                   "passes": prof["launches"]},
        "job_one_off_s": {"energy_table": t_table, "init": t_init, "observables": t_obs,
                          "charged_per_step_ms": (t_table + t_init + t_obs) / N * 1e3},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "result": {"p_success": obs["p_success"], "energy": obs["energy"], "norm": obs["norm"],
                   "steps_done": K},
    }
    out.update(extras)
    if cpu:
        out["gpu_over_cpu"] = value / cpu["value"]
    line = json.dumps(out)
    print(line, flush=True)
    if args.record:
        rec = dict(out)
        rec["record"] = {"time_unix": time.time(), "host_cpus": os.cpu_count(), "torch": torch.__version__,
                         "hip": torch.version.hip, "device": torch.cuda.get_device_name(dev),
                         "libqaa_version": qaa.qaa_version(), "kernel_source_sha256": kernel_source_sha(),
                         "argv": sys.argv[1:]}
        with open(args.record, "a") as f:
            f.write(json.dumps(rec) + "\n")


if __name__ == "__main__":
    main()
