/*
 * qaa.h -- C ABI of the MI355X (gfx950) library that evolves an n-qubit
 * state vector under the adiabatic 3-SAT Hamiltonian
 *
 *     H(s) = (1 - s) H_B + s H_P,   s = t / T            (Sec. 2.1, eq. 1)
 *     H_B  = sum_i (1 - sigma^x_i) / 2                    (ground state: the
 *            uniform superposition of Sec. 2.1)
 *     H_P |z> = E(z) |z>,  E(z) = number of clauses unsatisfied by z
 *                                                         (Sec. 4.3)
 *
 * with N second-order split steps: step k (0 <= k < N) evaluates the
 * schedule at the midpoint s_k = s((k + 1/2)/N), dt = T/N, and applies
 *     exp(-i dt/2 s_k H_P) exp(-i dt (1 - s_k) H_B) exp(-i dt/2 s_k H_P).
 * The schedule s(u), u = t/T, is the paper's linear s = u or a
 * caller-given piecewise-linear table (qaa_schedule).
 * The paper does not name its integrator; this splitting is the build's
 * reading and is what the test oracle computes.
 *
 * Conventions
 *  - Literals are DIMACS style (Sec. 2.2 K-SAT definition): +v is x_v,
 *    -v is "not x_v", 1 <= v <= n; three distinct variables per clause.
 *  - Variable x_i lives on qubit q_i = bit (i-1) of the basis index z
 *    (basis order |q_n ... q_1> of Sec. 2.1).
 *  - Amplitudes: 2^n complex numbers in device memory, interleaved
 *    (re, im), index z; complex64 (float pairs) or complex128.  Amplitude
 *    and energy-table buffers must be 16-byte aligned and live on the
 *    calling thread's current HIP device.
 *  - Every device pointer is caller-owned: the library never frees or
 *    reallocates a caller buffer.  Buffers must stay alive until the work
 *    queued on the stream has finished.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on it unless stated otherwise.
 *  - Library-owned device memory: a device copy of each instance's clause
 *    list, the 64 KiB scratch array of qaa_evolve_range_noalloc (one per
 *    device, held until the process ends), and per-call buffers (norm
 *    accumulators, reduction partials, batch descriptors, qaa_spectrum's
 *    Lanczos vectors) taken from the stream-ordered allocator and released
 *    in stream order by the call that took them.
 *  - Calls on different streams share no library state on the device and
 *    run concurrently, including the ones that read back results
 *    (qaa_energy_table, qaa_observables), which wait for their own stream
 *    only.
 *  - Errors: every call returns a qaa_status; nothing throws or aborts
 *    across the ABI.  qaa_last_error() returns a thread-local message for
 *    the last failing call of the calling thread.
 */
#ifndef QAA_H
#define QAA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum qaa_status {
    QAA_OK = 0,
    QAA_ERR_INVALID_ARG = 1,   /* argument outside the documented domain */
    QAA_ERR_UNSUPPORTED = 2,   /* valid but not supported (e.g. E_max > 255 with a uint8 table) */
    QAA_ERR_OUT_OF_MEMORY = 3, /* a library-owned allocation failed / request can never fit */
    QAA_ERR_DEVICE = 4,        /* a HIP runtime call or kernel launch failed */
    QAA_ERR_NOT_READY = 5,     /* a prerequisite call has not run (e.g. no energy table yet) */
    QAA_ERR_INTERNAL = 6,
    QAA_ERR_CANCELLED = 7      /* a served request was cancelled (qaa_server_cancel) */
} qaa_status;

typedef enum qaa_dtype {
    QAA_C64 = 0,    /* complex64: float re, float im */
    QAA_C128 = 1    /* complex128: double re, double im */
} qaa_dtype;

typedef enum qaa_etype {
    QAA_E_U8 = 0,   /* energy table entries as uint8 (requires E_max <= 255) */
    QAA_E_U16 = 1   /* energy table entries as uint16 (requires E_max <= 1023 for evolution) */
} qaa_etype;

/* Largest supported qubit count (2^34 complex64 = 128 GiB). */
#define QAA_MAX_QUBITS 34

/* ---------------------------------------------------------------------
 * Instances (Sec. 2.2 K-SAT definition, k = 3).
 * ------------------------------------------------------------------- */

typedef struct qaa_instance qaa_instance;

/*
 * Create an instance from a clause list.
 *   n    : number of variables / qubits, 1 <= n <= QAA_MAX_QUBITS.
 *   m    : number of clauses, 0 <= m <= 65535.
 *   lits : host array of 3*m signed literals (copied; may be freed after).
 *   out  : receives a host-owned handle; release with qaa_instance_destroy.
 * QAA_ERR_INVALID_ARG if n or m is out of range, a literal is 0 or |v| > n,
 * a clause repeats a variable, lits is NULL with m > 0, or out is NULL.
 * Duplicate clauses are allowed and counted once per copy.
 */
qaa_status qaa_instance_create(int32_t n, int32_t m, const int32_t *lits, qaa_instance **out);

/* Release an instance (NULL is ignored).  Frees the library-owned device
 * copy of the clause list; no queued work may still use the instance. */
void qaa_instance_destroy(qaa_instance *inst);

/*
 * Query an instance.  Any output pointer may be NULL.  e_min, e_max and
 * degeneracy (number of z with E(z) = e_min: the ground-manifold size of
 * Sec. 2.1) are -1 until qaa_energy_table has run once for the instance.
 */
qaa_status qaa_instance_info(const qaa_instance *inst, int32_t *n, int32_t *m,
                             int32_t *e_min, int32_t *e_max, int64_t *degeneracy);

/* ---------------------------------------------------------------------
 * Energy table: E(z) for all 2^n basis states (Sec. 4.3; the paper's GPU
 * kernel gives each thread basis states to score, Sec. 4.3 results).
 * ------------------------------------------------------------------- */

/*
 * Fill d_table[z] = E(z), z = 0 .. 2^n - 1, bit-exact.
 *   d_table : device buffer of 2^n uint8 (QAA_E_U8) or uint16 (QAA_E_U16).
 * SYNCHRONOUS: waits for the stream, then records e_min, e_max and the
 * degeneracy on the instance.  QAA_ERR_UNSUPPORTED if etype is QAA_E_U8 and
 * some E(z) > 255 (the table is then incomplete; use QAA_E_U16).
 */
qaa_status qaa_energy_table(qaa_instance *inst, void *d_table, qaa_etype etype, void *stream);

/*
 * Diagnostic: the energy kernel's arithmetic for one thread, run on the
 * host: out32[i] = E(z0 + i), i = 0..31 (z0 a multiple of 32 below 2^n; for
 * n < 5 only z0 = 0, and entries at i >= 2^n carry no meaning).  Host memory
 * only; exists so that host-side tests can check the bit-sliced counting
 * without a device.
 */
qaa_status qaa_debug_energy_block(const qaa_instance *inst, uint64_t z0, int32_t *out32);

/*
 * The statistics qaa_energy_table records (e_min, e_max, degeneracy) without
 * building a table: the energies are scored from the clause records and
 * discarded (two passes over the 2^n basis states).  Needed before a state
 * in recompute mode can evolve.  SYNCHRONOUS.
 */
qaa_status qaa_energy_stats(qaa_instance *inst, void *stream);

/* ---------------------------------------------------------------------
 * States.
 * ------------------------------------------------------------------- */

typedef struct qaa_state {
    const qaa_instance *inst;  /* instance the state evolves under */
    void *amp;                 /* device, 2^n interleaved complex amplitudes */
    qaa_dtype dtype;           /* QAA_C64 or QAA_C128 */
    const void *table;         /* device energy table filled by qaa_energy_table, or NULL:
                                  recompute mode (below) */
    qaa_etype etype;           /* element type of table (recompute mode: the width the
                                  energies are held in; QAA_E_U8 needs E_max <= 255) */
} qaa_state;

/*
 * Recompute mode.  A state whose table is NULL has the energy function
 * (Sec. 4.3: the number of violated clauses) scored from the instance's
 * clause records wherever it is needed -- in the evolution passes that
 * apply the diagonal phase, once per call for states held in one
 * workgroup, and in qaa_observables -- instead of being read from a
 * 2^n-entry table.  Results equal the table mode's to the bit (the same
 * integer counts).  It saves the table's 2^n (or 2 * 2^n) bytes of HBM at
 * the cost of ALU time in the phase passes.  qaa_energy_stats (or
 * qaa_energy_table) must have run for the instance.  Not offered by
 * qaa_evolve_batch, qaa_autotune and qaa_spectrum (QAA_ERR_UNSUPPORTED /
 * QAA_ERR_INVALID_ARG for a NULL table).
 */

/* psi(z) = 2^{-n/2}: the ground state of H_B (Sec. 2.1).  Needs only amp. */
qaa_status qaa_state_init_uniform(const qaa_state *st, void *stream);

/* psi = |z0>, a computational basis state (0 <= z0 < 2^n). */
qaa_status qaa_state_init_basis(const qaa_state *st, uint64_t z0, void *stream);

/* ---------------------------------------------------------------------
 * Evolution.
 * ------------------------------------------------------------------- */

/*
 * The interpolation schedule s(u) of H(s), u = t/T in [0, 1].
 *   QAA_SCHED_LINEAR: s(u) = u, the schedule of Sec. 2.1, eq. 1.
 *   QAA_SCHED_TABLE : s(u) is the piecewise-linear interpolant of
 *       count knots values[0..count) placed at u_j = j/(count - 1):
 *       with x = u (count - 1), j = min(floor(x), count - 2),
 *       s(u) = values[j] + (x - j) (values[j+1] - values[j]).
 *       A table lets the evolution slow down where the gap of H(s) is
 *       small (the paper only asks that s change slowly enough, Sec. 2.1);
 *       {0, 1} is the linear schedule, to the bit.
 *   count  : 2 <= count <= QAA_SCHED_MAX_KNOTS (TABLE only).
 *   values : host array of count knots, each finite and in [0, 1]; read
 *            during the call only (the library keeps its own copy).
 * A NULL qaa_schedule pointer means QAA_SCHED_LINEAR.  Step k evaluates
 * s at the step's midpoint u_k = (k + 1/2)/N.  QAA_ERR_INVALID_ARG for an
 * unknown kind, a count out of range, a NULL values array or a knot
 * outside [0, 1].
 */
typedef enum qaa_schedule_kind {
    QAA_SCHED_LINEAR = 0,
    QAA_SCHED_TABLE = 1
} qaa_schedule_kind;

#define QAA_SCHED_MAX_KNOTS 256

typedef struct qaa_schedule {
    int32_t kind;              /* qaa_schedule_kind */
    int32_t count;             /* TABLE: number of knots */
    const double *values;      /* TABLE: knot values s(u_j) */
} qaa_schedule;

/*
 * Apply all `steps` second-order steps of total time T to st->amp in place
 * (equivalent to qaa_evolve_range with k0 = 0, k1 = steps).
 *   sched : NULL (linear) or a qaa_schedule as described above.
 * steps == 0 is a no-op.  QAA_ERR_INVALID_ARG for T < 0, steps < 0, a NaN
 * T, a bad schedule, or a state without amp/table/inst.
 * QAA_ERR_UNSUPPORTED if the instance's E_max exceeds what the table type
 * allows.  Asynchronous.
 *
 * The state must have unit norm (as qaa_state_init_uniform / _basis leave
 * it; the evolution is unitary).  Norm control keeps it there against FP32
 * rounding: every measuring pass sums |psi|^2 as a 2^-60 fixed-point
 * integer, and the next one divides by the square root of what the
 * previous one measured -- so a state of another norm is rescaled to 1 as
 * it evolves (a multi-pass state of norm^2 >= 16 would overflow the
 * accumulator), and the norm that qaa_observables reports stays within
 * rounding of 1 rather than measuring the integration error.  States held
 * in one workgroup (n <= 13) are renormalised exactly once per 32 steps.
 */
qaa_status qaa_evolve(const qaa_state *st, const qaa_schedule *sched, double T,
                      int64_t steps, void *stream);

/*
 * Apply steps k0 .. k1-1 (0 <= k0 <= k1 <= steps) of the `steps`-step
 * evolution over total time T.  The state after range [k0, k1) is the state
 * after step k1 - 1 (both half phases applied), so
 * evolve_range(0, K); evolve_range(K, N) equals evolve(N) up to FP32 rounding
 * (the uninterrupted call merges the two half phases at K).  Asynchronous.
 */
qaa_status qaa_evolve_range(const qaa_state *st, const qaa_schedule *sched, double T,
                            int64_t steps, int64_t k0, int64_t k1, void *stream);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * evolution as qaa_evolve_range (same arguments, same kernels, bit-identical
 * results), but it allocates nothing.  The only device scratch an evolution
 * needs, the norm-control totals and partial sums (8192 + 16 64-bit words),
 * lives in a library-owned static device array of 64 KiB + 128 bytes per
 * device (held until the process
 * ends; its address is looked up once per device on the first call there).
 * Every state the library accepts fits it, so no size is refused beyond
 * what qaa_evolve_range refuses.  All calls on one device share that array
 * and a call clears it (with a kernel, not a memset) before use: calls that
 * overlap on one device -- on different streams or threads -- race and
 * must be serialised by the caller.  Asynchronous; errors as for
 * qaa_evolve_range, plus QAA_ERR_DEVICE if the array's address cannot be
 * obtained.
 */
qaa_status qaa_evolve_range_noalloc(const qaa_state *st, const qaa_schedule *sched, double T,
                                    int64_t steps, int64_t k0, int64_t k1, void *stream);

/*
 * Evolve `count` independent states together.  states[i], T[i] and
 * steps[i] (host arrays) as in qaa_evolve; the states may have different n.
 * scheds: NULL (every state linear) or a host array of `count` schedules,
 * scheds[i] for states[i], each as in qaa_evolve.
 * States whose whole vector fits one workgroup tile (n <= 13 for complex64,
 * 12 for complex128) run in one launch, one workgroup each; the others run
 * in lock step, one launch per pass and tile size covering every state
 * still running, with rotation and phase coefficients computed on the
 * device.  Each state follows the plan qaa_plan_get reports for its n.  Each result
 * equals what qaa_evolve gives for that state alone up to FP32 rounding
 * (same pass plan per n).  The call waits for the descriptor uploads (and
 * so for work already queued on the stream); the evolution itself is
 * asynchronous on the stream.  Internally the small states, and the launch
 * groups after the first (states sharing a number of qubit sets and tile
 * sizes, the heaviest split in two until each stream has a group), run on
 * library-owned streams of the device, forked from `stream` and joined
 * back into it: work queued on `stream` after the call waits for all of
 * them.  QAA_BATCH_STREAMS (0..3, default 2) sets how many streams the
 * launch groups after the first spread over; 0 keeps every group on
 * `stream`; QAA_BATCH_SPLIT=0 keeps one group per plan shape (results are
 * the same either way).
 */
qaa_status qaa_evolve_batch(int32_t count, const qaa_state *states, const qaa_schedule *scheds,
                            const double *T, const int64_t *steps, void *stream);

/* ---------------------------------------------------------------------
 * Spectrum of H(s).  How slowly the sweep must go is set by the gap
 * between the two lowest levels of H(s) along the path (Sec. 2.1); this
 * computes the lowest levels at given s.
 * ------------------------------------------------------------------- */

#define QAA_SPECTRUM_MAX_ITERS 1024

/*
 * The k lowest eigenvalues of H(s) = (1 - s) H_B + s H_P at each of `count`
 * values of s, by Lanczos with full reorthogonalisation (the three-term
 * recurrence, then one classical Gram-Schmidt sweep against every earlier
 * vector) in FP64 on the device; the Ritz values of
 * the tridiagonal matrix come from Sturm-sequence bisection on the host.
 *   inst, table, etype : an instance and its energy table (qaa_energy_table
 *                        must have run for it; table is device memory)
 *   s_values           : host array of count values, each in [0, 1]
 *   v0                 : device array of 2^n doubles, the start vector (not
 *                        modified).  A random vector reaches every level
 *                        with probability 1; a level whose eigenvectors
 *                        are orthogonal to v0 is never seen.
 *   iters              : Lanczos steps, 1 <= iters <= QAA_SPECTRUM_MAX_ITERS
 *                        (at most 2^n are taken)
 *   k                  : values per s, 1 <= k <= iters
 *   evals              : host array [count][k]: row i holds the k lowest
 *                        levels (distinct eigenvalues) at s_values[i],
 *                        ascending: Ritz values closer than 1e-10 of the
 *                        matrix scale (max_j |alpha_j| + 2 beta_j, about
 *                        the spectral radius) count as one level.  NaN
 *                        where the run found fewer than k levels.
 *   bounds             : NULL, or a host array [count][k] that receives
 *                        the residual norm |beta_m y_m| of each returned
 *                        Ritz value (y the unit eigenvector of the m x m
 *                        tridiagonal matrix): H(s) has an eigenvalue
 *                        within that distance of it.  Small bounds on the
 *                        two lowest levels mean the gap is resolved.
 * The accuracy of the Ritz values grows with iters (the lowest converge
 * first).  SYNCHRONOUS.  Takes about (iters + 2) * 2^n * 8 bytes of device
 * memory from the stream-ordered allocator for the call:
 * QAA_ERR_OUT_OF_MEMORY if that fails.  QAA_ERR_INVALID_ARG for bad
 * arguments or a zero / non-finite v0 (detected after the run);
 * QAA_ERR_NOT_READY if the instance has no energy table yet.
 */
qaa_status qaa_spectrum(const qaa_instance *inst, const void *table, qaa_etype etype, int32_t count,
                        const double *s_values, const double *v0, int32_t iters, int32_t k, double *evals,
                        double *bounds, void *stream);

/* ---------------------------------------------------------------------
 * Observables (Sec. 2.1: the result is read from the weight on the ground
 * manifold of H_P).  FP64 accumulation, deterministic order.
 * ------------------------------------------------------------------- */

typedef struct qaa_obs {
    double norm;          /* sum_z |psi(z)|^2 */
    double energy;        /* <H_P> = sum_z E(z) |psi(z)|^2 */
    double p_success;     /* sum over z with E(z) = e_min of |psi(z)|^2 */
    int32_t e_min;        /* minimum of E */
    int64_t degeneracy;   /* number of z with E(z) = e_min */
} qaa_obs;

/* SYNCHRONOUS: enqueues the reduction on the stream, waits for it, and
 * fills *out.  QAA_ERR_NOT_READY if the instance has no energy table yet. */
qaa_status qaa_observables(const qaa_state *st, qaa_obs *out, void *stream);

/* ---------------------------------------------------------------------
 * Serving: a solve-request server.  Requests are admitted in arrival order
 * when one of `slots` workers is free and their HBM footprint
 * (qaa_server_footprint) fits the budget beside the admitted ones; each worker runs its solve (energy table, uniform
 * start, qaa_evolve_range over chunks of steps, qaa_observables) on its own HIP stream, so solves
 * admitted while others run overlap on the device.  The server allocates
 * and frees each request's device buffers on the current device of the
 * thread that created it.
 * ------------------------------------------------------------------- */

typedef struct qaa_server qaa_server;

typedef struct qaa_server_config {
    uint64_t hbm_budget_bytes;  /* admitted requests' footprints never exceed this */
    int32_t slots;              /* concurrent solves (worker threads / streams), 1..64 */
    int32_t reserved;           /* set to 0 */
} qaa_server_config;

typedef struct qaa_server_result {
    qaa_status status;          /* QAA_OK once done without error (QAA_ERR_CANCELLED if cancelled) */
    int32_t done;               /* 1 when the solve finished, failed or was cancelled */
    qaa_obs obs;                /* observables of the final state (done == 1) */
    double queued_s;            /* time from submit to admission (so far, if not admitted) */
    double latency_s;           /* time from submit to completion (so far, if not done) */
    int64_t steps;              /* the request's step count */
    int64_t steps_done;         /* steps finished on the device so far (the solve evolves in
                                   chunks and records each; == steps once done without error) */
} qaa_server_result;

/* Device bytes a request of n qubits and m clauses is charged at
 * admission: the complex64 state (8 * 2^n), the energy table (2^n bytes, or
 * 2 * 2^n when m > 255, since only then can a count exceed 255 and the
 * solve widen the table), 16 bytes per clause record and 64 KiB of the
 * library's per-call scratch.  0 for n or m out of range. */
uint64_t qaa_server_footprint(int32_t n, int32_t m);

/* Start a server (threads and streams).  QAA_ERR_INVALID_ARG for a NULL
 * argument, slots outside 1..64 or a zero budget. */
qaa_status qaa_server_create(const qaa_server_config *cfg, qaa_server **out);

/* Queue a solve of the instance (n, m, lits; as qaa_instance_create) for
 * total time T and `steps` steps under schedule `sched` (NULL: linear; as
 * in qaa_evolve); *ticket identifies it.  Copies lits and the schedule's
 * knots.  QAA_ERR_OUT_OF_MEMORY if its footprint exceeds the whole budget
 * (it could never be admitted); QAA_ERR_INVALID_ARG for malformed arguments
 * or a bad schedule (clause errors are reported through the result). */
qaa_status qaa_server_submit(qaa_server *sv, int32_t n, int32_t m, const int32_t *lits,
                             const qaa_schedule *sched, double T, int64_t steps, int64_t *ticket);

/* Non-blocking status of a ticket.  A finished request's record (its
 * status, observables and times, about 100 bytes) is kept until destroy. */
qaa_status qaa_server_poll(qaa_server *sv, int64_t ticket, qaa_server_result *out);

/* Cancel a request.  Still queued: it leaves the queue at once and
 * finishes with status QAA_ERR_CANCELLED.  Running: the solve stops at its
 * next chunk boundary (see above; the device finishes the chunk in flight),
 * frees its buffers and finishes with QAA_ERR_CANCELLED, steps_done
 * telling how far it got; a solve already in its last chunk (at small n,
 * the whole solve is one chunk) runs to its end and finishes normally.  Already finished: nothing changes.  Either way
 * the call returns QAA_OK without waiting; QAA_ERR_INVALID_ARG for a NULL
 * server or an unknown ticket. */
qaa_status qaa_server_cancel(qaa_server *sv, int64_t ticket);

/* Block until the ticket's solve has finished, then fill *out. */
qaa_status qaa_server_wait(qaa_server *sv, int64_t ticket, qaa_server_result *out);

/* Queue length, running solves and admitted footprint in bytes (any may be NULL). */
qaa_status qaa_server_stats(qaa_server *sv, int64_t *queued, int64_t *running, uint64_t *bytes_in_use);

/* Stop the server: solves already admitted finish, queued ones are dropped,
 * then the server is freed.  No other call on this server may run
 * concurrently with or after this one.  NULL is ignored. */
void qaa_server_destroy(qaa_server *sv);

/* ---------------------------------------------------------------------
 * Plans (how a step is split into HBM passes) -- introspection.
 * ------------------------------------------------------------------- */

/*
 * Describe the pass plan used for n qubits of the given dtype:
 *   *tile_bits      : qubits held per workgroup tile (0 = whole state in one
 *                     workgroup, all steps in one launch)
 *   *sets           : qubit sets the n qubits are split into
 *   *passes_per_step: HBM read+write passes per step in steady state
 */
qaa_status qaa_plan_info(int32_t n, qaa_dtype dtype, int32_t *tile_bits, int32_t *sets,
                         int32_t *passes_per_step);

/*
 * How a plan with two or more sets assigns qubits and tiles:
 *   balance    : 1 = the top set also rotates set 0's highest qubits, up to
 *                as many as its tile can hold.
 *   passengers : 1 = with three or more sets, the low "passenger" qubits
 *                (1..4 for complex64, 0..3 for complex128), which ride in
 *                every set's tiles, rotate in the set-1 passes instead of
 *                the set-0 turn.
 *   tiles      : 0 = every set in the base tile (2^13 amplitudes for
 *                complex64, 2^12 for complex128); 1 = the top set's passes
 *                in 2^14-amplitude tiles (longer contiguous runs in the pass
 *                that gathers from the whole state); 2 = every set in
 *                2^14-amplitude tiles, the qubits above set 0 split evenly.
 *                Tiles 1 and 2 apply to complex64 states with a uint8 table
 *                and n >= 22 only (elsewhere the base tile is used whatever
 *                is recorded).
 * Beyond the choice, two things follow from the plan's shape: complex64
 * plans of two sets in 2^13-amplitude tiles (n = 14..21) run 512 threads
 * of 16 amplitudes per tile instead of 256 of 32, and three-set complex64
 * plans from n = 30 on give set 1 the four highest qubits as well as the
 * lowest high ones, the top set taking the run between them
 * (QAA_PLAN_SPREAD = a digit sets that count for every n; 0 turns it off).
 * Results do not depend on the choice beyond FP32 rounding order.  The
 * choice is process-wide per (n, dtype); the environment variables
 * QAA_PLAN_BALANCE / QAA_PLAN_PASSENGERS (0 or 1) and QAA_PLAN_TILES
 * (0, 1 or 2), if set, override it.
 */
typedef struct qaa_plan_choice {
    int32_t balance;
    int32_t passengers;
    int32_t tiles;
} qaa_plan_choice;

/* The choice in effect for (n, dtype) with a uint8 table: recorded, else
 * the built-in default (balance for two sets, passengers for three or
 * more, the tiles measured fastest for n). */
qaa_status qaa_plan_get(int32_t n, qaa_dtype dtype, qaa_plan_choice *out);

/* Record a choice for (n, dtype) (balance and passengers 0 or 1, tiles 0, 1
 * or 2); NULL restores the default.  Affects calls made after it returns. */
qaa_status qaa_plan_set(int32_t n, qaa_dtype dtype, const qaa_plan_choice *choice);

/*
 * Autotuner: time `steps` steps (step size 0.01) of every candidate choice
 * (balance x passengers x tiles, those that apply) for the scratch state's
 * (n, dtype) on the stream, record the fastest with qaa_plan_set, and
 * return it (*best, *ms_per_step may be NULL).  If the environment variable
 * QAA_AUTOTUNE_CACHE names a file, every recorded choice is then written
 * there (as qaa_plan_save), and a later process reads that file before its
 * first plan lookup, so tuned plans persist across runs; qaa_evolve_batch
 * follows the recorded balance and passengers for each n.  The scratch
 * state's amplitudes are overwritten; its energy table must have been
 * computed.  SYNCHRONOUS.
 */
qaa_status qaa_autotune(const qaa_state *scratch, int64_t steps, qaa_plan_choice *best, double *ms_per_step,
                        void *stream);

/* Write every recorded plan choice to a text file (one line per (n, dtype):
 * "n dtype balance passengers tiles"), or record the choices a file holds
 * (*count: lines recorded; malformed lines are skipped).  Host only.
 * QAA_ERR_INVALID_ARG if the file cannot be written / read. */
qaa_status qaa_plan_save(const char *path);
qaa_status qaa_plan_load(const char *path, int32_t *count);

/*
 * Diagnostic: the host half of qaa_spectrum on a given tridiagonal matrix
 * (diagonal alpha[0..m), off-diagonal beta[0..m-1), and beta[m-1] the
 * residual coefficient of the last Lanczos step): the k lowest levels and,
 * if bounds is not NULL, their residual norms, exactly as qaa_spectrum
 * returns them.  Host memory only; exists so that host-side tests can
 * check the eigenvalue and merging logic without a device.
 */
qaa_status qaa_debug_tridiag_levels(const double *alpha, const double *beta, int32_t m, int32_t k, double *evals,
                                    double *bounds);

/*
 * Diagnostic: the pass descriptors qaa_evolve_range would launch for an
 * n-qubit state (energies up to emax) over steps k0..k1-1 of `steps`
 * under schedule `sched` (NULL: linear).
 *   tile_bits : 0 for the library's own plan; otherwise the plan the same
 *               planner makes for base tiles of that many qubits (complex64
 *               9..13, complex128 8..12) and, where the plan choice asks for
 *               wider tiles (qaa_plan_choice.tiles, honoured from
 *               n >= tile_bits + 9), wide tiles one qubit larger.  Smaller
 *               tiles give the plan shapes of large n (three to five qubit
 *               sets, wide top sets) already at small n, so host-side
 *               replays can check them against a reference; no kernel runs
 *               such tiles.  QAA_ERR_INVALID_ARG outside that range.
 * Writes up to `capacity` descriptors of *desc_bytes bytes each into the
 * host buffer `out` (may be NULL to query the count) and the total number
 * into *count (0 when the whole state is one workgroup tile).  The record
 * layout is the library's internal pass descriptor and may change between
 * versions; it exists so that host-side tests can replay the index maps.
 */
qaa_status qaa_debug_pass_descs(int32_t n, qaa_dtype dtype, int32_t emax, const qaa_schedule *sched, double T,
                                int64_t steps, int64_t k0, int64_t k1, int32_t tile_bits, void *out,
                                int32_t capacity, int32_t *count, int32_t *desc_bytes);

/* ---------------------------------------------------------------------
 * Kernel timing (tracing).
 * ------------------------------------------------------------------- */

/*
 * While enabled (on != 0), every pass-kernel launch made by the calling
 * process carries a start and a stop HIP event on its own dispatch
 * (hipExtLaunchKernel: the events time that kernel alone, with no event
 * commands between launches).  Enabling adds one event pair per launch; it
 * does not change results.  Disabled by default.
 */
qaa_status qaa_profile_enable(int32_t on);

typedef struct qaa_profile {
    int64_t launches;       /* pass launches recorded since the last reset */
    double kernel_ms;       /* sum of their event-measured durations */
    double min_ms, max_ms;  /* shortest / longest single launch */
    double alg_bytes;       /* algorithmic HBM bytes of those launches:
                               2^n * (2 * sizeof(amplitude) + sizeof(energy)
                               if the pass applies the phase) each */
} qaa_profile;

/* SYNCHRONOUS: waits for the recorded events, fills *out, and clears the
 * record when reset != 0. */
qaa_status qaa_profile_read(qaa_profile *out, int32_t reset);

/* ---------------------------------------------------------------------
 * Errors and version.
 * ------------------------------------------------------------------- */

const char *qaa_status_str(qaa_status s);  /* static string, never NULL */
const char *qaa_last_error(void);          /* thread-local; "" if none */
int32_t qaa_version(void);                 /* major*10000 + minor*100 + patch */

#ifdef __cplusplus
}
#endif

#endif /* QAA_H */
