// qaa_api.hip -- host runtime behind include/qaa.h: argument validation,
// instance encoding, the pass planner, the per-step pass sequence and the
// per-device scratch used by reductions.
#include "qaa.h"
#include "qaa_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

using namespace qaa;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
namespace {

// A roctx range over the enclosing scope: host-side time of an API call or
// of one pass's launch, named in rocprofv3 traces taken with
// --marker-trace (the calls cost a few tens of nanoseconds when no tool
// listens).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    TraceRange(const char *fmt, int a, int b, long long c, long long d)
    {
        char buf[96];
        std::snprintf(buf, sizeof buf, fmt, a, b, c, d);
        roctxRangePushA(buf);
    }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace

namespace {

thread_local std::string g_last_error;

qaa_status fail(qaa_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

qaa_status ok()
{
    g_last_error.clear();
    return QAA_OK;
}

}  // namespace

// Shared with the server translation unit (same thread-local message).
qaa_status qaa::set_error(qaa_status st, const char *msg)
{
    if (st == QAA_OK)
        g_last_error.clear();
    else
        g_last_error = msg ? msg : "";
    return st;
}

namespace {

#define QAA_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(QAA_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

// ---------------------------------------------------------------------------
// Per-device context: the side stream that batched small states run on.
// Reductions (energy-table statistics, observables) take their scratch per
// call from the stream-ordered allocator, so concurrent calls on different
// streams share nothing and need no lock.
// ---------------------------------------------------------------------------
struct DeviceCtx {
    std::mutex mu;                          // enqueueing on `side`
    bool ready = false;
    hipStream_t side = nullptr;             // second stream for batched small states
    // streams for the second and later launch groups of a batch (see
    // run_batch_passes); created on first use, default priority
    std::mutex group_mu;
    std::vector<hipStream_t> group;
};

std::mutex g_dev_mu;
std::map<int, std::unique_ptr<DeviceCtx>> g_devs;

qaa_status device_ctx(DeviceCtx **out)
{
    int dev = 0;
    QAA_HIP(hipGetDevice(&dev));
    DeviceCtx *ctx;
    {
        std::lock_guard<std::mutex> lk(g_dev_mu);
        auto &p = g_devs[dev];
        if (!p) p.reset(new DeviceCtx());
        ctx = p.get();
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->ready) {
        QAA_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
        ctx->ready = true;
    }
    *out = ctx;
    return QAA_OK;
}

// Per-call device scratch from the stream-ordered allocator, released in
// stream order when the holder goes out of scope (every return path).
struct StreamScratch {
    void *p = nullptr;
    hipStream_t s = nullptr;
    ~StreamScratch()
    {
        if (p) (void)hipFreeAsync(p, s);
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// Instances
// ---------------------------------------------------------------------------
struct qaa_instance {
    int32_t n = 0;
    int32_t m = 0;
    std::vector<int32_t> lits;
    std::vector<ClauseRec> recs;
    std::mutex mu;
    std::map<int, ClauseRec *> dev_recs;   // device copy per device
    int32_t e_min = -1, e_max = -1;
    int64_t degeneracy = -1;
};

namespace {

// Encode one clause: violated iff every literal is false, i.e. iff
// x_v = 0 for each positive literal and x_v = 1 for each negated one
// (Sec. 2.2).  mask = the three variable bits, pat = the negated ones; the
// record splits the test at bit 5 (see ClauseRec).
ClauseRec encode_clause(const int32_t *c)
{
    uint64_t mask = 0, pat = 0;
    for (int j = 0; j < 3; ++j) {
        const int32_t v = c[j] > 0 ? c[j] : -c[j];
        const uint64_t bit = 1ull << (v - 1);
        mask |= bit;
        if (c[j] < 0) pat |= bit;
    }
    ClauseRec r;
    r.mhi = (uint32_t)(mask >> 5);
    r.phi = (uint32_t)(pat >> 5);
    r.low = 0;
    for (uint32_t i = 0; i < 32; ++i)
        if ((i & (uint32_t)(mask & 31)) == (uint32_t)(pat & 31)) r.low |= 1u << i;
    r.pad_ = 0;
    return r;
}

}  // namespace

extern "C" qaa_status qaa_instance_create(int32_t n, int32_t m, const int32_t *lits, qaa_instance **out)
{
    if (!out) return fail(QAA_ERR_INVALID_ARG, "qaa_instance_create: out is NULL");
    *out = nullptr;
    if (n < 1 || n > QAA_MAX_QUBITS)
        return fail(QAA_ERR_INVALID_ARG, "qaa_instance_create: n=%d outside [1, %d]", n, QAA_MAX_QUBITS);
    if (m < 0 || m > 65535) return fail(QAA_ERR_INVALID_ARG, "qaa_instance_create: m=%d outside [0, 65535]", m);
    if (m > 0 && !lits) return fail(QAA_ERR_INVALID_ARG, "qaa_instance_create: lits is NULL with m=%d", m);
    for (int c = 0; c < m; ++c) {
        int32_t vs[3];
        for (int j = 0; j < 3; ++j) {
            const int32_t l = lits[3 * c + j];
            const int32_t v = l > 0 ? l : -l;
            if (l == 0 || v > n)
                return fail(QAA_ERR_INVALID_ARG, "qaa_instance_create: clause %d literal %d out of range for n=%d", c,
                            l, n);
            vs[j] = v;
        }
        if (vs[0] == vs[1] || vs[0] == vs[2] || vs[1] == vs[2])
            return fail(QAA_ERR_INVALID_ARG, "qaa_instance_create: clause %d repeats a variable", c);
    }
    qaa_instance *inst = new (std::nothrow) qaa_instance();
    if (!inst) return fail(QAA_ERR_OUT_OF_MEMORY, "qaa_instance_create: host allocation failed");
    inst->n = n;
    inst->m = m;
    inst->lits.assign(lits, lits + 3 * (size_t)m);
    inst->recs.reserve(m);
    for (int c = 0; c < m; ++c) inst->recs.push_back(encode_clause(lits + 3 * c));
    *out = inst;
    return ok();
}

extern "C" void qaa_instance_destroy(qaa_instance *inst)
{
    if (!inst) return;
    int cur = 0;
    const bool have_dev = hipGetDevice(&cur) == hipSuccess;
    for (auto &kv : inst->dev_recs) {
        if (!kv.second) continue;
        if (have_dev) (void)hipSetDevice(kv.first);
        (void)hipFree(kv.second);
    }
    if (have_dev) (void)hipSetDevice(cur);
    delete inst;
}

extern "C" qaa_status qaa_instance_info(const qaa_instance *inst, int32_t *n, int32_t *m, int32_t *e_min,
                                        int32_t *e_max, int64_t *degeneracy)
{
    if (!inst) return fail(QAA_ERR_INVALID_ARG, "qaa_instance_info: inst is NULL");
    if (n) *n = inst->n;
    if (m) *m = inst->m;
    if (e_min) *e_min = inst->e_min;
    if (e_max) *e_max = inst->e_max;
    if (degeneracy) *degeneracy = inst->degeneracy;
    return ok();
}

extern "C" qaa_status qaa_debug_energy_block(const qaa_instance *inst, uint64_t z0, int32_t *out32)
{
    if (!inst || !out32) return fail(QAA_ERR_INVALID_ARG, "qaa_debug_energy_block: NULL argument");
    if (z0 % 32 || (inst->n >= 5 && z0 >= (1ull << inst->n)) || (inst->n < 5 && z0 != 0))
        return fail(QAA_ERR_INVALID_ARG, "qaa_debug_energy_block: z0 must be a multiple of 32 below 2^n");
    uint32_t e[32];
    energy_block_host(inst->recs.data(), inst->m, (uint32_t)(z0 >> 5), e);
    for (int i = 0; i < 32; ++i) out32[i] = (int32_t)e[i];
    return ok();
}

// ---------------------------------------------------------------------------
// Energy table
// ---------------------------------------------------------------------------
namespace {

// The instance's clause records on the calling thread's device (uploaded
// on first use, kept until the instance is destroyed).
qaa_status device_clauses(qaa_instance *inst, ClauseRec **out, const char *who)
{
    int dev = 0;
    QAA_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(inst->mu);
    auto it = inst->dev_recs.find(dev);
    if (it != inst->dev_recs.end()) {
        *out = it->second;
        return QAA_OK;
    }
    ClauseRec *recs = nullptr;
    const size_t bytes = sizeof(ClauseRec) * std::max<size_t>(1, inst->recs.size());
    QAA_HIP(hipMalloc(reinterpret_cast<void **>(&recs), bytes));
    if (!inst->recs.empty()) {
        hipError_t e = hipMemcpy(recs, inst->recs.data(), sizeof(ClauseRec) * inst->recs.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(recs);
            return fail(QAA_ERR_DEVICE, "%s: clause upload failed: %s", who, hipGetErrorString(e));
        }
    }
    inst->dev_recs[dev] = recs;
    *out = recs;
    return QAA_OK;
}

}  // namespace

extern "C" qaa_status qaa_energy_stats(qaa_instance *inst, void *stream)
{
    TraceRange trace_range("qaa_energy_stats");
    const char *who = "qaa_energy_stats";
    if (!inst) return fail(QAA_ERR_INVALID_ARG, "%s: inst is NULL", who);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ClauseRec *recs = nullptr;
    qaa_status r = device_clauses(inst, &recs, who);
    if (r != QAA_OK) return r;
    // the statistics of qaa_energy_table, with no table written: E_min and
    // E_max in one pass, then the number of z at E_min in a second
    StreamScratch scr;
    scr.s = s;
    QAA_HIP(hipMallocAsync(&scr.p, 64, s));
    uint32_t *stats = reinterpret_cast<uint32_t *>(scr.p);
    unsigned long long *count = reinterpret_cast<unsigned long long *>(stats + 4);
    uint32_t h[4] = {0, 0, 0, 0};
    bool wide = false;
    for (int pass = 0; pass < 2; ++pass) {
        QAA_HIP(launch_zero_u64(reinterpret_cast<unsigned long long *>(stats), 3, s));
        QAA_HIP(launch_energy(recs, inst->m, inst->n, nullptr, QAA_E_U16, wide, stats, 0, nullptr, s));
        QAA_HIP(hipMemcpyAsync(h, stats, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        QAA_HIP(hipStreamSynchronize(s));
        if (!h[3]) break;
        wide = true;              // some count passed 255: count again with 16 planes
    }
    const uint32_t emin = ~h[0], emax = h[1];
    QAA_HIP(launch_zero_u64(reinterpret_cast<unsigned long long *>(stats), 3, s));
    QAA_HIP(launch_energy(recs, inst->m, inst->n, nullptr, QAA_E_U16, wide, stats, (int)emin, count, s));
    unsigned long long hc = 0;
    QAA_HIP(hipMemcpyAsync(&hc, count, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    QAA_HIP(hipStreamSynchronize(s));
    inst->e_min = (int32_t)emin;
    inst->e_max = (int32_t)emax;
    inst->degeneracy = (int64_t)hc;
    return ok();
}

extern "C" qaa_status qaa_energy_table(qaa_instance *inst, void *d_table, qaa_etype etype, void *stream)
{
    TraceRange trace_range("qaa_energy_table");
    if (!inst) return fail(QAA_ERR_INVALID_ARG, "qaa_energy_table: inst is NULL");
    if (!d_table) return fail(QAA_ERR_INVALID_ARG, "qaa_energy_table: d_table is NULL");
    if (reinterpret_cast<uintptr_t>(d_table) % 16)
        return fail(QAA_ERR_INVALID_ARG, "qaa_energy_table: d_table must be 16-byte aligned");
    if (etype != QAA_E_U8 && etype != QAA_E_U16)
        return fail(QAA_ERR_INVALID_ARG, "qaa_energy_table: bad etype %d", (int)etype);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ClauseRec *recs = nullptr;
    qaa_status rc = device_clauses(inst, &recs, "qaa_energy_table");
    if (rc != QAA_OK) return rc;

    // stats[0] = ~E_min (max of complements), stats[1] = E_max, stats[2] =
    // uint8 overflow flag; count = number of z at E_min
    StreamScratch scr;
    scr.s = s;
    QAA_HIP(hipMallocAsync(&scr.p, 64, s));
    uint32_t *stats = reinterpret_cast<uint32_t *>(scr.p);
    unsigned long long *count = reinterpret_cast<unsigned long long *>(stats + 4);
    QAA_HIP(launch_zero_u64(reinterpret_cast<unsigned long long *>(stats), 3, s));
    QAA_HIP(launch_energy(recs, inst->m, inst->n, d_table, (int)etype, false, stats, 0, nullptr, s));
    uint32_t h[4] = {0, 0, 0, 0};
    QAA_HIP(hipMemcpyAsync(h, stats, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    QAA_HIP(hipStreamSynchronize(s));
    if (h[3] && etype == QAA_E_U16) {
        // some count passed 255: count again with 16 planes
        QAA_HIP(launch_zero_u64(reinterpret_cast<unsigned long long *>(stats), 3, s));
        QAA_HIP(launch_energy(recs, inst->m, inst->n, d_table, (int)etype, true, stats, 0, nullptr, s));
        QAA_HIP(hipMemcpyAsync(h, stats, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        QAA_HIP(hipStreamSynchronize(s));
    }
    const uint32_t emin = ~h[0], emax = h[1];
    if (etype == QAA_E_U8 && (h[2] || h[3] || emax > 255))
        return fail(QAA_ERR_UNSUPPORTED, "qaa_energy_table: E_max > 255 does not fit uint8; use QAA_E_U16");
    QAA_HIP(launch_count_equal(d_table, (int)etype, inst->n, (int)emin, count, s));
    unsigned long long hc = 0;
    QAA_HIP(hipMemcpyAsync(&hc, count, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    QAA_HIP(hipStreamSynchronize(s));
    inst->e_min = (int32_t)emin;
    inst->e_max = (int32_t)emax;
    inst->degeneracy = (int64_t)hc;
    return ok();
}

// ---------------------------------------------------------------------------
// State initialisation
// ---------------------------------------------------------------------------
namespace {

qaa_status check_state_amp(const qaa_state *st, const char *who)
{
    if (!st) return fail(QAA_ERR_INVALID_ARG, "%s: state is NULL", who);
    if (!st->inst) return fail(QAA_ERR_INVALID_ARG, "%s: state has no instance", who);
    if (!st->amp) return fail(QAA_ERR_INVALID_ARG, "%s: state has no amplitude buffer", who);
    if (st->dtype != QAA_C64 && st->dtype != QAA_C128)
        return fail(QAA_ERR_INVALID_ARG, "%s: bad dtype %d", who, (int)st->dtype);
    if (reinterpret_cast<uintptr_t>(st->amp) % 16)
        return fail(QAA_ERR_INVALID_ARG, "%s: amplitudes must be 16-byte aligned", who);
    return QAA_OK;
}

// A state with a table, or without one (recompute mode: the energies are
// scored from the clause records where they are needed; etype is then the
// width they are held in).  Either way the energy statistics must be known.
qaa_status check_state_table(const qaa_state *st, const char *who, bool allow_recompute = true)
{
    qaa_status r = check_state_amp(st, who);
    if (r != QAA_OK) return r;
    if (!st->table && !allow_recompute)
        return fail(QAA_ERR_UNSUPPORTED, "%s: needs an energy table (recompute mode is not offered here)", who);
    if (st->etype != QAA_E_U8 && st->etype != QAA_E_U16)
        return fail(QAA_ERR_INVALID_ARG, "%s: bad etype %d", who, (int)st->etype);
    if (reinterpret_cast<uintptr_t>(st->table) % 16)
        return fail(QAA_ERR_INVALID_ARG, "%s: energy table must be 16-byte aligned", who);
    if (st->inst->e_max < 0)
        return fail(QAA_ERR_NOT_READY, "%s: neither qaa_energy_table nor qaa_energy_stats has run for this instance",
                    who);
    return QAA_OK;
}

}  // namespace

extern "C" qaa_status qaa_state_init_uniform(const qaa_state *st, void *stream)
{
    qaa_status r = check_state_amp(st, "qaa_state_init_uniform");
    if (r != QAA_OK) return r;
    QAA_HIP(launch_init_uniform(st->amp, (int)st->dtype, st->inst->n, reinterpret_cast<hipStream_t>(stream)));
    return ok();
}

extern "C" qaa_status qaa_state_init_basis(const qaa_state *st, uint64_t z0, void *stream)
{
    qaa_status r = check_state_amp(st, "qaa_state_init_basis");
    if (r != QAA_OK) return r;
    if (z0 >> st->inst->n) return fail(QAA_ERR_INVALID_ARG, "qaa_state_init_basis: z0 >= 2^n");
    QAA_HIP(launch_init_basis(st->amp, (int)st->dtype, st->inst->n, z0, reinterpret_cast<hipStream_t>(stream)));
    return ok();
}

// ---------------------------------------------------------------------------
// Planner
// ---------------------------------------------------------------------------
namespace {

// Which XCD takes which tiles of a pass (PassDesc::xcd_map, pass_kernel).
// Over a state larger than the last-level cache: when the amplitude-index
// bits of byte-address bits 10..12 are tile-number bits, those name the
// XCD (each XCD streams its own 1 KiB-interleaved eighth of memory; n = 28
// copy probe, 256-, 512- and 1024-byte runs: 5.8-6.0 TB/s, against
// 5.0-5.3 with those bits at address bits 11..13 and 5.3-6.0 in the plain
// order); when they lie inside the tile (set 0), the grid's top bits do
// (64 KiB tiles: 5.0 -> 5.6 TB/s).  n = 28 passes: middle 0.82 -> 0.77 ms,
// set-0 turns 0.81 -> 0.80 ms.  The persistent passes (top set) and
// smaller states run better in the plain order (n = 28 top turns: 0.96 ms
// plain, 0.98-1.00 ms with the XCD on tile bits 1..6; n = 22: 4 % per
// step, its passes reusing what the previous pass left in the L2s).
int xcd_arrangement(const PassDesc &d, int n, int dtype)
{
    if (n < 26 || d.persist) return 0;
    const int xb = dtype == QAA_C64 ? 7 : 6;          // amplitude bit of byte-address bit 10
    const uint64_t three = 7ull << xb;
    if ((d.rest_mask & three) != three) return 1;
    return 2 + __builtin_popcountll(d.rest_mask & ((1ull << xb) - 1));
}

struct SetPlan {
    int tb = 0;                  // tile bits of this set's passes
    std::vector<int> tile;       // physical bits of the tile, ascending (size tb)
    std::vector<int> rot_local;  // tile-local indices of the rotated qubits
};

struct Plan {
    bool resident = false;
    int tile_bits = 0, reg_bits = 0;    // set 0's tile bits; register bits of every set
    std::vector<SetPlan> sets;
};

// Plan choices per (n, dtype).
//   balance: the top set takes set 0's highest qubits until it rotates as
//     many as it can hold.
//   passengers: with three or more sets, the passenger qubits (except
//     complex64's bit 0) rotate in the set-1 passes (see make_plan).
//   tiles (complex64 with a uint8 table, n >= 22 only): 0 = every set in
//     2^13-amplitude tiles; 1 = the top set's passes in 2^14-amplitude tiles
//     (7 or more passenger bits at n = 28: 1 KiB runs of state, 128-byte
//     runs of the table); 2 = every set in 2^14-amplitude tiles with the
//     high qubits split evenly over the sets above set 0.
// Defaults, measured per n (complex64): with two sets the turn over set 0
// otherwise rotates up to 13 qubits twice against a handful in the other
// turn, and balancing gains up to 6 % (n = 20); with three sets the top
// set's shorter contiguous runs cost as much as set 0 saves (n = 26 and 28
// lose about 1 %), so balancing is off there, while moving the passengers
// is 3 % faster at n = 28.  qaa_plan_set / qaa_autotune record other
// choices; the environment variables QAA_PLAN_BALANCE, QAA_PLAN_PASSENGERS
// (0 or 1) and QAA_PLAN_TILES (0, 1 or 2) override all.
struct PlanChoice {
    int balance, passengers, tiles;     // -1: the default for the plan's shape
};

std::mutex g_plan_mu;
std::map<std::pair<int, int>, PlanChoice> g_plan_choice;

// Default tiles per n (complex64, measured: ms per step at T = 50, 5000-step
// schedule).  Wide tiles pay where they remove a whole qubit set: n = 22
// runs two sets instead of three with a wide top set (0.063 -> 0.045 ms),
// n = 23 two sets with every set wide (0.091 -> 0.081 ms), n = 30 three
// instead of four with a wide top set (10.4 -> 8.0 ms), n = 31, 32 three
// with every set wide (20.7 -> 18.0 ms, 41.3 -> 38.5 ms).  Where the set
// count does not change, the 2^14 tiles' single workgroup per CU costs
// more than the longer runs gain (n = 28: 1.71 ms, 1.76 ms with the top
// set wide, 1.98 ms all wide; n = 24..29 likewise within 2 %).
int default_tiles(int n, int dtype)
{
    if (dtype != 0) return 0;
    if (n == 22 || n == 30) return 1;
    if (n == 23 || n == 31 || n == 32) return 2;
    return 0;
}
PlanChoice default_plan_choice(int sets) { return PlanChoice{sets == 2 ? 1 : 0, sets >= 3 ? 1 : 0, 0}; }

// With three sets, how many of the highest qubits set 1 takes (0: none, the
// top set takes them).  Set 1 then holds the lowest of the high qubits and
// the `spread` highest ones, the top set the run between.  Measured on
// complex64 (ms per step; set 1 takes 2..5 of the highest qubits): n = 30
// 7.74 -> 7.52 / 7.62 / 7.33 / 7.54, n = 31 18.06 -> 21.97 / 17.57 / 16.88 /
// 16.73 (the top set's tiles then gather runs from fewer, nearer rows, and
// set 1's passes, which take the spread qubits, lose less than the top set's
// gain); n = 28 and 29 within 1 % either way, so 4 from n = 30 on.
// QAA_PLAN_SPREAD (a digit, read at every call) overrides it for every n.
int plan_spread(int n, int dtype, int high_sets)
{
    if (const char *e = std::getenv("QAA_PLAN_SPREAD"))
        return (e[0] >= '0' && e[0] <= '9') ? e[0] - '0' : 0;
    return (dtype == 0 && n >= 30 && high_sets == 2) ? 4 : 0;
}

int env_knob(const char *name)
{
    const char *e = std::getenv(name);
    return e ? (e[0] >= '0' && e[0] <= '9' ? e[0] - '0' : 0) : -1;
}

// Plan-choice files (qaa_plan_save / qaa_plan_load, and the autotuner's
// cache named by QAA_AUTOTUNE_CACHE): one line per (n, dtype),
//     n dtype balance passengers tiles
// '#' starts a comment.  Reading records every well-formed line and
// skips the rest; returns the number recorded (-1: the file cannot be read).
int read_plan_file(const char *path)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return -1;
    char line[256];
    int count = 0;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        int n, dt, b, q, t;
        if (std::sscanf(line, "%d %d %d %d %d", &n, &dt, &b, &q, &t) != 5) continue;
        if (n < 1 || n > QAA_MAX_QUBITS || (dt != 0 && dt != 1) || (b != 0 && b != 1) || (q != 0 && q != 1) ||
            t < 0 || t > 2)
            continue;
        g_plan_choice[{n, dt}] = PlanChoice{b, q, t};
        ++count;
    }
    std::fclose(f);
    return count;
}

// Writes every recorded choice (caller holds g_plan_mu); false on failure.
bool write_plan_file(const char *path)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "# qaa plan choices: n dtype balance passengers tiles\n");
    for (const auto &kv : g_plan_choice) {
        const PlanChoice &c = kv.second;
        if (c.balance < 0 || c.passengers < 0 || c.tiles < 0) continue;
        std::fprintf(f, "%d %d %d %d %d\n", kv.first.first, kv.first.second, c.balance, c.passengers, c.tiles);
    }
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

// The autotuner's cache file, read once before the first plan lookup.
const char *autotune_cache_path()
{
    static const char *p = std::getenv("QAA_AUTOTUNE_CACHE");
    return p && p[0] ? p : nullptr;
}

void load_autotune_cache_once()
{
    static std::once_flag once;
    std::call_once(once, [] {
        if (const char *p = autotune_cache_path()) {
            std::lock_guard<std::mutex> lk(g_plan_mu);
            (void)read_plan_file(p);
        }
    });
}

// The recorded (or environment-forced) choice for (n, dtype); fields the
// caller did not fix are -1.
PlanChoice recorded_choice(int n, int dtype)
{
    load_autotune_cache_once();
    PlanChoice c{-1, -1, -1};
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plan_choice.find({n, dtype});
        if (it != g_plan_choice.end()) c = it->second;
    }
    static const int force_balance = env_knob("QAA_PLAN_BALANCE");
    static const int force_passengers = env_knob("QAA_PLAN_PASSENGERS");
    static const int force_tiles = env_knob("QAA_PLAN_TILES");
    if (force_balance >= 0) c.balance = force_balance ? 1 : 0;
    if (force_passengers >= 0) c.passengers = force_passengers ? 1 : 0;
    if (force_tiles >= 0) c.tiles = std::min(force_tiles, 2);
    return c;
}

// Whether 2^14-amplitude tiles can run this state: complex64 with a uint8
// table (tile, padding, phase table and energies fill 154 KiB of the 160 KiB
// of LDS), and n >= 22 (base tile + 9) so that plans below that keep their
// two sets of base tiles.
bool wide_tiles_ok(int n, int dtype, int etype, int base = kPassTileBits[0])
{
    return dtype == 0 && etype == 0 && n >= base + 9;
}

// The plan for n qubits.  etype matters only for the tile choice (wide
// tiles need a uint8 table); tile_override: 0 for the library's tile shape,
// otherwise a smaller base tile of that many bits (and a wide tile one bit
// larger), for host-side replay of the same plan shapes at small n
// (qaa_debug_pass_descs only: no kernel is built for such tiles).
Plan make_plan(int n, int dtype, int etype, int tile_override = 0, PlanChoice *used = nullptr)
{
    Plan p;
    if (n <= kResRegBits[dtype] + kResThrBits) {
        p.resident = true;
        return p;
    }
    const int base = tile_override ? tile_override : kPassTileBits[dtype];
    const int pas = kPassengerBits[dtype];
    PlanChoice c = recorded_choice(n, dtype);
    const int wide = tile_override ? tile_override + 1 : kWideTileBits;
    int tiles = c.tiles >= 0 ? c.tiles : (tile_override ? 0 : default_tiles(n, dtype));
    if (!wide_tiles_ok(n, dtype, etype, base)) tiles = 0;
    const int tb0 = tiles == 2 ? wide : base;
    const int tb_mid = tiles == 2 ? wide : base;
    const int tb_top = tiles >= 1 ? wide : base;
    const int q_mid = tb_mid - pas, q_top = tb_top - pas;   // qubits a high set can rotate
    // Qubits above set 0's tile go to the sets above it, ascending.  The
    // lower high sets take q_mid each and the top set the rest (tiles 0,
    // 1); with tiles 2 they are split evenly, the top set taking the
    // smaller share (its passes gather from the whole state, so its
    // passenger runs matter most).
    const int H = n - tb0;
    int h = 1;
    while ((h - 1) * q_mid + q_top < H) ++h;
    std::vector<int> sizes(h, 0);
    if (tiles == 2) {
        for (int j = 0; j < h; ++j) sizes[j] = H / h + (j < H % h ? 1 : 0);
    } else {
        int left = H;
        for (int j = 0; j < h - 1; ++j) {
            sizes[j] = std::min(q_mid, left);
            left -= sizes[j];
        }
        sizes[h - 1] = left;
    }
    std::vector<std::vector<int>> hi_sets;
    for (int j = 0, b = tb0; j < h; b += sizes[j], ++j) {
        std::vector<int> r;
        for (int q = b; q < b + sizes[j]; ++q) r.push_back(q);
        hi_sets.push_back(r);
    }
    const int spread = plan_spread(n, dtype, h);
    if (h == 2 && spread > 0 && spread < sizes[0]) {
        // set 1: the lowest sizes[0] - spread high qubits and the spread
        // highest; the top set: the run of sizes[1] qubits between them
        const int lo = tb0 + sizes[0] - spread;
        hi_sets[0].clear();
        hi_sets[1].clear();
        for (int q = tb0; q < lo; ++q) hi_sets[0].push_back(q);
        for (int q = lo; q < lo + sizes[1]; ++q) hi_sets[1].push_back(q);
        for (int q = lo + sizes[1]; q < n; ++q) hi_sets[0].push_back(q);
    }
    const PlanChoice def = default_plan_choice(1 + h);
    const int balance = c.balance >= 0 ? c.balance : def.balance;
    const int passengers = c.passengers >= 0 ? c.passengers : def.passengers;
    if (used) *used = PlanChoice{balance, passengers, tiles};
    p.tile_bits = tb0;
    // two sets of 2^13-amplitude tiles (complex64, n = 14..21): 4 register
    // bits, 512 threads per tile (n = 18: 14.9 -> 12.9 us per pass, n = 20:
    // 17.1 -> 15.9 us); replays with smaller tiles keep 5
    p.reg_bits = (dtype == 0 && h == 1 && tb0 == kPassTileBits[0] && tb_top == tb0) ? kSmallPlanRegBits
                                                                                     : kPassRegBits[dtype];
    // The top set takes set 0's highest qubits until it rotates q_top of
    // them (set 0 keeps at least the passenger bits, which only it
    // rotates): the turn passes over set 0 and over the top set then rotate
    // comparable numbers of qubits.
    int moved = 0;
    if (balance) moved = std::min(q_top - (int)hi_sets.back().size(), tb0 - pas);
    for (int j = 0; j < moved; ++j) hi_sets.back().push_back(tb0 - 1 - j);
    SetPlan s0;
    s0.tb = tb0;
    for (int b = 0; b < tb0; ++b) {
        s0.tile.push_back(b);
        if (b < tb0 - moved) s0.rot_local.push_back(b);
    }
    p.sets.push_back(s0);
    for (size_t j = 0; j < hi_sets.size(); ++j) {
        std::vector<int> r = hi_sets[j];
        std::sort(r.begin(), r.end());
        SetPlan st;
        st.tb = j + 1 == hi_sets.size() ? tb_top : tb_mid;
        const int extra = st.tb - (int)r.size();  // low passenger bits
        for (int b = 0; b < extra; ++b) st.tile.push_back(b);
        for (int b : r) st.tile.push_back(b);
        std::sort(st.tile.begin(), st.tile.end());
        for (int b = 0; b < st.tb; ++b)
            if (std::find(r.begin(), r.end(), st.tile[b]) != r.end()) st.rot_local.push_back(b);
        p.sets.push_back(st);
    }
    // With three or more sets, every step visits set 1 once, next to set 0
    // and with no phase in between, and set 1's tile holds the passenger
    // bits.  Those qubits' rotations move from set 0 to set 1: the turn
    // over set 0 then rotates 8 qubits twice instead of 13, the middle
    // passes (HBM-bound, with VALU to spare) 13 instead of 8.
    if (p.sets.size() >= 3 && passengers) {
        // (complex64: bit 0 stays with set 0; it is a register bit of every
        // group, so it costs set 0 no extra exchange)
        const int lo = dtype == 0 ? 1 : 0;
        std::vector<int> keep;
        for (int j : p.sets[0].rot_local)
            if (j < lo || j >= pas) keep.push_back(j);
        p.sets[0].rot_local = keep;
        std::vector<int> r1;
        for (int j = lo; j < pas; ++j) r1.push_back(j);     // tile-local = physical for passengers
        for (int j : p.sets[1].rot_local) r1.push_back(j);
        p.sets[1].rot_local = r1;
    }
    return p;
}

// The plan under an explicit choice, whatever is recorded for (n, dtype).
Plan make_plan_with(int n, int dtype, int etype, const PlanChoice &c)
{
    PlanChoice saved{-1, -1, -1};
    bool had = false;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plan_choice.find({n, dtype});
        if (it != g_plan_choice.end()) {
            saved = it->second;
            had = true;
        }
        g_plan_choice[{n, dtype}] = c;
    }
    Plan p = make_plan(n, dtype, etype);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (had)
        g_plan_choice[{n, dtype}] = saved;
    else
        g_plan_choice.erase({n, dtype});
    return p;
}

// Register groups for one qubit set.  The set's rotated tile-local bits are
// split, highest first, into groups that fill the rb register bits of a
// residency; bits a group does not rotate are fillers taken from the top of
// the tile.  For complex64 (vw = 2) register bit 0 is tile bit 0 in every
// group, so register pairs are adjacent in memory; tile bit 0 itself is
// rotated (if it belongs to the set) only in the first group.
struct Group {
    std::vector<int> bits;   // bits[i] = tile bit of register bit i (size rb)
    uint32_t rot;            // register bits this group rotates
};

bool contains(const std::vector<int> &v, int b) { return std::find(v.begin(), v.end(), b) != v.end(); }

std::vector<Group> make_groups(const std::vector<int> &rot, int tb, int rb, int vw)
{
    std::vector<int> members;
    bool rot0 = false;
    for (int b : rot) {
        if (vw == 2 && b == 0)
            rot0 = true;
        else
            members.push_back(b);
    }
    std::sort(members.rbegin(), members.rend());
    const int cap = vw == 2 ? rb - 1 : rb;
    // the first group must be able to talk to HBM (see io_capable): it takes
    // only members above the low bits, topped up with high filler bits
    const int lo_end = vw == 2 ? 5 : 4;
    size_t first = 0;
    while (first < members.size() && (int)first < cap && members[first] >= lo_end) ++first;
    std::vector<size_t> cuts{0};
    if (first > 0 || members.empty()) cuts.push_back(first);
    for (size_t i = cuts.back(); i < members.size();) {
        i = std::min(members.size(), i + cap);
        cuts.push_back(i);
    }
    std::vector<Group> gs;
    for (size_t c = 0; c + 1 < cuts.size() || (gs.empty() && rot0); ++c) {
        const size_t lo = c + 1 < cuts.size() ? cuts[c] : 0, hi = c + 1 < cuts.size() ? cuts[c + 1] : 0;
        Group g;
        g.rot = 0;
        if (vw == 2) {
            g.bits.push_back(0);
            if (rot0 && gs.empty()) g.rot |= 1u;
        }
        for (size_t j = lo; j < hi; ++j) {
            g.rot |= 1u << g.bits.size();
            g.bits.push_back(members[j]);
        }
        for (int b = tb - 1; b >= 0 && (int)g.bits.size() < rb; --b)
            if (!contains(g.bits, b)) g.bits.push_back(b);
        gs.push_back(g);
    }
    return gs;
}

// A group may talk to HBM directly when its thread-index bits start with
// the tile's low bits, so that each wave touches >= 256 contiguous bytes.
bool io_capable(const Group &g, int vw)
{
    for (int b = vw == 2 ? 1 : 0; b < (vw == 2 ? 5 : 4); ++b)
        if (contains(g.bits, b)) return false;
    return true;
}

// Step k: schedule midpoint s, driver angle theta, and the shear
// coefficients of the per-qubit rotation by phi = theta/2.  phi is reduced to
// [-pi/2, pi/2] first (a 2 pi shift changes nothing; M(phi) = -M(phi - pi)
// for the 2x2 block M), so |t| = |tan(phi/2)| <= 1 and the shears stay well
// conditioned; a reduction by pi flips the sign of every qubit's block,
// which the step's global phase absorbs (flip).
struct StepCoef {
    double s, theta, t, sn;
    bool flip;
};

StepCoef step_coef(double T, int64_t N, int64_t k, const SchedKnots &sc)
{
    StepCoef c;
    const double dt = T / (double)N;
    c.s = sched_mid(sc.v, sc.count, k, N);
    c.theta = dt * (1.0 - c.s);
    double phi = std::fmod(0.5 * c.theta, 2.0 * M_PI);
    if (phi > M_PI) phi -= 2.0 * M_PI;
    c.flip = false;
    if (phi > 0.5 * M_PI) {
        phi -= M_PI;
        c.flip = true;
    } else if (phi < -0.5 * M_PI) {
        phi += M_PI;
        c.flip = true;
    }
    c.t = std::tan(0.5 * phi);
    c.sn = std::sin(phi);
    return c;
}

double wrap_phase(double a);

// Global phase of step k's driver factor on n qubits: exp(-i n theta / 2),
// times (-1)^n when the rotation angle was reduced by pi.
double step_gphase(int n, const StepCoef &c)
{
    return wrap_phase(0.5 * n * c.theta + (c.flip ? M_PI * (n & 1) : 0.0));
}

double wrap_phase(double a)
{
    return std::fmod(a, 2.0 * M_PI);
}

uint32_t pad_index(uint32_t l, int dt) { return l + (uint32_t)kPadN[dt] * (l >> kPadS[dt]); }

// Residency list for one pass over set `sp`:
//   v1: rotate with coefficient set A before the phase,
//   ph: apply the phase,
//   v2: rotate with coefficient set B after the phase.
// The first and last residencies move the tile between HBM and registers,
// so both use a group whose register bits avoid the tile's low bits.
void fill_residencies(PassDesc &d, const SetPlan &sp, int tb, int rb, int dt, bool v1, bool ph, bool v2)
{
    const int vw = dt == 0 ? 2 : 1;
    std::vector<Group> gs = make_groups(sp.rot_local, tb, rb, vw);
    const int G = (int)gs.size();
    // Group order: the first group (always HBM-capable) first, then the
    // groups that cannot talk to HBM, then the other HBM-capable ones, so
    // that passes ending on the last group store directly when possible.
    {
        std::vector<Group> ord{gs[0]};
        for (int g = 1; g < G; ++g)
            if (!io_capable(gs[g], vw)) ord.push_back(gs[g]);
        for (int g = 1; g < G; ++g)
            if (io_capable(gs[g], vw)) ord.push_back(gs[g]);
        gs = ord;
    }
    struct Res {
        int g;
        uint32_t ma, mb;
        bool phase;
    };
    std::vector<Res> rs;
    if (v1 && ph && v2) {
        for (int g = 0; g < G - 1; ++g) rs.push_back({g, gs[g].rot, 0, false});
        rs.push_back({G - 1, gs[G - 1].rot, gs[G - 1].rot, true});
        for (int g = G - 2; g >= 0; --g) rs.push_back({g, 0, gs[g].rot, false});
    } else if (v1 && ph) {
        for (int g = 0; g < G - 1; ++g) rs.push_back({g, gs[g].rot, 0, false});
        rs.push_back({G - 1, gs[G - 1].rot, 0, true});
    } else if (ph && v2) {
        rs.push_back({0, 0, gs[0].rot, true});
        for (int g = 1; g < G; ++g) rs.push_back({g, 0, gs[g].rot, false});
    } else {
        for (int g = 0; g < G; ++g) rs.push_back({g, gs[g].rot, 0, false});
    }
    if (!io_capable(gs[rs.front().g], vw)) rs.insert(rs.begin(), Res{0, 0, 0, false});
    if (!io_capable(gs[rs.back().g], vw)) rs.push_back(Res{0, 0, 0, false});

    const int wb = tb - rb;
    const int R = 1 << rb;
    d.n_res = (int)rs.size();
    d.phase_at = -1;
    for (int r = 0; r < d.n_res; ++r) {
        const Group &g = gs[rs[r].g];
        int k = 0;
        for (int b = 0; b < tb; ++b)
            if (!contains(g.bits, b)) d.tpos[r][k++] = (uint8_t)b;
        for (int j = 0; j < R; ++j) {
            uint32_t l = 0;
            uint64_t gl = 0;
            for (int i = 0; i < rb; ++i)
                if ((j >> i) & 1) {
                    l |= 1u << g.bits[i];
                    gl |= 1ull << sp.tile[g.bits[i]];
                }
            d.lj[r][j] = (uint16_t)l;
            d.ljp[r][j] = (uint16_t)pad_index(l, dt);
            if (r == 0) d.goff_first[j] = gl;
            if (r == d.n_res - 1) d.goff_last[j] = gl;
        }
        if (r == 0)
            for (int kk = 0; kk < wb; ++kk) d.gpos_first[kk] = (uint8_t)sp.tile[d.tpos[0][kk]];
        if (r == d.n_res - 1)
            for (int kk = 0; kk < wb; ++kk) d.gpos_last[kk] = (uint8_t)sp.tile[d.tpos[r][kk]];
        d.masks[r] = rs[r].ma | (rs[r].mb << 8);
        if (rs[r].phase) d.phase_at = r;
    }
}

ResidentDesc make_resident_desc(const qaa_state *st, const SchedKnots &sc, double T, int64_t N, int64_t k0,
                                int64_t k1, int rb, const ClauseRec *clauses = nullptr)
{
    const int n = st->inst->n;
    ResidentDesc d;
    std::memset(&d, 0, sizeof d);
    d.sched = sc;
    d.amp = st->amp;
    d.table = st->table;
    d.clauses = clauses;
    d.m = st->inst->m;
    d.n = n;
    d.emax = st->inst->e_max;
    d.T = T;
    d.N = N;
    d.k0 = k0;
    d.k1 = k1;
    d.reg_bits = std::min(rb, n);
    d.thr_bits = n - d.reg_bits;
    std::vector<int> rot;
    for (int b = 0; b < n; ++b) rot.push_back(b);
    const std::vector<Group> gs = make_groups(rot, n, d.reg_bits, 1);
    d.n_groups = (int)gs.size();
    for (int g = 0; g < d.n_groups; ++g) {
        for (int i = 0; i < d.reg_bits; ++i) d.gbits[g][i] = (uint8_t)gs[g].bits[i];
        int k = 0;
        for (int b = 0; b < n; ++b)
            if (std::find(gs[g].bits.begin(), gs[g].bits.end(), b) == gs[g].bits.end()) d.tpos[g][k++] = (uint8_t)b;
        d.gmask[g] = (uint8_t)gs[g].rot;
    }
    return d;
}

qaa_status run_resident(const qaa_state *st, const SchedKnots &sc, double T, int64_t N, int64_t k0, int64_t k1,
                        hipStream_t s)
{
    int rb = 0, wb = 0;
    resident_shape(st->inst->n, &rb, &wb);
    ClauseRec *recs = nullptr;       // recompute mode: the kernel scores its energies once
    if (!st->table) {
        qaa_status rc = device_clauses(const_cast<qaa_instance *>(st->inst), &recs, "evolve");
        if (rc != QAA_OK) return rc;
    }
    const ResidentDesc d = make_resident_desc(st, sc, T, N, k0, k1, rb, recs);
    QAA_HIP(launch_resident(nullptr, &d, 1, (int)st->dtype, (int)st->etype, rb, wb, s));
    return QAA_OK;
}

// The pass sequence for steps k0..k1-1 (see PassDesc).  The qubit sets are
// visited forward on even steps (relative to k0) and backward on odd ones,
// so the set that ends step k also starts step k+1 and one pass applies
// both its rotations and the merged diagonal phase between them.
std::vector<PassDesc> build_passes(const Plan &p, int n, int dty, int emax, const SchedKnots &sc, double T,
                                   int64_t N, int64_t k0, int64_t k1)
{
    std::vector<PassDesc> out;
    const int RB = p.reg_bits;
    const int r = (int)p.sets.size();
    const double dt = T / (double)N;
    PassDesc base;
    std::memset(&base, 0, sizeof base);
    base.n = n;
    base.emax = emax;
    // The index maps depend only on the set and the pass kind (first pass,
    // turn, closing pass, rotations only): built once per (set, kind) and
    // copied, with each pass's coefficients written into the copy.
    std::vector<PassDesc> tmpl(4 * (size_t)r);
    std::vector<char> have(4 * (size_t)r, 0);
    auto templ = [&](int set, int kind) -> const PassDesc & {
        const size_t key = 4 * (size_t)set + (size_t)kind;
        if (!have[key]) {
            PassDesc d = base;
            const SetPlan &sp = p.sets[set];
            const int TB = sp.tb;
            for (int j = 0; j < TB; ++j) d.tile_pos[j] = (uint8_t)sp.tile[j];
            int nr = 0;
            d.rest_mask = 0;
            for (int b = 0; b < n; ++b)
                if (std::find(sp.tile.begin(), sp.tile.end(), b) == sp.tile.end()) {
                    d.rest_pos[nr++] = (uint8_t)b;
                    d.rest_mask |= 1ull << b;
                }
            d.n_rest = nr;
            d.set_id = set;
            d.reg_bits = RB;
            d.tile_begin = 0;
            d.tile_count = 1ull << nr;
            static const bool rot_a[4] = {false, true, true, true}, phase[4] = {true, true, true, false},
                              rot_b[4] = {true, true, false, false};
            fill_residencies(d, sp, TB, RB, dty, rot_a[kind], phase[kind], rot_b[kind]);
            tmpl[key] = d;
            have[key] = 1;
        }
        return tmpl[key];
    };
    out.reserve((size_t)(k1 - k0) * (size_t)std::max(1, r - 1) + 1);
    for (int64_t k = k0; k < k1; ++k) {
        const bool fwd = ((k - k0) & 1) == 0;
        const StepCoef ck = step_coef(T, N, k, sc);
        for (int idx = 0; idx < r; ++idx) {
            const int set = fwd ? idx : r - 1 - idx;
            const bool first = idx == 0, last = idx == r - 1;
            if (first && k > k0) continue;    // merged into the previous turn pass
            if (first) {
                // k == k0: half phase of step k0, then this set's rotations
                out.push_back(templ(set, 0));
                PassDesc &d = out.back();
                d.phi = 0.5 * dt * ck.s;
                d.gphase = 0.0;
                d.tB = ck.t;
                d.sB = ck.sn;
            } else if (last && k + 1 < k1) {
                out.push_back(templ(set, 1));
                PassDesc &d = out.back();
                const StepCoef cn = step_coef(T, N, k + 1, sc);
                d.tA = ck.t;
                d.sA = ck.sn;
                d.phi = 0.5 * dt * (ck.s + cn.s);
                d.gphase = step_gphase(n, ck);
                d.tB = cn.t;
                d.sB = cn.sn;
            } else if (last) {
                out.push_back(templ(set, 2));
                PassDesc &d = out.back();
                d.tA = ck.t;
                d.sA = ck.sn;
                d.phi = 0.5 * dt * ck.s;
                d.gphase = step_gphase(n, ck);
            } else {
                out.push_back(templ(set, 3));
                PassDesc &d = out.back();
                d.tA = ck.t;
                d.sA = ck.sn;
            }
        }
    }
    return out;
}

// Cache blocking.  Between two passes over the top qubit set, every other
// pass keeps the top bits of the index fixed inside each tile, so those
// passes can run group by group: all of them over the tiles whose top
// `cbits` index bits equal g, then all of them for g + 1, ...  A group of
// 2^(log2 bytes) bytes stays in the device's last-level caches between those
// passes, so only the first read and the final write of a group reach HBM.
// Off by default (measured slower at n = 28: each chunked launch is too
// short for the persistent pipeline); QAA_CHUNK_LOG2_BYTES = log2 of the
// group size in bytes turns it on.
int chunk_log2_bytes()
{
    const char *e = std::getenv("QAA_CHUNK_LOG2_BYTES");
    return e ? std::atoi(e) : 0;
}

std::vector<PassDesc> schedule_passes(const std::vector<PassDesc> &in, const Plan &p, int n, int amp_log2_bytes)
{
    const int top = (int)p.sets.size() - 1;
    const int lg = chunk_log2_bytes();
    if (lg <= 0 || top < 2) return in;
    // the group index is made of the highest index bits, which must all be
    // rotated by the top set (so that no other pass mixes groups)
    std::vector<int> top_rot;
    for (int j : p.sets[top].rot_local) top_rot.push_back(p.sets[top].tile[j]);
    int run = 0;
    while (run < n && contains(top_rot, n - 1 - run)) ++run;
    const int cbits = std::min(std::max(0, n + amp_log2_bytes - lg), run);
    if (cbits == 0) return in;
    std::vector<PassDesc> out;
    size_t i = 0;
    while (i < in.size()) {
        if (in[i].set_id == top) {
            out.push_back(in[i++]);
            continue;
        }
        size_t j = i;
        while (j < in.size() && in[j].set_id != top) ++j;
        // passes [i, j) never touch the top set: split them by chunk group,
        // when the top cbits of every tile-id are the top cbits of the index
        bool ok = true;
        for (size_t q = i; q < j && ok; ++q) {
            const PassDesc &d = in[q];
            if (d.n_rest < cbits) ok = false;
            for (int b = 0; b < cbits && ok; ++b)
                if (d.rest_pos[d.n_rest - cbits + b] != n - cbits + b) ok = false;
        }
        if (!ok || j - i < 2) {
            for (size_t q = i; q < j; ++q) out.push_back(in[q]);
        } else {
            for (uint64_t g = 0; g < (1ull << cbits); ++g)
                for (size_t q = i; q < j; ++q) {
                    PassDesc d = in[q];
                    d.tile_count = 1ull << (d.n_rest - cbits);
                    d.tile_begin = g * d.tile_count;
                    out.push_back(d);
                }
        }
        i = j;
    }
    return out;
}

// ---------------------------------------------------------------------------
// Kernel timing: event pairs around pass launches (qaa_profile_enable).
// ---------------------------------------------------------------------------
struct ProfRec {
    hipEvent_t a, b;
    double bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::deque<ProfRec> g_prof_live;      // recorded, not yet read (launch order)
std::vector<hipEvent_t> g_prof_pool;  // free events
int64_t g_prof_launches = 0;
double g_prof_ms = 0.0, g_prof_min = 0.0, g_prof_max = 0.0, g_prof_bytes = 0.0;

hipError_t prof_event(hipEvent_t *e)
{
    if (!g_prof_pool.empty()) {
        *e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// Collect finished records, oldest first; with wait = false only up to the
// first one still running (later launches on its stream cannot have
// finished), so a drain costs one query per record collected plus one.
hipError_t prof_drain(bool wait)
{
    while (!g_prof_live.empty()) {
        ProfRec r = g_prof_live.front();
        if (wait) {
            hipError_t e = hipEventSynchronize(r.b);
            if (e != hipSuccess) return e;
        } else if (hipEventQuery(r.b) != hipSuccess) {
            break;
        }
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return e;
        if (g_prof_launches == 0 || ms < g_prof_min) g_prof_min = ms;
        if (g_prof_launches == 0 || ms > g_prof_max) g_prof_max = ms;
        g_prof_launches += 1;
        g_prof_ms += ms;
        g_prof_bytes += r.bytes;
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
        g_prof_live.pop_front();
    }
    return hipSuccess;
}

std::vector<PassDesc> plan_passes(const Plan &p, int n, int dty, int emax, const SchedKnots &sc, double T,
                                  int64_t N, int64_t k0, int64_t k1)
{
    std::vector<PassDesc> v = build_passes(p, n, dty, emax, sc, T, N, k0, k1);
    if (chunk_log2_bytes() <= 0) return v;
    return schedule_passes(v, p, n, dty == 0 ? 3 : 4);
}

// Norm control (see PassDesc) is on unless QAA_NORM_CONTROL=0 is set in
// the environment (used to measure the uncorrected FP32 drift).
bool norm_control_enabled()
{
    static const bool on = [] {
        const char *e = std::getenv("QAA_NORM_CONTROL");
        return !(e && e[0] == '0');
    }();
    return on;
}

// fixed_acc: nullptr, or three norm-control accumulators the caller owns
// (qaa_evolve_range_noalloc); otherwise they come from the stream-ordered
// allocator for this call.
qaa_status run_passes(const qaa_state *st, const Plan &p, const SchedKnots &sc, double T, int64_t N, int64_t k0,
                      int64_t k1, hipStream_t s, unsigned long long *fixed_acc)
{
    std::vector<PassDesc> ps = plan_passes(p, st->inst->n, (int)st->dtype, st->inst->e_max, sc, T, N, k0, k1);
    ClauseRec *recs = nullptr;       // recompute mode: passes with a phase score their tiles
    if (!st->table) {
        qaa_status rc = device_clauses(const_cast<qaa_instance *>(st->inst), &recs, "evolve");
        if (rc != QAA_OK) return rc;
    }
    unsigned long long *acc = nullptr;
    const bool own_acc = fixed_acc == nullptr;
    if (norm_control_enabled()) {
        if (own_acc)
            QAA_HIP(hipMallocAsync(reinterpret_cast<void **>(&acc), kNormWords * sizeof(unsigned long long), s));
        else
            acc = fixed_acc;
        // a fill kernel, not a memset node: callers may capture this call
        QAA_HIP(launch_zero_u64(acc, kNormWords, s));
    }
    bool prof;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        prof = g_prof_on;
    }
    const double amp_bytes = st->dtype == QAA_C64 ? 8.0 : 16.0;
    const double e_bytes = st->etype == QAA_E_U8 ? 1.0 : 2.0;
    const double dim = std::ldexp(1.0, st->inst->n);
    int64_t gj = 0;     // index of the next norm-carrying pass
    const int top = (int)p.sets.size() - 1;
    // Passes over the sets below the top one keep the top set's index bits
    // as the high bits of their tile numbers, so the region a pass wrote
    // last is the region the next such pass visits first if it runs in the
    // opposite direction: consecutive lower-set passes alternate direction
    // and start on data still in the last-level cache.
    bool prev_low = false, prev_rev = false;
    bool reduce_next = false;   // the previous pass measured the norm
    for (PassDesc &d : ps) {
        d.clauses = recs;
        d.m = st->inst->m;
        const bool full = d.tile_begin == 0 && d.tile_count == (1ull << d.n_rest);
        const bool low = d.set_id != top && full;
        d.reverse = (low && prev_low && !prev_rev) ? 1 : 0;
        // One workgroup per tile streams fastest (n = 28: middle passes
        // 0.89 -> 0.82 ms, set-0 turns 0.84 -> 0.81 ms, top turns 0.96 ->
        // 0.94 ms; n = 16..21: 6-8 % per step), except over the top set of a
        // plan with three or more sets from n = 29 on (complex64; its tiles
        // are gathered from runs spread over the whole state, n = 29..31:
        // 1-5 % per step faster on the persistent grid, with the next
        // tile's loads in flight) and for complex128, measured on the
        // persistent grid only.
        d.persist = (top >= 2 && d.set_id == top && (st->dtype != QAA_C64 || st->inst->n >= 29)) ? 1 : 0;
        d.xcd_map = xcd_arrangement(d, st->inst->n, (int)st->dtype);
        prev_low = low;
        prev_rev = d.reverse != 0;
        // Norm control rides on the passes over the top qubit set: each one
        // measures the norm of its output, and rescales by the norm the
        // previous one measured (passes over other sets carry no norm work).
        if (acc && d.set_id == top) {
            d.acc_out = acc + kNormTotalsWords;
            d.acc_zero = acc + (gj + 1) % 3;
            d.acc_in = gj > 0 ? acc + (gj + 2) % 3 : nullptr;
            ++gj;
            reduce_next = true;
        } else if (reduce_next) {
            // the pass after a measuring pass reduces its partial slots into
            // the total the next measuring pass scales by (top-set passes
            // are never adjacent)
            d.red_src = acc + kNormTotalsWords;
            d.red_dst = acc + (gj - 1) % 3;
            reduce_next = false;
        }
        ProfRec rec{};
        if (prof) {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            if (g_prof_live.size() > 4096) QAA_HIP(prof_drain(false));
            QAA_HIP(prof_event(&rec.a));
            QAA_HIP(prof_event(&rec.b));
            rec.bytes = dim * (double)d.tile_count / std::ldexp(1.0, d.n_rest) *
                        (2.0 * amp_bytes + (d.phase_at >= 0 && st->table ? e_bytes : 0.0));
        }
        hipError_t e;
        {
            TraceRange tr("qaa pass: set %d, phase at residency %d, tiles %lld+%lld", d.set_id, d.phase_at,
                          (long long)d.tile_begin, (long long)d.tile_count);
            // profiling: the events are the dispatch's own start and stop
            e = launch_pass(st->amp, (int)st->dtype, st->table, (int)st->etype, d.n - d.n_rest, p.reg_bits, d, s,
                            prof ? rec.a : nullptr, prof ? rec.b : nullptr);
        }
        if (e != hipSuccess) {
            if (acc && own_acc) (void)hipFreeAsync(acc, s);
            return fail(QAA_ERR_DEVICE, "pass launch failed: %s", hipGetErrorString(e));
        }
        if (prof) {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            g_prof_live.push_back(rec);
        }
    }
    if (acc && own_acc) QAA_HIP(hipFreeAsync(acc, s));
    return QAA_OK;
}

int lut_limit(qaa_etype e) { return e == QAA_E_U8 ? kLutMaxU8 : kLutMax; }

}  // namespace

// Validates a caller's schedule and copies it into the form the planner and
// the kernels read (NULL and QAA_SCHED_LINEAR: count 0).
qaa_status qaa::to_knots(const qaa_schedule *sched, SchedKnots *out, const char *who)
{
    std::memset(out, 0, sizeof *out);
    if (!sched || sched->kind == QAA_SCHED_LINEAR) return QAA_OK;
    if (sched->kind != QAA_SCHED_TABLE)
        return fail(QAA_ERR_INVALID_ARG, "%s: unknown schedule kind %d", who, sched->kind);
    if (sched->count < 2 || sched->count > kMaxKnots)
        return fail(QAA_ERR_INVALID_ARG, "%s: schedule table needs 2..%d knots, got %d", who, kMaxKnots,
                    sched->count);
    if (!sched->values) return fail(QAA_ERR_INVALID_ARG, "%s: schedule table values is NULL", who);
    for (int j = 0; j < sched->count; ++j) {
        const double v = sched->values[j];
        if (!(v >= 0.0 && v <= 1.0))
            return fail(QAA_ERR_INVALID_ARG, "%s: schedule knot %d is not in [0, 1]", who, j);
        out->v[j] = v;
    }
    out->count = sched->count;
    return QAA_OK;
}

// ---------------------------------------------------------------------------
// Evolution without device allocation.  The three norm-control accumulators
// of a multi-pass evolution live in `scratch`, a static device array of this
// translation unit (each device the library runs on holds its own copy until
// the process ends), instead of the stream-ordered allocator.  Host code
// never uses the array's name as a device address: at a device's first call
// its address comes from hipGetSymbolAddress, with that device current, and
// is kept per device.  Every call on a device shares the array; it is
// cleared by a fill kernel at the start of each multi-pass call, so calls
// that overlap on one device race.
// ---------------------------------------------------------------------------
namespace {

constexpr int kScratchWords = kNormWords;     // 64 KiB + 128 B: the norm totals and partial slots
static __device__ __align__(256) unsigned long long scratch[kScratchWords];

std::mutex g_scratch_mu;
std::map<int, unsigned long long *> g_scratch_addr;

qaa_status scratch_address(unsigned long long **out, const char *who)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(QAA_ERR_DEVICE, "%s: hipGetDevice failed: %s", who, hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(QAA_ERR_DEVICE, "%s: hipGetSymbolAddress(scratch) failed on device %d: %s", who, dev,
                        hipGetErrorString(e));
        it = g_scratch_addr.emplace(dev, reinterpret_cast<unsigned long long *>(ptr)).first;
    }
    *out = it->second;
    return QAA_OK;
}


qaa_status evolve_common(const qaa_state *st, const qaa_schedule *sched, double T, int64_t steps, int64_t k0,
                         int64_t k1, void *stream, const char *who, bool noalloc = false)
{
    SchedKnots sc;
    qaa_status r = to_knots(sched, &sc, who);
    if (r != QAA_OK) return r;
    r = check_state_table(st, who);
    if (r != QAA_OK) return r;
    if (!(T >= 0.0) || !std::isfinite(T)) return fail(QAA_ERR_INVALID_ARG, "%s: T must be finite and >= 0", who);
    if (steps < 0) return fail(QAA_ERR_INVALID_ARG, "%s: steps < 0", who);
    if (k0 < 0 || k1 < k0 || k1 > steps)
        return fail(QAA_ERR_INVALID_ARG, "%s: need 0 <= k0 <= k1 <= steps", who);
    if (st->inst->e_max >= lut_limit(st->etype))
        return fail(QAA_ERR_UNSUPPORTED, "%s: E_max=%d exceeds the phase table limit %d", who, st->inst->e_max,
                    lut_limit(st->etype) - 1);
    if (k0 == k1) return ok();
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Plan p = make_plan(st->inst->n, (int)st->dtype, (int)st->etype);
    if (p.resident) {
        r = run_resident(st, sc, T, steps, k0, k1, s);
    } else {
        // the accumulators do not grow with n: every state the library
        // accepts (n <= QAA_MAX_QUBITS) fits the scratch array
        static_assert(kNormWords <= kScratchWords, "norm-control accumulators exceed the scratch array");
        unsigned long long *fixed_acc = nullptr;
        if (noalloc) {
            r = scratch_address(&fixed_acc, who);
            if (r != QAA_OK) return r;
        }
        r = run_passes(st, p, sc, T, steps, k0, k1, s, fixed_acc);
    }
    if (r != QAA_OK) return r;
    return ok();
}

}  // namespace

extern "C" qaa_status qaa_evolve(const qaa_state *st, const qaa_schedule *sched, double T, int64_t steps,
                                 void *stream)
{
    TraceRange tr("qaa_evolve");
    return evolve_common(st, sched, T, steps, 0, steps, stream, "qaa_evolve");
}

extern "C" qaa_status qaa_evolve_range(const qaa_state *st, const qaa_schedule *sched, double T, int64_t steps,
                                       int64_t k0, int64_t k1, void *stream)
{
    TraceRange tr("qaa_evolve_range");
    return evolve_common(st, sched, T, steps, k0, k1, stream, "qaa_evolve_range");
}

extern "C" qaa_status qaa_evolve_range_noalloc(const qaa_state *st, const qaa_schedule *sched, double T,
                                               int64_t steps, int64_t k0, int64_t k1, void *stream)
{
    TraceRange tr("qaa_evolve_range_noalloc");
    return evolve_common(st, sched, T, steps, k0, k1, stream, "qaa_evolve_range_noalloc", true);
}


namespace {

// Pass structures of one qubit count for the batched kernel, in the kind
// order documented at BatchInst.
void batch_structs(const Plan &p, int n, int dty, std::vector<PassDesc> &out)
{
    const int RB = p.reg_bits;
    const int r = (int)p.sets.size();
    auto make = [&](int set, bool v1, bool ph, bool v2) {
        PassDesc d;
        std::memset(&d, 0, sizeof d);
        d.n = n;
        const SetPlan &sp = p.sets[set];
        const int TB = sp.tb;
        for (int j = 0; j < TB; ++j) d.tile_pos[j] = (uint8_t)sp.tile[j];
        int nr = 0;
        for (int b = 0; b < n; ++b)
            if (!contains(sp.tile, b)) {
                d.rest_pos[nr++] = (uint8_t)b;
                d.rest_mask |= 1ull << b;
            }
        d.n_rest = nr;
        d.set_id = set;
        d.tile_count = 1ull << nr;
        fill_residencies(d, sp, TB, RB, dty, v1, ph, v2);
        out.push_back(d);
    };
    make(0, false, true, true);                          // kind 0: first pass
    for (int m = 1; m <= r - 2; ++m) make(m, true, false, false);
    make(r - 1, true, true, true);                       // turn at the top set
    make(0, true, true, true);                           // turn at set 0
    make(r - 1, true, true, false);                      // last pass at the top set
    make(0, true, true, false);                          // last pass at set 0
}

template <typename T>
qaa_status upload(const std::vector<T> &host, T **dev, hipStream_t s)
{
    const size_t bytes = sizeof(T) * std::max<size_t>(1, host.size());
    QAA_HIP(hipMallocAsync(reinterpret_cast<void **>(dev), bytes, s));
    void *pinned = nullptr;
    hipError_t e = hipHostMalloc(&pinned, bytes, hipHostMallocDefault);
    if (e == hipSuccess) {
        std::memcpy(pinned, host.data(), sizeof(T) * host.size());
        e = hipMemcpyAsync(*dev, pinned, sizeof(T) * host.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipHostFree(pinned);
    }
    if (e != hipSuccess) {
        (void)hipFreeAsync(*dev, s);
        *dev = nullptr;
        return fail(QAA_ERR_DEVICE, "descriptor upload failed: %s", hipGetErrorString(e));
    }
    return QAA_OK;
}

// Lock-step batched passes for states of one dtype/etype above the resident
// size.  States are grouped by their number of qubit sets r (a group runs
// r - 1 passes per step, r in the first); inside a group they are sorted by
// step count, longest first, so the states still running at step k are a
// prefix, and each state's tiles are cut into chunks of batch_chunk_tiles()
// (one workgroup each).
// Tiles per workgroup chunk: QAA_BATCH_CHUNK_TILES (1..64, read once), else 8.
int batch_chunk_tiles()
{
    static const int v = [] {
        const char *e = std::getenv("QAA_BATCH_CHUNK_TILES");
        const int x = e ? std::atoi(e) : 0;
        return x >= 1 && x <= 64 ? x : 8;
    }();
    return v;
}

// Extra streams for a batch's launch groups: QAA_BATCH_STREAMS (0..3, read
// once), else 2.  0 runs every group on the caller's stream.  (With the
// caller's stream and the side stream, 2 extra streams fill the four
// hardware queues a process gets by default.)
int batch_group_streams()
{
    static const int v = [] {
        const char *e = std::getenv("QAA_BATCH_STREAMS");
        const int x = e ? std::atoi(e) : 2;
        return x >= 0 && x <= 3 ? x : 2;
    }();
    return v;
}

// Split the heaviest launch groups in two until every stream has one
// (QAA_BATCH_SPLIT=0, read once: one launch group per plan shape).
bool batch_split()
{
    static const bool v = [] {
        const char *e = std::getenv("QAA_BATCH_SPLIT");
        return !(e && std::atoi(e) == 0);
    }();
    return v;
}

// The first `want` group streams of the device (created on first use).
qaa_status group_streams(DeviceCtx *ctx, int want, std::vector<hipStream_t> *out)
{
    std::lock_guard<std::mutex> lk(ctx->group_mu);
    while ((int)ctx->group.size() < want) {
        hipStream_t st = nullptr;
        QAA_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        ctx->group.push_back(st);
    }
    out->assign(ctx->group.begin(), ctx->group.begin() + want);
    return QAA_OK;
}

qaa_status run_batch_passes(const std::vector<int> &idx, const qaa_state *states, const SchedKnots *scs,
                            const double *T, const int64_t *steps, hipStream_t s, DeviceCtx *ctx)
{
    if (idx.empty()) return QAA_OK;
    const int dty = (int)states[idx[0]].dtype, ety = (int)states[idx[0]].etype;
    const int chunk_tiles = batch_chunk_tiles();
    // A launch group holds states whose plans have the same number of sets
    // and the same tile size per set, so that every pass of a step runs one
    // kernel variant for all of them.  Each state has a chunk table entry
    // per tile variant its sets use (base [0], wide [1]).
    struct GroupPlan {
        int r = 0, rb = 0;                        // qubit sets, register bits
        std::vector<int> tbs;                     // tile bits per set
        std::vector<int> order;                   // state indices, longest first
        size_t inst_base = 0, chunk_base[2] = {0, 0};
        std::vector<uint64_t> chunk_prefix[2];    // chunks of the first q states, per variant
    };
    std::map<std::vector<int>, GroupPlan> groups;
    for (int i : idx) {
        const Plan p = make_plan(states[i].inst->n, dty, ety);
        std::vector<int> key{p.reg_bits, (int)p.sets.size()};
        for (const SetPlan &sp : p.sets) key.push_back(sp.tb);
        GroupPlan &g = groups[key];
        g.rb = p.reg_bits;
        g.r = (int)p.sets.size();
        g.tbs.assign(key.begin() + 2, key.end());
        g.order.push_back(i);
    }
    // Splitting: while there are fewer launch groups than streams, the
    // group with the most amplitude-steps is split in two, its states
    // (longest first) dealt alternately, so each part runs on its own stream.
    if (batch_split()) {
        const size_t want = 1 + (size_t)batch_group_streams();
        auto work = [&](const GroupPlan &g) {
            double w = 0.0;
            for (int i : g.order) w += std::ldexp((double)steps[i], states[i].inst->n);
            return w;
        };
        std::map<std::vector<int>, GroupPlan> parts;
        for (auto &kv : groups) {
            std::vector<int> key = kv.first;
            key.push_back(0);
            parts[key] = kv.second;
        }
        int next_id = 1;
        while (parts.size() < want) {
            auto best = parts.end();
            for (auto it = parts.begin(); it != parts.end(); ++it)
                if (it->second.order.size() >= 2 && (best == parts.end() || work(it->second) > work(best->second)))
                    best = it;
            if (best == parts.end()) break;
            GroupPlan g = best->second;
            std::vector<int> key = best->first;
            parts.erase(best);
            std::stable_sort(g.order.begin(), g.order.end(), [&](int a, int b) { return steps[a] > steps[b]; });
            GroupPlan h[2];
            for (int q = 0; q < 2; ++q) {
                h[q].rb = g.rb;
                h[q].r = g.r;
                h[q].tbs = g.tbs;
            }
            for (size_t q = 0; q < g.order.size(); ++q) h[q & 1].order.push_back(g.order[q]);
            parts[key] = h[0];
            key.back() = next_id++;
            parts[key] = h[1];
        }
        groups.swap(parts);
    }
    std::vector<PassDesc> structs;
    std::map<int, int> base_of_n;
    std::vector<BatchInst> insts;
    std::vector<uint32_t> chunk_inst[2];
    int64_t maxN = 0;
    for (auto &kv : groups) {
        GroupPlan &g = kv.second;
        std::stable_sort(g.order.begin(), g.order.end(), [&](int a, int b) { return steps[a] > steps[b]; });
        g.inst_base = insts.size();
        bool uses[2] = {false, false};
        for (int tb : g.tbs) uses[tb == kWideTileBits ? 1 : 0] = true;
        for (int v = 0; v < 2; ++v) {
            g.chunk_base[v] = chunk_inst[v].size();
            g.chunk_prefix[v].assign(1, 0);
        }
        for (int i : g.order) {
            const int n = states[i].inst->n;
            if (!base_of_n.count(n)) {
                base_of_n[n] = (int)structs.size();
                batch_structs(make_plan(n, dty, ety), n, dty, structs);
            }
            BatchInst b;
            std::memset(&b, 0, sizeof b);
            b.amp = states[i].amp;
            b.table = states[i].table;
            b.T = T[i];
            b.N = steps[i];
            b.n = n;
            b.emax = states[i].inst->e_max;
            b.r = g.r;
            b.struct_base = base_of_n[n];
            b.sched = scs[i];
            for (int v = 0; v < 2; ++v) {
                b.chunk_offset[v] = g.chunk_prefix[v].back();
                uint64_t chunks = 0;
                if (uses[v]) {
                    const int tb = v ? kWideTileBits : kPassTileBits[dty];
                    chunks = ((1ull << (n - tb)) + chunk_tiles - 1) / chunk_tiles;
                }
                for (uint64_t c = 0; c < chunks; ++c) chunk_inst[v].push_back((uint32_t)(insts.size() - g.inst_base));
                g.chunk_prefix[v].push_back(g.chunk_prefix[v].back() + chunks);
            }
            insts.push_back(b);
            maxN = std::max(maxN, steps[i]);
        }
    }
    unsigned long long *acc = nullptr;
    const int cnt = (int)insts.size();
    if (norm_control_enabled()) {
        QAA_HIP(hipMallocAsync(reinterpret_cast<void **>(&acc), 3 * sizeof(unsigned long long) * cnt, s));
        QAA_HIP(launch_zero_u64(acc, 3 * cnt, s));
        for (int q = 0; q < cnt; ++q) insts[q].acc = acc + 3 * q;
    }
    BatchInst *d_insts = nullptr;
    PassDesc *d_structs = nullptr;
    uint32_t *d_chunks[2] = {nullptr, nullptr};
    // every buffer this call took goes back in stream order, on every path
    auto release = [&]() {
        if (d_insts) (void)hipFreeAsync(d_insts, s);
        if (d_structs) (void)hipFreeAsync(d_structs, s);
        for (int v = 0; v < 2; ++v)
            if (d_chunks[v]) (void)hipFreeAsync(d_chunks[v], s);
        if (acc) (void)hipFreeAsync(acc, s);
    };
    qaa_status r = upload(insts, &d_insts, s);
    if (r == QAA_OK) r = upload(structs, &d_structs, s);
    for (int v = 0; v < 2 && r == QAA_OK; ++v) r = upload(chunk_inst[v], &d_chunks[v], s);
    if (r != QAA_OK) {
        release();
        return r;
    }
    // Launch groups share no state, so each may run on a stream of its own:
    // the first on the caller's stream, the others on the device's group
    // streams, forked after the uploads and joined back before the buffers
    // are released.  A group's launches each drain before the next of that
    // group starts; on separate streams the device fills one group's
    // ragged last round of workgroups with another group's work.  (Calls
    // from several threads may share the group streams: their launches then
    // also wait for each other, in enqueue order, which only serialises.)
    std::vector<hipStream_t> gs;
    const int extra = std::min<int>(batch_group_streams(), (int)groups.size() - 1);
    if (extra > 0) {
        r = group_streams(ctx, extra, &gs);
        if (r != QAA_OK) {
            release();
            return r;
        }
    }
    std::vector<hipEvent_t> evs(gs.size(), nullptr);
    auto free_events = [&]() {
        for (hipEvent_t &e : evs)
            if (e) (void)hipEventDestroy(e);
    };
    for (size_t i = 0; i < gs.size(); ++i) {
        hipError_t e = hipEventCreateWithFlags(&evs[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(evs[i], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(gs[i], evs[i], 0);
        if (e != hipSuccess) {
            // the group streams forked so far hold no work of this call yet
            free_events();
            release();
            return fail(QAA_ERR_DEVICE, "batched passes: fork failed: %s", hipGetErrorString(e));
        }
    }
    // every group stream's work of this call is ordered before the caller's
    // stream continues (and before the buffers go back), on every path
    auto join = [&]() {
        hipError_t first = hipSuccess;
        for (size_t i = 0; i < gs.size(); ++i) {
            hipError_t e = hipEventRecord(evs[i], gs[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, evs[i], 0);
            if (e != hipSuccess && first == hipSuccess) first = e;
        }
        free_events();
        return first;
    };
    std::map<std::vector<int>, int> active;
    std::map<std::vector<int>, hipStream_t> stream_of;
    {
        int gi = 0;
        for (auto &kv : groups) {
            active[kv.first] = (int)kv.second.order.size();
            stream_of[kv.first] = gi == 0 || gs.empty() ? s : gs[(gi - 1) % gs.size()];
            ++gi;
        }
    }
    for (int64_t k = 0; k < maxN; ++k) {
        for (auto &kv : groups) {
            const GroupPlan &g = kv.second;
            const hipStream_t gst = stream_of[kv.first];
            int &a = active[kv.first];
            while (a > 0 && insts[g.inst_base + a - 1].N <= k) --a;
            if (a == 0) continue;
            const int jn = k == 0 ? g.r : g.r - 1;
            for (int j = 0; j < jn; ++j) {
                // the set this pass visits (zig-zag order, as the kernel derives it)
                const int pos = k == 0 ? j : j + 1;
                const int set = (k & 1) == 0 ? pos : g.r - 1 - pos;
                const int tb = g.tbs[set];
                const int v = tb == kWideTileBits ? 1 : 0;
                hipError_t e = launch_batch_pass(d_insts + g.inst_base, d_chunks[v] + g.chunk_base[v],
                                                 g.chunk_prefix[v][a], d_structs, k, j, chunk_tiles, dty, ety, tb, g.rb,
                                                 gst);
                if (e != hipSuccess) {
                    (void)join();
                    release();
                    return fail(QAA_ERR_DEVICE, "batched pass launch failed: %s", hipGetErrorString(e));
                }
            }
        }
    }
    const hipError_t je = join();
    release();
    if (je != hipSuccess) return fail(QAA_ERR_DEVICE, "batched passes: join failed: %s", hipGetErrorString(je));
    return QAA_OK;
}

}  // namespace

extern "C" qaa_status qaa_evolve_batch(int32_t count, const qaa_state *states, const qaa_schedule *scheds,
                                       const double *T, const int64_t *steps, void *stream)
{
    TraceRange trace_range("qaa_evolve_batch");
    if (count < 0) return fail(QAA_ERR_INVALID_ARG, "qaa_evolve_batch: count < 0");
    if (count == 0) return ok();
    if (!states || !T || !steps) return fail(QAA_ERR_INVALID_ARG, "qaa_evolve_batch: NULL array");
    std::vector<SchedKnots> scs((size_t)count);
    for (int i = 0; i < count; ++i) {
        qaa_status r = to_knots(scheds ? &scheds[i] : nullptr, &scs[i], "qaa_evolve_batch");
        if (r != QAA_OK) return r;
        r = check_state_table(&states[i], "qaa_evolve_batch", false);
        if (r != QAA_OK) return r;
        if (!(T[i] >= 0.0) || !std::isfinite(T[i]) || steps[i] < 0)
            return fail(QAA_ERR_INVALID_ARG, "qaa_evolve_batch: state %d has a bad T or step count", i);
        if (states[i].inst->e_max >= lut_limit(states[i].etype))
            return fail(QAA_ERR_UNSUPPORTED, "qaa_evolve_batch: state %d E_max exceeds the phase table", i);
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    DeviceCtx *ctx = nullptr;
    qaa_status r = device_ctx(&ctx);
    if (r != QAA_OK) return r;
    // small states: one resident launch per dtype/etype on the side stream;
    // larger ones: lock-step batched passes per dtype/etype on the caller's
    std::vector<ResidentDesc> small[2][2];
    std::vector<int> large[2][2];
    for (int i = 0; i < count; ++i) {
        if (steps[i] == 0) continue;
        const int dt = (int)states[i].dtype, et = (int)states[i].etype;
        if (make_plan(states[i].inst->n, dt, et).resident)
            small[dt][et].push_back(make_resident_desc(&states[i], scs[i], T[i], steps[i], 0, steps[i], kResRegBits[dt]));
        else
            large[dt][et].push_back(i);
    }
    // The small states go to the device's side stream, forked from and
    // joined back into the caller's stream with events of this call; the
    // lock covers only the enqueueing on the shared side stream.
    hipEvent_t fork = nullptr, join = nullptr;
    QAA_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    hipError_t he = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    if (he != hipSuccess) {
        (void)hipEventDestroy(fork);
        return fail(QAA_ERR_DEVICE, "qaa_evolve_batch: event creation failed: %s", hipGetErrorString(he));
    }
    auto done = [&](qaa_status st) {
        (void)hipEventDestroy(fork);
        (void)hipEventDestroy(join);
        return st;
    };
    bool joined = false;      // join recorded on the side stream
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        he = hipEventRecord(fork, s);
        if (he == hipSuccess) he = hipStreamWaitEvent(ctx->side, fork, 0);
        if (he != hipSuccess)
            return done(fail(QAA_ERR_DEVICE, "qaa_evolve_batch: fork failed: %s", hipGetErrorString(he)));
        for (int dt = 0; dt < 2 && he == hipSuccess && r == QAA_OK; ++dt)
            for (int et = 0; et < 2 && he == hipSuccess && r == QAA_OK; ++et) {
                if (small[dt][et].empty()) continue;
                ResidentDesc *d = nullptr;
                r = upload(small[dt][et], &d, ctx->side);
                if (r != QAA_OK) break;
                he = launch_resident(d, nullptr, (int)small[dt][et].size(), dt, et, kResRegBits[dt], kResThrBits,
                                     ctx->side);
                (void)hipFreeAsync(d, ctx->side);
            }
        joined = hipEventRecord(join, ctx->side) == hipSuccess;
    }
    if (r == QAA_OK && he != hipSuccess)
        r = fail(QAA_ERR_DEVICE, "qaa_evolve_batch: resident launch failed: %s", hipGetErrorString(he));
    for (int dt = 0; dt < 2 && r == QAA_OK; ++dt)
        for (int et = 0; et < 2 && r == QAA_OK; ++et) r = run_batch_passes(large[dt][et], states, scs.data(), T, steps, s, ctx);
    // the caller's stream waits for the side stream's work of this call on
    // every path, so none of it outlives the caller's stream unordered
    he = joined ? hipStreamWaitEvent(s, join, 0) : hipErrorUnknown;
    if (r != QAA_OK) return done(r);
    if (he != hipSuccess) return done(fail(QAA_ERR_DEVICE, "qaa_evolve_batch: join failed"));
    return done(ok());
}

// ---------------------------------------------------------------------------
// Spectrum of H(s)
// ---------------------------------------------------------------------------
extern "C" qaa_status qaa_spectrum(const qaa_instance *inst, const void *table, qaa_etype etype, int32_t count,
                                   const double *s_values, const double *v0, int32_t iters, int32_t k,
                                   double *evals, double *bounds, void *stream)
{
    TraceRange trace_range("qaa_spectrum");
    const char *who = "qaa_spectrum";
    if (!inst) return fail(QAA_ERR_INVALID_ARG, "%s: instance is NULL", who);
    if (!table || !v0) return fail(QAA_ERR_INVALID_ARG, "%s: table or v0 is NULL", who);
    if (etype != QAA_E_U8 && etype != QAA_E_U16) return fail(QAA_ERR_INVALID_ARG, "%s: bad etype %d", who, (int)etype);
    if (count < 0) return fail(QAA_ERR_INVALID_ARG, "%s: count < 0", who);
    if (count > 0 && (!s_values || !evals)) return fail(QAA_ERR_INVALID_ARG, "%s: NULL s_values or evals", who);
    if (iters < 1 || iters > QAA_SPECTRUM_MAX_ITERS)
        return fail(QAA_ERR_INVALID_ARG, "%s: iters must be in 1..%d", who, QAA_SPECTRUM_MAX_ITERS);
    if (k < 1 || k > iters) return fail(QAA_ERR_INVALID_ARG, "%s: k must be in 1..iters", who);
    for (int i = 0; i < count; ++i)
        if (!(s_values[i] >= 0.0 && s_values[i] <= 1.0))
            return fail(QAA_ERR_INVALID_ARG, "%s: s_values[%d] is not in [0, 1]", who, i);
    if (reinterpret_cast<uintptr_t>(v0) % 8) return fail(QAA_ERR_INVALID_ARG, "%s: v0 must be 8-byte aligned", who);
    if (inst->e_max < 0) return fail(QAA_ERR_NOT_READY, "%s: qaa_energy_table has not run for this instance", who);
    if (count == 0) return ok();
    qaa_status r = lanczos_lowest(inst->n, table, (int)etype, count, s_values, v0, iters, k, evals, bounds,
                                  reinterpret_cast<hipStream_t>(stream));
    if (r != QAA_OK) return r;
    return ok();
}

// ---------------------------------------------------------------------------
// Observables
// ---------------------------------------------------------------------------
extern "C" qaa_status qaa_observables(const qaa_state *st, qaa_obs *out, void *stream)
{
    TraceRange trace_range("qaa_observables");
    if (!out) return fail(QAA_ERR_INVALID_ARG, "qaa_observables: out is NULL");
    qaa_status r = check_state_table(st, "qaa_observables");
    if (r != QAA_OK) return r;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int nb = observables_blocks(st->inst->n);
    StreamScratch scr;
    scr.s = s;
    QAA_HIP(hipMallocAsync(&scr.p, sizeof(double) * (3 * (size_t)nb + 4), s));
    double *partials = reinterpret_cast<double *>(scr.p);
    double *res = partials + 3 * (size_t)nb;
    ClauseRec *recs = nullptr;       // recompute mode: energies scored from the clause records
    if (!st->table) {
        r = device_clauses(const_cast<qaa_instance *>(st->inst), &recs, "qaa_observables");
        if (r != QAA_OK) return r;
    }
    // (recompute mode: the etype argument picks the counter width, 8 planes
    // when every count is at most 255)
    const int et = st->table ? (int)st->etype : (st->inst->e_max <= 255 ? 0 : 1);
    QAA_HIP(launch_observables(st->amp, (int)st->dtype, st->table, et, recs, st->inst->m, st->inst->n,
                               st->inst->e_min, partials, nb, res, s));
    double h[3] = {0.0, 0.0, 0.0};
    QAA_HIP(hipMemcpyAsync(h, res, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    QAA_HIP(hipStreamSynchronize(s));
    out->norm = h[0];
    out->energy = h[1];
    out->p_success = h[2];
    out->e_min = st->inst->e_min;
    out->degeneracy = st->inst->degeneracy;
    return ok();
}

// ---------------------------------------------------------------------------
// Plan introspection, errors, version
// ---------------------------------------------------------------------------
extern "C" qaa_status qaa_plan_get(int32_t n, qaa_dtype dtype, qaa_plan_choice *out)
{
    if (n < 1 || n > QAA_MAX_QUBITS || (dtype != QAA_C64 && dtype != QAA_C128) || !out)
        return fail(QAA_ERR_INVALID_ARG, "qaa_plan_get: bad argument");
    PlanChoice c{0, 0, 0};
    const Plan p = make_plan(n, (int)dtype, QAA_E_U8, 0, &c);
    if (p.resident) c = default_plan_choice(1);
    out->balance = c.balance;
    out->passengers = c.passengers;
    out->tiles = c.tiles;
    return ok();
}

extern "C" qaa_status qaa_plan_set(int32_t n, qaa_dtype dtype, const qaa_plan_choice *choice)
{
    if (n < 1 || n > QAA_MAX_QUBITS || (dtype != QAA_C64 && dtype != QAA_C128))
        return fail(QAA_ERR_INVALID_ARG, "qaa_plan_set: bad argument");
    if (choice && ((choice->balance != 0 && choice->balance != 1) ||
                   (choice->passengers != 0 && choice->passengers != 1) || choice->tiles < 0 || choice->tiles > 2))
        return fail(QAA_ERR_INVALID_ARG, "qaa_plan_set: balance and passengers are 0 or 1, tiles 0, 1 or 2");
    load_autotune_cache_once();
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (choice)
        g_plan_choice[{n, (int)dtype}] = PlanChoice{choice->balance, choice->passengers, choice->tiles};
    else
        g_plan_choice.erase({n, (int)dtype});
    return ok();
}

extern "C" qaa_status qaa_plan_save(const char *path)
{
    if (!path || !path[0]) return fail(QAA_ERR_INVALID_ARG, "qaa_plan_save: no path");
    load_autotune_cache_once();
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (!write_plan_file(path)) return fail(QAA_ERR_INVALID_ARG, "qaa_plan_save: cannot write %s", path);
    return ok();
}

extern "C" qaa_status qaa_plan_load(const char *path, int32_t *count)
{
    if (!path || !path[0]) return fail(QAA_ERR_INVALID_ARG, "qaa_plan_load: no path");
    load_autotune_cache_once();
    std::lock_guard<std::mutex> lk(g_plan_mu);
    const int c = read_plan_file(path);
    if (c < 0) return fail(QAA_ERR_INVALID_ARG, "qaa_plan_load: cannot read %s", path);
    if (count) *count = c;
    return ok();
}

extern "C" qaa_status qaa_autotune(const qaa_state *scratch, int64_t steps, qaa_plan_choice *best,
                                   double *ms_per_step, void *stream)
{
    TraceRange trace_range("qaa_autotune");
    qaa_status r = check_state_table(scratch, "qaa_autotune", false);
    if (r != QAA_OK) return r;
    if (steps < 1) return fail(QAA_ERR_INVALID_ARG, "qaa_autotune: steps < 1");
    const int n = scratch->inst->n, dt = (int)scratch->dtype, et = (int)scratch->etype;
    const Plan p0 = make_plan(n, dt, et);
    std::vector<PlanChoice> cands;
    if (p0.resident || p0.sets.size() < 2) {
        cands.push_back(default_plan_choice(1));
    } else {
        const int max_tiles = wide_tiles_ok(n, dt, et) ? 2 : 0;
        for (int t = 0; t <= max_tiles; ++t)
            for (int b = 0; b <= 1; ++b)
                for (int q = 0; q <= 1; ++q) {
                    PlanChoice c{b, q, t};
                    // the passenger move applies only to three or more sets
                    if (q && make_plan_with(n, dt, et, c).sets.size() < 3) continue;
                    cands.push_back(c);
                }
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    QAA_HIP(hipEventCreate(&e0));
    QAA_HIP(hipEventCreate(&e1));
    const double T = 0.01 * (double)steps;     // the step size of the workloads
    float best_ms = 0.0f;
    PlanChoice best_c = cands[0];
    for (const PlanChoice &c : cands) {
        const qaa_plan_choice qc{c.balance, c.passengers, c.tiles};
        qaa_plan_set(n, scratch->dtype, &qc);
        r = qaa_state_init_uniform(scratch, stream);
        if (r == QAA_OK) r = qaa_evolve_range(scratch, nullptr, T, steps, 0, 1, stream);     // warm-up
        hipError_t he = r == QAA_OK ? hipEventRecord(e0, s) : hipSuccess;
        if (r == QAA_OK && he == hipSuccess) r = qaa_evolve_range(scratch, nullptr, T, steps, 0, steps, stream);
        if (r == QAA_OK && he == hipSuccess) he = hipEventRecord(e1, s);
        if (r == QAA_OK && he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (r == QAA_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (r != QAA_OK || he != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            qaa_plan_set(n, scratch->dtype, nullptr);
            return r != QAA_OK ? r : fail(QAA_ERR_DEVICE, "qaa_autotune: %s", hipGetErrorString(he));
        }
        if (&c == &cands[0] || ms < best_ms) {
            best_ms = ms;
            best_c = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const qaa_plan_choice qb{best_c.balance, best_c.passengers, best_c.tiles};
    qaa_plan_set(n, scratch->dtype, &qb);
    if (const char *cache = autotune_cache_path()) {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        if (!write_plan_file(cache)) return fail(QAA_ERR_INVALID_ARG, "qaa_autotune: cannot write the cache %s", cache);
    }
    if (best) *best = qb;
    if (ms_per_step) *ms_per_step = (double)best_ms / (double)steps;
    return ok();
}

extern "C" qaa_status qaa_plan_info(int32_t n, qaa_dtype dtype, int32_t *tile_bits, int32_t *sets,
                                    int32_t *passes_per_step)
{
    if (n < 1 || n > QAA_MAX_QUBITS) return fail(QAA_ERR_INVALID_ARG, "qaa_plan_info: n out of range");
    if (dtype != QAA_C64 && dtype != QAA_C128) return fail(QAA_ERR_INVALID_ARG, "qaa_plan_info: bad dtype");
    const Plan p = make_plan(n, (int)dtype, QAA_E_U8);
    if (tile_bits) *tile_bits = p.resident ? 0 : p.tile_bits;
    if (sets) *sets = p.resident ? 1 : (int32_t)p.sets.size();
    if (passes_per_step) *passes_per_step = p.resident ? 0 : (int32_t)p.sets.size() - 1;
    return ok();
}

extern "C" qaa_status qaa_debug_pass_descs(int32_t n, qaa_dtype dtype, int32_t emax, const qaa_schedule *sched,
                                           double T, int64_t steps, int64_t k0, int64_t k1, int32_t tile_bits,
                                           void *out, int32_t capacity, int32_t *count, int32_t *desc_bytes)
{
    if (n < 1 || n > QAA_MAX_QUBITS) return fail(QAA_ERR_INVALID_ARG, "qaa_debug_pass_descs: n out of range");
    if (dtype != QAA_C64 && dtype != QAA_C128) return fail(QAA_ERR_INVALID_ARG, "qaa_debug_pass_descs: bad dtype");
    // a replayed tile keeps >= 4 thread-index bits (the low four carry the
    // contiguous runs) and room for one rotated qubit beside the passengers
    if (tile_bits != 0 && (tile_bits < kPassRegBits[dtype] + 4 || tile_bits > kPassTileBits[dtype]))
        return fail(QAA_ERR_INVALID_ARG, "qaa_debug_pass_descs: tile_bits must be 0 or in %d..%d",
                    kPassRegBits[dtype] + 4, kPassTileBits[dtype]);
    if (steps < 0 || k0 < 0 || k1 < k0 || k1 > steps || !count)
        return fail(QAA_ERR_INVALID_ARG, "qaa_debug_pass_descs: bad step range");
    if (desc_bytes) *desc_bytes = (int32_t)sizeof(PassDesc);
    SchedKnots sc;
    qaa_status r = to_knots(sched, &sc, "qaa_debug_pass_descs");
    if (r != QAA_OK) return r;
    const Plan p = make_plan(n, (int)dtype, QAA_E_U8, tile_bits);
    if (p.resident || k0 == k1) {
        *count = 0;
        return ok();
    }
    const std::vector<PassDesc> ps = plan_passes(p, n, (int)dtype, emax, sc, T, steps, k0, k1);
    *count = (int32_t)ps.size();
    if (out && capacity > 0)
        std::memcpy(out, ps.data(), sizeof(PassDesc) * std::min<size_t>(ps.size(), (size_t)capacity));
    return ok();
}

extern "C" qaa_status qaa_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return ok();
}

extern "C" qaa_status qaa_profile_read(qaa_profile *out, int32_t reset)
{
    if (!out) return fail(QAA_ERR_INVALID_ARG, "qaa_profile_read: out is NULL");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    QAA_HIP(prof_drain(true));
    out->launches = g_prof_launches;
    out->kernel_ms = g_prof_ms;
    out->min_ms = g_prof_min;
    out->max_ms = g_prof_max;
    out->alg_bytes = g_prof_bytes;
    if (reset) {
        g_prof_launches = 0;
        g_prof_ms = g_prof_min = g_prof_max = g_prof_bytes = 0.0;
    }
    return ok();
}

extern "C" const char *qaa_status_str(qaa_status s)
{
    switch (s) {
    case QAA_OK: return "ok";
    case QAA_ERR_INVALID_ARG: return "invalid argument";
    case QAA_ERR_UNSUPPORTED: return "unsupported";
    case QAA_ERR_OUT_OF_MEMORY: return "out of memory";
    case QAA_ERR_DEVICE: return "device error";
    case QAA_ERR_NOT_READY: return "not ready";
    case QAA_ERR_INTERNAL: return "internal error";
    case QAA_ERR_CANCELLED: return "cancelled";
    }
    return "unknown status";
}

extern "C" const char *qaa_last_error(void) { return g_last_error.c_str(); }

extern "C" int32_t qaa_version(void) { return 100; }
