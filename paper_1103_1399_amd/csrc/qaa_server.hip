// qaa_server.hip -- solve-request server behind the qaa_server_* C ABI.
//
// Requests (a clause list, T and a step count) are admitted in arrival
// order when a worker slot is free and their HBM footprint fits the budget
// (qaa_server_footprint: complex64 state, energy table, clause records and
// the library's per-call scratch).  Each slot owns
// a HIP stream and runs the whole solve on it (energy table, uniform start,
// the steps in chunks, observables), so solves admitted while others are running
// overlap on the device and share it kernel by kernel.  Results do not
// depend on what else runs: every kernel is deterministic and works only on
// its request's buffers.
#include "qaa.h"
#include "qaa_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    int64_t id = 0;
    int32_t n = 0;
    std::vector<int32_t> lits;
    std::vector<double> knots;   // schedule table (empty: linear)
    double T = 0.0;
    int64_t steps = 0;
    int64_t steps_done = 0;      // steps the device has finished (updated per chunk)
    size_t footprint = 0;
    int state = 0;               // 0 queued, 1 running, 2 done, 3 failed or cancelled
    bool cancel = false;         // stop at the next chunk boundary
    qaa_status status = QAA_OK;
    std::string error;
    qaa_obs obs{};
    double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
};

}  // namespace

struct qaa_server {
    qaa_server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work;   // workers wait for admissible requests
    std::condition_variable cv_done;   // clients wait for completions
    std::deque<int64_t> queue;
    std::map<int64_t, Request> reqs;
    size_t in_use = 0;
    int64_t next_id = 1;
    bool stop = false;
    std::vector<std::thread> workers;
};

namespace {

// Device memory a solve can hold at once: the complex64 state, the energy
// table (uint8, or uint16 when the clause count allows counts above 255:
// the solve widens the table only then), the instance's clause records and
// the per-call reduction scratch of the library (observables partials and
// counters, under 64 KiB).
size_t footprint_of(int32_t n, int32_t m)
{
    const size_t dim = size_t(1) << n;
    return dim * 8 + dim * (m > 255 ? 2 : 1) + sizeof(qaa::ClauseRec) * (size_t)m + (size_t(64) << 10);
}

// Steps evolved per qaa_evolve_range call of a solve: about a tenth to a
// quarter of a second of device time at large n, the whole solve at small
// n.  The worker waits for each chunk and records the steps done, which
// qaa_server_poll reports; a chunk boundary costs one extra half-phase
// pass, under 1 % at these sizes.
int64_t chunk_steps(int32_t n)
{
    return n >= 29 ? 64 : (int64_t(1) << (35 - n));
}

// Run one solve on the worker's stream; returns a status and message.
// progress(k) is called with the steps finished after each chunk and
// returns false when the request has been cancelled.
template <typename Progress>
qaa_status solve(Request &rq, hipStream_t s, std::string &err, Progress &&progress)
{
    qaa_instance *inst = nullptr;
    qaa_status st = qaa_instance_create(rq.n, (int32_t)(rq.lits.size() / 3), rq.lits.data(), &inst);
    if (st != QAA_OK) {
        err = qaa_last_error();
        return st;
    }
    const size_t dim = size_t(1) << rq.n;
    void *amp = nullptr, *table = nullptr;
    hipError_t he = hipMallocAsync(&amp, dim * 8, s);
    if (he == hipSuccess) he = hipMallocAsync(&table, dim, s);
    if (he != hipSuccess) {
        err = std::string("device allocation failed: ") + hipGetErrorString(he);
        if (amp) (void)hipFreeAsync(amp, s);
        qaa_instance_destroy(inst);
        return QAA_ERR_OUT_OF_MEMORY;
    }
    qaa_etype et = QAA_E_U8;
    st = qaa_energy_table(inst, table, QAA_E_U8, s);
    if (st == QAA_ERR_UNSUPPORTED) {      // E_max > 255: widen the table
        (void)hipFreeAsync(table, s);
        table = nullptr;
        he = hipMallocAsync(&table, dim * 2, s);
        st = he == hipSuccess ? qaa_energy_table(inst, table, QAA_E_U16, s) : QAA_ERR_OUT_OF_MEMORY;
        et = QAA_E_U16;
    }
    if (st == QAA_OK) {
        qaa_state state{inst, amp, QAA_C64, table, et};
        st = qaa_state_init_uniform(&state, s);
        const qaa_schedule sched{rq.knots.empty() ? QAA_SCHED_LINEAR : QAA_SCHED_TABLE, (int32_t)rq.knots.size(),
                                 rq.knots.empty() ? nullptr : rq.knots.data()};
        const int64_t chunk = chunk_steps(rq.n);
        for (int64_t k0 = 0; st == QAA_OK && k0 < rq.steps; k0 += chunk) {
            const int64_t k1 = std::min(rq.steps, k0 + chunk);
            st = qaa_evolve_range(&state, &sched, rq.T, rq.steps, k0, k1, s);
            if (st == QAA_OK && k1 < rq.steps) {
                if (hipStreamSynchronize(s) != hipSuccess) {
                    st = QAA_ERR_DEVICE;
                    err = "stream synchronisation failed";
                    break;
                }
                if (!progress(k1)) {
                    st = QAA_ERR_CANCELLED;
                    err = "cancelled";
                }
            }
        }
        if (st == QAA_OK) st = qaa_observables(&state, &rq.obs, s);
    }
    if (st != QAA_OK && err.empty()) err = qaa_last_error();
    if (amp) (void)hipFreeAsync(amp, s);
    if (table) (void)hipFreeAsync(table, s);
    (void)hipStreamSynchronize(s);
    qaa_instance_destroy(inst);
    return st;
}

void worker_main(qaa_server *sv)
{
    (void)hipSetDevice(sv->device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        // admit the request at the head of the queue once its footprint fits
        sv->cv_work.wait(lk, [&] {
            if (sv->stop) return true;
            if (sv->queue.empty()) return false;
            const Request &h = sv->reqs[sv->queue.front()];
            return sv->in_use + h.footprint <= sv->cfg.hbm_budget_bytes;
        });
        if (sv->stop) break;
        const int64_t id = sv->queue.front();
        sv->queue.pop_front();
        Request &rq = sv->reqs[id];
        rq.state = 1;
        rq.t_start = now_s();
        sv->in_use += rq.footprint;
        Request work = rq;                 // solve on a copy, outside the lock
        lk.unlock();
        std::string err;
        auto progress = [&](int64_t k) {
            std::lock_guard<std::mutex> g(sv->mu);
            Request &r = sv->reqs[id];
            r.steps_done = k;
            return !r.cancel;
        };
        const qaa_status st = s ? solve(work, s, err, progress) : QAA_ERR_DEVICE;
        if (!s) err = "worker stream could not be created";
        lk.lock();
        Request &done = sv->reqs[id];
        done.status = st;
        done.error = err;
        done.obs = work.obs;
        done.t_done = now_s();
        done.state = st == QAA_OK ? 2 : 3;
        if (st == QAA_OK) done.steps_done = done.steps;
        std::vector<int32_t>().swap(done.lits);    // finished records keep only their results
        std::vector<double>().swap(done.knots);
        sv->in_use -= done.footprint;
        sv->cv_work.notify_all();
        sv->cv_done.notify_all();
    }
    lk.unlock();
    if (s) (void)hipStreamDestroy(s);
}

}  // namespace

extern "C" qaa_status qaa_server_create(const qaa_server_config *cfg, qaa_server **out)
{
    if (!cfg || !out) return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_create: NULL argument");
    *out = nullptr;
    if (cfg->slots < 1 || cfg->slots > 64)
        return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_create: slots outside [1, 64]");
    if (cfg->hbm_budget_bytes == 0) return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_create: zero budget");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return qaa::set_error(QAA_ERR_DEVICE, "qaa_server_create: no device");
    qaa_server *sv = new (std::nothrow) qaa_server();
    if (!sv) return qaa::set_error(QAA_ERR_OUT_OF_MEMORY, "qaa_server_create: host allocation failed");
    sv->cfg = *cfg;
    sv->device = dev;
    try {
        for (int i = 0; i < cfg->slots; ++i) sv->workers.emplace_back(worker_main, sv);
    } catch (...) {
        qaa_server_destroy(sv);
        return qaa::set_error(QAA_ERR_OUT_OF_MEMORY, "qaa_server_create: could not start worker threads");
    }
    *out = sv;
    return qaa::set_error(QAA_OK, nullptr);
}

extern "C" qaa_status qaa_server_submit(qaa_server *sv, int32_t n, int32_t m, const int32_t *lits,
                                        const qaa_schedule *sched, double T, int64_t steps, int64_t *ticket)
{
    if (!sv || !ticket) return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_submit: NULL argument");
    if (n < 1 || n > QAA_MAX_QUBITS || m < 0 || (m > 0 && !lits) || !(T >= 0.0) || steps < 0)
        return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_submit: malformed request");
    qaa::SchedKnots sc;
    if (qaa::to_knots(sched, &sc, "qaa_server_submit") != QAA_OK) return QAA_ERR_INVALID_ARG;
    const size_t fp = footprint_of(n, m);
    if (fp > sv->cfg.hbm_budget_bytes)    // could never be admitted
        return qaa::set_error(QAA_ERR_OUT_OF_MEMORY, "qaa_server_submit: footprint exceeds the HBM budget");
    std::lock_guard<std::mutex> lk(sv->mu);
    Request rq;
    rq.id = sv->next_id++;
    rq.n = n;
    rq.lits.assign(lits, lits + 3 * (size_t)m);
    rq.knots.assign(sc.v, sc.v + sc.count);
    rq.T = T;
    rq.steps = steps;
    rq.footprint = fp;
    rq.t_submit = now_s();
    sv->reqs[rq.id] = rq;
    sv->queue.push_back(rq.id);
    *ticket = rq.id;
    sv->cv_work.notify_all();
    return qaa::set_error(QAA_OK, nullptr);
}

extern "C" uint64_t qaa_server_footprint(int32_t n, int32_t m)
{
    if (n < 1 || n > QAA_MAX_QUBITS || m < 0 || m > 65535) return 0;
    return (uint64_t)footprint_of(n, m);
}

namespace {

void fill_result(const Request &rq, qaa_server_result *out)
{
    out->status = rq.state == 2 ? QAA_OK : rq.status;
    out->done = rq.state >= 2 ? 1 : 0;
    out->obs = rq.obs;
    out->queued_s = (rq.state >= 1 ? rq.t_start : now_s()) - rq.t_submit;
    out->latency_s = (rq.state >= 2 ? rq.t_done : now_s()) - rq.t_submit;
    out->steps = rq.steps;
    out->steps_done = rq.steps_done;
}

}  // namespace

extern "C" qaa_status qaa_server_poll(qaa_server *sv, int64_t ticket, qaa_server_result *out)
{
    if (!sv || !out) return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_poll: unknown ticket");
    fill_result(it->second, out);
    return qaa::set_error(QAA_OK, nullptr);
}

extern "C" qaa_status qaa_server_cancel(qaa_server *sv, int64_t ticket)
{
    if (!sv) return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_cancel: NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_cancel: unknown ticket");
    Request &rq = it->second;
    if (rq.state == 0) {
        for (auto q = sv->queue.begin(); q != sv->queue.end(); ++q)
            if (*q == ticket) {
                sv->queue.erase(q);
                break;
            }
        rq.state = 3;
        rq.status = QAA_ERR_CANCELLED;
        rq.error = "cancelled";
        rq.t_start = rq.t_done = now_s();
        std::vector<int32_t>().swap(rq.lits);
        std::vector<double>().swap(rq.knots);
        sv->cv_work.notify_all();     // the next request may be admissible now
        sv->cv_done.notify_all();
    } else if (rq.state == 1) {
        rq.cancel = true;
    }
    return qaa::set_error(QAA_OK, nullptr);
}

extern "C" qaa_status qaa_server_wait(qaa_server *sv, int64_t ticket, qaa_server_result *out)
{
    if (!sv || !out) return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_wait: NULL argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_wait: unknown ticket");
    Request &rq = it->second;    // std::map references stay valid while other entries are added
    sv->cv_done.wait(lk, [&] { return rq.state >= 2; });
    fill_result(rq, out);
    return qaa::set_error(QAA_OK, nullptr);
}

extern "C" qaa_status qaa_server_stats(qaa_server *sv, int64_t *queued, int64_t *running, uint64_t *bytes_in_use)
{
    if (!sv) return qaa::set_error(QAA_ERR_INVALID_ARG, "qaa_server_stats: NULL server");
    std::lock_guard<std::mutex> lk(sv->mu);
    int64_t q = 0, r = 0;
    for (auto &kv : sv->reqs) {
        if (kv.second.state == 0) ++q;
        if (kv.second.state == 1) ++r;
    }
    if (queued) *queued = q;
    if (running) *running = r;
    if (bytes_in_use) *bytes_in_use = sv->in_use;
    return qaa::set_error(QAA_OK, nullptr);
}

extern "C" void qaa_server_destroy(qaa_server *sv)
{
    if (!sv) return;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        // let admitted solves finish; queued ones are dropped
        sv->queue.clear();
        sv->stop = true;
        sv->cv_work.notify_all();
    }
    for (auto &t : sv->workers) t.join();
    delete sv;
}
