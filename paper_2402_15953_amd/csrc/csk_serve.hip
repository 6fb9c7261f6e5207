// Serving loop: live sketches resident in HBM, insert/delete update batches and
// estimate requests executed as they arrive (continuous batching).
//
// Semantics: an estimate of query q reflects exactly the updates of q submitted before
// it, whatever else shares the GPU.  Requests are taken in arrival order and cut into
// epochs: an epoch ends before an update of a query that already has an estimate in
// the epoch.  The scheduler thread launches each epoch's updates as ONE batched
// persistent launch (round robin over the server's update streams) and hands the
// epoch's estimates to the estimate thread, together with the event of the last launch
// that touched each query.  The estimate thread gathers every pending estimate into
// one batched estimate on its own stream, which first waits on those events.  A later
// update of a query with an estimate still in flight waits for that estimate (per-query
// counter), so no estimate ever sees a later update.  Updates of other queries keep
// flowing while estimates run.  Completion times are taken by host callbacks on the
// streams (update) and after the estimate's result is on the host.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "csk_handle.h"
#include "csk_internal.h"

using namespace csk;

namespace {

double now_us()
{
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket;
    int32_t kind;  // 0 update, 1 estimate
    int32_t qid;
    int32_t rel;
    int32_t flags;
    const uint32_t *keys;
    const int64_t *weights;
    uint64_t n;
    double submit_us;
};

struct LiveQuery {
    cs_sketch *sk = nullptr;
    uint64_t bytes = 0;
    int inflight_estimates = 0;   // estimates handed to the estimate thread, not finished
    uint64_t pending = 0;         // submitted requests of this query not yet completed
    hipEvent_t last_update = nullptr;  // recorded behind the query's latest update launch
    int last_stream = -1;              // update stream of that launch (-1: none yet)
    bool has_update_event = false;
    bool removed = false;
};

struct EstJob {
    Request req;
};

}  // namespace

struct cs_server {
    cs_server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_est, cv_done;
    std::deque<Request> queue;
    std::deque<EstJob> est_queue;
    std::vector<cs_completion> completions;
    std::map<int32_t, LiveQuery> queries;
    int32_t next_qid = 0;
    uint64_t next_ticket = 1;
    uint64_t used_bytes = 0;
    uint64_t submitted = 0, completed = 0;
    bool stop = false;
    std::vector<hipStream_t> upd_streams;
    hipStream_t est_stream = nullptr;
    int rr = 0;
    cs_batch *upd_batch = nullptr;
    std::vector<cs_batch *> upd_batches;  // one per update stream (tables live until reuse)
    cs_batch *est_batch = nullptr;
    std::thread sched, est;
    std::string last_error;
    // statistics
    uint64_t n_update_launches = 0, n_estimate_batches = 0, n_epochs = 0;
};

namespace {

struct UpdDone {
    cs_server *S;
    std::vector<cs_completion> done;
};

// One request of query qid completed (the caller holds S->mu).
void query_request_done(cs_server *S, int32_t qid)
{
    auto it = S->queries.find(qid);
    if (it != S->queries.end() && it->second.pending > 0) it->second.pending--;
}

void on_updates_done(void *p)
{
    UpdDone *u = static_cast<UpdDone *>(p);
    const double t = now_us();
    {
        std::lock_guard<std::mutex> lk(u->S->mu);
        for (auto &c : u->done) {
            c.done_us = t;
            u->S->completions.push_back(c);
            query_request_done(u->S, c.qid);
        }
        u->S->completed += u->done.size();
    }
    u->S->cv_done.notify_all();
    delete u;
}

void scheduler_loop(cs_server *S)
{
    hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_sched.wait(lk, [&] { return S->stop || !S->queue.empty(); });
        if (S->stop && S->queue.empty()) return;
        // ---- cut one epoch from the front of the queue
        std::vector<Request> epoch;
        std::map<int32_t, bool> estimated;
        int n_up = 0;
        const int max_items = S->cfg.max_batch_items > 0 ? S->cfg.max_batch_items : 4096;
        while (!S->queue.empty()) {
            const Request &r = S->queue.front();
            if (r.kind == 0) {
                if (estimated.count(r.qid) || n_up >= max_items) break;
                ++n_up;
            } else {
                estimated[r.qid] = true;
            }
            epoch.push_back(r);
            S->queue.pop_front();
        }
        // ---- queries updated in this epoch while an estimate of theirs is in flight are
        // deferred, with all their requests of the epoch, in order
        std::map<int32_t, bool> blocked;
        for (const Request &r : epoch) {
            if (r.kind != 0) continue;
            auto it = S->queries.find(r.qid);
            if (it != S->queries.end() && it->second.inflight_estimates > 0) blocked[r.qid] = true;
        }
        std::vector<Request> ups, ests, deferred;
        for (const Request &r : epoch) {
            if (blocked.count(r.qid)) deferred.push_back(r);
            else if (r.kind == 0) ups.push_back(r);
            else ests.push_back(r);
        }
        for (auto it = deferred.rbegin(); it != deferred.rend(); ++it) S->queue.push_front(*it);
        if (ups.empty() && ests.empty()) {
            // everything waits for an estimate in flight: sleep until one finishes
            S->cv_done.wait(lk, [&] {
                if (S->stop) return true;
                for (auto &kv : blocked) {
                    auto it = S->queries.find(kv.first);
                    if (it == S->queries.end() || it->second.inflight_estimates == 0) return true;
                }
                return false;
            });
            continue;
        }
        ++S->n_epochs;
        // ---- updates: one batched launch
        if (!ups.empty()) {
            std::vector<cs_update_item> items;
            auto *done = new UpdDone{S, {}};
            const double t_start = now_us();
            for (const Request &r : ups) {
                auto it = S->queries.find(r.qid);
                cs_completion c{};
                c.ticket = r.ticket;
                c.qid = r.qid;
                c.kind = 0;
                c.submit_us = r.submit_us;
                c.start_us = t_start;
                if (it == S->queries.end() || it->second.removed) {
                    c.status = CS_EINVAL;
                } else {
                    items.push_back({it->second.sk, r.rel, r.flags, r.keys, r.weights, r.n});
                    c.status = CS_OK;
                }
                done->done.push_back(c);
            }
            const int si = S->rr++ % (int)S->upd_streams.size();
            hipStream_t st = S->upd_streams[si];
            // A query's updates run in submission order: an earlier launch of one of
            // these queries on another update stream may still be running, so this
            // launch waits for it.  The query's last-update event then covers every
            // update of the query, and an estimate waiting on it sees all of them.
            {
                std::map<int32_t, bool> waited;  // queries already waited for
                for (const Request &r : ups) {
                    auto it = S->queries.find(r.qid);
                    if (it == S->queries.end() || !it->second.has_update_event) continue;
                    if (it->second.last_stream == si || waited[r.qid]) continue;  // same stream: ordered by it
                    hipStreamWaitEvent(st, it->second.last_update, 0);
                    waited[r.qid] = true;
                }
            }
            lk.unlock();
            cs_status rc = cs_batch_update(S->upd_batches[si], items.data(), (int32_t)items.size(), st);
            lk.lock();
            if (rc != CS_OK) {
                S->last_error = cs_last_error();
                for (auto &c : done->done) c.status = rc;
            }
            ++S->n_update_launches;
            // the event every later estimate of these queries waits on
            for (const Request &r : ups) {
                auto it = S->queries.find(r.qid);
                if (it == S->queries.end()) continue;
                if (!it->second.last_update) hipEventCreateWithFlags(&it->second.last_update, hipEventDisableTiming);
                hipEventRecord(it->second.last_update, st);
                it->second.has_update_event = true;
                it->second.last_stream = si;
            }
            hipLaunchHostFunc(st, on_updates_done, done);
        }
        // ---- estimates: hand over; while one is in flight no later update of its query
        // is launched, so the query's last-update event stays the one it must wait for
        if (!ests.empty()) {
            for (const Request &r : ests) {
                auto it = S->queries.find(r.qid);
                if (it != S->queries.end()) it->second.inflight_estimates++;
                S->est_queue.push_back(EstJob{r});
            }
            S->cv_est.notify_all();
        }
    }
}

void estimate_loop(cs_server *S)
{
    hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_est.wait(lk, [&] { return S->stop || !S->est_queue.empty(); });
        if (S->stop && S->est_queue.empty()) return;
        std::vector<EstJob> jobs(S->est_queue.begin(), S->est_queue.end());
        S->est_queue.clear();
        std::vector<cs_sketch *> hs;
        std::vector<int> valid;
        std::map<int32_t, bool> waited;
        for (size_t i = 0; i < jobs.size(); ++i) {
            auto it = S->queries.find(jobs[i].req.qid);
            if (it != S->queries.end() && !it->second.removed) {
                hs.push_back(it->second.sk);
                valid.push_back((int)i);
                if (it->second.has_update_event && !waited[it->first]) {
                    hipStreamWaitEvent(S->est_stream, it->second.last_update, 0);
                    waited[it->first] = true;
                }
            }
        }
        const double t_start = now_us();
        lk.unlock();
        std::vector<cs_estimate_t> outs(hs.size());
        cs_status rc = CS_OK;
        if (!hs.empty()) rc = cs_batch_estimate(S->est_batch, hs.data(), (int32_t)hs.size(), S->est_stream,
                                                outs.data(), nullptr);
        const double t_done = now_us();
        lk.lock();
        ++S->n_estimate_batches;
        std::vector<char> ok(jobs.size(), 0);
        for (size_t v = 0; v < valid.size(); ++v) ok[valid[v]] = 1;
        size_t vi = 0;
        for (size_t i = 0; i < jobs.size(); ++i) {
            cs_completion c{};
            c.ticket = jobs[i].req.ticket;
            c.qid = jobs[i].req.qid;
            c.kind = 1;
            c.submit_us = jobs[i].req.submit_us;
            c.start_us = t_start;
            c.done_us = t_done;
            if (ok[i]) {
                c.status = rc;
                if (rc == CS_OK) c.estimate = outs[vi];
                ++vi;
            } else {
                c.status = CS_EINVAL;
            }
            S->completions.push_back(c);
            auto it = S->queries.find(jobs[i].req.qid);
            if (it != S->queries.end()) it->second.inflight_estimates--;
            query_request_done(S, jobs[i].req.qid);
        }
        if (rc != CS_OK) S->last_error = cs_last_error();
        S->completed += jobs.size();
        S->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

cs_status cs_server_create(const cs_server_config *cfg, cs_server **out)
{
    if (!out) return fail(CS_EINVAL, "null output");
    cs_server *S = new (std::nothrow) cs_server();
    if (!S) return fail(CS_ENOMEM, "host allocation failed");
    if (cfg) S->cfg = *cfg;
    if (S->cfg.n_streams <= 0) S->cfg.n_streams = 2;
    if (S->cfg.max_batch_items <= 0) S->cfg.max_batch_items = 4096;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return fail(CS_EDEVICE, "no HIP device");
    }
    for (int i = 0; i < S->cfg.n_streams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            delete S;
            return fail(CS_EDEVICE, "stream creation failed");
        }
        S->upd_streams.push_back(st);
        cs_batch *b = nullptr;
        if (cs_batch_create(&b) != CS_OK) {
            delete S;
            return CS_EDEVICE;
        }
        S->upd_batches.push_back(b);
    }
    if (hipStreamCreateWithFlags(&S->est_stream, hipStreamNonBlocking) != hipSuccess ||
        cs_batch_create(&S->est_batch) != CS_OK) {
        delete S;
        return fail(CS_EDEVICE, "estimate stream creation failed");
    }
    S->sched = std::thread(scheduler_loop, S);
    S->est = std::thread(estimate_loop, S);
    *out = S;
    return CS_OK;
}

cs_status cs_server_drain(cs_server *S)
{
    if (!S) return fail(CS_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->completed >= S->submitted; });
    return CS_OK;
}

cs_status cs_server_destroy(cs_server *S)
{
    if (!S) return CS_OK;
    cs_server_drain(S);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_sched.notify_all();
    S->cv_est.notify_all();
    if (S->sched.joinable()) S->sched.join();
    if (S->est.joinable()) S->est.join();
    hipDeviceSynchronize();
    for (auto &kv : S->queries) {
        if (kv.second.last_update) hipEventDestroy(kv.second.last_update);
        if (kv.second.sk) cs_destroy(kv.second.sk);
    }
    for (auto st : S->upd_streams) hipStreamDestroy(st);
    for (auto b : S->upd_batches) cs_batch_destroy(b);
    if (S->est_stream) hipStreamDestroy(S->est_stream);
    if (S->est_batch) cs_batch_destroy(S->est_batch);
    delete S;
    return CS_OK;
}

cs_status cs_server_add_query(cs_server *S, const cs_graph *graph, uint32_t m, uint32_t d, uint64_t seed,
                              int32_t *qid)
{
    if (!S || !qid) return fail(CS_EINVAL, "null argument");
    const uint64_t bytes = cs_sketch_bytes(graph, m, d);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->cfg.memory_budget && S->used_bytes + bytes > S->cfg.memory_budget)
            return fail(CS_EBUSY, "admission refused: sketch memory budget exhausted");
        S->used_bytes += bytes;  // reserve
    }
    cs_sketch *sk = nullptr;
    cs_status st = create_handle(graph, m, d, seed, false, &sk);
    std::lock_guard<std::mutex> lk(S->mu);
    if (st != CS_OK) {
        S->used_bytes -= bytes;
        return st;
    }
    const int32_t id = S->next_qid++;
    LiveQuery &q = S->queries[id];
    q.sk = sk;
    q.bytes = bytes;
    *qid = id;
    return CS_OK;
}

cs_status cs_server_remove_query(cs_server *S, int32_t qid)
{
    if (!S) return fail(CS_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    {
        auto it = S->queries.find(qid);
        if (it == S->queries.end()) return fail(CS_EINVAL, "unknown query");
        if (it->second.removed) return fail(CS_EINVAL, "query is already being removed");
        // later submissions of the query complete with CS_EINVAL without touching it
        it->second.removed = true;
    }
    // wait for this query's own requests only (others keep flowing); the map entry
    // stays until then, so it is looked up again after the wait
    S->cv_done.wait(lk, [&] {
        auto it = S->queries.find(qid);
        return it == S->queries.end() || it->second.pending == 0;
    });
    auto it = S->queries.find(qid);
    if (it == S->queries.end()) return fail(CS_EINVAL, "unknown query");
    LiveQuery q = it->second;
    S->queries.erase(it);
    S->used_bytes -= q.bytes;
    lk.unlock();
    // every update of the query has passed its stream (its completion callback ran) and
    // every estimate has returned; the event may still be queued behind them, so wait
    // for it before releasing the counters
    if (q.last_update) {
        hipEventSynchronize(q.last_update);
        hipEventDestroy(q.last_update);
    }
    cs_destroy(q.sk);
    return CS_OK;
}

cs_status cs_server_sketch(cs_server *S, int32_t qid, cs_sketch **out)
{
    if (!S || !out) return fail(CS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->queries.find(qid);
    if (it == S->queries.end()) return fail(CS_EINVAL, "unknown query");
    *out = it->second.sk;
    return CS_OK;
}

static cs_status submit(cs_server *S, Request r, uint64_t *ticket)
{
    std::lock_guard<std::mutex> lk(S->mu);
    auto qit = S->queries.find(r.qid);
    if (qit == S->queries.end()) return fail(CS_EINVAL, "unknown query");
    if (qit->second.removed) return fail(CS_EINVAL, "query is being removed");
    if (r.kind == 0 && r.n > 0) {
        const Handle &h = qit->second.sk->h;
        if (r.rel < 0 || r.rel >= h.g.n_rel) return fail(CS_EINVAL, "relation out of range");
        cs_status chk = check_device_array(r.keys, r.n * h.g.rel[r.rel].n_cols * sizeof(uint32_t), h.device, "keys");
        if (chk == CS_OK && r.weights)
            chk = check_device_array(r.weights, r.n * sizeof(int64_t), h.device, "weights");
        if (chk != CS_OK) return chk;
    }
    if (S->cfg.max_pending > 0 && (int64_t)(S->submitted - S->completed) >= S->cfg.max_pending)
        return fail(CS_EBUSY, "request queue full");
    r.ticket = S->next_ticket++;
    r.submit_us = now_us();
    S->queue.push_back(r);
    S->submitted++;
    qit->second.pending++;
    if (ticket) *ticket = r.ticket;
    S->cv_sched.notify_one();
    return CS_OK;
}

cs_status cs_server_submit_update(cs_server *S, int32_t qid, int32_t rel, const uint32_t *keys,
                                  const int64_t *weights, uint64_t n, int32_t flags, uint64_t *ticket)
{
    if (!S || (n > 0 && !keys)) return fail(CS_EINVAL, "null argument");
    Request r{};
    r.kind = 0;
    r.qid = qid;
    r.rel = rel;
    r.flags = flags;
    r.keys = keys;
    r.weights = weights;
    r.n = n;
    return submit(S, r, ticket);
}

cs_status cs_server_submit_estimate(cs_server *S, int32_t qid, uint64_t *ticket)
{
    if (!S) return fail(CS_EINVAL, "null server");
    Request r{};
    r.kind = 1;
    r.qid = qid;
    return submit(S, r, ticket);
}

cs_status cs_server_poll(cs_server *S, cs_completion *out, int32_t max, int32_t *n_out)
{
    if (!S || !n_out || (max > 0 && !out)) return fail(CS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    const int32_t n = (int32_t)std::min<size_t>((size_t)max, S->completions.size());
    for (int32_t i = 0; i < n; ++i) out[i] = S->completions[i];
    S->completions.erase(S->completions.begin(), S->completions.begin() + n);
    *n_out = n;
    return CS_OK;
}

cs_status cs_server_stats(cs_server *S, cs_server_stats_t *out)
{
    if (!S || !out) return fail(CS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->used_bytes = S->used_bytes;
    out->live_queries = (int32_t)S->queries.size();
    out->update_launches = S->n_update_launches;
    out->estimate_batches = S->n_estimate_batches;
    out->epochs = S->n_epochs;
    return CS_OK;
}

}  // extern "C"
