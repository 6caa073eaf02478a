// Serving form of libnpm (include/npm_serve.h): resident sessions, a scheduler
// thread that forms rounds of requests while earlier rounds run, persistent
// multi-session kernels per round, and a completion thread that stamps
// latencies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "npm_internal.h"
#include "npm_serve.h"
#include "serve_internal.h"

using namespace npm;

namespace {

double now_us()
{
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

npm_status sfail(npm_status st, const std::string &m)
{
    npm::set_error(m.c_str());
    return st;
}

struct Request {
    uint64_t id = 0;
    int32_t sid = 0;
    int32_t kind = 0;            // 0 query, 1 train
    int64_t n = 0;
    const float *pos = nullptr, *dir = nullptr, *rad = nullptr, *spdf = nullptr;
    float *lobes = nullptr, *pdf = nullptr, *sdir = nullptr, *spdf_out = nullptr;
    double *stats = nullptr;
    uint64_t seed = 0;
    uint32_t stream_id = 0;
    double submit_us = 0, launch_us = 0, done_us = 0;
    int64_t round = -1;
    bool done = false;
    bool failed = false;
};

struct Session {
    npm_ctx *ctx = nullptr;
    bool alive = false;
    bool reserved = false;       // taken by a create still allocating its context
    bool shared = false;         // served by the persistent kernels
    int64_t bytes = 0;
    int64_t outstanding = 0;     // submitted, not yet completed
};

struct Round {
    int64_t id;
    std::vector<uint64_t> reqs;
    hipEvent_t done_ev = nullptr;
    int slot = -1;               // descriptor buffer used
    double launch_us = 0;
    bool failed = false;
};

constexpr int kSlots = 4;        // descriptor buffers, i.e. rounds in flight

}  // namespace

struct npm_server {
    npm_server_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_slot;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Request> reqs;
    std::vector<Session> sessions;
    std::deque<Round> inflight;
    std::condition_variable cv_inflight;
    bool slot_busy[kSlots] = {false, false, false, false};
    RoundBuffers bufs[kSlots];
    uint64_t next_id = 1;
    int64_t next_round = 0;
    int64_t bytes_in_use = 0;
    npm_server_stats stats{};
    bool stop = false;
    bool held = false;            // npm_server_hold: no round is formed
    std::thread sched, completer;
};

namespace {

// Forms the next round from the pending queue (lock held): requests in
// arrival order; per session order is kept (a request is skipped, and the
// session blocked for this round, once an earlier request of the session
// could not join); at most one training batch per session, and nothing of
// that session after it; at most round_vertices vertices, except that the
// first request always joins.
std::vector<uint64_t> form_round(npm_server *s)
{
    std::vector<uint64_t> out;
    std::vector<char> blocked(s->sessions.size(), 0);
    int64_t verts = 0;
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        Request &r = s->reqs[*it];
        if (blocked[r.sid] || (int)out.size() >= kMaxRoundRequests) {
            blocked[r.sid] = 1;
            ++it;
            continue;
        }
        if (!out.empty() && verts + r.n > s->cfg.round_vertices) {
            blocked[r.sid] = 1;
            ++it;
            continue;
        }
        out.push_back(r.id);
        verts += r.n;
        if (r.kind == 1) blocked[r.sid] = 1;     // later requests of this session wait
        it = s->pending.erase(it);
    }
    return out;
}

// The per-session path: each request through its session's own calls.
hipError_t execute_plain(const std::vector<ServeRequest> &work, hipStream_t stream)
{
    for (const ServeRequest &r : work) {
        npm_status st;
        if (r.kind == 0)
            st = npm_query(r.ctx, r.n, r.pos, r.dir, r.seed, r.stream_id, r.lobes, r.pdf, r.sdir,
                           r.spdf_out, stream);
        else
            st = npm_train_step(r.ctx, r.n, r.pos, r.dir, r.rad, r.spdf, r.stats, stream);
        if (st != NPM_OK) return hipErrorUnknown;
    }
    return hipSuccess;
}

void scheduler(npm_server *s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_sched.wait(lk, [&] { return s->stop || (!s->pending.empty() && !s->held); });
        if (s->pending.empty() && s->stop) break;
        // a free descriptor buffer (bounds the rounds in flight)
        int slot = -1;
        s->cv_slot.wait(lk, [&] {
            for (int i = 0; i < kSlots; ++i) if (!s->slot_busy[i]) { slot = i; return true; }
            return false;
        });
        std::vector<uint64_t> ids = form_round(s);
        if (ids.empty()) continue;
        s->slot_busy[slot] = true;
        Round rd;
        rd.id = s->next_round++;
        rd.reqs = ids;
        rd.slot = slot;
        rd.launch_us = now_us();
        for (uint64_t id : ids) {
            Request &r = s->reqs[id];
            r.round = rd.id;
            r.launch_us = rd.launch_us;
        }
        // snapshot of what the launch needs, then launch without the lock
        std::vector<ServeRequest> work;
        std::vector<npm_ctx *> trained;
        bool plain = s->cfg.plain_path != 0;
        for (uint64_t id : ids) {
            const Request &r = s->reqs[id];
            const Session &se = s->sessions[r.sid];
            if (!se.shared) plain = true;
            ServeRequest w{};
            w.kind = r.kind;
            w.n = r.n;
            w.pos = r.pos; w.dir = r.dir; w.rad = r.rad; w.spdf = r.spdf;
            w.lobes = r.lobes; w.pdf = r.pdf; w.sdir = r.sdir; w.spdf_out = r.spdf_out;
            w.stats = r.stats;
            w.seed = r.seed;
            w.stream_id = r.stream_id;
            w.ctx = se.ctx;
            w.session = r.sid;
            work.push_back(w);
        }
        lk.unlock();
        const hipError_t e = plain ? execute_plain(work, s->stream)
                                   : serve_launch_round(&s->bufs[slot], work, s->stream);
        // The event follows whatever part of the round did launch (also when
        // a later launch failed): the completion thread releases the round's
        // descriptor buffer only after the device has passed it.  Without an
        // event the stream is drained here instead.
        hipEvent_t ev = nullptr;
        hipError_t ee = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (ee == hipSuccess) ee = hipEventRecord(ev, s->stream);
        if (ee != hipSuccess) {
            if (ev) (void)hipEventDestroy(ev);
            ev = nullptr;
            (void)hipStreamSynchronize(s->stream);   // the round is marked failed either way
        }
        lk.lock();
        rd.failed = e != hipSuccess || ee != hipSuccess;
        rd.done_ev = ev;
        s->inflight.push_back(rd);
        s->cv_inflight.notify_all();
    }
    s->inflight.push_back(Round{-1, {}, nullptr, -1, 0});   // completion thread: end
    s->cv_inflight.notify_all();
}

void completer(npm_server *s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_inflight.wait(lk, [&] { return !s->inflight.empty(); });
        Round rd = s->inflight.front();
        s->inflight.pop_front();
        if (rd.id < 0) break;
        lk.unlock();
        if (rd.done_ev) {
            // a round whose work the device did not complete fails its requests
            if (hipEventSynchronize(rd.done_ev) != hipSuccess) rd.failed = true;
            (void)hipEventDestroy(rd.done_ev);
        }
        const double t = now_us();
        lk.lock();
        for (uint64_t id : rd.reqs) {
            Request &r = s->reqs[id];
            r.done = true;
            r.failed = rd.failed;
            r.done_us = t;
            s->sessions[r.sid].outstanding -= 1;
            s->stats.requests_done += 1;
            s->stats.vertices_done += r.n;
        }
        s->stats.rounds += 1;
        s->stats.busy_us += t - rd.launch_us;
        s->slot_busy[rd.slot] = false;
        s->cv_slot.notify_all();
        s->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

npm_status npm_server_create(const npm_server_config *cfg, npm_server **out)
{
    if (!cfg || !out) return sfail(NPM_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (cfg->budget_bytes <= 0 || cfg->max_sessions < 1 || cfg->max_sessions > 256 ||
        cfg->round_vertices < 1024)
        return sfail(NPM_ERR_INVALID_ARG, "invalid server config");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return sfail(NPM_ERR_NO_DEVICE, "no HIP device");
    npm_server *s = new (std::nothrow) npm_server();
    if (!s) return sfail(NPM_ERR_OOM, "host allocation");
    s->cfg = *cfg;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    for (int i = 0; i < kSlots && e == hipSuccess; ++i) e = round_buffers_init(&s->bufs[i]);
    if (e != hipSuccess) {
        for (int i = 0; i < kSlots; ++i) round_buffers_free(&s->bufs[i]);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return sfail(NPM_ERR_HIP, std::string("server create: ") + hipGetErrorString(e));
    }
    s->sessions.resize(cfg->max_sessions);
    s->sched = std::thread(scheduler, s);
    s->completer = std::thread(completer, s);
    *out = s;
    return NPM_OK;
}

npm_status npm_server_hold(npm_server *s, int32_t hold)
{
    if (!s) return sfail(NPM_ERR_INVALID_ARG, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->held = hold != 0;
    }
    s->cv_sched.notify_all();
    return NPM_OK;
}

npm_status npm_drain(npm_server *s)
{
    if (!s) return sfail(NPM_ERR_INVALID_ARG, "null server");
    npm_server_hold(s, 0);
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] {
        for (auto &kv : s->reqs) if (!kv.second.done) return false;
        return true;
    });
    return NPM_OK;
}

npm_status npm_server_destroy(npm_server *s)
{
    if (!s) return NPM_OK;
    npm_drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    s->sched.join();
    s->completer.join();
    (void)hipStreamSynchronize(s->stream);
    for (auto &se : s->sessions)
        if (se.alive) npm_destroy(se.ctx);
    for (int i = 0; i < kSlots; ++i) round_buffers_free(&s->bufs[i]);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return NPM_OK;
}

npm_status npm_session_create(npm_server *s, const npm_config *cfg, int32_t *sid)
{
    if (!s || !cfg || !sid) return sfail(NPM_ERR_INVALID_ARG, "null argument");
    npm_config c = *cfg;
    if (c.sh_degree != 0)
        return sfail(NPM_ERR_INVALID_ARG, "sessions take radiance-based networks (sh_degree 0)");
    if (c.learn_selection != 0)
        return sfail(NPM_ERR_INVALID_ARG, "sessions take networks without the selection output");
    const bool shared = s->cfg.plain_path == 0 && c.precision == NPM_PREC_BF16 &&
                        serve_supports(&c);
    if (s->cfg.plain_path) {
        c.precision = NPM_PREC_FP32;
        c.exec_mode = NPM_EXEC_STAGED;
    }
    npm_layout lay;
    npm_status st = npm_get_layout(&c, &lay);
    if (st != NPM_OK) return st;
    const int64_t bytes = lay.device_bytes;
    std::unique_lock<std::mutex> lk(s->mu);
    int slot = -1;
    for (int i = 0; i < (int)s->sessions.size(); ++i)
        if (!s->sessions[i].alive && !s->sessions[i].reserved) { slot = i; break; }
    if (slot < 0) return sfail(NPM_ERR_BUDGET, "no free session slot");
    if (s->bytes_in_use + bytes > s->cfg.budget_bytes)
        return sfail(NPM_ERR_BUDGET, "session does not fit the HBM budget");
    // the slot and the bytes are taken before the (slow) allocation, so that
    // a concurrent create picks another slot
    s->bytes_in_use += bytes;
    s->sessions[slot].reserved = true;
    lk.unlock();
    npm_ctx *ctx = nullptr;
    st = npm_create(&c, &ctx);
    lk.lock();
    Session &se = s->sessions[slot];
    se.reserved = false;
    if (st != NPM_OK) {
        s->bytes_in_use -= bytes;
        return st;
    }
    se.ctx = ctx;
    se.alive = true;
    se.shared = shared;
    se.bytes = bytes;
    se.outstanding = 0;
    s->stats.sessions += 1;
    *sid = slot;
    return NPM_OK;
}

npm_status npm_session_destroy(npm_server *s, int32_t sid)
{
    if (!s) return sfail(NPM_ERR_INVALID_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    if (sid < 0 || sid >= (int)s->sessions.size() || !s->sessions[sid].alive)
        return sfail(NPM_ERR_INVALID_ARG, "no such session");
    s->cv_done.wait(lk, [&] { return s->sessions[sid].outstanding == 0; });
    Session &se = s->sessions[sid];
    npm_ctx *ctx = se.ctx;
    se.alive = false;
    se.ctx = nullptr;
    s->bytes_in_use -= se.bytes;
    s->stats.sessions -= 1;
    lk.unlock();
    (void)hipStreamSynchronize(s->stream);   // npm_destroy synchronises the device as well
    return npm_destroy(ctx);
}

npm_status npm_session_ctx(npm_server *s, int32_t sid, npm_ctx **ctx)
{
    if (!s || !ctx) return sfail(NPM_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (sid < 0 || sid >= (int)s->sessions.size() || !s->sessions[sid].alive)
        return sfail(NPM_ERR_INVALID_ARG, "no such session");
    *ctx = s->sessions[sid].ctx;
    return NPM_OK;
}

static npm_status submit(npm_server *s, Request r, uint64_t *req)
{
    if (!s || !req) return sfail(NPM_ERR_INVALID_ARG, "null argument");
    if (r.n < 0 || r.n > ((int64_t)1 << 31) - 1) return sfail(NPM_ERR_INVALID_ARG, "n out of range");
    if (r.n > 0 && !r.pos) return sfail(NPM_ERR_INVALID_ARG, "pos required");
    if (r.kind == 0 && r.pdf && !r.dir) return sfail(NPM_ERR_INVALID_ARG, "pdf needs dir");
    if (r.kind == 1 && r.n > 0 && (!r.dir || !r.rad || !r.spdf))
        return sfail(NPM_ERR_INVALID_ARG, "dir, radiance and sampling_pdf are required");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return sfail(NPM_ERR_STATE, "server stopping");
    if (r.sid < 0 || r.sid >= (int)s->sessions.size() || !s->sessions[r.sid].alive)
        return sfail(NPM_ERR_INVALID_ARG, "no such session");
    r.id = s->next_id++;
    r.submit_us = now_us();
    s->reqs[r.id] = r;
    s->sessions[r.sid].outstanding += 1;
    s->pending.push_back(r.id);
    *req = r.id;
    s->cv_sched.notify_one();
    return NPM_OK;
}

npm_status npm_submit_query(npm_server *s, int32_t sid, int64_t n, const float *pos,
                            const float *dir, uint64_t rng_seed, uint32_t rng_stream,
                            float *lobes, float *pdf, float *sample_dir, float *sample_pdf,
                            uint64_t *req)
{
    Request r;
    r.sid = sid; r.kind = 0; r.n = n;
    r.pos = pos; r.dir = dir;
    r.lobes = lobes; r.pdf = pdf; r.sdir = sample_dir; r.spdf_out = sample_pdf;
    r.seed = rng_seed; r.stream_id = rng_stream;
    return submit(s, r, req);
}

npm_status npm_submit_train(npm_server *s, int32_t sid, int64_t n, const float *pos,
                            const float *dir, const float *radiance, const float *sampling_pdf,
                            double *stats_out, uint64_t *req)
{
    Request r;
    r.sid = sid; r.kind = 1; r.n = n;
    r.pos = pos; r.dir = dir; r.rad = radiance; r.spdf = sampling_pdf;
    r.stats = stats_out;
    return submit(s, r, req);
}

npm_status npm_wait(npm_server *s, uint64_t req, int64_t timeout_us)
{
    if (!s) return sfail(NPM_ERR_INVALID_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req);
    if (it == s->reqs.end()) return sfail(NPM_ERR_INVALID_ARG, "unknown request");
    auto ready = [&] { return s->reqs[req].done; };
    if (timeout_us < 0 && s->held && s->reqs[req].round < 0)
        return sfail(NPM_ERR_STATE, "the server is held and the request not yet in a round: "
                                    "release it (npm_server_hold 0) before waiting");
    if (timeout_us < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
        return sfail(NPM_ERR_TIMEOUT, "request not complete");
    if (s->reqs[req].failed) return sfail(NPM_ERR_HIP, "the request's round failed to launch");
    return NPM_OK;
}

npm_status npm_request_info_get(npm_server *s, uint64_t req, npm_request_info *out)
{
    if (!s || !out) return sfail(NPM_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req);
    if (it == s->reqs.end()) return sfail(NPM_ERR_INVALID_ARG, "unknown request");
    const Request &r = it->second;
    if (!r.done) return sfail(NPM_ERR_STATE, "request not complete");
    out->submit_us = r.submit_us;
    out->launch_us = r.launch_us;
    out->done_us = r.done_us;
    out->round = r.round;
    out->n = r.n;
    out->kind = r.kind;
    out->session = r.sid;
    return NPM_OK;
}

npm_status npm_server_stats_get(npm_server *s, npm_server_stats *out)
{
    if (!s || !out) return sfail(NPM_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->bytes_in_use = s->bytes_in_use;
    return NPM_OK;
}

}  // extern "C"
