// Serving loop: requests are admitted in arrival order, skipping over ones
// whose HBM footprint does not fit yet (size-aware FIFO), while the
// footprints of the running requests stay within the context's HBM budget and
// a slot is free.  Each slot is a worker thread with its own stream (default
// priority), workspace arenas and graph cache; admitted requests run
// concurrently on the slots.  The footprint model follows the paper's memory
// accounting (section 5.3: grid plus per-source and per-output arrays),
// re-based on this library's buffers: inputs, outputs, target table and the
// NUFFT workspace of the request's frequencies.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "ctx.h"
#include "fv_internal.h"

namespace fv {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t id = 0;
    fv_problem p;
    double *vis = nullptr;
    bool dev = false;  // arrays (and vis) on the device
    size_t footprint = 0;
    Clock::time_point t_submit;
    bool done = false;
    fv_status status = FV_OK;
    std::string err;
    fv_report rep;
};

struct Server {
    fv_ctx *ctx = nullptr;
    std::vector<std::unique_ptr<Slot>> slots;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs;
    size_t in_use = 0;
    int running = 0;
    bool stopping = false, stopped = false;
    uint64_t next_id = 1;
};

// Bytes a request holds on the device while it runs (footprint_bytes, with
// the geometry plan from the context's cache).
// With src_on_host false the whole direction cube is an upper bound of the
// grid, and so of the footprint.
size_t request_footprint(fv_ctx *ctx, const fv_problem &p, bool src_on_host) {
    const int dim = choose_dim(p.ant_enu, p.n_ant, p.eps, p.freq_hz, p.n_freq, p.flags);
    const int prec = choose_prec(p.eps, p.flags);
    const size_t cap = std::max<size_t>(ctx->chunk_bytes, 1 << 20);
    GeomPlan g;
    if (p.n_src > 0 && (p.flags & FV_METHOD_MASK) == FV_METHOD_NUFFT) {
        double s_c[3] = {0, 0, 0}, S[3] = {1, 1, 1};
        if (src_on_host) src_box(p.src_lmn, p.n_src, dim, s_c, S);
        g = ctx_geometry(ctx, p.ant_enu, p.n_ant, dim, p.eps, s_c, S, !(p.flags & FV_NO_FOLD));
    }
    return footprint_bytes(p, g, dim, prec, cap);
}

namespace {

void worker(Server *S, Slot *slot) {
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        std::shared_ptr<Request> r;
        while (!S->stopping) {
            // first queued request that fits next to the running ones
            for (auto it = S->queue.begin(); it != S->queue.end(); ++it)
                if (S->in_use + (*it)->footprint <= S->ctx->budget) {
                    r = *it;
                    S->queue.erase(it);
                    break;
                }
            if (r) break;
            if (!S->queue.empty() && S->running == 0) {
                // the head can never fit: fail it rather than wait forever
                auto h = S->queue.front();
                S->queue.pop_front();
                h->done = true;
                h->status = FV_ENOMEM;
                h->err = "request footprint of " + std::to_string(h->footprint) + " bytes exceeds the HBM budget";
                S->cv_done.notify_all();
                continue;
            }
            S->cv_work.wait(lk);
        }
        if (!r) break;  // stopping
        S->in_use += r->footprint;
        ++S->running;
        lk.unlock();
        fv_status st = FV_OK;
        std::string err;
        fv_report rep;
        std::memset(&rep, 0, sizeof(rep));
        try {
            if (r->dev)
                simulate_dev_sync(S->ctx, *slot, r->p, r->vis, &rep);
            else
                simulate_host(S->ctx, *slot, &r->p, r->vis, &rep);
        } catch (const Error &e) {
            st = e.code;
            err = e.msg;
        } catch (const std::bad_alloc &) {
            st = FV_ENOMEM;
            err = "host allocation failed";
        } catch (const std::exception &e) {
            st = FV_EDEVICE;
            err = e.what();
        }
        rep.t_total_ms = std::chrono::duration<double, std::milli>(Clock::now() - r->t_submit).count();
        lk.lock();
        S->in_use -= r->footprint;
        --S->running;
        r->status = st;
        r->err = err;
        r->rep = rep;
        r->done = true;
        S->cv_done.notify_all();
        S->cv_work.notify_all();  // memory was freed: others may fit now
    }
}

void stop_server(Server *S) {
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stopped) return;
        S->stopping = true;
        for (auto &r : S->queue) {
            r->done = true;
            r->status = FV_ECANCELLED;
            r->err = "request cancelled by fv_server_stop";
        }
        S->queue.clear();
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
    for (auto &t : S->workers) t.join();
    S->workers.clear();
    S->slots.clear();
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopped = true;
}

}  // namespace

void server_free(Server *s) {
    if (!s) return;
    stop_server(s);
    delete s;
}

}  // namespace fv

using namespace fv;

#define FV_SERVER_GUARD(body)                          \
    try {                                              \
        body                                           \
    } catch (const fv::Error &e) {                     \
        fv::set_last_error(e.msg);                     \
        return e.code;                                 \
    } catch (const std::bad_alloc &) {                 \
        fv::set_last_error("host allocation failed");  \
        return FV_ENOMEM;                              \
    } catch (const std::exception &e) {                \
        fv::set_last_error(e.what());                  \
        return FV_EDEVICE;                             \
    }

extern "C" {

fv_status fv_server_start(fv_ctx *ctx, int max_slots) {
    FV_SERVER_GUARD({
        if (!ctx) fail(FV_EINVAL, "null context");
        if (max_slots < 1 || max_slots > 16) fail(FV_EINVAL, "max_slots must be in 1..16");
        if (ctx->server && !ctx->server->stopped) fail(FV_EBUSY, "server already running");
        server_free(ctx->server);
        ctx->server = nullptr;
        FV_HIP(hipSetDevice(ctx->device));
        Server *S = new Server();
        S->ctx = ctx;
        try {
            for (int i = 0; i < max_slots; ++i) {
                std::unique_ptr<Slot> sl(new Slot());
                FV_HIP(hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking));
                sl->own_stream = true;
                S->slots.push_back(std::move(sl));
            }
            for (auto &sl : S->slots) S->workers.emplace_back(worker, S, sl.get());
        } catch (...) {
            server_free(S);
            throw;
        }
        ctx->server = S;
        return FV_OK;
    })
}

}  // extern "C"

namespace {
fv_status enqueue(fv_ctx *ctx, std::shared_ptr<Request> r, uint64_t *ticket) {
    Server *S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopped || S->stopping) fail(FV_EBUSY, "server not running");
    if (S->queue.size() >= 65536) fail(FV_EBUSY, "queue full");
    r->id = S->next_id++;
    S->reqs[r->id] = r;
    S->queue.push_back(r);
    *ticket = r->id;
    S->cv_work.notify_one();
    return FV_OK;
}
}  // namespace

extern "C" {

fv_status fv_submit(fv_ctx *ctx, const fv_problem *p, double *vis, uint64_t *ticket) {
    FV_SERVER_GUARD({
        if (!ctx || !p || !vis || !ticket) fail(FV_EINVAL, "null argument");
        Server *S = ctx->server;
        if (!S || S->stopped || S->stopping) fail(FV_EBUSY, "server not running");
        validate_host(p);
        auto r = std::make_shared<Request>();
        r->p = *p;
        r->vis = vis;
        r->t_submit = Clock::now();
        r->footprint = request_footprint(ctx, *p);
        return enqueue(ctx, r, ticket);
    })
}

fv_status fv_submit_dev(fv_ctx *ctx, const fv_problem *p, double *vis, uint64_t *ticket) {
    FV_SERVER_GUARD({
        if (!ctx || !p || !ticket) fail(FV_EINVAL, "null argument");
        Server *S = ctx->server;
        if (!S || S->stopped || S->stopping) fail(FV_EBUSY, "server not running");
        check_dev_args(*p, vis);
        auto r = std::make_shared<Request>();
        r->p = *p;
        r->vis = vis;
        r->dev = true;
        r->t_submit = Clock::now();
        // the footprint needs the array and the frequencies on the host: two
        // small copies now (the full check runs on the request's slot)
        FV_HIP(hipSetDevice(ctx->device));
        std::vector<double> ant(3 * (size_t)p->n_ant);
        std::vector<double> freq((size_t)p->n_freq);
        FV_HIP(hipMemcpy(ant.data(), p->ant_enu, ant.size() * sizeof(double), hipMemcpyDeviceToHost));
        FV_HIP(hipMemcpy(freq.data(), p->freq_hz, freq.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (double a : ant)
            if (!std::isfinite(a)) fail(FV_EINVAL, "non-finite antenna position");
        for (double f : freq)
            if (!(std::isfinite(f) && f > 0)) fail(FV_EINVAL, "frequency must be finite and > 0");
        fv_problem meta = *p;
        meta.ant_enu = ant.data();
        meta.freq_hz = freq.data();
        r->footprint = request_footprint(ctx, meta, false);
        return enqueue(ctx, r, ticket);
    })
}

fv_status fv_wait(fv_ctx *ctx, uint64_t ticket, double timeout_s, fv_report *rep) {
    FV_SERVER_GUARD({
        if (!ctx) fail(FV_EINVAL, "null context");
        Server *S = ctx->server;
        if (!S) fail(FV_EBUSY, "no server");
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end()) fail(FV_EINVAL, "unknown ticket");
        std::shared_ptr<Request> r = it->second;
        auto ready = [&] { return r->done; };
        if (timeout_s < 0) {
            S->cv_done.wait(lk, ready);
        } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
            set_last_error("fv_wait timed out");
            return FV_ETIMEOUT;
        }
        S->reqs.erase(ticket);
        if (rep) *rep = r->rep;
        if (r->status != FV_OK) set_last_error(r->err);
        return r->status;
    })
}

fv_status fv_server_stop(fv_ctx *ctx) {
    FV_SERVER_GUARD({
        if (!ctx) fail(FV_EINVAL, "null context");
        if (ctx->server) stop_server(ctx->server);
        return FV_OK;
    })
}

}  // extern "C"
