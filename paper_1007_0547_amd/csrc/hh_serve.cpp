// Continuous batching of detection requests on one context.
//
// Each lane is a worker thread with a context of its own (own HIP stream,
// pool and arena): a slot.  A free lane takes the pending requests in
// arrival order while their predicted device footprint fits what the
// batches already running leave of the context's device-memory budget, runs
// them as one batch, brings every result's cells and statistics to the host
// and completes the tickets.  Requests arriving while batches run are taken
// by the next lane that is free once memory allows, so batches of different
// lanes overlap on the device.  A batch that fails as a whole is run again
// request by request, so that each request gets its own status.
#include "hh_serve.hpp"

#include <algorithm>
#include <exception>
#include <new>

#include "hh_engine.hpp"

namespace hh {

namespace {

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

template <typename F>
hh_status capture(F&& f, std::string& error)
{
    try {
        return f();
    } catch (const Error& e) {
        error = e.what;
        return e.status;
    } catch (const std::bad_alloc&) {
        error = "host allocation failed";
        return HH_ENOMEM;
    } catch (const std::exception& e) {
        error = e.what();
        return HH_EINTERNAL;
    }
}

// E * 2^depth of a request (E estimated from the edge density seen so far
// when it is not known).
double work_units(const Server* sv, const Request& r)
{
    const double e = r.points >= 0 ? (double)r.points : sv->density * (double)r.pixels;
    return std::max(1.0, e) * (double)((int64_t)1 << std::max(0, r.depth));
}

void run_lane(Server* sv, int lane)
{
    hh_ctx* c = sv->lanes[(size_t)lane];
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        int64_t batch_bytes = 0;
        double units = 0.0;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            auto predicted = [&](const Request& r) { return (int64_t)(sv->beta * work_units(sv, r)); };
            sv->work_cv.wait(lk, [&] {
                return sv->stop || (!sv->pending.empty() &&
                                    (sv->in_flight == 0 || sv->in_flight + predicted(*sv->pending.front()) <= sv->budget));
            });
            if (sv->stop) return;
            const int32_t kind = sv->pending.front()->in.kind;
            int64_t pixels = 0;
            while (!sv->pending.empty() && (int32_t)batch.size() < sv->cfg.max_batch) {
                const auto& r = sv->pending.front();
                if (r->in.kind != kind) break;   // one kind per batch
                const int64_t b = predicted(*r);
                if (!batch.empty() && (sv->in_flight + batch_bytes + b > sv->budget ||
                                       (sv->cfg.max_batch_pixels > 0 && pixels + r->pixels > sv->cfg.max_batch_pixels)))
                    break;
                r->bytes = b;
                batch_bytes += b;
                units += work_units(sv, *r);
                pixels += r->pixels;
                batch.push_back(r);
                sv->pending.pop_front();
            }
            sv->in_flight += batch_bytes;
            if (!sv->pending.empty()) sv->work_cv.notify_one();   // another lane may take the rest
        }
        const Clock::time_point t_start = Clock::now();
        const int32_t n = (int32_t)batch.size();
        std::vector<hh_input> ins((size_t)n);
        for (int32_t k = 0; k < n; ++k) ins[(size_t)k] = batch[(size_t)k]->in;
        std::vector<hh_result*> outs((size_t)n, nullptr);
        std::vector<hh_status> status((size_t)n, HH_OK);
        std::vector<std::string> error((size_t)n);
        {
            std::lock_guard<std::mutex> g(c->mu);
            std::string err;
            hh_status st = capture([&] { return engine_detect_batch(c, ins.data(), n, outs.data()); }, err);
            if (st == HH_OK) {
                for (int32_t k = 0; k < n; ++k) {
                    status[(size_t)k] = capture([&] { return engine_host_cells(outs[(size_t)k]); }, error[(size_t)k]);
                }
            } else if (n == 1) {
                status[0] = st;
                error[0] = err;
            } else {
                for (int32_t k = 0; k < n; ++k) {
                    hh_result* r = nullptr;
                    status[(size_t)k] = capture([&] { return engine_detect(c, &ins[(size_t)k], &r); }, error[(size_t)k]);
                    outs[(size_t)k] = r;
                    if (status[(size_t)k] == HH_OK)
                        status[(size_t)k] = capture([&] { return engine_host_cells(r); }, error[(size_t)k]);
                }
            }
            for (int32_t k = 0; k < n; ++k) {
                if (status[(size_t)k] != HH_OK && outs[(size_t)k]) {
                    {
                        std::lock_guard<std::mutex> r(c->results_mu);
                        c->live_results.erase(outs[(size_t)k]);
                    }
                    delete outs[(size_t)k];
                    outs[(size_t)k] = nullptr;
                }
            }
        }
        const Clock::time_point t_done = Clock::now();
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->in_flight -= batch_bytes;
            // learn the footprint per unit and the edge density from this batch
            if (c->last_call_bytes > 0 && units > 0.0)
                sv->beta = std::min(1e4, std::max(0.05, 0.7 * sv->beta + 0.3 * (double)c->last_call_bytes / units));
            for (int32_t k = 0; k < n; ++k)
                if (outs[(size_t)k] && batch[(size_t)k]->pixels > 0 && batch[(size_t)k]->in.kind != 0)
                    sv->density = 0.9 * sv->density +
                                  0.1 * (double)outs[(size_t)k]->info.n_points / (double)batch[(size_t)k]->pixels;
            for (int32_t k = 0; k < n; ++k) {
                Request& r = *batch[(size_t)k];
                r.t_start = t_start;
                r.t_done = t_done;
                r.status = status[(size_t)k];
                r.error = error[(size_t)k];
                r.result = outs[(size_t)k];
                if (r.result) {
                    r.result->timing.queue_ms = ms_between(r.t_submit, t_start);
                    r.result->timing.service_ms = ms_between(t_start, t_done);
                }
                r.done = true;
            }
        }
        sv->done_cv.notify_all();
        sv->work_cv.notify_all();   // memory freed up: a waiting lane may admit now
    }
}

}  // namespace

hh_status serve_start(hh_ctx* ctx, const hh_serve_config* cfg_in)
{
    if (ctx->server) throw Error{HH_EINVAL, "the context is already serving"};
    if (ctx->cfg.arena) throw Error{HH_EINVAL, "a context with a caller arena cannot serve"};
    hh_serve_config cfg{};
    if (cfg_in) cfg = *cfg_in;
    if (cfg.lanes == 0) cfg.lanes = 2;
    if (cfg.max_batch == 0) cfg.max_batch = 32;
    if (cfg.queue_capacity == 0) cfg.queue_capacity = 4096;
    if (cfg.lanes < 1 || cfg.lanes > 8 || cfg.max_batch < 1 || cfg.max_batch > kMaxTrees ||
        cfg.max_batch_pixels < 0 || cfg.queue_capacity < 1)
        throw Error{HH_EINVAL, "bad serving configuration"};
    if ((int64_t)cfg.max_batch * __builtin_popcount(ctx->cfg.passes) > kMaxTrees)
        throw Error{HH_EINVAL, "max_batch times the enabled passes exceeds 2048 trees"};
    auto sv = std::make_unique<Server>();
    sv->cfg = cfg;
    // the device-memory budget of all lanes together; one lane's arena may
    // take all of it when it runs alone
    int64_t budget = (int64_t)ctx->cfg.hbm_budget_bytes;
    if (budget <= 0 && ctx->cfg.arena_limit_mib > 0) budget = (int64_t)ctx->cfg.arena_limit_mib << 20;
    if (budget <= 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            total_b = (size_t)64 << 30;
        }
        budget = (int64_t)(0.35 * (double)total_b);
    }
    sv->budget = budget;
    auto cleanup = [&] {
        for (hh_ctx* l : sv->lanes) engine_destroy(l);
        for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
    };
    for (int i = 0; i < cfg.lanes; ++i) {
        hipStream_t s = nullptr;
        if (hipSetDevice(ctx->device) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            cleanup();
            throw Error{HH_EDEVICE, "hipStreamCreateWithFlags failed"};
        }
        sv->streams.push_back(s);
        hh_config lc = ctx->cfg;
        lc.stream = s;
        lc.hbm_budget_bytes = (uint64_t)budget;
        hh_ctx* lane = nullptr;
        const hh_status st = engine_create(&lc, &lane);
        if (st != HH_OK) {
            cleanup();
            throw Error{st, "lane context creation failed"};
        }
        lane->compact_results = true;   // a queued result holds its cells and voters only
        lane->task_steps = ctx->task_steps;
        lane->queue_batch = ctx->queue_batch;
        lane->wg_per_cu = ctx->wg_per_cu;
        sv->lanes.push_back(lane);
    }
    Server* raw = sv.get();
    for (int i = 0; i < cfg.lanes; ++i) raw->workers.emplace_back(run_lane, raw, i);
    ctx->server = std::move(sv);
    return HH_OK;
}

hh_status serve_submit(hh_ctx* ctx, const hh_input* in, uint64_t* ticket)
{
    Server* sv = ctx->server.get();
    if (!sv) throw Error{HH_EINVAL, "the context is not serving (hough_hier_serve_start)"};
    if (in->kind < 0 || in->kind > 2) throw Error{HH_EINVAL, "input kind must be 0 (points), 1 or 2 (images)"};
    if (in->width < 1 || in->height < 1) throw Error{HH_EINVAL, "width and height must be >= 1"};
    auto r = std::make_shared<Request>();
    r->in = *in;
    r->pixels = in->kind != 0 ? (int64_t)in->width * in->height : std::max<int64_t>(in->n_points, 1);
    if (in->kind == 0) {
        r->points = in->n_points;
    } else if (in->kind == 1 && !in->on_device && in->image) {   // a host binary image: count its edge points
        const int64_t stride = in->row_stride ? in->row_stride : in->width;
        int64_t e = 0;
        for (int32_t y = 0; y < in->height; ++y) {
            const uint8_t* row = in->image + (int64_t)y * stride;
            for (int32_t x = 0; x < in->width; ++x) e += row[x] != 0;
        }
        r->points = e;
    }
    {
        const int32_t side = std::max(in->width, in->height);
        int32_t s2 = 0;
        while ((1 << s2) < side) ++s2;
        const int32_t d = in->max_depth == INT32_MIN ? ctx->cfg.max_depth : in->max_depth;
        r->depth = d == 0 ? s2 : std::max(d, 0);
    }
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if ((int64_t)sv->tickets.size() >= sv->cfg.queue_capacity) return HH_EBUSY;
        r->ticket = sv->next_ticket++;
        sv->tickets.emplace(r->ticket, r);
        sv->pending.push_back(r);
    }
    sv->work_cv.notify_one();
    *ticket = r->ticket;
    return HH_OK;
}

hh_status serve_poll(hh_ctx* ctx, uint64_t ticket, int32_t wait_us, hh_result** out)
{
    Server* sv = ctx->server.get();
    if (!sv) throw Error{HH_EINVAL, "the context is not serving (hough_hier_serve_start)"};
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) throw Error{HH_EINVAL, "unknown ticket"};
    std::shared_ptr<Request> r = it->second;
    if (!r->done && wait_us != 0) {
        auto ready = [&] { return r->done || sv->stop; };
        if (wait_us < 0) sv->done_cv.wait(lk, ready);
        else sv->done_cv.wait_for(lk, std::chrono::microseconds(wait_us), ready);
    }
    if (!r->done) return HH_PENDING;
    sv->tickets.erase(ticket);
    if (r->status != HH_OK) throw Error{r->status, r->error};
    *out = r->result;
    return HH_OK;
}

void serve_stop(hh_ctx* ctx)
{
    Server* sv = ctx->server.get();
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->work_cv.notify_all();
    sv->done_cv.notify_all();
    for (auto& t : sv->workers)
        if (t.joinable()) t.join();
    // unclaimed results live in their lane's context and go with it
    for (hh_ctx* l : sv->lanes) engine_destroy(l);
    for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
    ctx->server.reset();
}

}  // namespace hh
