// Continuous batching of detection requests on one context.
//
// Each lane is a worker thread with a context of its own (own HIP stream,
// events and host buffers): a slot.  The lanes' device memory comes from
// one slab allocated when serving starts.  A free lane takes the pending
// requests in arrival order while their predicted footprint fits the slab's
// free space, runs them as one batch with its pool drawing from the slab,
// brings every result's cells and statistics to the host and completes the
// tickets; the results keep their blocks until they are freed.  Requests
// arriving while batches run are taken by the next lane that is free once
// slab space allows, so batches of different lanes overlap on the device
// and serving allocates no device memory.  A batch that finds the slab
// full gives its second half back to the head of the queue and runs its
// first half again; a single request waits for space to come back and runs
// again, and one that still finds the slab full while no batch runs (the
// slab held by results not yet freed for a second, or a request larger than
// the slab) runs outside the slab, in device memory returned as soon as its
// results are freed.  A
// batch that fails as a whole is run again request by request, so that each
// request gets its own status.
#include "hh_serve.hpp"

#include <algorithm>
#include <cstring>
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

// Predicted device bytes of a request: beta * units plus the fixed part of
// a call (level records, descriptors).
int64_t predicted_bytes(const Server* sv, const Request& r)
{
    return (int64_t)(sv->beta * work_units(sv, r)) + ((int64_t)4 << 20);
}

constexpr int kMaxRetries = 64;   // waits for slab space before a batch runs outside it

// One call of the lane on its stream, its pool drawing from the slab (or
// not), released blocks going back only after the stream is drained.
template <typename F>
hh_status lane_call(hh_ctx* c, bool outside, F&& f, std::string& err)
{
    c->pool.draw_outside(outside);
    c->pool.begin_call();
    const hh_status st = capture(std::forward<F>(f), err);
    (void)hipStreamSynchronize(c->stream);
    c->pool.end_call();
    c->pool.draw_outside(false);
    return st;
}

void run_lane(Server* sv, int lane)
{
    hh_ctx* c = sv->lanes[(size_t)lane];
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        int64_t want = 0;    // the batch's predicted bytes
        double units = 0.0;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            // a request whose footprint fits free slab space, or any request
            // while no batch runs (the call itself then finds out); slab space
            // comes back without this lock, hence the timed waits
            for (;;) {
                if (sv->stop) return;
                if (!sv->pending.empty() &&
                    (sv->running == 0 || predicted_bytes(sv, *sv->pending.front()) <= sv->space.largest()))
                    break;
                sv->work_cv.wait_for(lk, std::chrono::milliseconds(5));
            }
            const int32_t kind = sv->pending.front()->in.kind;
            // a batch predicted to take at most half a lane's share of the slab
            // (after the first request): room for the prediction to fall short
            // while the other lanes run
            const int64_t share = sv->space.total() / (2 * (int64_t)sv->lanes.size());
            const int64_t room = std::min(sv->space.largest(), share);
            int64_t pixels = 0;
            while (!sv->pending.empty() && (int32_t)batch.size() < sv->cfg.max_batch) {
                const auto& r = sv->pending.front();
                if (r->in.kind != kind) break;   // one kind per batch
                const int64_t b = predicted_bytes(sv, *r);
                if (!batch.empty() && (want + b > room || (sv->cfg.max_batch_pixels > 0 &&
                                                          pixels + r->pixels > sv->cfg.max_batch_pixels)))
                    break;
                r->bytes = b;
                want += b;
                units += work_units(sv, *r);
                pixels += r->pixels;
                batch.push_back(r);
                sv->pending.pop_front();
            }
            ++sv->running;
            if (!sv->pending.empty()) sv->work_cv.notify_one();   // another lane may take the rest
        }
        const Clock::time_point t_start = Clock::now();
        int32_t n = (int32_t)batch.size();
        std::vector<hh_input> ins((size_t)n);
        for (int32_t k = 0; k < n; ++k) ins[(size_t)k] = batch[(size_t)k]->in;
        std::vector<hh_result*> outs((size_t)n, nullptr);
        std::vector<hh_status> status((size_t)n, HH_OK);
        std::vector<std::string> error((size_t)n);
        {
            std::lock_guard<std::mutex> g(c->mu);
            c->arena_hint_bytes = want;
            std::string err;
            hh_status st = HH_OK;
            bool outside = false, reran = false;
            for (int attempt = 0;; ++attempt) {
                st = lane_call(c, outside, [&] { return engine_detect_batch(c, ins.data(), n, outs.data()); }, err);
                if (st == HH_EINTERNAL) {
                    // a consistency check of the kernels failed (no result was
                    // made): counted, its first text kept, and the batch run
                    // once more
                    std::lock_guard<std::mutex> lk(sv->mu);
                    if (sv->first_internal_error.empty()) sv->first_internal_error = err;
                    if (!reran) {
                        ++sv->internal_reruns;
                        reran = true;
                        continue;
                    }
                    ++sv->internal_failures;
                }
                if (st != HH_ENOMEM || outside) break;
                std::unique_lock<std::mutex> lk(sv->mu);
                ++sv->retries;
                if (n > 1) {
                    // the slab is full: the batch's second half goes back to the
                    // head of the queue, the first half runs again at once
                    const int32_t keep = n / 2;
                    for (int32_t k = n - 1; k >= keep; --k) sv->pending.push_front(batch[(size_t)k]);
                    batch.resize((size_t)keep);
                    n = keep;
                    ins.resize((size_t)n);
                    outs.assign((size_t)n, nullptr);
                    status.assign((size_t)n, HH_OK);
                    error.assign((size_t)n, std::string());
                    want = 0;
                    units = 0.0;
                    for (const auto& r : batch) {
                        want += r->bytes;
                        units += work_units(sv, *r);
                    }
                    c->arena_hint_bytes = want;
                    sv->work_cv.notify_one();
                    continue;
                }
                // one request: wait for space to come back while other batches
                // run, else (or after many waits) run it outside the slab
                if (sv->running > 1 && attempt < kMaxRetries) {
                    sv->work_cv.wait_for(lk, std::chrono::milliseconds(50));
                } else if (attempt < 10) {
                    // only results not yet freed hold the slab: wait for their owners
                    sv->work_cv.wait_for(lk, std::chrono::milliseconds(100));
                } else {
                    outside = true;
                }
            }
            if (outside) {
                std::lock_guard<std::mutex> lk(sv->mu);
                ++sv->outside_batches;
            } else if (st == HH_OK) {
                std::lock_guard<std::mutex> lk(sv->mu);
                ++sv->slab_batches;
            }
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
                    c->arena_hint_bytes = batch[(size_t)k]->bytes;
                    status[(size_t)k] = lane_call(c, outside, [&] { return engine_detect(c, &ins[(size_t)k], &r); },
                                                  error[(size_t)k]);
                    outs[(size_t)k] = r;
                    if (status[(size_t)k] == HH_OK)
                        status[(size_t)k] = capture([&] { return engine_host_cells(r); }, error[(size_t)k]);
                }
            }
            c->arena_hint_bytes = 0;
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
            --sv->running;
            // learn the footprint per unit and the edge density from this batch
            if (c->last_call_need > 0 && units > 0.0)
                sv->beta = std::min(1e4, std::max(0.05, 0.7 * sv->beta + 0.3 * (double)c->last_call_need / units));
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
        sv->work_cv.notify_all();   // a lane may admit now
    }
}

}  // namespace

hh_status serve_start(hh_ctx* ctx, const hh_serve_config* cfg_in)
{
    if (ctx->server) throw Error{HH_EINVAL, "the context is already serving"};
    if (ctx->cfg.arena) throw Error{HH_EINVAL, "a context with a caller arena cannot serve"};
    hh_serve_config cfg{};
    if (cfg_in) cfg = *cfg_in;
    // defaults: on a burst of mixed 256..4096-pixel images, three lanes of
    // batches of up to four served about twice the images per second of
    // per-request launches; larger batches of large images lost to the
    // memory they hold at once
    if (cfg.lanes == 0) cfg.lanes = 3;
    if (cfg.max_batch == 0) cfg.max_batch = 4;
    if (cfg.queue_capacity == 0) cfg.queue_capacity = 4096;
    if (cfg.lanes < 1 || cfg.lanes > 8 || cfg.max_batch < 1 || cfg.max_batch > kMaxTrees ||
        cfg.max_batch_pixels < 0 || cfg.queue_capacity < 1)
        throw Error{HH_EINVAL, "bad serving configuration"};
    if ((int64_t)cfg.max_batch * __builtin_popcount(ctx->cfg.passes) > kMaxTrees)
        throw Error{HH_EINVAL, "max_batch times the enabled passes exceeds 2048 trees"};
    auto sv = std::make_unique<Server>();
    sv->cfg = cfg;
    // the device-memory budget of all lanes together: the slab
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
    if (hipSetDevice(ctx->device) != hipSuccess || hipMalloc(&sv->slab, (size_t)budget) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{HH_ENOMEM, "device allocation of the serving slab (" + std::to_string(budget) + " bytes) failed"};
    }
    sv->space.init(sv->slab, budget, &sv->work_cv);
    auto cleanup = [&] {
        for (hh_ctx* l : sv->lanes) engine_destroy(l);
        for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
        (void)hipFree(sv->slab);
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
        lane->pool.set_caching(false);   // memory outside the slab is returned as soon as it is released
        lane->pool.back_with(&sv->space);
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

hh_status serve_stats(hh_ctx* ctx, hh_serve_stats* out)
{
    Server* sv = ctx->server.get();
    if (!sv) throw Error{HH_EINVAL, "the context is not serving (hough_hier_serve_start)"};
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = hh_serve_stats{};
    out->slab_bytes = sv->space.total();
    out->slab_used = sv->space.used();
    out->slab_batches = sv->slab_batches;
    out->outside_batches = sv->outside_batches;
    out->retries = sv->retries;
    out->pending = (int64_t)sv->pending.size();
    out->bytes_per_unit = sv->beta;
    out->internal_reruns = sv->internal_reruns;
    out->internal_failures = sv->internal_failures;
    const size_t nt = std::min(sv->first_internal_error.size(), sizeof(out->first_internal_error) - 1);
    std::memcpy(out->first_internal_error, sv->first_internal_error.data(), nt);
    out->first_internal_error[nt] = 0;
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
    // unclaimed results live in their lane's context and go with it (their
    // slab intervals return first), then the slab
    for (hh_ctx* l : sv->lanes) engine_destroy(l);
    for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
    (void)hipFree(sv->slab);
    ctx->server.reset();
}

}  // namespace hh
