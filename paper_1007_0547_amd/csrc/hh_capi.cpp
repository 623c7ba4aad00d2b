// C ABI of the hierarchical Hough vote library (declarations and contracts in
// include/hough_hier.h).  Every entry point converts internal errors into an
// hh_status and records the message on the context.
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hh_engine.hpp"

namespace {

hh_status fail(hh_ctx* ctx, hh_status s, const std::string& msg)
{
    if (ctx) {
        std::lock_guard<std::mutex> g(ctx->err_mu);
        ctx->last_error = msg;
    }
    return s;
}

void clear_error(hh_ctx* ctx)
{
    std::lock_guard<std::mutex> g(ctx->err_mu);
    ctx->last_error.clear();
}

template <typename F>
hh_status guarded(hh_ctx* ctx, F&& f)
{
    try {
        return f();
    } catch (const hh::Error& e) {
        return fail(ctx, e.status, e.what);
    } catch (const std::bad_alloc&) {
        return fail(ctx, HH_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(ctx, HH_EINTERNAL, e.what());
    } catch (...) {
        return fail(ctx, HH_EINTERNAL, "unknown error");
    }
}

}  // namespace

extern "C" {

hh_status hough_hier_create(const hh_config* cfg, hh_ctx** out)
{
    if (!cfg || !out) return HH_EINVAL;
    *out = nullptr;
    if (cfg->threshold < 0 || cfg->max_depth < -1 || cfg->max_depth > HH_MAX_DEPTH ||
        (cfg->variant != HH_VARIANT_CODE && cfg->variant != HH_VARIANT_CIRCLE) ||
        (cfg->passes & ~(HH_PASS_0 | HH_PASS_1)) != 0 || (cfg->membership != 0 && cfg->membership != 1) ||
        cfg->arena_limit_mib < 0 || (cfg->arena && (cfg->arena_bytes == 0 || (uintptr_t)cfg->arena % 256)) ||
        (!cfg->arena && cfg->arena_bytes))
        return HH_EINVAL;
    try {
        return hh::engine_create(cfg, out);
    } catch (...) {
        return HH_EINTERNAL;
    }
}

void hough_hier_destroy(hh_ctx* ctx)
{
    try {
        hh::engine_destroy(ctx);
    } catch (...) {
    }
}

hh_status hough_hier_set_launch(hh_ctx* ctx, const hh_launch* launch)
{
    if (!ctx || !launch) return HH_EINVAL;
    const int32_t steps = launch->task_steps ? launch->task_steps : 8;
    if (steps < 1 || steps > hh::kMaxTaskSteps || launch->queue_batch < 0 || launch->queue_batch > 1024 ||
        launch->wg_per_cu < 0 || launch->wg_per_cu > 64)
        return fail(ctx, HH_EINVAL, "launch shape out of range");
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->task_steps = steps;
    ctx->queue_batch = launch->queue_batch;
    ctx->wg_per_cu = launch->wg_per_cu;
    return HH_OK;
}

hh_status hough_hier_autotune(hh_ctx* ctx, const hh_input* inputs, int32_t n, hh_launch* chosen,
                              int32_t* from_cache)
{
    if (!ctx) return HH_EINVAL;
    if (!inputs || !chosen || n < 1) return fail(ctx, HH_EINVAL, "inputs and chosen must not be NULL, n >= 1");
    clear_error(ctx);
    std::lock_guard<std::mutex> g(ctx->mu);
    int32_t cached = 0;
    const hh_status s = guarded(ctx, [&] { return hh::engine_autotune(ctx, inputs, n, chosen, &cached); });
    if (from_cache) *from_cache = cached;
    return s;
}

hh_status hough_hier_get_launch(const hh_ctx* ctx, hh_launch* launch)
{
    if (!ctx || !launch) return HH_EINVAL;
    launch->task_steps = ctx->task_steps;
    launch->queue_batch = ctx->queue_batch;
    launch->wg_per_cu = ctx->wg_per_cu;
    launch->reserved = 0;
    return HH_OK;
}

const char* hough_hier_last_error(const hh_ctx* ctx)
{
    if (!ctx) return "";
    return ctx->last_error.c_str();
}

hh_status hough_hier_serve_start(hh_ctx* ctx, const hh_serve_config* cfg)
{
    if (!ctx) return HH_EINVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    return guarded(ctx, [&] { return hh::serve_start(ctx, cfg); });
}

hh_status hough_hier_serve_stats(hh_ctx* ctx, hh_serve_stats* out)
{
    if (!ctx) return HH_EINVAL;
    if (!out) return fail(ctx, HH_EINVAL, "output pointer must not be NULL");
    return guarded(ctx, [&] { return hh::serve_stats(ctx, out); });
}

hh_status hough_hier_submit(hh_ctx* ctx, const hh_input* in, uint64_t* ticket)
{
    if (!ctx) return HH_EINVAL;
    if (!in || !ticket) return fail(ctx, HH_EINVAL, "input and ticket pointers must not be NULL");
    return guarded(ctx, [&] { return hh::serve_submit(ctx, in, ticket); });
}

hh_status hough_hier_poll(hh_ctx* ctx, uint64_t ticket, int32_t wait_us, hh_result** out)
{
    if (!ctx) return HH_EINVAL;
    if (!out) return fail(ctx, HH_EINVAL, "output pointer must not be NULL");
    *out = nullptr;
    return guarded(ctx, [&] { return hh::serve_poll(ctx, ticket, wait_us, out); });
}

hh_status hough_hier_detect(hh_ctx* ctx, const hh_input* in, hh_result** out)
{
    if (!ctx) return HH_EINVAL;
    if (!in || !out) return fail(ctx, HH_EINVAL, "input and output pointers must not be NULL");
    *out = nullptr;
    clear_error(ctx);
    std::lock_guard<std::mutex> g(ctx->mu);
    return guarded(ctx, [&] { return hh::engine_detect(ctx, in, out); });
}

hh_status hough_hier_detect_noalloc(hh_ctx* ctx, const hh_input* in, hh_cell* cells, int64_t cells_cap,
                                    int32_t* members, int64_t members_cap, hh_level_stats* stats, int64_t* n_cells,
                                    int64_t* n_members)
{
    if (!ctx) return HH_EINVAL;
    if (!in || !stats || !n_cells || !n_members)
        return fail(ctx, HH_EINVAL, "input, stats and count pointers must not be NULL");
    clear_error(ctx);
    std::lock_guard<std::mutex> g(ctx->mu);
    return guarded(ctx, [&] {
        return hh::engine_detect_noalloc(ctx, in, cells, cells_cap, members, members_cap, stats, n_cells, n_members);
    });
}

hh_status hough_hier_detect_batch(hh_ctx* ctx, const hh_input* inputs, int32_t n, hh_result** out)
{
    if (!ctx) return HH_EINVAL;
    if (!inputs || !out) return fail(ctx, HH_EINVAL, "input and output pointers must not be NULL");
    if (n < 1) return fail(ctx, HH_EINVAL, "a batch needs at least one input");
    for (int32_t k = 0; k < n; ++k) out[k] = nullptr;
    clear_error(ctx);
    std::lock_guard<std::mutex> g(ctx->mu);
    return guarded(ctx, [&] { return hh::engine_detect_batch(ctx, inputs, n, out); });
}

hh_status hough_hier_result_cells(hh_result* res, int32_t pass, int32_t on_device, const hh_cell** cells,
                                  int64_t* n)
{
    if (!res || !cells || !n || (pass != 0 && pass != 1)) return HH_EINVAL;
    *cells = nullptr;
    *n = 0;
    int64_t before = 0;
    bool enabled = false;
    for (int t = 0; t < res->n_trees; ++t) {
        if (res->tree_pass[t] == pass) {
            enabled = true;
            break;
        }
        before += res->info.n_cells[res->tree_pass[t]];
    }
    if (!enabled) return HH_OK;
    const int64_t count = res->info.n_cells[pass];
    std::lock_guard<std::mutex> g(res->ctx->mu);
    if (on_device) {
        const hh::Cell* dc = nullptr;
        hh_status s = guarded(res->ctx, [&] {
            dc = hh::engine_device_cells(res);
            return HH_OK;
        });
        if (s != HH_OK) return s;
        if (count > 0) *cells = reinterpret_cast<const hh_cell*>(dc) + before;
        *n = count;
        return HH_OK;
    }
    hh_status s = guarded(res->ctx, [&] { return hh::engine_host_cells(res); });
    if (s != HH_OK) return s;
    if (count > 0) *cells = res->host_cells.data() + before;
    *n = count;
    return HH_OK;
}

hh_status hough_hier_result_members(hh_result* res, int32_t on_device, const int32_t** ids, int64_t* n)
{
    if (!res || !ids || !n) return HH_EINVAL;
    *ids = nullptr;
    *n = 0;
    if (!res->have_members) return fail(res->ctx, HH_EINVAL, "membership was not kept");
    std::lock_guard<std::mutex> g(res->ctx->mu);
    if (on_device) {
        hh_status s = guarded(res->ctx, [&] { return hh::engine_device_ids(res); });
        if (s != HH_OK) return s;
        *ids = res->dev_ids ? res->dev_ids.as<const int32_t>() : nullptr;
        *n = res->info.member_slots;
        return HH_OK;
    }
    hh_status s = guarded(res->ctx, [&] { return hh::engine_host_members(res); });
    if (s != HH_OK) return s;
    *ids = res->host_members.data();
    *n = (int64_t)res->host_members.size();
    return HH_OK;
}

hh_status hough_hier_result_member_points(const hh_result* res, const void** entries, int64_t* n,
                                         int32_t* entry_bytes)
{
    if (!res || !entries || !n || !entry_bytes) return HH_EINVAL;
    *entries = nullptr;
    *n = 0;
    *entry_bytes = res->entry_bytes;
    if (!res->have_members) return fail(res->ctx, HH_EINVAL, "membership was not kept");
    *entries = res->members;
    *n = res->info.member_slots;
    return HH_OK;
}

hh_status hough_hier_result_stats(const hh_result* res, int32_t pass, const hh_level_stats** levels,
                                  int32_t* n_levels)
{
    if (!res || !levels || !n_levels || (pass != 0 && pass != 1)) return HH_EINVAL;
    *levels = res->stats[pass].empty() ? nullptr : res->stats[pass].data();
    *n_levels = (int32_t)res->stats[pass].size();
    return HH_OK;
}

hh_status hough_hier_result_info(const hh_result* res, hh_result_info* info)
{
    if (!res || !info) return HH_EINVAL;
    *info = res->info;
    return HH_OK;
}

hh_status hough_hier_result_timing(const hh_result* res, hh_timing* timing)
{
    if (!res || !timing) return HH_EINVAL;
    *timing = res->timing;
    return HH_OK;
}

hh_status hough_hier_solution(hh_result* const* results, int32_t n, double* kernel_ms)
{
    if (kernel_ms) *kernel_ms = 0.0;
    if (n < 0 || (n > 0 && !results)) return HH_EINVAL;
    for (int32_t k = 0; k < n; ++k)
        if (!results[k]) return HH_EINVAL;
    // results of one context run in one launch; a serving context's results
    // belong to the lane that made them
    std::vector<bool> done((size_t)n, false);
    for (int32_t k = 0; k < n; ++k) {
        if (done[(size_t)k]) continue;
        hh_ctx* ctx = results[k]->ctx;
        std::vector<hh_result*> group;
        for (int32_t q = k; q < n; ++q) {
            if (!done[(size_t)q] && results[q]->ctx == ctx) {
                group.push_back(results[q]);
                done[(size_t)q] = true;
            }
        }
        double ms = 0.0;
        hh_status s;
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            s = guarded(ctx, [&] { return hh::engine_solution(ctx, group.data(), (int32_t)group.size(), &ms); });
        }
        if (s != HH_OK) return s;
        if (kernel_ms) *kernel_ms += ms;
    }
    return HH_OK;
}

hh_status hough_hier_result_solution(hh_result* res, int32_t pass, int32_t on_device, hh_solution* out)
{
    if (!res || !out || (pass != 0 && pass != 1)) return HH_EINVAL;
    *out = hh_solution{};
    if (!res->sol_ready) return fail(res->ctx, HH_EINVAL, "hough_hier_solution has not run on this result");
    bool enabled = false;
    for (int t = 0; t < res->n_trees; ++t) enabled = enabled || res->tree_pass[t] == pass;
    if (!enabled) return HH_OK;
    out->n_cells = res->info.n_cells[pass];
    out->n_points = res->info.n_points;
    out->kept = res->sol_kept[pass];
    out->plotted_points = res->sol_plotted[pass];
    out->rounds = res->sol_rounds;
    if (on_device) {
        out->keep = res->sol + res->sol_keep_off[pass];
        out->plotted = res->sol + res->sol_plot_off[pass];
        return HH_OK;
    }
    std::lock_guard<std::mutex> g(res->ctx->mu);
    hh_status s = guarded(res->ctx, [&] { return hh::engine_host_solution(res, pass); });
    if (s != HH_OK) return s;
    out->keep = res->host_keep[pass].data();
    out->plotted = res->host_plotted[pass].data();
    return HH_OK;
}

hh_status hough_hier_result_solution_image(hh_result* res, uint8_t* image, int64_t row_stride, int32_t on_device)
{
    if (!res || !image) return HH_EINVAL;
    if (!res->sol_ready) return fail(res->ctx, HH_EINVAL, "hough_hier_solution has not run on this result");
    if (row_stride < res->info.width) return fail(res->ctx, HH_EINVAL, "row_stride is below the image width");
    std::lock_guard<std::mutex> g(res->ctx->mu);
    return guarded(res->ctx, [&] { return hh::engine_solution_image(res, image, row_stride, on_device); });
}

const char* hough_hier_result_last_error(const hh_result* res)
{
    if (!res || !res->ctx) return "";
    std::lock_guard<std::mutex> g(res->ctx->err_mu);
    return res->ctx->last_error.c_str();
}

void hough_hier_result_free(hh_result* res)
{
    if (!res) return;
    try {
        // the pool has a lock of its own: a free never waits for a running call
        {
            std::lock_guard<std::mutex> g(res->ctx->results_mu);
            res->ctx->live_results.erase(res);
            if (res->in_arena) --res->ctx->arena_results;
        }
        delete res;
    } catch (...) {
    }
}

}  // extern "C"
