// Level-synchronous driver of the hierarchical Hough vote on one gfx950.
//
// One call runs every enabled pass of one image as a separate quadtree; the
// trees share every launch.  Per level l (0 .. depth-1): a fill kernel
// clears the level's look-back words, k_vote counts and compacts the child
// voter lists, k_decide applies the threshold and writes the level-(l+1)
// region table (or the detected cells at the finest level), and the host
// reads the level's totals to size level l+1.
#include "hh_engine.hpp"

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>

#include "hh_kernels.hpp"

namespace hh {

// ---------------------------------------------------------------- pool

DevicePool::~DevicePool()
{
    trim();
    for (auto& kv : size_of_) (void)hipFree(kv.first);
}

size_t DevicePool::round_size(size_t bytes)
{
    if (bytes < 256) return 256;
    int hb = 63 - __builtin_clzll((unsigned long long)bytes);
    size_t step = hb >= 3 ? ((size_t)1 << (hb - 3)) : 1;
    return (bytes + step - 1) / step * step;
}

void* DevicePool::alloc(size_t bytes)
{
    const size_t sz = round_size(bytes);
    auto it = free_.find(sz);
    if (it != free_.end() && !it->second.empty()) {
        void* p = it->second.back();
        it->second.pop_back();
        cached_ -= sz;
        live_ += sz;
        return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
        (void)hipGetLastError();
        trim();
        if (hipMalloc(&p, sz) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    size_of_[p] = sz;
    live_ += sz;
    return p;
}

void DevicePool::release(void* p)
{
    if (!p) return;
    auto it = size_of_.find(p);
    if (it == size_of_.end()) return;
    free_[it->second].push_back(p);
    live_ -= it->second;
    cached_ += it->second;
}

void DevicePool::trim()
{
    for (auto& kv : free_) {
        for (void* p : kv.second) {
            (void)hipFree(p);
            size_of_.erase(p);
        }
        kv.second.clear();
    }
    cached_ = 0;
}

DevBuf::DevBuf(DevicePool* pool, size_t bytes) : pool_(pool), bytes_(bytes)
{
    ptr_ = pool->alloc(bytes ? bytes : 1);
    if (!ptr_) throw Error{HH_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
}

DevBuf& DevBuf::operator=(DevBuf&& o) noexcept
{
    if (this != &o) {
        reset();
        pool_ = o.pool_;
        ptr_ = o.ptr_;
        bytes_ = o.bytes_;
        o.pool_ = nullptr;
        o.ptr_ = nullptr;
        o.bytes_ = 0;
    }
    return *this;
}

void DevBuf::reset()
{
    if (pool_ && ptr_) pool_->release(ptr_);
    pool_ = nullptr;
    ptr_ = nullptr;
    bytes_ = 0;
}

// ---------------------------------------------------------------- helpers

namespace {

constexpr size_t kErrorOff = 64;     // uint32 error word in d_small
constexpr size_t kTotalsOff = 128;   // LevelTotals in d_small
constexpr size_t kScalarOff = 192;   // int64 scratch in d_small
constexpr size_t kSmallBytes = 256;

void check(hipError_t e, const char* what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{HH_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
    }
}

uint32_t* d_error(hh_ctx* c) { return reinterpret_cast<uint32_t*>(c->d_small.as<char>() + kErrorOff); }
LevelTotals* d_totals(hh_ctx* c)
{
    return reinterpret_cast<LevelTotals*>(c->d_small.as<char>() + kTotalsOff);
}
int64_t* d_scalar(hh_ctx* c) { return reinterpret_cast<int64_t*>(c->d_small.as<char>() + kScalarOff); }

int ceil_log2(int64_t n)
{
    int d = 0;
    while (((int64_t)1 << d) < n) ++d;
    return d;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

void sync(hh_ctx* c) { check(hipStreamSynchronize(c->stream), "hipStreamSynchronize"); }

void mark(hh_ctx* c, int k)
{
    if (!c->events.empty()) check(hipEventRecord(c->events[(size_t)k], c->stream), "hipEventRecord");
}

double elapsed(hh_ctx* c, int a, int b)
{
    float ms = 0.f;
    check(hipEventElapsedTime(&ms, c->events[(size_t)a], c->events[(size_t)b]), "hipEventElapsedTime");
    return ms;
}

void fetch_totals(hh_ctx* c)
{
    check(hipMemcpyAsync(c->h_totals, d_totals(c), sizeof(LevelTotals), hipMemcpyDeviceToHost, c->stream),
          "copy level totals");
    sync(c);
}

}  // namespace

// ---------------------------------------------------------------- context

hh_status engine_create(const hh_config* cfg, hh_ctx** out)
{
    std::unique_ptr<hh_ctx> ctx(new (std::nothrow) hh_ctx());
    if (!ctx) return HH_ENOMEM;
    ctx->cfg = *cfg;
    if (ctx->cfg.passes == 0) ctx->cfg.passes = HH_PASS_0 | HH_PASS_1;
    ctx->device = cfg->device;
    ctx->stream = static_cast<hipStream_t>(cfg->stream);
    try {
        int n = 0;
        check(hipGetDeviceCount(&n), "hipGetDeviceCount");
        if (cfg->device < 0 || cfg->device >= n) throw Error{HH_EDEVICE, "no such HIP device"};
        check(hipSetDevice(cfg->device), "hipSetDevice");
        hipDeviceProp_t prop;
        check(hipGetDeviceProperties(&prop, cfg->device), "hipGetDeviceProperties");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            throw Error{HH_EDEVICE, std::string("device is ") + prop.gcnArchName + ", not gfx950"};
        ctx->cu_count = prop.multiProcessorCount;
        check(hipHostMalloc((void**)&ctx->h_totals, sizeof(LevelTotals), hipHostMallocDefault),
              "hipHostMalloc");
        check(hipHostMalloc((void**)&ctx->h_trees, 2 * sizeof(TreeDesc), hipHostMallocDefault),
              "hipHostMalloc");
        check(hipHostMalloc((void**)&ctx->h_scalar, 64 * sizeof(int64_t), hipHostMallocDefault),
              "hipHostMalloc");
        check(hipHostMalloc((void**)&ctx->h_error, sizeof(uint32_t), hipHostMallocDefault),
              "hipHostMalloc");
        if (cfg->flags & HH_FLAG_TIMING) {
            ctx->events.resize(3 + 3 * kMaxLevels, nullptr);
            for (auto& e : ctx->events) check(hipEventCreate(&e), "hipEventCreate");
        }
        ctx->d_small = DevBuf(&ctx->pool, kSmallBytes);
        check(launch_fill_u64(ctx->d_small.as<uint64_t>(), kSmallBytes / 8, 0, ctx->stream), "fill");
        sync(ctx.get());
    } catch (const Error& e) {
        engine_destroy(ctx.release());
        return e.status;
    }
    *out = ctx.release();
    return HH_OK;
}

void engine_destroy(hh_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    ctx->events.clear();
    for (hh_result* r : ctx->live_results) delete r;
    ctx->live_results.clear();
    ctx->d_small.reset();
    if (ctx->h_totals) (void)hipHostFree(ctx->h_totals);
    if (ctx->h_trees) (void)hipHostFree(ctx->h_trees);
    if (ctx->h_scalar) (void)hipHostFree(ctx->h_scalar);
    if (ctx->h_error) (void)hipHostFree(ctx->h_error);
    delete ctx;
}

// ---------------------------------------------------------------- detect

namespace {

struct Plan {
    int32_t W, H;
    int64_t S;
    int32_t s_log2;
    int32_t dmax;
    int32_t T;
    uint32_t passes;
    int32_t variant;
    bool wide;
    bool membership;
};

Plan make_plan(const hh_ctx* ctx, const hh_input* in)
{
    Plan p{};
    if (in->width < 1 || in->height < 1) throw Error{HH_EINVAL, "width and height must be >= 1"};
    const int32_t side = std::max(in->width, in->height);
    if (side > HH_MAX_SIDE) throw Error{HH_EINVAL, "max(width, height) exceeds 16384"};
    p.W = in->width;
    p.H = in->height;
    p.s_log2 = ceil_log2(side);
    p.S = (int64_t)1 << p.s_log2;
    p.T = in->threshold >= 0 ? in->threshold : ctx->cfg.threshold;
    if (p.T < 0) throw Error{HH_EINVAL, "threshold must be >= 0"};
    int32_t d = in->max_depth == INT32_MIN ? ctx->cfg.max_depth : in->max_depth;
    if (d == 0) d = p.s_log2;
    if (d < 0) d = 0;
    if (d > HH_MAX_DEPTH) throw Error{HH_EINVAL, "depth exceeds 15"};
    if ((p.S << d) > ((int64_t)1 << 28)) throw Error{HH_EINVAL, "S * 2^depth exceeds 2^28"};
    p.dmax = d;
    p.passes = ctx->cfg.passes;
    p.variant = ctx->cfg.variant;
    p.wide = (ctx->cfg.flags & HH_FLAG_WIDE_COMPARE) != 0;
    p.membership = ctx->cfg.membership != 0;
    return p;
}

}  // namespace

hh_status engine_detect(hh_ctx* ctx, const hh_input* in, hh_result** out)
{
    std::unique_ptr<hh_result> res(new (std::nothrow) hh_result());
    if (!res) return HH_ENOMEM;
    res->ctx = ctx;
    hipStream_t st = ctx->stream;
    DevicePool* pool = &ctx->pool;
    check(hipSetDevice(ctx->device), "hipSetDevice");
    const Plan plan = make_plan(ctx, in);

    // clear tickets, error word and totals
    check(launch_fill_u64(ctx->d_small.as<uint64_t>(), kSmallBytes / 8, 0, st), "fill");
    const bool timing = !ctx->events.empty();
    hh_timing& tm = res->timing;
    mark(ctx, 0);

    // ---- edge staging
    DevBuf xb, yb, imgb, sync0;
    const int32_t* dx = nullptr;
    const int32_t* dy = nullptr;
    int64_t E = 0;
    if (in->kind == 0) {
        if (in->n_points < 0 || in->n_points > INT32_MAX) throw Error{HH_EINVAL, "bad n_points"};
        E = in->n_points;
        if (E > 0 && (!in->x || !in->y)) throw Error{HH_EINVAL, "x and y must not be NULL"};
        if (in->on_device) {
            dx = in->x;
            dy = in->y;
            check(launch_validate(dx, dy, E, plan.W, plan.H, d_error(ctx), st), "validate");
        } else {
            for (int64_t k = 0; k < E; ++k)
                if (in->x[k] < 0 || in->x[k] >= plan.W || in->y[k] < 0 || in->y[k] >= plan.H)
                    throw Error{HH_EINVAL, "point " + std::to_string(k) + " outside the image"};
            xb = DevBuf(pool, (size_t)std::max<int64_t>(E, 1) * 4);
            yb = DevBuf(pool, (size_t)std::max<int64_t>(E, 1) * 4);
            if (E > 0) {
                check(hipMemcpyAsync(xb.get(), in->x, (size_t)E * 4, hipMemcpyHostToDevice, st), "copy x");
                check(hipMemcpyAsync(yb.get(), in->y, (size_t)E * 4, hipMemcpyHostToDevice, st), "copy y");
            }
            dx = xb.as<int32_t>();
            dy = yb.as<int32_t>();
        }
    } else if (in->kind == 1) {
        if (!in->image) throw Error{HH_EINVAL, "image must not be NULL"};
        const int64_t stride = in->row_stride ? in->row_stride : plan.W;
        if (stride < plan.W) throw Error{HH_EINVAL, "row_stride < width"};
        const int64_t n_pix = (int64_t)plan.W * plan.H;
        const uint8_t* img = in->image;
        int64_t dstride = stride;
        if (!in->on_device) {
            imgb = DevBuf(pool, (size_t)n_pix);
            check(hipMemcpy2DAsync(imgb.get(), (size_t)plan.W, in->image, (size_t)stride, (size_t)plan.W,
                                   (size_t)plan.H, hipMemcpyHostToDevice, st),
                  "copy image");
            img = imgb.as<uint8_t>();
            dstride = plan.W;
        }
        xb = DevBuf(pool, (size_t)n_pix * 4);
        yb = DevBuf(pool, (size_t)n_pix * 4);
        const int32_t n_tiles = (int32_t)cdiv(n_pix, kPixTile);
        sync0 = DevBuf(pool, (size_t)(n_tiles + 1) * 8);
        check(launch_fill_u64(sync0.as<uint64_t>(), n_tiles + 1, 0, st), "fill");
        ExtractArgs ea{};
        ea.image = img;
        ea.row_stride = dstride;
        ea.width = plan.W;
        ea.height = plan.H;
        ea.n_pix = n_pix;
        ea.x = xb.as<int32_t>();
        ea.y = yb.as<int32_t>();
        ea.status = sync0.as<uint64_t>();
        ea.ticket = reinterpret_cast<uint32_t*>(sync0.as<uint64_t>() + n_tiles);
        ea.n_tiles = n_tiles;
        ea.total = d_scalar(ctx);
        ea.error = d_error(ctx);
        check(launch_extract(ea, st), "extract");
        mark(ctx, 1);
        check(hipMemcpyAsync(ctx->h_scalar, d_scalar(ctx), 8, hipMemcpyDeviceToHost, st), "copy E");
        sync(ctx);
        E = ctx->h_scalar[0];
        if (E > INT32_MAX) throw Error{HH_ECAPACITY, "more than 2^31-1 edge points"};
        dx = xb.as<int32_t>();
        dy = yb.as<int32_t>();
    } else {
        throw Error{HH_EINVAL, "input kind must be 0 (points) or 1 (image)"};
    }

    // ---- trees (one per enabled pass)
    int32_t n_trees = 0;
    for (int p = 0; p < 2; ++p) {
        if (!(plan.passes & (1u << p))) continue;
        TreeDesc& t = ctx->h_trees[n_trees];
        t.u = p == 0 ? dx : dy;   // pass 1 reads (x0, y0) as (y0, x0)
        t.v = p == 0 ? dy : dx;
        t.n_points = E;
        t.s_log2 = plan.s_log2;
        t.dmax = plan.dmax;
        t.threshold = plan.T;
        t.pass = p;
        t.image = 0;
        t.pad = 0;
        res->tree_pass[n_trees] = p;
        ++n_trees;
    }
    res->n_trees = n_trees;
    DevBuf d_trees(pool, sizeof(TreeDesc) * 2);
    check(hipMemcpyAsync(d_trees.get(), ctx->h_trees, sizeof(TreeDesc) * n_trees, hipMemcpyHostToDevice, st),
          "copy trees");
    const int64_t n_stats = (int64_t)n_trees * kMaxLevels * kNumStats;
    DevBuf d_stats(pool, (size_t)n_stats * 8);
    check(launch_fill_u64(d_stats.as<uint64_t>(), n_stats, 0, st), "fill");

    const bool root_votes = E > plan.T;   // every line crosses the root (code 0011)
    int64_t n_cells_total = 0;
    DevBuf cells, members, iota;

    if (root_votes && plan.dmax > 0) {
        // ---- level loop
        int64_t P = n_trees;
        int64_t L = (int64_t)n_trees * E;
        DevBuf regions(pool, sizeof(Region) * (size_t)P);
        int32_t n_tiles = (int32_t)cdiv(L, kTile);
        DevBuf tile_first(pool, (size_t)n_tiles * 4);
        iota = DevBuf(pool, (size_t)E * 4);
        check(launch_init_level0(regions.as<Region>(), tile_first.as<int32_t>(), iota.as<int32_t>(), n_trees, E,
                                 n_tiles, st),
              "init level 0");
        DevBuf list;   // level list buffer (level 0 uses iota)
        const int32_t* list_ptr = iota.as<int32_t>();
        for (int l = 0; l < plan.dmax; ++l) {
            const bool last = (l + 1 == plan.dmax);
            n_tiles = (int32_t)cdiv(L, kTile);
            const int32_t n_ptiles = (int32_t)cdiv(P, kBlock);
            const bool write_out = !last || plan.membership;
            DevBuf outb;
            if (write_out) outb = DevBuf(pool, (size_t)L * 4 * 4);
            DevBuf pstart(pool, (size_t)P * 4 * 8);
            const int64_t n_sync = (int64_t)n_tiles * 4 + (int64_t)n_ptiles * 3 + 2;
            DevBuf syncb(pool, (size_t)n_sync * 8);
            uint64_t* sw = syncb.as<uint64_t>();
            check(launch_fill_u64(sw, n_sync, 0, st), "fill");
            DevBuf next_regions, next_tile_first, cellb;
            int64_t next_tile_cap = 0;
            if (!last) {
                next_regions = DevBuf(pool, sizeof(Region) * (size_t)(4 * P));
                next_tile_cap = cdiv(4 * L, kTile) + 1;
                next_tile_first = DevBuf(pool, (size_t)next_tile_cap * 4);
            } else {
                cellb = DevBuf(pool, sizeof(Cell) * (size_t)(4 * P));
            }

            VoteArgs va{};
            va.regions = regions.as<Region>();
            va.n_regions = (int32_t)P;
            va.tile_first = tile_first.as<int32_t>();
            va.n_tiles = n_tiles;
            va.list = list_ptr;
            va.trees = d_trees.as<TreeDesc>();
            va.n_entries = L;
            va.level = l;
            va.write_out = write_out ? 1 : 0;
            va.out = write_out ? outb.as<int32_t>() : nullptr;
            va.out_cap = L;
            va.pstart = pstart.as<int64_t>();
            va.status = sw;
            va.ticket = reinterpret_cast<uint32_t*>(sw + (int64_t)n_tiles * 4 + (int64_t)n_ptiles * 3);
            va.totals = d_totals(ctx);
            va.error = d_error(ctx);
            mark(ctx, 3 + 3 * l);
            check(launch_vote(va, plan.variant, plan.wide, st), "vote");
            mark(ctx, 4 + 3 * l);

            DecideArgs da{};
            da.regions = regions.as<Region>();
            da.n_regions = (int32_t)P;
            da.trees = d_trees.as<TreeDesc>();
            da.level = l;
            da.pstart = pstart.as<int64_t>();
            da.out_cap = L;
            da.status = sw + (int64_t)n_tiles * 4;
            da.ticket = va.ticket + 2;   // next uint64 word
            da.n_tiles = n_ptiles;
            da.totals = d_totals(ctx);
            da.next_regions = last ? nullptr : next_regions.as<Region>();
            da.next_tile_first = last ? nullptr : next_tile_first.as<int32_t>();
            da.next_tile_cap = next_tile_cap;
            da.cells = last ? cellb.as<Cell>() : nullptr;
            da.stats = d_stats.as<int64_t>();
            da.keep_members = plan.membership ? 1 : 0;
            da.error = d_error(ctx);
            check(launch_decide(da, st), "decide");
            mark(ctx, 5 + 3 * l);
            fetch_totals(ctx);
            const LevelTotals tot = *ctx->h_totals;
            if (timing) {
                tm.vote_ms += elapsed(ctx, 3 + 3 * l, 4 + 3 * l);
                tm.decide_ms += elapsed(ctx, 4 + 3 * l, 5 + 3 * l);
                tm.vote_launches += 1;
                tm.decide_launches += 1;
            }
            tm.vote_entries += L;
            if (write_out) tm.vote_written += tot.votes[0] + tot.votes[1] + tot.votes[2] + tot.votes[3];

            if (last) {
                n_cells_total = tot.n_cells;
                cells = std::move(cellb);
                if (write_out) members = std::move(outb);
                res->info.member_slots = write_out ? 4 * L : 0;
                break;
            }
            // advance to level l+1
            list = std::move(outb);
            list_ptr = list.as<int32_t>();
            if (l == 0) iota.reset();
            regions = std::move(next_regions);
            tile_first = std::move(next_tile_first);
            P = tot.n_next;
            L = tot.len_next;
            if (P == 0) break;
        }
    } else if (root_votes) {
        // depth 0: the root is the finest region, every line votes for it
        iota = DevBuf(pool, (size_t)E * 4);
        DevBuf dummy_regions(pool, sizeof(Region) * 2);
        DevBuf dummy_tiles(pool, 4 * 2);
        check(launch_init_level0(dummy_regions.as<Region>(), dummy_tiles.as<int32_t>(), iota.as<int32_t>(),
                                 n_trees, E, 1, st),
              "init level 0");
        std::vector<Cell> hc(n_trees);
        for (int t = 0; t < n_trees; ++t) {
            hc[t].i = 0;
            hc[t].j = 0;
            hc[t].votes = (int32_t)E;
            hc[t].pass = res->tree_pass[t];
            hc[t].key = 0;
            hc[t].member_off = plan.membership ? 0 : -1;
        }
        cells = DevBuf(pool, sizeof(Cell) * n_trees);
        check(hipMemcpyAsync(cells.get(), hc.data(), sizeof(Cell) * n_trees, hipMemcpyHostToDevice, st),
              "copy cells");
        n_cells_total = n_trees;
        if (plan.membership) {
            members = std::move(iota);
            res->info.member_slots = E;
        }
        sync(ctx);
    }

    // ---- statistics and error word
    mark(ctx, 2);
    std::vector<int64_t> hs((size_t)n_stats);
    check(hipMemcpyAsync(hs.data(), d_stats.get(), (size_t)n_stats * 8, hipMemcpyDeviceToHost, st), "copy stats");
    check(hipMemcpyAsync(ctx->h_error, d_error(ctx), 4, hipMemcpyDeviceToHost, st), "copy error");
    sync(ctx);
    if (timing) {
        tm.total_ms = elapsed(ctx, 0, 2);
        if (in->kind == 1) tm.extract_ms = elapsed(ctx, 0, 1);
    }
    if (*ctx->h_error & kErrPointRange) throw Error{HH_EINVAL, "a device point lies outside the image"};
    if (*ctx->h_error & kErrLookback) throw Error{HH_EINTERNAL, "look-back wait timed out"};
    if (*ctx->h_error & kErrInternal) throw Error{HH_EINTERNAL, "a kernel index failed its range check"};

    res->info.n_points = E;
    res->info.width = plan.W;
    res->info.height = plan.H;
    res->info.side_pow2 = (int32_t)plan.S;
    res->info.depth = plan.dmax;
    res->info.threshold = plan.T;
    res->info.passes = plan.passes;
    res->info.compare_bits = (plan.variant == HH_VARIANT_CIRCLE || plan.wide) ? 64 : 32;
    int64_t code_tests = 0;
    for (int t = 0; t < n_trees; ++t) {
        const int p = res->tree_pass[t];
        auto& v = res->stats[p];
        v.assign((size_t)plan.dmax + 1, hh_level_stats{});
        v[0].evaluated = 1;
        v[0].votes = E;
        v[0].code_tests = E;
        if (root_votes && plan.dmax > 0) {
            v[0].split = 1;
            v[0].entries = E;
        }
        if (root_votes && plan.dmax == 0) v[0].detected = 1;
        for (int l = 1; l <= plan.dmax; ++l) {
            const int64_t* s = &hs[((size_t)t * kMaxLevels + l) * kNumStats];
            v[l].evaluated = s[0];
            v[l].votes = s[1];
            v[l].split = s[2];
            v[l].detected = s[3];
            v[l].code_tests = s[4];
            v[l].entries = s[5];
        }
        for (const auto& lv : v) code_tests += lv.code_tests;
        res->info.n_cells[p] = v[plan.dmax].detected;
    }
    res->info.code_tests = code_tests;
    res->n_cells_total = n_cells_total;
    if (res->info.n_cells[0] + res->info.n_cells[1] != n_cells_total)
        throw Error{HH_EINTERNAL, "cell count does not match the statistics"};
    res->cells = std::move(cells);
    res->members = std::move(members);
    res->have_members = plan.membership;
    ctx->live_results.insert(res.get());
    *out = res.release();
    return HH_OK;
}

hh_status engine_host_copy(hh_result* res)
{
    if (res->host_ready) return HH_OK;
    hh_ctx* ctx = res->ctx;
    hipStream_t st = ctx->stream;
    check(hipSetDevice(ctx->device), "hipSetDevice");
    const int64_t n = res->n_cells_total;
    res->host_cells.resize((size_t)n);
    if (n > 0)
        check(hipMemcpyAsync(res->host_cells.data(), res->cells.get(), (size_t)n * sizeof(hh_cell),
                             hipMemcpyDeviceToHost, st),
              "copy cells");
    sync(ctx);
    std::vector<int64_t> off((size_t)n);
    int64_t total = 0;
    for (int64_t c = 0; c < n; ++c) {
        off[(size_t)c] = total;
        total += res->host_cells[(size_t)c].votes;
    }
    if (res->have_members && n > 0) {
        DevBuf d_off(&ctx->pool, (size_t)n * 8);
        DevBuf d_dst(&ctx->pool, (size_t)std::max<int64_t>(total, 1) * 4);
        check(hipMemcpyAsync(d_off.get(), off.data(), (size_t)n * 8, hipMemcpyHostToDevice, st), "copy offsets");
        check(launch_gather_members(res->cells.as<Cell>(), n, d_off.as<int64_t>(), res->members.as<int32_t>(),
                                    d_dst.as<int32_t>(), st),
              "gather members");
        res->host_members.resize((size_t)total);
        check(hipMemcpyAsync(res->host_members.data(), d_dst.get(), (size_t)total * 4, hipMemcpyDeviceToHost, st),
              "copy members");
        sync(ctx);
    }
    for (int64_t c = 0; c < n; ++c)
        res->host_cells[(size_t)c].member_off = res->have_members ? off[(size_t)c] : -1;
    res->host_ready = true;
    return HH_OK;
}

}  // namespace hh
