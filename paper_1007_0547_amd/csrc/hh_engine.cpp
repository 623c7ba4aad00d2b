// Level-synchronous driver of the hierarchical Hough vote on one gfx950.
//
// One call runs every enabled pass of one image as a separate quadtree; the
// trees share every launch.  The host enqueues the whole call without
// waiting: edge staging, the root setup, then per level l (0 .. depth-1) the
// count, decide, emit and compaction launches.  Level sizes stay on the
// device (LevelInfo records in the call's arena); the host waits once, at
// the end, and reads the level records, the tree records (the per-pass
// statistics follow from them) and the error word.  If a level did not fit
// the arena the call is run again with a larger arena (sizes learnt this way
// are kept for the next calls on the context).
#include "hh_engine.hpp"

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>

#include "hh_kernels.hpp"
#include "hh_serve.hpp"
#include "hh_solution.hpp"

namespace hh {

// ---------------------------------------------------------------- pool

void SlabSpace::init(char* base, int64_t bytes, std::condition_variable* freed)
{
    std::lock_guard<std::mutex> g(mu_);
    base_ = base;
    freed_ = freed;
    free_.clear();
    live_.clear();
    total_ = bytes & ~(int64_t)255;
    used_ = 0;
    if (total_ > 0) free_[0] = total_;
}

int64_t SlabSpace::take(int64_t bytes)
{
    bytes = (std::max<int64_t>(bytes, 256) + 255) & ~(int64_t)255;
    std::lock_guard<std::mutex> g(mu_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < bytes) continue;
        const int64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        live_[off] = bytes;
        used_ += bytes;
        return off;
    }
    return -1;
}

void SlabSpace::give(int64_t off)
{
    {
        std::lock_guard<std::mutex> g(mu_);
        auto it = live_.find(off);
        if (it == live_.end()) return;
        int64_t bytes = it->second;
        live_.erase(it);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {   // merge with the interval after
            bytes += next->second;
            next = free_.erase(next);
        }
        bool merged = false;
        if (next != free_.begin()) {   // and with the one before
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                merged = true;
            }
        }
        if (!merged) free_[off] = bytes;
    }
    if (freed_) freed_->notify_all();
}

int64_t SlabSpace::largest()
{
    std::lock_guard<std::mutex> g(mu_);
    int64_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
}

int64_t SlabSpace::used()
{
    std::lock_guard<std::mutex> g(mu_);
    return used_;
}

DevicePool::~DevicePool()
{
    trim_locked();
    for (auto& kv : size_of_) {
        if (slab_ && slab_->holds(kv.first)) slab_->give(static_cast<char*>(kv.first) - slab_->base());
        else (void)hipFree(kv.first);
    }
    for (void* p : deferred_) slab_->give(static_cast<char*>(p) - slab_->base());
}

void DevicePool::free_locked(void* p, size_t sz)
{
    live_ -= sz;
    size_of_.erase(p);
    if (slab_ && slab_->holds(p)) {
        if (in_call_) deferred_.push_back(p);
        else slab_->give(static_cast<char*>(p) - slab_->base());
    } else {
        (void)hipFree(p);
    }
}

void DevicePool::begin_call()
{
    std::lock_guard<std::mutex> g(mu_);
    in_call_ = true;
}

void DevicePool::end_call()
{
    std::vector<void*> back;
    {
        std::lock_guard<std::mutex> g(mu_);
        in_call_ = false;
        back.swap(deferred_);
    }
    for (void* p : back) slab_->give(static_cast<char*>(p) - slab_->base());
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
    std::lock_guard<std::mutex> g(mu_);
    const size_t sz = round_size(bytes);
    if (slab_ && !outside_) {
        const int64_t off = slab_->take((int64_t)sz);
        if (off >= 0) {
            void* p = slab_->base() + off;
            size_of_[p] = sz;
            live_ += sz;
            return p;
        }
        // a full slab fails a call (its lane waits for space); a block made
        // on request between calls (a result's ids or rebased cells) comes
        // from hipMalloc instead
        if (in_call_) return nullptr;
    }
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
        trim_locked();
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
    std::lock_guard<std::mutex> g(mu_);
    auto it = size_of_.find(p);
    if (it == size_of_.end()) return;
    if (!caching_ || (slab_ && slab_->holds(p))) {
        free_locked(p, it->second);
        return;
    }
    live_ -= it->second;
    free_[it->second].push_back(p);
    cached_ += it->second;
}

void DevicePool::discard(void* p)
{
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    auto it = size_of_.find(p);
    if (it == size_of_.end()) return;
    free_locked(p, it->second);
}

void DevicePool::trim()
{
    std::lock_guard<std::mutex> g(mu_);
    trim_locked();
}

void DevicePool::trim_locked()
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
    if (!ptr_) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) (void)hipGetLastError();
        throw Error{HH_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed (this context holds " +
                                   std::to_string(pool->live_bytes()) + " bytes; device free " +
                                   std::to_string(free_b) + " of " + std::to_string(total_b) + ")"};
    }
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

void DevBuf::discard()
{
    if (pool_ && ptr_) pool_->discard(ptr_);
    pool_ = nullptr;
    ptr_ = nullptr;
    bytes_ = 0;
}

void DevBuf::reset()
{
    if (pool_ && ptr_) pool_->release(ptr_);
    pool_ = nullptr;
    ptr_ = nullptr;
    bytes_ = 0;
}

DevBuf CallMem::get(size_t bytes, const char* what)
{
    taken += (int64_t)bytes;
    if (!base) return DevBuf(pool, bytes);
    const int64_t n = align256(std::max<int64_t>((int64_t)bytes, 1));
    if (used + n > cap)
        throw Error{HH_ECAPACITY, std::string("the caller's arena (") + std::to_string(cap) +
                                      " bytes) cannot hold the call's " + what};
    DevBuf b = DevBuf::view(base + used, bytes);
    used += n;
    return b;
}

// ---------------------------------------------------------------- helpers

namespace {

void check(hipError_t e, const char* what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{HH_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
    }
}

int ceil_log2(int64_t n)
{
    int d = 0;
    while (((int64_t)1 << d) < n) ++d;
    return d;
}

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

// A call's descriptor block (host and device alike): trees at 0, the staging
// error word at `err`, the input table at `desc`.
struct CallLayout {
    int64_t err, desc, bytes;
};

CallLayout call_layout(int32_t n_trees, int32_t n_inputs)
{
    CallLayout c{};
    c.err = align256((int64_t)n_trees * (int64_t)sizeof(TreeDesc));
    c.desc = c.err + 256;
    c.bytes = c.desc + (int64_t)n_inputs * (int64_t)std::max(sizeof(ImageDesc), sizeof(PointsDesc));
    return c;
}

// Fixed part of an arena: level records, tree records, error word, scratch,
// then the cells.  Everything before the cells is copied back in one piece.
struct FixedLayout {
    int64_t info, rec, error, scalar, head_bytes, cells, bytes;
};

FixedLayout fixed_layout(int32_t n_trees, int64_t cells_cap)
{
    FixedLayout f{};
    int64_t off = 0;
    f.info = off;
    off += align256((int64_t)(kMaxLevels + 1) * (int64_t)sizeof(LevelInfo));
    f.rec = off;
    off += align256((int64_t)n_trees * kMaxLevels * kRecCh * 8);
    f.error = off;
    off += 256;
    f.scalar = off;
    off += 256;
    f.head_bytes = off;
    f.cells = off;
    off += align256(cells_cap * (int64_t)sizeof(Cell));
    f.bytes = off;
    return f;
}

struct Caps {
    int64_t cells, mem, half, work;   // cells, member entries, bytes per half, scratch bytes
};

// An arena has two parts: the front (the fixed part, the cells and the
// voters), which the results of a group keep, and the back (the two level
// halves and the per-level scratch), which only the group's levels use.
int64_t arena_front_bytes(const FixedLayout& f, const Caps& c, int32_t entry_bytes)
{
    return f.bytes + align256(c.mem * entry_bytes);
}

int64_t arena_back_bytes(const Caps& c) { return 2 * c.half + c.work; }

int64_t arena_bytes(const FixedLayout& f, const Caps& c, int32_t entry_bytes)
{
    return arena_front_bytes(f, c, entry_bytes) + arena_back_bytes(c);
}

// The parts of an arena whose front and back start at `front` and `back`
// (one block holds both when back = front + arena_front_bytes).
Arena carve(char* front, char* back, const FixedLayout& f, int32_t n_trees, const Caps& c, int32_t entry_bytes)
{
    Arena a{};
    a.info = reinterpret_cast<LevelInfo*>(front + f.info);
    a.rec = reinterpret_cast<int64_t*>(front + f.rec);
    a.error = reinterpret_cast<uint32_t*>(front + f.error);
    a.scalar = reinterpret_cast<int64_t*>(front + f.scalar);
    a.cells = reinterpret_cast<Cell*>(front + f.cells);
    a.cells_cap = c.cells;
    a.members = front + f.bytes;
    a.mem_cap = c.mem;
    a.half[0] = back;
    a.half[1] = back + c.half;
    a.half_cap = c.half;
    a.work = back + 2 * c.half;
    a.work_cap = c.work;
    a.n_trees = n_trees;
    a.entry_bytes = entry_bytes;
    for (const void* q : {(const void*)a.cells, (const void*)a.members, (const void*)a.half[0], (const void*)a.half[1],
                          (const void*)a.work})
        if (reinterpret_cast<uintptr_t>(q) & 255u) throw Error{HH_EINTERNAL, "arena part not 256-byte aligned"};
    return a;
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
        if (cfg->arena_hint) {
            const int64_t h = std::max<int64_t>(4096, align256((int64_t)std::min<uint64_t>(cfg->arena_hint, 1ull << 40)));
            ctx->half_cap = h;
            ctx->work_cap = std::max<int64_t>(4096, align256(h / 4));
            ctx->mem_cap = std::max<int64_t>(1024, h / 16);
            ctx->cells_cap = std::max<int64_t>(256, h / 256);
        }
        if (cfg->arena_limit_mib > 0) {
            // start within a quarter of the limit (the arena grows up to the limit)
            const int64_t lim = (int64_t)cfg->arena_limit_mib << 18;
            while (2 * ctx->half_cap + ctx->work_cap + 8 * ctx->mem_cap + 32 * ctx->cells_cap > lim &&
                   ctx->half_cap > 4096) {
                ctx->half_cap = std::max<int64_t>(4096, align256(ctx->half_cap / 2));
                ctx->work_cap = std::max<int64_t>(4096, align256(ctx->work_cap / 2));
                ctx->mem_cap = std::max<int64_t>(1024, ctx->mem_cap / 2);
                ctx->cells_cap = std::max<int64_t>(256, ctx->cells_cap / 2);
            }
        }
        ctx->grid = std::max(1, ctx->cu_count) * 8;
        noalloc_scratch(cfg->device);   // the device address of the fixed scratch, once per device
        const FixedLayout f = fixed_layout(kMaxTrees, 0);
        check(hipHostMalloc((void**)&ctx->h_fixed, (size_t)f.head_bytes, hipHostMallocDefault), "hipHostMalloc");
        check(hipHostMalloc((void**)&ctx->h_call, (size_t)call_layout(kMaxTrees * 2, kMaxTrees).bytes,
                            hipHostMallocDefault),
              "hipHostMalloc");
        ctx->h_trees = reinterpret_cast<TreeDesc*>(ctx->h_call);
        if (cfg->flags & HH_FLAG_TIMING) {
            ctx->events.resize(3 + 4 * kMaxLevels, nullptr);
            for (auto& e : ctx->events) check(hipEventCreate(&e), "hipEventCreate");
        }
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
    serve_stop(ctx);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    ctx->events.clear();
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    ctx->graph_exec = nullptr;
    {
        std::lock_guard<std::mutex> g(ctx->results_mu);
        for (hh_result* r : ctx->live_results) delete r;
        ctx->live_results.clear();
    }
    if (ctx->h_fixed) (void)hipHostFree(ctx->h_fixed);
    if (ctx->h_call) (void)hipHostFree(ctx->h_call);
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

// The message of an internal error: the checks that failed and their levels,
// the values the first failure recorded (scratch: the arena head's scratch
// words as read back), and the resumes the call made.
std::string internal_error_text(uint32_t err, const int64_t* scratch, int32_t resumes)
{
    std::string m = "a kernel index failed its range check";
    const std::pair<uint32_t, const char*> at[] = {
        {kErrAtCountTask, "k_count: a task's region or range out of bounds"},
        {kErrAtWriteTask, "k_write: a task's region or range out of bounds"},
        {kErrAtWriteVotes, "k_write: a kept child's votes differ from its count"},
        {kErrAtEmit, "emit: a region or task index past the level's totals"},
    };
    std::string what;
    for (const auto& a : at)
        if (err & a.first) what += (what.empty() ? "" : "; ") + std::string(a.second);
    std::string levels;
    for (int l = 0; l < kMaxLevels && kErrLevelShift + l < 32; ++l)
        if (err & (1u << (kErrLevelShift + l))) levels += (levels.empty() ? "" : ",") + std::to_string(l);
    if (!what.empty()) m += " (" + what + (levels.empty() ? "" : "; level " + levels) + ")";
    if (scratch && scratch[0] == 1) {
        m += "; first failure: check " + std::to_string(scratch[1] & 0xFFFFFFFF) + " at level " +
             std::to_string(scratch[1] >> 32) + ", values";
        for (int k = 2; k < 7; ++k) m += " " + std::to_string(scratch[k]);
    }
    m += "; resumes " + std::to_string(resumes);
    return m;
}

// The stage of a call whose sizes did not fit the caps c, from the level
// records the call left (the same checks the kernels make): -1 the root setup
// (level 0), l >= 0 the split decision of level l (its children's sizes are
// in info[l + 1]), -2 if every recorded size fits.
int failing_stage(const LevelInfo* info, int32_t dmax, const Caps& c, bool members, int32_t eb)
{
    auto fits = [&](const LevelInfo& x) {
        return half_layout(nullptr, x.P, x.L, x.NT, eb).end <= c.half && work_layout(nullptr, x.P, x.NT).end <= c.work;
    };
    if (!fits(info[0])) return -1;
    for (int l = 0; l < dmax; ++l) {
        const LevelInfo& x = info[l + 1];
        if (!fits(x) || x.cells_base + x.cells > c.cells || (members && x.mem_base + x.mem > c.mem)) return l;
    }
    return -2;
}

// Caps that hold the sizes x of the failing stage: each size that did not
// fit becomes `factor` times its need (the next levels are not known yet; a
// later overflow resumes again), rounded so that every part of an arena
// starts on a 256-byte boundary.
Caps grown_caps(const Caps& c, const LevelInfo& x, bool members, int32_t eb, double factor)
{
    auto grow = [&](int64_t cur, int64_t need) {
        return need <= cur ? cur : align256((int64_t)((double)need * factor));
    };
    Caps g = c;
    g.half = grow(c.half, half_layout(nullptr, x.P, x.L, x.NT, eb).end);
    g.work = grow(c.work, work_layout(nullptr, x.P, x.NT).end);
    g.cells = grow(c.cells, x.cells_base + x.cells);
    if (members) g.mem = grow(c.mem, x.mem_base + x.mem);
    return g;
}

}  // namespace

namespace {

// Host-side view of one image of a call.
struct ImagePlan {
    Plan plan;
    int32_t kind;
    int64_t n_points;          // point lists: from the input; images: known after the call
    int64_t xy_base;           // point lists: position of its points
};

// Statistics of one tree from the level and tree records (levels 0 .. D):
// level 0 is the root; level l+1 sums the parents of the tree at level l,
// delimited by the tree's record and the next tree's record at level l (or
// the level totals for the last tree).
std::vector<hh_level_stats> tree_stats(const LevelInfo* info, const int64_t* rec, int32_t t, int32_t n_trees,
                                       int32_t D, int64_t E, int32_t T)
{
    std::vector<hh_level_stats> v((size_t)D + 1, hh_level_stats{});
    const bool root_votes = E > T;   // every line crosses the root (code 0011)
    v[0].evaluated = 1;
    v[0].votes = E;
    v[0].code_tests = E;
    if (root_votes && D > 0) {
        v[0].split = 1;
        v[0].entries = E;
    }
    if (root_votes && D == 0) v[0].detected = 1;
    for (int l = 0; l < D; ++l) {
        const int64_t* r = rec + ((int64_t)t * kMaxLevels + l) * kRecCh;
        if (r[0] < 0) continue;   // the tree had no parent at level l
        int64_t nx[kRecCh] = {info[l].P, info[l].L, info[l + 1].P, info[l + 1].L, info[l + 1].cells,
                              info[l].votes, info[l + 1].mem};
        for (int t2 = t + 1; t2 < n_trees; ++t2) {
            const int64_t* r2 = rec + ((int64_t)t2 * kMaxLevels + l) * kRecCh;
            if (r2[0] >= 0) {
                for (int c = 0; c < kRecCh; ++c) nx[c] = r2[c];
                break;
            }
        }
        hh_level_stats& s = v[(size_t)l + 1];
        s.evaluated = 4 * (nx[0] - r[0]);
        s.code_tests = 4 * (nx[1] - r[1]);
        s.split = nx[2] - r[2];
        s.entries = nx[3] - r[3];
        s.detected = nx[4] - r[4];
        s.votes = nx[5] - r[5];
    }
    return v;
}

// [lo, hi) of the tree's cells (channel 4) or member entries (channel 6) at
// its finest level D, in the call's numbering.
void tree_range(const LevelInfo* info, const int64_t* rec, int32_t t, int32_t n_trees, int32_t D, int ch,
                int64_t& lo, int64_t& hi)
{
    const int l = D - 1;
    const int64_t base = ch == 4 ? info[D].cells_base : info[D].mem_base;
    const int64_t total = ch == 4 ? info[D].cells : info[D].mem;
    const int64_t* r = rec + ((int64_t)t * kMaxLevels + l) * kRecCh;
    lo = hi = -1;
    if (r[0] < 0) return;
    lo = base + r[ch];
    hi = base + total;
    for (int t2 = t + 1; t2 < n_trees; ++t2) {
        const int64_t* r2 = rec + ((int64_t)t2 * kMaxLevels + l) * kRecCh;
        if (r2[0] >= 0) {
            hi = base + r2[ch];
            break;
        }
    }
}

}  // namespace

namespace {

// A group's level pipeline needs more device memory than one arena may take.
struct BudgetExceeded {
    double budget;
};

// The level pipeline of one group of trees (trees[0 .. n_trees), points
// staged in xy) in an arena of its own.  When a level does not fit the
// arena, the group resumes at that level in a larger arena holding a copy of
// everything the finished stages left (level records, cells, voters, the
// level's tables, list and count results); a failure of the root setup
// reruns it.  On return the level and tree records are in ctx->h_fixed and
// the first back_bytes of the trees' block (the trees with their point
// counts, for the first group also the staging error word) in h_trees.
struct GroupRun {
    DevBuf arena;   // the front part (or the whole caller-arena view)
    DevBuf back;    // the back part (pool arenas only)
    FixedLayout fl{};
    Arena ar{};
    uint32_t err = 0;
};

// The part sizes of a level arena of `avail` bytes in the proportions of c
// (every part scaled by one factor).
Caps fit_caps(const Caps& c, int64_t avail, int32_t n_trees, int32_t eb, bool members)
{
    const double need = (double)arena_bytes(fixed_layout(n_trees, c.cells), c, eb);
    double f = (double)avail / need;
    for (int k = 0; k < 64; ++k, f *= 0.97) {
        Caps s{};
        s.cells = std::max<int64_t>(256, (int64_t)((double)c.cells * f));
        s.mem = members ? std::max<int64_t>(1024, (int64_t)((double)c.mem * f)) : 0;
        s.half = std::max<int64_t>(4096, (int64_t)((double)c.half * f) & ~(int64_t)255);
        s.work = std::max<int64_t>(4096, (int64_t)((double)c.work * f) & ~(int64_t)255);
        if (arena_bytes(fixed_layout(n_trees, s.cells), s, eb) <= avail) return s;
    }
    throw Error{HH_ECAPACITY, "the caller's arena (" + std::to_string(avail) +
                                  " bytes left after the call's inputs) is too small for a level arena"};
}

void run_group(hh_ctx* ctx, CallMem& mem, const Plan& p0, int32_t entry_bytes, TreeDesc* trees, int32_t n_trees,
               int32_t dmax, const uint32_t* xy, const int32_t* ids, TreeDesc* h_trees, int64_t back_bytes,
               hh_timing& tm, GroupRun& g)
{
    hipStream_t st = ctx->stream;
    DevicePool* pool = &ctx->pool;
    const bool members = p0.membership;
    const bool timing = !ctx->events.empty();
    const int64_t n_rec = (int64_t)n_trees * kMaxLevels * kRecCh;
    const int32_t task_steps = ctx->task_steps;   // fixed for the whole run: a resume reuses built tasks
    int count_grid = level_grid(0, p0.variant, p0.wide, entry_bytes, ctx->cu_count);
    int write_grid = level_grid(1, p0.variant, p0.wide, entry_bytes, ctx->cu_count);
    if (ctx->wg_per_cu > 0) {
        count_grid = std::min(count_grid, ctx->wg_per_cu * ctx->cu_count);
        write_grid = std::min(write_grid, ctx->wg_per_cu * ctx->cu_count);
    }
    // the launches from stage `from` (-1: the root setup; l: level l's split
    // decision) to the finest level, then the copies of the level records
    // back to the host (enqueued only)
    auto enqueue_levels = [&](int from) {
        if (from < 0) check(launch_roots(g.ar, trees, n_trees, xy, ids, task_steps, ctx->grid, st), "roots");
        LevelArgs la{};
        la.ar = g.ar;
        la.trees = trees;
        la.xy = xy;
        la.keep_members = members ? 1 : 0;
        la.task_steps = task_steps;
        la.queue_batch = ctx->queue_batch;
        for (int l = std::max(from, 0); l < dmax; ++l) {
            la.level = l;
            mark(ctx, 3 + 4 * l);
            if (l != from) check(launch_count(la, p0.variant, p0.wide, count_grid, st), "count");
            mark(ctx, 4 + 4 * l);
            if (l != from) check(launch_decide(la, kRangeGrid, st), "decide");
            check(launch_emit(la, kRangeGrid, st), "emit");
            mark(ctx, 5 + 4 * l);
            if (l + 1 < dmax || members) check(launch_write(la, p0.variant, p0.wide, write_grid, st), "write");
            mark(ctx, 6 + 4 * l);
        }
        mark(ctx, 2);
        check(hipMemcpyAsync(ctx->h_fixed, g.ar.info, (size_t)g.fl.head_bytes, hipMemcpyDeviceToHost, st),
              "copy level records");
        check(hipMemcpyAsync(h_trees, trees, (size_t)back_bytes, hipMemcpyDeviceToHost, st), "copy trees back");
    };
    // wait for them; false if a level outgrew the arena
    auto collect = [&]() {
        sync(ctx);
        g.err = *reinterpret_cast<const uint32_t*>(ctx->h_fixed + g.fl.error);
        return !(g.err & kErrArena) || (g.err & (kErrPointRange | kErrInternal));
    };
    auto launch_levels = [&](int from) {
        enqueue_levels(from);
        return collect();
    };
    auto account = [&](int first) {
        const LevelInfo* info = reinterpret_cast<const LevelInfo*>(ctx->h_fixed + g.fl.info);
        if (timing) {
            for (int l = first; l < dmax; ++l) {
                const double c = elapsed(ctx, 3 + 4 * l, 4 + 4 * l), w = elapsed(ctx, 5 + 4 * l, 6 + 4 * l);
                tm.count_ms += c;
                tm.write_ms += w;
                tm.vote_ms += c + w;
                tm.decide_ms += elapsed(ctx, 4 + 4 * l, 5 + 4 * l);
            }
            tm.vote_launches += dmax + (members ? dmax : dmax - 1);
            tm.decide_launches += 2 * dmax;
        }
        for (int l = 0; l < dmax; ++l) {
            tm.vote_entries += info[l].L;
            if (l + 1 < dmax) tm.vote_written += info[l + 1].L;
            if (members) tm.vote_written += info[l + 1].mem;
        }
    };
    // part sizes that hold the needs of the stage that overflowed (factor x need)
    auto learn = [&](const Caps& caps, double factor, Caps& grown) {
        const LevelInfo* info = reinterpret_cast<const LevelInfo*>(ctx->h_fixed + g.fl.info);
        const int f = failing_stage(info, dmax, caps, members, entry_bytes);
        if (f == -2) throw Error{HH_EINTERNAL, "arena overflow reported but every level fits"};
        grown = grown_caps(caps, info[f + 1], members, entry_bytes, factor);   // f = -1: the root level
        return f;
    };

    if (mem.base) {
        // the caller's arena: the rest of it is the level arena; up to three
        // reruns from the root, each with the parts re-split by the sizes the
        // runs so far measured.  With HH_FLAG_GRAPH the first run's launches
        // are a captured graph, replayed when the next call bakes in the same
        // addresses and sizes.
        const bool graph = (ctx->cfg.flags & HH_FLAG_GRAPH) && !timing && mem.graph_ok && st != nullptr;
        const int64_t avail = mem.left() & ~(int64_t)255;
        DevBuf whole = mem.get((size_t)std::max<int64_t>(avail, 256), "level arena");
        mem.taken -= (int64_t)whole.bytes();
        mem.arena_peak = std::max<int64_t>(mem.arena_peak, avail);
        for (int attempt = 0; attempt < 4; ++attempt) {
            const Caps want{ctx->cells_cap, members ? ctx->mem_cap : 0, ctx->half_cap, ctx->work_cap};
            const Caps caps = fit_caps(want, avail, n_trees, entry_bytes, members);
            g.fl = fixed_layout(n_trees, caps.cells);
            g.ar = carve(whole.as<char>(), whole.as<char>() + arena_front_bytes(g.fl, caps, entry_bytes), g.fl, n_trees,
                         caps, entry_bytes);
            g.arena = DevBuf::view(whole.get(), whole.bytes());
            bool ok;
            if (graph && attempt == 0) {
                // every address and size the launches bake in
                std::string key;
                auto put = [&](const auto& v) { key.append(reinterpret_cast<const char*>(&v), sizeof(v)); };
                for (const auto& v : {(int64_t)(intptr_t)whole.get(), caps.cells, caps.mem, caps.half, caps.work,
                                      (int64_t)(intptr_t)trees, (int64_t)(intptr_t)xy, (int64_t)(intptr_t)ids,
                                      (int64_t)(intptr_t)h_trees, back_bytes, (int64_t)n_trees, (int64_t)dmax,
                                      (int64_t)entry_bytes, (int64_t)p0.variant, (int64_t)p0.wide,
                                      (int64_t)members, (int64_t)task_steps, (int64_t)ctx->queue_batch,
                                      (int64_t)count_grid, (int64_t)write_grid})
                    put(v);
                if (!ctx->graph_exec || ctx->graph_key != key) {
                    if (ctx->graph_exec) check(hipGraphExecDestroy(ctx->graph_exec), "hipGraphExecDestroy");
                    ctx->graph_exec = nullptr;
                    check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
                    hipGraph_t gr = nullptr;
                    try {
                        check(launch_clear(g.ar, n_rec, st), "clear");
                        enqueue_levels(-1);
                    } catch (...) {
                        (void)hipStreamEndCapture(st, &gr);
                        if (gr) (void)hipGraphDestroy(gr);
                        throw;
                    }
                    check(hipStreamEndCapture(st, &gr), "hipStreamEndCapture");
                    const hipError_t e = hipGraphInstantiate(&ctx->graph_exec, gr, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(gr);
                    check(e, "hipGraphInstantiate");
                    ctx->graph_key = key;
                } else {
                    ++ctx->graph_replays;
                    tm.graph_replayed = 1;
                }
                check(hipGraphLaunch(ctx->graph_exec, st), "hipGraphLaunch");
                ok = collect();
            } else {
                check(launch_clear(g.ar, n_rec, st), "clear");
                ok = launch_levels(-1);
            }
            if (ok) {
                account(0);
                return;
            }
            Caps grown{};
            learn(caps, 1.25, grown);
            ++tm.resumes;
            ctx->half_cap = std::max(ctx->half_cap, grown.half);
            ctx->work_cap = std::max(ctx->work_cap, grown.work);
            ctx->cells_cap = std::max(ctx->cells_cap, grown.cells);
            if (members) ctx->mem_cap = std::max(ctx->mem_cap, grown.mem);
        }
        throw Error{HH_ECAPACITY, "the caller's arena (" + std::to_string(mem.cap) +
                                      " bytes) cannot hold the call's level lists"};
    }

    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        total_b = (size_t)64 << 30;
    }
    // one arena; a resume holds two for a moment
    const double budget = ctx->cfg.hbm_budget_bytes > 0 ? (double)ctx->cfg.hbm_budget_bytes
                          : ctx->cfg.arena_limit_mib > 0 ? (double)ctx->cfg.arena_limit_mib * (1 << 20)
                                                         : 0.35 * (double)total_b;
    int from = -1;   // -1: from the root setup; l: from level l's split decision
    for (int run = 0;; ++run) {
        if (run >= 64) throw Error{HH_ECAPACITY, "arena sizing did not converge"};
        Caps caps{ctx->cells_cap, members ? ctx->mem_cap : 0, ctx->half_cap, ctx->work_cap};
        if (run == 0 && ctx->arena_hint_bytes > 0) {
            // a size expected for this call (serving lanes): the parts in the
            // learnt proportions, scaled to it; a resume grows what overflows
            try {
                caps = fit_caps(caps, ctx->arena_hint_bytes, n_trees, entry_bytes, members);
            } catch (const Error&) {
            }
        }
        const FixedLayout nfl = fixed_layout(n_trees, caps.cells);
        if (run == 0 && (double)arena_bytes(nfl, caps, entry_bytes) > budget) throw BudgetExceeded{budget};
        DevBuf nfront(pool, (size_t)arena_front_bytes(nfl, caps, entry_bytes));
        DevBuf nback(pool, (size_t)arena_back_bytes(caps));
        mem.arena_peak = std::max<int64_t>(mem.arena_peak, arena_bytes(nfl, caps, entry_bytes));
        const Arena nar = carve(nfront.as<char>(), nback.as<char>(), nfl, n_trees, caps, entry_bytes);
        if (from < 0) {
            check(launch_clear(nar, n_rec, st), "clear");
        } else {
            // carry the finished stages over (both arenas have the same fixed head)
            const LevelInfo* info = reinterpret_cast<const LevelInfo*>(ctx->h_fixed + g.fl.info);
            const LevelInfo& lv = info[from];
            const LevelInfo& nx = info[from + 1];
            auto copy = [&](void* dst, const void* src, int64_t bytes) {
                if (bytes > 0) check(hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice, st), "resume copy");
            };
            copy(nar.info, g.ar.info, g.fl.head_bytes);
            check(hipMemsetAsync(nar.error, 0, sizeof(uint32_t), st), "resume clear");
            copy(nar.cells, g.ar.cells, nx.cells_base * (int64_t)sizeof(Cell));
            if (members) copy(nar.members, g.ar.members, nx.mem_base * entry_bytes);
            copy(nar.half[from & 1], g.ar.half[from & 1], half_layout(nullptr, lv.P, lv.L, lv.NT, entry_bytes).end);
            copy(nar.work, g.ar.work, work_layout(nullptr, lv.P, lv.NT).end);
            sync(ctx);   // the old arena goes back to the pool only once it is read
        }
        if (run > 0) {   // a smaller arena is of no further use
            g.arena.discard();
            g.back.discard();
        }
        g.arena = std::move(nfront);
        g.back = std::move(nback);
        g.ar = nar;
        g.fl = nfl;
        if (launch_levels(from)) {
            account(std::max(from, 0));
            return;
        }
        // lists about double per level while most regions split: twice the
        // need, less if that exceeds the budget
        Caps grown{};
        bool ok = false;
        int f = -2;
        for (double factor : {2.0, 1.25, 1.0}) {
            f = learn(caps, factor, grown);
            if ((double)arena_bytes(fixed_layout(n_trees, grown.cells), grown, entry_bytes) <= budget) {
                ok = true;
                break;
            }
        }
        if (!ok) throw BudgetExceeded{budget};
        ++tm.resumes;
        ctx->half_cap = grown.half;
        ctx->work_cap = grown.work;
        ctx->cells_cap = grown.cells;
        if (members) ctx->mem_cap = grown.mem;
        from = f;
    }
}

}  // namespace

hh_status engine_detect(hh_ctx* ctx, const hh_input* in, hh_result** out)
{
    return engine_detect_batch(ctx, in, 1, out);
}

hh_status engine_detect_batch(hh_ctx* ctx, const hh_input* inputs, int32_t n, hh_result** out, CallMem* ext)
{
    hipStream_t st = ctx->stream;
    DevicePool* pool = &ctx->pool;
    check(hipSetDevice(ctx->device), "hipSetDevice");
    const bool timing = !ctx->events.empty();
    const uint32_t passes = ctx->cfg.passes;
    const int32_t n_pass = __builtin_popcount(passes);
    if (n < 1) throw Error{HH_EINVAL, "a call needs at least one input"};
    if ((int64_t)n * n_pass > kMaxTrees) throw Error{HH_ECAPACITY, "too many images in one call"};
    const int32_t n_trees = n * n_pass;
    // device memory of the call: the pool, or the caller's arena front to back
    CallMem mem;
    mem.pool = pool;
    if (ext) {
        mem = *ext;
    } else if (ctx->cfg.arena) {
        std::lock_guard<std::mutex> g(ctx->results_mu);
        if (ctx->arena_results > 0)
            throw Error{HH_EBUSY, "results of an earlier call still live in the caller's arena: free them first"};
        mem.base = static_cast<char*>(ctx->cfg.arena);
        mem.cap = (int64_t)ctx->cfg.arena_bytes;
    }

    // ---- plans; every input of a call is of one kind
    std::vector<ImagePlan> ip((size_t)n);
    int32_t dmax_all = 0;
    for (int32_t k = 0; k < n; ++k) {
        const hh_input* in = &inputs[k];
        ip[(size_t)k].plan = make_plan(ctx, in);
        ip[(size_t)k].kind = in->kind;
        if (in->kind != 0 && in->kind != 1 && in->kind != 2)
            throw Error{HH_EINVAL, "input kind must be 0 (points), 1 (binary image) or 2 (gray image)"};
        if (in->kind == 2 && in->edge_threshold < 0) throw Error{HH_EINVAL, "edge_threshold must be >= 0"};
        if (in->kind == 2 && ip[(size_t)k].plan.dmax == 0)
            throw Error{HH_EINVAL, "gray images need depth >= 1"};
        if (in->kind != inputs[0].kind) throw Error{HH_EINVAL, "all inputs of a call must be of one kind"};
        dmax_all = std::max(dmax_all, ip[(size_t)k].plan.dmax);
    }
    mem.graph_ok = true;
    for (int32_t k = 0; k < n; ++k) mem.graph_ok = mem.graph_ok && inputs[k].on_device;
    const Plan& p0 = ip[0].plan;   // variant, compares and membership are the context's
    const int32_t kind = inputs[0].kind;
    // point lists and gray images keep their point ids in the entries
    const int32_t entry_bytes = kind == 1 ? 4 : 8;

    auto store = std::make_shared<CallStore>();
    DevBuf hx, hy, himg, tcount, tpre, d_ids;
    int64_t n_tiles = 0, total_points = 0;
    const CallLayout cl = call_layout(n_trees, n);
    PointsDesc* const h_lists = reinterpret_cast<PointsDesc*>(ctx->h_call + cl.desc);
    ImageDesc* const h_images = reinterpret_cast<ImageDesc*>(ctx->h_call + cl.desc);
    uint32_t* const h_err = reinterpret_cast<uint32_t*>(ctx->h_call + cl.err);
    if (kind == 0) {
        // point lists: host lists are gathered into one upload
        int64_t host_points = 0;
        for (int32_t k = 0; k < n; ++k) {
            const hh_input* in = &inputs[k];
            if (in->n_points < 0 || in->n_points > INT32_MAX) throw Error{HH_EINVAL, "bad n_points"};
            if (in->n_points > 0 && (!in->x || !in->y)) throw Error{HH_EINVAL, "x and y must not be NULL"};
            if (!in->on_device) {
                for (int64_t q = 0; q < in->n_points; ++q)
                    if (in->x[q] < 0 || in->x[q] >= in->width || in->y[q] < 0 || in->y[q] >= in->height)
                        throw Error{HH_EINVAL, "point " + std::to_string(q) + " of input " + std::to_string(k) +
                                                   " outside the image"};
                host_points += in->n_points;
            }
            ip[(size_t)k].n_points = in->n_points;
            ip[(size_t)k].xy_base = total_points;
            total_points += in->n_points;
        }
        if (host_points > 0) {
            std::vector<int32_t> hxv((size_t)host_points), hyv((size_t)host_points);
            int64_t at = 0;
            for (int32_t k = 0; k < n; ++k) {
                const hh_input* in = &inputs[k];
                if (in->on_device || in->n_points == 0) continue;
                std::copy(in->x, in->x + in->n_points, hxv.begin() + at);
                std::copy(in->y, in->y + in->n_points, hyv.begin() + at);
                at += in->n_points;
            }
            hx = mem.get((size_t)host_points * 4, "staged x");
            hy = mem.get((size_t)host_points * 4, "staged y");
            check(hipMemcpyAsync(hx.get(), hxv.data(), (size_t)host_points * 4, hipMemcpyHostToDevice, st), "copy x");
            check(hipMemcpyAsync(hy.get(), hyv.data(), (size_t)host_points * 4, hipMemcpyHostToDevice, st), "copy y");
            check(hipStreamSynchronize(st), "copy points");   // the host vectors end here
        }
        int64_t at = 0;
        for (int32_t k = 0; k < n; ++k) {
            const hh_input* in = &inputs[k];
            PointsDesc& d = h_lists[k];
            d.x = in->on_device ? in->x : hx.as<int32_t>() + at;
            d.y = in->on_device ? in->y : hy.as<int32_t>() + at;
            if (!in->on_device) at += in->n_points;
            d.n = in->n_points;
            d.base = ip[(size_t)k].xy_base;
            d.width = in->width;
            d.height = in->height;
        }
        store->points = mem.get((size_t)std::max<int64_t>(total_points, 1) * 4, "packed points");
    } else {
        // binary or gray images: host images are packed into one upload
        int64_t host_bytes = 0, pix_all = 0;
        for (int32_t k = 0; k < n; ++k) {
            const hh_input* in = &inputs[k];
            if (!in->image) throw Error{HH_EINVAL, "image must not be NULL"};
            const int64_t stride = in->row_stride ? in->row_stride : in->width;
            if (stride < in->width) throw Error{HH_EINVAL, "row_stride < width"};
            if (!in->on_device) host_bytes += (int64_t)in->width * in->height;
            pix_all += (int64_t)in->width * in->height;
        }
        if (host_bytes > 0) himg = mem.get((size_t)host_bytes, "staged images");
        int64_t at = 0;
        for (int32_t k = 0; k < n; ++k) {
            const hh_input* in = &inputs[k];
            const int64_t stride = in->row_stride ? in->row_stride : in->width;
            ImageDesc& d = h_images[k];
            d.width = in->width;
            d.height = in->height;
            d.n_pix = (int64_t)in->width * in->height;
            d.tile0 = n_tiles;
            d.edge_threshold = kind == 2 ? in->edge_threshold : 0;
            d.pad = 0;
            n_tiles += cdiv(d.n_pix, kPixTile);
            if (in->on_device) {
                d.image = in->image;
                d.row_stride = stride;
            } else {
                check(hipMemcpy2DAsync(himg.as<uint8_t>() + at, (size_t)in->width, in->image, (size_t)stride,
                                       (size_t)in->width, (size_t)in->height, hipMemcpyHostToDevice, st),
                      "copy image");
                d.image = himg.as<uint8_t>() + at;
                d.row_stride = in->width;
                at += d.n_pix;
            }
            ip[(size_t)k].n_points = -1;
        }
        store->points = mem.get((size_t)std::max<int64_t>(pix_all, 1) * 4, "packed points");
        const int64_t sets = kind == 2 ? 2 : 1;   // gray images count ALPHA and BETA apart
        tcount = mem.get((size_t)std::max<int64_t>(n_tiles * sets, 1) * 4, "tile counts");
        tpre = mem.get((size_t)std::max<int64_t>(n_tiles * sets, 1) * 8, "tile prefixes");
        if (kind == 2) d_ids = mem.get((size_t)std::max<int64_t>(pix_all, 1) * 4, "point ids");
    }
    uint32_t* xy = store->points.as<uint32_t>();

    // ---- trees: image k, enabled pass p
    int32_t tree_pass[2] = {-1, -1};
    {
        int32_t t = 0;
        for (int32_t k = 0; k < n; ++k)
            for (int p = 0; p < 2; ++p) {
                if (!(passes & (1u << p))) continue;
                TreeDesc& T = ctx->h_trees[t++];
                const Plan& pl = ip[(size_t)k].plan;
                T.xy_base = kind == 0 ? ip[(size_t)k].xy_base : 0;   // images: set on the device
                T.n_points = kind == 0 ? ip[(size_t)k].n_points : 0;
                T.s_log2 = pl.s_log2;
                T.dmax = pl.dmax;
                T.threshold = pl.T;
                T.pass = p;
                T.image = k;
                T.image_points = kind == 0 ? (int32_t)ip[(size_t)k].n_points : 0;
            }
        int32_t c = 0;
        for (int p = 0; p < 2; ++p)
            if (passes & (1u << p)) tree_pass[c++] = p;
    }
    // trees, a cleared staging error word and the input table in one upload
    *h_err = 0;
    const int64_t call_bytes = cl.desc + (int64_t)n * (kind == 0 ? sizeof(PointsDesc) : sizeof(ImageDesc));
    DevBuf d_call = mem.get((size_t)call_bytes, "descriptors");
    check(hipMemcpyAsync(d_call.get(), ctx->h_call, (size_t)call_bytes, hipMemcpyHostToDevice, st), "copy descriptors");
    TreeDesc* const d_trees = d_call.as<TreeDesc>();
    uint32_t* const d_err = reinterpret_cast<uint32_t*>(d_call.as<char>() + cl.err);
    char* const d_desc = d_call.as<char>() + cl.desc;

    // ---- edge staging of every input (the groups below share it)
    hh_timing tm{};
    mark(ctx, 0);
    if (kind == 0) {
        check(launch_pack_points(reinterpret_cast<const PointsDesc*>(d_desc), n, total_points, xy, d_err, st), "pack");
    } else if (kind == 2) {
        SobelArgs sa{};
        sa.images = reinterpret_cast<const ImageDesc*>(d_desc);
        sa.n_images = n;
        sa.n_tiles = n_tiles;
        sa.xy = xy;
        sa.ids = d_ids.as<int32_t>();
        sa.tile_count = tcount.as<int32_t>();
        sa.tile_pre = tpre.as<int64_t>();
        sa.trees = d_trees;
        sa.n_trees = n_trees;
        check(launch_sobel(sa, st), "sobel");
    } else {
        ExtractArgs ea{};
        ea.images = reinterpret_cast<const ImageDesc*>(d_desc);
        ea.n_images = n;
        ea.n_tiles = n_tiles;
        ea.xy = xy;
        ea.tile_count = tcount.as<int32_t>();
        ea.tile_pre = tpre.as<int64_t>();
        ea.trees = d_trees;
        ea.n_trees = n_trees;
        check(launch_extract(ea, st), "extract");
    }
    mark(ctx, 1);

    // ---- groups of consecutive inputs whose level lists fit one arena.
    // One group holds the whole call unless an earlier call on the context
    // learnt a point limit; a group that exceeds the budget halves the limit
    // and the remaining inputs are grouped again.
    bool counts_known = kind == 0;
    auto points_of = [&](int32_t k) { return (int64_t)ctx->h_trees[(size_t)k * n_pass].image_points; };
    auto ensure_counts = [&] {
        if (counts_known) return;
        check(hipMemcpyAsync(ctx->h_trees, d_trees, (size_t)(cl.err + 4), hipMemcpyDeviceToHost, st),
              "copy trees back");
        sync(ctx);
        counts_known = true;
    };
    std::vector<std::unique_ptr<hh_result>> res((size_t)n);
    int32_t n_groups = 0;
    for (int32_t k0 = 0; k0 < n;) {
        int32_t k1 = n;
        if (ctx->group_points > 0 && n > 1 && !mem.base) {
            ensure_counts();
            int64_t sum = points_of(k0);
            for (k1 = k0 + 1; k1 < n && sum + points_of(k1) <= ctx->group_points; ++k1) sum += points_of(k1);
        }
        int32_t dmax = 0;
        for (int32_t k = k0; k < k1; ++k) dmax = std::max(dmax, ip[(size_t)k].plan.dmax);
        const int32_t t0g = k0 * n_pass, ntg = (k1 - k0) * n_pass;
        GroupRun g;
        try {
            // the first group also brings back the staging error word
            const int64_t back = k0 == 0 ? cl.err + 4 : (int64_t)ntg * (int64_t)sizeof(TreeDesc);
            run_group(ctx, mem, p0, entry_bytes, d_trees + t0g, ntg, dmax, xy,
                      kind == 2 ? d_ids.as<int32_t>() : nullptr, ctx->h_trees + t0g, back, tm, g);
        } catch (const BudgetExceeded& b) {
            if (k1 - k0 <= 1)
                throw Error{HH_ECAPACITY, "input " + std::to_string(k0) + " needs more than " +
                                              std::to_string((int64_t)(b.budget / 1e9)) +
                                              " GB of device memory for its level lists"};
            counts_known = true;   // run_group copied the group's trees back
            int64_t sum = 0;
            for (int32_t k = k0; k < k1; ++k) sum += points_of(k);
            ctx->group_points = std::max<int64_t>(1, sum / 2);
            continue;
        }
        if (g.err & kErrInternal)
            throw Error{HH_EINTERNAL,
                        internal_error_text(g.err, reinterpret_cast<const int64_t*>(ctx->h_fixed + g.fl.scalar),
                                            tm.resumes)};
        if (*h_err & kErrPointRange) throw Error{HH_EINVAL, "a device point lies outside the image"};
        counts_known = true;

        const LevelInfo* info = reinterpret_cast<const LevelInfo*>(ctx->h_fixed + g.fl.info);
        const int64_t* rec = reinterpret_cast<const int64_t*>(ctx->h_fixed + g.fl.rec);
        {
            // the level arena this group needed at least: its largest level, its cells and voters
            Caps need{info[dmax].cells_base + info[dmax].cells, p0.membership ? info[dmax].mem_base + info[dmax].mem : 0,
                      0, 0};
            for (int l = 0; l <= dmax; ++l) {
                need.half = std::max(need.half, half_layout(nullptr, info[l].P, info[l].L, info[l].NT, entry_bytes).end);
                need.work = std::max(need.work, work_layout(nullptr, info[l].P, info[l].NT).end);
            }
            mem.arena_need = std::max(mem.arena_need, arena_bytes(fixed_layout(ntg, need.cells), need, entry_bytes));
        }
        auto gs = std::make_shared<GroupStore>();
        gs->call = store;
        const Cell* gcells = g.ar.cells;
        const void* gmembers = g.ar.members;
        if ((k0 == 0 && k1 == n) || !mem.base) {
            // one group, or a pool arena: the results keep the front part
            // (cells and voters) and point into it; the back part returns to
            // the pool when the group ends
            gs->arena = std::move(g.arena);
        } else {
            // several groups in the caller's arena: keep exact copies of the
            // cells and voters, and let the next group reuse the arena
            const int64_t nc = info[dmax].cells_base + info[dmax].cells;
            const int64_t nm = p0.membership ? info[dmax].mem_base + info[dmax].mem : 0;
            gs->cells = DevBuf(pool, (size_t)std::max<int64_t>(nc, 1) * sizeof(Cell));
            if (nc > 0)
                check(hipMemcpyAsync(gs->cells.get(), g.ar.cells, (size_t)nc * sizeof(Cell), hipMemcpyDeviceToDevice,
                                     st),
                      "copy cells");
            if (nm > 0) {
                gs->members = DevBuf(pool, (size_t)nm * entry_bytes);
                check(hipMemcpyAsync(gs->members.get(), g.ar.members, (size_t)nm * entry_bytes,
                                     hipMemcpyDeviceToDevice, st),
                      "copy members");
            }
            gcells = gs->cells.as<Cell>();
            gmembers = gs->members.get();
        }
        ++n_groups;

        // ---- one result per image of the group
        for (int32_t k = k0; k < k1; ++k) {
            auto r = std::make_unique<hh_result>();
            r->ctx = ctx;
            r->store = gs;
            r->n_trees = n_pass;
            r->tree_pass[0] = tree_pass[0];
            r->tree_pass[1] = tree_pass[1];
            r->entry_bytes = entry_bytes;
            r->have_members = p0.membership;
            const Plan& pl = ip[(size_t)k].plan;
            const int32_t tl = (k - k0) * n_pass;   // the image's first tree in the group
            const int64_t E = points_of(k);
            r->xy = xy + ctx->h_trees[(size_t)k * n_pass].xy_base;
            r->members_base = gmembers;
            int64_t code_tests = 0, cells_lo = -1, cells_hi = -1, mem_lo = -1, mem_hi = -1;
            for (int32_t q = 0; q < n_pass; ++q) {
                const int32_t t = tl + q;
                const int p = tree_pass[q];
                // a tree's own points (a gray image's passes see different sets)
                r->stats[p] = tree_stats(info, rec, t, ntg, pl.dmax, ctx->h_trees[(size_t)(t0g + t)].n_points, pl.T);
                for (const auto& lv : r->stats[p]) code_tests += lv.code_tests;
                r->info.n_cells[p] = r->stats[p][(size_t)pl.dmax].detected;
                if (pl.dmax > 0 && r->info.n_cells[p] > 0) {
                    int64_t lo, hi, mlo, mhi;
                    tree_range(info, rec, t, ntg, pl.dmax, 4, lo, hi);
                    tree_range(info, rec, t, ntg, pl.dmax, 6, mlo, mhi);
                    if (hi - lo != r->info.n_cells[p])
                        throw Error{HH_EINTERNAL, "cell count does not match the statistics"};
                    if (cells_lo < 0) {
                        cells_lo = lo;
                        mem_lo = mlo;
                    }
                    cells_hi = hi;
                    mem_hi = mhi;
                }
            }
            r->n_cells_total = r->info.n_cells[0] + r->info.n_cells[1];
            if (pl.dmax > 0) {
                r->cells = cells_lo >= 0 ? gcells + cells_lo : nullptr;
                if (cells_lo >= 0 && cells_hi - cells_lo != r->n_cells_total)
                    throw Error{HH_EINTERNAL, "an image's cells are not contiguous"};
                if (p0.membership && mem_lo >= 0) {
                    r->mem_base = mem_lo;
                    r->members = static_cast<const char*>(gmembers) + mem_lo * entry_bytes;
                    r->info.member_slots = mem_hi - mem_lo;
                }
            } else if (r->n_cells_total > 0) {
                // depth 0: the root is the finest region; every line votes for it
                r->depth0 = true;
                r->depth0_cells = mem.get(sizeof(Cell) * (size_t)n_pass, "cells");
                std::vector<Cell> hc;
                for (int32_t q = 0; q < n_pass; ++q) {
                    if (r->info.n_cells[tree_pass[q]] == 0) continue;
                    Cell c{};
                    c.votes = (int32_t)E;
                    c.pass = tree_pass[q];
                    c.member_off = p0.membership ? 0 : -1;
                    hc.push_back(c);
                }
                check(hipMemcpyAsync(r->depth0_cells.get(), hc.data(), sizeof(Cell) * hc.size(),
                                     hipMemcpyHostToDevice, st),
                      "copy cells");
                r->cells = r->depth0_cells.as<Cell>();
                if (p0.membership) {
                    r->members = r->xy;   // the voters are all points, in order
                    r->entry_bytes = 4;
                    r->info.member_slots = E;
                }
                sync(ctx);
            }
            r->info.n_points = E;
            r->info.width = pl.W;
            r->info.height = pl.H;
            r->info.side_pow2 = (int32_t)pl.S;
            r->info.depth = pl.dmax;
            r->info.threshold = pl.T;
            r->info.passes = passes;
            r->info.compare_bits = (p0.variant == HH_VARIANT_CIRCLE || p0.wide) ? 64 : 32;
            r->info.code_tests = code_tests;
            res[(size_t)k] = std::move(r);
        }
        k0 = k1;
    }
    sync(ctx);   // the copies of the last group
    ctx->last_call_bytes = mem.taken + mem.arena_peak;
    ctx->last_call_need = mem.taken + mem.arena_need;
    if (timing) {
        tm.total_ms = elapsed(ctx, 0, 2);
        tm.extract_ms = elapsed(ctx, 0, 1);
    }
    std::lock_guard<std::mutex> g(ctx->results_mu);
    for (int32_t k = 0; k < n; ++k) {
        res[(size_t)k]->timing = tm;
        res[(size_t)k]->timing.groups = n_groups;
        res[(size_t)k]->in_arena = mem.base != nullptr && !ext;
        out[k] = res[(size_t)k].release();
        ctx->live_results.insert(out[k]);
        if (out[k]->in_arena) ++ctx->arena_results;
    }
    return HH_OK;
}

hh_status engine_detect_noalloc(hh_ctx* ctx, const hh_input* in, hh_cell* cells, int64_t cells_cap,
                                int32_t* members, int64_t members_cap, hh_level_stats* stats, int64_t* n_cells,
                                int64_t* n_members)
{
    check(hipSetDevice(ctx->device), "hipSetDevice");
    if (cells_cap < 0 || members_cap < 0 || (cells_cap > 0 && !cells) || (members_cap > 0 && !members))
        throw Error{HH_EINVAL, "bad output buffers"};
    CallMem mem;
    mem.base = static_cast<char*>(noalloc_scratch(ctx->device));
    mem.cap = kNoAllocScratchBytes;
    hh_result* raw = nullptr;
    engine_detect_batch(ctx, in, 1, &raw, &mem);
    // the result lives only for this call
    {
        std::lock_guard<std::mutex> g(ctx->results_mu);
        ctx->live_results.erase(raw);
    }
    std::unique_ptr<hh_result> r(raw);
    const hh_result_info& info = r->info;
    const int64_t nc = r->n_cells_total;
    // voters, compact: a depth-0 cell holds every point
    const int64_t nm = !r->have_members ? 0 : r->depth0 ? (int64_t)info.n_points * nc : info.member_slots;
    n_cells[0] = info.n_cells[0];
    n_cells[1] = info.n_cells[1];
    *n_members = nm;
    for (int p = 0; p < 2; ++p)
        for (int l = 0; l <= HH_MAX_DEPTH; ++l)
            stats[p * (HH_MAX_DEPTH + 1) + l] =
                l < (int)r->stats[p].size() ? r->stats[p][(size_t)l] : hh_level_stats{};
    if (nc > cells_cap) throw Error{HH_ECAPACITY, "the cell buffer holds " + std::to_string(cells_cap) +
                                                      " cells; the call found " + std::to_string(nc)};
    if (r->have_members && members && nm > members_cap)
        throw Error{HH_ECAPACITY, "the member buffer holds " + std::to_string(members_cap) +
                                      " ids; the call found " + std::to_string(nm)};
    hipStream_t st = ctx->stream;
    if (r->depth0) {
        // the root is the only level: one cell per pass, every point votes
        hh_cell h[2]{};
        int64_t c = 0;
        for (int p = 0; p < 2; ++p) {
            if (info.n_cells[p] == 0) continue;
            h[c].votes = (int32_t)info.n_points;
            h[c].pass = p;
            h[c].member_off = r->have_members ? c * info.n_points : -1;
            ++c;
        }
        if (nc > 0) check(hipMemcpyAsync(cells, h, (size_t)nc * sizeof(hh_cell), hipMemcpyHostToDevice, st), "cells");
        if (r->have_members && members)
            for (int64_t c = 0; c < nc; ++c)
                check(launch_iota(members + c * info.n_points, info.n_points, st), "member ids");
    } else if (nc > 0) {
        // cells after cells, voters dense: member_off counted from the image's first voter
        check(launch_rebase_cells(r->cells, nc, r->have_members ? r->mem_base : 0, reinterpret_cast<Cell*>(cells),
                                  st),
              "cells");
        if (r->have_members && members)
            check(launch_member_ids(r->cells, nc, nullptr, r->mem_base, r->members_base, r->entry_bytes, r->xy,
                                    info.n_points, members, st),
                  "member ids");
    }
    sync(ctx);
    return HH_OK;
}

// Cells of a result whose member_off index this result's members (made on
// request when its voters do not start the call's member buffer).
const Cell* engine_device_cells(hh_result* res)
{
    if (res->depth0 || res->mem_base == 0 || !res->have_members || res->n_cells_total == 0) return res->cells;
    if (!res->dev_cells) {
        hh_ctx* ctx = res->ctx;
        check(hipSetDevice(ctx->device), "hipSetDevice");
        DevBuf d(&ctx->pool, sizeof(Cell) * (size_t)res->n_cells_total);
        check(launch_rebase_cells(res->cells, res->n_cells_total, res->mem_base, d.as<Cell>(), ctx->stream),
              "rebase cells");
        sync(ctx);
        res->dev_cells = std::move(d);
    }
    return res->dev_cells.as<Cell>();
}

hh_status engine_device_ids(hh_result* res)
{
    if (res->dev_ids || !res->have_members) return HH_OK;
    hh_ctx* ctx = res->ctx;
    check(hipSetDevice(ctx->device), "hipSetDevice");
    const int64_t slots = std::max<int64_t>(res->info.member_slots, 1);
    res->dev_ids = DevBuf(&ctx->pool, (size_t)slots * 4);
    if (res->depth0) {
        check(launch_iota(res->dev_ids.as<int32_t>(), res->info.member_slots, ctx->stream), "iota");
    } else if (res->entry_bytes == 4) {   // packed points: ids through a table of ranks per pixel
        DevBuf table(&ctx->pool, (size_t)res->info.width * (size_t)res->info.height * 4);
        if (!table) throw Error{HH_ENOMEM, "pixel rank table"};
        check(launch_ids_by_pixel(res->xy, res->info.n_points, res->info.width, res->info.height,
                                  table.as<int32_t>(), static_cast<const uint32_t*>(res->members),
                                  res->info.member_slots, res->dev_ids.as<int32_t>(), ctx->stream),
              "member ids");
        sync(ctx);   // the table returns to the pool when this scope ends
    } else {
        check(launch_member_ids(res->cells, res->n_cells_total, nullptr, res->mem_base, res->members_base,
                                res->entry_bytes, res->xy, res->info.n_points, res->dev_ids.as<int32_t>(),
                                ctx->stream),
              "member ids");
    }
    sync(ctx);
    return HH_OK;
}

// Host copy of the cells, member_off rewritten to the compact host layout
// (cells after cells, in (pass, key) order).
hh_status engine_host_cells(hh_result* res)
{
    if (res->host_cells_ready) return HH_OK;
    hh_ctx* ctx = res->ctx;
    check(hipSetDevice(ctx->device), "hipSetDevice");
    const int64_t n = res->n_cells_total;
    res->host_cells.resize((size_t)n);
    if (n > 0)
        check(hipMemcpyAsync(res->host_cells.data(), res->cells, (size_t)n * sizeof(hh_cell), hipMemcpyDeviceToHost,
                             ctx->stream),
              "copy cells");
    sync(ctx);
    int64_t total = 0;
    for (int64_t c = 0; c < n; ++c) {
        hh_cell& h = res->host_cells[(size_t)c];
        h.member_off = res->have_members ? total : -1;
        total += h.votes;
    }
    res->host_member_total = total;
    res->host_cells_ready = true;
    return HH_OK;
}

// Host copy of the voters' point ids in the compact host layout.
hh_status engine_host_members(hh_result* res)
{
    if (res->host_members_ready) return HH_OK;
    engine_host_cells(res);
    hh_ctx* ctx = res->ctx;
    hipStream_t st = ctx->stream;
    const int64_t n = res->n_cells_total, total = res->host_member_total;
    if (res->have_members && n > 0) {
        res->host_members.resize((size_t)total);
        if (res->depth0) {   // every point votes for the root: ids 0 .. E-1 per cell
            for (int64_t c = 0; c < n; ++c) {
                const hh_cell& h = res->host_cells[(size_t)c];
                for (int32_t k = 0; k < h.votes; ++k) res->host_members[(size_t)(h.member_off + k)] = k;
            }
        } else {
            std::vector<int64_t> off((size_t)n);
            for (int64_t c = 0; c < n; ++c) off[(size_t)c] = res->host_cells[(size_t)c].member_off;
            DevBuf d_off(&ctx->pool, (size_t)n * 8);
            DevBuf d_dst(&ctx->pool, (size_t)std::max<int64_t>(total, 1) * 4);
            check(hipMemcpyAsync(d_off.get(), off.data(), (size_t)n * 8, hipMemcpyHostToDevice, st), "copy offsets");
            check(launch_member_ids(res->cells, n, d_off.as<int64_t>(), 0, res->members_base, res->entry_bytes,
                                    res->xy, res->info.n_points, d_dst.as<int32_t>(), st),
                  "member ids");
            check(hipMemcpyAsync(res->host_members.data(), d_dst.get(), (size_t)total * 4, hipMemcpyDeviceToHost, st),
                  "copy members");
            sync(ctx);
        }
    }
    res->host_members_ready = true;
    return HH_OK;
}

// solution() with removal (Sec. 3): one walk per tree of every result, in
// one launch per bitmap kind.  A result's pass p owns keep flags for its
// cells and plotted flags for its n_points ids.  The voter ids, rebased cells
// and pixel rank table the walk reads live only for the call, in one buffer
// each; the flags of all results share one buffer, held by every result.
hh_status engine_solution(hh_ctx* ctx, hh_result* const* res, int32_t n, double* kernel_ms)
{
    if (kernel_ms) *kernel_ms = 0.0;
    check(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = ctx->stream;
    std::vector<hh_result*> todo;
    for (int32_t k = 0; k < n; ++k) {
        hh_result* r = res[k];
        if (!r) throw Error{HH_EINVAL, "null result"};
        if (r->ctx != ctx) throw Error{HH_EINTERNAL, "result of another context"};
        if (!r->have_members) throw Error{HH_EINVAL, "membership was not kept"};
        if (r->sol_ready || std::find(todo.begin(), todo.end(), r) != todo.end()) continue;
        todo.push_back(r);
    }
    if (todo.empty()) return HH_OK;
    // sizes: ids (4-aligned per result, for 16-byte loads), rebased cells, table, flags
    const size_t nr = todo.size();
    std::vector<int64_t> ids_off(nr), cells_off(nr, -1), flags_off(nr);
    int64_t n_ids = 0, n_cells = 0, max_pix = 1, flag_bytes = 0;
    for (size_t k = 0; k < nr; ++k) {
        hh_result* r = todo[k];
        ids_off[k] = n_ids;
        n_ids += (std::max<int64_t>(r->info.member_slots, 1) + 3) & ~(int64_t)3;
        if (!r->depth0 && r->mem_base != 0 && r->n_cells_total > 0) {
            cells_off[k] = n_cells;
            n_cells += r->n_cells_total;
        }
        if (!r->depth0 && r->entry_bytes == 4)
            max_pix = std::max<int64_t>(max_pix, (int64_t)r->info.width * r->info.height);
        // flags: keep per cell, plotted per point and pass, then 4 counts
        flags_off[k] = flag_bytes;
        int64_t before = 0;
        for (int q = 0; q < r->n_trees; ++q) {
            const int32_t p = r->tree_pass[q];
            r->sol_keep_off[p] = before;
            before += r->info.n_cells[p];
        }
        int64_t bytes = align256(std::max<int64_t>(before, 1));
        for (int q = 0; q < r->n_trees; ++q) {
            r->sol_plot_off[r->tree_pass[q]] = bytes;
            bytes += align256(std::max<int64_t>(r->info.n_points, 1));
        }
        r->sol_counts_off = bytes;
        flag_bytes += bytes + 256;
    }
    DevBuf ids(&ctx->pool, (size_t)n_ids * 4);
    DevBuf cells(&ctx->pool, (size_t)std::max<int64_t>(n_cells, 1) * sizeof(Cell));
    DevBuf table(&ctx->pool, (size_t)max_pix * 4);
    auto flags = std::make_shared<DevBuf>(&ctx->pool, (size_t)flag_bytes);
    if (!ids || !cells || !table || !*flags) throw Error{HH_ENOMEM, "solution buffers"};
    std::vector<SolTree> lds, dev;
    int64_t max_lds_points = 0;
    for (size_t k = 0; k < nr; ++k) {
        hh_result* r = todo[k];
        const int64_t E = r->info.n_points, slots = r->info.member_slots;
        int32_t* dst = ids.as<int32_t>() + ids_off[k];
        if (r->depth0) {
            check(launch_iota(dst, slots, st), "iota");
        } else if (r->entry_bytes == 4) {   // packed points: ids through the table of ranks per pixel
            check(launch_ids_by_pixel(r->xy, E, r->info.width, r->info.height, table.as<int32_t>(),
                                      static_cast<const uint32_t*>(r->members), slots, dst, st),
                  "member ids");
        } else {
            check(launch_member_ids(r->cells, r->n_cells_total, nullptr, r->mem_base, r->members_base,
                                    r->entry_bytes, r->xy, E, dst, st),
                  "member ids");
        }
        const Cell* rc = r->cells;   // member_off counted from the result's first voter
        if (cells_off[k] >= 0) {
            Cell* d = cells.as<Cell>() + cells_off[k];
            check(launch_rebase_cells(r->cells, r->n_cells_total, r->mem_base, d, st), "rebase cells");
            rc = d;
        }
        r->sol_store = flags;
        r->sol = flags->as<uint8_t>() + flags_off[k];
        uint8_t* base = const_cast<uint8_t*>(r->sol);
        int64_t cbefore = 0;
        for (int q = 0; q < r->n_trees; ++q) {
            const int32_t p = r->tree_pass[q];
            SolTree t{};
            t.cells = rc ? rc + cbefore : nullptr;
            t.ids = dst;
            t.n_cells = r->info.n_cells[p];
            t.n_points = E;
            t.n_slots = slots;
            t.keep = base + r->sol_keep_off[p];
            t.plotted = base + r->sol_plot_off[p];
            t.counts = reinterpret_cast<int64_t*>(base + r->sol_counts_off) + 2 * p;
            t.threshold = r->info.threshold;
            cbefore += t.n_cells;
            if (t.n_cells > 0 && !t.cells) throw Error{HH_EINTERNAL, "solution inputs missing"};
            if (E <= solution_lds_points()) {
                max_lds_points = std::max(max_lds_points, E);
                lds.push_back(t);
            } else {
                dev.push_back(t);
            }
        }
    }
    // Segments: consecutive cells of about kSolSegSlots voter entries, at most
    // kSolMaxSegs per tree, and only as many as it takes
    // for two segments per compute unit over all trees (a batch of many
    // trees walks each in one segment, in one round); LDS trees first.
    // Bitmaps per segment: in, out (and a work bitmap for device-bitmap
    // trees); per tree: all.
    constexpr int64_t kSolSegSlots = 1 << 16;
    std::vector<SolTree> all(lds);
    all.insert(all.end(), dev.begin(), dev.end());
    const int32_t n_trees = (int32_t)all.size(), n_lds_trees = (int32_t)lds.size();
    const int64_t seg_cap = std::max<int64_t>(1, 2 * (int64_t)ctx->cu_count / std::max<int32_t>(n_trees, 1));
    std::vector<SolSeg> segs;
    std::vector<int64_t> seg_words;   // bitmap word offsets of each segment: in, out, work
    int64_t words_total = 0, max_words = 1, max_segs = 1;
    int32_t n_lds = 0;
    std::vector<int64_t> all_off((size_t)n_trees);
    for (int32_t k = 0; k < n_trees; ++k) {
        SolTree& t = all[(size_t)k];
        const int64_t words = ((t.n_points + 31) >> 5 | 1) + 63 & ~(int64_t)63;
        max_words = std::max(max_words, (t.n_points + 31) >> 5);
        all_off[(size_t)k] = words_total;
        words_total += words;
        const int64_t K = t.n_cells == 0 ? 0
                          : std::min({(int64_t)kSolMaxSegs, seg_cap, t.n_cells,
                                      std::max<int64_t>(1, (t.n_slots + kSolSegSlots - 1) / kSolSegSlots)});
        max_segs = std::max(max_segs, K);
        t.seg0 = (int32_t)segs.size();
        t.n_segs = (int32_t)K;
        for (int64_t q = 0; q < K; ++q) {
            SolSeg g{};
            g.tree = k;
            g.c0 = t.n_cells * q / K;   // by cell count here; by voter entries on the device
            g.c1 = t.n_cells * (q + 1) / K;
            segs.push_back(g);
            seg_words.push_back(words_total);
            words_total += (k < n_lds_trees ? 2 : 3) * words;
        }
        if (k < n_lds_trees) n_lds = (int32_t)segs.size();
    }
    const int32_t n_segs = (int32_t)segs.size(), n_dev = n_segs - n_lds;
    DevBuf bitmaps(&ctx->pool, (size_t)std::max<int64_t>(words_total, 1) * 4);
    if (!bitmaps) throw Error{HH_ENOMEM, "solution bitmaps"};
    check(hipMemsetAsync(bitmaps.get(), 0, (size_t)std::max<int64_t>(words_total, 1) * 4, st), "clear bitmaps");
    uint32_t* const bw = bitmaps.as<uint32_t>();
    for (int32_t k = 0; k < n_trees; ++k) all[(size_t)k].all = bw + all_off[(size_t)k];
    for (int32_t q = 0; q < n_segs; ++q) {
        SolSeg& g = segs[(size_t)q];
        const SolTree& t = all[(size_t)g.tree];
        const int64_t words = ((t.n_points + 31) >> 5 | 1) + 63 & ~(int64_t)63;
        g.in = bw + seg_words[(size_t)q];
        g.out = g.in + words;
        g.work = q >= n_lds ? g.out + words : nullptr;
        g.counts = nullptr;   // set below, in the table buffer
    }
    const size_t trees_bytes = (size_t)align256((int64_t)(std::max<int32_t>(n_trees, 1) * sizeof(SolTree)));
    const size_t segs_bytes = (size_t)align256((int64_t)(std::max<int32_t>(n_segs, 1) * sizeof(SolSeg)));
    const size_t cnt_bytes = (size_t)align256((int64_t)std::max<int32_t>(n_segs, 1) * 16);
    const size_t list_bytes = (size_t)align256((int64_t)std::max<int32_t>(n_segs, 1) * 4);
    const size_t tree_int_bytes = (size_t)align256((int64_t)std::max<int32_t>(n_trees, 1) * 4);
    const size_t flag_seg_bytes = (size_t)align256((int64_t)std::max<int32_t>(n_segs, 1));
    DevBuf d(&ctx->pool, trees_bytes + segs_bytes + cnt_bytes + 4 * list_bytes + tree_int_bytes + flag_seg_bytes + 256);
    if (!d) throw Error{HH_ENOMEM, "solution table"};
    char* dp = d.as<char>();
    SolTree* const d_trees = reinterpret_cast<SolTree*>(dp);
    dp += trees_bytes;
    SolSeg* const d_segs = reinterpret_cast<SolSeg*>(dp);
    dp += segs_bytes;
    int64_t* const d_cnt = reinterpret_cast<int64_t*>(dp);
    dp += cnt_bytes;
    int32_t* lists[4];   // two rounds' lists: LDS, device, LDS, device
    for (auto& l : lists) {
        l = reinterpret_cast<int32_t*>(dp);
        dp += list_bytes;
    }
    int32_t* const d_first = reinterpret_cast<int32_t*>(dp);
    dp += tree_int_bytes;
    uint8_t* const d_changed = reinterpret_cast<uint8_t*>(dp);
    dp += flag_seg_bytes;
    uint32_t* const d_err = reinterpret_cast<uint32_t*>(dp);   // error, then the list sizes of both rounds
    int32_t* const d_nlist = reinterpret_cast<int32_t*>(dp + 16);
    for (int32_t q = 0; q < n_segs; ++q) segs[(size_t)q].counts = d_cnt + 2 * q;
    // the first round walks every segment
    std::vector<int32_t> first_list((size_t)std::max<int32_t>(n_segs, 1));
    for (int32_t q = 0; q < n_segs; ++q) first_list[(size_t)q] = q;
    const std::vector<int32_t> no_walk((size_t)std::max<int32_t>(n_trees, 1), INT32_MAX);
    const int32_t first_n[4] = {n_lds, n_dev, 0, 0};
    if (n_trees > 0) {
        check(hipMemcpyAsync(d_trees, all.data(), (size_t)n_trees * sizeof(SolTree), hipMemcpyHostToDevice, st),
              "copy trees");
        check(hipMemcpyAsync(d_first, no_walk.data(), (size_t)n_trees * 4, hipMemcpyHostToDevice, st), "copy marks");
    }
    if (n_segs > 0) {
        check(hipMemcpyAsync(d_segs, segs.data(), (size_t)n_segs * sizeof(SolSeg), hipMemcpyHostToDevice, st),
              "copy segments");
        check(launch_solution_cut(d_trees, d_segs, n_segs, st), "segment bounds");
        if (n_lds > 0)
            check(hipMemcpyAsync(lists[0], first_list.data(), (size_t)n_lds * 4, hipMemcpyHostToDevice, st),
                  "copy list");
        if (n_dev > 0)
            check(hipMemcpyAsync(lists[1], first_list.data() + n_lds, (size_t)n_dev * 4, hipMemcpyHostToDevice, st),
                  "copy list");
        check(hipMemsetAsync(d_changed, 0, (size_t)n_segs, st), "clear marks");
    }
    check(hipMemsetAsync(d_err, 0, 16, st), "clear error");
    check(hipMemcpyAsync(d_nlist, first_n, sizeof(first_n), hipMemcpyHostToDevice, st), "copy list sizes");
    hipEvent_t ev[2];
    check(hipEventCreate(&ev[0]), "event");
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        throw Error{HH_EDEVICE, "event"};
    }
    struct Events {
        hipEvent_t* e;
        ~Events()
        {
            (void)hipEventDestroy(e[0]);
            (void)hipEventDestroy(e[1]);
        }
    } guard{ev};
    // Rounds until no segment's input changes (at most one per segment, plus
    // one), queued 2, 4, 8, 8, ... at a time between checks on the host; a
    // round with empty lists costs only its launches.
    SolRound rd{};
    rd.trees = d_trees;
    rd.segs = d_segs;
    rd.n_trees = n_trees;
    rd.n_segs = n_segs;
    rd.n_lds = n_lds;
    rd.grid = 2 * ctx->cu_count;
    rd.max_lds_points = max_lds_points;
    rd.max_words = max_words;
    rd.first_walked = d_first;
    rd.changed = d_changed;
    rd.error = d_err;
    check(hipEventRecord(ev[0], st), "event");
    int rounds = 0, parity = 0;
    for (int batch = 2;; batch = std::min(batch * 2, 8)) {
        for (int b = 0; b < batch; ++b) {
            rd.list_lds = lists[2 * parity];
            rd.list_dev = lists[2 * parity + 1];
            rd.n_list = d_nlist + 2 * parity;
            rd.next_lds = lists[2 * (1 - parity)];
            rd.next_dev = lists[2 * (1 - parity) + 1];
            rd.n_next = d_nlist + 2 * (1 - parity);
            check(launch_solution_round(rd, st), "solution round");
            parity = 1 - parity;
            ++rounds;
        }
        uint32_t h[4] = {0, 0, 0, 0};   // error, pad, list sizes of the next round
        check(hipMemcpyAsync(h, d_err, 4, hipMemcpyDeviceToHost, st), "copy error");
        check(hipMemcpyAsync(h + 2, d_nlist + 2 * parity, 8, hipMemcpyDeviceToHost, st), "copy list sizes");
        sync(ctx);
        if (h[0]) throw Error{HH_EINTERNAL, "solution: malformed cells or member ids"};
        if (h[2] == 0 && h[3] == 0) break;
        if (rounds > max_segs + 16) throw Error{HH_EINTERNAL, "solution: the segment rounds did not settle"};
    }
    check(launch_solution_finish(d_trees, n_trees, d_segs, st), "solution finish");
    check(hipEventRecord(ev[1], st), "event");
    // the counts of every result come back in one copy each
    std::vector<int64_t> counts(4 * nr, 0);
    sync(ctx);
    float ms = 0.f;
    check(hipEventElapsedTime(&ms, ev[0], ev[1]), "event time");
    if (kernel_ms) *kernel_ms = ms;
    for (size_t k = 0; k < nr; ++k) {
        hh_result* r = todo[k];
        check(hipMemcpyAsync(&counts[4 * k], r->sol + r->sol_counts_off, 32, hipMemcpyDeviceToHost, st),
              "copy counts");
    }
    sync(ctx);
    for (size_t k = 0; k < nr; ++k) {
        hh_result* r = todo[k];
        for (int p = 0; p < 2; ++p) {
            r->sol_kept[p] = counts[4 * k + 2 * p];
            r->sol_plotted[p] = counts[4 * k + 2 * p + 1];
        }
        r->sol_rounds = rounds;
        r->sol_ready = true;
    }
    return HH_OK;
}

hh_status engine_host_solution(hh_result* res, int32_t pass)
{
    if (res->host_sol_ready[pass]) return HH_OK;
    hh_ctx* ctx = res->ctx;
    check(hipSetDevice(ctx->device), "hipSetDevice");
    const int64_t nc = res->info.n_cells[pass], E = res->info.n_points;
    res->host_keep[pass].assign((size_t)nc, 0);
    res->host_plotted[pass].assign((size_t)E, 0);
    if (nc > 0)
        check(hipMemcpyAsync(res->host_keep[pass].data(), res->sol + res->sol_keep_off[pass], (size_t)nc,
                             hipMemcpyDeviceToHost, ctx->stream),
              "copy keep");
    if (E > 0)
        check(hipMemcpyAsync(res->host_plotted[pass].data(), res->sol + res->sol_plot_off[pass], (size_t)E,
                             hipMemcpyDeviceToHost, ctx->stream),
              "copy plotted");
    sync(ctx);
    res->host_sol_ready[pass] = true;
    return HH_OK;
}

hh_status engine_solution_image(hh_result* res, uint8_t* image, int64_t row_stride, int32_t on_device)
{
    hh_ctx* ctx = res->ctx;
    check(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = ctx->stream;
    const int32_t W = res->info.width, H = res->info.height;
    DevBuf img(&ctx->pool, (size_t)W * (size_t)H);
    if (!img) throw Error{HH_ENOMEM, "output image"};
    check(hipMemsetAsync(img.get(), 0, (size_t)W * (size_t)H, st), "clear image");
    const Cell* cells = engine_device_cells(res);   // member_off counted from res->members
    int64_t before = 0;
    for (int q = 0; q < res->n_trees; ++q) {
        const int32_t p = res->tree_pass[q];
        const int64_t nc = res->info.n_cells[p];
        check(launch_paint(cells + before, nc, res->sol + res->sol_keep_off[p], res->members, res->entry_bytes, W, H,
                           img.as<uint8_t>(), st),
              "paint");
        before += nc;
    }
    check(hipMemcpy2DAsync(image, (size_t)row_stride, img.get(), (size_t)W, (size_t)W, (size_t)H,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st),
          "copy image");
    sync(ctx);
    return HH_OK;
}

}  // namespace hh
