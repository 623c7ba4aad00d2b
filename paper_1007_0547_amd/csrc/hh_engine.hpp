// Host engine of the hierarchical Hough vote: device memory pool, context,
// and the level-synchronous driver behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <condition_variable>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/hough_hier.h"
#include "hh_types.hpp"

namespace hh {

// Intervals of one device slab shared by several pools, handed out first
// fit (256-byte aligned), with a lock of its own.  `freed` (if set) is
// notified whenever an interval comes back.
class SlabSpace {
public:
    void init(char* base, int64_t bytes, std::condition_variable* freed);
    int64_t take(int64_t bytes);    // offset of a free interval of `bytes`, or -1
    void give(int64_t off);         // return the interval at off
    int64_t largest();              // the largest free interval
    int64_t total() const { return total_; }
    int64_t used();
    char* base() const { return base_; }
    bool holds(const void* p) const
    {
        return p >= base_ && static_cast<const char*>(p) < base_ + total_;
    }

private:
    std::mutex mu_;
    std::map<int64_t, int64_t> free_;   // offset -> bytes
    std::map<int64_t, int64_t> live_;   // offset -> bytes
    char* base_ = nullptr;
    int64_t total_ = 0, used_ = 0;
    std::condition_variable* freed_ = nullptr;
};

// Caching allocator over hipMalloc.  Sizes are rounded up to one of eight
// steps per power of two; freed blocks wait in per-size free lists and are
// handed out again without a hipMalloc.  All device work that uses a pool's
// blocks runs on its context's stream, so reuse is ordered by the stream.
// The pool is locked on its own, so that releasing a result's blocks never
// waits for a call running on the context.
//
// A pool may instead draw its blocks from a slab that other pools (on other
// streams) share: no caching, and a block released while a call runs goes
// back to the slab only when the call has ended (its stream synchronized),
// so no other stream can reuse it while this one's work may still touch it.
// With the slab full, an allocation inside a call fails; one between calls
// (made on request for a result) falls back to hipMalloc.
class DevicePool {
public:
    ~DevicePool();
    void* alloc(size_t bytes);
    void release(void* p);
    void discard(void* p);   // hipFree a live block instead of caching it
    void trim();
    void set_caching(bool on) { caching_ = on; }   // off: a released block is freed at once
    void back_with(SlabSpace* slab) { slab_ = slab; }
    void draw_outside(bool on) { outside_ = on; }   // new blocks from hipMalloc even when backed
    void begin_call();
    void end_call();         // after the call's stream is synchronized
    size_t live_bytes() const { return live_; }
    size_t cached_bytes() const { return cached_; }

private:
    static size_t round_size(size_t bytes);
    void trim_locked();
    void free_locked(void* p, size_t sz);
    std::mutex mu_;
    std::unordered_map<size_t, std::vector<void*>> free_;
    std::unordered_map<void*, size_t> size_of_;
    size_t live_ = 0, cached_ = 0;
    bool caching_ = true;
    SlabSpace* slab_ = nullptr;
    bool outside_ = false;
    bool in_call_ = false;
    std::vector<void*> deferred_;   // slab blocks released during a call
};

// A pool block that returns to its pool on destruction.
class DevBuf {
public:
    DevBuf() = default;
    DevBuf(DevicePool* pool, size_t bytes);
    // a view of memory the DevBuf does not own (nothing is released)
    static DevBuf view(void* p, size_t bytes)
    {
        DevBuf b;
        b.ptr_ = p;
        b.bytes_ = bytes;
        return b;
    }
    ~DevBuf() { reset(); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
    DevBuf& operator=(DevBuf&& o) noexcept;
    void reset();
    void discard();   // free the block outright (it is not cached for reuse)
    template <typename T> T* as() const { return static_cast<T*>(ptr_); }
    void* get() const { return ptr_; }
    size_t bytes() const { return bytes_; }
    explicit operator bool() const { return ptr_ != nullptr; }

private:
    DevicePool* pool_ = nullptr;
    void* ptr_ = nullptr;
    size_t bytes_ = 0;
};

struct Error {
    hh_status status;
    std::string what;
};

// Device memory of one call: blocks of the context's pool, or views carved
// front to back (256-byte aligned) from a caller's arena.
struct CallMem {
    DevicePool* pool = nullptr;
    char* base = nullptr;   // the caller's arena, or nullptr
    int64_t cap = 0, used = 0;
    bool graph_ok = false;  // every input is device resident (HH_FLAG_GRAPH may capture)
    int64_t taken = 0;      // bytes handed out (both kinds), for the footprint of the call
    int64_t arena_peak = 0; // largest level arena the call held
    int64_t arena_need = 0; // largest level arena the call's groups needed (measured)
    DevBuf get(size_t bytes, const char* what);
    int64_t left() const { return cap - used; }
};

}  // namespace hh

namespace hh {

// Device memory of one call, shared by the results of its images and
// released with the last of them: the packed edge points, image after image.
struct CallStore {
    DevBuf points;
};

// Device memory of one group of a call's images (the images whose levels
// ran in one arena).  A group keeps its arena's front part (level records,
// cells and voters; the level halves and scratch of the back part go back to
// the pool when the group ends), except in several groups of a call in the
// caller's arena, which reuse that arena: there each group keeps exact
// copies of its cells and voters.
struct GroupStore {
    std::shared_ptr<CallStore> call;
    DevBuf arena;
    DevBuf cells;
    DevBuf members;
    std::function<void()> on_release;   // run when the last result of the group goes (serving slab space)
    ~GroupStore()
    {
        if (on_release) on_release();
    }
};

}  // namespace hh

// The result of one image of a call.
struct hh_result {
    hh_ctx* ctx = nullptr;
    std::shared_ptr<hh::GroupStore> store;
    hh_result_info info{};
    int32_t n_trees = 0;
    int32_t tree_pass[2] = {-1, -1};
    std::vector<hh_level_stats> stats[2];
    const hh::Cell* cells = nullptr;     // this image's cells, (pass, key) order, member_off into the call's buffer
    int64_t n_cells_total = 0;
    const void* members = nullptr;       // this image's voter entries, cell after cell
    const void* members_base = nullptr;  // the call's member buffer
    int64_t mem_base = 0;                // member_off of this image's first voter
    const uint32_t* xy = nullptr;        // this image's packed edge points
    int32_t entry_bytes = 4;             // 4: packed point; 8: id << 32 | packed point
    bool have_members = false;
    bool in_arena = false;               // made in the caller's arena (counted in ctx->arena_results)
    bool depth0 = false;                 // the root is the only level: every point votes
    hh::DevBuf depth0_cells;             // depth 0: the cells, made on the host
    hh::DevBuf dev_cells;                // cells with member_off relative to this image (made on request)
    hh::DevBuf dev_ids;                  // point ids in the layout of member_off (made on request)
    // solution() with removal (hough_hier_solution): per pass, keep flags of
    // its cells and plotted flags of the point ids, then the counts
    bool sol_ready = false;
    std::shared_ptr<hh::DevBuf> sol_store;   // the flags of every result of one hough_hier_solution call
    const uint8_t* sol = nullptr;            // this result's part
    int64_t sol_keep_off[2] = {0, 0};
    int64_t sol_plot_off[2] = {0, 0};
    int64_t sol_counts_off = 0;
    int64_t sol_kept[2] = {0, 0};
    int64_t sol_plotted[2] = {0, 0};
    int64_t sol_rounds = 0;
    bool host_sol_ready[2] = {false, false};
    std::vector<uint8_t> host_keep[2];
    std::vector<uint8_t> host_plotted[2];
    hh_timing timing{};
    // lazily filled host copies
    bool host_cells_ready = false;
    bool host_members_ready = false;
    int64_t host_member_total = 0;
    std::vector<hh_cell> host_cells;
    std::vector<int32_t> host_members;
};

namespace hh {
struct Server;
}

struct hh_ctx {
    hh_config cfg{};
    // serialises the calls that use this context's stream, pool and results
    std::mutex mu;
    std::mutex err_mu;       // last_error
    std::mutex results_mu;   // live_results
    // serving lanes (hough_hier_serve_start); stopped before the context goes
    std::unique_ptr<hh::Server> server;
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    hh::DevicePool pool;
    int cu_count = 0;
    // pinned host copies: an arena's fixed part (level records, tree records,
    // error), the trees of a call, the descriptors of its inputs
    char* h_fixed = nullptr;
    // a call's descriptors in one block, uploaded with one copy: the trees,
    // the staging error word, then the input table (see call_layout)
    char* h_call = nullptr;
    hh::TreeDesc* h_trees = nullptr;    // = h_call
    // arena sizes that worked before (grown when a call overflows)
    int64_t half_cap = 64ll << 20;      // bytes per level half
    int64_t work_cap = 16ll << 20;      // bytes of per-level scratch
    int64_t mem_cap = 16ll << 20;       // member entries
    int64_t cells_cap = 1ll << 20;
    // most edge points one group of a batch may hold (0: no limit), learnt
    // when a group's level lists exceeded the memory budget
    int64_t group_points = 0;
    int32_t grid = 0;          // workgroups of the root-list kernel
    // launch shape of the list kernels: steps (512 entries) per task, tasks a
    // wavefront takes from the level's queue at once (0: a fixed share), and
    // resident workgroups per compute unit (0: as many as fit)
    int32_t task_steps = 8;
    int32_t queue_batch = 0;
    int32_t wg_per_cu = 0;
    int64_t arena_hint_bytes = 0;   // > 0: size of a call's first level arena (serving lanes set it per batch)
    // HIP events for HH_FLAG_TIMING: [0] call start, [1] staging end, [2] call end,
    // then four per level: before count, after count, after emit, after the compaction
    std::vector<hipEvent_t> events;
    // results not yet freed; destroyed with the context
    std::unordered_set<hh_result*> live_results;
    // results made in the caller's arena (hh_config.arena) and not yet freed
    int64_t arena_results = 0;
    // device bytes the last detection call held at most (inputs, staging,
    // level arena), for serving admission
    int64_t last_call_bytes = 0;
    int64_t last_call_need = 0;   // device bytes the last call needed at least (inputs and level arena)
    // HH_FLAG_GRAPH: the captured level launches of the last call and what
    // they were captured for (sizes, parameters, addresses)
    hipGraphExec_t graph_exec = nullptr;
    std::string graph_key;
    int64_t graph_replays = 0;
};

namespace hh {

hh_status engine_create(const hh_config* cfg, hh_ctx** out);
void engine_destroy(hh_ctx* ctx);
hh_status engine_detect(hh_ctx* ctx, const hh_input* in, hh_result** out);
// n inputs in one call; out[k] is the result of in[k] (all or none are made).
// With ext, the call's device memory is carved from ext's region (no
// allocation) and its results are not counted as the caller arena's.
hh_status engine_detect_batch(hh_ctx* ctx, const hh_input* in, int32_t n, hh_result** out,
                              CallMem* ext = nullptr);
// One detection whose device memory is the library's fixed scratch array of
// this device (hough_hier_detect_noalloc): outputs go to the caller's
// buffers; nothing is allocated on the device.
hh_status engine_detect_noalloc(hh_ctx* ctx, const hh_input* in, hh_cell* cells, int64_t cells_cap,
                                int32_t* members, int64_t members_cap, hh_level_stats* stats, int64_t* n_cells,
                                int64_t* n_members);
// Autotuner (hh_tune.cpp): the launch shape for calls like in[0 .. n), from
// the cache or by timing candidates on this call; set on ctx and returned.
hh_status engine_autotune(hh_ctx* ctx, const hh_input* in, int32_t n, hh_launch* chosen, int32_t* from_cache);
// The fixed scratch array of the current device (its device address, taken
// once per device with hipGetSymbolAddress) and its size.
void* noalloc_scratch(int device);
extern const int64_t kNoAllocScratchBytes;
hh_status engine_host_cells(hh_result* res);
hh_status engine_host_members(hh_result* res);
hh_status engine_device_ids(hh_result* res);
// The result's device cells with member_off counted from its own first voter.
const Cell* engine_device_cells(hh_result* res);
// solution() with removal over the detected cells of results of this context
// (one launch for all their trees); *kernel_ms gets the walk's duration.
hh_status engine_solution(hh_ctx* ctx, hh_result* const* res, int32_t n, double* kernel_ms);
// Host copies of one pass's keep and plotted flags.
hh_status engine_host_solution(hh_result* res, int32_t pass);
// The output image of solution() (plotted points of every pass = 255, else 0)
// into image (host or device memory, rows of row_stride bytes).
hh_status engine_solution_image(hh_result* res, uint8_t* image, int64_t row_stride, int32_t on_device);

// Serving (hh_serve.cpp).
hh_status serve_start(hh_ctx* ctx, const hh_serve_config* cfg);
hh_status serve_submit(hh_ctx* ctx, const hh_input* in, uint64_t* ticket);
hh_status serve_poll(hh_ctx* ctx, uint64_t ticket, int32_t wait_us, hh_result** out);
void serve_stop(hh_ctx* ctx);
hh_status serve_stats(hh_ctx* ctx, hh_serve_stats* out);

}  // namespace hh
