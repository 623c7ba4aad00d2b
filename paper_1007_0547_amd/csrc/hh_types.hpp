// Types and memory layout shared by the device kernels and the host engine
// of the hierarchical Hough vote library.  Nothing here is part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hh {

constexpr int kWave = 64;                   // CDNA wavefront width
constexpr int kBlock = 256;                 // threads per workgroup (4 wavefronts)
constexpr int kWaves = kBlock / kWave;
constexpr int kStep = 8 * kWave;            // 512 list entries: the unit a task's length is counted in
constexpr int kMaxTaskSteps = 64;           // a task covers 1 .. 64 steps of one region's list
constexpr int kPixPerThread = 16;           // image bytes per lane in edge staging
constexpr int kPixTile = kBlock * kPixPerThread;
constexpr int kMaxLevels = 16;              // depth <= 15
constexpr int kNumStats = 6;                // evaluated, votes, split, detected, code_tests, entries
constexpr int kAggCh = 6;                   // decision sums: next regions, next entries, cells, member entries, votes, next tasks
constexpr int kRecCh = 7;                   // tree record: p, start, then the decision prefixes
constexpr int kRangeGrid = 512;             // region ranges of the split-decision launches
constexpr int kMaxTrees = 2048;             // trees (image passes) in one call

// Error bits set by kernels (the host reports them after the call).
constexpr uint32_t kErrPointRange = 2u;     // an input point lies outside [0,W)x[0,H)
constexpr uint32_t kErrInternal = 4u;       // an index failed a range check
constexpr uint32_t kErrArena = 8u;          // a level did not fit its arena; rerun larger
constexpr uint32_t kErrStop = kErrArena | kErrInternal;   // later kernels do nothing
// With kErrInternal, the check that failed (bits 8..11) and the level it
// failed at (bit 16 + level), so that the error message names them.
constexpr uint32_t kErrAtCountTask = 1u << 8;    // k_count: a task's region or range out of bounds
constexpr uint32_t kErrAtWriteTask = 1u << 9;    // k_write: a task's region or range out of bounds
constexpr uint32_t kErrAtWriteVotes = 1u << 10;  // k_write: a kept child's votes differ from its count
constexpr uint32_t kErrAtEmit = 1u << 11;        // emit: a region or task index past the level's totals
constexpr int kErrLevelShift = 16;

// Edge points are stored packed: x in bits 0..15, y in bits 16..31, so the
// packed value orders points row-major (y, then x).
__host__ __device__ inline uint32_t pack_xy(int32_t x, int32_t y) { return (uint32_t)x | ((uint32_t)y << 16); }

// One quadtree: one pass over one image's edge points.
struct TreeDesc {
    int64_t xy_base;    // first point of the image in the packed coordinate array
    int64_t n_points;
    int32_t s_log2;     // S = 2^s_log2
    int32_t dmax;       // finest level
    int32_t threshold;  // a region splits (or is detected) iff votes > threshold
    int32_t pass;       // 0: (u, v) = (x, y); 1: (u, v) = (y, x)
    int32_t image;      // index of the image in its batch
    int32_t image_points;   // edge points of the whole image (both sets of a gray image)
};

// One point list of a batch: n points (x[k], y[k]) in [0, W) x [0, H), packed
// to xy[base + k].
struct PointsDesc {
    const int32_t* x;
    const int32_t* y;
    int64_t n;
    int64_t base;
    int32_t width, height;
};

// One image of a batch for the edge staging: its pixel tiles are
// tile0 .. tile0 + ceil(n_pix / kPixTile) - 1 of the batch's tile range.
struct ImageDesc {
    const uint8_t* image;
    int64_t row_stride;
    int32_t width, height;
    int64_t tile0;
    int64_t n_pix;
    int32_t edge_threshold;   // gray images: Sobel magnitude threshold
    int32_t pad;
};

// Region.meta bits
constexpr uint32_t kMetaPass = 1u;               // pass 1: axes swapped
constexpr int kMetaSlogShift = 1;                // s_log2 in bits 1..4
constexpr uint32_t kMetaChildFinest = 1u << 5;   // the region's children are at the finest level

// A region that split at its level.  Its voters are entries
// [start, start + len) of the level's list.
struct Region {
    int64_t start;
    uint32_t ij;        // i | j << 16, indices at its level
    int32_t len;        // votes = list length
    int32_t tree;
    uint32_t meta;      // kMeta* bits
};

// Sizes of one level, filled in on the device as the levels run.
struct LevelInfo {
    int64_t P;          // regions that split at this level
    int64_t L;          // their total list length
    int64_t votes;      // summed votes of their children
    int64_t cells;      // cells detected at this level
    int64_t cells_base; // cells detected at shallower levels
    int64_t mem;        // voter entries of the cells detected at this level
    int64_t mem_base;   // voter entries of the cells detected at shallower levels
    int64_t NT;         // tasks over the level's list
    int64_t task_steps; // steps (kStep entries) per task of this level
    int64_t queue[2];   // work queue heads of the count and compaction launches
    int64_t pad;
};

// A task of a level: steps [c * task_steps, (c + 1) * task_steps) of region
// r's list (the last task of a region may be shorter).  The tasks of a
// region are consecutive, c = 0, 1, ..., so task t - c is its first.
struct Task {
    int32_t r;
    int32_t c;
};

// A detected cell; layout equal to the public hh_cell.
struct Cell {
    int32_t i, j;
    int32_t votes;
    int32_t pass;
    int64_t key;
    int64_t member_off;
};

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t align256(int64_t bytes) { return (bytes + 255) & ~(int64_t)255; }

// A level's data inside its arena half (l & 1): the region table, the task
// table and the child-vote totals (zeroed), written by the previous level's
// split decision (or the root setup), then the level's list, written by the
// previous level's compaction.  cv[r][q] collects the votes of child q of
// region r.
struct HalfLayout {
    Region* regions;
    Task* tasks;
    int32_t* cv;
    void* list;
    int64_t end;        // bytes used from the half's start
};

__host__ __device__ inline HalfLayout half_layout(char* half, int64_t P, int64_t L, int64_t NT, int entry_bytes)
{
    HalfLayout y;
    int64_t off = 0;
    y.regions = reinterpret_cast<Region*>(half + off);
    off += align256(P * (int64_t)sizeof(Region));
    y.tasks = reinterpret_cast<Task*>(half + off);
    off += align256(NT * (int64_t)sizeof(Task));
    y.cv = reinterpret_cast<int32_t*>(half + off);
    off += align256(P * 16);
    y.list = half + off;
    off += align256(L * entry_bytes);
    y.end = off;
    return y;
}

// Tasks of a region with n list entries.
__host__ __device__ inline int64_t region_tasks(int64_t n, int64_t task_steps)
{
    return n > 0 ? cdiv(n, task_steps * kStep) : 0;
}

// Per-level scratch, reused by every level.
//   dst  [P][4]  where the child's voters go (next list or member buffer), -1: dropped
//   tcnt [NT][4] child votes counted by each task
//   agg  [kRangeGrid][kAggCh] decision sums per range of regions
struct WorkLayout {
    int64_t* dst;
    int32_t* tcnt;
    int64_t* agg;
    int64_t end;
};

__host__ __device__ inline WorkLayout work_layout(char* work, int64_t P, int64_t NT)
{
    WorkLayout w;
    int64_t off = 0;
    w.dst = reinterpret_cast<int64_t*>(work + off);
    off += align256(P * 32);
    w.tcnt = reinterpret_cast<int32_t*>(work + off);
    off += align256(NT * 16);
    w.agg = reinterpret_cast<int64_t*>(work + off);
    off += align256((int64_t)kRangeGrid * kAggCh * 8);
    w.end = off;
    return w;
}

// All device memory of one call: a fixed part, the member buffer, two level
// halves used in turn and the per-level scratch.
struct Arena {
    LevelInfo* info;       // [kMaxLevels + 1]
    int64_t* rec;          // [n_trees][kMaxLevels][kRecCh] tree boundary records (-1: none)
    uint32_t* error;
    int64_t* scalar;       // [8] the first internal failure: claim, check and level, six values
    Cell* cells;
    int64_t cells_cap;
    void* members;         // voters of the detected cells, cell after cell
    int64_t mem_cap;       // entries
    char* half[2];
    int64_t half_cap;      // bytes per half
    char* work;
    int64_t work_cap;      // bytes
    int32_t n_trees;
    int32_t entry_bytes;   // 4: packed points; 8: (id, packed point)
};

}  // namespace hh
