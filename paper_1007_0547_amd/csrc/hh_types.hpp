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
constexpr int kRows = 8;                    // 64-entry rows per wavefront in a tile
constexpr int kTileRows = kWaves * kRows;   // 32 rows
constexpr int kTile = kTileRows * kWave;    // 2048 list entries per tile
constexpr int kStage = 256;                 // regions of a tile whose fields are staged in LDS
constexpr int kPixPerThread = 16;           // image bytes per lane in edge staging
constexpr int kPixTile = kBlock * kPixPerThread;
constexpr int kMaxLevels = 16;              // depth <= 15
constexpr int kNumStats = 6;                // evaluated, votes, split, detected, code_tests, entries
constexpr int kAggCh = 5;                   // decision sums: next regions, next entries, cells, member entries, votes
constexpr int kRecCh = 7;                   // tree record: p, start, then the decision prefixes
constexpr int kRangeGrid = 512;             // region ranges of the split-decision launches
constexpr int kMaxTrees = 2048;             // trees (image passes) in one call

// Error bits set by kernels (the host reports them after the call).
constexpr uint32_t kErrPointRange = 2u;     // an input point lies outside [0,W)x[0,H)
constexpr uint32_t kErrInternal = 4u;       // an index failed a range check
constexpr uint32_t kErrArena = 8u;          // a level did not fit its arena; rerun larger
constexpr uint32_t kErrStop = kErrArena | kErrInternal;   // later kernels do nothing

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
    int64_t pad;
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

// The part of the corner test (Sec. 2) a region shares with all its lines,
// for the 4-bit code variant with 32-bit compares: M0 = M of the first corner
// column of its children's grid and nB_r = -B_r - 1 for the three corner rows,
// at the children's level.
struct CodeConsts {
    int32_t M0, nB0, nB1, nB2;
};

__host__ __device__ inline CodeConsts code_consts(uint32_t ij, uint32_t meta, int lc)
{
    const int s_log2 = (int)((meta >> 1) & 15u);
    const int32_t S = 1 << s_log2;
    const int32_t pi = (int32_t)(ij & 0xFFFFu), pj = (int32_t)(ij >> 16);
    const int32_t B0 = 6 * S * pj - (S << lc);
    CodeConsts c;
    c.M0 = 4 * pi - (1 << lc);
    c.nB0 = -B0 - 1;
    c.nB1 = -(B0 + 3 * S) - 1;
    c.nB2 = -(B0 + 6 * S) - 1;
    return c;
}

// A level's data inside its arena half (l & 1): the region table, the tile
// map, the regions' code constants and the child-vote totals (zeroed),
// written by the previous level's split decision (or the root setup), then
// the level's list, written by the previous level's compaction.
// tile_first[t] is the region holding entry t * kTile; cv[r][q] collects the
// votes of child q of region r.
struct HalfLayout {
    Region* regions;
    int32_t* tile_first;
    CodeConsts* cc;
    int32_t* cv;
    void* list;
    int64_t end;        // bytes used from the half's start
};

__host__ __device__ inline HalfLayout half_layout(char* half, int64_t P, int64_t L, int entry_bytes)
{
    HalfLayout y;
    int64_t off = 0;
    y.regions = reinterpret_cast<Region*>(half + off);
    off += align256(P * (int64_t)sizeof(Region));
    y.tile_first = reinterpret_cast<int32_t*>(half + off);
    off += align256((cdiv(L, kTile) + 1) * 4);
    y.cc = reinterpret_cast<CodeConsts*>(half + off);
    off += align256(P * (int64_t)sizeof(CodeConsts));
    y.cv = reinterpret_cast<int32_t*>(half + off);
    off += align256(P * 16);
    y.list = half + off;
    off += align256(L * entry_bytes);
    y.end = off;
    return y;
}

// Per-level scratch, reused by every level.
//   head  [P][4]  child votes of a region in the tile where it starts, for
//                 regions that run past that tile
//   dst   [P][4]  where the child's voters go (next list or member buffer), -1: dropped
//   tcar  [nt][4] child votes of the region carried into tile t from earlier tiles
//   woff  [nt][kWaves][4] child votes of the region open at each wavefront's
//                 first entry, counted from its first entry in the tile
//   vbits [nt][kBlock] the vote bits of the count pass for the compaction
//                 pass: lane t of a tile, bits 4k .. 4k+3 = votes of the
//                 entry in its wavefront's row k for the children NE, NW, SW, SE
//   agg   [kRangeGrid][kAggCh] decision sums per range of regions
struct WorkLayout {
    int32_t* head;
    int64_t* dst;
    int32_t* tcar;
    int32_t* woff;
    uint32_t* vbits;
    int64_t* agg;
    int64_t end;
};

__host__ __device__ inline WorkLayout work_layout(char* work, int64_t P, int64_t L)
{
    WorkLayout w;
    const int64_t nt = cdiv(L, kTile);
    int64_t off = 0;
    w.head = reinterpret_cast<int32_t*>(work + off);
    off += align256(P * 16);
    w.dst = reinterpret_cast<int64_t*>(work + off);
    off += align256(P * 32);
    w.tcar = reinterpret_cast<int32_t*>(work + off);
    off += align256(nt * 16);
    w.woff = reinterpret_cast<int32_t*>(work + off);
    off += align256(nt * kWaves * 16);
    w.vbits = reinterpret_cast<uint32_t*>(work + off);
    off += align256(nt * kBlock * 4);
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
    int64_t* scalar;       // [8] scratch (edge count, ...)
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
