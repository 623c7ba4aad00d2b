// Types and memory layout shared by the device kernels and the host engine
// of the hierarchical Hough vote library.  Nothing here is part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hh {

constexpr int kWave = 64;                 // CDNA wavefront width
constexpr int kBlock = 256;               // threads per workgroup (4 wavefronts)
constexpr int kWaves = kBlock / kWave;
constexpr int kEpt = 8;                   // list entries per lane in the vote kernel
constexpr int kWaveSpan = kWave * kEpt;   // 512 consecutive entries per wavefront
constexpr int kTile = kBlock * kEpt;      // 2048 entries per vote tile
constexpr int kStage = 128;               // regions of a tile whose data is staged in LDS
constexpr int kPixPerThread = 16;         // image bytes per lane in edge staging
constexpr int kPixTile = kBlock * kPixPerThread;
constexpr int kMaxLevels = 16;            // depth <= 15
constexpr int kNumStats = 6;              // evaluated, votes, split, detected, code_tests, entries
constexpr int kDecCh = 4;                 // decision channels: n_next, len_next, cells, votes
constexpr int kRecCh = 6;                 // tree record: p, start, then the decision prefixes

// Error bits set by kernels (the host reports them after the call).
constexpr uint32_t kErrLookback = 1u;     // a bounded wait timed out
constexpr uint32_t kErrPointRange = 2u;   // an input point lies outside [0,W)x[0,H)
constexpr uint32_t kErrInternal = 4u;     // an index failed a range check
constexpr uint32_t kErrArena = 8u;        // a level did not fit its arena; rerun larger
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
    int32_t image;
    int32_t pad;
};

// Region.meta bits
constexpr uint32_t kMetaPass = 1u;            // pass 1: axes swapped
constexpr int kMetaSlogShift = 1;             // s_log2 in bits 1..4
constexpr uint32_t kMetaChildFinest = 1u << 5;   // the region's children are at the finest level

// A region that split: its voters form one list of the level.
struct Region {
    int64_t start;      // first flat entry index of its list within the level
    int64_t in_base;    // entry e of the level lives at list[in_base + e]; for the
                        // root lists (level 0) in_base + e indexes the point array
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
    int64_t pad[3];
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

// Buffers of level l inside its arena half (l & 1).  regions / tile_first
// are written by the split decision of level l-1 (or the root setup) and
// sized from level l-1; the rest is written by the launches of level l.
//   out    children's voter lists: child q of the parent with flat start s
//          and length n occupies out[4 s + q n, 4 s + q n + votes)
//   cv     [P][4] child votes
//   dvw    [P][4] decision values of the parents before it whose list ends in
//          the same wavefront span (exclusive prefix)
//   wpre   [tiles][kWaves][4] exclusive prefix of the decision values of the
//          wavefront spans of a tile
//   vts    [tiles][4] decision totals per tile;  vtp: their exclusive prefix
struct LevelLayout {
    Region* regions;
    int64_t regions_cap;
    int32_t* tile_first;
    int64_t tile_cap;
    void* out;          // 4 L entries of entry_bytes
    int32_t* cv;
    int32_t* dvw;
    int32_t* wpre;
    int32_t* vts;
    int64_t* vtp;
    int64_t end;        // bytes used from the half's start
};

__host__ __device__ inline LevelLayout level_layout(char* half, int level, int64_t P_prev, int64_t L_prev,
                                                    int64_t P, int64_t L, int32_t n_trees, int entry_bytes)
{
    LevelLayout y;
    y.regions_cap = level == 0 ? n_trees : 4 * P_prev;
    y.tile_cap = (level == 0 ? cdiv(L, kTile) : cdiv(4 * L_prev, kTile)) + 1;
    const int64_t nt = cdiv(L, kTile);
    int64_t off = 0;
    y.regions = reinterpret_cast<Region*>(half + off);
    off += align256(y.regions_cap * (int64_t)sizeof(Region));
    y.tile_first = reinterpret_cast<int32_t*>(half + off);
    off += align256(y.tile_cap * 4);
    y.out = half + off;
    off += align256(4 * L * entry_bytes);
    y.cv = reinterpret_cast<int32_t*>(half + off);
    off += align256(4 * P * 4);
    y.dvw = reinterpret_cast<int32_t*>(half + off);
    off += align256(4 * P * 4);
    y.wpre = reinterpret_cast<int32_t*>(half + off);
    off += align256(nt * kWaves * kDecCh * 4);
    y.vts = reinterpret_cast<int32_t*>(half + off);
    off += align256(nt * kDecCh * 4);
    y.vtp = reinterpret_cast<int64_t*>(half + off);
    off += align256(nt * kDecCh * 8);
    y.end = off;
    return y;
}

// All device memory of one call: a fixed part and two level halves used in
// turn.
struct Arena {
    LevelInfo* info;       // [kMaxLevels + 1]
    int64_t* rec;          // [n_trees][kMaxLevels][kRecCh] tree boundary records (-1: none)
    uint32_t* error;
    int64_t* scalar;       // [8] scratch (edge count, ...)
    Cell* cells;
    int64_t cells_cap;
    char* half[2];
    int64_t half_cap;      // bytes per half
    int32_t n_trees;
    int32_t entry_bytes;   // 4: packed points; 8: (id, packed point)
};

}  // namespace hh
