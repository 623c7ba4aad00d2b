// Types shared by the device kernels and the host engine of the
// hierarchical Hough vote library.  Nothing here is part of the public ABI.
#pragma once

#include <stdint.h>

namespace hh {

constexpr int kWave = 64;                 // CDNA wavefront width
constexpr int kBlock = 256;               // threads per workgroup (4 wavefronts)
constexpr int kWaves = kBlock / kWave;
constexpr int kEpt = 8;                   // list entries per lane in the vote kernel
constexpr int kWaveSpan = kWave * kEpt;   // 512 consecutive entries per wavefront
constexpr int kTile = kBlock * kEpt;      // 2048 entries per vote tile
constexpr int kPixPerThread = 16;         // image bytes per lane in edge staging
constexpr int kPixTile = kBlock * kPixPerThread;
constexpr int kMaxLevels = 16;            // depth <= 15
constexpr int kNumStats = 6;              // evaluated, votes, split, detected, code_tests, entries

// Error bits set by kernels (host reports them after the call).
constexpr uint32_t kErrLookback = 1u;     // a look-back wait hit its spin limit
constexpr uint32_t kErrPointRange = 2u;   // an input point lies outside [0,W)x[0,H)
constexpr uint32_t kErrInternal = 4u;     // an index failed a range check

// One quadtree: one pass over one image's edge points.
struct TreeDesc {
    const int32_t* u;   // slope-axis coordinate (x for pass 0, y for pass 1)
    const int32_t* v;   // intercept-axis coordinate (y for pass 0, x for pass 1)
    int64_t n_points;
    int32_t s_log2;     // S = 2^s_log2
    int32_t dmax;       // finest level
    int32_t threshold;  // a region splits (or is detected) iff votes > threshold
    int32_t pass;
    int32_t image;
    int32_t pad;
};

// A region that split: its voters form one list of the level.
struct Region {
    int64_t start;      // first flat entry index of its list within the level
    int64_t off;        // position of its list in the level's list buffer
    int32_t i, j;       // indices at its level
    int32_t len;        // votes = list length
    int32_t tree;
};

// Totals a level's kernels leave for the host (one struct per level).
struct LevelTotals {
    int64_t votes[4];   // summed votes per child slot (NE, NW, SW, SE)
    int64_t n_next;     // children that split
    int64_t len_next;   // total list length of those children
    int64_t n_cells;    // children detected at the finest level
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

}  // namespace hh
