// Host-side launchers for the gfx950 kernels of the hierarchical Hough vote.
#pragma once

#include <hip/hip_runtime.h>

#include "hh_types.hpp"

namespace hh {

struct VoteArgs {
    const Region* regions;     // level-l split regions in (tree, key) order
    int32_t n_regions;
    const int32_t* tile_first; // region containing each tile's first entry
    int32_t n_tiles;
    const int32_t* list;       // the level's list buffer
    const TreeDesc* trees;
    int64_t n_entries;         // L_l
    int32_t level;             // l: the parents' level; children are at l + 1
    int32_t write_out;         // 0: count only (no voter lists for the children)
    int32_t* out;              // 4 slices (NE, NW, SW, SE) of out_cap entries
    int64_t out_cap;
    int64_t* pstart;           // [n_regions][4]: exclusive slice prefix at each region's first entry
    uint64_t* status;          // [n_tiles][4] look-back words, zeroed
    uint32_t* ticket;          // tile ticket, zeroed
    LevelTotals* totals;
    uint32_t* error;
};

struct DecideArgs {
    const Region* regions;
    int32_t n_regions;
    const TreeDesc* trees;
    int32_t level;
    const int64_t* pstart;
    int64_t out_cap;
    uint64_t* status;          // [n_tiles][3] look-back words, zeroed
    uint32_t* ticket;
    int32_t n_tiles;
    LevelTotals* totals;       // reads votes[], writes n_next, len_next, n_cells
    Region* next_regions;      // level l+1 split regions (may be null when none can split)
    int32_t* next_tile_first;
    int64_t next_tile_cap;
    Cell* cells;               // detected cells (may be null when none can be detected)
    int64_t* stats;            // [tree][kMaxLevels][kNumStats]
    int32_t keep_members;      // 0: cells get member_off = -1
    uint32_t* error;
};

struct ExtractArgs {
    const uint8_t* image;
    int64_t row_stride;
    int32_t width, height;
    int64_t n_pix;
    int32_t* x;
    int32_t* y;
    uint64_t* status;          // [n_tiles] look-back words, zeroed
    uint32_t* ticket;
    int32_t n_tiles;
    int64_t* total;
    uint32_t* error;
};

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t value, hipStream_t s);
hipError_t launch_init_level0(Region* regions, int32_t* tile_first, int32_t* iota,
                              int32_t n_trees, int64_t n_points, int32_t n_tiles, hipStream_t s);
hipError_t launch_vote(const VoteArgs& a, int variant, bool wide, hipStream_t s);
hipError_t launch_decide(const DecideArgs& a, hipStream_t s);
hipError_t launch_extract(const ExtractArgs& a, hipStream_t s);
hipError_t launch_validate(const int32_t* x, const int32_t* y, int64_t n, int32_t W, int32_t H,
                           uint32_t* error, hipStream_t s);
hipError_t launch_gather_members(const Cell* cells, int64_t n_cells, const int64_t* dst_off,
                                 const int32_t* src, int32_t* dst, hipStream_t s);

}  // namespace hh
