// Host-side launchers for the gfx950 kernels of the hierarchical Hough vote.
#pragma once

#include <hip/hip_runtime.h>

#include "hh_types.hpp"

namespace hh {

// Arguments of one level's launches.  Sizes are not passed: the kernels read
// them from ar.info, filled in by earlier launches.
struct LevelArgs {
    Arena ar;
    const TreeDesc* trees;
    const uint32_t* xy;        // packed edge points
    int32_t level;             // l: the parents' level; children are at l + 1
    int32_t keep_members;      // 0: detected cells get member_off = -1 and keep no voters
};

struct ExtractArgs {
    const uint8_t* image;
    int64_t row_stride;
    int32_t width, height;
    int64_t n_pix;
    uint32_t* xy;              // packed output points
    int32_t* tile_count;       // [n_tiles] edge pixels per tile
    int64_t* tile_pre;         // [n_tiles] exclusive prefix of tile_count
    int32_t n_tiles;
    int64_t* total;            // edge count
};

// Zero the fixed part of an arena (level records, error word, scratch) and
// mark every tree record as absent.
hipError_t launch_clear(const Arena& ar, int64_t n_rec, hipStream_t s);
hipError_t launch_pack_points(const int32_t* x, const int32_t* y, int64_t n, int32_t W, int32_t H,
                              uint32_t* xy, uint32_t* error, hipStream_t s);
// Edge staging in three launches: edge pixels per tile, their exclusive
// prefix, then the row-major compaction.
hipError_t launch_extract(const ExtractArgs& a, hipStream_t s);
// Root setup: level-0 sizes, root regions, tile map and root lists.
// n_points < 0 takes the edge count from ar.scalar[0] (left there by the
// edge staging).
hipError_t launch_begin(const Arena& ar, TreeDesc* trees, int32_t n_trees, int64_t n_points, int32_t threshold,
                        int32_t dmax, const uint32_t* xy, int grid, hipStream_t s);
// One level: child-vote counts per tile, per-region totals and decisions,
// the next level's tables, then the compaction of the voters of the kept
// children (skipped by the host at the finest level without members).
// Resident workgroups of the count (which = 0) or compaction (which = 1)
// kernel of the given form on a device with cu_count compute units (the
// compaction kernel depends on the entry size only).
int level_grid(int which, int variant, bool wide, int entry_bytes, int cu_count);
hipError_t launch_count(const LevelArgs& a, int variant, bool wide, int grid, hipStream_t s);
hipError_t launch_decide(const LevelArgs& a, int grid, hipStream_t s);
hipError_t launch_emit(const LevelArgs& a, int grid, hipStream_t s);
hipError_t launch_write(const LevelArgs& a, int grid, hipStream_t s);
// Point ids of the voters of detected cells (see k_member_ids): into the
// member buffer's layout (dst_off == nullptr) or compacted at dst_off[c].
hipError_t launch_member_ids(const Cell* cells, int64_t n_cells, const int64_t* dst_off, const void* src,
                             int entry_bytes, const uint32_t* xy, int64_t n_points, int32_t* dst, hipStream_t s);
hipError_t launch_iota(int32_t* dst, int64_t n, hipStream_t s);

}  // namespace hh
