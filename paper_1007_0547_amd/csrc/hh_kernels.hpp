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
    int32_t task_steps;        // steps per task of the tasks the emit step makes for the next level
    int32_t queue_batch;       // tasks a wavefront takes from the level's queue at once; 0: fixed share
};

// Edge staging of a batch of binary images: the nonzero pixels of image k,
// row-major, become its packed points at xy[trees' xy_base], and every tree of
// image k (tree.image == k) receives its point range.
struct ExtractArgs {
    const ImageDesc* images;
    int32_t n_images;
    int64_t n_tiles;           // pixel tiles of all images
    uint32_t* xy;              // packed output points, image after image
    int32_t* tile_count;       // [n_tiles] edge pixels per tile
    int64_t* tile_pre;         // [n_tiles] exclusive prefix of tile_count
    TreeDesc* trees;
    int32_t n_trees;
};

// Edge front end of a batch of gray images (Sec. 3: Sobel's operator sorts
// the edge points into ALPHA and BETA).  Image k's ALPHA points, row-major,
// then its BETA points become xy[image base ...], with ids[] holding each
// point's rank among all edge points of its image; the tree of pass 0 gets
// the ALPHA range and the tree of pass 1 the BETA range.
struct SobelArgs {
    const ImageDesc* images;
    int32_t n_images;
    int64_t n_tiles;
    uint32_t* xy;
    int32_t* ids;
    int32_t* tile_count;       // [2][n_tiles] ALPHA, BETA edge pixels per tile
    int64_t* tile_pre;         // [2][n_tiles] their exclusive prefixes
    TreeDesc* trees;
    int32_t n_trees;
};

// Zero the fixed part of an arena (level records, error word, scratch) and
// mark every tree record as absent.
hipError_t launch_clear(const Arena& ar, int64_t n_rec, hipStream_t s);
// Pack the point lists of a batch (total points n_total) into xy; a point
// outside its image raises kErrPointRange.
hipError_t launch_pack_points(const PointsDesc* lists, int32_t n_lists, int64_t n_total, uint32_t* xy,
                              uint32_t* error, hipStream_t s);
// Edge staging in three launches: edge pixels per tile, their exclusive
// prefix (which also fills the trees' point ranges), then the row-major
// compaction.
hipError_t launch_extract(const ExtractArgs& a, hipStream_t s);
// Gray images: Sobel gradients, the two point sets and the trees' ranges, in
// three launches like launch_extract.
hipError_t launch_sobel(const SobelArgs& a, hipStream_t s);
// Root setup: level-0 sizes, root regions and their tasks (task_steps steps
// each) for every tree whose root splits (more than T points and depth > 0),
// from the trees' point ranges; then the root lists (the trees' points in
// input order).
// With ids != nullptr (8-byte entries) a root entry takes its point id from
// ids[] instead of its position in the tree's range.
hipError_t launch_roots(const Arena& ar, const TreeDesc* trees, int32_t n_trees, const uint32_t* xy,
                        const int32_t* ids, int32_t task_steps, int grid, hipStream_t s);
// One level: child-vote counts per task and per-region totals, the split
// decisions, the next level's region and task tables, then the compaction of
// the voters of the kept children (skipped by the host at the finest level
// without members).  Resident workgroups of the count (which = 0) or
// compaction (which = 1) kernel of the given form on a device with cu_count
// compute units.
int level_grid(int which, int variant, bool wide, int entry_bytes, int cu_count);
hipError_t launch_count(const LevelArgs& a, int variant, bool wide, int grid, hipStream_t s);
hipError_t launch_decide(const LevelArgs& a, int grid, hipStream_t s);
hipError_t launch_emit(const LevelArgs& a, int grid, hipStream_t s);
hipError_t launch_write(const LevelArgs& a, int variant, bool wide, int grid, hipStream_t s);
// Point ids of the voters of detected cells (see k_member_ids): cell c's
// voters are src[cells[c].member_off ...]; they go to dst[dst_off[c] ...], or
// with dst_off == nullptr to dst[cells[c].member_off - dst_base ...].
hipError_t launch_member_ids(const Cell* cells, int64_t n_cells, const int64_t* dst_off, int64_t dst_base,
                             const void* src, int entry_bytes, const uint32_t* xy, int64_t n_points, int32_t* dst,
                             hipStream_t s);
// dst[c] = src[c] with member_off - base (cells whose member_off < 0 keep it).
hipError_t launch_rebase_cells(const Cell* src, int64_t n, int64_t base, Cell* dst, hipStream_t s);
hipError_t launch_iota(int32_t* dst, int64_t n, hipStream_t s);

}  // namespace hh
