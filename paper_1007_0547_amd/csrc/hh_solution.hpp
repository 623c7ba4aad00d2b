// Host-side launcher of the solution() walk (point removal, Sec. 3).
#pragma once

#include <hip/hip_runtime.h>

#include "hh_types.hpp"

namespace hh {

// One tree (one pass of one image) for the walk.
struct SolTree {
    const Cell* cells;      // the pass's detected cells in key order, voters back to back
    const int32_t* ids;     // voter point ids; cell c's are ids[cells[c].member_off ...]
    int64_t n_cells;
    int64_t n_points;       // ids lie in [0, n_points)
    int64_t n_slots;        // length of ids
    uint8_t* keep;          // [n_cells] 1 = the cell survives removal
    uint8_t* plotted;       // [n_points] 1 = the point was plotted
    uint32_t* bitmap;       // n_points bits of zeroed device memory, or null: the walk keeps them in LDS
    int64_t* counts;        // [2] kept cells, plotted points
    int32_t threshold;
    int32_t pad;
};

// Point ids a walk keeps in LDS; trees with more points need a device bitmap.
int64_t solution_lds_points();
// The walk of n_lds trees with LDS bitmaps (trees[0 .. n_lds)) and n_dev
// trees with device bitmaps (trees[n_lds ...]); max_lds_points is the
// largest n_points among the first.  A malformed tree (cells not back to back,
// an id out of range) raises kErrInternal in *error.
hipError_t launch_solution(const SolTree* trees, int32_t n_lds, int64_t max_lds_points, int32_t n_dev,
                           uint32_t* error, hipStream_t s);

// Point ids of packed-point voter entries (binary-image inputs, whose ids are
// the row-major ranks of their edge points xy[0 .. n_points)): a W x H table
// of ranks (table, W * H int32) is filled from xy, then dst[e] is the rank of
// the point in src[e] for e < n_slots (-1 for an entry outside the image).
hipError_t launch_ids_by_pixel(const uint32_t* xy, int64_t n_points, int32_t width, int32_t height,
                               int32_t* table, const uint32_t* src, int64_t n_slots, int32_t* dst, hipStream_t s);

// The output image: image[y * width + x] = 255 for the voters of the kept
// cells (keep[c] = 1) among n_cells cells whose voters are entries of
// entry_bytes bytes at members[cells[c].member_off ...] (the packed point in
// the low 32 bits); other pixels are left as they are.
hipError_t launch_paint(const Cell* cells, int64_t n_cells, const uint8_t* keep, const void* members,
                        int entry_bytes, int32_t width, int32_t height, uint8_t* image, hipStream_t s);

}  // namespace hh
