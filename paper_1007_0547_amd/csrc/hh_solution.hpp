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
    uint32_t* all;          // n_points bits: every point plotted by the tree's segments (after a merge)
    int64_t* counts;        // [2] kept cells, plotted points
    int32_t threshold;
    int32_t seg0, n_segs;   // its segments: segs[seg0 .. seg0 + n_segs)
    int32_t pad;
};

// One segment of a tree: cells [c0, c1), walked from the points in `in`.
struct SolSeg {
    int32_t tree;
    int32_t pad;
    int64_t c0, c1;
    uint32_t* in;           // n_points bits: points taken as plotted before the segment
    uint32_t* out;          // n_points bits: points the segment plotted beyond `in`
    uint32_t* work;         // n_points bits of device memory for the walk, or null: it keeps them in LDS
    int64_t* counts;        // [2] kept cells, plotted points of the segment
};

// Point ids a walk keeps in LDS; trees with more points need device bitmaps.
int64_t solution_lds_points();

constexpr int kSolMaxSegs = 128;   // segments of one tree (the fastest of 64, 128 and 256 on the 1024x1024 image)

// One round of segment walks and what follows them.  Segments of a tree are
// consecutive in segs, in cell order; segs[0 .. n_lds) are of trees that keep
// their bitmap in LDS (at most max_lds_points points), the rest use device
// bitmaps.
struct SolRound {
    const SolTree* trees;
    const SolSeg* segs;
    int32_t n_trees, n_segs, n_lds;
    int32_t grid;                 // most workgroups of a walk launch
    int64_t max_lds_points;
    int64_t max_words;            // the largest bitmap, in 32-bit words
    const int32_t* list_lds;      // this round's segments: LDS ones, device ones,
    const int32_t* list_dev;
    const int32_t* n_list;        // and their numbers ([0], [1])
    int32_t* next_lds;            // the next round's, made by this one
    int32_t* next_dev;
    int32_t* n_next;
    int32_t* first_walked;        // [n_trees] INT_MAX between rounds
    uint8_t* changed;             // [n_segs] zero between rounds
    uint32_t* error;              // kErrInternal: a malformed tree (cells not back to back, an id out of range)
};

// The walks of the round's segments, then per tree with a walked segment the
// inputs of the segments from it on (the union of the outputs before each;
// `all`, the union of every output), and the next round's lists: the
// segments whose input changed.  No segment in the next lists: every input
// stands, and the walk is done.
hipError_t launch_solution_round(const SolRound& r, hipStream_t s);
// Each tree's segment bounds (c0, c1) by voter entries: segment q of a tree
// with K segments starts at the first cell whose voters start at or past
// q / K of its entries.  Before the first round.
hipError_t launch_solution_cut(const SolTree* trees, SolSeg* segs, int32_t n_segs, hipStream_t s);
// Once a merge changed nothing: per tree, plotted flags from `all` and the
// counts summed over its segments.
hipError_t launch_solution_finish(const SolTree* trees, int32_t n_trees, const SolSeg* segs, hipStream_t s);

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
