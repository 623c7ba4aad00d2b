// gfx950 kernels of the hierarchical slope-intercept Hough vote
// (Singh and Bhatia, arXiv:1007.0547).
//
// Level-synchronous form of the paper's depth-first search (Sec. 3): all
// regions that split at level l (of every tree = pass of an image) are
// processed together.  Their voter lists are stored back to back; a flat
// entry index e in [0, L_l) walks all (parent region, line) pairs.
//
//   k_vote    one read of every (parent, line) entry: the 4-bit corner codes
//             of the line for the four children (Sec. 2, getcode()), the vote
//             rule (code not 0000 / 1111, steps 5 and 12.v), wave ballots for
//             the child vote counts, a decoupled look-back scan over tiles,
//             and a stable stream compaction of the crossing lines into four
//             slices (one per child position NE, NW, SW, SE).  The list of
//             child q of parent R is the run of slice q between the slice
//             prefixes at R's first entry and at the next region's first entry.
//   k_decide  per parent: the four child vote counts from those prefixes,
//             the threshold rule (step 13: split below the finest level,
//             detected at it), a look-back scan over the children that split,
//             and the level-(l+1) region table (in quad order, so key order is
//             kept) or the detected cells.
//
// Look-back status words pack a 2-bit flag with a 62-bit value and are read
// and written with agent-scope atomics; a tile id comes from an atomic ticket
// so every tile a tile waits on is already owned by a running workgroup.
// Every wait is bounded: on timeout a kernel raises kErrLookback and goes on.

#include <hip/hip_runtime.h>

#include "hh_kernels.hpp"

namespace hh {
namespace {

constexpr uint64_t kFlagAggregate = 1ull << 62;
constexpr uint64_t kFlagInclusive = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;
constexpr uint64_t kWaitTicks = 50000000;   // 0.5 s of the 100 MHz wall clock

__device__ inline uint64_t load_status(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void store_status(uint64_t* p, uint64_t w)
{
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled look-back for one channel of one tile.  Publishes the tile's
// aggregate, sums predecessors until one with an inclusive prefix, publishes
// its own inclusive prefix and returns its exclusive prefix.
__device__ int64_t lookback(uint64_t* status, int64_t tile, int nch, int ch, int64_t agg,
                            uint32_t* error)
{
    uint64_t* mine = status + tile * nch + ch;
    if (tile == 0) {
        store_status(mine, kFlagInclusive | (uint64_t)agg);
        return 0;
    }
    store_status(mine, kFlagAggregate | (uint64_t)agg);
    int64_t excl = 0;
    const uint64_t deadline = wall_clock64() + kWaitTicks;
    for (int64_t k = tile - 1; k >= 0; --k) {
        uint64_t w = 0;
        for (;;) {
            w = load_status(status + k * nch + ch);
            if (w >> 62) break;
            if (wall_clock64() > deadline) {
                atomicOr(error, kErrLookback);
                w = kFlagInclusive;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        excl += (int64_t)(w & kValueMask);
        if ((w >> 62) == 2) break;
    }
    store_status(mine, kFlagInclusive | (uint64_t)(excl + agg));
    return excl;
}

__device__ inline uint32_t lanes_below(uint64_t b)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
}

__device__ inline int code_votes(uint32_t code) { return code != 0u && code != 15u; }

// Child crossing mask of one line for the four children of parent (pi, pj),
// children at level lc.  Bit q set <=> the line votes for child q, where
// q = 0 NE (east 1, north 1), 1 NW (0, 1), 2 SW (0, 0), 3 SE (1, 0).
//
// Code variant (Sec. 2).  The children's corners form the parent's 3x3
// corner grid at level lc: columns ic = 2 pi + c and rows jc = 2 pj + r,
// c, r in {0, 1, 2}, at m = M_c / 2^lc and b = B_r / 2^lc with
// M_c = 2 ic - 2^lc and B_r = -S 2^lc + 3 S jc.  Corner (c, r) is below the
// line b = v - u m iff B_r < t_c with t_c = v 2^lc - u M_c; consecutive
// columns differ by 2 in M, so t_{c+1} = t_c - 2u.  Nine exact compares give
// the four codes (NE bit leftmost).
template <typename CT>
__device__ inline uint32_t code_mask(int32_t u, int32_t v, int32_t pi, int32_t pj, int lc,
                                     int s_log2)
{
    const CT S = (CT)1 << s_log2;
    const CT scale = (CT)1 << lc;
    const CT M0 = (CT)4 * (CT)pi - scale;
    const CT t0 = ((CT)v << lc) - (CT)u * M0;
    const CT du = (CT)2 * (CT)u;
    const CT t1 = t0 - du;
    const CT t2 = t1 - du;
    const CT B0 = (CT)6 * S * (CT)pj - (S << lc);
    const CT B1 = B0 + (CT)3 * S;
    const CT B2 = B1 + (CT)3 * S;
    // below[c][r]
    const uint32_t b00 = B0 < t0, b01 = B1 < t0, b02 = B2 < t0;
    const uint32_t b10 = B0 < t1, b11 = B1 < t1, b12 = B2 < t1;
    const uint32_t b20 = B0 < t2, b21 = B1 < t2, b22 = B2 < t2;
    // code = NE<<3 | NW<<2 | SW<<1 | SE with NE = (e+1, n+1), NW = (e, n+1),
    // SW = (e, n), SE = (e+1, n) for the child at (e, n)
    const uint32_t cNE = (b22 << 3) | (b12 << 2) | (b11 << 1) | b21;   // e = 1, n = 1
    const uint32_t cNW = (b12 << 3) | (b02 << 2) | (b01 << 1) | b11;   // e = 0, n = 1
    const uint32_t cSW = (b11 << 3) | (b01 << 2) | (b00 << 1) | b10;   // e = 0, n = 0
    const uint32_t cSE = (b21 << 3) | (b11 << 2) | (b10 << 1) | b20;   // e = 1, n = 0
    return (uint32_t)code_votes(cNE) | ((uint32_t)code_votes(cNW) << 1) |
           ((uint32_t)code_votes(cSW) << 2) | ((uint32_t)code_votes(cSE) << 3);
}

// Circumscribed-circle variant (comparison method of the paper's ref. [9]).
// For child (lc, i, j) with centre m = -1 + (2i+1)/2^lc,
// b = -S + 3S(2j+1)/2^(lc+1), in units where the cell is a unit square, the
// line is within the circumradius iff D^2 <= 2 (9 S^2 + 4 u^2) with
// D = 3S(2j+1) + 2u(2i+1) - (v + u + S) 2^(lc+1).
__device__ inline uint32_t circle_mask(int32_t u, int32_t v, int32_t pi, int32_t pj, int lc,
                                       int s_log2)
{
    const int64_t S = (int64_t)1 << s_log2;
    const int64_t U = u;
    const int64_t base = ((int64_t)v + U + S) << (lc + 1);
    const int64_t a_s = 3 * S * (4 * (int64_t)pj + 1) - base;   // north = 0: 2j+1 = 4 pj + 1
    const int64_t a_n = a_s + 6 * S;                             // north = 1: 4 pj + 3
    const int64_t c_w = 2 * U * (4 * (int64_t)pi + 1);           // east = 0
    const int64_t c_e = c_w + 4 * U;                             // east = 1
    const int64_t rhs = 2 * (9 * S * S + 4 * U * U);
    const int64_t dNE = a_n + c_e, dNW = a_n + c_w, dSW = a_s + c_w, dSE = a_s + c_e;
    return (uint32_t)(dNE * dNE <= rhs) | ((uint32_t)(dNW * dNW <= rhs) << 1) |
           ((uint32_t)(dSW * dSW <= rhs) << 2) | ((uint32_t)(dSE * dSE <= rhs) << 3);
}

template <int kVariant, typename CT>
__device__ inline uint32_t child_mask(int32_t u, int32_t v, int32_t pi, int32_t pj, int lc,
                                      int s_log2)
{
    if constexpr (kVariant == 0)
        return code_mask<CT>(u, v, pi, pj, lc, s_log2);
    else
        return circle_mask(u, v, pi, pj, lc, s_log2);
}

template <int kVariant, typename CT>
__global__ __launch_bounds__(kBlock) void k_vote(VoteArgs a)
{
    __shared__ uint16_t s_rel[kTile + 1];     // region starts relative to the tile
    __shared__ int32_t s_wcnt[kWaves][4];
    __shared__ int64_t s_excl[4];
    __shared__ int32_t s_tile;

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if (tid == 0) s_tile = (int32_t)atomicAdd(a.ticket, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t t0 = tile * kTile;
    const int r0 = a.tile_first[tile];
    const int r1 = (tile + 1 < a.n_tiles) ? a.tile_first[tile + 1] : a.n_regions - 1;
    int nr = r1 - r0 + 1;   // <= kTile + 1: every region holds at least one entry
    if (nr < 1 || nr > kTile + 1) {
        if (tid == 0) atomicOr(a.error, kErrInternal);
        nr = nr < 1 ? 1 : kTile + 1;
    }
    for (int k = tid; k < nr; k += kBlock) {
        const int64_t rel = a.regions[r0 + k].start - t0;
        s_rel[k] = (uint16_t)(rel < 0 ? 0 : (rel > kTile ? kTile : rel));
    }
    __syncthreads();

    const int64_t wbase = t0 + (int64_t)wave * kWaveSpan;
    int32_t ids[kEpt];
    int32_t reg[kEpt];
    uint32_t masks = 0;      // 4 bits per entry
    uint32_t starts = 0;     // bit k: entry k is the first entry of its region
    int32_t cnt[4] = {0, 0, 0, 0};

#pragma unroll
    for (int k = 0; k < kEpt; ++k) {
        const int64_t e = wbase + k * kWave + lane;
        uint32_t m = 0;
        ids[k] = 0;
        reg[k] = 0;
        if (e < a.n_entries) {
            const int er = (int)(e - t0);
            int lo = 0, hi = nr - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((int)s_rel[mid] <= er) lo = mid; else hi = mid - 1;
            }
            const int r = r0 + lo;
            const Region R = a.regions[r];
            const int64_t at = e - R.start;
            if ((uint64_t)at < (uint64_t)R.len) {
                const int32_t id = a.list[R.off + at];
                const TreeDesc* T = a.trees + R.tree;
                if ((uint64_t)id < (uint64_t)T->n_points) {
                    const int32_t u = T->u[id];
                    const int32_t v = T->v[id];
                    m = child_mask<kVariant, CT>(u, v, R.i, R.j, a.level + 1, T->s_log2);
                } else {
                    atomicOr(a.error, kErrInternal);
                }
                ids[k] = id;
                reg[k] = r;
                if (at == 0) starts |= 1u << k;
            } else {
                atomicOr(a.error, kErrInternal);
            }
        }
        masks |= m << (4 * k);
#pragma unroll
        for (int q = 0; q < 4; ++q) cnt[q] += (int32_t)__popcll(__ballot((m >> q) & 1u));
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s_wcnt[wave][q] = cnt[q];
    }
    __syncthreads();
    if (tid < 4) {
        int64_t agg = 0;
        for (int w = 0; w < kWaves; ++w) agg += s_wcnt[w][tid];
        const int64_t excl = lookback(a.status, tile, 4, tid, agg, a.error);
        s_excl[tid] = excl;
        if (tile == a.n_tiles - 1) a.totals->votes[tid] = excl + agg;
    }
    __syncthreads();

    int64_t base[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int64_t b = s_excl[q];
        for (int w = 0; w < wave; ++w) b += s_wcnt[w][q];
        base[q] = b;
    }
#pragma unroll
    for (int k = 0; k < kEpt; ++k) {
        const uint32_t m = (masks >> (4 * k)) & 15u;
        const bool first = (starts >> k) & 1u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t bit = (m >> q) & 1u;
            const uint64_t b = __ballot(bit);
            const int64_t pos = base[q] + lanes_below(b);
            if (bit && a.write_out) a.out[(int64_t)q * a.out_cap + pos] = ids[k];
            if (first) a.pstart[(int64_t)reg[k] * 4 + q] = pos;
            base[q] += (int64_t)__popcll(b);
        }
    }
}

__device__ inline int64_t wave_incl_scan(int64_t x, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ inline int64_t wave_sum(int64_t x)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// quad digit of child (east, north): NE = 0, NW = 1, SW = 2, SE = 3
__device__ inline int64_t key_of(int32_t i, int32_t j, int depth)
{
    int64_t key = 0;
    for (int b = depth - 1; b >= 0; --b) {
        const int e = (i >> b) & 1, n = (j >> b) & 1;
        key = key * 4 + (((n ^ 1) << 1) | (e ^ n));
    }
    return key;
}

__global__ __launch_bounds__(kBlock) void k_decide(DecideArgs a)
{
    __shared__ int64_t s_wtot[kWaves][3];
    __shared__ int64_t s_excl[3];
    __shared__ int32_t s_tile;

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if (tid == 0) s_tile = (int32_t)atomicAdd(a.ticket, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t p = tile * kBlock + tid;
    const bool valid = p < a.n_regions;
    const int lc = a.level + 1;

    int64_t glo[4] = {0, 0, 0, 0}, votes[4] = {0, 0, 0, 0};
    Region R{};
    int32_t thr = 0, pass = 0, tree = 0;
    bool finest = false;
    if (valid) {
        R = a.regions[p];
        tree = R.tree;
        const TreeDesc T = a.trees[R.tree];
        thr = T.threshold;
        pass = T.pass;
        finest = (lc == T.dmax);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            glo[q] = a.pstart[p * 4 + q];
            const int64_t ghi = (p + 1 < a.n_regions) ? a.pstart[(p + 1) * 4 + q] : a.totals->votes[q];
            votes[q] = ghi - glo[q];
        }
    }
    int64_t n_next = 0, len_next = 0, n_cells = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (valid && votes[q] > thr) {
            if (finest) ++n_cells;
            else { ++n_next; len_next += votes[q]; }
        }
    }

    // per-tree, per-level statistics for the children's level
    {
        int64_t st[kNumStats] = {valid ? 4 : 0,
                                 votes[0] + votes[1] + votes[2] + votes[3],
                                 n_next, n_cells,
                                 valid ? 4 * (int64_t)R.len : 0,
                                 len_next};
        const int32_t tree0 = __shfl(tree, 0, kWave);
        const bool uniform = __all(!valid || tree == tree0);
        if (uniform) {
#pragma unroll
            for (int s = 0; s < kNumStats; ++s) {
                const int64_t tot = wave_sum(st[s]);
                if (lane == 0 && tot != 0)
                    atomicAdd((unsigned long long*)&a.stats[((int64_t)tree0 * kMaxLevels + lc) * kNumStats + s],
                              (unsigned long long)tot);
            }
        } else if (valid) {
            for (int s = 0; s < kNumStats; ++s)
                if (st[s] != 0)
                    atomicAdd((unsigned long long*)&a.stats[((int64_t)tree * kMaxLevels + lc) * kNumStats + s],
                              (unsigned long long)st[s]);
        }
    }

    // block-wide exclusive scan of (n_next, len_next, n_cells)
    const int64_t in0 = wave_incl_scan(n_next, lane);
    const int64_t in1 = wave_incl_scan(len_next, lane);
    const int64_t in2 = wave_incl_scan(n_cells, lane);
    if (lane == kWave - 1) {
        s_wtot[wave][0] = in0;
        s_wtot[wave][1] = in1;
        s_wtot[wave][2] = in2;
    }
    __syncthreads();
    if (tid < 3) {
        int64_t agg = 0;
        for (int w = 0; w < kWaves; ++w) agg += s_wtot[w][tid];
        const int64_t excl = lookback(a.status, tile, 3, tid, agg, a.error);
        s_excl[tid] = excl;
        if (tile == a.n_tiles - 1) {
            if (tid == 0) a.totals->n_next = excl + agg;
            if (tid == 1) a.totals->len_next = excl + agg;
            if (tid == 2) a.totals->n_cells = excl + agg;
        }
    }
    __syncthreads();
    int64_t ri = s_excl[0] + in0 - n_next;
    int64_t start = s_excl[1] + in1 - len_next;
    int64_t ci = s_excl[2] + in2 - n_cells;
    for (int w = 0; w < wave; ++w) {
        ri += s_wtot[w][0];
        start += s_wtot[w][1];
        ci += s_wtot[w][2];
    }
    if (!valid) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (votes[q] <= thr) continue;
        const int32_t e = (q == 0 || q == 3) ? 1 : 0;
        const int32_t n = (q <= 1) ? 1 : 0;
        const int32_t ci_ = 2 * R.i + e, cj = 2 * R.j + n;
        const int64_t off = (int64_t)q * a.out_cap + glo[q];
        if (finest) {
            if (!a.cells) {
                atomicOr(a.error, kErrInternal);
                continue;
            }
            Cell c;
            c.i = ci_;
            c.j = cj;
            c.votes = (int32_t)votes[q];
            c.pass = pass;
            c.key = key_of(ci_, cj, lc);
            c.member_off = a.keep_members ? off : -1;
            a.cells[ci++] = c;
        } else {
            if (!a.next_regions) {
                atomicOr(a.error, kErrInternal);
                continue;
            }
            Region C;
            C.start = start;
            C.off = off;
            C.i = ci_;
            C.j = cj;
            C.len = (int32_t)votes[q];
            C.tree = tree;
            a.next_regions[ri] = C;
            // next-level tiles whose first entry falls inside this region
            for (int64_t t = (start + kTile - 1) / kTile; t * kTile < start + votes[q]; ++t)
                if (t < a.next_tile_cap) a.next_tile_first[t] = (int32_t)ri;
            ++ri;
            start += votes[q];
        }
    }
}

// Edge staging: nonzero pixels of a row-major binary image, in row-major
// order, by a stable compaction (look-back over tiles of kPixTile pixels).
__global__ __launch_bounds__(kBlock) void k_extract(ExtractArgs a)
{
    __shared__ int64_t s_wtot[kWaves];
    __shared__ int64_t s_excl;
    __shared__ int32_t s_tile;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if (tid == 0) s_tile = (int32_t)atomicAdd(a.ticket, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t p0 = tile * kPixTile + (int64_t)tid * kPixPerThread;
    int32_t row = 0, col = 0;
    uint32_t bits = 0;
    if (p0 < a.n_pix) {
        row = (int32_t)(p0 / a.width);
        col = (int32_t)(p0 - (int64_t)row * a.width);
        int32_t r = row, c = col;
        for (int k = 0; k < kPixPerThread && p0 + k < a.n_pix; ++k) {
            if (a.image[(int64_t)r * a.row_stride + c]) bits |= 1u << k;
            if (++c == a.width) { c = 0; ++r; }
        }
    }
    const int64_t cnt = __popc(bits);
    const int64_t incl = wave_incl_scan(cnt, lane);
    if (lane == kWave - 1) s_wtot[wave] = incl;
    __syncthreads();
    if (tid == 0) {
        int64_t agg = 0;
        for (int w = 0; w < kWaves; ++w) agg += s_wtot[w];
        const int64_t excl = lookback(a.status, tile, 1, 0, agg, a.error);
        s_excl = excl;
        if (tile == a.n_tiles - 1) *a.total = excl + agg;
    }
    __syncthreads();
    int64_t pos = s_excl + incl - cnt;
    for (int w = 0; w < wave; ++w) pos += s_wtot[w];
    int32_t r = row, c = col;
    for (int k = 0; k < kPixPerThread; ++k) {
        if ((bits >> k) & 1u) {
            a.x[pos] = c;
            a.y[pos] = r;
            ++pos;
        }
        if (++c == a.width) { c = 0; ++r; }
    }
}

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t value)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = value;
}

__global__ void k_init_level0(Region* regions, int32_t* tile_first, int32_t* iota, int32_t n_trees,
                              int64_t n_points, int32_t n_tiles)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_points; k += stride)
        iota[k] = (int32_t)k;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_tiles; k += stride)
        tile_first[k] = (int32_t)((k * kTile) / n_points);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_trees; k += stride) {
        Region R;
        R.start = k * n_points;
        R.off = 0;
        R.i = 0;
        R.j = 0;
        R.len = (int32_t)n_points;
        R.tree = (int32_t)k;
        regions[k] = R;
    }
}

__global__ void k_validate(const int32_t* x, const int32_t* y, int64_t n, int32_t W, int32_t H,
                           uint32_t* error)
{
    bool bad = false;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        bad |= (x[k] < 0) | (x[k] >= W) | (y[k] < 0) | (y[k] >= H);
    if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(error, kErrPointRange);
}

// one wavefront per cell copies its voters to their compact position
__global__ void k_gather_members(const Cell* cells, int64_t n_cells, const int64_t* dst_off,
                                 const int32_t* src, int32_t* dst)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t c = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; c < n_cells;
         c += waves) {
        const Cell cell = cells[c];
        const int32_t* s = src + cell.member_off;
        int32_t* d = dst + dst_off[c];
        for (int32_t k = lane; k < cell.votes; k += kWave) d[k] = s[k];
    }
}

int grid_for(int64_t n, int per_block)
{
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

}  // namespace

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t value, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_u64<<<grid_for(n, kBlock), kBlock, 0, s>>>(p, n, value);
    return hipGetLastError();
}

hipError_t launch_init_level0(Region* regions, int32_t* tile_first, int32_t* iota, int32_t n_trees,
                              int64_t n_points, int32_t n_tiles, hipStream_t s)
{
    const int64_t n = n_points > n_tiles ? n_points : n_tiles;
    k_init_level0<<<grid_for(n, kBlock), kBlock, 0, s>>>(regions, tile_first, iota, n_trees, n_points,
                                                          n_tiles);
    return hipGetLastError();
}

hipError_t launch_vote(const VoteArgs& a, int variant, bool wide, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    if (variant == 1)
        k_vote<1, int64_t><<<a.n_tiles, kBlock, 0, s>>>(a);
    else if (wide)
        k_vote<0, int64_t><<<a.n_tiles, kBlock, 0, s>>>(a);
    else
        k_vote<0, int32_t><<<a.n_tiles, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_decide(const DecideArgs& a, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    k_decide<<<a.n_tiles, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_extract(const ExtractArgs& a, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    k_extract<<<a.n_tiles, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_validate(const int32_t* x, const int32_t* y, int64_t n, int32_t W, int32_t H,
                           uint32_t* error, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_validate<<<grid_for(n, kBlock), kBlock, 0, s>>>(x, y, n, W, H, error);
    return hipGetLastError();
}

hipError_t launch_gather_members(const Cell* cells, int64_t n_cells, const int64_t* dst_off,
                                 const int32_t* src, int32_t* dst, hipStream_t s)
{
    if (n_cells <= 0) return hipSuccess;
    k_gather_members<<<grid_for(n_cells, kWaves), kBlock, 0, s>>>(cells, n_cells, dst_off, src, dst);
    return hipGetLastError();
}

}  // namespace hh
