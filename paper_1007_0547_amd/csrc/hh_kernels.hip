// gfx950 kernels of the hierarchical slope-intercept Hough vote
// (Singh and Bhatia, arXiv:1007.0547).
//
// Level-synchronous form of the paper's depth-first search (Sec. 3): all
// regions that split at level l (of every tree = pass of an image) are
// processed together.  Their voter lists are stored back to back; a flat
// entry index e in [0, L_l) walks all (parent region, line) pairs.  A list
// entry carries the line itself (the packed edge point, or the point id and
// the packed point), so no launch gathers coordinates.
//
//   k_vote   one read of every (parent, line) entry: the 4-bit corner codes
//            of the line for the four children (Sec. 2, getcode()) and the
//            vote rule (code not 0000 / 1111, steps 5 and 12.v), evaluated as
//            wavefront lane masks; a stable compaction of the voting lines
//            into each child's list at a position fixed by the parent alone
//            (child q of a parent with flat start s and length n starts at
//            4 s + q n), so workgroups never wait on each other: a tile whose
//            first parent began in an earlier tile recounts that prefix
//            itself.  The tile holding a parent's last entry records the
//            child votes and the parent's split decisions (step 13).
//   k_scan   one workgroup: exclusive prefix of the per-tile decision totals.
//   k_emit   per parent: the level-(l+1) region table in quad order (so key
//            order is kept), or the detected cells at the finest level.
//
// Level sizes never travel to the host: each launch reads them from the
// arena's LevelInfo records written by the launches before it, and walks its
// tiles with a fixed grid.  No launch uses atomics or waits on another
// workgroup.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "hh_kernels.hpp"

namespace hh {
namespace {

// Pointers reached through argument structs are generic; the kernels access
// device memory through these casts so the compiler emits global (not flat)
// loads, stores and atomics.
template <typename T>
__device__ inline T* G(T* p)
{
    return (T*)(__attribute__((address_space(1))) T*)p;
}

__device__ inline bool stopped(uint32_t* error)
{
    return (__hip_atomic_load(G(error), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrStop) != 0;
}

__device__ inline void raise_error(uint32_t* error, uint32_t bits)
{
    __hip_atomic_fetch_or(G(error), bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint32_t lanes_below(uint64_t b)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
}

template <typename Entry> struct EntryOps;
template <> struct EntryOps<uint32_t> {   // the packed edge point
    __device__ static uint32_t point(uint32_t e) { return e; }
    __device__ static uint32_t root(const uint32_t* pts, int64_t k) { return pts[k]; }
};
template <> struct EntryOps<uint64_t> {   // point id << 32 | packed edge point
    __device__ static uint32_t point(uint64_t e) { return (uint32_t)e; }
    __device__ static uint64_t root(const uint32_t* pts, int64_t k) { return ((uint64_t)k << 32) | pts[k]; }
};

// The lines of a wavefront against the four children of each lane's parent
// (pi, pj), children at level lc: cm[q] holds one bit per lane, set when the
// lane's line votes for child q (q = 0 NE, 1 NW, 2 SW, 3 SE).
//
// Code variant (Sec. 2).  The children's corners form the parent's 3x3
// corner grid at level lc: columns ic = 2 pi + c and rows jc = 2 pj + r,
// c, r in {0, 1, 2}, at m = M_c / 2^lc and b = B_r / 2^lc with
// M_c = 2 ic - 2^lc and B_r = -S 2^lc + 3 S jc.  Corner (c, r) is below the
// line b = v - u m iff B_r < t_c with t_c = v 2^lc - u M_c (a corner on the
// line is above); consecutive columns differ by 2 in M, so
// t_{c+1} = t_c - 2u.  The nine compares become nine lane masks b_cr, and a
// child's code (NE, NW, SW, SE corner bits) votes iff it is neither 0000 nor
// 1111: some corner below and not all of them.
template <typename CT>
__device__ inline void code_masks(bool valid, int32_t u, int32_t v, int32_t pi, int32_t pj, int lc, int s_log2,
                                  uint64_t (&cm)[4])
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
    const uint64_t b00 = __ballot(valid && B0 < t0), b01 = __ballot(valid && B1 < t0),
                   b02 = __ballot(valid && B2 < t0);
    const uint64_t b10 = __ballot(valid && B0 < t1), b11 = __ballot(valid && B1 < t1),
                   b12 = __ballot(valid && B2 < t1);
    const uint64_t b20 = __ballot(valid && B0 < t2), b21 = __ballot(valid && B1 < t2),
                   b22 = __ballot(valid && B2 < t2);
    // child at (east e, north n): NE = (e+1, n+1), NW = (e, n+1), SW = (e, n), SE = (e+1, n)
    cm[0] = (b22 | b12 | b11 | b21) & ~(b22 & b12 & b11 & b21);   // NE child, e = 1, n = 1
    cm[1] = (b12 | b02 | b01 | b11) & ~(b12 & b02 & b01 & b11);   // NW child, e = 0, n = 1
    cm[2] = (b11 | b01 | b00 | b10) & ~(b11 & b01 & b00 & b10);   // SW child, e = 0, n = 0
    cm[3] = (b21 | b11 | b10 | b20) & ~(b21 & b11 & b10 & b20);   // SE child, e = 1, n = 0
}

// Circumscribed-circle variant (comparison method of the paper's ref. [9]).
// For child (lc, i, j) with centre m = -1 + (2i+1)/2^lc,
// b = -S + 3S(2j+1)/2^(lc+1), in units where the cell is a unit square, the
// line is within the circumradius iff D^2 <= 2 (9 S^2 + 4 u^2) with
// D = 3S(2j+1) + 2u(2i+1) - (v + u + S) 2^(lc+1).
__device__ inline void circle_masks(bool valid, int32_t u, int32_t v, int32_t pi, int32_t pj, int lc,
                                    int s_log2, uint64_t (&cm)[4])
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
    cm[0] = __ballot(valid && dNE * dNE <= rhs);
    cm[1] = __ballot(valid && dNW * dNW <= rhs);
    cm[2] = __ballot(valid && dSW * dSW <= rhs);
    cm[3] = __ballot(valid && dSE * dSE <= rhs);
}

template <int kVariant, typename CT>
__device__ inline void child_masks(bool valid, uint32_t point, uint32_t meta, uint32_t ij, int lc,
                                   uint64_t (&cm)[4])
{
    const int32_t x = (int32_t)(point & 0xFFFFu), y = (int32_t)(point >> 16);
    const bool swap = meta & kMetaPass;   // pass 1 reads (x0, y0) as (y0, x0)
    const int32_t u = swap ? y : x, v = swap ? x : y;
    const int s_log2 = (int)((meta >> kMetaSlogShift) & 15u);
    const int32_t pi = (int32_t)(ij & 0xFFFFu), pj = (int32_t)(ij >> 16);
    if constexpr (kVariant == 0)
        code_masks<CT>(valid, u, v, pi, pj, lc, s_log2, cm);
    else
        circle_masks(valid, u, v, pi, pj, lc, s_log2, cm);
}

__device__ inline LevelLayout layout_of(const Arena& ar, int l)
{
    const int64_t Pp = l ? ar.info[l - 1].P : 0, Lp = l ? ar.info[l - 1].L : 0;
    return level_layout(ar.half[l & 1], l, Pp, Lp, ar.info[l].P, ar.info[l].L, ar.n_trees, ar.entry_bytes);
}

__device__ inline int32_t wave_incl_scan32(int32_t x, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ inline int64_t wave_incl_scan64(int64_t x, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// LDS of one vote tile.
struct VoteLds {
    uint16_t rel[kTile + 1];       // region starts relative to the tile (0: at or before it)
    uint16_t roff[kTile + 1][4];   // tile prefix of each child slot at the region's first entry
    int64_t inb[kStage];           // staged region data (tiles with at most kStage regions)
    int64_t obase[kStage];         //   4 * start
    int32_t len[kStage];
    uint32_t ij[kStage];
    uint32_t meta[kStage];
    int32_t tree[kStage];
    int32_t cnt[kWaves][4];
    int32_t dec[kWaves][kDecCh];
};

// Region fields of the tile's regions: from LDS when every region of the tile
// is staged, otherwise from the region table.
template <bool kStaged>
struct RegionView {
    const VoteLds& S;
    const Region* regions;
    int r0;
    __device__ int64_t inb(int i) const { if constexpr (kStaged) return S.inb[i]; else return regions[r0 + i].in_base; }
    __device__ int64_t obase(int i) const { if constexpr (kStaged) return S.obase[i]; else return 4 * regions[r0 + i].start; }
    __device__ int32_t len(int i) const { if constexpr (kStaged) return S.len[i]; else return regions[r0 + i].len; }
    __device__ uint32_t ij(int i) const { if constexpr (kStaged) return S.ij[i]; else return regions[r0 + i].ij; }
    __device__ uint32_t meta(int i) const { if constexpr (kStaged) return S.meta[i]; else return regions[r0 + i].meta; }
    __device__ int32_t tree(int i) const { if constexpr (kStaged) return S.tree[i]; else return regions[r0 + i].tree; }
};

struct VoteTile {
    int64_t tile, t0, t_end, L;
    int r0, nr, lc;
    bool before;            // the first region began in an earlier tile
    int32_t carry[4];       // its votes per child slot before this tile
};

// The entries of one tile: region, line, child masks, block prefix, stable
// compaction into the children's lists, and the parents that end here.
template <typename Entry, int kVariant, typename CT, bool kStaged>
__device__ __forceinline__ void vote_tile(const LevelArgs& a, const LevelLayout& lay, VoteLds& S,
                                          const Entry* list, Entry* out, const Region* regions,
                                          const uint32_t* pts, const TreeDesc* trees, const VoteTile& t)
{
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const RegionView<kStaged> rv{S, regions, t.r0};
    const int64_t wb = t.t0 + (int64_t)wave * kWaveSpan;

    // region of every entry (binary search over the region starts)
    uint32_t ridx[kEpt];
    uint32_t valid = 0;
    {
        int lo_prev = 0;
#pragma unroll
        for (int k = 0; k < kEpt; ++k) {
            const int64_t e = wb + k * kWave + lane;
            ridx[k] = 0;
            if (e < t.t_end) {
                const int rel = (int)(e - t.t0);
                int lo = lo_prev, hi = t.nr - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if ((int)S.rel[mid] <= rel) lo = mid; else hi = mid - 1;
                }
                lo_prev = lo;
                ridx[k] = (uint32_t)lo;
                valid |= 1u << k;
            }
        }
    }
    // the lines, all loads issued before any use
    Entry ent[kEpt];
#pragma unroll
    for (int k = 0; k < kEpt; ++k) {
        ent[k] = 0;
        if ((valid >> k) & 1u) {
            const int64_t i = rv.inb((int)ridx[k]) + wb + k * kWave + lane;
            ent[k] = list ? list[i] : EntryOps<Entry>::root(pts, i);
        }
    }
    // child masks and per-wave counts
    uint32_t bits = 0;   // 4 child bits per entry, entry k at bits 4k .. 4k+3
    int32_t cnt[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kEpt; ++k) {
        const int idx = (int)ridx[k];
        uint64_t cm[4];
        child_masks<kVariant, CT>((valid >> k) & 1u, EntryOps<Entry>::point(ent[k]), rv.meta(idx), rv.ij(idx),
                                  t.lc, cm);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            cnt[q] += (int32_t)__popcll(cm[q]);
            bits |= (uint32_t)((cm[q] >> lane) & 1u) << (4 * k + q);
        }
        // keep the rounds apart: their lane masks live in scalar registers
        __builtin_amdgcn_sched_barrier(0);
    }
    if (lane == 0)
        for (int q = 0; q < 4; ++q) S.cnt[wave][q] = cnt[q];
    __syncthreads();
    int32_t base[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        base[q] = 0;
        for (int w = 0; w < wave; ++w) base[q] += S.cnt[w][q];
    }
    // tile prefix of each child slot at the first entry of each region that starts here
    {
        int32_t run[4] = {base[0], base[1], base[2], base[3]};
#pragma unroll
        for (int k = 0; k < kEpt; ++k) {
            const int idx = (int)ridx[k];
            const int64_t e = wb + k * kWave + lane;
            const bool first = ((valid >> k) & 1u) && (int)(e - t.t0) == (int)S.rel[idx] && !(idx == 0 && t.before);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint64_t m = __ballot((bits >> (4 * k + q)) & 1u);
                if (first) S.roff[idx][q] = (uint16_t)(run[q] + (int32_t)lanes_below(m));
                run[q] += (int32_t)__popcll(m);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    __syncthreads();

    // stable compaction into each child's list; the entry that closes a region
    // records the child votes and the region's split decisions
    int32_t run[4] = {base[0], base[1], base[2], base[3]};
    int32_t dec_run[kDecCh] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kEpt; ++k) {
        const int64_t e = wb + k * kWave + lane;
        const bool ok = (valid >> k) & 1u;
        const int idx = (int)ridx[k];
        const int64_t obase = ok ? rv.obase(idx) : 0;
        const int32_t len = ok ? rv.len(idx) : 0;
        const bool carried = idx == 0 && t.before;
        int32_t votes[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t bit = (bits >> (4 * k + q)) & 1u;
            const uint64_t m = __ballot(bit);
            const int32_t X = run[q] + (int32_t)lanes_below(m);
            const int32_t rank = carried ? X + t.carry[q] : X - (int32_t)S.roff[idx][q];
            if (bit && a.write_out) out[obase + (int64_t)q * len + rank] = ent[k];
            votes[q] = rank + (int32_t)bit;   // votes of child q up to and including e
            run[q] += (int32_t)__popcll(m);
        }
        const bool last =
            ok && ((idx + 1 < t.nr) ? ((int)S.rel[idx + 1] == (int)(e - t.t0) + 1) : (e + 1 == t.L));
        if (__ballot(last)) {
            int32_t dv[kDecCh] = {0, 0, 0, 0};
            if (last) {
                const int64_t p = t.r0 + idx;
                const int32_t thr = trees[rv.tree(idx)].threshold;
                const bool finest = rv.meta(idx) & kMetaChildFinest;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    G(lay.cv)[p * 4 + q] = votes[q];
                    dv[3] += votes[q];
                    if (votes[q] > thr) {
                        if (finest) dv[2] += 1;
                        else {
                            dv[0] += 1;
                            dv[1] += votes[q];
                        }
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < kDecCh; ++c) {
                const int32_t incl = wave_incl_scan32(dv[c], lane);
                if (last) G(lay.dvw)[(int64_t)(t.r0 + idx) * kDecCh + c] = dec_run[c] + incl - dv[c];
                dec_run[c] += __shfl(incl, kWave - 1, kWave);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (lane == 0)
        for (int c = 0; c < kDecCh; ++c) S.dec[wave][c] = dec_run[c];
    __syncthreads();
    if (tid < kWaves * kDecCh) {
        const int w = tid / kDecCh, c = tid % kDecCh;
        int32_t pre = 0;
        for (int v = 0; v < w; ++v) pre += S.dec[v][c];
        G(lay.wpre)[(t.tile * kWaves + w) * kDecCh + c] = pre;
        if (w == kWaves - 1) G(lay.vts)[t.tile * kDecCh + c] = pre + S.dec[w][c];
    }
}

template <typename Entry, int kVariant, typename CT>
__global__ __launch_bounds__(kBlock) void k_vote(LevelArgs a)
{
    __shared__ VoteLds S;
    const Arena& ar = a.ar;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if (stopped(ar.error)) return;
    const int l = a.level;
    const int64_t P = ar.info[l].P, L = ar.info[l].L;
    if (P == 0) return;
    const LevelLayout lay = layout_of(ar, l);
    if (lay.end > ar.half_cap) {
        if (tid == 0 && blockIdx.x == 0) raise_error(ar.error, kErrArena);
        return;
    }
    const Entry* const list = G(l ? static_cast<const Entry*>(layout_of(ar, l - 1).out) : nullptr);
    Entry* const out = G(static_cast<Entry*>(lay.out));
    const Region* const regions = G(static_cast<const Region*>(lay.regions));
    const int32_t* tile_first = G(static_cast<const int32_t*>(lay.tile_first));
    const uint32_t* const pts = G(a.xy);
    const TreeDesc* const trees = G(a.trees);
    const int64_t n_tiles = cdiv(L, kTile);

    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        VoteTile t;
        t.tile = tile;
        t.t0 = tile * kTile;
        t.t_end = std::min<int64_t>(t.t0 + kTile, L);
        t.L = L;
        t.lc = l + 1;
        t.r0 = tile_first[tile];
        const int r1 = (tile + 1 < n_tiles) ? tile_first[tile + 1] : (int)(P - 1);
        t.nr = r1 - t.r0 + 1;   // <= kTile + 1: every region holds at least one entry
        if (t.r0 < 0 || r1 >= P || t.nr < 1 || t.nr > kTile + 1) {
            if (tid == 0) raise_error(ar.error, kErrInternal);
            continue;
        }
        __syncthreads();   // LDS of the previous tile is free
        for (int k = tid; k < t.nr; k += kBlock) {
            const Region R = regions[t.r0 + k];
            const int64_t rel = R.start - t.t0;
            S.rel[k] = (uint16_t)(rel <= 0 ? 0 : (rel > kTile ? kTile : rel));
            if (k < kStage) {
                S.inb[k] = R.in_base;
                S.obase[k] = 4 * R.start;
                S.len[k] = R.len;
                S.ij[k] = R.ij;
                S.meta[k] = R.meta;
                S.tree[k] = R.tree;
            }
        }
        const int64_t start0 = regions[t.r0].start;
        t.before = start0 < t.t0;
        __syncthreads();

        // lines of the first region before this tile: their child-slot counts
        for (int q = 0; q < 4; ++q) t.carry[q] = 0;
        if (t.before) {
            const int64_t inb = S.inb[0];
            const uint32_t ij = S.ij[0], meta = S.meta[0];
            int32_t c[4] = {0, 0, 0, 0};
            for (int64_t b = start0; b < t.t0; b += kTile) {
                Entry ent[kEpt];
#pragma unroll
                for (int k = 0; k < kEpt; ++k) {
                    const int64_t e = b + k * kBlock + tid;
                    ent[k] = 0;
                    if (e < t.t0) ent[k] = list ? list[inb + e] : EntryOps<Entry>::root(pts, inb + e);
                }
#pragma unroll
                for (int k = 0; k < kEpt; ++k) {
                    const int64_t e = b + k * kBlock + tid;
                    uint64_t cm[4];
                    child_masks<kVariant, CT>(e < t.t0, EntryOps<Entry>::point(ent[k]), meta, ij, t.lc, cm);
#pragma unroll
                    for (int q = 0; q < 4; ++q) c[q] += (int32_t)__popcll(cm[q]);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            if (lane == 0)
                for (int q = 0; q < 4; ++q) S.cnt[wave][q] = c[q];
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 4; ++q)
                for (int w = 0; w < kWaves; ++w) t.carry[q] += S.cnt[w][q];
            __syncthreads();
        }
        if (t.nr <= kStage)
            vote_tile<Entry, kVariant, CT, true>(a, lay, S, list, out, regions, pts, trees, t);
        else
            vote_tile<Entry, kVariant, CT, false>(a, lay, S, list, out, regions, pts, trees, t);
    }
}

// One workgroup: exclusive prefix of the per-tile decision totals of level l
// and the sizes of level l+1.
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void k_scan(LevelArgs a)
{
    __shared__ int64_t s_w[kScanThreads / kWave][kDecCh];
    const Arena& ar = a.ar;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if (stopped(ar.error)) return;
    const int l = a.level;
    const int lc = l + 1;
    const int64_t P = ar.info[l].P, L = ar.info[l].L;
    const int64_t cells_base = ar.info[l].cells_base + ar.info[l].cells;
    if (P == 0) {
        if (tid == 0) {
            LevelInfo& nx = ar.info[lc];
            nx.P = 0;
            nx.L = 0;
            nx.cells = 0;
            nx.cells_base = cells_base;
        }
        return;
    }
    const LevelLayout lay = layout_of(ar, l);
    const int64_t nt = cdiv(L, kTile);
    const int64_t chunk = cdiv(nt, kScanThreads);
    const int64_t b = std::min<int64_t>(nt, tid * chunk), e = std::min<int64_t>(nt, b + chunk);
    int64_t sum[kDecCh] = {0, 0, 0, 0};
    for (int64_t t = b; t < e; ++t)
#pragma unroll
        for (int c = 0; c < kDecCh; ++c) sum[c] += G(lay.vts)[t * kDecCh + c];
    int64_t incl[kDecCh];
#pragma unroll
    for (int c = 0; c < kDecCh; ++c) {
        incl[c] = wave_incl_scan64(sum[c], lane);
        if (lane == kWave - 1) s_w[wave][c] = incl[c];
    }
    __syncthreads();
    int64_t run[kDecCh];
#pragma unroll
    for (int c = 0; c < kDecCh; ++c) {
        run[c] = incl[c] - sum[c];
        for (int w = 0; w < wave; ++w) run[c] += s_w[w][c];
    }
    for (int64_t t = b; t < e; ++t)
#pragma unroll
        for (int c = 0; c < kDecCh; ++c) {
            G(lay.vtp)[t * kDecCh + c] = run[c];
            run[c] += G(lay.vts)[t * kDecCh + c];
        }
    if (tid == kScanThreads - 1) {
        LevelInfo& nx = ar.info[lc];
        nx.P = run[0];
        nx.L = run[1];
        nx.cells = run[2];
        nx.cells_base = cells_base;
        ar.info[l].votes = run[3];
    }
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

__global__ __launch_bounds__(kBlock) void k_emit(LevelArgs a)
{
    const Arena& ar = a.ar;
    if (stopped(ar.error)) return;
    const int l = a.level;
    const int lc = l + 1;
    const int64_t P = ar.info[l].P, L = ar.info[l].L;
    if (P == 0) return;
    const LevelLayout lay = layout_of(ar, l);
    const LevelLayout nxt = level_layout(ar.half[lc & 1], lc, P, L, 0, 0, ar.n_trees, ar.entry_bytes);
    if (nxt.end > ar.half_cap) {
        if (threadIdx.x == 0 && blockIdx.x == 0) raise_error(ar.error, kErrArena);
        return;
    }
    const int64_t cells_base = ar.info[lc].cells_base;
    for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < P; p += (int64_t)gridDim.x * kBlock) {
        const Region R = G(lay.regions)[p];
        const int64_t le = R.start + R.len - 1;   // the region's last entry
        const int64_t tile = le / kTile;
        const int64_t w = (le - tile * kTile) / kWaveSpan;
        int64_t pre[kDecCh];
#pragma unroll
        for (int c = 0; c < kDecCh; ++c)
            pre[c] = G(lay.vtp)[tile * kDecCh + c] + G(lay.wpre)[(tile * kWaves + w) * kDecCh + c] +
                     G(lay.dvw)[p * kDecCh + c];
        int32_t cv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) cv[q] = G(lay.cv)[p * 4 + q];
        const TreeDesc T = G(a.trees)[R.tree];
        const bool finest = R.meta & kMetaChildFinest;
        const int32_t pi = (int32_t)(R.ij & 0xFFFFu), pj = (int32_t)(R.ij >> 16);
        int64_t ri = pre[0], start = pre[1], ci = cells_base + pre[2];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (cv[q] <= T.threshold) continue;
            const int32_t e = (q == 0 || q == 3) ? 1 : 0;
            const int32_t n = (q <= 1) ? 1 : 0;
            const int32_t ci_ = 2 * pi + e, cj = 2 * pj + n;
            const int64_t off = 4 * R.start + (int64_t)q * R.len;   // the child's list in this level's output
            if (finest) {
                if (ci >= ar.cells_cap) {
                    raise_error(ar.error, kErrArena);
                    continue;
                }
                Cell c;
                c.i = ci_;
                c.j = cj;
                c.votes = cv[q];
                c.pass = T.pass;
                c.key = key_of(ci_, cj, lc);
                c.member_off = a.keep_members ? off : -1;
                G(ar.cells)[ci++] = c;
            } else {
                if (ri >= nxt.regions_cap) {
                    raise_error(ar.error, kErrInternal);
                    continue;
                }
                Region C;
                C.start = start;
                C.in_base = off - start;
                C.ij = (uint32_t)ci_ | ((uint32_t)cj << 16);
                C.len = cv[q];
                C.tree = R.tree;
                C.meta = (R.meta & ~kMetaChildFinest) | (lc + 1 == T.dmax ? kMetaChildFinest : 0u);
                G(nxt.regions)[ri] = C;
                // next-level tiles whose first entry falls inside this region
                for (int64_t t = cdiv(start, kTile); t * kTile < start + cv[q]; ++t)
                    if (t < nxt.tile_cap) G(nxt.tile_first)[t] = (int32_t)ri;
                ++ri;
                start += cv[q];
            }
        }
        // the first parent of each tree records where its tree's sums begin
        if (p == 0 || G(lay.regions)[p - 1].tree != R.tree) {
            int64_t* r = G(ar.rec + ((int64_t)R.tree * kMaxLevels + l) * kRecCh);
            r[0] = p;
            r[1] = R.start;
            r[2] = pre[0];
            r[3] = pre[1];
            r[4] = pre[2];
            r[5] = pre[3];
        }
    }
}

// Edge staging: nonzero pixels of a row-major binary image in row-major order.
__device__ inline uint32_t pixel_bits(const ExtractArgs& a, int64_t p0, int32_t& row, int32_t& col)
{
    uint32_t bits = 0;
    row = 0;
    col = 0;
    if (p0 < a.n_pix) {
        row = (int32_t)(p0 / a.width);
        col = (int32_t)(p0 - (int64_t)row * a.width);
        int32_t r = row, c = col;
        for (int k = 0; k < kPixPerThread && p0 + k < a.n_pix; ++k) {
            if (a.image[(int64_t)r * a.row_stride + c]) bits |= 1u << k;
            if (++c == a.width) {
                c = 0;
                ++r;
            }
        }
    }
    return bits;
}

__device__ inline int32_t block_excl_scan32(int32_t x, int32_t* s_w, int32_t& total)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int32_t incl = wave_incl_scan32(x, lane);
    if (lane == kWave - 1) s_w[wave] = incl;
    __syncthreads();
    int32_t pre = 0;
    total = 0;
    for (int w = 0; w < kWaves; ++w) {
        if (w < wave) pre += s_w[w];
        total += s_w[w];
    }
    return pre + incl - x;
}

__global__ __launch_bounds__(kBlock) void k_extract_count(ExtractArgs a)
{
    __shared__ int32_t s_w[kWaves];
    for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        int32_t row, col;
        const uint32_t bits = pixel_bits(a, tile * kPixTile + (int64_t)threadIdx.x * kPixPerThread, row, col);
        int32_t total;
        __syncthreads();
        block_excl_scan32(__popc(bits), s_w, total);
        if (threadIdx.x == 0) a.tile_count[tile] = total;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_counts(const int32_t* cnt, int64_t n, int64_t* pre,
                                                              int64_t* total)
{
    __shared__ int64_t s_w[kScanThreads / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t chunk = cdiv(n, kScanThreads);
    const int64_t b = std::min<int64_t>(n, tid * chunk), e = std::min<int64_t>(n, b + chunk);
    int64_t sum = 0;
    for (int64_t t = b; t < e; ++t) sum += cnt[t];
    const int64_t incl = wave_incl_scan64(sum, lane);
    if (lane == kWave - 1) s_w[wave] = incl;
    __syncthreads();
    int64_t run = incl - sum;
    for (int w = 0; w < wave; ++w) run += s_w[w];
    for (int64_t t = b; t < e; ++t) {
        pre[t] = run;
        run += cnt[t];
    }
    if (tid == kScanThreads - 1) *total = run;
}

__global__ __launch_bounds__(kBlock) void k_extract_write(ExtractArgs a)
{
    __shared__ int32_t s_w[kWaves];
    for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        int32_t row, col;
        const uint32_t bits = pixel_bits(a, tile * kPixTile + (int64_t)threadIdx.x * kPixPerThread, row, col);
        int32_t total;
        __syncthreads();
        int64_t pos = a.tile_pre[tile] + block_excl_scan32(__popc(bits), s_w, total);
        int32_t r = row, c = col;
        for (int k = 0; k < kPixPerThread; ++k) {
            if ((bits >> k) & 1u) a.xy[pos++] = pack_xy(c, r);
            if (++c == a.width) {
                c = 0;
                ++r;
            }
        }
    }
}

__global__ void k_clear(Arena ar, int64_t n_rec)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t info_words = (int64_t)(kMaxLevels + 1) * (int64_t)sizeof(LevelInfo) / 8;
    for (int64_t k = g; k < info_words; k += stride) reinterpret_cast<int64_t*>(ar.info)[k] = 0;
    for (int64_t k = g; k < n_rec; k += stride) ar.rec[k] = -1;
    for (int64_t k = g; k < 8; k += stride) ar.scalar[k] = 0;
    if (g == 0) *ar.error = 0;
}

__global__ void k_pack_points(const int32_t* x, const int32_t* y, int64_t n, int32_t W, int32_t H,
                              uint32_t* xy, uint32_t* error)
{
    bool bad = false;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t xk = x[k], yk = y[k];
        const bool outside = (xk < 0) | (xk >= W) | (yk < 0) | (yk >= H);
        bad |= outside;
        xy[k] = outside ? 0u : pack_xy(xk, yk);
    }
    if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) raise_error(error, kErrPointRange | kErrInternal);
}

__global__ void k_begin(Arena ar, TreeDesc* trees, int32_t n_trees, int64_t n_points, int32_t threshold,
                        int32_t dmax)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t E = n_points >= 0 ? n_points : ar.scalar[0];
    const int64_t P0 = (E > threshold && dmax > 0) ? n_trees : 0;
    const int64_t L0 = P0 * E;
    if (g == 0) {
        LevelInfo& in = ar.info[0];
        in.P = P0;
        in.L = L0;
        in.votes = 0;
        in.cells = 0;
        in.cells_base = 0;
        if (n_points >= 0) ar.scalar[0] = E;
    }
    if (g < n_trees) trees[g].n_points = E;
    if (P0 == 0) return;
    const LevelLayout lay = level_layout(ar.half[0], 0, 0, 0, P0, L0, n_trees, ar.entry_bytes);
    if (lay.end > ar.half_cap) {
        if (g == 0) raise_error(ar.error, kErrArena);
        return;
    }
    for (int64_t t = g; t < P0; t += stride) {
        const TreeDesc T = trees[t];
        Region R;
        R.start = t * E;
        R.in_base = T.xy_base - t * E;   // root lists are the point array itself
        R.ij = 0;
        R.len = (int32_t)E;
        R.tree = (int32_t)t;
        R.meta = (T.pass ? kMetaPass : 0u) | ((uint32_t)T.s_log2 << kMetaSlogShift) |
                 (T.dmax == 1 ? kMetaChildFinest : 0u);
        lay.regions[t] = R;
    }
    for (int64_t k = g; k < cdiv(L0, kTile); k += stride) lay.tile_first[k] = (int32_t)((k * kTile) / E);
}

// Point ids of the voters of detected cells, one wavefront per cell.  A
// packed-point entry's id is its position in the row-major point array xy
// (binary search); an (id, point) entry carries it.  dst_off == nullptr keeps
// the layout of the entry buffer; otherwise cell c goes to dst_off[c].
__device__ inline int32_t entry_id(uint32_t v, const uint32_t* xy, int64_t n_points)
{
    int64_t lo = 0, hi = n_points;   // first position with xy[pos] >= v
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (xy[mid] < v) lo = mid + 1; else hi = mid;
    }
    return (int32_t)lo;
}

__device__ inline int32_t entry_id(uint64_t v, const uint32_t*, int64_t) { return (int32_t)(v >> 32); }

template <typename Entry>
__global__ void k_member_ids(const Cell* cells, int64_t n_cells, const int64_t* dst_off, const Entry* src,
                             const uint32_t* xy, int64_t n_points, int32_t* dst)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t c = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; c < n_cells;
         c += waves) {
        const Cell cell = cells[c];
        const Entry* s = src + cell.member_off;
        int32_t* d = dst + (dst_off ? dst_off[c] : cell.member_off);
        for (int32_t k = lane; k < cell.votes; k += kWave) d[k] = entry_id(s[k], xy, n_points);
    }
}

__global__ void k_iota(int32_t* dst, int64_t n)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = (int32_t)k;
}

int grid_for(int64_t n, int per_block, int max_grid = 4096)
{
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > max_grid) g = max_grid;
    return (int)g;
}

}  // namespace

hipError_t launch_clear(const Arena& ar, int64_t n_rec, hipStream_t s)
{
    k_clear<<<grid_for(std::max<int64_t>(n_rec, 256), kBlock, 1024), kBlock, 0, s>>>(ar, n_rec);
    return hipGetLastError();
}

hipError_t launch_pack_points(const int32_t* x, const int32_t* y, int64_t n, int32_t W, int32_t H,
                              uint32_t* xy, uint32_t* error, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_pack_points<<<grid_for(n, kBlock), kBlock, 0, s>>>(x, y, n, W, H, xy, error);
    return hipGetLastError();
}

hipError_t launch_extract(const ExtractArgs& a, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(a.n_tiles, 2048);
    k_extract_count<<<grid, kBlock, 0, s>>>(a);
    k_scan_counts<<<1, kScanThreads, 0, s>>>(a.tile_count, a.n_tiles, a.tile_pre, a.total);
    k_extract_write<<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_begin(const Arena& ar, TreeDesc* trees, int32_t n_trees, int64_t n_points, int32_t threshold,
                        int32_t dmax, int64_t work_bound, hipStream_t s)
{
    k_begin<<<grid_for(work_bound, kBlock, 1024), kBlock, 0, s>>>(ar, trees, n_trees, n_points, threshold, dmax);
    return hipGetLastError();
}

hipError_t launch_vote(const LevelArgs& a, int variant, bool wide, int grid, hipStream_t s)
{
    const bool ids = a.ar.entry_bytes == 8;
    if (variant == 1) {
        if (ids) k_vote<uint64_t, 1, int64_t><<<grid, kBlock, 0, s>>>(a);
        else k_vote<uint32_t, 1, int64_t><<<grid, kBlock, 0, s>>>(a);
    } else if (wide) {
        if (ids) k_vote<uint64_t, 0, int64_t><<<grid, kBlock, 0, s>>>(a);
        else k_vote<uint32_t, 0, int64_t><<<grid, kBlock, 0, s>>>(a);
    } else {
        if (ids) k_vote<uint64_t, 0, int32_t><<<grid, kBlock, 0, s>>>(a);
        else k_vote<uint32_t, 0, int32_t><<<grid, kBlock, 0, s>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_scan(const LevelArgs& a, hipStream_t s)
{
    k_scan<<<1, kScanThreads, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_emit(const LevelArgs& a, int grid, hipStream_t s)
{
    k_emit<<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_member_ids(const Cell* cells, int64_t n_cells, const int64_t* dst_off, const void* src,
                             int entry_bytes, const uint32_t* xy, int64_t n_points, int32_t* dst, hipStream_t s)
{
    if (n_cells <= 0) return hipSuccess;
    if (entry_bytes == 8)
        k_member_ids<uint64_t><<<grid_for(n_cells, kWaves), kBlock, 0, s>>>(
            cells, n_cells, dst_off, static_cast<const uint64_t*>(src), xy, n_points, dst);
    else
        k_member_ids<uint32_t><<<grid_for(n_cells, kWaves), kBlock, 0, s>>>(
            cells, n_cells, dst_off, static_cast<const uint32_t*>(src), xy, n_points, dst);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t* dst, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_iota<<<grid_for(n, kBlock), kBlock, 0, s>>>(dst, n);
    return hipGetLastError();
}

}  // namespace hh
