// gfx950 kernels of the hierarchical slope-intercept Hough vote
// (Singh and Bhatia, arXiv:1007.0547).
//
// Level-synchronous form of the paper's depth-first search (Sec. 3): all
// regions that split at level l (of every tree = pass of an image) are
// processed together.  Their voter lists are stored back to back in one
// dense list per level, so a flat entry index e in [0, L_l) walks all
// (parent region, line) pairs and every load is a plain streaming load.  An
// entry carries the line itself (the packed edge point, or the point id and
// the packed point), so no launch gathers coordinates.
//
// Per level, four launches:
//   k_count   one read of every entry: the 4-bit corner codes of the line for
//             the four children (Sec. 2, getcode()) and the vote rule (code
//             not 0000 / 1111, Sec. 3) as wavefront lane masks, and
//             per tile of kTile entries the child-vote counts of every
//             region piece in it.
//   k_decide  per region: its child votes (its pieces summed), the split
//             decisions (votes > T, Sec. 3) and their sums per range of regions.
//   k_emit    per region: offsets from those sums; the next level's region
//             table in quad order (so key order is kept) and tile map, or the
//             detected cells at the finest level.
//   k_write   a second read of every entry: each vote for a kept child is
//             written, in list order, to that child's list in the next
//             level (or to the member buffer at the finest level).
//
// Level sizes never travel to the host: each launch reads them from the
// arena's LevelInfo records written by the launches before it, and walks its
// work with a fixed grid.  No launch waits on another workgroup.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "hh_kernels.hpp"

namespace hh {
namespace {

constexpr int kScanThreads = 1024;   // the one-workgroup prefix of the edge staging

// Pointers reached through argument structs are generic; the kernels access
// device memory through these casts so the compiler emits global (not flat)
// loads, stores and atomics.
template <typename T>
__device__ inline T* G(T* p)
{
    return (T*)(__attribute__((address_space(1))) T*)p;
}

// Whether an earlier launch stopped the call.  A plain load: errors of earlier
// launches are visible at the kernel boundary, and an error raised by a
// concurrent workgroup of this launch need not stop the others.  Kernels load
// it together with their level sizes, so the check costs no extra round trip.
__device__ inline bool stopped(uint32_t err) { return (err & kErrStop) != 0; }

__device__ inline void raise_error(uint32_t* error, uint32_t bits)
{
    __hip_atomic_fetch_or(G(error), bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup barrier that orders LDS only.  The level kernels share nothing
// but LDS inside a workgroup, so their barriers need not wait for the
// wavefront's outstanding global stores (a full __syncthreads would drain
// them at every tile).
__device__ inline void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// set bits of b at lanes below this lane
__device__ inline uint32_t lanes_below(uint64_t b)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
}

__device__ inline uint64_t bits_below(int p) { return ((uint64_t)1 << p) - 1; }   // p in 0..63

// v (equal in every lane) as a wavefront-uniform value.  readfirstlane
// returns int: widen through uint32_t so bit 31 does not sign-extend.
__device__ inline uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

template <typename T>
__device__ inline T pick4(const T (&v)[4], int k)
{
    return k == 0 ? v[0] : k == 1 ? v[1] : k == 2 ? v[2] : v[3];
}

// A list entry carries its line as (u, v) packed u | v << 16: the edge point
// (x, y) in pass 0 and (y, x) in pass 1 (Sec. 3, BETA reads the point with
// its axes swapped), so no kernel tests the pass per entry.  swap16 turns one
// form into the other.
__device__ inline uint32_t swap16(uint32_t p) { return (p >> 16) | (p << 16); }

template <typename Entry> struct EntryOps;
template <> struct EntryOps<uint32_t> {   // the packed line
    __device__ static uint32_t point(uint32_t e) { return e; }
    __device__ static uint32_t root(const uint32_t* pts, int64_t k, bool swap)
    {
        return swap ? swap16(pts[k]) : pts[k];
    }
    __device__ static uint32_t natural(uint32_t e, bool swap) { return swap ? swap16(e) : e; }
};
template <> struct EntryOps<uint64_t> {   // point id << 32 | packed line
    __device__ static uint32_t point(uint64_t e) { return (uint32_t)e; }
    __device__ static uint64_t root(const uint32_t* pts, int64_t k, bool swap)
    {
        return ((uint64_t)k << 32) | (swap ? swap16(pts[k]) : pts[k]);
    }
    __device__ static uint64_t natural(uint64_t e, bool swap)
    {
        return swap ? ((e & 0xFFFFFFFF00000000ull) | swap16((uint32_t)e)) : e;
    }
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
// t_{c+1} = t_c - 2u.  Since u >= 0, t_c does not grow with c while B_r
// grows with r: a corner below the line has every corner west or south of it
// below too.  So a child's code (NE, NW, SW, SE corner bits) is some-but-not-
// all below -- neither 0000 nor 1111, the vote rule -- exactly when its SW
// corner is below and its NE corner is not; the other two bits never decide.
// Seven of the nine corner compares are needed, each one lane mask b_cr.
template <typename CT>
__device__ inline void code_masks(uint64_t vm, int32_t u, int32_t v, int32_t pi, int32_t pj, int lc, int s_log2,
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
    const uint64_t b00 = __ballot(B0 < t0), b01 = __ballot(B1 < t0);
    const uint64_t b10 = __ballot(B0 < t1), b11 = __ballot(B1 < t1), b12 = __ballot(B2 < t1);
    const uint64_t b21 = __ballot(B1 < t2), b22 = __ballot(B2 < t2);
    // child at (east e, north n): SW corner (e, n), NE corner (e+1, n+1)
    cm[0] = vm & b11 & ~b22;   // NE child, e = 1, n = 1
    cm[1] = vm & b01 & ~b12;   // NW child, e = 0, n = 1
    cm[2] = vm & b00 & ~b11;   // SW child, e = 0, n = 0
    cm[3] = vm & b10 & ~b21;   // SE child, e = 1, n = 0
}

// Circumscribed-circle variant (comparison method of the paper's ref. [9]).
// For child (lc, i, j) with centre m = -1 + (2i+1)/2^lc,
// b = -S + 3S(2j+1)/2^(lc+1), in units where the cell is a unit square, the
// line is within the circumradius iff D^2 <= 2 (9 S^2 + 4 u^2) with
// D = 3S(2j+1) + 2u(2i+1) - (v + u + S) 2^(lc+1).
__device__ inline void circle_masks(uint64_t vm, int32_t u, int32_t v, int32_t pi, int32_t pj, int lc,
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
    cm[0] = vm & __ballot(dNE * dNE <= rhs);
    cm[1] = vm & __ballot(dNW * dNW <= rhs);
    cm[2] = vm & __ballot(dSW * dSW <= rhs);
    cm[3] = vm & __ballot(dSE * dSE <= rhs);
}

template <int kVariant, typename CT>
__device__ inline void child_masks(uint64_t vm, uint32_t point, uint32_t meta, uint32_t ij, int lc,
                                   uint64_t (&cm)[4])
{
    const int32_t u = (int32_t)(point & 0xFFFFu), v = (int32_t)(point >> 16);
    const int s_log2 = (int)((meta >> kMetaSlogShift) & 15u);
    const int32_t pi = (int32_t)(ij & 0xFFFFu), pj = (int32_t)(ij >> 16);
    if constexpr (kVariant == 0)
        code_masks<CT>(vm, u, v, pi, pj, lc, s_log2, cm);
    else
        circle_masks(vm, u, v, pi, pj, lc, s_log2, cm);
}

// The open region's part of the vote test, computed once per region and kept
// in scalar registers; masks() evaluates a whole row of lines against it as
// lane masks, votes() (code variant) as per-lane bits without any scalar
// work.  With d_cr = t_c - B_r - 1, corner (c, r) is below the line iff
// d_cr >= 0, so a child votes iff the sign bit of ~d_SW & d_NE is set.
template <int kVariant, typename CT>
struct OpenMasks {
    uint32_t ij, meta;
    CT M0, B0, B1, B2;      // code variant: scaled corner values of the children's grid
    CT nB0, nB1, nB2;       //   -B_r - 1
    __device__ void set(uint32_t ij_, uint32_t meta_, int lc)
    {
        ij = ij_;
        meta = meta_;
        const int s_log2 = (int)((meta >> kMetaSlogShift) & 15u);
        const CT S = (CT)1 << s_log2;
        const int32_t pi = (int32_t)(ij & 0xFFFFu), pj = (int32_t)(ij >> 16);
        M0 = (CT)4 * (CT)pi - ((CT)1 << lc);
        B0 = (CT)6 * S * (CT)pj - (S << lc);
        B1 = B0 + (CT)3 * S;
        B2 = B1 + (CT)3 * S;
        nB0 = -B0 - 1;
        nB1 = -B1 - 1;
        nB2 = -B2 - 1;
    }
    __device__ void masks(uint64_t vm, uint32_t point, int lc, uint64_t (&cm)[4]) const
    {
        if constexpr (kVariant == 0) {
            const CT u = (CT)(point & 0xFFFFu), v = (CT)(point >> 16);
            const CT t0 = (v << lc) - mul(u, M0);
            const CT du = 2 * u;
            const CT t1 = t0 - du;
            const CT t2 = t1 - du;
            const uint64_t b00 = __ballot(B0 < t0), b01 = __ballot(B1 < t0);
            const uint64_t b10 = __ballot(B0 < t1), b11 = __ballot(B1 < t1), b12 = __ballot(B2 < t1);
            const uint64_t b21 = __ballot(B1 < t2), b22 = __ballot(B2 < t2);
            cm[0] = vm & b11 & ~b22;
            cm[1] = vm & b01 & ~b12;
            cm[2] = vm & b00 & ~b11;
            cm[3] = vm & b10 & ~b21;
        } else {
            child_masks<kVariant, CT>(vm, point, meta, ij, lc, cm);
        }
    }
    // code variant: vote bits of one lane (NE, NW, SW, SE in bits 0..3)
    // |u| < 2^14 and |M0| <= 2^15: a 24-bit multiply is exact for 32-bit compares
    __device__ static CT mul(CT u, CT m)
    {
        if constexpr (sizeof(CT) == 4) return __mul24(u, m);
        else return u * m;
    }
    template <bool kAllValid>
    __device__ uint32_t votes(bool valid, uint32_t point, int lc) const
    {
        const CT u = (CT)(point & 0xFFFFu), v = (CT)(point >> 16);
        CT t0 = (v << lc) - mul(u, M0);
        const CT du = 2 * u;
        CT t1 = t0 - du;
        CT t2 = t1 - du;
        if (!kAllValid && !valid) t0 = t1 = t2 = -((CT)1 << 30);   // below every corner: no vote
        const CT d00 = t0 + nB0, d01 = t0 + nB1;
        const CT d10 = t1 + nB0, d11 = t1 + nB1, d12 = t1 + nB2;
        const CT d21 = t2 + nB1, d22 = t2 + nB2;
        constexpr int kSign = 8 * (int)sizeof(CT) - 1;
        using U = typename std::conditional<sizeof(CT) == 8, uint64_t, uint32_t>::type;
        const uint32_t ne = (uint32_t)((U)(~d11 & d22) >> kSign);
        const uint32_t nw = (uint32_t)((U)(~d01 & d12) >> kSign);
        const uint32_t sw = (uint32_t)((U)(~d00 & d11) >> kSign);
        const uint32_t se = (uint32_t)((U)(~d10 & d21) >> kSign);
        return ne | (nw << 1) | (sw << 2) | (se << 3);
    }
};

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

__device__ inline int64_t wave_sum64(int64_t x)
{
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

__device__ inline int32_t wave_sum32(int32_t x)
{
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// ------------------------------------------------------------------ tiles
//
// A tile is kTile consecutive entries of a level's list: 32 rows of 64,
// wavefront w taking rows 8w .. 8w+7.  Its regions are tile_first[t] ..
// tile_first[t+1] (local indices 0 .. nr-1; local 0 holds the tile's first
// entry).  In LDS the tile keeps a bitmap of the entries (other than the
// first) that begin a region, so the local region of an entry is the number
// of marked entries up to it, and a row's marks form one 64-bit word.  A row
// with no mark belongs entirely to the wavefront's open region, whose fields
// the wavefront keeps in scalar registers; only rows with a mark look up
// region fields per lane.  Region fields come from LDS when the tile has at
// most kStage regions, otherwise from the region table (a separate
// instantiation, so no load has to choose between the two at run time).
// Each workgroup walks its tiles with the next tile's entries and bounds
// already in flight.

__device__ inline uint32_t rfl(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

template <typename Entry>
__device__ inline void load_rows(const Entry* list, int64_t L, int64_t tile, int wave, int lane, Entry (&ent)[kRows])
{
    const int64_t rb = tile * kTile + (int64_t)wave * (kRows * kWave);
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int64_t e = rb + k * kWave + lane;
        ent[k] = e < L ? list[e] : Entry(0);
    }
}

struct TileBounds {
    int r0, r1;
};

__device__ inline TileBounds tile_bounds(const int32_t* tile_first, int64_t tile, int64_t nt, int64_t P)
{
    TileBounds b{0, -1};
    if (tile < nt) {
        b.r0 = tile_first[tile];
        b.r1 = tile + 1 < nt ? tile_first[tile + 1] : (int)(P - 1);
    }
    return b;
}

// <= kTile + 1 regions: every region holds at least one entry
__device__ inline bool bounds_ok(const TileBounds& b, int64_t P)
{
    const int nr = b.r1 - b.r0 + 1;
    return b.r0 >= 0 && b.r1 < P && nr >= 1 && nr <= kTile + 1;
}

__device__ inline uint64_t row_word(const uint32_t* bm, int row)
{
    return uniform64((uint64_t)bm[2 * row] | ((uint64_t)bm[2 * row + 1] << 32));
}

// marked entries in the rows before wavefront `wave`
__device__ inline int starts_before(const uint32_t* bm, int wave, int lane)
{
    const int nw = 2 * kRows * wave;   // bitmap words before the wavefront's rows (< 64)
    const int c = lane < nw ? __popc(bm[lane]) : 0;
    return __builtin_amdgcn_readfirstlane(wave_sum32(c));
}

// Staged fields of a tile's first kStage regions.
struct StagedRegions {
    uint32_t ij[kStage];
    uint32_t meta[kStage];
};

// Fields of local region `local`: from LDS (kStaged) or the region table.
template <bool kStaged>
struct RegionSource {
    const StagedRegions& S;
    const Region* regions;
    int r0;
    __device__ void fields(int local, uint32_t& ij, uint32_t& meta) const
    {
        if constexpr (kStaged) {
            ij = S.ij[local];
            meta = S.meta[local];
        } else {
            ij = regions[r0 + local].ij;
            meta = regions[r0 + local].meta;
        }
    }
};

// Region marks and staged fields of one tile; returns whether local region 0
// began in an earlier tile.
__device__ inline bool stage_tile(uint32_t* bm, StagedRegions& sr, const Region* regions, int64_t t0,
                                  const TileBounds& tb)
{
    const int nr = tb.r1 - tb.r0 + 1;
    for (int k = threadIdx.x; k < nr; k += kBlock) {
        const Region R = regions[tb.r0 + k];
        const int64_t rel = R.start - t0;
        if (rel >= 1 && rel < kTile) atomicOr(&bm[rel >> 5], 1u << (rel & 31));
        if (k < kStage) {
            sr.ij[k] = R.ij;
            sr.meta[k] = R.meta;
        }
    }
    return regions[tb.r0].start < t0;
}

// ------------------------------------------------------------------ k_count
//
// Child-vote counts of every region piece of a tile.  A wavefront walks its
// rows keeping the counts of the region open at the current entry in scalar
// registers.  A region that begins and ends inside one tile has its total
// stored in cv at once (by the wavefront where it ends, or by the tile's
// combine step when it crosses wavefronts); the pieces of a region that
// crosses tiles are added to cv atomically, and the tile keeps for the
// compaction pass: head (the piece in the region's first tile), tcar (the
// piece of the region carried in from earlier tiles) and woff (the votes of
// each wavefront's first region counted before that wavefront in the tile).

// Vote bits (NE, NW, SW, SE in bits 0..3) of the line `point` for the
// children of a region with constants c, 32-bit compares.  With
// d_cr = t_c - B_r - 1, corner (c, r) is below iff d_cr >= 0, so a child votes
// iff the sign bit of ~d_SW & d_NE is set (see code_masks).
__device__ inline uint32_t code_votes(uint32_t point, const CodeConsts& c, int lc)
{
    const int32_t u = (int32_t)(point & 0xFFFFu), v = (int32_t)(point >> 16);
    const int32_t t0 = (v << lc) - __mul24(u, c.M0);   // |u| < 2^14, |M0| <= 2^15
    const int32_t du = 2 * u;
    const int32_t t1 = t0 - du;
    const int32_t t2 = t1 - du;
    const int32_t d00 = t0 + c.nB0, d01 = t0 + c.nB1;
    const int32_t d10 = t1 + c.nB0, d11 = t1 + c.nB1, d12 = t1 + c.nB2;
    const int32_t d21 = t2 + c.nB1, d22 = t2 + c.nB2;
    const uint32_t ne = (uint32_t)(~d11 & d22) >> 31;
    const uint32_t nw = (uint32_t)(~d01 & d12) >> 31;
    const uint32_t sw = (uint32_t)(~d00 & d11) >> 31;
    const uint32_t se = (uint32_t)(~d10 & d21) >> 31;
    return ne | (nw << 1) | (sw << 2) | (se << 3);
}

struct CountLds {
    uint32_t bm[kTile / 32];
    StagedRegions sr;
    CodeConsts cc[kStage];
    int32_t wfirst[kWaves][4];   // per wavefront: votes of the region open at its first entry (up to its close)
    int32_t wlast[kWaves][4];    //   votes of the region open at its end, from that region's start
    int32_t wlocal[kWaves];      //   local index of that region
    int32_t wclosed[kWaves];     //   whether the region open at its first entry ended inside it
};

struct WaveCount {
    int open;          // local index of the open region
    bool closed;       // the first region ended inside the wavefront
    int32_t run[4];    // votes of the open region counted inside the wavefront
    int32_t first[4];  // votes of the first region inside the wavefront
    uint32_t vword;    // this lane's vote bits, row k in bits 4k .. 4k+3
};

__device__ inline uint32_t lane_bits(const uint64_t (&cm)[4], int lane)
{
    uint32_t b = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) b |= (uint32_t)((cm[q] >> lane) & 1u) << q;
    return b;
}

// Vote bits of one lane's line for the children of its region (local index
// `local`): the staged code constants for 32-bit compares, otherwise the
// general lane-mask form.
template <int kVariant, typename CT, bool kStaged>
__device__ inline uint32_t lane_votes(const RegionSource<kStaged>& src, const CodeConsts* cc, int local,
                                      uint32_t point, uint64_t vm, int lc, int lane)
{
    if constexpr (kVariant == 0 && sizeof(CT) == 4) {
        // staged: cc is the tile's LDS copy; otherwise the level's table from
        // region r0.  Lanes past the list end compute on a zero entry and are
        // masked afterwards (no branch).
        const uint32_t vb = code_votes(point, cc[local], lc);
        return ((vm >> lane) & 1u) ? vb : 0u;
    } else {
        uint32_t ij, meta;
        src.fields(local, ij, meta);
        uint64_t cm[4];
        child_masks<kVariant, CT>(vm, point, meta, ij, lc, cm);
        return lane_bits(cm, lane);
    }
}

template <typename Entry, int kVariant, typename CT, bool kStaged>
__device__ __forceinline__ void count_rows(const RegionSource<kStaged>& src, const CodeConsts* cc, const uint32_t* bm,
                                           const Entry (&ent)[kRows], int64_t rb, int64_t L, int lc, int wave,
                                           int lane, int nr, int32_t* cv, WaveCount& wc)
{
    int open = starts_before(bm, wave, lane);
    bool open_here = false;   // the open region began inside this wavefront
    bool closed = false;
    int32_t run[4] = {0, 0, 0, 0}, first[4] = {0, 0, 0, 0};
    uint32_t vword = 0;
    const int lim = (int)std::max<int64_t>(0, std::min<int64_t>(L - rb, kRows * kWave));   // valid entries
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int left = lim - k * kWave;
        const uint64_t vm = left >= kWave ? ~0ull : (left <= 0 ? 0ull : bits_below(left));
        const uint64_t W = row_word(bm, wave * kRows + k);
        const int local = std::min(open + (int)__popcll(W & ((2ull << lane) - 1)), nr - 1);
        const uint32_t vb = lane_votes<kVariant, CT, kStaged>(src, cc, local, EntryOps<Entry>::point(ent[k]), vm, lc,
                                                                lane);
        vword |= vb << (4 * k);
        uint64_t cm[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) cm[q] = __ballot((vb >> q) & 1u);
        uint64_t rest = W;
        int prev = 0;
        while (rest) {   // regions that end inside this row
            const int p = __builtin_ctzll(rest);
            rest &= rest - 1;
            const uint64_t seg = bits_below(p) & ~bits_below(prev);
#pragma unroll
            for (int q = 0; q < 4; ++q) run[q] += (int32_t)__popcll(cm[q] & seg);
            if (open_here) {   // began and ended in this wavefront: its total
                if (lane == 0)
                    *reinterpret_cast<int4*>(cv + (int64_t)(src.r0 + open) * 4) = int4{run[0], run[1], run[2], run[3]};
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) first[q] = run[q];
                closed = true;
            }
            ++open;
            open_here = true;
            prev = p;
#pragma unroll
            for (int q = 0; q < 4; ++q) run[q] = 0;
        }
        const uint64_t tail = ~bits_below(prev);
#pragma unroll
        for (int q = 0; q < 4; ++q) run[q] += (int32_t)__popcll(cm[q] & tail);
    }
    wc.open = open;
    wc.closed = closed;
    wc.vword = vword;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        wc.run[q] = run[q];
        wc.first[q] = closed ? first[q] : run[q];
    }
}

// Register budgets: k_count at 6 wavefronts per SIMD (80 VGPRs, no spills) and
// k_write at 7 (65 VGPRs, scalar spills to VGPR lanes only) hide more latency
// than the compiler's defaults; both measured faster (-7% and -5%).
template <typename Entry, int kVariant, typename CT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_count(LevelArgs a)
{
    __shared__ CountLds S;
    const Arena& ar = a.ar;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int l = a.level;
    const int lc = l + 1;
    const uint32_t err = *G(ar.error);
    const int64_t P = ar.info[l].P, L = ar.info[l].L;
    if (stopped(err) || P == 0) return;
    const HalfLayout hl = half_layout(ar.half[l & 1], P, L, ar.entry_bytes);
    const WorkLayout wl = work_layout(ar.work, P, L);
    if (hl.end > ar.half_cap || wl.end > ar.work_cap) {
        if (tid == 0 && blockIdx.x == 0) raise_error(ar.error, kErrArena);
        return;
    }
    const Entry* const list = G(static_cast<const Entry*>(hl.list));
    const Region* const regions = G(static_cast<const Region*>(hl.regions));
    const int32_t* const tile_first = G(static_cast<const int32_t*>(hl.tile_first));
    int32_t* const cv = G(hl.cv);
    const CodeConsts* const ccg = G(static_cast<const CodeConsts*>(hl.cc));
    int32_t* const head = G(wl.head);
    int32_t* const tcar = G(wl.tcar);
    int32_t* const woff = G(wl.woff);
    const int64_t nt = cdiv(L, kTile);
    int64_t tile = blockIdx.x;
    if (tile >= nt) return;

    if (tid < kTile / 32) S.bm[tid] = 0u;
    Entry ent[kRows];
    load_rows(list, L, tile, wave, lane, ent);
    TileBounds tb = tile_bounds(tile_first, tile, nt, P);
    for (;;) {
        const int64_t next = tile + gridDim.x;
        const int64_t t0 = tile * kTile;
        const int64_t rb = t0 + (int64_t)wave * (kRows * kWave);
        if (!bounds_ok(tb, P)) {
            if (tid == 0) raise_error(ar.error, kErrInternal);
            return;
        }
        const int r0 = tb.r0, nr = tb.r1 - tb.r0 + 1;
        lds_barrier();   // the previous tile is done with S (its bitmap is clear again)
        const bool carried = stage_tile(S.bm, S.sr, regions, t0, tb);
        if constexpr (kVariant == 0 && sizeof(CT) == 4)
            for (int k = tid; k < nr && k < kStage; k += kBlock) S.cc[k] = ccg[r0 + k];
        lds_barrier();
        // the next tile's entries and bounds, issued only now: loads complete in
        // order, so a wait for this tile's region fields would otherwise wait
        // for them too
        Entry nent[kRows];
        load_rows(list, L, next, wave, lane, nent);
        const TileBounds ntb = tile_bounds(tile_first, next, nt, P);
        WaveCount wc;
        if (nr <= kStage)
            count_rows<Entry, kVariant, CT, true>(RegionSource<true>{S.sr, regions, r0}, S.cc, S.bm, ent, rb, L, lc,
                                                  wave, lane, nr, cv, wc);
        else
            count_rows<Entry, kVariant, CT, false>(RegionSource<false>{S.sr, regions, r0}, ccg + r0, S.bm, ent, rb,
                                                   L, lc, wave, lane, nr, cv, wc);
        G(wl.vbits)[tile * kBlock + tid] = wc.vword;
        if (lane < 4) {
            S.wfirst[wave][lane] = pick4(wc.first, lane);
            S.wlast[wave][lane] = pick4(wc.run, lane);
        }
        if (lane == 0) {
            S.wlocal[wave] = wc.open;
            S.wclosed[wave] = wc.closed ? 1 : 0;
        }
        lds_barrier();
        if (tid < 4) {   // one thread per child slot
            const int q = tid;
            int cur = 0;
            bool cur_carried = carried;
            int32_t cnt = 0;
            for (int w = 0; w < kWaves; ++w) {
                woff[(tile * kWaves + w) * 4 + q] = cnt;
                cnt += S.wfirst[w][q];
                if (S.wclosed[w]) {
                    if (cur_carried) {   // the last piece of a region from earlier tiles
                        tcar[tile * 4 + q] = cnt;
                        atomicAdd(&cv[(int64_t)r0 * 4 + q], cnt);
                    } else {
                        cv[(int64_t)(r0 + cur) * 4 + q] = cnt;   // began and ended in this tile
                    }
                    cur = S.wlocal[w];
                    cur_carried = false;
                    cnt = S.wlast[w][q];
                }
            }
            // the region open at the tile's end (it may continue in the next tile)
            if (cur_carried) tcar[tile * 4 + q] = cnt;
            else head[(int64_t)(r0 + cur) * 4 + q] = cnt;
            atomicAdd(&cv[(int64_t)(r0 + cur) * 4 + q], cnt);
        }
        if (tid < kTile / 32) S.bm[tid] = 0u;   // every wavefront has read the bitmap

        if (next >= nt) break;
        tile = next;
        tb = ntb;
#pragma unroll
        for (int k = 0; k < kRows; ++k) ent[k] = nent[k];
    }
}

// ------------------------------------------------------------------ k_decide / k_emit
//
// Both launches split the P regions into blocks of kBlock and the blocks
// into kRangeGrid contiguous ranges, range g going to workgroup g of either
// launch.  k_decide leaves one sum per range and channel; k_emit takes the
// exclusive prefix of those sums as its range's starting offsets, so no
// launch scans all regions.

__device__ inline void range_of(int64_t nb, int g, int64_t& b0, int64_t& b1)
{
    if (nb <= kRangeGrid) {   // one block per range, in the first workgroups dispatched
        b0 = std::min<int64_t>(g, nb);
        b1 = std::min<int64_t>(g + 1, nb);
    } else {
        b0 = nb * g / kRangeGrid;
        b1 = nb * (g + 1) / kRangeGrid;
    }
}

// Decision channels of one region from its child votes.
__device__ inline void decision(const int32_t (&cv)[4], int32_t thr, bool finest, int64_t (&dv)[kAggCh])
{
#pragma unroll
    for (int c = 0; c < kAggCh; ++c) dv[c] = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        dv[4] += cv[q];
        if (cv[q] > thr) {
            if (finest) {
                dv[2] += 1;
                dv[3] += cv[q];
            } else {
                dv[0] += 1;
                dv[1] += cv[q];
            }
        }
    }
}

__device__ inline void region_decision(const Region* regions, const int32_t* cvi, const TreeDesc* trees, int64_t r,
                                       Region& R, int32_t (&cv)[4], int32_t& thr, int64_t (&dv)[kAggCh])
{
    R = regions[r];
    const int4 c = reinterpret_cast<const int4*>(cvi)[r];
    cv[0] = c.x;
    cv[1] = c.y;
    cv[2] = c.z;
    cv[3] = c.w;
    thr = trees[R.tree].threshold;
    decision(cv, thr, (R.meta & kMetaChildFinest) != 0, dv);
}

__global__ __launch_bounds__(kBlock) void k_decide(LevelArgs a)
{
    __shared__ int64_t s_red[kWaves][kAggCh];
    const Arena& ar = a.ar;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int l = a.level;
    const uint32_t err = *G(ar.error);
    const int64_t P = ar.info[l].P, L = ar.info[l].L;
    if (stopped(err) || P == 0) return;
    const HalfLayout hl = half_layout(ar.half[l & 1], P, L, ar.entry_bytes);
    const WorkLayout wl = work_layout(ar.work, P, L);
    if (hl.end > ar.half_cap || wl.end > ar.work_cap) return;   // k_count raised the error
    const Region* const regions = G(static_cast<const Region*>(hl.regions));
    const int32_t* const cvi = G(static_cast<const int32_t*>(hl.cv));
    const TreeDesc* const trees = G(a.trees);
    const int64_t nb = cdiv(P, kBlock);

    for (int g = blockIdx.x; g < kRangeGrid; g += gridDim.x) {
        int64_t b0, b1;
        range_of(nb, g, b0, b1);
        int64_t acc[kAggCh] = {0, 0, 0, 0, 0};
        for (int64_t r = b0 * kBlock + tid; r < std::min(P, b1 * kBlock); r += kBlock) {
            Region R;
            int32_t cv[4], thr;
            int64_t dv[kAggCh];
            region_decision(regions, cvi, trees, r, R, cv, thr, dv);
#pragma unroll
            for (int c = 0; c < kAggCh; ++c) acc[c] += dv[c];
        }
#pragma unroll
        for (int c = 0; c < kAggCh; ++c) {
            const int64_t s = wave_sum64(acc[c]);
            if (lane == 0) s_red[wave][c] = s;
        }
        __syncthreads();
        if (tid < kAggCh) {
            int64_t s = 0;
            for (int w = 0; w < kWaves; ++w) s += s_red[w][tid];
            G(wl.agg)[(int64_t)g * kAggCh + tid] = s;
        }
        __syncthreads();
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
    __shared__ int64_t s_red[kWaves][2 * kAggCh];
    __shared__ int64_t s_w[kWaves][kAggCh];
    const Arena& ar = a.ar;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int l = a.level;
    const int lc = l + 1;
    const uint32_t err = *G(ar.error);
    const int64_t P = ar.info[l].P, L = ar.info[l].L;
    if (stopped(err)) return;
    const int64_t cells_base = ar.info[l].cells_base + ar.info[l].cells;
    const int64_t mem_base = ar.info[l].mem_base + ar.info[l].mem;
    if (P == 0) {
        if (tid == 0 && blockIdx.x == 0) {
            LevelInfo& nx = ar.info[lc];
            nx.P = 0;
            nx.L = 0;
            nx.cells = 0;
            nx.mem = 0;
            nx.cells_base = cells_base;
            nx.mem_base = mem_base;
        }
        return;
    }
    const HalfLayout hl = half_layout(ar.half[l & 1], P, L, ar.entry_bytes);
    const WorkLayout wl = work_layout(ar.work, P, L);
    if (hl.end > ar.half_cap || wl.end > ar.work_cap) return;
    const int64_t* const agg = G(static_cast<const int64_t*>(wl.agg));
    const Region* const regions = G(static_cast<const Region*>(hl.regions));
    const int32_t* const cvi = G(static_cast<const int32_t*>(hl.cv));
    int64_t* const dsto = G(wl.dst);
    const TreeDesc* const trees = G(a.trees);
    const int64_t nb = cdiv(P, kBlock);

    for (int g = blockIdx.x; g < kRangeGrid; g += gridDim.x) {
        int64_t b0, b1;
        range_of(nb, g, b0, b1);
        if (b0 == b1 && g != 0) continue;   // nothing here, and the level totals are written by range 0
        // this range's offsets and the level totals
        int64_t pre[kAggCh], tot[kAggCh];
        {
            int64_t p2[2 * kAggCh];
#pragma unroll
            for (int c = 0; c < 2 * kAggCh; ++c) p2[c] = 0;
            for (int k = tid; k < kRangeGrid; k += kBlock)
#pragma unroll
                for (int c = 0; c < kAggCh; ++c) {
                    const int64_t v = agg[(int64_t)k * kAggCh + c];
                    if (k < g) p2[c] += v;
                    p2[kAggCh + c] += v;
                }
#pragma unroll
            for (int c = 0; c < 2 * kAggCh; ++c) {
                const int64_t s = wave_sum64(p2[c]);
                if (lane == 0) s_red[wave][c] = s;
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < kAggCh; ++c) {
                pre[c] = 0;
                tot[c] = 0;
                for (int w = 0; w < kWaves; ++w) {
                    pre[c] += s_red[w][c];
                    tot[c] += s_red[w][kAggCh + c];
                }
            }
            __syncthreads();
        }
        const int64_t P2 = tot[0], L2 = tot[1];
        const HalfLayout nx = half_layout(ar.half[lc & 1], P2, L2, ar.entry_bytes);
        const bool fits = nx.end <= ar.half_cap && work_layout(ar.work, P2, L2).end <= ar.work_cap &&
                          cells_base + tot[2] <= ar.cells_cap &&
                          (!a.keep_members || mem_base + tot[3] <= ar.mem_cap);
        if (g == 0 && tid == 0) {
            LevelInfo& ni = ar.info[lc];
            ni.P = P2;
            ni.L = L2;
            ni.cells = tot[2];
            ni.cells_base = cells_base;
            ni.mem = tot[3];
            ni.mem_base = mem_base;
            ar.info[l].votes = tot[4];
            if (!fits) raise_error(ar.error, kErrArena);
        }
        if (!fits) return;
        Region* const nreg = G(nx.regions);
        int32_t* const ntf = G(nx.tile_first);
        int32_t* const ncv = G(nx.cv);
        const int64_t n_ntiles = cdiv(L2, kTile);
        for (int64_t b = b0; b < b1; ++b) {
            const int64_t r = b * kBlock + tid;
            const bool valid = r < P;
            Region R{};
            int32_t cv[4] = {0, 0, 0, 0};
            int32_t thr = 0;
            int64_t dv[kAggCh] = {0, 0, 0, 0, 0};
            if (valid) region_decision(regions, cvi, trees, r, R, cv, thr, dv);
            int64_t ex[kAggCh], inc[kAggCh];
#pragma unroll
            for (int c = 0; c < kAggCh; ++c) {
                inc[c] = wave_incl_scan64(dv[c], lane);
                if (lane == kWave - 1) s_w[wave][c] = inc[c];
            }
            __syncthreads();
            int64_t btot[kAggCh];
#pragma unroll
            for (int c = 0; c < kAggCh; ++c) {
                int64_t wp = 0;
                btot[c] = 0;
                for (int w = 0; w < kWaves; ++w) {
                    if (w < wave) wp += s_w[w][c];
                    btot[c] += s_w[w][c];
                }
                ex[c] = pre[c] + wp + inc[c] - dv[c];
            }
            __syncthreads();
            if (valid) {
                const TreeDesc T = trees[R.tree];
                const bool finest = R.meta & kMetaChildFinest;
                const int32_t pi = (int32_t)(R.ij & 0xFFFFu), pj = (int32_t)(R.ij >> 16);
                int64_t ri = ex[0], start = ex[1], ci = cells_base + ex[2], mo = mem_base + ex[3];
                int64_t dq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    dq[q] = -1;
                    if (cv[q] <= thr) continue;
                    const int32_t e = (q == 0 || q == 3) ? 1 : 0;
                    const int32_t n = (q <= 1) ? 1 : 0;
                    const int32_t ci_ = 2 * pi + e, cj = 2 * pj + n;
                    if (finest) {
                        Cell c;
                        c.i = ci_;
                        c.j = cj;
                        c.votes = cv[q];
                        c.pass = T.pass;
                        c.key = key_of(ci_, cj, lc);
                        c.member_off = a.keep_members ? mo : -1;
                        G(ar.cells)[ci++] = c;
                        if (a.keep_members) dq[q] = mo;
                        mo += cv[q];
                    } else {
                        if (ri >= P2) {
                            raise_error(ar.error, kErrInternal);
                            continue;
                        }
                        Region C;
                        C.start = start;
                        C.ij = (uint32_t)ci_ | ((uint32_t)cj << 16);
                        C.len = cv[q];
                        C.tree = R.tree;
                        C.meta = (R.meta & ~kMetaChildFinest) | (lc + 1 == T.dmax ? kMetaChildFinest : 0u);
                        nreg[ri] = C;
                        G(nx.cc)[ri] = code_consts(C.ij, C.meta, lc + 1);
                        reinterpret_cast<int4*>(ncv)[ri] = int4{0, 0, 0, 0};
                        // next-level tiles whose first entry falls inside this region
                        for (int64_t t = cdiv(start, kTile); t * kTile < start + cv[q] && t < n_ntiles; ++t)
                            ntf[t] = (int32_t)ri;
                        dq[q] = start;
                        ++ri;
                        start += cv[q];
                    }
                }
                int4* const d4 = reinterpret_cast<int4*>(dsto + r * 4);
                d4[0] = int4{(int32_t)dq[0], (int32_t)(dq[0] >> 32), (int32_t)dq[1], (int32_t)(dq[1] >> 32)};
                d4[1] = int4{(int32_t)dq[2], (int32_t)(dq[2] >> 32), (int32_t)dq[3], (int32_t)(dq[3] >> 32)};
                // the first parent of each tree records where its tree's sums begin
                if (r == 0 || regions[r - 1].tree != R.tree) {
                    int64_t* rc = G(ar.rec + ((int64_t)R.tree * kMaxLevels + l) * kRecCh);
                    rc[0] = r;
                    rc[1] = R.start;
                    rc[2] = ex[0];
                    rc[3] = ex[1];
                    rc[4] = ex[2];
                    rc[5] = ex[4];
                    rc[6] = ex[3];
                }
            }
#pragma unroll
            for (int c = 0; c < kAggCh; ++c) pre[c] += btot[c];
        }
    }
}

// ------------------------------------------------------------------ k_write
//
// Second read of every entry.  A vote of the entry for child q of its region
// r goes to dst[r][q] + its rank among the votes of r for q in list order.
// Within a row the rank is a lane count: for the lanes of the region open at
// the row's first entry the wavefront's running count plus the lanes below,
// for a region that begins in the row the lanes below minus the lanes below
// its first entry.  A wavefront starts its running counts from woff, plus,
// for a region carried in from earlier tiles, its votes in those tiles
// (head of its first tile and tcar of the tiles between), so wavefronts never
// exchange counts.

struct WriteLds {
    uint32_t bm[2][kTile / 32];  // alternate tiles: one is cleared while the other is in use
    StagedRegions sr;
    int64_t dst[kStage][4];
    int32_t cv[kStage][4];
    int32_t tpre[4];             // votes of the carried region before this tile
};

// Child destinations and child votes of local region `local`.
template <bool kStaged>
struct KidSource {
    const int64_t (*s_dst)[4];
    const int32_t (*s_cv)[4];
    const int64_t* dsti;
    const int32_t* cvi;
    int r0;
    __device__ int64_t dst(int local, int q) const
    {
        if constexpr (kStaged) return s_dst[local][q];
        else return dsti[(int64_t)(r0 + local) * 4 + q];
    }
    __device__ int32_t votes(int local, int q) const
    {
        if constexpr (kStaged) return s_cv[local][q];
        else return cvi[(int64_t)(r0 + local) * 4 + q];
    }
};

// Rows of one wavefront.  Per child slot q the open region keeps bq[q], the
// start of that child's list (in the next level's list, or the member buffer
// at the finest level), run[q], its votes for q so far, and cv[q], its total
// votes for q from the count pass (the emit step checked every child's slot
// [dst, dst + cv) against its buffer).  The lanes voting for q write at
// run[q] + their rank in the row, the offset clamped to cv[q] - 1 so that no
// store leaves the child's slot; when a region closes, run must equal cv
// (else the call fails with an internal error).  A row without a region start
// continues the open region's counts; in a row where regions start, each lane
// takes its destination on its own: the lanes of the region open at the row
// start continue its counts, the others count from their region's first lane
// in the row.
template <typename Entry, bool kStaged>
__device__ __forceinline__ void write_rows(const RegionSource<kStaged>& src, const KidSource<kStaged>& kids,
                                           const uint32_t* bm, const Entry (&ent)[kRows], uint32_t vword, int wave,
                                           int lane, int nr, const int32_t (&run0)[4], int open, Entry* nlist,
                                           Entry* members, bool& bad)
{
    Entry* bq[4];
    int32_t run[4], cv[4];
    uint32_t keep;     // bit q: child q's voters are kept
    bool unswap;       // member entries are stored as (x, y) whatever the pass
    auto open_fields = [&]() {
        const int o = std::min(open, nr - 1);
        uint32_t ij, meta;
        src.fields(o, ij, meta);
        meta = rfl(meta);
        const bool finest = meta & kMetaChildFinest;
        Entry* const out = finest ? members : nlist;
        unswap = finest && (meta & kMetaPass);
        keep = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t d = (int64_t)uniform64((uint64_t)kids.dst(o, q));
            keep |= (d >= 0 ? 1u : 0u) << q;
            bq[q] = out + (d >= 0 ? d : 0);
            cv[q] = (int32_t)rfl((uint32_t)kids.votes(o, q));
            run[q] = 0;
        }
    };
    auto close_check = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (((keep >> q) & 1u) && run[q] != cv[q]) bad = true;
    };
    open_fields();
#pragma unroll
    for (int q = 0; q < 4; ++q) run[q] = run0[q];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const uint32_t vb = (vword >> (4 * k)) & 15u;
        uint64_t cm[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) cm[q] = __ballot((vb >> q) & 1u);
        const uint64_t W = row_word(bm, wave * kRows + k);
        const int starts = (int)__popcll(W);
        if (starts == 0) {   // the whole row belongs to the open region
            const Entry e_out = EntryOps<Entry>::natural(ent[k], unswap);
            const uint32_t vk = vb & keep;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if ((vk >> q) & 1u) bq[q][std::min(run[q] + (int32_t)lanes_below(cm[q]), cv[q] - 1)] = e_out;
                run[q] += (int32_t)__popcll(cm[q]);
            }
            continue;
        }
        // a region starts in this row: per-lane destinations
        const uint64_t le = W & ((2ull << lane) - 1);
        const bool seg0 = le == 0;
        const int local = std::min(open + (int)__popcll(le), nr - 1);
        const int p = seg0 ? 0 : 63 - __builtin_clzll(le);   // first lane of this lane's region in the row
        uint32_t ij, meta;
        src.fields(local, ij, meta);
        uint32_t m[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) m[q] = lanes_below(cm[q]);
        const uint32_t packed = m[0] | (m[1] << 8) | (m[2] << 16) | (m[3] << 24);
        const uint32_t at_p = (uint32_t)__shfl((int)packed, p, kWave);
        const bool finest = meta & kMetaChildFinest;
        Entry* const out = finest ? members : nlist;
        const Entry e_out = EntryOps<Entry>::natural(ent[k], finest && (meta & kMetaPass));
        const uint64_t first = bits_below(__builtin_ctzll(W));   // the lanes of the region open at the row start
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!((vb >> q) & 1u)) continue;
            const int32_t rank = (int32_t)m[q] - (int32_t)((at_p >> (8 * q)) & 255u);
            if (seg0) {
                if ((keep >> q) & 1u) bq[q][std::min(run[q] + rank, cv[q] - 1)] = e_out;
            } else {
                const int64_t d = kids.dst(local, q);
                if (d >= 0) out[d + std::min(rank, kids.votes(local, q) - 1)] = e_out;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) run[q] += (int32_t)__popcll(cm[q] & first);
        close_check();
        open += starts;
        const int h = 63 - __builtin_clzll(W);
        open_fields();
#pragma unroll
        for (int q = 0; q < 4; ++q) run[q] = (int32_t)__popcll(cm[q] & ~bits_below(h));
    }
}

template <typename Entry>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) void k_write(LevelArgs a)
{
    __shared__ WriteLds S;
    const Arena& ar = a.ar;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int l = a.level;
    const int lc = l + 1;
    const uint32_t err = *G(ar.error);
    const int64_t P = ar.info[l].P, L = ar.info[l].L;
    if (stopped(err) || P == 0) return;
    const HalfLayout hl = half_layout(ar.half[l & 1], P, L, ar.entry_bytes);
    const WorkLayout wl = work_layout(ar.work, P, L);
    if (hl.end > ar.half_cap || wl.end > ar.work_cap) return;
    // the next level's list and the member buffer were checked by the emit step
    const HalfLayout nx = half_layout(ar.half[lc & 1], ar.info[lc].P, ar.info[lc].L, ar.entry_bytes);
    const Entry* const list = G(static_cast<const Entry*>(hl.list));
    const Region* const regions = G(static_cast<const Region*>(hl.regions));
    const int32_t* const tile_first = G(static_cast<const int32_t*>(hl.tile_first));
    const int64_t* const dsti = G(static_cast<const int64_t*>(wl.dst));
    const int32_t* const head = G(static_cast<const int32_t*>(wl.head));
    const int32_t* const tcar = G(static_cast<const int32_t*>(wl.tcar));
    const int32_t* const woff = G(static_cast<const int32_t*>(wl.woff));
    const int32_t* const cvi = G(static_cast<const int32_t*>(hl.cv));
    Entry* const nlist = G(static_cast<Entry*>(nx.list));
    Entry* const members = G(static_cast<Entry*>(ar.members));
    const int64_t nt = cdiv(L, kTile);
    int64_t tile = blockIdx.x;
    if (tile >= nt) return;

    if (tid < kTile / 32) {
        S.bm[0][tid] = 0u;
        S.bm[1][tid] = 0u;
    }
    const uint32_t* const vbits = G(static_cast<const uint32_t*>(wl.vbits));
    Entry ent[kRows];
    load_rows(list, L, tile, wave, lane, ent);
    uint32_t vword = vbits[tile * kBlock + tid];
    TileBounds tb = tile_bounds(tile_first, tile, nt, P);
    bool bad = false;
    for (int it = 0;; ++it) {
        const int64_t next = tile + gridDim.x;
        const int64_t t0 = tile * kTile;
        if (!bounds_ok(tb, P)) {
            if (tid == 0) raise_error(ar.error, kErrInternal);
            return;
        }
        const int r0 = tb.r0, nr = tb.r1 - tb.r0 + 1;
        uint32_t* const bm = S.bm[it & 1];
        lds_barrier();   // the previous tile is done with S
        if (tid < kTile / 32) S.bm[(it + 1) & 1][tid] = 0u;   // last read two tiles ago
        const bool carried = stage_tile(bm, S.sr, regions, t0, tb);
        for (int k = tid; k < nr && k < kStage; k += kBlock) {
#pragma unroll
            for (int q = 0; q < 4; ++q) S.dst[k][q] = dsti[(int64_t)(r0 + k) * 4 + q];
            *reinterpret_cast<int4*>(S.cv[k]) = reinterpret_cast<const int4*>(cvi)[r0 + k];
        }
        if (carried && wave == 0) {
            // votes of the carried region before this tile: its first tile's
            // piece plus the whole tiles in between
            const int64_t ts = regions[r0].start / kTile;
            int32_t c[4] = {0, 0, 0, 0};
            for (int64_t t = ts + 1 + lane; t < tile; t += kWave) {
                const int4 v = reinterpret_cast<const int4*>(tcar)[t];
                c[0] += v.x;
                c[1] += v.y;
                c[2] += v.z;
                c[3] += v.w;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) c[q] = wave_sum32(c[q]);
            if (lane < 4) S.tpre[lane] = pick4(c, lane) + head[(int64_t)r0 * 4 + lane];
        }
        lds_barrier();

        const int open = starts_before(bm, wave, lane);
        int32_t run[4];
        {
            const bool first_carried = open == 0 && carried;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                run[q] = woff[(tile * kWaves + wave) * 4 + q] + (first_carried ? S.tpre[q] : 0);
        }
        // the next tile's entries, vote bits and bounds, issued only once this
        // tile's tables are read (loads complete in order)
        Entry nent[kRows];
        load_rows(list, L, next, wave, lane, nent);
        const uint32_t nvword = next < nt ? vbits[next * kBlock + tid] : 0u;
        const TileBounds ntb = tile_bounds(tile_first, next, nt, P);
        if (nr <= kStage)
            write_rows<Entry, true>(RegionSource<true>{S.sr, regions, r0},
                                    KidSource<true>{S.dst, S.cv, dsti, cvi, r0}, bm, ent, vword, wave, lane, nr, run,
                                    open, nlist, members, bad);
        else
            write_rows<Entry, false>(RegionSource<false>{S.sr, regions, r0},
                                     KidSource<false>{S.dst, S.cv, dsti, cvi, r0}, bm, ent, vword, wave, lane, nr,
                                     run, open, nlist, members, bad);

        if (next >= nt) break;
        tile = next;
        tb = ntb;
        vword = nvword;
#pragma unroll
        for (int k = 0; k < kRows; ++k) ent[k] = nent[k];
    }
    if (__any(bad) && lane == 0) raise_error(ar.error, kErrInternal);
}

// Edge staging: nonzero pixels of each image of a batch, row-major.  A
// pixel tile (kPixTile pixels) belongs to one image, found by binary search
// over the images' first tiles.
__device__ inline int image_of_tile(const ImageDesc* images, int32_t n_images, int64_t tile)
{
    int lo = 0, hi = n_images - 1;   // last image with tile0 <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (images[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline uint32_t pixel_bits(const ImageDesc& im, int64_t p0, int32_t& row, int32_t& col)
{
    uint32_t bits = 0;
    row = 0;
    col = 0;
    if (p0 < im.n_pix) {
        row = (int32_t)(p0 / im.width);
        col = (int32_t)(p0 - (int64_t)row * im.width);
        int32_t r = row, c = col;
        for (int k = 0; k < kPixPerThread && p0 + k < im.n_pix; ++k) {
            if (im.image[(int64_t)r * im.row_stride + c]) bits |= 1u << k;
            if (++c == im.width) {
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
        const ImageDesc im = a.images[image_of_tile(a.images, a.n_images, tile)];
        int32_t row, col;
        const uint32_t bits =
            pixel_bits(im, (tile - im.tile0) * kPixTile + (int64_t)threadIdx.x * kPixPerThread, row, col);
        int32_t total;
        __syncthreads();
        block_excl_scan32(__popc(bits), s_w, total);
        if (threadIdx.x == 0) a.tile_count[tile] = total;
    }
}

// One workgroup: exclusive prefix of the tile counts, then each tree's point
// range (its image's first tile prefix and edge count).
__global__ __launch_bounds__(kScanThreads) void k_scan_counts(ExtractArgs a)
{
    __shared__ int64_t s_w[kScanThreads / kWave];
    __shared__ int64_t s_total;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t n = a.n_tiles;
    const int64_t chunk = cdiv(n, kScanThreads);
    const int64_t b = std::min<int64_t>(n, tid * chunk), e = std::min<int64_t>(n, b + chunk);
    int64_t sum = 0;
    for (int64_t t = b; t < e; ++t) sum += a.tile_count[t];
    const int64_t incl = wave_incl_scan64(sum, lane);
    if (lane == kWave - 1) s_w[wave] = incl;
    __syncthreads();
    int64_t run = incl - sum;
    for (int w = 0; w < wave; ++w) run += s_w[w];
    for (int64_t t = b; t < e; ++t) {
        a.tile_pre[t] = run;
        run += a.tile_count[t];
    }
    if (tid == kScanThreads - 1) s_total = run;
    __syncthreads();   // tile_pre is complete (workgroup-scope ordering of global memory)
    for (int t = tid; t < a.n_trees; t += kScanThreads) {
        const int k = a.trees[t].image;
        const int64_t lo = a.images[k].tile0 < n ? a.tile_pre[a.images[k].tile0] : s_total;
        const int64_t hi = k + 1 < a.n_images && a.images[k + 1].tile0 < n ? a.tile_pre[a.images[k + 1].tile0]
                                                                            : s_total;
        a.trees[t].xy_base = lo;
        a.trees[t].n_points = hi - lo;
        a.trees[t].image_points = (int32_t)(hi - lo);
    }
}

__global__ __launch_bounds__(kBlock) void k_extract_write(ExtractArgs a)
{
    __shared__ int32_t s_w[kWaves];
    for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const ImageDesc im = a.images[image_of_tile(a.images, a.n_images, tile)];
        int32_t row, col;
        const uint32_t bits =
            pixel_bits(im, (tile - im.tile0) * kPixTile + (int64_t)threadIdx.x * kPixPerThread, row, col);
        int32_t total;
        __syncthreads();
        int64_t pos = a.tile_pre[tile] + block_excl_scan32(__popc(bits), s_w, total);
        int32_t r = row, c = col;
        for (int k = 0; k < kPixPerThread; ++k) {
            if ((bits >> k) & 1u) a.xy[pos++] = pack_xy(c, r);
            if (++c == im.width) {
                c = 0;
                ++r;
            }
        }
    }
}

// Gray images (Sec. 3: the edge points are sorted into ALPHA and BETA while
// Sobel's gradient operator is applied).  A pixel with a full 3x3
// neighbourhood is an edge point iff Gx^2 + Gy^2 > t^2; the image line through
// it runs across the gradient, with slope -Gx/Gy, so it belongs to ALPHA
// (|slope| <= 1) iff |Gx| <= |Gy|.  Bits k of `a` / `b` mark the ALPHA / BETA
// edge points among a lane's kPixPerThread consecutive pixels.
__device__ inline void sobel_bits(const ImageDesc& im, int64_t p0, uint32_t& a, uint32_t& b, int32_t& row,
                                  int32_t& col)
{
    a = b = 0;
    row = col = 0;
    if (p0 >= im.n_pix) return;
    row = (int32_t)(p0 / im.width);
    col = (int32_t)(p0 - (int64_t)row * im.width);
    const int64_t t2 = (int64_t)im.edge_threshold * im.edge_threshold;
    int32_t r = row, c = col;
    for (int k = 0; k < kPixPerThread && p0 + k < im.n_pix; ++k) {
        if (r >= 1 && r + 1 < im.height && c >= 1 && c + 1 < im.width) {
            const uint8_t* const up = im.image + (int64_t)(r - 1) * im.row_stride + c;
            const uint8_t* const mid = up + im.row_stride;
            const uint8_t* const dn = mid + im.row_stride;
            const int32_t nw = up[-1], n = up[0], ne = up[1];
            const int32_t w = mid[-1], e = mid[1];
            const int32_t sw = dn[-1], s_ = dn[0], se = dn[1];
            const int32_t gx = (ne + 2 * e + se) - (nw + 2 * w + sw);
            const int32_t gy = (sw + 2 * s_ + se) - (nw + 2 * n + ne);
            if ((int64_t)gx * gx + (int64_t)gy * gy > t2) {
                if (abs(gx) > abs(gy)) b |= 1u << k;
                else a |= 1u << k;
            }
        }
        if (++c == im.width) {
            c = 0;
            ++r;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_sobel_count(SobelArgs a)
{
    __shared__ int32_t s_w[kWaves];
    for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const ImageDesc im = a.images[image_of_tile(a.images, a.n_images, tile)];
        uint32_t ba, bb;
        int32_t row, col;
        sobel_bits(im, (tile - im.tile0) * kPixTile + (int64_t)threadIdx.x * kPixPerThread, ba, bb, row, col);
        int32_t na, nb;
        __syncthreads();
        block_excl_scan32(__popc(ba), s_w, na);
        __syncthreads();
        block_excl_scan32(__popc(bb), s_w, nb);
        if (threadIdx.x == 0) {
            a.tile_count[tile] = na;
            a.tile_count[a.n_tiles + tile] = nb;
        }
    }
}

// One workgroup: the exclusive prefixes of both counts over the tiles, then
// each tree's range: pass 0 the image's ALPHA points, pass 1 its BETA points.
__global__ __launch_bounds__(kScanThreads) void k_sobel_scan(SobelArgs a)
{
    __shared__ int64_t s_w[kScanThreads / kWave];
    __shared__ int64_t s_total[2];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t n = a.n_tiles;
    const int64_t chunk = cdiv(n, kScanThreads);
    const int64_t b = std::min<int64_t>(n, tid * chunk), e = std::min<int64_t>(n, b + chunk);
    for (int set = 0; set < 2; ++set) {
        const int32_t* const cnt = a.tile_count + set * n;
        int64_t* const pre = a.tile_pre + set * n;
        int64_t sum = 0;
        for (int64_t t = b; t < e; ++t) sum += cnt[t];
        const int64_t incl = wave_incl_scan64(sum, lane);
        __syncthreads();   // s_w of the previous set has been read
        if (lane == kWave - 1) s_w[wave] = incl;
        __syncthreads();
        int64_t run = incl - sum;
        for (int w = 0; w < wave; ++w) run += s_w[w];
        for (int64_t t = b; t < e; ++t) {
            pre[t] = run;
            run += cnt[t];
        }
        if (tid == kScanThreads - 1) s_total[set] = run;
    }
    __syncthreads();   // tile_pre is complete (workgroup-scope ordering of global memory)
    const int64_t* const pa = a.tile_pre;
    const int64_t* const pb = a.tile_pre + n;
    for (int t = tid; t < a.n_trees; t += kScanThreads) {
        const int k = a.trees[t].image;
        const int64_t t0 = a.images[k].tile0, t1 = k + 1 < a.n_images ? a.images[k + 1].tile0 : n;
        const int64_t a0 = t0 < n ? pa[t0] : s_total[0], a1 = t1 < n ? pa[t1] : s_total[0];
        const int64_t b0 = t0 < n ? pb[t0] : s_total[1], b1 = t1 < n ? pb[t1] : s_total[1];
        const int64_t base = a0 + b0;   // points of the images before k
        a.trees[t].image_points = (int32_t)((a1 - a0) + (b1 - b0));
        if (a.trees[t].pass == 0) {
            a.trees[t].xy_base = base;
            a.trees[t].n_points = a1 - a0;
        } else {
            a.trees[t].xy_base = base + (a1 - a0);
            a.trees[t].n_points = b1 - b0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_sobel_write(SobelArgs a)
{
    __shared__ int32_t s_w[kWaves];
    const int64_t n = a.n_tiles;
    for (int64_t tile = blockIdx.x; tile < n; tile += gridDim.x) {
        const int k = image_of_tile(a.images, a.n_images, tile);
        const ImageDesc im = a.images[k];
        uint32_t ba, bb;
        int32_t row, col;
        sobel_bits(im, (tile - im.tile0) * kPixTile + (int64_t)threadIdx.x * kPixPerThread, ba, bb, row, col);
        const int64_t t0 = im.tile0, t1 = k + 1 < a.n_images ? a.images[k + 1].tile0 : n;
        const int64_t* const pa = a.tile_pre;
        const int64_t* const pb = a.tile_pre + n;
        // the image's ALPHA count: the prefix at its last tile plus that tile's count
        const int64_t a_img = pa[t1 - 1] + a.tile_count[t1 - 1] - pa[t0];
        const int64_t base = pa[t0] + pb[t0];
        int32_t tot;
        __syncthreads();
        const int32_t ra = block_excl_scan32(__popc(ba), s_w, tot);
        __syncthreads();
        const int32_t rb = block_excl_scan32(__popc(bb), s_w, tot);
        int64_t pos_a = base + (pa[tile] - pa[t0]) + ra;
        int64_t pos_b = base + a_img + (pb[tile] - pb[t0]) + rb;
        int32_t id_a = (int32_t)((pa[tile] - pa[t0]) + (pb[tile] - pb[t0]));   // rank among the image's edges
        int32_t r = row, c = col;
        int32_t seen = 0;
        // the lane's edges before pixel j, of both sets, come before it in the image
        int32_t id0 = 0;
        {
            __syncthreads();
            id0 = block_excl_scan32(__popc(ba | bb), s_w, tot);
        }
        for (int j = 0; j < kPixPerThread; ++j) {
            const uint32_t bit = 1u << j;
            if ((ba | bb) & bit) {
                const int32_t id = id_a + id0 + seen;
                if (ba & bit) {
                    a.xy[pos_a] = pack_xy(c, r);
                    a.ids[pos_a] = id;
                    ++pos_a;
                } else {
                    a.xy[pos_b] = pack_xy(c, r);
                    a.ids[pos_b] = id;
                    ++pos_b;
                }
                ++seen;
            }
            if (++c == im.width) {
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

__global__ void k_pack_points(const PointsDesc* lists, int32_t n_lists, int64_t n_total, uint32_t* xy,
                              uint32_t* error)
{
    bool bad = false;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_total;
         g += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = n_lists - 1;   // last list with base <= g
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (lists[mid].base <= g) lo = mid; else hi = mid - 1;
        }
        const PointsDesc d = lists[lo];
        const int64_t k = g - d.base;
        const int32_t xk = d.x[k], yk = d.y[k];
        const bool outside = (xk < 0) | (xk >= d.width) | (yk < 0) | (yk >= d.height);
        bad |= outside;
        xy[g] = outside ? 0u : pack_xy(xk, yk);
    }
    if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) raise_error(error, kErrPointRange | kErrInternal);
}

// Root setup: level 0 holds one region per tree whose root splits (every
// line crosses the root, code 0011, so it splits iff the tree has more than T
// points and depth > 0), its list the tree's points in input order.
// k_roots (one workgroup) lays the regions out; k_root_lists writes the lists
// and the tile map.
constexpr int kRootThreads = 1024;

__global__ __launch_bounds__(kRootThreads) void k_roots(Arena ar, const TreeDesc* trees, int32_t n_trees)
{
    __shared__ int64_t s_w[kRootThreads / kWave][2];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    constexpr int kPer = kMaxTrees / kRootThreads;   // trees per thread
    int64_t len[kPer], cnt = 0, sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int t = tid * kPer + k;
        len[k] = 0;
        if (t < n_trees) {
            const TreeDesc T = trees[t];
            if (T.n_points > T.threshold && T.dmax > 0) len[k] = T.n_points;
        }
        cnt += len[k] > 0;
        sum += len[k];
    }
    const int64_t ci = wave_incl_scan64(cnt, lane), si = wave_incl_scan64(sum, lane);
    if (lane == kWave - 1) {
        s_w[wave][0] = ci;
        s_w[wave][1] = si;
    }
    __syncthreads();
    int64_t r = ci - cnt, start = si - sum, P0 = 0, L0 = 0;
    for (int w = 0; w < kRootThreads / kWave; ++w) {
        if (w < wave) {
            r += s_w[w][0];
            start += s_w[w][1];
        }
        P0 += s_w[w][0];
        L0 += s_w[w][1];
    }
    if (tid == 0) {
        LevelInfo& in = ar.info[0];
        in.P = P0;
        in.L = L0;
        in.votes = 0;
        in.cells = 0;
        in.cells_base = 0;
        in.mem = 0;
        in.mem_base = 0;
    }
    if (P0 == 0) return;
    const HalfLayout hl = half_layout(ar.half[0], P0, L0, ar.entry_bytes);
    if (hl.end > ar.half_cap || work_layout(ar.work, P0, L0).end > ar.work_cap) {
        if (tid == 0) raise_error(ar.error, kErrArena);
        return;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int t = tid * kPer + k;
        if (len[k] == 0) continue;
        const TreeDesc T = trees[t];
        Region R;
        R.start = start;
        R.ij = 0;
        R.len = (int32_t)len[k];
        R.tree = t;
        R.meta = (T.pass ? kMetaPass : 0u) | ((uint32_t)T.s_log2 << kMetaSlogShift) |
                 (T.dmax == 1 ? kMetaChildFinest : 0u);
        G(hl.regions)[r] = R;
        G(hl.cc)[r] = code_consts(R.ij, R.meta, 1);
        reinterpret_cast<int4*>(G(hl.cv))[r] = int4{0, 0, 0, 0};
        ++r;
        start += len[k];
    }
}

template <typename Entry>
__global__ __launch_bounds__(kBlock) void k_root_lists(Arena ar, const TreeDesc* trees, const uint32_t* xy,
                                                        const int32_t* ids)
{
    __shared__ int64_t s_start[kMaxTrees];
    const uint32_t err = *G(ar.error);
    const int64_t P0 = ar.info[0].P, L0 = ar.info[0].L;
    if (stopped(err) || P0 == 0) return;
    const HalfLayout hl = half_layout(ar.half[0], P0, L0, ar.entry_bytes);
    const Region* const regions = G(static_cast<const Region*>(hl.regions));
    for (int64_t r = threadIdx.x; r < P0; r += kBlock) s_start[r] = regions[r].start;
    __syncthreads();
    auto region_of = [&](int64_t e) {   // last region with start <= e
        int lo = 0, hi = (int)P0 - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= e) lo = mid; else hi = mid - 1;
        }
        return lo;
    };
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    for (int64_t t = g; t < cdiv(L0, kTile); t += stride) G(hl.tile_first)[t] = region_of(t * kTile);
    Entry* const list = G(static_cast<Entry*>(hl.list));
    int cur = -1;
    int64_t lo = 0, hi = -1, base = 0;
    bool swap = false;
    for (int64_t e = g; e < L0; e += stride) {
        if (e < lo || e >= hi) {
            cur = region_of(e);
            const Region R = regions[cur];
            const TreeDesc T = trees[R.tree];
            lo = R.start;
            hi = R.start + R.len;
            base = T.xy_base;
            swap = T.pass != 0;
        }
        Entry v = EntryOps<Entry>::root(xy + base, e - lo, swap);
        if constexpr (sizeof(Entry) == 8)
            if (ids) v = (v & 0xFFFFFFFFull) | ((uint64_t)(uint32_t)ids[base + (e - lo)] << 32);
        list[e] = v;
    }
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
__global__ void k_member_ids(const Cell* cells, int64_t n_cells, const int64_t* dst_off, int64_t dst_base,
                             const Entry* src, const uint32_t* xy, int64_t n_points, int32_t* dst)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t c = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; c < n_cells;
         c += waves) {
        const Cell cell = cells[c];
        const Entry* s = src + cell.member_off;
        int32_t* d = dst + (dst_off ? dst_off[c] : cell.member_off - dst_base);
        for (int32_t k = lane; k < cell.votes; k += kWave) d[k] = entry_id(s[k], xy, n_points);
    }
}

__global__ void k_rebase_cells(const Cell* src, int64_t n, int64_t base, Cell* dst)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        Cell x = src[c];
        if (x.member_off >= 0) x.member_off -= base;
        dst[c] = x;
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

// The level kernels in their three forms: code variant with 32-bit or
// 64-bit compares, circle variant; entries of 4 or 8 bytes.
#define HH_LEVEL_LAUNCH(kernel)                                                                  \
    do {                                                                                         \
        const bool ids = a.ar.entry_bytes == 8;                                                  \
        if (variant == 1) {                                                                      \
            if (ids) kernel<uint64_t, 1, int64_t><<<grid, kBlock, 0, s>>>(a);                    \
            else kernel<uint32_t, 1, int64_t><<<grid, kBlock, 0, s>>>(a);                        \
        } else if (wide) {                                                                       \
            if (ids) kernel<uint64_t, 0, int64_t><<<grid, kBlock, 0, s>>>(a);                    \
            else kernel<uint32_t, 0, int64_t><<<grid, kBlock, 0, s>>>(a);                        \
        } else {                                                                                 \
            if (ids) kernel<uint64_t, 0, int32_t><<<grid, kBlock, 0, s>>>(a);                    \
            else kernel<uint32_t, 0, int32_t><<<grid, kBlock, 0, s>>>(a);                        \
        }                                                                                        \
    } while (0)

}  // namespace

hipError_t launch_clear(const Arena& ar, int64_t n_rec, hipStream_t s)
{
    k_clear<<<grid_for(std::max<int64_t>(n_rec, 256), kBlock, 1024), kBlock, 0, s>>>(ar, n_rec);
    return hipGetLastError();
}

hipError_t launch_pack_points(const PointsDesc* lists, int32_t n_lists, int64_t n_total, uint32_t* xy,
                              uint32_t* error, hipStream_t s)
{
    if (n_total <= 0) return hipSuccess;
    k_pack_points<<<grid_for(n_total, kBlock), kBlock, 0, s>>>(lists, n_lists, n_total, xy, error);
    return hipGetLastError();
}

hipError_t launch_sobel(const SobelArgs& a, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(a.n_tiles, 2048);
    k_sobel_count<<<grid, kBlock, 0, s>>>(a);
    k_sobel_scan<<<1, kScanThreads, 0, s>>>(a);
    k_sobel_write<<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_extract(const ExtractArgs& a, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(a.n_tiles, 2048);
    k_extract_count<<<grid, kBlock, 0, s>>>(a);
    k_scan_counts<<<1, kScanThreads, 0, s>>>(a);
    k_extract_write<<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_roots(const Arena& ar, const TreeDesc* trees, int32_t n_trees, const uint32_t* xy,
                        const int32_t* ids, int grid, hipStream_t s)
{
    if (n_trees > kMaxTrees) return hipErrorInvalidValue;
    k_roots<<<1, kRootThreads, 0, s>>>(ar, trees, n_trees);
    if (ar.entry_bytes == 8) k_root_lists<uint64_t><<<grid, kBlock, 0, s>>>(ar, trees, xy, ids);
    else k_root_lists<uint32_t><<<grid, kBlock, 0, s>>>(ar, trees, xy, nullptr);
    return hipGetLastError();
}

// Workgroups of the count / compaction kernels that fit on the device at
// once: each walks its share of the tiles, so a grid larger than what is
// resident would run in two rounds.
template <typename K>
int resident_grid(K kernel, int cu_count)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    return per_cu * cu_count;
}

#define HH_LEVEL_GRID(kernel)                                                                   \
    do {                                                                                        \
        if (variant == 1)                                                                       \
            return ids ? resident_grid(kernel<uint64_t, 1, int64_t>, cu_count)                  \
                       : resident_grid(kernel<uint32_t, 1, int64_t>, cu_count);                 \
        if (wide)                                                                               \
            return ids ? resident_grid(kernel<uint64_t, 0, int64_t>, cu_count)                  \
                       : resident_grid(kernel<uint32_t, 0, int64_t>, cu_count);                 \
        return ids ? resident_grid(kernel<uint64_t, 0, int32_t>, cu_count)                      \
                   : resident_grid(kernel<uint32_t, 0, int32_t>, cu_count);                     \
    } while (0)

int level_grid(int which, int variant, bool wide, int entry_bytes, int cu_count)
{
    const bool ids = entry_bytes == 8;
    if (which == 0) HH_LEVEL_GRID(k_count);
    return ids ? resident_grid(k_write<uint64_t>, cu_count) : resident_grid(k_write<uint32_t>, cu_count);
}

hipError_t launch_count(const LevelArgs& a, int variant, bool wide, int grid, hipStream_t s)
{
    HH_LEVEL_LAUNCH(k_count);
    return hipGetLastError();
}

hipError_t launch_decide(const LevelArgs& a, int grid, hipStream_t s)
{
    k_decide<<<std::min(grid, kRangeGrid), kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_emit(const LevelArgs& a, int grid, hipStream_t s)
{
    k_emit<<<std::min(grid, kRangeGrid), kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_write(const LevelArgs& a, int grid, hipStream_t s)
{
    if (a.ar.entry_bytes == 8) k_write<uint64_t><<<grid, kBlock, 0, s>>>(a);
    else k_write<uint32_t><<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_member_ids(const Cell* cells, int64_t n_cells, const int64_t* dst_off, int64_t dst_base,
                             const void* src, int entry_bytes, const uint32_t* xy, int64_t n_points, int32_t* dst,
                             hipStream_t s)
{
    if (n_cells <= 0) return hipSuccess;
    if (entry_bytes == 8)
        k_member_ids<uint64_t><<<grid_for(n_cells, kWaves), kBlock, 0, s>>>(
            cells, n_cells, dst_off, dst_base, static_cast<const uint64_t*>(src), xy, n_points, dst);
    else
        k_member_ids<uint32_t><<<grid_for(n_cells, kWaves), kBlock, 0, s>>>(
            cells, n_cells, dst_off, dst_base, static_cast<const uint32_t*>(src), xy, n_points, dst);
    return hipGetLastError();
}

hipError_t launch_rebase_cells(const Cell* src, int64_t n, int64_t base, Cell* dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_rebase_cells<<<grid_for(n, kBlock), kBlock, 0, s>>>(src, n, base, dst);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t* dst, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_iota<<<grid_for(n, kBlock), kBlock, 0, s>>>(dst, n);
    return hipGetLastError();
}

}  // namespace hh
