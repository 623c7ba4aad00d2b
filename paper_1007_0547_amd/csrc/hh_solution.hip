// solution() with point removal (Sec. 3) on gfx950.
//
// In the paper's depth-first search a detected finest cell calls solution():
// its voters are plotted (they form the output image) and their codes are
// zeroed at every level, so no region visited afterwards counts them.  The
// search visits cells in key order, and it reaches a cell whenever the cell
// itself has more than T unplotted voters (each ancestor, visited earlier with
// fewer points plotted, has at least those voters).  So the kept cells are
// those of a walk over the detected cells of the search without removal, in
// key order, that keeps a cell iff more than T of its voters are not yet
// plotted and then plots them.
//
// The walk is sequential by definition.  It runs here as a fixpoint of
// independent walks: a tree's cells are cut into segments of consecutive
// cells holding about equal numbers of voters (k_solution_cut), one
// workgroup each, and every segment walks its cells starting from
// an input set of points taken as plotted before it.  After a round, each
// segment's input becomes the union of the points the segments before it
// plotted in that round; when no input changes, every segment walked from
// exactly the points the cells before it plot, so the rounds reproduce the
// sequential walk (the first segment's input is always empty, so after r
// rounds the first r segments are exact, and at most one round per segment
// plus one is needed).  Kept cells are few and each one's influence reaches
// few segments, so a handful of rounds suffice in practice.
//
// One workgroup walks one segment.  It
// streams the segment's voter ids in windows of kSolCh entries held in registers
// (kSolR consecutive entries per lane, the next window's loaded while this one
// is processed).  Each lane tests its entries against the plotted set and
// stores its live bits into the window's live bitmap in LDS; the lane of each
// cell of the window counts the cell's live entries there (popcounts over its
// range), the first cell above T is plotted, and the window's remaining
// entries are tested again from registers until no cell of the window is above
// T.  A cell that runs past the window carries its count into the next one.
// The plotted set is a bitmap over the tree's point ids: in LDS when it fits,
// else in device memory behind atomics at workgroup scope (performed in L2,
// one copy for all waves of the workgroup).
//
// The walk of one segment runs on one compute unit and is bound by its vector
// ALU issue (the live test, the window setup) and by the latency of each
// window's loads; many segments fill the device.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <type_traits>

#include "hh_solution.hpp"

namespace hh {
namespace {

constexpr int kSolThreads = 1024;
constexpr int kSolWaves = kSolThreads / kWave;
constexpr int kSolR = 8;                        // voter entries per lane in a window
constexpr int kSolCh = kSolThreads * kSolR;     // entries per window
constexpr int kSolMaxCells = 256;               // cells per window, one per lane of the first lanes
constexpr int64_t kSolLdsBytes = 40 << 10;      // LDS for the plotted bitmap
constexpr int64_t kSolLdsPoints = kSolLdsBytes * 8;
// A lane's live bits are kSolR consecutive bits of the window's live bitmap.
using LaneBits = std::conditional_t<kSolR == 8, uint8_t, uint16_t>;
static_assert(kSolR == 8 || kSolR == 16, "a lane's live bits are one byte or one half-word");
static_assert(kSolMaxCells <= kSolThreads, "one lane per window cell");

template <typename T>
__device__ inline T* G(T* p)
{
    return (T*)(__attribute__((address_space(1))) T*)p;
}

// Loads and stores through global-address-space pointers: global (not flat)
// instructions count only in vmcnt, so a wait for an LDS read never waits for
// the next window's loads still in flight.
template <typename T>
__device__ inline T ldg(const T* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}

template <typename T>
__device__ inline void stg(T* p, T v)
{
    *(__attribute__((address_space(1))) T*)p = v;
}

// A workgroup barrier for data exchanged through LDS only: it does not wait
// for the wavefront's outstanding global loads (the next window's prefetch).
__device__ inline void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// With the bitmap in device memory the waves also exchange global data.
template <bool kLds>
__device__ inline void sol_barrier()
{
    if constexpr (kLds) lds_barrier();
    else __syncthreads();
}

template <bool kLds>
__device__ inline uint32_t bit_word(uint32_t* bits, int64_t w)
{
    if constexpr (kLds) return bits[w];
    else return __hip_atomic_fetch_or(G(bits) + w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Sets bits m of word w; returns the word before.
template <bool kLds>
__device__ inline uint32_t bit_set(uint32_t* bits, int64_t w, uint32_t m)
{
    if constexpr (kLds) return atomicOr(bits + w, m);
    else return __hip_atomic_fetch_or(G(bits) + w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The ids of window base ab held by this lane: ab + kSolR * tid + j (-1 past
// the buffer).
__device__ inline void load_ids(const int32_t* ids, int64_t n_slots, int64_t ab, int tid, int32_t (&v)[kSolR])
{
    const int64_t q0 = ab + (int64_t)kSolR * tid;
    const int64_t left = n_slots - q0;
    const int32_t* src = ids + q0;
    if (left >= kSolR) {
        typedef int v4i __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int g = 0; g < kSolR; g += 4) {
            const v4i x = ldg(reinterpret_cast<const v4i*>(src + g));
            v[g] = x.x;
            v[g + 1] = x.y;
            v[g + 2] = x.z;
            v[g + 3] = x.w;
        }
    } else {
        const int n = left > 0 ? (int)left : 0;
#pragma unroll
        for (int j = 0; j < kSolR; ++j) v[j] = j < n ? ldg(src + j) : -1;
    }
}

// Voter range of cell c (off, votes) and the start of the cell after it
// (next; -1: c is the last cell of the segment, which ends before c_end).
// Kept as loaded, so that a prefetch is not waited for before the values are
// used.
struct SolCell {
    int64_t off, next;
    int32_t votes;
};

__device__ inline SolCell load_cell(const SolTree& t, int64_t c, int64_t c_end)
{
    SolCell r{0, -1, 0};
    if (c < c_end) {
        r.off = ldg(&t.cells[c].member_off);
        r.votes = ldg(&t.cells[c].votes);
        if (c + 1 < c_end) r.next = ldg(&t.cells[c + 1].member_off);
    }
    return r;
}

// Live bits of this lane's entries (bit j: entry j is an id of the tree and
// not plotted); *valid gets the bits of entries that are ids of the tree.
// Entries before window position skip_below are not read.
template <bool kLds>
__device__ inline uint32_t live_bits(uint32_t* bits, const int32_t (&id)[kSolR], uint32_t n_points, int x0,
                                     int skip_below, uint32_t* valid)
{
    uint32_t m = 0, v = 0;
#pragma unroll
    for (int j = 0; j < kSolR; ++j) {
        const bool ok = (uint32_t)id[j] < n_points;   // negative ids wrap above n_points
        v |= (ok ? 1u : 0u) << j;
        const bool take = ok && x0 + j >= skip_below;
        if constexpr (kLds) {
            const uint32_t k = take ? (uint32_t)id[j] : 0u;   // LDS: read unconditionally, mask after
            m |= (take ? ((bits[k >> 5] >> (k & 31)) & 1u) ^ 1u : 0u) << j;
        } else if (take) {
            m |= (((bit_word<kLds>(bits, id[j] >> 5) >> (id[j] & 31)) & 1u) ^ 1u) << j;
        }
    }
    *valid = v;
    return m;
}

// Live entries of the window in positions [cs, ce), from the window's live
// bitmap (entry e is bit e % 32 of word e / 32).
__device__ inline int32_t live_in(const uint32_t* live, int32_t cs, int32_t ce)
{
    if (cs >= ce) return 0;
    const int32_t w0 = cs >> 5, w1 = (ce - 1) >> 5;
    int32_t n = 0;
    for (int32_t w = w0; w <= w1; ++w) {
        uint32_t v = live[w];
        if (w == w0) v &= ~0u << (cs & 31);
        if (w == w1 && (ce & 31)) v &= (1u << (ce & 31)) - 1u;
        n += __popc(v);
    }
    return n;
}

// The walks of the segments in list[0 .. *n_list), a workgroup taking list
// entries blockIdx.x, blockIdx.x + gridDim.x, ...; each walked segment
// lowers its tree's first_walked to its index.
template <bool kLds>
__global__ __launch_bounds__(kSolThreads) void k_solution(const SolTree* trees, const SolSeg* segs, const int32_t* list,
                                                           const int32_t* n_list, int32_t* first_walked,
                                                           uint32_t* error)
{
    extern __shared__ uint32_t s_bits[];
    __shared__ uint32_t s_live[kSolCh / 32];     // the window's live bitmap, kSolR bits per lane
    __shared__ int32_t s_cs[kSolMaxCells];       // window cells: first and end window position
    __shared__ int32_t s_ce[kSolMaxCells];
    __shared__ int32_t s_first[kSolWaves];
    __shared__ int64_t s_wend, s_off0;
    __shared__ int32_t s_nw, s_carry, s_last_done, s_bad_cells, s_bad_ids, s_bad_mark, s_plotted;

    const int32_t n_walk = ldg(n_list);
    for (int32_t li = blockIdx.x; li < n_walk; li += gridDim.x) {
    const int32_t si = ldg(list + li);
    const SolSeg sg = segs[si];
    const SolTree t = trees[sg.tree];
    const int64_t c_end = sg.c1;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    uint32_t* bits = kLds ? s_bits : sg.work;
    const int64_t words = (t.n_points + 31) >> 5;
    // the points plotted before the segment
    for (int64_t w = tid; w < words; w += kSolThreads) {
        if constexpr (kLds) s_bits[w] = ldg(sg.in + w);
        else stg(sg.work + w, ldg(sg.in + w));
    }
    if (tid == 0) {
        s_bad_cells = 0;
        s_bad_ids = 0;
        s_bad_mark = 0;
        s_plotted = 0;
        s_carry = 0;   // unplotted voters of the first undecided cell before pos
    }
    sol_barrier<kLds>();

    const int32_t T = t.threshold;
    const uint32_t n_points = (uint32_t)t.n_points;              // ids are 32-bit
    LaneBits* live_byte = reinterpret_cast<LaneBits*>(s_live) + tid;
    const int x0 = kSolR * tid;                                   // this lane's first window position
    int64_t c_cur = sg.c0;                                        // first undecided cell
    int64_t pos = c_cur < c_end ? ldg(&t.cells[c_cur].member_off) : 0;   // its first untested voter
    int64_t kept = 0;
    int32_t plotted = 0;                                          // bits this lane set
    bool bad = false;
    // this window's and the next window's cells and ids, loaded one window ahead
    SolCell cell = tid < kSolMaxCells ? load_cell(t, c_cur + tid, c_end) : SolCell{0, -1, 0};
    int32_t id[kSolR], nid[kSolR];
    if (c_cur < c_end) load_ids(t.ids, t.n_slots, pos & ~(int64_t)3, tid, nid);
    while (c_cur < c_end) {
        const int64_t ab = pos & ~(int64_t)3;   // window base, aligned for 16-byte loads
        const int64_t limit = ab + kSolCh;
        // The window's cells: c_cur and the cells that start before limit.  The
        // last one knows it is last: the cell after it starts at or past limit
        // (or there is none, or no lane for it).
        const int64_t c = c_cur + tid;
        const int64_t off = cell.off, end = cell.off + cell.votes;
        const int64_t next = cell.next < 0 ? end : cell.next;
        if (tid < kSolMaxCells && c < c_end) {
            const bool in = tid == 0 || off < limit;
            const bool ok = end > off && off >= 0 && end <= t.n_slots && next == end &&
                            (tid > 0 || (pos >= off && pos < end));
            if (in && !ok) s_bad_cells = 1;
            if (in && (tid == kSolMaxCells - 1 || c + 1 >= c_end || next >= limit)) {
                s_nw = tid + 1;
                s_wend = end < limit ? end : limit;
                s_last_done = end <= limit;
            }
        }
        if (tid == 0) s_off0 = off;
        // The window's entries and their live bits (every loaded entry; only
        // those of the window's cells are counted).
#pragma unroll
        for (int j = 0; j < kSolR; ++j) id[j] = nid[j];
        uint32_t valid = 0;
        uint32_t m = live_bits<kLds>(bits, id, n_points, x0, 0, &valid);
        *live_byte = (LaneBits)m;
        sol_barrier<kLds>();
        if (s_bad_cells) {
            bad = true;
            break;
        }
        const int32_t n_w = s_nw;
        const int32_t carry = s_carry;
        const int64_t w_end = s_wend;
        const bool last_done = s_last_done;
        const bool complete = tid < n_w && end <= w_end;
        int32_t cs = 0, ce = 0;
        if (tid < n_w) {
            cs = (int32_t)((off > pos ? off : pos) - ab);
            ce = (int32_t)((end < w_end ? end : w_end) - ab);
            s_cs[tid] = cs;
            s_ce[tid] = ce;
        }
        {   // every id of the window's cells must name a point of the tree
            const int64_t lo64 = pos - (ab + x0), hi64 = w_end - (ab + x0);
            const int lo = lo64 < 0 ? 0 : lo64 > kSolR ? kSolR : (int)lo64;
            const int hi = hi64 < 0 ? 0 : hi64 > kSolR ? kSolR : (int)hi64;
            const uint32_t in_cells = hi > lo ? ((1u << hi) - 1u) & ~((1u << lo) - 1u) : 0u;
            if (in_cells & ~valid) s_bad_ids = 1;
        }
        // Prefetch the next window (its first cell and base are known now).
        const int64_t c_next = last_done ? c_cur + n_w : c_cur + n_w - 1;
        if (c_next < c_end) {
            if (tid < kSolMaxCells) cell = load_cell(t, c_next + tid, c_end);
            load_ids(t.ids, t.n_slots, w_end & ~(int64_t)3, tid, nid);
        }
        // Take the first cell above T, plot it, test again; until none is left.
        int32_t k_from = 0, cnt = 0;
        bool my_keep = false;
        for (;;) {
            bool cand = false;
            if (tid < n_w) {
                cnt = live_in(s_live, cs, ce) + (tid == 0 ? carry : 0);
                cand = complete && tid >= k_from && cnt > T;
            }
            const uint64_t bc = __ballot(cand);
            if (lane == 0) s_first[wave] = bc ? wave * kWave + __ffsll((unsigned long long)bc) - 1 : INT_MAX;
            sol_barrier<kLds>();
            if (s_bad_ids) {
                bad = true;
                break;
            }
            int32_t f = INT_MAX;
#pragma unroll
            for (int w = 0; w < kSolWaves; ++w) f = s_first[w] < f ? s_first[w] : f;
            if (f == INT_MAX) break;
            // Plot cell f: its live voters in this window, and for a cell that
            // began in an earlier window, its voters before pos.
            const int32_t fs = s_cs[f], fe = s_ce[f];
#pragma unroll
            for (int j = 0; j < kSolR; ++j) {
                if (x0 + j >= fs && x0 + j < fe && ((m >> j) & 1u)) {
                    const uint32_t b = 1u << (id[j] & 31);
                    plotted += (bit_set<kLds>(bits, id[j] >> 5, b) & b) ? 0 : 1;
                }
            }
            if (f == 0 && s_off0 < pos) {
                for (int64_t q = s_off0 + tid; q < pos; q += kSolThreads) {
                    const int32_t p = ldg(t.ids + q);
                    if (p < 0 || (int64_t)p >= t.n_points) {
                        s_bad_mark = 1;
                        continue;
                    }
                    const uint32_t b = 1u << (p & 31);
                    plotted += (bit_set<kLds>(bits, p >> 5, b) & b) ? 0 : 1;
                }
            }
            my_keep = my_keep || tid == f;
            ++kept;
            k_from = f + 1;
            sol_barrier<kLds>();
            if (s_bad_mark) {
                bad = true;
                break;
            }
            // entries up to cell f's end are decided; test the rest again
            m = live_bits<kLds>(bits, id, n_points, x0, fe, &valid);
            *live_byte = (LaneBits)m;
            sol_barrier<kLds>();
        }
        if (bad) break;
        // The next window reads the carry after its first barrier, and writes
        // its tables only after that barrier, when every lane is done with
        // this window's.
        if (tid == n_w - 1) s_carry = last_done ? 0 : cnt;
        if (complete) stg(t.keep + c, (uint8_t)(my_keep ? 1 : 0));
        c_cur = c_next;
        pos = w_end;
    }

    // Output: the points this segment plotted (beyond its input), its kept
    // cells and plotted points.
    for (int d = kWave / 2; d > 0; d >>= 1) plotted += __shfl_xor(plotted, d, kWave);
    if (lane == 0) atomicAdd(&s_plotted, plotted);
    sol_barrier<kLds>();
    for (int64_t w = tid; w < words; w += kSolThreads) stg(sg.out + w, bit_word<kLds>(bits, w) & ~ldg(sg.in + w));
    if (tid == 0) {
        stg(sg.counts, kept);
        stg(sg.counts + 1, (int64_t)s_plotted);
        atomicMin(first_walked + sg.tree, si);
        if (bad) __hip_atomic_fetch_or(G(error), kErrInternal, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    sol_barrier<kLds>();   // the next segment sets up the workgroup's tables again
    }
}

// After a round: in each tree with a walked segment, the input of every
// segment becomes the union of what the segments before it plotted (an
// exclusive OR-scan over the tree's segments, one thread per segment, for
// kMergeWords bitmap words per workgroup), and the tree's `all` the union of
// every segment's; a segment whose input changed is marked in changed[].
constexpr int kMergeThreads = kSolMaxSegs;   // one thread per segment of a tree
constexpr int kMergeWords = 4;

__global__ __launch_bounds__(kMergeThreads) void k_solution_merge(const SolTree* trees, const SolSeg* segs,
                                                                  int64_t blocks_per_tree,
                                                                  const int32_t* first_walked, uint8_t* changed)
{
    __shared__ uint32_t s_wave[kMergeThreads / kWave];
    const int32_t k = (int32_t)(blockIdx.x / blocks_per_tree);
    const int64_t w0 = (blockIdx.x - (int64_t)k * blocks_per_tree) * kMergeWords;
    const SolTree& t = trees[k];
    const int32_t f = ldg(first_walked + k);
    const int64_t words = (t.n_points + 31) >> 5;
    if (f < t.seg0 || f >= t.seg0 + t.n_segs || w0 >= words) return;   // uniform: nothing walked here
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const bool mine = tid < t.n_segs;
    const SolSeg* sg = segs + t.seg0 + (mine ? tid : 0);
    bool moved = false;
    for (int64_t w = w0; w < w0 + kMergeWords && w < words; ++w) {
        const uint32_t o = mine ? ldg(sg->out + w) : 0u;
        // inclusive OR-scan within the wave, then across the waves
        uint32_t x = o;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)x, d, kWave);
            if (lane >= d) x |= y;
        }
        if (lane == kWave - 1) s_wave[wave] = x;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int v = 0; v < kMergeThreads / kWave; ++v) {
            if (v < wave) before |= s_wave[v];
            total |= s_wave[v];
        }
        __syncthreads();   // s_wave is rewritten for the next word
        const uint32_t below = (uint32_t)__shfl_up((int)x, 1, kWave);   // inclusive scan of the lane before
        const uint32_t in_new = before | (lane > 0 ? below : 0u);
        if (mine && ldg(sg->in + w) != in_new) {
            stg(sg->in + w, in_new);
            moved = true;
        }
        if (tid == 0) stg(t.all + w, total);
    }
    if (moved) stg(changed + t.seg0 + tid, (uint8_t)1);
}

// The next round's lists: the segments marked changed (marks cleared), LDS
// segments (index < n_lds) and device-bitmap ones apart, appended at the
// counters n_next[0] and n_next[1] (zero before); every tree's first_walked
// goes back to INT_MAX.
__global__ void k_solution_collect(int32_t n_segs, int32_t n_lds, uint8_t* changed, int32_t* next_lds,
                                   int32_t* next_dev, int32_t* n_next, int32_t* first_walked, int32_t n_trees)
{
    const int64_t n = n_segs > n_trees ? n_segs : n_trees;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        if (q < n_trees) stg(first_walked + q, (int32_t)INT_MAX);
        if (q < n_segs && ldg(changed + q)) {
            stg(changed + q, (uint8_t)0);
            if (q < n_lds) next_lds[atomicAdd(n_next, 1)] = (int32_t)q;
            else next_dev[atomicAdd(n_next + 1, 1)] = (int32_t)q;
        }
    }
}

// Once no input changes: per tree, the plotted flag of every point and the
// kept cells and plotted points over its segments.
__global__ void k_solution_finish(const SolTree* trees, int32_t n_trees, const SolSeg* segs)
{
    const SolTree& t = trees[blockIdx.x];
    for (int64_t k = threadIdx.x; k < t.n_points; k += blockDim.x)
        stg(t.plotted + k, (uint8_t)((ldg(t.all + (k >> 5)) >> (k & 31)) & 1u));
    if (threadIdx.x == 0) {
        int64_t kept = 0, plotted = 0;
        for (int32_t s = t.seg0; s < t.seg0 + t.n_segs; ++s) {
            kept += ldg(segs[s].counts);
            plotted += ldg(segs[s].counts + 1);
        }
        stg(t.counts, kept);
        stg(t.counts + 1, plotted);
    }
}

// Segment bounds of every tree by voter entries: segment q of K starts at
// the first cell whose voters start at or past q / K of the tree's entries
// (cells hold very different numbers of voters, and a round lasts as long as
// its longest walk).  One thread per segment; member_off grows from cell to
// cell (voters are back to back), so a binary search finds each bound.  An
// empty segment (one cell holding two bounds) walks nothing.
__global__ void k_solution_cut(const SolTree* trees, SolSeg* segs, int32_t n_segs)
{
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_segs) return;
    const SolTree t = trees[segs[g].tree];
    const int64_t q = g - t.seg0, K = t.n_segs, n = t.n_cells;
    if (n <= 0 || K <= 0) return;
    const int64_t first = ldg(&t.cells[0].member_off);
    const int64_t total = ldg(&t.cells[n - 1].member_off) + ldg(&t.cells[n - 1].votes) - first;
    auto bound = [&](int64_t k) -> int64_t {
        if (k <= 0) return 0;
        if (k >= K) return n;
        const int64_t target = first + total * k / K;
        int64_t lo = 0, hi = n;   // first cell with member_off >= target
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (ldg(&t.cells[mid].member_off) < target) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    segs[g].c0 = bound(q);
    segs[g].c1 = bound(q + 1);
}

// The rank table of an image's edge points: table[y * W + x] = k for
// xy[k] = x | y << 16.
__global__ void k_pixel_rank(const uint32_t* xy, int64_t n_points, int32_t width, int32_t height, int32_t* table)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_points;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = ldg(xy + k);
        const int32_t x = (int32_t)(p & 0xFFFFu), y = (int32_t)(p >> 16);
        if (x < width && y < height) stg(table + (int64_t)y * width + x, (int32_t)k);
    }
}

__global__ void k_ids_by_pixel(const int32_t* table, int32_t width, int32_t height, const uint32_t* src,
                               int64_t n_slots, int32_t* dst)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_slots;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = ldg(src + e);
        const int32_t x = (int32_t)(p & 0xFFFFu), y = (int32_t)(p >> 16);
        stg(dst + e, x < width && y < height ? ldg(table + (int64_t)y * width + x) : -1);
    }
}

// One wavefront per cell; kept cells paint their voters.
template <typename Entry>
__global__ void k_paint(const Cell* cells, int64_t n_cells, const uint8_t* keep, const Entry* members,
                        int32_t width, int32_t height, uint8_t* image)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t c = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; c < n_cells; c += waves) {
        if (!ldg(keep + c)) continue;
        const int64_t off = ldg(&cells[c].member_off);
        const int32_t votes = ldg(&cells[c].votes);
        for (int32_t k = lane; k < votes; k += kWave) {
            const uint32_t p = (uint32_t)ldg(members + off + k);
            const int32_t x = (int32_t)(p & 0xFFFFu), y = (int32_t)(p >> 16);
            if (x < width && y < height) stg(image + (int64_t)y * width + x, (uint8_t)255);
        }
    }
}

}  // namespace

hipError_t launch_paint(const Cell* cells, int64_t n_cells, const uint8_t* keep, const void* members,
                        int entry_bytes, int32_t width, int32_t height, uint8_t* image, hipStream_t s)
{
    if (n_cells <= 0) return hipSuccess;
    constexpr int kThreads = 256;
    const int grid = (int)std::min<int64_t>((n_cells + kThreads / kWave - 1) / (kThreads / kWave), 4096);
    if (entry_bytes == 8)
        k_paint<uint64_t><<<grid, kThreads, 0, s>>>(cells, n_cells, keep, static_cast<const uint64_t*>(members),
                                                     width, height, image);
    else
        k_paint<uint32_t><<<grid, kThreads, 0, s>>>(cells, n_cells, keep, static_cast<const uint32_t*>(members),
                                                     width, height, image);
    return hipGetLastError();
}

hipError_t launch_ids_by_pixel(const uint32_t* xy, int64_t n_points, int32_t width, int32_t height,
                               int32_t* table, const uint32_t* src, int64_t n_slots, int32_t* dst, hipStream_t s)
{
    constexpr int kThreads = 256;
    auto grid = [](int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + kThreads - 1) / kThreads, 1), 8192); };
    if (n_points > 0) k_pixel_rank<<<grid(n_points), kThreads, 0, s>>>(xy, n_points, width, height, table);
    if (n_slots > 0) k_ids_by_pixel<<<grid(n_slots), kThreads, 0, s>>>(table, width, height, src, n_slots, dst);
    return hipGetLastError();
}

int64_t solution_lds_points() { return kSolLdsPoints; }

hipError_t launch_solution_round(const SolRound& r, hipStream_t s)
{
    if (r.max_lds_points > kSolLdsPoints) return hipErrorInvalidValue;
    if (r.n_lds > 0) {
        const size_t lds = (size_t)((r.max_lds_points + 31) >> 5) * 4;
        k_solution<true><<<std::min(r.n_lds, r.grid), kSolThreads, lds, s>>>(r.trees, r.segs, r.list_lds, r.n_list,
                                                                            r.first_walked, r.error);
    }
    if (r.n_segs > r.n_lds)
        k_solution<false><<<std::min(r.n_segs - r.n_lds, r.grid), kSolThreads, 0, s>>>(
            r.trees, r.segs, r.list_dev, r.n_list + 1, r.first_walked, r.error);
    const int64_t per_tree = (r.max_words + kMergeWords - 1) / kMergeWords;
    if (r.n_trees > 0 && per_tree > 0)
        k_solution_merge<<<(unsigned)(r.n_trees * per_tree), kMergeThreads, 0, s>>>(r.trees, r.segs, per_tree,
                                                                                    r.first_walked, r.changed);
    hipError_t e = hipMemsetAsync(r.n_next, 0, 8, s);
    if (e != hipSuccess) return e;
    const int64_t m = std::max<int64_t>(r.n_segs, r.n_trees);
    if (m > 0)
        k_solution_collect<<<(int)std::min<int64_t>((m + 255) / 256, 4096), 256, 0, s>>>(
            r.n_segs, r.n_lds, r.changed, r.next_lds, r.next_dev, r.n_next, r.first_walked, r.n_trees);
    return hipGetLastError();
}

hipError_t launch_solution_cut(const SolTree* trees, SolSeg* segs, int32_t n_segs, hipStream_t s)
{
    if (n_segs <= 0) return hipSuccess;
    k_solution_cut<<<(n_segs + 255) / 256, 256, 0, s>>>(trees, segs, n_segs);
    return hipGetLastError();
}

hipError_t launch_solution_finish(const SolTree* trees, int32_t n_trees, const SolSeg* segs, hipStream_t s)
{
    if (n_trees <= 0) return hipSuccess;
    k_solution_finish<<<n_trees, 256, 0, s>>>(trees, n_trees, segs);
    return hipGetLastError();
}

}  // namespace hh
