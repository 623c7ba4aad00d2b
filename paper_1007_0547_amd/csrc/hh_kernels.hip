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
//             not 0000 / 1111, Sec. 3) as wavefront lane masks, counted per
//             task (a run of one region's list) and summed per region.
//   k_decide  per region: the split decisions (votes > T, Sec. 3) and their
//             sums per range of regions.
//   k_emit    per region: offsets from those sums; the next level's region
//             table in quad order (so key order is kept) and its tasks, or
//             the detected cells at the finest level.
//   k_write   a second read of every entry of a region with a kept child:
//             each vote for a kept child is written, in list order, to that
//             child's list in the next level (or to the member buffer at the
//             finest level).
//
// Level sizes never travel to the host: each launch reads them from the
// arena's LevelInfo records written by the launches before it.  The list
// launches run a resident grid whose wavefronts draw tasks until the
// level's are all taken; the others walk their work with a fixed grid.  No
// launch waits on another workgroup.

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

// Element k of an array no launch writes while the caller runs, read through
// the constant address space: with a wavefront-uniform index the compiler
// emits a scalar load into scalar registers.
template <typename T>
__device__ __forceinline__ T ld_const(const T* p, int64_t k)
{
#if __HIP_DEVICE_COMPILE__
    return ((const __attribute__((address_space(4))) T*)p)[k];
#else
    return p[k];   // the host pass only parses device code
#endif
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

// The first internal failure of a call leaves its check, level and six
// values in the arena's scratch words (slot 0 is the claim), which the host
// reads back with the level records and puts in the error message.
__device__ inline void record_failure(int64_t* scratch, uint32_t at, int level, int64_t a, int64_t b, int64_t c,
                                      int64_t d, int64_t e)
{
    unsigned long long* const claim = reinterpret_cast<unsigned long long*>(G(scratch));
    if (atomicCAS(claim, 0ull, 1ull) != 0ull) return;
    int64_t* const v = G(scratch);
    v[1] = (int64_t)at | ((int64_t)level << 32);
    v[2] = a;
    v[3] = b;
    v[4] = c;
    v[5] = d;
    v[6] = e;
}

// set bits of b at lanes below this lane
__device__ inline uint32_t lanes_below(uint64_t b)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
}

__device__ inline uint64_t bits_below(int p) { return ((uint64_t)1 << p) - 1; }   // p in 0..63

// acc + (this lane's bit of mask): one vector add with the mask as its
// carry-in (the compiler makes a select and an add of `acc + bit`); no
// memory access in the asm
__device__ __forceinline__ int32_t add_lane_bit(int32_t acc, uint64_t mask)
{
    int32_t out;
    uint64_t carry;
    asm("v_addc_co_u32_e64 %0, %1, %2, 0, %3" : "=v"(out), "=s"(carry) : "v"(acc), "s"(mask));
    return out;
}

// This lane's bit of a wavefront-uniform lane mask, as a lane predicate: the
// mask itself serves as the execution mask, with no vector instruction.
__device__ inline bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

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

// A region's part of the vote test, computed once per task and kept in
// scalar registers; masks() evaluates a whole row of lines against it as lane
// masks, one per child (see code_masks and circle_masks).
template <int kVariant, typename CT>
struct RegionTest {
    uint32_t ij, meta;
    CT M0, B0, B1, B2;      // code variant: scaled corner values of the children's grid
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
    // |u| < 2^14 and |M0| <= 2^15: a 24-bit multiply is exact for 32-bit compares
    __device__ static CT mul(CT u, CT m)
    {
        if constexpr (sizeof(CT) == 4) return __mul24(u, m);
        else return u * m;
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

// ------------------------------------------------------------------ tasks
//
// A level's list is cut into tasks: up to task_steps consecutive steps of
// one region's list, a step being 512 entries.  A wavefront takes tasks one
// after another -- from a fixed share (task = its wavefront index + k * all
// wavefronts of the grid) or from the level's work queue (an atomic head in
// its LevelInfo, queue_batch tasks at a time, the next batch requested while
// the current one runs) -- and streams a task one chunk of rows at a time,
// the next chunk's entries already in flight while it tests the current
// one.  All lines of a task belong to one region, so the region's
// part of the vote test is wavefront-uniform and sits in scalar registers,
// and a row is one test per lane.  Workgroups share nothing: a workgroup is
// only a unit of launch.

__device__ inline uint32_t rfl(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// Task ids of one wavefront.
struct TaskFeed {
    int64_t* head;
    int64_t NT, cur, end, stride;
    int64_t req;     // queue mode, lane 0: start of the batch requested in advance
    int32_t batch;   // 0: fixed share

    __device__ __forceinline__ int64_t request() const
    {
        int64_t v = 0;
        if ((threadIdx.x & (kWave - 1)) == 0)
            v = (int64_t)__hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(G(head)),
                                                (unsigned long long)batch, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
        return v;
    }
    __device__ __forceinline__ void init(int64_t* h, int64_t nt, int32_t b, int64_t wave_id, int64_t waves)
    {
        head = h;
        NT = nt;
        batch = b;
        stride = waves;
        req = 0;
        if (batch <= 0) {
            cur = wave_id;
            end = 0;
        } else {
            cur = (int64_t)uniform64((uint64_t)request());
            end = cur + batch;
            req = request();
        }
    }
    // the next task id (wavefront-uniform), or -1 when the level's tasks are
    // all taken
    __device__ __forceinline__ int64_t take()
    {
        int64_t t;
        if (batch <= 0) {
            t = cur;
            cur += stride;
        } else {
            if (cur >= end && cur < NT) {
                cur = (int64_t)uniform64((uint64_t)req);
                end = cur + batch;
                if (cur < NT) req = request();
            }
            t = cur;
            if (cur < NT) ++cur;
        }
        return (int64_t)uniform64((uint64_t)(t < NT ? t : -1));
    }
};

// A task as a wavefront sees it (all fields wavefront-uniform).
struct TaskView {
    int64_t t;       // task id
    int64_t b;       // first entry in the level's list
    int32_t n;       // entries
    int32_t r;       // region
    int32_t c;       // task index within the region
    bool last;       // the region's last task
};

// Reads task t (scalar loads); false if its fields are out of range.
__device__ __forceinline__ bool view_task(const Task* tasks, const Region* regions, int64_t P, int64_t L,
                                          int64_t task_len, int64_t t, TaskView& v)
{
    const Task tk = ld_const(tasks, t);
    v.t = t;
    v.r = tk.r;
    v.c = tk.c;
    if (tk.r < 0 || tk.r >= P || tk.c < 0 || tk.c > t) return false;
    const Region R = ld_const(regions, (int64_t)tk.r);
    const int64_t off = (int64_t)tk.c * task_len;
    if (off >= R.len || R.start < 0 || R.start + R.len > L) return false;
    v.b = R.start + off;
    v.n = (int32_t)std::min<int64_t>(task_len, R.len - off);
    v.last = off + task_len >= R.len;
    return true;
}

// The region's indices and meta bits (read when its task becomes current, so
// they do not occupy registers while the previous task runs).
__device__ __forceinline__ void region_code(const Region* regions, int32_t r, uint32_t& ij, uint32_t& meta)
{
    const Region R = ld_const(regions, (int64_t)r);
    ij = R.ij;
    meta = R.meta;
}

// An entry whose line votes for no region in the code variant: u = 0,
// v = 65535 is the horizontal parameter line b = 65535, above every corner
// (b <= 2S <= 32768), so every corner is below it (code 1111).  Lanes past a
// task's end hold it and need no mask.  The circle variant masks them.
template <typename Entry, int kVariant>
__device__ constexpr Entry pad_entry()
{
    return kVariant == 0 ? (Entry)0xFFFF0000u : (Entry)0;
}

// A wavefront holds a chunk of R rows of 64 entries of a task in registers,
// and loads the next chunk while it tests this one.  k_count keeps 8 rows;
// k_write, with more arithmetic per row, keeps 16 rows of 4-byte entries
// (8 KB of the list in flight per wavefront) and 8 of 8-byte ones.  Measured
// on the 4096x4096 image and the 512-image batch, each choice was the
// faster of the two for its kernel.
constexpr int kCountRows = 8;
template <typename Entry>
constexpr int kWriteRows = sizeof(Entry) == 4 ? 16 : 8;

// Entries of chunk s (R rows) of a task (n entries from b); a full chunk
// loads without lane masks.
template <int R, typename Entry, int kVariant>
__device__ __forceinline__ void load_chunk(const Entry* list, int64_t b, int32_t n, int s, int lane, Entry (&ent)[R])
{
    constexpr int kChunk = R * kWave;
    const Entry* const p = list + b + (int64_t)s * kChunk;
    const int32_t rem = n - s * kChunk;
    if (rem >= kChunk) {
#pragma unroll
        for (int k = 0; k < R; ++k) ent[k] = p[k * kWave + lane];
    } else {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int32_t o = k * kWave + lane;
            ent[k] = o < rem ? p[o] : pad_entry<Entry, kVariant>();
        }
    }
}

// Valid lanes of row k of a step with rem entries left (circle variant only).
__device__ inline uint64_t row_mask(int32_t rem, int k)
{
    const int32_t left = rem - k * kWave;
    return left >= kWave ? ~0ull : (left <= 0 ? 0ull : bits_below(left));
}

// ------------------------------------------------------------------ k_count
//
// One read of every entry: per task, the votes of its lines for each child
// of its region (the 4-bit code of Sec. 2 and the vote rule of Sec. 3 as
// lane masks).  Each lane counts its own votes per child, one vector add
// with carry-in per row and child, and the task's four counts are summed over the
// wavefront at its end: this keeps the per-row work on the vector unit,
// which issues as often as the scalar unit but had slack.  A task stores its
// four counts (for the ranks of the compaction pass) and adds them to its
// region's totals: a plain store when it is the region's only task, atomics
// otherwise.

template <int R, typename Entry, int kVariant, typename CT, bool kFull>
__device__ __forceinline__ void count_rows(const RegionTest<kVariant, CT>& rt, const Entry (&ent)[R], int32_t rem,
                                           int lc, int32_t (&lacc)[4])
{
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if (!kFull && k * kWave >= rem) break;
        const uint64_t vm = (kFull || kVariant == 0) ? ~0ull : row_mask(rem, k);
        uint64_t cm[4];
        rt.masks(vm, EntryOps<Entry>::point(ent[k]), lc, cm);
#pragma unroll
        for (int q = 0; q < 4; ++q) lacc[q] = add_lane_bit(lacc[q], cm[q]);
    }
}

// The rows of a chunk with rem entries left in the task: a full chunk runs
// without per-row bounds.
template <int R, typename Entry, int kVariant, typename CT>
__device__ __forceinline__ void count_chunk(const RegionTest<kVariant, CT>& rt, const Entry (&ent)[R], int32_t rem,
                                            int lc, int32_t (&lacc)[4])
{
    if (rem >= R * kWave) count_rows<R, Entry, kVariant, CT, true>(rt, ent, rem, lc, lacc);
    else count_rows<R, Entry, kVariant, CT, false>(rt, ent, rem, lc, lacc);
}

// The four per-lane counts summed over the wavefront (every lane gets the
// sums).  Two counts share a 32-bit word, 16 bits each: a task's count for
// one child is at most its length, kMaxTaskSteps * kStep = 32768 < 2^16.
__device__ __forceinline__ void wave_sum4(const int32_t (&x)[4], int32_t (&sum)[4])
{
    static_assert(kMaxTaskSteps * kStep < (1 << 16), "a task's count must fit 16 bits");
    uint32_t a = (uint32_t)x[0] | ((uint32_t)x[1] << 16);
    uint32_t b = (uint32_t)x[2] | ((uint32_t)x[3] << 16);
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        a += (uint32_t)__shfl_xor((int)a, d, kWave);
        b += (uint32_t)__shfl_xor((int)b, d, kWave);
    }
    sum[0] = (int32_t)(a & 0xFFFFu);
    sum[1] = (int32_t)(a >> 16);
    sum[2] = (int32_t)(b & 0xFFFFu);
    sum[3] = (int32_t)(b >> 16);
}

template <typename Entry, int kVariant, typename CT>
__global__ __launch_bounds__(kBlock) void k_count(LevelArgs a)
{
    const Arena& ar = a.ar;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = (int)rfl(threadIdx.x / kWave);
    const int l = a.level;
    const int lc = l + 1;
    const uint32_t err = *G(ar.error);
    LevelInfo* const info = ar.info + l;
    const int64_t P = info->P, L = info->L, NT = info->NT, steps = info->task_steps;
    if (stopped(err) || P == 0) return;
    const HalfLayout hl = half_layout(ar.half[l & 1], P, L, NT, ar.entry_bytes);
    const WorkLayout wl = work_layout(ar.work, P, NT);
    if (hl.end > ar.half_cap || wl.end > ar.work_cap || steps < 1 || steps > kMaxTaskSteps) {
        if (threadIdx.x == 0 && blockIdx.x == 0) raise_error(ar.error, kErrArena);
        return;
    }
    const Entry* const list = G(static_cast<const Entry*>(hl.list));
    const Region* const regions = G(static_cast<const Region*>(hl.regions));
    const Task* const tasks = G(static_cast<const Task*>(hl.tasks));
    int32_t* const cv = G(hl.cv);
    int32_t* const tcnt = G(wl.tcnt);
    const int64_t task_len = steps * kStep;

    TaskFeed feed;
    feed.init(&info->queue[0], NT, a.queue_batch, (int64_t)blockIdx.x * kWaves + wave, (int64_t)gridDim.x * kWaves);
    TaskView cur;
    {
        const int64_t t = feed.take();
        if (t < 0) return;
        if (!view_task(tasks, regions, P, L, task_len, t, cur)) {
            if (lane == 0) raise_error(ar.error, kErrInternal | kErrAtCountTask | (1u << (kErrLevelShift + l)));
            return;
        }
    }
    RegionTest<kVariant, CT> rt;
    {
        uint32_t ij, meta;
        region_code(regions, cur.r, ij, meta);
        rt.set(ij, meta, lc);
    }
    constexpr int R = kCountRows;
    Entry ent[R];
    load_chunk<R, Entry, kVariant>(list, cur.b, cur.n, 0, lane, ent);
    int s = 0;
    int32_t lacc[4] = {0, 0, 0, 0};    // this lane's votes per child in this task
    for (;;) {
        // the next chunk: this task's, or the first of the next task
        const bool more = (s + 1) * R * kWave < cur.n;
        TaskView nxt;
        bool have_next = false;
        Entry nent[R];
        if (more) {
            load_chunk<R, Entry, kVariant>(list, cur.b, cur.n, s + 1, lane, nent);
        } else {
            const int64_t t = feed.take();
            if (t >= 0) {
                if (!view_task(tasks, regions, P, L, task_len, t, nxt)) {
                    if (lane == 0) raise_error(ar.error, kErrInternal | kErrAtCountTask | (1u << (kErrLevelShift + l)));
                    return;
                }
                have_next = true;
                load_chunk<R, Entry, kVariant>(list, nxt.b, nxt.n, 0, lane, nent);
            }
        }
        count_chunk<R, Entry, kVariant, CT>(rt, ent, cur.n - s * R * kWave, lc, lacc);
        if (more) {
            ++s;
        } else {
            // the task's counts (ranks of the compaction pass) and the
            // region's totals: a plain store for a one-task region, else atomics
            int32_t acc[4];
            wave_sum4(lacc, acc);
            if (lane < 4) {
                const int32_t v = pick4(acc, lane);
                tcnt[cur.t * 4 + lane] = v;
                if (cur.c == 0 && cur.last) cv[(int64_t)cur.r * 4 + lane] = v;
                else if (v) atomicAdd(&cv[(int64_t)cur.r * 4 + lane], v);
            }
            if (!have_next) break;
            {
                uint32_t ij, meta;
                region_code(regions, nxt.r, ij, meta);
                rt.set(ij, meta, lc);
            }
            cur = nxt;
            s = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) lacc[q] = 0;
        }
#pragma unroll
        for (int k = 0; k < R; ++k) ent[k] = nent[k];
    }
}

// ------------------------------------------------------------------ k_write
//
// Second read of every entry of a region with a kept child.  A vote of the
// entry for kept child q of its region r goes to dst[r][q] + its rank among
// the votes of r for q in list order: the votes counted by the region's
// earlier tasks (summed from tcnt), plus those of the earlier rows of this
// task (a running count in scalar registers), plus the voting lanes below
// it in its row (mbcnt).  No store leaves the destination buffer: a task
// whose every kept child has room in the buffer for all of the task's
// entries stores without further checks (a task of n entries adds at most
// n votes to a child); any other task checks each row's run against the
// region's slots and drops a run that would leave them.  The region's last
// task checks that each kept child got exactly its count, else the call
// fails with an internal error.  Tasks of regions without a kept child are
// skipped without reading their entries.

// Kept children of a task's region.  The emit step lays a region's kept
// children out one after another in quad order (in the next level's list, or
// in the member buffer at the finest level), so one base pointer serves all
// four: pos[q] is the slot (counted from base) of the next vote for child q.
template <typename Entry>
struct Kids {
    Entry* base;
    int32_t pos[4];
    int32_t total;      // votes of the kept children: the region's slots are [0, total)
    uint32_t keep;      // bit q: child q's voters are kept
    bool unswap;        // member entries are stored as (x, y) whatever the pass
    bool roomy;         // every kept child has room in the buffer for the whole task
};

// Where each kept child's slot starts (from the first kept child's) and
// the region's kept votes.
__device__ __forceinline__ void kid_slots(const int32_t (&c)[4], uint32_t keep, int32_t (&lo)[4], int32_t& total)
{
    total = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        lo[q] = total;
        if ((keep >> q) & 1u) total += c[q];
    }
}

__device__ __forceinline__ uint32_t keep_bits(const int64_t* dsti, int32_t r)
{
    uint32_t keep = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) keep |= (ld_const(dsti, (int64_t)r * 4 + q) >= 0 ? 1u : 0u) << q;
    return keep;
}

// nlist_cap / mem_cap: entries the next level's list / the member buffer
// can hold.
template <typename Entry>
__device__ __forceinline__ void load_kids(const TaskView& v, uint32_t meta, const int64_t* dsti, const int32_t* cvi,
                                          const int32_t* tcnt, Entry* nlist, int64_t nlist_cap, Entry* members,
                                          int64_t mem_cap, Kids<Entry>& k)
{
    const bool finest = (meta & kMetaChildFinest) != 0;
    k.unswap = finest && (meta & kMetaPass);
    k.keep = keep_bits(dsti, v.r);
    const int4 c4 = ld_const(reinterpret_cast<const int4*>(cvi), (int64_t)v.r);
    const int32_t c[4] = {c4.x, c4.y, c4.z, c4.w};
    int32_t lo[4];
    kid_slots(c, k.keep, lo, k.total);
    const int q0 = __builtin_ctz(k.keep | 16u);   // first kept child (keep != 0 here)
    const int64_t dst = q0 < 4 ? ld_const(dsti, (int64_t)v.r * 4 + q0) : 0;
    k.base = (finest ? members : nlist) + dst;
    const int64_t cap = finest ? mem_cap : nlist_cap;
#pragma unroll
    for (int q = 0; q < 4; ++q) k.pos[q] = lo[q];
    if (v.c > 0) {
        // votes of the region's earlier tasks, by scalar loads: a vector load
        // here would wait for every store the wavefront still has in flight
        const int4* const tc = reinterpret_cast<const int4*>(tcnt);
        for (int64_t t = v.t - v.c; t < v.t; ++t) {
            const int4 x = ld_const(tc, t);
            k.pos[0] += x.x;
            k.pos[1] += x.y;
            k.pos[2] += x.z;
            k.pos[3] += x.w;
        }
    }
    k.roomy = dst >= 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if ((k.keep >> q) & 1u) k.roomy = k.roomy && k.pos[q] >= 0 && dst + k.pos[q] + v.n <= cap;
}

// At a region's last task each kept child must have got exactly its votes.
template <typename Entry>
__device__ __forceinline__ bool kids_complete(const TaskView& v, const int32_t* cvi, const Kids<Entry>& k)
{
    const int4 c4 = ld_const(reinterpret_cast<const int4*>(cvi), (int64_t)v.r);
    const int32_t c[4] = {c4.x, c4.y, c4.z, c4.w};
    int32_t lo[4], total;
    kid_slots(c, k.keep, lo, total);
    bool ok = true;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if ((k.keep >> q) & 1u) ok = ok && k.pos[q] == lo[q] + c[q];
    return ok;
}

// One row of a chunk into the kept children's lists; vm = the lanes that
// hold an entry of the task.  kChecked: each run is checked against the
// region's slots (tasks without room for all their entries, and partial
// chunks).
template <bool kChecked, typename Entry, int kVariant, typename CT>
__device__ __forceinline__ void write_row(const RegionTest<kVariant, CT>& rt, Entry e, uint64_t vm, int lc,
                                          Kids<Entry>& k)
{
    uint64_t cm[4];
    rt.masks(vm, EntryOps<Entry>::point(e), lc, cm);
    const Entry e_out = EntryOps<Entry>::natural(e, k.unswap);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!((k.keep >> q) & 1u)) continue;
        // The row's voters for child q fill slots pos .. pos + n - 1, a lane
        // taking pos + (voting lanes below it).  A checked run that would
        // leave the region's slots [0, total) is not stored (a negative pos
        // wraps to a large unsigned value); pos still advances, so the
        // region's closing check reports it.
        const int32_t n = (int32_t)__popcll(cm[q]);
        const bool fits = !kChecked || (uint32_t)(k.pos[q] + n) <= (uint32_t)k.total;
        if (fits && lane_bit(cm[q])) k.base[(uint32_t)k.pos[q] + lanes_below(cm[q])] = e_out;
        k.pos[q] += n;
    }
}

// A full chunk of a task with room runs unrolled without bounds; any other
// chunk (the last, partial one of a task, or any chunk of a task without
// room) runs row by row with checks in a rolled loop (rare, so kept small).
// rem = the entries left in the task from this chunk on: the chunk's rows
// are the first min(R, rem / 64 rounded up) of them.
template <int R, typename Entry, int kVariant, typename CT>
__device__ __forceinline__ void write_chunk(const RegionTest<kVariant, CT>& rt, const Entry (&ent)[R], int32_t rem,
                                            int lc, int lane, Kids<Entry>& k)
{
    if (rem >= R * kWave && k.roomy) {
#pragma unroll
        for (int r = 0; r < R; ++r) write_row<false, Entry, kVariant, CT>(rt, ent[r], ~0ull, lc, k);
    } else {
#pragma nounroll
        for (int r = 0; r < R && r * kWave < rem; ++r)
            write_row<true, Entry, kVariant, CT>(rt, ent[r], kVariant == 0 ? ~0ull : row_mask(rem, r), lc, k);
    }
}

template <typename Entry, int kVariant, typename CT>
__global__ __launch_bounds__(kBlock) void k_write(LevelArgs a)
{
    const Arena& ar = a.ar;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = (int)rfl(threadIdx.x / kWave);
    const int l = a.level;
    const int lc = l + 1;
    const uint32_t err = *G(ar.error);
    LevelInfo* const info = ar.info + l;
    const int64_t P = info->P, L = info->L, NT = info->NT, steps = info->task_steps;
    if (stopped(err) || P == 0) return;
    const HalfLayout hl = half_layout(ar.half[l & 1], P, L, NT, ar.entry_bytes);
    const WorkLayout wl = work_layout(ar.work, P, NT);
    if (hl.end > ar.half_cap || wl.end > ar.work_cap || steps < 1 || steps > kMaxTaskSteps) return;
    // the next level's list and the member buffer were checked by the emit step
    const LevelInfo* const ni = ar.info + lc;
    const HalfLayout nx = half_layout(ar.half[lc & 1], ni->P, ni->L, ni->NT, ar.entry_bytes);
    const Entry* const list = G(static_cast<const Entry*>(hl.list));
    const Region* const regions = G(static_cast<const Region*>(hl.regions));
    const Task* const tasks = G(static_cast<const Task*>(hl.tasks));
    const int64_t* const dsti = G(static_cast<const int64_t*>(wl.dst));
    const int32_t* const tcnt = G(static_cast<const int32_t*>(wl.tcnt));
    const int32_t* const cvi = G(static_cast<const int32_t*>(hl.cv));
    Entry* const nlist = G(static_cast<Entry*>(nx.list));
    Entry* const members = G(static_cast<Entry*>(ar.members));
    const int64_t nlist_cap = (ar.half_cap - (static_cast<char*>(nx.list) - ar.half[lc & 1])) / (int64_t)sizeof(Entry);
    const int64_t task_len = steps * kStep;

    TaskFeed feed;
    feed.init(&info->queue[1], NT, a.queue_batch, (int64_t)blockIdx.x * kWaves + wave, (int64_t)gridDim.x * kWaves);
    uint32_t bad = 0;   // kErrAt* bits of the checks that failed
    // the next task whose region keeps a child, false at the end
    auto next_task = [&](TaskView& v) -> bool {
        for (;;) {
            const int64_t t = feed.take();
            if (t < 0) return false;
            if (!view_task(tasks, regions, P, L, task_len, t, v)) {
                bad |= kErrAtWriteTask;
                return false;
            }
            if (keep_bits(dsti, v.r)) return true;
        }
    };
    TaskView cur;
    if (next_task(cur)) {
        RegionTest<kVariant, CT> rt;
        Kids<Entry> kc;
        // a task becomes current: its region's test and kept children, and
        // the votes of the region's tasks before it
        auto enter = [&]() {
            uint32_t ij, meta;
            region_code(regions, cur.r, ij, meta);
            rt.set(ij, meta, lc);
            load_kids(cur, meta, dsti, cvi, tcnt, nlist, nlist_cap, members, ar.mem_cap, kc);
        };
        enter();
        constexpr int R = kWriteRows<Entry>;
        Entry ent[R];
        load_chunk<R, Entry, kVariant>(list, cur.b, cur.n, 0, lane, ent);
        int s = 0;
        for (;;) {
            const bool more = (s + 1) * R * kWave < cur.n;
            TaskView nxt;
            bool have_next = false;
            Entry nent[R];
            if (more) {
                load_chunk<R, Entry, kVariant>(list, cur.b, cur.n, s + 1, lane, nent);
            } else if (next_task(nxt)) {
                have_next = true;
                load_chunk<R, Entry, kVariant>(list, nxt.b, nxt.n, 0, lane, nent);
            }
            write_chunk<R, Entry, kVariant, CT>(rt, ent, cur.n - s * R * kWave, lc, lane, kc);
            if (more) {
                ++s;
            } else {
                if (cur.last && !kids_complete(cur, cvi, kc)) {
                    bad |= kErrAtWriteVotes;
                    if (lane == 0) {
                        const int4 c4 = ld_const(reinterpret_cast<const int4*>(cvi), (int64_t)cur.r);
                        record_failure(ar.scalar, kErrAtWriteVotes, l, cur.r, cur.t, kc.keep,
                                       ((int64_t)kc.pos[0] << 32) | (uint32_t)kc.pos[1],
                                       ((int64_t)c4.x << 48) | ((int64_t)(c4.y & 0xFFFF) << 32) |
                                           ((int64_t)(c4.z & 0xFFFF) << 16) | (c4.w & 0xFFFF));
                    }
                }
                if (!have_next) break;
                cur = nxt;
                enter();
                s = 0;
            }
#pragma unroll
            for (int k = 0; k < R; ++k) ent[k] = nent[k];
        }
    }
    if (bad && lane == 0) raise_error(ar.error, kErrInternal | bad | (1u << (kErrLevelShift + l)));
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

// Decision channels of one region from its child votes: regions, list
// entries and tasks of the next level (children that split), cells and
// their voters (children detected at the finest level), votes.
__device__ inline void decision(const int32_t (&cv)[4], int32_t thr, bool finest, int64_t steps,
                                int64_t (&dv)[kAggCh])
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
                dv[5] += region_tasks(cv[q], steps);
            }
        }
    }
}

__device__ inline void region_decision(const Region* regions, const int32_t* cvi, const TreeDesc* trees, int64_t r,
                                       int64_t steps, Region& R, int32_t (&cv)[4], int32_t& thr,
                                       int64_t (&dv)[kAggCh])
{
    R = regions[r];
    const int4 c = reinterpret_cast<const int4*>(cvi)[r];
    cv[0] = c.x;
    cv[1] = c.y;
    cv[2] = c.z;
    cv[3] = c.w;
    thr = trees[R.tree].threshold;
    decision(cv, thr, (R.meta & kMetaChildFinest) != 0, steps, dv);
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
    const int64_t P = ar.info[l].P, L = ar.info[l].L, NT = ar.info[l].NT;
    if (stopped(err) || P == 0) return;
    const HalfLayout hl = half_layout(ar.half[l & 1], P, L, NT, ar.entry_bytes);
    const WorkLayout wl = work_layout(ar.work, P, NT);
    if (hl.end > ar.half_cap || wl.end > ar.work_cap) return;   // k_count raised the error
    const Region* const regions = G(static_cast<const Region*>(hl.regions));
    const int32_t* const cvi = G(static_cast<const int32_t*>(hl.cv));
    const TreeDesc* const trees = G(a.trees);
    const int64_t nb = cdiv(P, kBlock);

    for (int g = blockIdx.x; g < kRangeGrid; g += gridDim.x) {
        int64_t b0, b1;
        range_of(nb, g, b0, b1);
        int64_t acc[kAggCh] = {0, 0, 0, 0, 0, 0};
        for (int64_t r = b0 * kBlock + tid; r < std::min(P, b1 * kBlock); r += kBlock) {
            Region R;
            int32_t cv[4], thr;
            int64_t dv[kAggCh];
            region_decision(regions, cvi, trees, r, a.task_steps, R, cv, thr, dv);
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
    const int64_t P = ar.info[l].P, L = ar.info[l].L, NT = ar.info[l].NT;
    if (stopped(err)) return;
    const int64_t cells_base = ar.info[l].cells_base + ar.info[l].cells;
    const int64_t mem_base = ar.info[l].mem_base + ar.info[l].mem;
    if (P == 0) {
        if (tid == 0 && blockIdx.x == 0) {
            LevelInfo& nx = ar.info[lc];
            nx.P = 0;
            nx.L = 0;
            nx.NT = 0;
            nx.task_steps = a.task_steps;
            nx.queue[0] = nx.queue[1] = 0;
            nx.cells = 0;
            nx.mem = 0;
            nx.cells_base = cells_base;
            nx.mem_base = mem_base;
        }
        return;
    }
    const HalfLayout hl = half_layout(ar.half[l & 1], P, L, NT, ar.entry_bytes);
    const WorkLayout wl = work_layout(ar.work, P, NT);
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
        const int64_t P2 = tot[0], L2 = tot[1], NT2 = tot[5];
        const HalfLayout nx = half_layout(ar.half[lc & 1], P2, L2, NT2, ar.entry_bytes);
        const bool fits = nx.end <= ar.half_cap && work_layout(ar.work, P2, NT2).end <= ar.work_cap &&
                          cells_base + tot[2] <= ar.cells_cap &&
                          (!a.keep_members || mem_base + tot[3] <= ar.mem_cap);
        if (g == 0 && tid == 0) {
            LevelInfo& ni = ar.info[lc];
            ni.P = P2;
            ni.L = L2;
            ni.NT = NT2;
            ni.task_steps = a.task_steps;
            ni.queue[0] = ni.queue[1] = 0;
            ni.cells = tot[2];
            ni.cells_base = cells_base;
            ni.mem = tot[3];
            ni.mem_base = mem_base;
            ar.info[l].votes = tot[4];
            if (!fits) raise_error(ar.error, kErrArena);
        }
        if (!fits) return;
        Region* const nreg = G(nx.regions);
        Task* const ntask = G(nx.tasks);
        int32_t* const ncv = G(nx.cv);
        for (int64_t b = b0; b < b1; ++b) {
            const int64_t r = b * kBlock + tid;
            const bool valid = r < P;
            Region R{};
            int32_t cv[4] = {0, 0, 0, 0};
            int32_t thr = 0;
            int64_t dv[kAggCh] = {0, 0, 0, 0, 0, 0};
            if (valid) region_decision(regions, cvi, trees, r, a.task_steps, R, cv, thr, dv);
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
                int64_t ri = ex[0], start = ex[1], ci = cells_base + ex[2], mo = mem_base + ex[3], tk = ex[5];
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
                        const int64_t nt = region_tasks(cv[q], a.task_steps);
                        if (ri >= P2 || tk + nt > NT2) {
                            raise_error(ar.error, kErrInternal | kErrAtEmit | (1u << (kErrLevelShift + l)));
                            record_failure(ar.scalar, kErrAtEmit, l, r, ri, P2, tk + nt, NT2);
                            continue;
                        }
                        Region C;
                        C.start = start;
                        C.ij = (uint32_t)ci_ | ((uint32_t)cj << 16);
                        C.len = cv[q];
                        C.tree = R.tree;
                        C.meta = (R.meta & ~kMetaChildFinest) | (lc + 1 == T.dmax ? kMetaChildFinest : 0u);
                        nreg[ri] = C;
                        reinterpret_cast<int4*>(ncv)[ri] = int4{0, 0, 0, 0};
                        for (int64_t k = 0; k < nt; ++k) ntask[tk + k] = Task{(int32_t)ri, (int32_t)k};
                        tk += nt;
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
// k_roots (one workgroup) lays the regions and their tasks out;
// k_root_lists writes the lists.
constexpr int kRootThreads = 1024;

__global__ __launch_bounds__(kRootThreads) void k_roots(Arena ar, const TreeDesc* trees, int32_t n_trees,
                                                        int32_t task_steps)
{
    __shared__ int64_t s_w[kRootThreads / kWave][3];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    constexpr int kPer = kMaxTrees / kRootThreads;   // trees per thread
    int64_t len[kPer], cnt = 0, sum = 0, tsum = 0;
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
        tsum += region_tasks(len[k], task_steps);
    }
    const int64_t ci = wave_incl_scan64(cnt, lane), si = wave_incl_scan64(sum, lane);
    const int64_t ti = wave_incl_scan64(tsum, lane);
    if (lane == kWave - 1) {
        s_w[wave][0] = ci;
        s_w[wave][1] = si;
        s_w[wave][2] = ti;
    }
    __syncthreads();
    int64_t r = ci - cnt, start = si - sum, tk = ti - tsum, P0 = 0, L0 = 0, NT0 = 0;
    for (int w = 0; w < kRootThreads / kWave; ++w) {
        if (w < wave) {
            r += s_w[w][0];
            start += s_w[w][1];
            tk += s_w[w][2];
        }
        P0 += s_w[w][0];
        L0 += s_w[w][1];
        NT0 += s_w[w][2];
    }
    if (tid == 0) {
        LevelInfo& in = ar.info[0];
        in.P = P0;
        in.L = L0;
        in.NT = NT0;
        in.task_steps = task_steps;
        in.queue[0] = in.queue[1] = 0;
        in.votes = 0;
        in.cells = 0;
        in.cells_base = 0;
        in.mem = 0;
        in.mem_base = 0;
    }
    if (P0 == 0) return;
    const HalfLayout hl = half_layout(ar.half[0], P0, L0, NT0, ar.entry_bytes);
    if (hl.end > ar.half_cap || work_layout(ar.work, P0, NT0).end > ar.work_cap) {
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
        reinterpret_cast<int4*>(G(hl.cv))[r] = int4{0, 0, 0, 0};
        const int64_t nt = region_tasks(len[k], task_steps);
        for (int64_t c = 0; c < nt; ++c) G(hl.tasks)[tk + c] = Task{(int32_t)r, (int32_t)c};
        tk += nt;
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
    const HalfLayout hl = half_layout(ar.half[0], P0, L0, ar.info[0].NT, ar.entry_bytes);
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
                        const int32_t* ids, int32_t task_steps, int grid, hipStream_t s)
{
    if (n_trees > kMaxTrees || task_steps < 1 || task_steps > kMaxTaskSteps) return hipErrorInvalidValue;
    k_roots<<<1, kRootThreads, 0, s>>>(ar, trees, n_trees, task_steps);
    if (ar.entry_bytes == 8) k_root_lists<uint64_t><<<grid, kBlock, 0, s>>>(ar, trees, xy, ids);
    else k_root_lists<uint32_t><<<grid, kBlock, 0, s>>>(ar, trees, xy, nullptr);
    return hipGetLastError();
}

// Workgroups of the count / compaction kernels that fit on the device at
// once (each wavefront walks tasks until the level's are all taken, so a
// larger grid would only queue behind the resident one).
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
    HH_LEVEL_GRID(k_write);
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

hipError_t launch_write(const LevelArgs& a, int variant, bool wide, int grid, hipStream_t s)
{
    HH_LEVEL_LAUNCH(k_write);
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
