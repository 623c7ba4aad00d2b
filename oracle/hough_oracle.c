/*
 * CPU oracle for the hierarchical slope-intercept Hough vote of
 * C. Singh and N. Bhatia, "A Fast Decision Technique for Hierarchical Hough
 * Transform for Line Detection" (arXiv:1007.0547).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the GPU library never calls it
 * and shares no code with it.
 *
 * What it computes (per enabled pass):
 *   - Sec. 1 / Sec. 3 (ALPHA/BETA): pass 0 maps edge point (x, y) to the
 *     parameter line b = y - x*m; pass 1 swaps the roles of the axes and
 *     maps it to b = x - y*m.  Below, (u, v) is (x, y) or (y, x).
 *   - Sec. 3: level 0 is the whole parameter space; each level splits a
 *     region into the quadrants quad1..quad4 = NE, NW, SW, SE.  The finest
 *     level is ceil(log2 N) for an N x N image.  The parameter space is read
 *     as m in [-1, 1] by b in [-S, 2S] with S = 2^ceil(log2(max(W, H))), so
 *     region (l, i, j) spans m in [-1 + 2i/2^l, -1 + 2(i+1)/2^l] and
 *     b in [-S + 3S*j/2^l, -S + 3S*(j+1)/2^l]; east is +m, north is +b.
 *   - Sec. 2 / getcode(): a 4-bit code per (region, line), one bit per
 *     corner in the order NE, NW, SW, SE (NE is the leftmost bit); a bit is
 *     1 when the corner is below the line, and a corner on the line counts as
 *     above (F = b_c + u*m_c - v >= 0).  Corners are dyadic, so each test is
 *     an exact integer compare after scaling m and b by 2^l.
 *   - Sec. 3, the vote test of the pseudo-code: a line votes for a region iff its
 *     code is neither 0000 nor 1111.
 *   - Sec. 3, the descent of the pseudo-code: a child region only tests the lines
 *     that voted for its parent.
 *   - Sec. 3, the threshold test of the pseudo-code: a region with votes > THRESHOLD is split,
 *     or, at the finest level, handed to solution(), which reports its voting
 *     edge points.  Regions are visited depth first in quad order.
 *   - Sec. 2 / Sec. 3 (comparison method of the paper's ref. [9]): the
 *     circumscribed-circle test, votes iff the distance from the region's
 *     centre to the line is at most the circumradius.  Distances are taken in
 *     units where a region is a square (one grid cell per side); the test is
 *     an exact integer inequality with no square root.
 *
 * The solution() removal (Sec. 3) is not applied here: cells are reported
 * with their full vote lists.  The greedy removal pass is a separate
 * function below (hough_oracle_solution).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

#define OR_VARIANT_CODE 0
#define OR_VARIANT_CIRCLE 1

#define OR_MAX_DEPTH 15
#define OR_NSTAT 6 /* evaluated, votes, split, detected, code_tests, entries */

typedef struct {
    int32_t pass, i, j, votes;
    int64_t key, member_off;
} or_cell;

/* keep_members: 0 = counts only, 1 = every cell's voters stored,
 * 2 = voters folded into a per-pass checksum instead of stored (see
 * push_cell), for searches whose voter lists do not fit in host memory. */
#define OR_MEMBERS_DIGEST 2

typedef struct {
    int32_t status;
    int32_t n_levels;                               /* Dmax + 1 */
    int64_t S;
    int64_t stats[2][OR_MAX_DEPTH + 1][OR_NSTAT];
    or_cell* cells;
    int64_t n_cells, cap_cells;
    int32_t* members;
    int64_t n_members, cap_members;
    int32_t keep_members;
    uint64_t member_digest[2];                      /* keep_members = 2 */
    int64_t pass_members[2];                        /* voters reported per pass */
} or_result;

typedef struct {
    const int32_t* u;
    const int32_t* v;
    int64_t S;
    int32_t dmax, threshold, variant, pass;
    int32_t** level_list;      /* level_list[l]: lines voting for the region open at level l */
    or_result* res;
} or_walk;

/* ---- Sec. 2: position of a corner relative to a parameter line ---------- */

/* Corner (ic, jc) of the level-l grid sits at m = (2*ic - 2^l)/2^l and
 * b = (-S*2^l + 3*S*jc)/2^l.  It is below the line b = v - u*m iff
 * b_c < v - u*m_c; multiplying by 2^l keeps the compare exact. */
static int corner_below(int64_t S, int l, int64_t ic, int64_t jc, int64_t u, int64_t v)
{
    const int64_t scale = (int64_t)1 << l;
    const int64_t Mc = 2 * ic - scale;
    const int64_t Bc = -S * scale + 3 * S * jc;
    return Bc < v * scale - u * Mc;
}

/* getcode(): bit 1 (leftmost) NE, bit 2 NW, bit 3 SW, bit 4 SE. */
static int getcode(int64_t S, int l, int64_t i, int64_t j, int64_t u, int64_t v)
{
    int code = 0;
    if (corner_below(S, l, i + 1, j + 1, u, v)) code |= 8; /* North East */
    if (corner_below(S, l, i, j + 1, u, v))     code |= 4; /* North West */
    if (corner_below(S, l, i, j, u, v))         code |= 2; /* South West */
    if (corner_below(S, l, i + 1, j, u, v))     code |= 1; /* South East */
    return code;
}

/* Circumscribed-circle test of ref. [9], in grid-cell units.
 * Centre: m_c = -1 + (2i+1)/2^l, b_c = -S + 3S(2j+1)/2^(l+1).  With
 * dm = 2/2^l and db = 3S/2^l, the signed distance from the centre to the
 * line in units where the cell is a unit square is
 *     (b_c + u*m_c - v) / sqrt(db^2 + u^2 dm^2),
 * and the circumradius is sqrt(2)/2.  Scaling by 2^(l+1):
 *     D = 3S(2j+1) + 2u(2i+1) - (v + u + S) 2^(l+1),
 * and the test (distance <= radius) becomes D^2 <= 2 (9 S^2 + 4 u^2). */
static int circle_votes(int64_t S, int l, int64_t i, int64_t j, int64_t u, int64_t v)
{
    const int64_t D = 3 * S * (2 * j + 1) + 2 * u * (2 * i + 1) - ((v + u + S) << (l + 1));
    const __int128 lhs = (__int128)D * D;
    const __int128 rhs = (__int128)2 * (9 * (__int128)S * S + 4 * (__int128)u * u);
    return lhs <= rhs;
}

static int votes_for_region(const or_walk* w, int l, int64_t i, int64_t j, int32_t k)
{
    const int64_t u = w->u[k], v = w->v[k];
    if (w->variant == OR_VARIANT_CIRCLE)
        return circle_votes(w->S, l, i, j, u, v);
    {
        const int code = getcode(w->S, l, i, j, u, v);
        return code != 0 && code != 15;           /* Sec. 3 vote test */
    }
}

/* ---- result storage ----------------------------------------------------- */

/* Checksum of a pass's voters in the order a stored member list holds them
 * (cells in visiting order, each cell's voters ascending): the sum over
 * positions t of (t * A + B) * (id + 1), modulo 2^64.  It is a record of the
 * output, not part of the method. */
#define OR_DIGEST_A 0x9E3779B97F4A7C15ull
#define OR_DIGEST_B 0x632BE59BD9B4E019ull

static int push_cell(or_result* r, const or_cell* c, const int32_t* mem, int64_t n)
{
    const int p = c->pass & 1;
    if (r->keep_members == OR_MEMBERS_DIGEST) {
        uint64_t d = r->member_digest[p];
        const uint64_t t0 = (uint64_t)r->pass_members[p];
        for (int64_t t = 0; t < n; ++t)
            d += ((t0 + (uint64_t)t) * OR_DIGEST_A + OR_DIGEST_B) * ((uint64_t)(uint32_t)mem[t] + 1u);
        r->member_digest[p] = d;
    }
    r->pass_members[p] += n;
    if (r->n_cells == r->cap_cells) {
        int64_t cap = r->cap_cells ? 2 * r->cap_cells : 1024;
        or_cell* p = (or_cell*)realloc(r->cells, (size_t)cap * sizeof(or_cell));
        if (!p) return OR_ENOMEM;
        r->cells = p;
        r->cap_cells = cap;
    }
    r->cells[r->n_cells] = *c;
    r->cells[r->n_cells].member_off = r->keep_members == 1 ? r->n_members : -1;
    r->n_cells++;
    if (r->keep_members == 1) {
        if (r->n_members + n > r->cap_members) {
            int64_t cap = r->cap_members ? r->cap_members : 4096;
            while (cap < r->n_members + n) cap *= 2;
            int32_t* p = (int32_t*)realloc(r->members, (size_t)cap * sizeof(int32_t));
            if (!p) return OR_ENOMEM;
            r->members = p;
            r->cap_members = cap;
        }
        memcpy(r->members + r->n_members, mem, (size_t)n * sizeof(int32_t));
        r->n_members += n;
    }
    return OR_OK;
}

/* ---- Sec. 3: depth-first traversal -------------------------------------- */

/* Evaluate region (l, i, j) against the lines in cand[0..n).  Its voting
 * lines go to level_list[l]; if it collects more than THRESHOLD votes it is
 * either split (its four children evaluated in quad order against that list)
 * or, at the finest level, reported.  key holds the quad digits of the path
 * (NE = 0, NW = 1, SW = 2, SE = 3), most significant first. */
static int evaluate(or_walk* w, int l, int64_t i, int64_t j, const int32_t* cand,
                    int64_t n, int64_t key)
{
    int64_t* st = w->res->stats[w->pass][l];
    int32_t* voters = w->level_list[l];
    int64_t votes = 0;
    st[0] += 1;          /* regions evaluated  */
    st[4] += n;          /* codes computed     */
    for (int64_t t = 0; t < n; ++t)
        if (votes_for_region(w, l, i, j, cand[t]))
            voters[votes++] = cand[t];
    st[1] += votes;
    if (votes <= w->threshold)
        return OR_OK;
    if (l == w->dmax) {  /* one-cell region: solution() reports its edge points */
        or_cell c;
        c.pass = w->pass;
        c.i = (int32_t)i;
        c.j = (int32_t)j;
        c.votes = (int32_t)votes;
        c.key = key;
        c.member_off = -1;
        st[3] += 1;
        return push_cell(w->res, &c, voters, votes);
    }
    st[2] += 1;
    st[5] += votes;
    {
        /* quad1..quad4 = NE, NW, SW, SE: (east, north) = (1,1), (0,1), (0,0), (1,0) */
        static const int east[4] = {1, 0, 0, 1};
        static const int north[4] = {1, 1, 0, 0};
        for (int q = 0; q < 4; ++q) {
            int rc = evaluate(w, l + 1, 2 * i + east[q], 2 * j + north[q], voters, votes,
                              key * 4 + q);
            if (rc != OR_OK) return rc;
        }
    }
    return OR_OK;
}

static int64_t pow2_ceil(int64_t side)
{
    int64_t S = 1;
    while (S < side) S <<= 1;
    return S;
}

static int log2_exact(int64_t S)
{
    int d = 0;
    while (((int64_t)1 << d) < S) ++d;
    return d;
}

/* Run the vote for the enabled passes (bit 0: pass 0, bit 1: pass 1).
 * dmax = 0 selects ceil(log2(max(W, H))); dmax < 0 selects depth 0.
 * Returns a result handle (check ->status) or NULL when out of memory. */
or_result* hough_oracle_detect(const int32_t* x, const int32_t* y, int64_t E, int32_t W,
                               int32_t H, int32_t threshold, int32_t dmax, int32_t variant,
                               uint32_t passes, int32_t keep_members)
{
    or_result* r = (or_result*)calloc(1, sizeof(or_result));
    if (!r) return NULL;
    r->keep_members = keep_members;
    if (W < 1 || H < 1 || E < 0 || threshold < 0 || (variant != 0 && variant != 1) ||
        (E > 0 && (!x || !y)) || E > INT32_MAX) {
        r->status = OR_EINVAL;
        return r;
    }
    r->S = pow2_ceil(W > H ? W : H);
    if (dmax == 0) dmax = log2_exact(r->S);
    if (dmax < 0) dmax = 0;
    if (dmax > OR_MAX_DEPTH) {
        r->status = OR_EINVAL;
        return r;
    }
    r->n_levels = dmax + 1;
    for (int64_t k = 0; k < E; ++k)
        if (x[k] < 0 || x[k] >= W || y[k] < 0 || y[k] >= H) {
            r->status = OR_EINVAL;
            return r;
        }

    int32_t* all = (int32_t*)malloc((size_t)(E > 0 ? E : 1) * sizeof(int32_t));
    int32_t** lists = (int32_t**)calloc((size_t)dmax + 1, sizeof(int32_t*));
    int rc = (all && lists) ? OR_OK : OR_ENOMEM;
    for (int l = 0; rc == OR_OK && l <= dmax; ++l) {
        lists[l] = (int32_t*)malloc((size_t)(E > 0 ? E : 1) * sizeof(int32_t));
        if (!lists[l]) rc = OR_ENOMEM;
    }
    for (int64_t k = 0; rc == OR_OK && k < E; ++k) all[k] = (int32_t)k;

    for (int pass = 0; rc == OR_OK && pass < 2; ++pass) {
        if (!(passes & (1u << pass))) continue;
        or_walk w;
        w.u = pass == 0 ? x : y;   /* pass 1: (x0, y0) is read as (y0, x0) */
        w.v = pass == 0 ? y : x;
        w.S = r->S;
        w.dmax = dmax;
        w.threshold = threshold;
        w.variant = variant;
        w.pass = pass;
        w.level_list = lists;
        w.res = r;
        rc = evaluate(&w, 0, 0, 0, all, E, 0);
    }
    if (lists)
        for (int l = 0; l <= dmax; ++l) free(lists[l]);
    free(lists);
    free(all);
    r->status = rc;
    return r;
}

/* One subtree of one pass: region (level, i, j), evaluated against the lines
 * cand[0..n_cand) -- in the search, the lines that voted for its parent (all
 * lines for the root) -- and everything the search visits below it, in the
 * same order and with the same arithmetic as hough_oracle_detect.  key is
 * the region's quad-digit key; its cells' keys extend it.  Statistics cover
 * levels >= level only.  A part of a large search can so be run (or timed)
 * on its own. */
or_result* hough_oracle_detect_subtree(const int32_t* x, const int32_t* y, int64_t E, int32_t W,
                                       int32_t H, int32_t threshold, int32_t dmax, int32_t variant,
                                       int32_t pass, int32_t level, int64_t i, int64_t j, int64_t key,
                                       const int32_t* cand, int64_t n_cand, int32_t keep_members)
{
    or_result* r = (or_result*)calloc(1, sizeof(or_result));
    if (!r) return NULL;
    r->keep_members = keep_members;
    if (W < 1 || H < 1 || E < 0 || threshold < 0 || (variant != 0 && variant != 1) ||
        (pass != 0 && pass != 1) || (E > 0 && (!x || !y)) || E > INT32_MAX || n_cand < 0 ||
        n_cand > E || (n_cand > 0 && !cand)) {
        r->status = OR_EINVAL;
        return r;
    }
    r->S = pow2_ceil(W > H ? W : H);
    if (dmax == 0) dmax = log2_exact(r->S);
    if (dmax < 0) dmax = 0;
    if (dmax > OR_MAX_DEPTH || level < 0 || level > dmax || i < 0 || j < 0 ||
        i >= ((int64_t)1 << level) || j >= ((int64_t)1 << level)) {
        r->status = OR_EINVAL;
        return r;
    }
    r->n_levels = dmax + 1;
    for (int64_t k = 0; k < E; ++k)
        if (x[k] < 0 || x[k] >= W || y[k] < 0 || y[k] >= H) {
            r->status = OR_EINVAL;
            return r;
        }
    for (int64_t t = 0; t < n_cand; ++t)
        if (cand[t] < 0 || cand[t] >= E) {
            r->status = OR_EINVAL;
            return r;
        }
    int32_t** lists = (int32_t**)calloc((size_t)dmax + 1, sizeof(int32_t*));
    int rc = lists ? OR_OK : OR_ENOMEM;
    for (int l = level; rc == OR_OK && l <= dmax; ++l) {
        lists[l] = (int32_t*)malloc((size_t)(n_cand > 0 ? n_cand : 1) * sizeof(int32_t));
        if (!lists[l]) rc = OR_ENOMEM;
    }
    if (rc == OR_OK) {
        or_walk w;
        w.u = pass == 0 ? x : y;
        w.v = pass == 0 ? y : x;
        w.S = r->S;
        w.dmax = dmax;
        w.threshold = threshold;
        w.variant = variant;
        w.pass = pass;
        w.level_list = lists;
        w.res = r;
        rc = evaluate(&w, level, i, j, cand, n_cand, key);
    }
    if (lists)
        for (int l = 0; l <= dmax; ++l) free(lists[l]);
    free(lists);
    r->status = rc;
    return r;
}

/* ---- accessors ---------------------------------------------------------- */

int32_t hough_oracle_status(const or_result* r) { return r->status; }
int32_t hough_oracle_n_levels(const or_result* r) { return r->n_levels; }
int64_t hough_oracle_S(const or_result* r) { return r->S; }
int64_t hough_oracle_n_cells(const or_result* r) { return r->n_cells; }
int64_t hough_oracle_n_members(const or_result* r) { return r->n_members; }
uint64_t hough_oracle_member_digest(const or_result* r, int32_t pass) { return r->member_digest[pass & 1]; }
int64_t hough_oracle_pass_members(const or_result* r, int32_t pass) { return r->pass_members[pass & 1]; }

void hough_oracle_cells(const or_result* r, int32_t* pass, int32_t* i, int32_t* j,
                        int64_t* key, int32_t* votes, int64_t* member_off)
{
    for (int64_t c = 0; c < r->n_cells; ++c) {
        pass[c] = r->cells[c].pass;
        i[c] = r->cells[c].i;
        j[c] = r->cells[c].j;
        key[c] = r->cells[c].key;
        votes[c] = r->cells[c].votes;
        member_off[c] = r->cells[c].member_off;
    }
}

void hough_oracle_members(const or_result* r, int32_t* out)
{
    if (r->n_members) memcpy(out, r->members, (size_t)r->n_members * sizeof(int32_t));
}

/* out[l*6 + s] for l in [0, n_levels): evaluated, votes, split, detected,
 * code_tests, entries (the summed votes of the regions split at level l). */
void hough_oracle_stats(const or_result* r, int32_t pass, int64_t* out)
{
    for (int l = 0; l < r->n_levels; ++l)
        for (int s = 0; s < OR_NSTAT; ++s)
            out[l * OR_NSTAT + s] = r->stats[pass & 1][l][s];
}

void hough_oracle_free(or_result* r)
{
    if (!r) return;
    free(r->cells);
    free(r->members);
    free(r);
}

/* Lines that vote for one region (l, i, j) of one pass, by testing every
 * edge point against that region directly (no hierarchy).  Writes their ids
 * in ascending order to out (if not NULL) and returns their number, or -1 on
 * bad arguments. */
int64_t hough_oracle_region_voters(const int32_t* x, const int32_t* y, int64_t E, int32_t W,
                                   int32_t H, int32_t pass, int32_t l, int64_t i, int64_t j,
                                   int32_t variant, int32_t* out)
{
    if (W < 1 || H < 1 || l < 0 || l > OR_MAX_DEPTH || i < 0 || j < 0 ||
        i >= ((int64_t)1 << l) || j >= ((int64_t)1 << l))
        return -1;
    or_walk w;
    w.u = pass == 0 ? x : y;
    w.v = pass == 0 ? y : x;
    w.S = pow2_ceil(W > H ? W : H);
    w.variant = variant;
    int64_t n = 0;
    for (int64_t k = 0; k < E; ++k)
        if (votes_for_region(&w, l, i, j, (int32_t)k)) {
            if (out) out[n] = (int32_t)k;
            ++n;
        }
    return n;
}

/* The 4-bit code of one line for one region (Sec. 2), for tests. */
int32_t hough_oracle_getcode(int64_t S, int32_t l, int64_t i, int64_t j, int64_t u, int64_t v)
{
    return getcode(S, l, i, j, u, v);
}

/* The circle test of one line for one region, for tests. */
int32_t hough_oracle_circle(int64_t S, int32_t l, int64_t i, int64_t j, int64_t u, int64_t v)
{
    return circle_votes(S, l, i, j, u, v);
}

/* solution() with removal (Sec. 3): walk the detected cells of one pass in
 * depth-first (key) order; a cell is kept when more than THRESHOLD of its
 * voters have not been plotted by an earlier kept cell, and then its voters
 * are plotted.  keep[c] receives 1 for kept cells; plotted[k] receives 1 for
 * every plotted edge point.  Cells must be one pass, sorted by key, with
 * members available.  Returns the number of kept cells or -1. */
int64_t hough_oracle_solution(const or_result* r, int32_t pass, int32_t threshold, int64_t E,
                              uint8_t* keep, uint8_t* plotted)
{
    if (r->keep_members != 1) return -1;
    memset(plotted, 0, (size_t)E);
    int64_t kept = 0, c_out = 0;
    for (int64_t c = 0; c < r->n_cells; ++c) {
        const or_cell* cell = &r->cells[c];
        if (cell->pass != pass) continue;
        const int32_t* m = r->members + cell->member_off;
        int64_t live = 0;
        for (int32_t t = 0; t < cell->votes; ++t) live += !plotted[m[t]];
        keep[c_out] = live > threshold;
        if (live > threshold) {
            for (int32_t t = 0; t < cell->votes; ++t) plotted[m[t]] = 1;
            ++kept;
        }
        ++c_out;
    }
    return kept;
}
