/*
 * hough_hier.h -- C ABI of the MI355X (gfx950) hierarchical slope-intercept
 * Hough vote of C. Singh and N. Bhatia, "A Fast Decision Technique for
 * Hierarchical Hough Transform for Line Detection" (arXiv:1007.0547).
 *
 * What the library computes (per image and enabled pass):
 *   - Sec. 1 and Sec. 3 (ALPHA/BETA): pass 0 maps each edge point (x, y) to
 *     the parameter line b = y - x*m with |m| <= 1; pass 1 swaps the axes and
 *     maps it to b = x - y*m.  Every edge point enters both passes.
 *   - Sec. 3: a quadtree over the parameter space.  Level 0 is the whole
 *     space m in [-1, 1], b in [-S, 2S] with S = 2^ceil(log2(max(W, H))).
 *     Region (l, i, j) spans m in [-1 + 2i/2^l, -1 + 2(i+1)/2^l] and
 *     b in [-S + 3S j/2^l, -S + 3S (j+1)/2^l]; east is +m, north is +b, and
 *     its children are taken in the order quad1..quad4 = NE, NW, SW, SE.
 *   - Sec. 2, getcode(): for every (region, line) pair a 4-bit code, one bit
 *     per corner in the order NE, NW, SW, SE (NE leftmost), 1 when the corner
 *     is below the line; a corner on the line counts as above.  Corners are
 *     dyadic, so each bit is an exact integer compare with m and b scaled by
 *     2^level.
 *   - Sec. 3 pseudo-code (vote test, descent, threshold test): a line votes for a region
 *     iff its code is neither 0000 nor 1111; a child only tests the lines
 *     that voted for its parent; a region with votes > threshold splits, and
 *     at the finest level (default ceil(log2 N)) it is reported as a
 *     detected cell together with its voters (solution(), without removal).
 *   - Sec. 2 / Sec. 3, comparison method of the paper's ref. [9]
 *     (HH_VARIANT_CIRCLE): a line votes iff its distance from the region's
 *     centre is at most the circumradius, distances measured in units where a
 *     region is a square, as an exact integer inequality with no square root.
 *
 * Conventions for every entry point:
 *   - Every call returns hh_status; nothing throws or aborts across the ABI.
 *     hough_hier_last_error() returns the text of the last failure on a
 *     context.
 *   - Point ids are positions in the input point list (for an image input:
 *     rank in a row-major scan, y then x).  Ids are int32.
 *   - Output cells are sorted by (pass, key), where key holds the quad digits
 *     NE=0, NW=1, SW=2, SE=3 of the path from level 1 down, most significant
 *     first (the paper's depth-first visiting order).  Each cell's voters are
 *     ascending point ids.
 *   - All GPU work of a call runs on the context's stream.  A call returns
 *     when its result (cells, members, statistics) is complete on the device.
 *   - Calls on one context are serialised by a lock inside the context;
 *     hough_hier_submit and hough_hier_poll may be called from any thread.
 */
#ifndef HOUGH_HIER_H
#define HOUGH_HIER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define HH_API __attribute__((visibility("default")))
#else
#define HH_API
#endif

typedef struct hh_ctx hh_ctx;
typedef struct hh_result hh_result;

typedef enum {
    HH_PENDING = 1,      /* hough_hier_poll: the request has not completed (not an error) */
    HH_OK = 0,
    HH_EINVAL = -1,      /* bad argument: null pointer, W or H < 1, point outside
                            [0,W)x[0,H), threshold < 0, depth out of range, size limit */
    HH_ENOMEM = -2,      /* device or host allocation failed                          */
    HH_ECAPACITY = -3,   /* a size limit of the implementation was exceeded          */
    HH_EDEVICE = -4,     /* HIP error, or the device is not a gfx950                  */
    HH_EBUSY = -5,       /* no free slot                                              */
    HH_ECANCELED = -6,
    HH_EINTERNAL = -7    /* an internal consistency check failed; the error text names
                            the check, its level, the first failure's indices and
                            totals, and the call's arena resumes                      */
} hh_status;

typedef enum {
    HH_VARIANT_CODE = 0,     /* 4-bit corner code (Sec. 2)                    */
    HH_VARIANT_CIRCLE = 1    /* circumscribed-circle test (comparison method) */
} hh_variant;

#define HH_PASS_0 1u         /* |m| <= 1 as given (ALPHA)                   */
#define HH_PASS_1 2u         /* axes swapped (BETA)                         */

/* hh_config.flags */
#define HH_FLAG_WIDE_COMPARE 1   /* code variant: use 64-bit compares even where 32-bit
                                    compares are provably exact                         */
#define HH_FLAG_TIMING 2         /* record HIP events around every kernel launch; read them
                                    with hough_hier_result_timing()                    */
#define HH_FLAG_GRAPH 4          /* with a caller arena (hh_config.arena), a stream (not
                                    the null stream) and device-resident
                                    inputs: capture a call's level launches (arena
                                    clear, root setup, every level's four launches and
                                    the copy of the level records) into a HIP graph, and
                                    replay it for the next call whose sizes, parameters
                                    and memory are the same (its addresses are then the
                                    same too); otherwise the launches run one by one.
                                    Results do not depend on it.  Not with TIMING.     */

/* Limits: max(W, H) <= 16384, depth <= 15 and S * 2^depth <= 2^28 (keeps every
 * scaled corner value inside 31 bits and the circle test inside 63 bits);
 * number of points <= 2^31 - 1. */
#define HH_MAX_SIDE 16384
#define HH_MAX_DEPTH 15

typedef struct {
    int32_t threshold;        /* default T >= 0 for inputs that give threshold < 0     */
    int32_t max_depth;        /* default depth: 0 = ceil(log2(max(W,H))), -1 = depth 0  */
    uint32_t passes;          /* HH_PASS_0 | HH_PASS_1; 0 is taken as both              */
    int32_t variant;          /* hh_variant                                             */
    int32_t membership;       /* 1: keep each detected cell's voters; 0: counts only    */
    int32_t device;           /* HIP device ordinal; the device must be a gfx950        */
    void* stream;             /* hipStream_t for all work, or NULL for the null stream  */
    int32_t flags;            /* HH_FLAG_*                                              */
    int32_t arena_limit_mib;  /* most MiB one arena may take (0: 35% of the device
                                 memory).  A batch whose level lists need more runs in
                                 groups of inputs; one input that needs more fails
                                 with HH_ECAPACITY.                                    */
    uint64_t arena_hint;      /* initial bytes of each level-list half of a call's arena
                                 (0: 64 MiB); the other parts start in proportion.  A
                                 call whose levels outgrow the arena continues in a
                                 larger one, and later calls keep the larger sizes.   */
    void* arena;              /* caller-owned device memory (e.g. a torch tensor's) for
                                 every detection call on this context, or NULL (the
                                 library allocates from its own pool).  A call carves
                                 its staged inputs, descriptors and level arena from it
                                 front to back and allocates no device memory; the
                                 level arena's parts are split in the proportions the
                                 context has learnt.  When a level does not fit, the
                                 call reruns from the root with the parts re-split by
                                 the sizes measured so far (at most three reruns), then
                                 fails with HH_ECAPACITY (nothing is grouped or resumed
                                 in a larger arena).  The results of
                                 a call point into the arena: free them before the
                                 next call (that call fails with HH_EBUSY otherwise).
                                 The memory stays the caller's; it must stay valid
                                 while results of the context live.  A context with an
                                 arena cannot serve.  256-byte aligned.                */
    uint64_t arena_bytes;     /* size of arena in bytes                                 */
    uint64_t hbm_budget_bytes;/* device-memory budget of one call's level arena (a
                                 batch beyond it runs in groups) and the admission
                                 budget of serving (sum of the predicted footprints of
                                 the requests in flight); 0: arena_limit_mib if set,
                                 else 35% of the device memory                         */
} hh_config;

typedef struct {
    int32_t kind;             /* 0: point list (x, y, n_points); 1: binary image;
                                 2: gray image through the Sobel front end (Sec. 3):
                                 the edge points are the pixels with a full 3x3
                                 neighbourhood and Gx^2 + Gy^2 > edge_threshold^2;
                                 pass 0 takes those with |Gx| <= |Gy| (ALPHA, image
                                 lines with |slope| <= 1), pass 1 the others (BETA).
                                 Point ids are ranks among all edge points, row-major;
                                 depth must be >= 1                                    */
    int32_t width, height;    /* W, H >= 1                                              */
    int32_t on_device;        /* 1: x, y, image are device pointers valid on the stream */
    const int32_t* x;         /* kind 0: x[k] in [0, W)                                 */
    const int32_t* y;         /* kind 0: y[k] in [0, H)                                 */
    int64_t n_points;         /* kind 0: number of points (0 allowed)                   */
    const uint8_t* image;     /* kind 1: H rows of W bytes, nonzero = edge pixel;
                                 kind 2: H rows of W gray levels                        */
    int64_t row_stride;       /* kinds 1, 2: bytes between rows (>= W; 0 means W)        */
    int32_t threshold;        /* T for this input; < 0 takes the context default        */
    int32_t max_depth;        /* depth for this input: 0 = ceil(log2(max(W,H))),
                                 -1 = depth 0, INT32_MIN takes the context default      */
    int32_t edge_threshold;   /* kind 2: Sobel magnitude threshold (>= 0)               */
    int32_t reserved;
} hh_input;

/* One detected finest-level cell.  member_off indexes the members array that
 * hough_hier_result_members() returns with the same on_device value. */
typedef struct {
    int32_t i, j;             /* cell indices at the finest level                       */
    int32_t votes;            /* number of voters (lines crossing the cell)             */
    int32_t pass;             /* 0 or 1                                                 */
    int64_t key;              /* quad-digit path key                                    */
    int64_t member_off;       /* first voter in the members array, or -1 if not kept    */
} hh_cell;

/* Per-level statistics of one pass (level 0 = root). */
typedef struct {
    int64_t evaluated;        /* regions whose votes were counted                       */
    int64_t votes;            /* sum of their votes (the paper's "number of votes")     */
    int64_t split;            /* regions with votes > T below the finest level          */
    int64_t detected;         /* regions with votes > T at the finest level             */
    int64_t code_tests;       /* (region, line) codes computed at this level            */
    int64_t entries;          /* summed votes of the regions split at this level        */
} hh_level_stats;

typedef struct {
    int64_t n_points;         /* E                                                      */
    int32_t width, height;
    int32_t side_pow2;        /* S                                                      */
    int32_t depth;            /* finest level                                           */
    int32_t threshold;
    uint32_t passes;
    int64_t n_cells[2];       /* detected cells per pass                                */
    int64_t code_tests;       /* summed over levels and passes                          */
    int64_t member_slots;     /* length of the device members array                     */
    int32_t compare_bits;     /* 32 or 64: width of the corner compares used            */
    int32_t reserved;
} hh_result_info;

/* Kernel timings of one call (HH_FLAG_TIMING), from HIP events recorded on
 * the context's stream around the launches of each level; zero without the
 * flag.  The events themselves add a few microseconds per level.  The entry
 * counts, groups and resumes are filled in with or without the flag. */
typedef struct {
    int32_t vote_launches;    /* per-level count and compaction launches            */
    int32_t decide_launches;  /* per-level split-decision launches                  */
    double vote_ms;           /* count_ms + write_ms                                */
    double decide_ms;         /* summed duration of the split-decision launches     */
    double extract_ms;        /* edge staging (image inputs)                        */
    double total_ms;          /* first to last event of the call                    */
    int64_t vote_entries;     /* (parent, line) entries read by the count launches  */
    int64_t vote_written;     /* entries written by the compaction launches         */
    double count_ms;          /* summed duration of the count launches              */
    double write_ms;          /* summed duration of the compaction launches         */
    int32_t groups;           /* groups of inputs whose levels ran in one arena     */
    int32_t resumes;          /* levels that outgrew the arena and resumed larger   */
    double queue_ms;          /* served requests: submission to the start of its batch */
    double service_ms;        /* served requests: batch start to cells and statistics
                                 on the host                                           */
    int32_t graph_replayed;   /* HH_FLAG_GRAPH: 1 if the call replayed the graph captured
                                 by an earlier call, 0 if it captured or ran launches  */
    int32_t reserved;
} hh_timing;

/* Launch shape of the two list kernels of every level (the count pass and
 * the compaction pass).  A level's list is cut into tasks, each a run of at
 * most task_steps * 512 entries of one region's list; the kernels run a
 * resident grid (wg_per_cu workgroups of 256 threads per compute unit) whose
 * wavefronts take tasks until the level's are all taken: from a fixed share
 * (queue_batch = 0: wavefront w takes tasks w, w + W, w + 2W, ... of the W
 * wavefronts), or from the level's device work queue, an atomic head that
 * hands out queue_batch consecutive tasks at a time.  Results do not depend
 * on the launch shape; only the time does. */
typedef struct {
    int32_t task_steps;       /* 512-entry steps per task, 1..64 (0: default 8)       */
    int32_t queue_batch;      /* 0: fixed share; 1..1024: tasks per take from the queue */
    int32_t wg_per_cu;        /* resident workgroups per compute unit, 0: as many as fit */
    int32_t reserved;
} hh_launch;

/* Set or read the launch shape of the list kernels on ctx (applies to the
 * calls that start afterwards; serving lanes take it when they start).
 * Errors: HH_EINVAL (NULL arguments, a field out of range). */
HH_API hh_status hough_hier_set_launch(hh_ctx* ctx, const hh_launch* launch);
HH_API hh_status hough_hier_get_launch(const hh_ctx* ctx, hh_launch* launch);

/* Pick the launch shape for calls like inputs[0 .. n) (the same kind, count,
 * sizes, depth and context settings) and set it on ctx.  The choice is read
 * from a cache file keyed by the device (architecture, compute units, HIP
 * runtime version) and the shape of the call, or, for a new key, made by
 * running the call once per candidate shape (task_steps 1, 2, 4, 8, 16 with
 * wg_per_cu 0 or 4, fixed shares) -- once to warm up, then twice timed, the
 * fastest kept -- and written to the cache.  The cache file is
 * $HH_TUNE_CACHE, else $HOME/.cache/hough_hier_tune.json (a JSON object of
 * key -> shape and milliseconds).  Inputs are borrowed for the call; the
 * results of the timed runs are freed.  *from_cache (may be NULL) is 1 when
 * the cache had the key.
 * Errors: as hough_hier_detect_batch. */
HH_API hh_status hough_hier_autotune(hh_ctx* ctx, const hh_input* inputs, int32_t n, hh_launch* chosen,
                                     int32_t* from_cache);

/* Create a context on cfg->device.  Checks the device is a gfx950.
 * Errors: HH_EINVAL (cfg or out NULL, bad defaults), HH_EDEVICE. */
HH_API hh_status hough_hier_create(const hh_config* cfg, hh_ctx** out);

/* Destroy a context and release all its device memory, including the memory
 * of results not yet freed (those handles must not be used afterwards).
 * NULL is accepted. */
HH_API void hough_hier_destroy(hh_ctx* ctx);

/* Text of the last error on ctx (never NULL; empty if none). */
HH_API const char* hough_hier_last_error(const hh_ctx* ctx);

/* Run the hierarchical vote (Sec. 3) on one input: edge staging (image
 * inputs), then levels 0 .. depth-1 for every enabled pass.  Inputs are
 * borrowed for the duration of the call.  On HH_OK *out owns the result;
 * release it with hough_hier_result_free().  The result keeps the call's
 * arena (its cells and voters are inside) until it is freed, so free results
 * promptly when calls are many or large.
 * Errors: HH_EINVAL (see hh_status; also for device point lists with a point
 * out of range), HH_ENOMEM, HH_EDEVICE, HH_EINTERNAL. */
HH_API hh_status hough_hier_detect(hh_ctx* ctx, const hh_input* in, hh_result** out);

/* Run the vote on n inputs of one kind (all point lists or all images) in one
 * call.  Every enabled pass of every input is its own quadtree (Sec. 3) and
 * all trees share each level's launches, so a batch of small inputs pays the
 * per-level launch cost once.  Each input keeps its own size, threshold and
 * depth; the call runs to the deepest of them.  out[k] (an array of n
 * handles owned by the caller) receives the result of inputs[k], with the
 * same cells, members and statistics that hough_hier_detect(&inputs[k])
 * returns.  Each handle is freed on its own; the device memory the handles
 * share is released with the last of them.  n * (enabled passes) <= 2048.
 * Errors: as hough_hier_detect; HH_EINVAL also for n < 1 or inputs of mixed
 * kinds, HH_ECAPACITY for more than 2048 trees.  On an error no handle is
 * returned (out[] is all NULL). */
HH_API hh_status hough_hier_detect_batch(hh_ctx* ctx, const hh_input* inputs, int32_t n, hh_result** out);

/* ---- Serving: continuous batching of requests on one context.
 *
 * hough_hier_serve_start allocates one device slab of the context's budget
 * (hbm_budget_bytes, else arena_limit_mib, else 35% of the device memory)
 * and starts `lanes` worker lanes (slots), each with its own HIP stream
 * (default-priority streams); the lanes draw all their device memory from
 * the slab.  A free lane takes the pending requests in arrival order, as
 * many as fit (at most max_batch requests, at most max_batch_pixels image
 * pixels if that is not 0, and -- the admission by device memory -- while
 * their predicted footprint fits the slab's largest free interval and, past
 * the first request, half of 1/lanes of the slab; any request while no
 * batch runs), runs them as one batch
 * (hough_hier_detect_batch), copies each result's cells and statistics to
 * the host and completes the tickets.  A request's footprint is predicted
 * as beta * E * 2^depth bytes, E its edge points (counted at submission for
 * a host binary image or a point list, else its pixels times the edge
 * density seen so far), beta a running average over completed batches of
 * their measured need per unit; the prediction also sizes the batch's
 * first level arena, which grows from the level that overflows.  Requests
 * that arrive while batches run are admitted by the next lane that is free
 * once slab space allows, so batches of different lanes overlap on the
 * device; serving allocates no device memory.  A served result keeps its
 * device memory (cells and voters) until the last result of its batch is
 * freed: free served results promptly.  A batch that finds the slab full
 * gives its second half back to the head of the queue and runs its first
 * half again; a single request runs again once space comes back, and if it
 * still finds the slab full while no batch runs (the slab held by results
 * not yet freed for a second, or a request larger than the slab) it runs
 * outside the slab, in device memory returned as soon as its results are
 * freed.  A request's result is identical to what
 * hough_hier_detect returns for the same input.  The context stays usable
 * for plain calls.  Served results carry queue_ms and service_ms in
 * hh_timing. */
typedef struct {
    int32_t lanes;            /* concurrent batches, 1..8 (0: 3)                       */
    int32_t max_batch;        /* most requests in one batch, 1..2048 (0: 4)            */
    int64_t max_batch_pixels; /* most image pixels (points of lists) in a batch, 0: no
                                 limit besides the memory budget                        */
    int32_t queue_capacity;   /* most tickets not yet claimed by poll (0: 4096)        */
    int32_t reserved;
} hh_serve_config;

/* Start serving on ctx (once per context).  cfg may be NULL for defaults.
 * Errors: HH_EINVAL (bad config, already serving), HH_EDEVICE, HH_ENOMEM
 * (the slab could not be allocated). */
HH_API hh_status hough_hier_serve_start(hh_ctx* ctx, const hh_serve_config* cfg);

/* Queue one input (borrowed until its ticket completes; device inputs must be
 * ready, since lanes run on their own streams).  *ticket identifies it.
 * Errors: HH_EINVAL (not serving, bad input form), HH_EBUSY (queue_capacity
 * tickets outstanding). */
HH_API hh_status hough_hier_submit(hh_ctx* ctx, const hh_input* in, uint64_t* ticket);

/* Wait up to wait_us microseconds (< 0: until done, 0: do not wait) for a
 * ticket.  HH_PENDING: not completed yet (ask again).  Otherwise the ticket
 * is consumed: on HH_OK *out owns the result (free it with
 * hough_hier_result_free), on an error the request's status is returned
 * and hough_hier_last_error() holds its text.
 * Errors: HH_EINVAL (unknown ticket, not serving), any error of the request. */
HH_API hh_status hough_hier_poll(hh_ctx* ctx, uint64_t ticket, int32_t wait_us, hh_result** out);

/* Serving counters of ctx (hough_hier_serve_stats). */
typedef struct {
    int64_t slab_bytes;        /* the slab allocated by hough_hier_serve_start        */
    int64_t slab_used;         /* bytes of it held now by running batches and results */
    int64_t slab_batches;      /* batches run inside the slab                         */
    int64_t outside_batches;   /* batches run outside the slab                        */
    int64_t retries;           /* runs that found the slab full and ran again         */
    int64_t pending;           /* requests waiting for a lane                         */
    double bytes_per_unit;     /* the footprint model's beta (bytes per E * 2^depth)  */
    int64_t internal_reruns;   /* batches whose kernels' consistency check failed
                                  (HH_EINTERNAL, no result made) and that ran again  */
    int64_t internal_failures; /* of those, reruns that failed the same way (their
                                  requests then run one by one)                       */
    char first_internal_error[512];   /* the first such failure's text, or ""       */
} hh_serve_stats;

/* Copy the serving counters of ctx into *out.
 * Errors: HH_EINVAL (not serving, out NULL). */
HH_API hh_status hough_hier_serve_stats(hh_ctx* ctx, hh_serve_stats* out);

/* Cells of one pass (0 or 1), sorted by key.  on_device = 1 returns a device
 * pointer (member_off indexes the device members array); on_device = 0 copies
 * to host memory owned by the result (member_off indexes the host members
 * array).  A pass that was not enabled has no cells.
 * Errors: HH_EINVAL, HH_EDEVICE. */
HH_API hh_status hough_hier_result_cells(hh_result* res, int32_t pass, int32_t on_device,
                                  const hh_cell** cells, int64_t* n);

/* Point ids of the voters of the detected cells (ascending within a cell).
 * on_device = 1: a device array of *n slots in the layout of the device
 * cells' member_off (slots no cell references are unspecified), made on the
 * first request; on_device = 0: a compact host array, cells in (pass, key)
 * order.  Both stay valid until hough_hier_result_free().
 * Errors: HH_EINVAL (membership was not kept), HH_EDEVICE. */
HH_API hh_status hough_hier_result_members(hh_result* res, int32_t on_device, const int32_t** ids,
                                    int64_t* n);

/* The voters as the kernels left them, with no conversion: a device array of
 * *n entries in the layout of the device cells' member_off.  *entry_bytes = 4:
 * each entry is an edge point packed as x | y << 16 (image inputs; ascending
 * packed value = ascending id); *entry_bytes = 8: (id << 32) | packed point
 * (point-list inputs).  Valid until hough_hier_result_free().
 * Errors: HH_EINVAL (membership was not kept). */
HH_API hh_status hough_hier_result_member_points(const hh_result* res, const void** entries, int64_t* n,
                                          int32_t* entry_bytes);

/* Host per-level statistics of one pass: *n_levels = depth + 1 entries. */
HH_API hh_status hough_hier_result_stats(const hh_result* res, int32_t pass,
                                  const hh_level_stats** levels, int32_t* n_levels);

/* Sizes and parameters of a result. */
HH_API hh_status hough_hier_result_info(const hh_result* res, hh_result_info* info);

/* Kernel timings of the call that produced res (see hh_timing). */
HH_API hh_status hough_hier_result_timing(const hh_result* res, hh_timing* timing);

/* solution() with point removal (Sec. 3, the procedure called at a detected
 * finest region).  The depth-first search plots the voters of a detected cell
 * and zeroes their codes at every level, so no region visited after it counts
 * them.  Per pass this keeps a detected cell (in key order, the search's
 * visiting order) iff more than T of its voters were not plotted by an earlier
 * kept cell, and then plots its voters; the plotted points are the output
 * image.  Passes are independent (each has its own plotted set).
 * hough_hier_solution computes this on the device for n results (all their
 * passes together; results of a serving context are walked on the lane that
 * made them); a result already solved is skipped.  The walk of a pass is cut
 * into segments of consecutive cells, each walked by one workgroup from the
 * points the segments before it plotted in the previous round; rounds repeat
 * until no segment's starting points change, which gives exactly the
 * sequential walk.  *kernel_ms (may be NULL) receives the device time from
 * the first round to the outputs, the host's checks between rounds
 * included.  While it runs the
 * call holds device memory for the voter ids of all its results (4 bytes per
 * voter, kept in the context's pool for later calls); the flags (a byte per
 * cell, and per point and pass) stay with the results until they are freed.
 * Errors: HH_EINVAL (null arguments, membership was not kept), HH_ENOMEM,
 * HH_EDEVICE, HH_EINTERNAL (malformed result). */
HH_API hh_status hough_hier_solution(hh_result* const* results, int32_t n, double* kernel_ms);

/* The outcome of hough_hier_solution for one pass of a result. */
typedef struct {
    const uint8_t* keep;      /* [n_cells] 1 = the cell is kept, in the order of hough_hier_result_cells */
    int64_t n_cells;
    const uint8_t* plotted;   /* [n_points] 1 = point id k was plotted by this pass              */
    int64_t n_points;
    int64_t kept;             /* number of kept cells                                              */
    int64_t plotted_points;   /* number of plotted points                                          */
    int64_t rounds;           /* rounds of segment walks of the hough_hier_solution call           */
} hh_solution;

/* on_device = 1 returns device arrays, on_device = 0 host copies owned by the
 * result; both stay valid until hough_hier_result_free().  A pass that was not
 * enabled has no cells and no plotted points.
 * Errors: HH_EINVAL (bad pass, hough_hier_solution not run on res), HH_EDEVICE. */
HH_API hh_status hough_hier_result_solution(hh_result* res, int32_t pass, int32_t on_device, hh_solution* out);

/* The output image of solution() (Sec. 3: the plotted points make up the
 * output image): height rows of width bytes, row r at image + r *
 * row_stride, set to 255 where a point plotted by any enabled pass lies and 0
 * elsewhere.  image is caller-owned host memory (on_device = 0) or device
 * memory (on_device = 1); the call waits until it is written.
 * Errors: HH_EINVAL (null arguments, row_stride < width, hough_hier_solution not
 * run on res), HH_ENOMEM, HH_EDEVICE. */
HH_API hh_status hough_hier_result_solution_image(hh_result* res, uint8_t* image, int64_t row_stride,
                                                  int32_t on_device);

/* ---- For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.
 *
 * hough_hier_detect_noalloc runs one detection like hough_hier_detect (same
 * cells, voters and statistics) but takes every device buffer it needs from
 * a fixed scratch array inside the library, HH_NOALLOC_SCRATCH_BYTES per
 * device (held by each device the library runs on until the process ends),
 * and calls no device allocation or free.  The caller passes the input and
 * the output buffers:
 *   cells    device array of cells_cap hh_cell: the detected cells in
 *            (pass, key) order, member_off indexing `members`;
 *   members  device array of members_cap int32 point ids (each cell's voters,
 *            ascending, cells after cells), or NULL when membership is off;
 *   stats    host array of 2 * (HH_MAX_DEPTH + 1) hh_level_stats: pass p's
 *            level l at stats[p * (HH_MAX_DEPTH + 1) + l], zero past the
 *            finest level and for a pass not enabled;
 *   n_cells  host int64[2]: detected cells per pass; *n_members: voter ids.
 * A host input is staged into the scratch by copies.  The call waits until
 * the outputs are written.  Every call on a device uses that device's one
 * scratch array (the contents of the last call stay there): calls that
 * overlap on one device -- on two contexts, or on two threads -- race, so
 * serialise them.  Calls on one context are serialised by its lock.
 * Errors: as hough_hier_detect; HH_ECAPACITY when the call needs more scratch
 * than HH_NOALLOC_SCRATCH_BYTES, or more cells or ids than the output buffers
 * hold (then n_cells and *n_members report what the call found). */
#define HH_NOALLOC_SCRATCH_BYTES (256ull << 20)
HH_API hh_status hough_hier_detect_noalloc(hh_ctx* ctx, const hh_input* in, hh_cell* cells, int64_t cells_cap,
                                           int32_t* members, int64_t members_cap, hh_level_stats* stats,
                                           int64_t* n_cells, int64_t* n_members);

/* Text of the last error recorded by a call on res (its accessors, solution
 * and image calls).  Results of a serving context record their errors on the
 * serving lane that made them, not on the context passed to poll, so read
 * them here (never NULL; empty if none). */
HH_API const char* hough_hier_result_last_error(const hh_result* res);

/* Release a result (its device memory returns to the context, where the
 * context's next call may reuse it: finish any work that reads the result's
 * device arrays first).  Does not wait for calls running on the context.
 * NULL is accepted. */
HH_API void hough_hier_result_free(hh_result* res);

#ifdef __cplusplus
}
#endif

#endif /* HOUGH_HIER_H */
