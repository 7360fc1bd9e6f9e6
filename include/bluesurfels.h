/*
 * bluesurfels.h -- C ABI of the MI355X (gfx950) greedy blue-noise surfel
 * ordering library (libbluesurfels.so).
 *
 * The operation is the progressive ordering of candidate surfels from
 * "Rendering of Complex Heterogenous Scenes using Progressive Blue Surfels"
 * (Brandt, Jaehn, Fischer, Meyer auf der Heide; arXiv 1904.08225), Sec. 3.2
 * and Sec. 3.3: start at a random candidate, then repeatedly append the
 * remaining candidate whose distance to its nearest already chosen surfel is
 * largest, and remove it, until k surfels are chosen.  The result is a
 * greedy permutation (farthest-first traversal): every prefix of the
 * ordered array is an r-net of the candidates (Sec. 4.1), so a renderer
 * picks a level of detail by drawing a prefix.
 *
 * Exactness contract (the paper does not fix the arithmetic; these are the
 * library's readings):
 *   - distances are squared Euclidean in binary32 with a fixed association
 *     and no contraction:  d2 = ((dx*dx + dy*dy) + dz*dz),  dx = a.x - b.x;
 *   - the selection compares d2 values; ties go to the lowest index;
 *   - out_radius[t] = sqrtf(d2 of out_order[t] to its nearest earlier pick),
 *     correctly rounded; out_radius[0] = +inf;
 *   - a chosen candidate is never chosen again, also at distance 0;
 *   - the start is SplitMix64(seed) mod n (first output of SplitMix64,
 *     Steele, Lea and Flood 2014) unless an explicit start is given.
 * Every entry point returns the same orders and radii, bit for bit, for the
 * same (points, k, start), whichever kernel or tiling it uses.
 *
 * Conventions for every entry point:
 *   - pointers named d_* or documented as device pointers are device memory
 *     (hipMalloc / PyTorch CUDA tensors) on the current HIP device; h_*
 *     pointers are host memory;
 *   - the caller owns every input, output and workspace buffer; the library
 *     never frees them;
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue
 *     work and return without waiting; errors that the host can detect
 *     (null pointers, bad sizes, too small workspace) are returned
 *     synchronously and nothing is enqueued;
 *   - candidates with a non-finite coordinate are detected on the device;
 *     the outputs are then out_order[:] = -1 and out_radius[:] = NaN;
 *   - the cooperative kernels wait for one another at every step with a
 *     bounded wait (about a second); if one gives up, every workgroup
 *     leaves and the outputs become out_order[:] = -2, out_radius[:] = NaN
 *     (bs_order_status reports it as BS_ERR_TIMEOUT).
 *   - normals and colours are accepted for interface completeness (a surfel
 *     is position + normal + material, Sec. 3.1) but the selection ignores
 *     them, as the paper's sampling does (Sec. 5 limitations); they may be
 *     NULL.
 * All functions are thread-safe except where a handle is shared without
 * external locking.
 */
#ifndef BLUESURFELS_H
#define BLUESURFELS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef enum {
    BS_OK = 0,
    BS_ERR_INVALID_ARG = -1,   /* bad pointer / size / argument */
    BS_ERR_OUT_OF_MEMORY = -2, /* device allocation failed */
    BS_ERR_HIP = -3,           /* a HIP runtime call failed */
    BS_ERR_OVER_BUDGET = -4,   /* server: job exceeds the HBM budget */
    BS_ERR_NOT_READY = -5,     /* server: job not finished yet */
    BS_ERR_UNSUPPORTED = -6,   /* no kernel for this size / device */
    BS_ERR_TIMEOUT = -7,       /* a wait exceeded its deadline */
    BS_ERR_DEVICE = -8         /* a kernel reported an internal error */
} bs_status;

/* Human readable name of a status code (static string). */
const char* bs_error_string(int code);
/* Detail message of the last error on the calling thread (static storage
 * per thread, valid until the next call on that thread). */
const char* bs_last_error_message(void);
/* Library version as "major.minor.patch". */
const char* bs_version(void);

/* ---------------------------------------------------------------- tuning */
typedef enum {
    BS_KERNEL_AUTO = 0,  /* library picks (autotuned table; without one: up to 4,096
                            candidates BS_KERNEL_WG, from 4,097 (two workgroups) to
                            4,194,304 BS_KERNEL_COOP with 256 picks per step (128 below
                            64 workgroups), above
                            that BS_KERNEL_GRID) */
    BS_KERNEL_WG = 1,    /* one workgroup, candidates resident in registers */
    BS_KERNEL_COOP = 2,  /* cooperative workgroups, resident, full scan (several picks
                            per step with tuning picks > 1) */
    BS_KERNEL_GRID = 3   /* uniform-grid radius-pruned kernel */
} bs_kernel;

typedef struct {
    int32_t kernel;        /* bs_kernel */
    int32_t block;         /* threads per workgroup (0 = auto) */
    int32_t per_thread;    /* candidates per thread for resident kernels (0 = auto) */
    int32_t groups;        /* workgroups of a cooperative launch (0 = auto) */
    float cell_points;     /* grid kernel: target mean candidates per cell (0 = auto) */
    int32_t picks;         /* grid kernel: most picks per round, 0 = auto, 1 = one pick
                              per round, 2..32 = several exact picks per round (same
                              result; see bs_order_ex).  Cooperative full scan
                              (BS_KERNEL_COOP; 1024-thread workgroups with 1, 2, 4, 8, 12 or
                              16 per thread, or 512-thread with 24 or 32; 2..256
                              workgroups): 2..256 = several exact picks per step over
                              the candidates in Morton order, every workgroup a bucket
                              offering its four best keys, five in the 128-pick
                              kernel.  Batch plans: most exact picks per round of
                              each object, 1..32 (same result); 0 = 24, or 16 for
                              an object whose cells average more than 64
                              candidates */
    int32_t lead_picks;    /* grid kernel with several picks per round: the first picks
                              come from the cooperative full scan over all CUs, which
                              then hands every candidate's distance to the grid kernel
                              (same result).  0 = auto (n / 1024 picks from n >= 2^18
                              candidates when a cooperative scan holds n), -1 = none,
                              >= 2 = that many (capped at k; BS_ERR_UNSUPPORTED if no
                              cooperative scan holds n) */
    int32_t batch_wide;    /* batch plans: how many of the objects with the largest k are
                              ordered by 1024-thread workgroups (a second persistent
                              kernel beside the 256-thread one, on `groups` CUs; same
                              result).  0 = auto (objects with k >= 65536 and more than
                              half the mean k per 256-thread workgroup slot), -1 = none.
                              For batch plans `groups` is the number of those 1024-thread
                              workgroups (one CU each; 0 = three quarters of the CUs) */
    int32_t spin_limit;    /* cooperative kernels: polls of a bounded wait for the other
                              workgroups before giving up (0 = default, about a second).
                              A small value forces the give-up path from the host (tests
                              of the error contract); results are unchanged otherwise */
    int32_t reserved[3];   /* must be zero */
} bs_tuning;

/* ------------------------------------------------------- single instance */

/*
 * Greedy permutation of n candidates (paper Sec. 3.2, 3.3).
 *   d_points   device float[n][3] (AoS, row-major, 12-byte stride)
 *   d_normals  device float[n][3] or NULL (not read by the ordering)
 *   d_colors   device uint8[n][3] or NULL (not read by the ordering)
 *   n          number of candidates, 1 <= n < 2^31 (n may be 0 when k == 0)
 *   k          number of surfels to order, 0 <= k <= n (k == 0: no-op)
 *   seed       start = SplitMix64(seed) mod n
 *   d_out_order   device int32[k]: candidate indices in greedy order
 *   d_out_radius  device float[k] or NULL: distance of each pick to its
 *                 nearest earlier pick (covering radius of the prefix)
 * The library allocates its workspace from a stream-ordered pool
 * (hipMallocAsync) and frees it stream-ordered.  Errors: BS_ERR_INVALID_ARG
 * (null pointers, k < 0, k > n, n >= 2^31), BS_ERR_OUT_OF_MEMORY, BS_ERR_HIP.
 */
int bs_order(const float* d_points, const float* d_normals, const uint8_t* d_colors,
             int64_t n, int64_t k, uint64_t seed,
             int32_t* d_out_order, float* d_out_radius, void* stream);

/*
 * As bs_order with an explicit start, a caller-owned workspace and an
 * optional tuning override.
 *   start_index   0 <= start_index < n, or -1 to derive it from `seed`
 *   d_workspace   device buffer of at least bs_workspace_size(n, k, tuning)
 *                 bytes, 256-byte aligned; its contents on entry do not
 *                 matter; concurrent calls must not share it
 *   tuning        NULL = automatic choice
 * Errors: as bs_order, plus BS_ERR_INVALID_ARG for a too small or
 * misaligned workspace and BS_ERR_UNSUPPORTED if the forced kernel cannot
 * hold n candidates.
 */
int bs_order_ex(const float* d_points, const float* d_normals, const uint8_t* d_colors,
                int64_t n, int64_t k, uint64_t seed, int64_t start_index,
                int32_t* d_out_order, float* d_out_radius,
                void* d_workspace, size_t workspace_bytes,
                const bs_tuning* tuning, void* stream);

/*
 * Profiling form of bs_order_ex (same ordering, same workspace size, same
 * kernels).  Two optional instruments:
 *   d_step_ticks  NULL or device uint64[k]: the device wall clock (see
 *                 bs_wall_clock_hz) right after pick t is emitted, so that
 *                 consecutive differences are per-step latencies;
 *   event_begin,  NULL or hipEvent_t handles created by the caller: recorded
 *   event_end     on `stream` immediately before and after the launch of the
 *                 ordering kernel itself (after validation and grid build),
 *                 so hipEventElapsedTime gives that kernel's duration.
 * start_index as in bs_order_ex, with -1 meaning SplitMix64(0) mod n.
 * Errors: as bs_order_ex; BS_ERR_HIP if an event cannot be recorded.
 */
int bs_order_profile(const float* d_points, int64_t n, int64_t k, int64_t start_index,
                     int32_t* d_out_order, float* d_out_radius, uint64_t* d_step_ticks,
                     void* event_begin, void* event_end,
                     void* d_workspace, size_t workspace_bytes, const bs_tuning* tuning,
                     void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * ordering of bs_order_ex with the workspace taken from a device array the
 * library holds, one per GPU, from module load to process exit
 * (bs_noalloc_max_bytes() bytes: 64 MiB, the several-picks scan up to
 * 524,288 candidates).  The call allocates nothing and frees nothing; the
 * caller passes inputs and outputs.  Every call on one GPU shares that GPU's
 * array, so calls that overlap on one GPU race: order them (one stream, or
 * events).  Arguments as bs_order_ex (start_index -1 = from seed; tuning
 * NULL = automatic).  Errors: as bs_order_ex; BS_ERR_UNSUPPORTED when
 * bs_workspace_size(n, k, tuning) exceeds the array; BS_ERR_HIP if the
 * array's device address cannot be found (looked up on a device's first
 * call, with that device current).
 */
int bs_order_noalloc(const float* d_points, int64_t n, int64_t k, uint64_t seed, int64_t start_index,
                     int32_t* d_out_order, float* d_out_radius, const bs_tuning* tuning, void* stream);
/* Bytes of the per-GPU array bs_order_noalloc uses as its workspace. */
size_t bs_noalloc_max_bytes(void);

/*
 * Status of the last ordering enqueued on `d_workspace` (bs_order_ex,
 * bs_order_profile): waits for `stream` (a hipStream_t), then reads the
 * workspace's device header.  Returns BS_OK; BS_ERR_INVALID_ARG if a
 * coordinate was not finite (outputs -1 / NaN); BS_ERR_TIMEOUT if a
 * cooperative kernel's bounded wait gave up (outputs -2 / NaN);
 * BS_ERR_HIP if the stream reports an error.  Synchronous.
 */
int bs_order_status(const void* d_workspace, void* stream);

/* Frequency of the device wall clock used by bs_order_profile (Hz); 0 on error. */
double bs_wall_clock_hz(void);

/* Workspace bytes bs_order_ex needs for (n, k, tuning); 0 if unsupported. */
size_t bs_workspace_size(int64_t n, int64_t k, const bs_tuning* tuning);

/* The start index bs_order uses for (seed, n): SplitMix64(seed) mod n;
 * -1 if n < 1. */
int64_t bs_start_index(uint64_t seed, int64_t n);

/* Which kernel the automatic choice uses for (n, k) (a bs_kernel value). */
int bs_auto_kernel(int64_t n, int64_t k);

/*
 * The plan bs_order_ex follows for (n, k, tuning), every automatic choice
 * resolved into *out: kernel; for the resident kernels block, per_thread and
 * groups; for the grid kernel block, cell_points, picks and lead_picks (-1
 * when no leading scan runs), and with a leading scan per_thread and groups
 * of that cooperative scan (1024-thread workgroups).  A NULL tuning takes the
 * autotuner's table entry as bs_order does.  Reads no device memory.
 * Errors: BS_ERR_INVALID_ARG (null out, bad sizes or tuning),
 * BS_ERR_UNSUPPORTED (no kernel for this size and tuning).
 */
int bs_plan_describe(int64_t n, int64_t k, const bs_tuning* tuning, bs_tuning* out);

/* ------------------------------------------------- ordered surfel buffer */

/*
 * One surfel of an ordered vertex buffer: the paper stores an approximation
 * as one contiguous buffer of surfels (position, normal, material) whose
 * every prefix is a level of detail (Sec. 3); Table 1 implies 20 bytes per
 * surfel.  The packing is this library's reading (the paper does not give
 * it): position as binary32; the normal as an octahedral code (Meyer et al.
 * 2010): p = (n.x, n.y) / (|n.x| + |n.y| + |n.z|), folded to
 * ((1 - |p.y|) sgn p.x, (1 - |p.x|) sgn p.y) for n.z < 0 (sgn 0 = +1), each
 * component round-to-nearest-even(clamp(p, -1, 1) * 32767); colour r, g, b
 * and a = 255.
 */
typedef struct {
    float x, y, z;
    int16_t normal[2];  /* octahedral code; (0, 0) for a zero / non-finite normal or no normals */
    uint8_t rgba[4];    /* (255, 255, 255, 255) without colours */
} bs_surfel;

/*
 * Gather the ordered surfels: d_out[t] = record of candidate d_order[t],
 * t < k.  d_normals (float[n][3]) and d_colors (uint8[n][3]) may be NULL.
 * An order entry outside [0, n) (a non-finite input's -1) gives a record
 * with NaN position, normal (0, 0) and colour (0, 0, 0, 0).  All pointers
 * are device memory; the call enqueues one kernel on `stream`.
 * Errors: BS_ERR_INVALID_ARG (null pointers with k > 0, k < 0, n < 0),
 * BS_ERR_HIP.
 */
int bs_emit_surfels(const float* d_points, const float* d_normals, const uint8_t* d_colors, int64_t n,
                    const int32_t* d_order, int64_t k, bs_surfel* d_out, void* stream);

/*
 * r_m of the prefix-length estimate (Sec. 4.1): the median, over the first
 * p_m ordered surfels, of each one's distance to its nearest other surfel in
 * that prefix (binary32, d2 = (dx*dx + dy*dy) + dz*dz, correctly rounded
 * sqrt; an even count takes 0.5f * (a + b) of the middle two).  Writes one
 * float to d_out_rm (device memory) on `stream`; NaN if an order entry lies
 * outside [0, n).  2 <= p_m <= 4096.
 * Errors: BS_ERR_INVALID_ARG, BS_ERR_HIP.
 */
int bs_prefix_median_nn(const float* d_points, int64_t n, const int32_t* d_order, int64_t p_m, float* d_out_rm,
                        void* stream);

/*
 * Estimated prefix length for surfel radius r (Sec. 4.1):
 * p(r) = p_m (r_m / r)^2, rounded up and clamped to [1, k]; k when r <= 0.
 * Host only.
 */
int64_t bs_prefix_length(double r, double r_m, int64_t p_m, int64_t k);

/*
 * Exact prefix length for radius r from an ordering's radii (host memory,
 * h_radius[t] = covering radius of the t-prefix, non-increasing): the least
 * t >= 1 with h_radius[t] <= r, so that every candidate lies within r of the
 * first t surfels; k if there is none.  Host only.
 */
int64_t bs_prefix_for_radius(const float* h_radius, int64_t k, float r);

/*
 * The Morton (Z-order) layout the ordering kernels keep candidates in.  This
 * is not an operation of the paper (it is how this library lays out the
 * candidates for the pruned update): 30-bit codes from a 2^10-per-axis
 * quantization of the bounding box, scaled by its longest side
 * (binary32: q = (int)((p - lo) * (1024.0f / extent)), clamped to
 * [0, 1023]; x in the lowest bit of each triple), sorted stably, so equal
 * codes stay in index order.  Exposed for spatially coherent surfel layouts
 * and to check the sort.
 *   bs_morton_order: d_out_perm[i] = index of the i-th candidate in that
 *     order (device int32[n]); workspace of bs_morton_workspace_size(n)
 *     bytes, 256-byte aligned, owned by the caller.  n = 0 is a no-op.
 *   (bs_batch_morton_order, with the batch functions below, does the same
 *     for every object of a batch plan.)
 * Enqueued on `stream`.  Errors: BS_ERR_INVALID_ARG (null pointers, n < 0,
 * n >= 2^31, small or misaligned workspace), BS_ERR_HIP.
 */
size_t bs_morton_workspace_size(int64_t n);
int bs_morton_order(const float* d_points, int64_t n, int32_t* d_out_perm, void* d_workspace, size_t workspace_bytes,
                    void* stream);

/* ------------------------------------------------------------ autotuner */

/*
 * Autotuner: times candidate configurations (resident full scan, cooperative
 * full scan, grid kernel with 512/1024 threads, cell occupancies 4..32, one
 * or several picks per round) on the caller's points for a prefix of the
 * ordering (max(1024, k/8) picks), and keeps the fastest in a per-device
 * table keyed by (floor(log2 n), floor(log2 k)).  Calls with a NULL tuning
 * (bs_order, bs_order_ex, bs_workspace_size, bs_auto_kernel) use the table
 * entry of their size when there is one; query bs_workspace_size after
 * tuning.  Every configuration gives the same ordering; only speed differs.
 *   d_points     device float[n][3]
 *   1 <= k <= n  the ordering to tune for; seed as in bs_order
 *   out_tuning   host: receives the chosen configuration
 * Synchronous: allocates scratch from the stream-ordered pool, runs the
 * candidates on `stream` and waits for them.  Errors: BS_ERR_INVALID_ARG
 * (also: the tuning cache file named below could not be written; the
 * in-memory entry and *out_tuning are still set), BS_ERR_OUT_OF_MEMORY,
 * BS_ERR_UNSUPPORTED (no candidate fits), BS_ERR_HIP.
 *
 * Environment:
 *   BS_TUNE_CACHE=path   bs_autotune also records its winner in this text
 *                        file, one line per (GPU architecture, floor(log2 n),
 *                        floor(log2 k)); calls with a NULL tuning read it when
 *                        the in-memory table has no entry for their size, so
 *                        a later process reuses earlier tuning runs.
 *   BS_FORCE_KERNEL=wg|scan|several|grid
 *                        calls with a NULL tuning take this kernel instead of
 *                        the automatic choice (one resident workgroup, the
 *                        cooperative full scan with one pick per step or with
 *                        several, the grid-pruned kernel).  Any other value
 *                        makes them fail with BS_ERR_INVALID_ARG.
 */
int bs_autotune(const float* d_points, int64_t n, int64_t k, uint64_t seed,
                bs_tuning* out_tuning, void* stream);

/* The table entry for (n, k) on the current device: BS_OK and *out_tuning,
 * or BS_ERR_NOT_READY when that size has not been tuned. */
int bs_autotune_lookup(int64_t n, int64_t k, bs_tuning* out_tuning);

/* Forget every tuned entry (all devices); the next lookup reads the
 * BS_TUNE_CACHE file again. */
void bs_autotune_clear(void);

/*
 * Autotuner for a batch (arguments as bs_batch_plan_create, plus the
 * device candidates d_points): orders a sample of the objects (the four with
 * the largest k and twelve spread over the rest, each cut to at most 4096
 * picks) as batches with cell occupancies 4, 8, 16 and 32 candidates and
 * returns the fastest in out_tuning->cell_points (kernel = BS_KERNEL_GRID),
 * to pass to bs_batch_plan_create.  When the batch has objects for the
 * 1024-thread workgroups (bs_tuning.batch_wide) and at most 2^27 picks in
 * all, it then orders the whole batch once for each share of the CUs given
 * to those workgroups (4/8 .. 7/8) and returns the fastest in
 * out_tuning->groups (this needs the batch's workspace and outputs a second
 * time, allocated from the stream-ordered pool).  Synchronous; errors as
 * bs_autotune.
 */
int bs_batch_autotune(const int64_t* h_offsets, const int64_t* h_k, const uint64_t* h_seed,
                      int32_t m, const float* d_points, bs_tuning* out_tuning, void* stream);

/* -------------------------------------------------------------- batched */

/*
 * Batched ordering of many independent objects (the per-node approximations
 * of a scene, paper Sec. 3.4 and Sec. 5: the sampling parallelises over the
 * objects of a scene).  Every object's result is bit-identical to ordering
 * it alone with bs_order(seed = h_seed[j]).
 *
 * Candidates of all objects lie in one device array in CSR form: object j
 * owns rows h_offsets[j] .. h_offsets[j+1]-1 of d_points (float[N][3]).
 * Its k_j = h_k[j] picks are written to rows out_off[j] .. out_off[j]+k_j-1
 * of d_out_order / d_out_radius, where out_off is the exclusive prefix sum
 * of h_k (bs_batch_out_offsets); indices are local to the object
 * (0 .. n_j-1).
 *
 * The plan copies its host arrays; it owns a few small device arrays and,
 * after the first execute, a captured hipGraph of the ordering launch (one
 * persistent work-queue kernel whose 256-thread workgroups order objects
 * largest-k first).  Preprocessing (per-object grids) and the queue reset
 * are enqueued as ordinary launches before the graph.  The objects with the
 * longest chains (bs_tuning.batch_wide) are ordered meanwhile by a second
 * persistent kernel of 1024-thread workgroups on a stream of the plan,
 * forked from and joined back into `stream`.
 *
 *   h_offsets  host int64[m+1], non-decreasing, h_offsets[0] = 0, total < 2^31
 *   h_k        host int64[m], 0 <= k_j <= n_j
 *   h_seed     host uint64[m] or NULL (all 0): start_j = SplitMix64(seed_j) mod n_j
 *   tuning     NULL or cell_points (target candidates per grid cell, >= 8)
 * Errors: BS_ERR_INVALID_ARG (bad sizes), BS_ERR_OUT_OF_MEMORY, BS_ERR_HIP.
 */
typedef struct bs_batch_plan bs_batch_plan;
int bs_batch_plan_create(const int64_t* h_offsets, const int64_t* h_k, const uint64_t* h_seed,
                         int32_t m, const bs_tuning* tuning, bs_batch_plan** out_plan);
/* Device workspace bytes bs_batch_plan_execute needs (256-byte aligned). */
size_t bs_batch_workspace_size(const bs_batch_plan* plan);
/* Sum of k over the objects (length of the output arrays). */
int64_t bs_batch_total_k(const bs_batch_plan* plan);
/* Writes the m+1 output offsets (exclusive prefix sum of h_k) to host memory. */
int bs_batch_out_offsets(const bs_batch_plan* plan, int64_t* h_out_offsets);
/*
 * Enqueue the batched ordering on `stream`.  d_out_radius may be NULL.
 * Objects whose candidates contain a non-finite coordinate get order -1 and
 * radius NaN; the others are unaffected.  Calls with the same plan are
 * serialised by the plan; distinct plans may run concurrently on distinct
 * workspaces.
 */
int bs_batch_plan_execute(bs_batch_plan* plan, const float* d_points, int32_t* d_out_order,
                          float* d_out_radius, void* d_workspace, size_t workspace_bytes,
                          void* stream);

/*
 * Each object's candidates in the Morton layout of bs_morton_order, every
 * object sorted within its own rows: row i of object j (rows h_offsets[j] ..
 * h_offsets[j+1]-1 of d_out_perm, device int32[N]) receives an index local
 * to the object.  Workspace as for bs_batch_plan_execute.  Enqueued on
 * `stream`.  Errors: BS_ERR_INVALID_ARG, BS_ERR_HIP.
 */
int bs_batch_morton_order(bs_batch_plan* plan, const float* d_points, int32_t* d_out_perm, void* d_workspace,
                          size_t workspace_bytes, void* stream);
void bs_batch_plan_destroy(bs_batch_plan* plan);
/*
 * The randomized sampler (bs_sample, paper Sec. 3.2) over the plan's objects
 * instead of the exact ordering: one persistent launch whose 256-thread
 * workgroups take objects largest k first.  Object j's picks are bit-identical
 * to bs_sample on it alone with seed h_seed[j].  Outputs and workspace as
 * bs_batch_plan_execute; d_out_count: NULL or device int32[m] (objects as
 * given; 0 for objects with k = 0).  params NULL = bs_sampler_defaults().
 * Defined after the sampler's parameter struct below.
 */

/* ----------------------------- visible-surface capture (paper Sec. 3.1) */

/*
 * An analytic primitive of a node (world = rot * local + center).
 *   kind 0 sphere: prm[0] radius;  kind 1 box: prm = half extents;
 *   kind 2 cylinder along local z: prm[0] radius, prm[1] half height (capped).
 */
typedef struct {
    int32_t kind;
    float center[3];
    float rot[9];      /* row-major 3 x 3, local -> world */
    float prm[3];
    uint8_t rgb[4];    /* colour; rgb[3] unused */
} bs_primitive;

/* Device workspace bytes of bs_capture at `resolution` pixels per side
 * (a G-buffer of 32 B per pixel of the eight views); 0 if out of 1..8192. */
size_t bs_capture_workspace_size(int32_t resolution);

/*
 * The initial surfel set of a node (Sec. 3.1): its visible surface seen from
 * the eight corners of its bounding box with orthographic projection towards
 * the box centre, resolution^2 pixels per view (the paper uses 1024^2); every
 * covered pixel gives one candidate: the first primitive surface its ray
 * meets (position, unit normal, the primitive's colour).  The camera of view
 * v (bits x, y, z of v pick hi over lo): c = (lo + hi) / 2, s = |hi - lo| / 2,
 * d = (c - corner) / |c - corner|, u = d x (0,0,1) normalised (d x (0,1,0)
 * when that is shorter than 1e-6), w = u x d; pixel (i, j) casts along d from
 * c + a u + b w - 2 s d, a = ((2 i + 1) / resolution - 1) s, b likewise.
 * Nearest t > 0 wins, the lower primitive index on equal t.  Binary32 with a
 * fixed operation order; candidates in view, row, column order.  Spheres,
 * boxes and capped cylinders (no tori).
 *   d_prims          device bs_primitive[count]
 *   h_lo, h_hi       host float[3]: the node's bounding box (finite, lo <= hi)
 *   d_out_points     device float[8 resolution^2][3] (capacity)
 *   d_out_normals    device float[8 resolution^2][3] or NULL
 *   d_out_colors     device uint8[8 resolution^2][3] or NULL
 *   d_out_count      device int64[1]: candidates written
 *   d_workspace      bs_capture_workspace_size(resolution) bytes, 256-byte aligned
 * The outputs feed bs_order / bs_sample directly (the count stays on the
 * device; read it back to size the ordering).  Enqueues three kernels.
 * Errors: BS_ERR_INVALID_ARG, BS_ERR_HIP.
 */
int bs_capture(const bs_primitive* d_prims, int32_t count, const float* h_lo, const float* h_hi, int32_t resolution,
               float* d_out_points, float* d_out_normals, uint8_t* d_out_colors, int64_t* d_out_count,
               void* d_workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------ randomized sampler (paper Sec. 3.2) */

/*
 * Parameters of the paper's randomized progressive sampler (Sec. 3.2), which
 * approximates the greedy permutation with rounds of random samples.
 */
typedef struct {
    int32_t sample_size;    /* candidates drawn per round, 1..256 (the paper: about 200); 0 = the
                               whole remaining set, which makes every pick the exact greedy one */
    int32_t growth_rounds;  /* after every growth_rounds rounds one more pick is taken from each
                               sample (the paper: 500); < 0 = one pick per round; 0 is invalid */
    float vicinity;         /* v > 0: after a round, its sample members whose squared distance to
                               the nearest chosen surfel is below v^2 times that of the round's
                               first pick are removed from the input (the paper's optional removal
                               of samples near the chosen ones, for which it gives no threshold);
                               0 = no removal (needs sample_size > 0 otherwise) */
    int32_t reserved[5];    /* must be zero */
} bs_sampler;

/* The paper's values: 200 samples per round, one more pick every 500 rounds, no removal. */
bs_sampler bs_sampler_defaults(void);

/* Device workspace bytes bs_sample needs for n candidates (0 if n is out of range). */
size_t bs_sample_workspace_size(int64_t n);

/*
 * The paper's randomized approximation of the greedy permutation (Sec. 3.2):
 * the start (SplitMix64(seed) mod n, or start_index >= 0), then rounds
 * i = 0, 1, ...: draw a random sample of the remaining candidates; append the
 * member whose distance to all chosen surfels is largest (binary32 d2 as in
 * the exact ordering, lowest index on ties) and remove it, 1 + floor(i /
 * growth_rounds) times from the same sample; optionally remove sample members
 * near the chosen surfels; stop after k picks or when the input is empty.
 * The draws: slot j of round i tries up to 16 times the candidate
 * floor(u * n / 2^32), u the first output word of Philox4x32-10 (Salmon et
 * al., SC 2011) with counter (i, j, attempt, 0) and key (low, high 32 bits of
 * seed), and keeps the first one that remains; a candidate named by two slots
 * counts once; a round whose slots all miss takes the farthest remaining
 * candidate.  The result depends only on (points, k, seed, start, params).
 *   params        NULL = bs_sampler_defaults()
 *   d_out_order   device int32[k]: picks; entries from the count on (the input ran
 *                 out, only with vicinity > 0) are -3, their radius NaN
 *   d_out_radius  device float[k] or NULL: each pick's distance to the surfels
 *                 chosen before it (+inf for the start)
 *   d_out_count   device int32[1] or NULL: picks made (not written when k == 0)
 *   d_workspace   device, at least bs_sample_workspace_size(n) bytes, 256-byte aligned
 * Non-finite coordinates give order -1, radius NaN, count 0.  Enqueues on
 * `stream` (one workgroup orders the object).  Errors: BS_ERR_INVALID_ARG
 * (sizes, pointers, parameters, workspace), BS_ERR_HIP.
 */
int bs_sample(const float* d_points, int64_t n, int64_t k, uint64_t seed, int64_t start_index,
              const bs_sampler* params, int32_t* d_out_order, float* d_out_radius, int32_t* d_out_count,
              void* d_workspace, size_t workspace_bytes, void* stream);

/*
 * Sec. 3.3 compares orderings by each prefix surfel's distance to its nearest
 * other surfel of the prefix: d_out[a] = sqrtf(min over b != a, b < p of
 * d2(points[order[a]], points[order[b]])), a < p (binary32 with the fixed d2;
 * +inf for p = 1); NaN everywhere if an order entry lies outside [0, n).
 * 1 <= p <= min(n, 2^20); all pointers device memory; one kernel on `stream`.
 */
int bs_prefix_nn(const float* d_points, int64_t n, const int32_t* d_order, int64_t p, float* d_out,
                 void* stream);

/* The sampler over a batch plan (see bs_batch_plan_execute above). */
int bs_batch_plan_execute_sample(bs_batch_plan* plan, const bs_sampler* params, const float* d_points,
                                 int32_t* d_out_order, float* d_out_radius, int32_t* d_out_count,
                                 void* d_workspace, size_t workspace_bytes, void* stream);

/* ------------------------------ hierarchical generation (paper Sec. 3.4) */

/*
 * Bottom-up generation over a scene hierarchy (Sec. 3.4): the paper makes one
 * approximation per complex subtree and, bottom-up, takes the surfels already
 * chosen for a node's children as that node's initial candidates.  Here node
 * j's candidates are, for a leaf (a node no other node names as parent), its
 * own rows h_leaf_offsets[j] .. h_leaf_offsets[j+1]-1 of d_points; for an
 * inner node, the k picks of each child, children in increasing node order,
 * each child's picks in order.  Every node is then ordered like a batch object
 * (exact greedy, or the randomized sampler), so node j's picks equal
 * bs_order (or bs_sample) with seed h_seed[j] on that candidate array.  Nodes
 * of equal depth form one batched launch (a single node: the single-object
 * path over all CUs); depths run leaves first.
 *   m               nodes, numbered so that a parent comes after its children
 *   h_parent        host int32[m]: the parent, or -1
 *   h_leaf_offsets  host int64[m+1], non-decreasing from 0: leaves' rows (inner nodes
 *                   have empty ranges); total < 2^31
 *   h_k             host int64[m]: picks of node j, 0 <= k_j <= its candidate count
 *                   (the paper's budget for a subtree of T triangles is min(200,000, T/2))
 *   h_seed          host uint64[m] or NULL (0)
 *   tuning          NULL or as bs_batch_plan_create (cell_points, batch_wide)
 * Errors: BS_ERR_INVALID_ARG (a parent before its child, k outside its range,
 * rows given for an inner node, sizes), BS_ERR_UNSUPPORTED, BS_ERR_HIP.
 */
typedef struct bs_hier_plan bs_hier_plan;
int bs_hier_plan_create(int32_t m, const int32_t* h_parent, const int64_t* h_leaf_offsets, const int64_t* h_k,
                        const uint64_t* h_seed, const bs_tuning* tuning, bs_hier_plan** out_plan);
/* Device workspace bytes bs_hier_plan_execute needs (256-byte aligned). */
size_t bs_hier_workspace_size(const bs_hier_plan* plan);
/* Sum of k over the nodes (length of the outputs). */
int64_t bs_hier_total_k(const bs_hier_plan* plan);
/* Writes the m+1 output offsets (exclusive prefix sum of h_k) to host memory. */
int bs_hier_out_offsets(const bs_hier_plan* plan, int64_t* h_out_offsets);
/*
 * Enqueue the generation on `stream`.  Node j's picks go to rows
 * out_off[j] .. out_off[j]+k_j-1 of d_out_order (indices into the node's own
 * candidate array), d_out_radius (NULL allowed) and d_out_source (device
 * int32[total_k]: the row of d_points each pick came from, so that normals
 * and colours of the original candidates follow the surfel up the tree).
 * sampler NULL = exact greedy; else the randomized sampler with those
 * parameters.  A node whose candidates hold a non-finite coordinate gets
 * order -1 and source -1, and so do its ancestors.
 */
int bs_hier_plan_execute(bs_hier_plan* plan, const float* d_points, const bs_sampler* sampler,
                         int32_t* d_out_order, float* d_out_radius, int32_t* d_out_source, void* d_workspace,
                         size_t workspace_bytes, void* stream);
void bs_hier_plan_destroy(bs_hier_plan* plan);

/* -------------------------------------------------------------- serving */

/*
 * A serving loop with continuous batching under an HBM budget (the paper
 * generates approximations per scene node ahead of rendering, Sec. 3.4 and
 * Sec. 5.2; here orderings are requested and answered while others run).
 * Jobs are submitted from any host thread.  A persistent kernel of
 * `workgroups` ordering workers (1024 threads each) stays resident on the
 * device, leaving the other compute units to the preprocessing; a dispatcher
 * thread admits pending jobs, in arrival order, into micro-batches while the
 * job fits the remaining budget, builds their grids on a preprocessing
 * stream and publishes them into a device ring, from which each idle worker
 * claims the next job (largest k first within a micro-batch).  A job never
 * waits for another job to finish, only for a free worker (and, if the
 * device runs a micro-batch's preprocessing behind the resident workers, for
 * the stop that stall_us triggers; while workers are being stopped no new
 * micro-batch starts, and a full set is relaunched once they have left).
 * Each job is timed
 * from submit to the moment its completion flag (written by its worker into
 * pinned host memory) is observed.  Results are bit-identical to bs_order on
 * the same job.  Workers exit a few milliseconds after the last job and are
 * relaunched on demand (so a device-wide synchronisation waits at most that
 * long for them).
 */
typedef struct {
    size_t hbm_budget_bytes;     /* device bytes the server may hold at once (> 0) */
    int32_t device;              /* HIP device ordinal */
    int32_t max_inflight;        /* micro-batches admitted and not finished; 0 = 64 */
    int32_t max_jobs_per_batch;  /* 0 = 512 */
    int32_t poll_us;             /* dispatcher polling period while busy; 0 = 50 */
    float cell_points;           /* grid cell target, 0 = 8 */
    int32_t workgroups;          /* resident 1024-thread ordering workers (each holds a whole
                                    compute unit), 0 = three quarters of the compute units;
                                    at most seven eighths (the rest run the preprocessing) */
    int32_t stall_us;            /* a micro-batch whose preprocessing has not begun on the device
                                    this long after every earlier micro-batch was published stops
                                    the workers (the device is then running it behind them on one
                                    in-order hardware queue); they restart once it is published.
                                    0 = 5,000 */
    int32_t reserved[5];         /* must be zero */
} bs_server_config;

typedef struct {
    const float* d_points;   /* device float[n][3]; must stay valid until the job is done */
    int64_t n;
    int64_t k;               /* 0 <= k <= n */
    uint64_t seed;           /* start = SplitMix64(seed) mod n */
    int32_t* d_out_order;    /* device int32[k] */
    float* d_out_radius;     /* device float[k] or NULL */
    void* ready_event;       /* hipEvent_t recorded after the work that writes d_points, or
                                NULL when the points are complete at submit: the server reads
                                them on its own stream, after waiting for this event (which
                                must stay valid until the job is done) */
} bs_job;

typedef struct {
    int64_t submitted, admitted, completed, rejected;
    int64_t queued;            /* waiting for admission now */
    int64_t inflight_batches;  /* micro-batches on the device now */
    int64_t batches;           /* micro-batches launched so far */
    int64_t ordered_surfels;   /* sum of k over completed jobs */
    double p50_us, p99_us, mean_us, max_us;  /* submit -> done latency */
    double elapsed_s;          /* first submit -> last completion */
    double surfels_per_s;      /* ordered_surfels / elapsed_s */
    size_t hbm_in_use, hbm_peak;
    int64_t worker_launches;   /* sets of persistent workers launched so far */
    int64_t stall_stops;       /* times an overdue publication stopped the workers */
} bs_serving_stats;

typedef struct bs_server bs_server;
/* Errors: BS_ERR_INVALID_ARG, BS_ERR_HIP. */
int bs_server_create(const bs_server_config* cfg, bs_server** out_server);
/* Enqueue a job; returns a ticket.  BS_ERR_OVER_BUDGET if the job alone can
 * never fit the budget (it is then not queued). */
int bs_server_submit(bs_server* server, const bs_job* job, uint64_t* ticket);
/* *done = 1 once the job's outputs are complete (returns the job's status). */
int bs_server_poll(bs_server* server, uint64_t ticket, int* done);
/* Block until the job is done or timeout_us passes (< 0: no limit);
 * BS_ERR_TIMEOUT on timeout. */
int bs_server_wait(bs_server* server, uint64_t ticket, int64_t timeout_us);
/* Block until no job is queued or in flight. */
int bs_server_drain(bs_server* server, int64_t timeout_us);
int bs_server_stats(bs_server* server, bs_serving_stats* out);
/* Finishes the jobs still queued or in flight, then releases everything. */
void bs_server_destroy(bs_server* server);

#ifdef __cplusplus
}
#endif

#endif /* BLUESURFELS_H */
