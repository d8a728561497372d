/*
 * powersort_hip.h -- C ABI of the MI355X (gfx950) powersort library.
 *
 * Powersort is the stable natural mergesort of Munro & Wild, "Nearly-Optimal
 * Mergesorts: Fast, Practical Sorting Methods That Optimally Adapt to
 * Existing Runs" (ESA 2018).  It
 *   - splits the input into runs (Sec. 2: maximal weakly increasing blocks, or
 *     strictly decreasing blocks, which are reversed), extending runs shorter
 *     than a minimum run length w by insertion sort (App. B.3/B.4);
 *   - gives every boundary between adjacent runs its node power
 *     (Def. "Node Power");
 *   - merges adjacent runs stably in the order of the min-oriented Cartesian
 *     tree of the powers (Cor. "Cartesian tree", Alg. PowerSort), whose merge
 *     cost M = sum of merge result sizes (Sec. 2.2) is at most H n + 2 n
 *     (Thm. "powersort").
 *
 * Conventions for every entry point:
 *   - Pointers named d_* and the key/payload arrays are DEVICE pointers of the
 *     current HIP device; everything else is host memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *     enqueued on it; results are valid once the stream has been
 *     synchronised.  Argument checks happen before anything is enqueued: an
 *     error status means nothing was launched.
 *   - The caller owns every array passed in.  Unless ps_options.workspace is
 *     given, the library keeps one scratch allocation per stream (grown on
 *     demand, reused across calls) until ps_release(stream).
 *   - Calls on one stream are serialised by the stream; calls on different
 *     streams use different scratch memory and may overlap.
 *   - Keys: int32, uint32, int64, uint64 in their natural order; float32 in
 *     IEEE-754 totalOrder (-NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN;
 *     NaNs ordered by payload bits).  Output keys keep their bit patterns.
 *   - Limits: every segment (and every ps_sort, ps_merge_cost and
 *     ps_inspect input) holds fewer than 2^31 elements; a segmented batch
 *     may hold up to 2^63 - 1 elements in all (uint64 offsets).
 *   - No exceptions or aborts cross this ABI.
 */
#ifndef POWERSORT_HIP_H
#define POWERSORT_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PS_OK = 0,
    PS_ERR_INVALID_ARG = -1,   /* null pointer, bad key type, bad segment offsets, ... */
    PS_ERR_TOO_LARGE = -2,     /* a segment of 2^31 or more elements, n_total >= 2^63, or a
                                  sort too large for the fixed scratch of ps_sort_no_alloc */
    PS_ERR_OUT_OF_MEMORY = -3, /* scratch allocation failed (nothing enqueued) */
    PS_ERR_HIP = -4,           /* a HIP runtime call failed; see ps_last_error() */
    PS_ERR_UNSUPPORTED = -5    /* option outside the supported range (e.g. min_run > 64) */
} ps_status;

typedef enum {
    PS_KEY_I32 = 0,
    PS_KEY_U32 = 1,
    PS_KEY_I64 = 2,
    PS_KEY_U64 = 3,
    PS_KEY_F32 = 4
} ps_key_type;

/* ps_options.flags: merge by Alg. PeekSort (Sec. 3.1) instead of powersort.
 * The leaves are the same (runs of the Sec. 2 convention extended to the
 * minimum run length); the merge tree is the one Alg. PeekSort's recursion
 * builds over them (Mehlhorn's Method 1, proof of Thm. "peeksort"): a range
 * of leaves A[l..r] with first leaf A[l..e] and last leaf A[s..r] is cut,
 * with m = l + floor((r - l) / 2), after its first leaf if m <= e, before its
 * last leaf if m >= s, and otherwise before the leaf A[i..j] holding m if
 * m - i < j - m, else after it.  Every entry point takes it; the output is
 * the same stable sort, the merge cost M (and ps_inspect's tree) are
 * peeksort's.  For ps_inspect, powers[j] then holds depth(j) + 1 of node j. */
#define PS_FLAG_PEEKSORT 1u

/* ps_options.flags: use one scratch copy of the data instead of two.  By
 * default the scratch holds two copies of keys (and payload), so that every
 * leaf longer than 4096 elements is merged from where it lies; with this flag
 * it holds one, and such a leaf is first copied to it when its depth in the
 * merge tree is odd.  Results are identical; only ps_workspace_bytes and
 * the data moved change. */
#define PS_FLAG_COMPACT_SCRATCH 2u

/* Options; a NULL pointer means all defaults.  struct_size must be
 * sizeof(ps_options). */
typedef struct {
    uint32_t struct_size;
    uint32_t min_run;          /* w of App. B.3/B.4; 0 = default 24 (the paper's
                                  setting); 1 = pure natural runs; at most 64 */
    uint32_t flags;            /* 0, or PS_FLAG_PEEKSORT and/or PS_FLAG_COMPACT_SCRATCH;
                                  other bits are rejected */
    uint32_t reserved;
    void *workspace;           /* optional caller-owned device scratch */
    uint64_t workspace_bytes;  /* its size; must be >= ps_workspace_bytes(...) */
} ps_options;

/* Bytes of device scratch one call needs for n_total elements in
 * num_segments segments (ps_sort: num_segments = 1).  has_payload is 0 or 1.
 * About 2 n_total (key bytes + 4 if has_payload) plus metadata, or half the
 * data part with PS_FLAG_COMPACT_SCRATCH in opt->flags.  A batch above
 * 2^31 - 1 elements runs in chunks of at most 2^31 - 1 (see
 * ps_segmented_sort), so its figure is that of 2^31 - 1 elements.  Returns 0
 * for invalid arguments. */
size_t ps_workspace_bytes(uint64_t n_total, uint64_t num_segments, ps_key_type key_type, int has_payload,
                          const ps_options *opt);

/* Sort keys[0..n) ascending and stably with powersort, in place; payload
 * (nullable, uint32 per key) is permuted alongside.  Sec. 2 (problem
 * statement and run convention), Alg. PowerSort, App. B.
 * d_merge_cost (nullable, 1 x uint64) receives the merge cost M of
 * Sec. 2.2: the sum of the result sizes of all r - 1 merges. */
ps_status ps_sort(void *keys, uint32_t *payload, uint64_t n, ps_key_type key_type, const ps_options *opt,
                  uint64_t *d_merge_cost, void *stream);

/* Sort each segment [d_offsets[g], d_offsets[g+1]) independently, as a whole
 * powersort with its own n and origin (the paper's nodePower takes the
 * subarray bounds, App. B.4), all segments in one batch of launches.
 * d_offsets: num_segments + 1 uint64 on the device, non-decreasing, with
 * d_offsets[0] = 0 and d_offsets[num_segments] = n_total; every segment
 * below 2^31 elements.  Empty segments are allowed.  d_merge_costs
 * (nullable): num_segments uint64, M per segment.  d_status (nullable,
 * 1 x int32): receives PS_OK, or PS_ERR_INVALID_ARG / PS_ERR_TOO_LARGE when
 * the offsets fail validation on the device; in that case the keys are left
 * in an unspecified order (no out-of-bounds access).
 * Batches of n_total >= 2^31 (up to 2^63 - 1): the library reads the offsets
 * back to the host once (this synchronises `stream`, so such a call cannot
 * be captured into a graph), validates them there (invalid offsets: the
 * error status is returned, nothing further is enqueued) and sorts the batch
 * as consecutive chunks of whole segments, each below 2^31 elements, one
 * after another on `stream` in one workspace.  Results are those of one
 * call. */
ps_status ps_segmented_sort(void *keys, uint32_t *payload, const uint64_t *d_offsets, uint64_t num_segments,
                            uint64_t n_total, ps_key_type key_type, const ps_options *opt,
                            uint64_t *d_merge_costs, int32_t *d_status, void *stream);

/* Merge cost M (Sec. 2.2) that ps_sort would incur on keys[0..n), computed
 * from the run partition, the node powers and the merge tree alone; keys
 * are not modified and no data moves.  d_merge_cost: 1 x uint64. */
ps_status ps_merge_cost(const void *keys, uint64_t n, ps_key_type key_type, const ps_options *opt,
                        uint64_t *d_merge_cost, void *stream);

/* Per-segment merge costs of ps_segmented_sort without sorting.
 * d_merge_costs: num_segments uint64.  d_status, and batches of 2^31 or
 * more elements, as in ps_segmented_sort. */
ps_status ps_segmented_merge_cost(const void *keys, const uint64_t *d_offsets, uint64_t num_segments,
                                  uint64_t n_total, ps_key_type key_type, const ps_options *opt,
                                  uint64_t *d_merge_costs, int32_t *d_status, void *stream);

/* Intermediate results of the method, for tests and tools (device arrays,
 * capacities in elements).  Leaves are the runs after min-run extension;
 * boundary j (1 <= j < r) separates leaves j-1 and j. */
typedef struct {
    uint32_t *starts;      /* n_total + 1: leaf starts, starts[r] = n_total */
    uint8_t *powers;       /* n_total + 1: powers[j] (Def. "Node Power"); 0 at
                              j = 0, j = r and between segments */
    uint32_t *node_left;   /* n_total: first leaf below node j */
    uint32_t *node_right;  /* n_total: one past the last leaf below node j */
    uint8_t *leaf_depth;   /* n_total: depth of leaf i in its segment's tree */
    uint32_t *r;           /* 1: number of leaves */
} ps_inspect_out;

/* Runs the non-moving part of the method (partition, powers, tree) on keys
 * and copies its intermediate arrays into `out` (each member nullable).
 * d_offsets may be NULL for one segment [0, n_total).  n_total < 2^31. */
ps_status ps_inspect(const void *keys, const uint64_t *d_offsets, uint64_t num_segments, uint64_t n_total,
                     ps_key_type key_type, const ps_options *opt, ps_inspect_out *out, void *stream);

/* Mehlhorn's Method 2' as a standalone nearly-optimal alphabetic tree
 * builder (App. A; Def. "Node Power"; Cor. "Cartesian tree"): for leaf
 * weights w[0..r) (device uint32, every w_i >= 1, sum W < 2^31) with leaf
 * probabilities w_i / W, computes the node powers, the tree they define (the
 * min-oriented Cartesian tree of the powers) and the leaf depths, and the
 * weighted path length sum_i depth_i * w_i, i.e. W times the search cost C
 * of Thm. "Nearly-Optimal BSTs" (iii), C <= H + 2.  This is powersort's tree
 * for runs of lengths w_i, without keys.  Outputs are device arrays, each
 * nullable: d_powers (r+1 bytes; node j between leaves j-1 and j has power
 * d_powers[j], d_powers[0] = d_powers[r] = 0), d_node_left / d_node_right
 * (r entries; node j merges leaves [d_node_left[j], j) and [j,
 * d_node_right[j]); entry 0 is unused), d_leaf_depth (r bytes), d_cost (one
 * uint64), d_status (one int32: PS_OK, PS_ERR_INVALID_ARG for a zero weight,
 * PS_ERR_TOO_LARGE for W >= 2^31; on error the outputs are those of unit
 * weights).  num_leaves in [1, 2^28], else an error is returned with nothing
 * enqueued.  Uses the per-stream scratch pool; asynchronous on stream. */
ps_status ps_alphabetic_tree(const uint32_t *d_weights, uint64_t num_leaves, uint8_t *d_powers,
                             uint32_t *d_node_left, uint32_t *d_node_right, uint8_t *d_leaf_depth, uint64_t *d_cost,
                             int32_t *d_status, void *stream);

/* ps_sort for callers that cannot allocate device memory (code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * allocation): the same sort, merge cost and arguments as ps_sort, with
 * scratch taken from a fixed array of 128 MiB that the library keeps on
 * every device it runs on (until the process ends) instead of the per-stream
 * pool.  It calls no hipMalloc, hipFree or other allocating routine; the
 * first call on a device looks up the array's address there.  The caller
 * still owns keys, payload and d_merge_cost.  opt->workspace must be NULL
 * (PS_ERR_INVALID_ARG otherwise).  A sort whose ps_workspace_bytes(n, 1,
 * key_type, payload != NULL, opt) exceeds 128 MiB returns PS_ERR_TOO_LARGE
 * with nothing enqueued; at the default minimum run that is above 6 404 640
 * 4-byte keys with a payload (10 359 840 without) or 4 645 728 8-byte keys
 * with a payload (6 414 287 without).  All calls on one device share that device's
 * array, and each call rewrites what it needs: calls that overlap on one
 * device (on different streams or from different threads) race and give
 * undefined results, so the caller serialises them, e.g. on one stream.
 * Profiling (ps_profile_enable) does not time these calls. */
ps_status ps_sort_no_alloc(void *keys, uint32_t *payload, uint64_t n, ps_key_type key_type, const ps_options *opt,
                           uint64_t *d_merge_cost, void *stream);

/* Launch shape of the data-movement kernels (process-wide).  Every value
 * changes only speed, never results: grids are workgroup counts of
 * grid-stride kernels; merge_tile is the outputs per merge-path tile, 2048,
 * 4096 or 8192 (8192 applies to 4-byte keys; 8-byte keys then use 4096);
 * merge_levels is the number of tree levels one merge pass does, 1 or 2:
 * with 2 (4-byte keys only) a node of more than 4096 elements at odd depth
 * in the merge tree is not written out but merged in the same pass as its
 * parent, which then merges up to four inputs.
 * Defaults: merge_tile 8192, merge_levels 1, grid_merge 2048, grid_split
 * 2048, grid_fused 2048, grid_big_leaf 2048.
 * Zero fields keep their current value.  Written by the project's
 * autotuner for a workload; read back with ps_get_tuning. */
typedef struct {
    uint32_t struct_size;
    uint32_t grid_big_leaf;
    uint32_t grid_fused;
    uint32_t grid_merge;
    uint32_t grid_split;
    uint32_t merge_tile;
    uint32_t merge_levels;
} ps_tuning;

/* Set (tuning != NULL) or reset to defaults (NULL) the launch shape.
 * Returns PS_ERR_INVALID_ARG for a bad struct_size, merge_tile or merge_levels, and
 * PS_ERR_UNSUPPORTED for a grid above 65536. */
ps_status ps_set_tuning(const ps_tuning *tuning);

/* Current launch shape. */
ps_status ps_get_tuning(ps_tuning *out);

/* Kernel groups timed by the profiling mode. */
enum {
    PS_PROF_PARTITION = 0, /* run detection and leaf partition */
    PS_PROF_TREE = 1,      /* powers, depths, merge cost */
    PS_PROF_LISTS = 2,     /* node ranges and work lists */
    PS_PROF_BIG_LEAF = 3,  /* copy / reversal of leaves longer than a fused subtree */
    PS_PROF_FUSED = 4,     /* leaf formation and merges of subtrees held in LDS */
    PS_PROF_MERGE = 5,     /* merge-path passes, one launch per node power */
    PS_PROF_SPLIT = 6,     /* co-ranks of the merge-path tiles, one launch per node power */
    PS_PROF_GROUPS = 7
};

/* Accumulated profile.  ms[g] is the summed duration of group g measured
 * with HIP events recorded on the caller's stream around its launches;
 * launches[g] counts those launches; elems[g] counts the elements the group
 * processed (for PS_PROF_MERGE: merge outputs, i.e. the part of the merge cost
 * M done by the merge-path passes; for PS_PROF_FUSED: elements of fused
 * subtrees; for PS_PROF_BIG_LEAF: elements copied or reversed; otherwise n). */
typedef struct {
    uint32_t struct_size;
    uint32_t calls;
    uint32_t launches[PS_PROF_GROUPS];
    double ms[PS_PROF_GROUPS];
    uint64_t elems[PS_PROF_GROUPS];
} ps_profile;

/* Turn the profiling mode off (0) or on for subsequent calls of this process,
 * for tools such as benchmarks: 1 times every group, any other value is a
 * mask of groups to time (bit g for group g; a mask holding only group 0 is
 * not expressible, as 1 means all).  Groups of one launch (big leaf, fused,
 * merge, split) are timed by the start and end events of the launch's own
 * dispatch, the others by events recorded around their launches, which
 * costs some microseconds per group.  Element counts are kept for every
 * group while profiling is on (a few device atomics).  Results are
 * unchanged. */
ps_status ps_profile_enable(int on);

/* Wait for the profiled work, add it to the running totals and copy them to
 * *out; reset != 0 clears the totals afterwards. */
ps_status ps_profile_read(ps_profile *out, int reset);

/* Cap the scratch the library's per-stream pool may hold for one stream
 * (bytes; 0 = no cap, the default).  A call whose scratch (as given by
 * ps_workspace_bytes) exceeds the cap returns PS_ERR_OUT_OF_MEMORY with
 * nothing enqueued, as it would if the allocation failed; calls with a
 * caller workspace or through ps_sort_no_alloc are not affected.  Existing
 * pool entries are kept until they must grow.  Process-wide. */
ps_status ps_set_pool_limit(uint64_t bytes);

/* Free the scratch memory the library holds for `stream` (synchronises it). */
ps_status ps_release(void *stream);

/* Static description of a status code. */
const char *ps_status_string(ps_status status);

/* Message of the last error on the calling thread ("" if none). */
const char *ps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* POWERSORT_HIP_H */
