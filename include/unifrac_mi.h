/*
 * unifrac_mi.h -- C ABI of the MI355X (gfx950) UniFrac distance library.
 *
 * The library computes the condensed matrix of pairwise UniFrac distances between
 * microbiome samples, given a phylogenetic tree that relates the features (Section 1 of
 * "Porting and optimizing UniFrac for GPUs", Sfiligoi, McDonald & Knight, 2020) and a
 * sample x feature count table.  The computation follows the Striped UniFrac structure the
 * paper ports to GPUs (Sections 2-3, Figs. 1-3): every branch of the tree contributes an
 * embedding (per-sample abundance below the branch), and every embedding is folded,
 * weighted by the branch length, into numerator and denominator accumulators laid out as
 * stripes (stripe s pairs sample k with sample (k+s+1) mod n).  The paper ships its code
 * as a C shared library linkable from any language (Abstract); this header is that
 * surface for this implementation.
 *
 * Conventions shared by every entry point
 *  - Status codes: every function returns uf_status (UF_OK = 0).  No C++ exception, abort
 *    or signal crosses the ABI.  A failing call leaves a message retrievable with
 *    uf_last_error().
 *  - Ownership: the caller owns every input array; they are read during the call only and
 *    never retained, except that uf_plan_create copies what it needs into the plan.
 *    Output buffers are caller-owned too.  Contexts, plans and batches are library-owned
 *    opaque objects released with their destroy function; plans and batches must be
 *    destroyed before the context they were made on.
 *  - Pointers: tree and table arrays are HOST pointers.  Output pointers are host or device
 *    pointers as the `out_on_device` flag says (device = memory of the context's GPU).
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *    device work is enqueued on it; the call returns after the output is complete.
 *  - Condensed order: pair (i, j), i < j, sits at index n*i - i*(i+1)/2 + (j - i - 1)
 *    (row i ascending, then j ascending), n = number of samples = CSR rows.
 *  - Threading: a context and its plans must not be used by two host threads at once.
 */
#ifndef UNIFRAC_MI_H
#define UNIFRAC_MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    UF_OK = 0,
    UF_E_ARG = 1,          /* null pointer, bad enum, size out of range                     */
    UF_E_TREE = 2,         /* parent array: not exactly one root, cycle, index out of range,
                              or a branch length that is negative / not finite              */
    UF_E_TABLE = 3,        /* CSR: bad indptr, feature id out of range, negative count,
                              feature mapped to a non-leaf node, per-sample total > INT32_MAX */
    UF_E_EMPTY_SAMPLE = 4, /* a sample whose total count is zero                             */
    UF_E_DEVICE = 5,       /* HIP runtime error                                              */
    UF_E_OOM = 6,          /* device allocation failed                                       */
    UF_E_UNSUPPORTED = 7,  /* method/precision combination not provided                      */
    UF_E_INTERNAL = 8
} uf_status;

/* UniFrac variant.  Unweighted: per pair, branch length seen in exactly one sample over
 * branch length seen in either.  Weighted normalized: per pair, sum over branches of
 * L * |p - q| over sum of L * (p + q), with p, q the fractions of each sample's reads below
 * the branch.  Weighted unnormalized: the numerator sum of L * |p - q| alone (the variant
 * of the Striped UniFrac work the paper builds on, reference [3]).  The root has no
 * branch. */
typedef enum {
    UF_UNWEIGHTED = 0,
    UF_WEIGHTED_NORMALIZED = 1,
    UF_WEIGHTED_UNNORMALIZED = 2
} uf_method;

/* Arithmetic of the hot path (the fp64 / fp32 code paths of Section 4, plus a matrix-core
 * form of the unweighted variant):
 *  UF_PREC_FP64       embeddings, products and accumulation in FP64 (striped kernel).
 *  UF_PREC_FP32       FP32 embeddings and products, FP32 sums within an embedding batch,
 *                     FP64 accumulation across batches, FP64 final division.
 *  UF_PREC_MFMA_BF16X2 unweighted only: shared branch length as P diag(L) P^T over 0/1
 *                     presence P on bf16 matrix cores, with every length split into two
 *                     bf16 terms (hi + lo), FP32 accumulation inside chunks of branches and
 *                     FP64 across chunks; FP64 final division. */
typedef enum { UF_PREC_FP64 = 0, UF_PREC_FP32 = 1, UF_PREC_MFMA_BF16X2 = 2 } uf_precision;

typedef enum { UF_F64 = 0, UF_F32 = 1 } uf_dtype;

/* Tree as a parent array.  parent[v] in [0, n_nodes) or -1 for the single root; every
 * node must reach the root.  length[v] >= 0 and finite is the length of the branch above v;
 * length[root] is ignored. */
typedef struct {
    int32_t n_nodes;
    const int32_t *parent;
    const double *length;
} uf_tree;

/* Sample x feature counts in CSR form, one row per sample (row order = sample order).
 * indptr[0] == 0, indptr non-decreasing, indptr[n_samples] = nnz.  indices[e] in
 * [0, n_features); duplicates within a row are summed.  counts[e] >= 0.  feature_node[f]
 * is the tree node of feature f and must be a leaf; NULL means feature f is node f.
 * Every sample needs a positive total, and a sample's total must fit in int32. */
typedef struct {
    int32_t n_samples;
    int32_t n_features;
    const int64_t *indptr;
    const int32_t *indices;
    const int32_t *counts;
    const int32_t *feature_node;
} uf_table;

/* Optional knobs; a NULL pointer or a zero field means "library default / tuned value". */
typedef struct {
    int32_t emb_batch;  /* branches per embedding batch streamed through the striped kernel
                           (the batch depth of Section 3, Fig. 2)                            */
    int32_t k_chunk;    /* matrix-core path: branches per FP32 accumulation chain (rounded
                           to an even number of 128-branch stages; default 4096).  Variant 1
                           adds every chain's sum into FP64.  Variant 0 adds four consecutive
                           chain sums together in FP32 (three roundings) before one FP64 add,
                           so each FP64 add takes 4 * k_chunk branches, while the FP32 error
                           stays that of one k_chunk chain plus three roundings              */
    int32_t den_mode;   /* striped path: 0 = numerator and denominator stripes (default);
                           1 = numerator stripes only, denominator from per-sample sums
                           (weighted normalized: sum_b L_b p_ib + sum_b L_b p_jb)            */
    int32_t variant;    /* striped path: 0 = fused kernel that transforms count rows while
                           staging them and loops over every batch in one launch (default);
                           1 = separate transform launch into an embedding buffer and one
                           striped launch per batch (single plans only; batches ignore it).
                           matrix-core path: 0 = four consecutive chunk sums are added
                           together in FP32, then into the FP64 output (two work-groups per
                           CU, default); 1 = every chunk sum goes into FP64 registers, written
                           once at the end (one work-group per CU)                           */
    int32_t tile;       /* striped fused/queued kernels: per-lane tile shape (samples x
                           stripes), 0, 1 or 2; den_mode 0: FP64 4x8 | 2x12 | 2x8,
                           FP32 4x16 | 8x8 | 4x8; den_mode 1: FP64 4x16 | 2x24 | 4x8,
                           FP32 4x24 | 8x16 | 4x16; shape 2 runs three work-groups per CU
                           (four for FP32 4x16; the others two).  A NULL tuning selects
                           shape 2 (fastest measured for den_mode 0); a zero field here
                           means shape 0                                                     */
    int32_t count_width; /* striped path: bytes per embedding count; 0 = 2 when every sample
                           total fits in 16 bits (halves count memory and traffic), else 4;
                           4 = int32; 2 = uint16 (UF_E_ARG if a total exceeds 65535)         */
    int32_t k_split;    /* fused and queued striped kernels: the branches are split into
                           this many contiguous ranges, each accumulated by its own grid
                           slice into its own copy of the stripe state, and the copies are
                           summed in order afterwards (more work-groups when the stripe
                           tiles alone do not fill the device many times over); 0 =
                           automatic (about twenty device rounds from the whole problem's
                           stripe tiles, also for stripe ranges; at most 32 splits, 64 when
                           16 would not fill the device once; at least two batches per
                           split, an FP64 batch depth left at its default shrinking to as
                           few as 64 branches to allow that; the state copies within 4 GB;
                           in a batch only while all its jobs' stripe tiles come to fewer
                           than ten device rounds and the extra state copies of all its
                           automatically split jobs stay within 16 GB, so a job splits as
                           it would alone), 1 = no split                                     */
} uf_tuning;

typedef struct {
    int32_t n_samples;
    int32_t n_nodes;
    int32_t n_branches;  /* n_nodes - 1 */
    int32_t n_leaves;
    int32_t n_levels;    /* height of the tree + 1: kernel launches of the propagation    */
    int32_t n_stripes;   /* floor(n_samples / 2)                                          */
    int64_t n_pairs;     /* n_samples * (n_samples - 1) / 2                               */
    int64_t nnz;
} uf_plan_info;

typedef struct uf_context uf_context;
typedef struct uf_plan uf_plan;

/* Human-readable name of a status code (static string, never NULL). */
const char *uf_status_string(uf_status s);

/* Message of the last failure: of `ctx` when non-NULL, else of the calling thread's last
 * context-free call (uf_validate).  Valid until the next call on the same object/thread. */
const char *uf_last_error(const uf_context *ctx);

/* Validate a tree and a table on the host; touches no device.  Returns UF_OK or the first
 * error found (UF_E_TREE, UF_E_TABLE, UF_E_EMPTY_SAMPLE, UF_E_ARG). */
uf_status uf_validate(const uf_tree *tree, const uf_table *table);

/* Create a context on HIP device `device`.  On success *out owns the device selection and
 * a message buffer; release with uf_context_destroy. */
uf_status uf_context_create(int32_t device, uf_context **out);
void uf_context_destroy(uf_context *ctx);

/* Validate and preprocess (tree levels, child lists, leaf slots of every CSR entry,
 * per-sample totals), then upload the inputs to the device on `stream`.  After it returns
 * the plan's inputs are resident in device memory and the host arrays may be freed. */
uf_status uf_plan_create(uf_context *ctx, const uf_tree *tree, const uf_table *table,
                         void *stream, uf_plan **out);
void uf_plan_destroy(uf_plan *plan);
uf_status uf_plan_query(const uf_plan *plan, uf_plan_info *info);

/* Embedding propagation only (the per-branch input buffers of Section 3): out[v][k] =
 * reads of sample k on tips at or below node v, for every node v (root row = totals),
 * as int32 in node-id order, [n_nodes][n_samples] row-major. */
uf_status uf_plan_embedding_counts(uf_plan *plan, int32_t *out, int32_t out_on_device,
                                   void *stream);

/* The same through the 16-bit count rows (every sample total must be <= 65535, else
 * UF_E_ARG); the output is int32 like uf_plan_embedding_counts. */
uf_status uf_plan_embedding_counts16(uf_plan *plan, int32_t *out, int32_t out_on_device,
                                     void *stream);

/* Presence bits of the same embedding: bit (k % 32) of out[v][k / 32] is set iff sample k
 * has a read at or below node v; [n_nodes][ceil(n_samples / 32)] uint32, node-id order. */
uf_status uf_plan_embedding_presence(uf_plan *plan, uint32_t *out, int32_t out_on_device,
                                     void *stream);

/* The full hot path on resident inputs: embedding propagation, transform, striped (or
 * matrix-core) accumulation, normalize/condense.  `out` receives n*(n-1)/2 values of
 * `out_dtype` in condensed order.  UF_PREC_MFMA_BF16X2 with a weighted method returns
 * UF_E_UNSUPPORTED.  Device scratch is allocated on first use and kept by the plan. */
uf_status uf_plan_distance(uf_plan *plan, uf_method method, uf_precision prec,
                           const uf_tuning *tuning, uf_dtype out_dtype, void *out,
                           int32_t out_on_device, void *stream);

/* Stripe-range subproblem: the independent chunks the paper distributes over many chips
 * (Section 1; Table 2 runs 128 and 4 chunks).  Computes only stripes [s_begin, s_end)
 * (0 <= s_begin <= s_end <= n/2) and writes the distances of the pairs those stripes hold
 * into `out`, a FULL condensed array of n*(n-1)/2 elements; all other entries are left
 * as they were.  A host output receives only the range's pairs: they are laid out
 * compactly in condensed order on the device, copied back once, and each condensed row's
 * (at most two) runs copied into place.  Ranges that partition [0, n/2) fill the whole
 * matrix with exactly the values of uf_plan_distance (same per-element arithmetic).
 * Striped precisions only; tuning->variant is ignored. */
uf_status uf_plan_distance_stripes(uf_plan *plan, uf_method method, uf_precision prec,
                                   const uf_tuning *tuning, int32_t s_begin, int32_t s_end,
                                   uf_dtype out_dtype, void *out, int32_t out_on_device,
                                   void *stream);

/* The same stripe range as a compact block, the partial result one chunk job keeps or
 * ships (Section 1, Table 2): out is [s_end - s_begin][n] values of out_dtype, row r,
 * column k = distance of the pair (k, (k + s_begin + r + 1) mod n); for even n the last
 * stripe's columns k >= n/2 repeat its first half.  Host or device output.  Blocks from
 * independent plans, contexts or processes assemble into the full matrix with
 * uf_merge_block. */
uf_status uf_plan_distance_block(uf_plan *plan, uf_method method, uf_precision prec,
                                 const uf_tuning *tuning, int32_t s_begin, int32_t s_end,
                                 uf_dtype out_dtype, void *out, int32_t out_on_device, void *stream);

/* Merge of a block of uf_plan_distance_block (stripes [s_begin, s_end) of an n-sample
 * problem, [s_end - s_begin][n] values of dtype, host or device) into `condensed`, a DEVICE
 * array of n*(n-1)/2 values of dtype: the block's pairs are written, every other entry is
 * left as it was.  Blocks of ranges that partition [0, n/2) reproduce uf_plan_distance bit
 * for bit.  A host block is staged through a device buffer allocated for the call.
 * Blocks until done. */
uf_status uf_merge_block(uf_context *ctx, int32_t n, int32_t s_begin, int32_t s_end, uf_dtype dtype,
                         const void *block, int32_t block_on_device, void *condensed, void *stream);

/* Raw stripe accumulators of the striped path (for inspection): num and den, each
 * [n_stripes][n_samples] FP64 row-major on the host, where row s, column k holds the sums
 * for the pair (k, (k + s + 1) mod n).  Only UF_PREC_FP64 / UF_PREC_FP32. */
uf_status uf_plan_stripes(uf_plan *plan, uf_method method, uf_precision prec,
                          const uf_tuning *tuning, double *num, double *den, void *stream);

/* Release the plan's cached device scratch (embeddings, stripes); inputs stay resident. */
uf_status uf_plan_trim(uf_plan *plan);

/* Device memory the plan may hold, in bytes, inputs included (0 = no limit but the
 * device's).  When all embedding count rows (striped precisions) or presence bits
 * (matrix-core precision) would not fit beside the inputs and the accumulators, the plan
 * generates them batch by batch instead: each batch of branch rows is computed from the
 * table on a second stream (the tips below a node form one range of a depth-first order,
 * so a row is a difference of two prefix sums over the sample's entries) while the previous
 * batch is accumulated, in two alternating buffers.  The same happens, without a limit,
 * when allocating the full rows fails.  Generated rows equal the propagated ones exactly;
 * striped results then run without branch splits (as with k_split = 1), and the
 * matrix-core path takes its branches in chunks of a multiple of 4 * k_chunk.  Returns
 * UF_E_ARG for a negative limit; a limit too small even for generated batches makes the
 * distance calls fail with UF_E_OOM. */
uf_status uf_plan_set_memory_limit(uf_plan *plan, int64_t max_device_bytes);

/* Per-kernel timing with HIP events recorded on the launch stream around every device
 * launch of the plan, grouped by kernel class ("propagate", "transform", "stripe", "reduce"
 * (the sum of the branch splits' state copies), "rowdot", "condense", "bits_transpose",
 * "mfma", "normalize").  enable != 0 turns it on
 * and clears the totals; enable == 0 turns it off.  Costs one event pair per launch. */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
} uf_kernel_stat;
uf_status uf_plan_set_profiling(uf_plan *plan, int32_t enable);
/* Copies up to `cap` classes with at least one launch into `out`; *n_out = classes copied. */
uf_status uf_plan_get_profile(uf_plan *plan, uf_kernel_stat *out, int32_t cap, int32_t *n_out);

/* Autotuner for the grouping parameters (Section 3: tile and batch sizes decide the run
 * time), on one plan.  Times candidate settings of `prec` on this plan's resident inputs
 * with HIP events (one warm-up, then `reps` calls each; reps <= 0 means 3): striped paths
 * try the three tile shapes with embedding-batch depths 128, 64 and 32 (FP32; deeper FP32
 * batches would loosen the worst-case bound of the in-batch FP32 sums, (E - 1) * 2^-24 of
 * the distance, past 1e-5) or 1024, 256 and 4096 (FP64); the matrix-core path tries variants
 * 0 and 1 with k_chunk 4096 and 16384.  den_mode is taken from `base` (NULL = 0).  A
 * candidate whose output differs from the first candidate's by more than the path's
 * tolerance (FP64 1e-12, else 1e-5) is rejected.  The winner goes to *best (and its
 * milliseconds per call to *best_ms if non-NULL).  With a non-NULL cache_path the winner is
 * appended to that text file under a key of device architecture, method, precision,
 * den_mode and log2 size buckets, and a later call with the same key returns the cached
 * entry without timing.  Uses the default stream. */
uf_status uf_plan_autotune(uf_plan *plan, uf_method method, uf_precision prec,
                           const uf_tuning *base, int32_t reps, const char *cache_path,
                           uf_tuning *best, double *best_ms);

/* Mantel test between two condensed matrices (the paper's fp32-vs-fp64 check, Section 4:
 * Mantel R^2 0.99999).  x, y: DEVICE arrays of n*(n-1)/2 FP64 values in condensed order
 * (n >= 3).  *r_out = Pearson correlation over all pairs.  perms: DEVICE array of n_perm
 * rows of n int32, each a permutation of 0..n-1 supplied by the caller (a row that is not
 * a permutation gives UF_E_ARG); for each row the labels of y are permuted and the
 * correlation recomputed; *p_out = (1 + #{|r_perm| >= |r|}) / (1 + n_perm) (two-sided;
 * 1 when n_perm = 0).  r_perm_out (host, n_perm values) may be NULL.  Arithmetic in FP64
 * with deterministic reductions.  Blocks until done; allocates its own scratch. */
uf_status uf_mantel(uf_context *ctx, const double *x, const double *y, int32_t n,
                    const int32_t *perms, int32_t n_perm, double *r_out, double *r_perm_out,
                    double *p_out, void *stream);

/* ---- Batches of independent jobs ------------------------------------------------------
 * Many UniFrac problems of uneven size computed together (the batching of Section 3 taken
 * one level up: many jobs per launch instead of many branches per launch).  Every job is
 * validated and made resident at creation; a run is a fixed sequence of launches shared by
 * all jobs (one gather per tree level for every job together, one persistent
 * queue-driven striped launch per precision and one for the matrix-core jobs, largest job
 * first), which uf_batch_capture records once into a HIP graph for replay. */
typedef struct {
    uf_tree tree;
    uf_table table;
    uf_method method;
    uf_precision prec;      /* FP64 / FP32 striped, or MFMA_BF16X2 (unweighted only)     */
    uf_dtype out_dtype;
    void *out;              /* n*(n-1)/2 elements of out_dtype.  A DEVICE pointer must stay
                               valid for the life of the batch (graphs replay it); a HOST
                               pointer is written by uf_batch_run after the device work,
                               through a device staging buffer the batch owns             */
    int32_t out_on_device;  /* 1: `out` is device memory of the context's GPU; 0: host     */
} uf_job;
typedef struct uf_batch uf_batch;
/* tuning: when non-NULL its knobs (emb_batch, den_mode, tile, count_width, k_chunk,
 * variant, k_split) apply to every job; when NULL every job takes the knobs uf_autotune
 * stored in the context for a problem of its kind and size, or the library defaults.  A
 * striped job's branch splits are queue items of their own, each into its own copy of the
 * job's stripe state, summed in split order before the condense. */
uf_status uf_batch_create(uf_context *ctx, const uf_job *jobs, int32_t n_jobs,
                          const uf_tuning *tuning, void *stream, uf_batch **out);
/* Runs every job (replaying the captured graph if there is one) and waits for it. */
uf_status uf_batch_run(uf_batch *batch, void *stream);
/* Records the batch's device work into a HIP graph (on a private stream); later runs
 * launch the graph.  Nothing is allocated while capturing or replaying. */
uf_status uf_batch_capture(uf_batch *batch);
uf_status uf_batch_set_profiling(uf_batch *batch, int32_t enable);
uf_status uf_batch_get_profile(uf_batch *batch, uf_kernel_stat *out, int32_t cap, int32_t *n_out);
void uf_batch_destroy(uf_batch *batch);
/* One-shot: create, run on `stream`, wait for the stream, destroy.  Blocks until every
 * output is valid; the same errors as uf_batch_create and uf_batch_run. */
uf_status uf_distance_batch(uf_context *ctx, const uf_job *jobs, int32_t n_jobs, void *stream);

/* One-shot convenience: plan_create + plan_distance + plan_destroy. */
uf_status uf_distance(uf_context *ctx, const uf_tree *tree, const uf_table *table,
                      uf_method method, uf_precision prec, uf_dtype out_dtype, void *out,
                      int32_t out_on_device, void *stream);

/* Embedding counts of every branch, for inspection (the per-branch input buffers of
 * Section 3): out_counts[b][k] = reads of sample k on the tips at or below the b-th non-root
 * node, nodes taken in ascending id order with the root skipped; [n_nodes - 1][n_samples]
 * int32 row-major in HOST memory, owned by the caller.  Validates the inputs first (the
 * status codes of uf_validate); computes on the context's GPU with the level-synchronous
 * propagation of the distance path, on the default stream; blocks until done. */
uf_status uf_debug_embedding_counts(uf_context *ctx, const uf_tree *tree, const uf_table *table,
                                    int32_t *out_counts);

/* Autotuner over representative jobs (Section 3: the grouping parameters "drastically"
 * change the run time, so they are tuned per kind of problem).  For each of the n jobs the
 * knobs of its (method, precision) are timed on its inputs (a temporary plan; tree, table,
 * method and prec are read, out is ignored): striped precisions try tile shapes 0-2 x
 * embedding-batch depths (FP32 32, 64, 128; FP64 256, 1024, 4096) x den_mode 0 and 1 (one
 * warm-up and two timed calls each); the matrix-core precision tries variants 0-1 x k_chunk
 * 4096 and 16384.  Candidates whose output differs from the first candidate's by more than
 * the path's tolerance (FP64 1e-12, else 1e-5) are rejected.  The winner is stored in the
 * context under (method, precision, log2 of the sample count, log2 of the node count); from
 * then on uf_plan_distance, uf_plan_distance_stripes and uf_distance with a NULL tuning, and
 * uf_batch_create with a NULL tuning, use the stored knobs for a problem in the same
 * bucket.  A later tuning of the same bucket replaces the entry.  Blocks until done. */
uf_status uf_autotune(uf_context *ctx, const uf_job *representative, int32_t n);

/* The knobs uf_autotune stored for a problem of this kind and size: *found = 1 and *out =
 * the knobs, or *found = 0 when the context has none (library defaults apply). */
uf_status uf_autotune_lookup(const uf_context *ctx, uf_method method, uf_precision prec,
                             int32_t n_samples, int32_t n_nodes, uf_tuning *out, int32_t *found);

/* ---- Without device allocation ------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The library holds one fixed scratch
 * array of UF_NOALLOC_SCRATCH_BYTES on every GPU it runs on (until the process ends); its
 * address is resolved per device when a context is created there. */
#define UF_NOALLOC_SCRATCH_BYTES (128u << 20)

/* uf_plan_distance for the striped precisions (UF_PREC_FP64, UF_PREC_FP32) with every
 * scratch buffer (count rows, reciprocal totals, per-sample sums, stripe state) taken from
 * that array: no hipMalloc, hipFree, memset node or other allocating call.  `out` is a
 * DEVICE pointer of n*(n-1)/2 elements of out_dtype.  The knobs are uf_plan_distance's
 * (fused kernel only; tuning->variant is ignored); the automatic branch split is lowered
 * until the state copies fit.  Returns UF_E_ARG when the problem needs more scratch than the
 * array holds (the message gives the size), UF_E_UNSUPPORTED for UF_PREC_MFMA_BF16X2.
 * Asynchronous: the work is enqueued on `stream` and `out` is complete when the stream's
 * work is.  Every call on one GPU shares its array and leaves its contents behind (each
 * call clears what must start at zero), so calls that overlap on one GPU, from several
 * streams or threads, race: serialize them. */
uf_status uf_plan_distance_noalloc(uf_plan *plan, uf_method method, uf_precision prec,
                                   const uf_tuning *tuning, uf_dtype out_dtype, void *out,
                                   void *stream);

#ifdef __cplusplus
}
#endif

#endif /* UNIFRAC_MI_H */
