// Internal declarations shared by the host runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "unifrac_mi.h"

namespace ufmi {

// ------------------------------------------------------------------ host preprocessing

// Node slots: nodes are renumbered by height (0 = leaf, else 1 + max child height), ties
// by node id.  Leaves occupy slots [0, n_leaf); height level h occupies slots
// [level_ptr[h], level_ptr[h+1]); the root is the last slot (it alone has the maximum
// height).  Branch slots are [0, n_nodes - 1).
struct HostPrep {
    int32_t n_nodes = 0, n_samples = 0, n_features = 0;
    int32_t root = -1, n_leaf = 0, n_levels = 0;
    int64_t nnz = 0;
    std::vector<int32_t> slot_of_node, node_of_slot;
    std::vector<int32_t> level_ptr;          // n_levels + 1
    std::vector<int32_t> child_ptr;          // per internal slot (slot - n_leaf), + 1
    std::vector<int32_t> child_slot;
    std::vector<double> length_slot;         // branch length per slot; 0 at the root slot
    std::vector<int64_t> indptr;             // n_samples + 1
    std::vector<int32_t> entry_slot;         // leaf slot of every CSR entry
    std::vector<int32_t> entry_count;
    std::vector<int32_t> totals;             // per-sample total reads (> 0, fits int32)
};

uf_status validate_and_prepare(const uf_tree *tree, const uf_table *table, HostPrep *hp,
                               std::string *err);

// Tip ranges of a depth-first order and per-sample sorted entries, for generating count
// rows batch by batch: the tips below slot s are positions [lo[s], hi[s]); the entries of
// sample k (CSR range of the table) sorted by tip position are spos, with running count
// sums scum (each sample starting from zero).
struct RangeTables {
    std::vector<int32_t> lo, hi;     // per slot
    std::vector<int32_t> spos, scum; // per CSR entry, sorted within each sample
};
void range_tables(const HostPrep &hp, RangeTables *rt);

// ------------------------------------------------------------------ device launches

// All launches are asynchronous on `st` and return the launch status.
hipError_t launch_fill_u32(void *p, uint32_t value, size_t n_words, hipStream_t st);
// *out = max_i |a[i] - b[i]| (NaN counts as infinity).
hipError_t launch_max_abs_diff(const double *a, const double *b, int64_t n, double *out, hipStream_t st);

// Embedding propagation (count form): C is [n_nodes][cstride] int32 in slot order.
// C: [n_nodes][cstride] counts of cw bytes (4 = int32, 2 = uint16 packed two per word;
// uint16 needs every sample total <= 65535, so packed halves never carry into each other).
hipError_t launch_scatter_counts(const int64_t *indptr, const int32_t *entry_slot,
                                 const int32_t *entry_count, void *C, int32_t cw, int64_t cstride,
                                 int32_t n_samples, hipStream_t st);
// stride_words: uint32 words per row (the gather adds whole words, i.e. both packed halves)
hipError_t launch_level_sum(void *C, int64_t stride_words, int32_t slot_begin, int32_t n_rows,
                            int32_t n_leaf, const int32_t *child_ptr, const int32_t *child_slot,
                            hipStream_t st);
// The narrow top of the tree (levels from HostPrep-derived tail_level up, each with few
// nodes) as one launch.  Its topology, level by level: node records (slot, first kid, end
// kid, 0) indexing the child slots `kid`, record boundaries per tail level `lvl`, and chunks of
// whole levels whose records and kids fit the kernel's LDS staging.
constexpr int kTailMaxLevels = 1024, kTailMaxNodes = 1024, kTailMaxKids = 2048;
struct TailProgram {
    const int32_t *lvl;      // tail levels + 1 record boundaries
    const int4 *rec;
    const int32_t *kid;
    const int2 *chunks;      // [first level, end level) of each chunk, tail-relative
    int32_t n_chunks, pad;
};
struct TailProgramHost {
    std::vector<int32_t> lvl, kid;
    std::vector<int32_t> rec;      // 4 ints per node
    std::vector<int32_t> chunks;   // 2 ints per chunk
};
// Builds the program of levels [h0, n_levels); false when a level alone exceeds the limits.
bool tail_program(const HostPrep &hp, int32_t h0, TailProgramHost *tp);
hipError_t launch_level_tail(bool is_or, uint32_t *X, int64_t stride_words, const TailProgram &tp,
                             hipStream_t st);
// First level of the narrow top of the tree: every level from it on holds at most
// `max_nodes` nodes (n_levels when the top level itself is wider).
int32_t narrow_tail_level(const HostPrep &hp, int32_t max_nodes);
// out[v][0..width) = (int32) src16[slot_of_node[v]][0..width)
hipError_t launch_gather_rows_u16(const uint16_t *src, int64_t sstride, const int32_t *slot_of_node,
                                  int32_t n_nodes, int32_t width, int32_t *out, hipStream_t st);
// Presence form: B is [n_nodes][bstride] uint32, bit k%32 of word k/32.
hipError_t launch_scatter_bits(const int64_t *indptr, const int32_t *entry_slot,
                               const int32_t *entry_count, uint32_t *B, int64_t bstride,
                               int32_t n_samples, hipStream_t st);
hipError_t launch_level_or(uint32_t *B, int64_t bstride, int32_t slot_begin, int32_t n_rows,
                           int32_t n_leaf, const int32_t *child_ptr, const int32_t *child_slot,
                           hipStream_t st);
// Batched propagation over many jobs: mode 0 = int32 counts, 1 = presence bits,
// 2 = uint16 counts packed two per word.
struct PropJob {
    uint32_t *X;              // counts or presence words, slot-major rows
    int64_t stride;           // uint32 words per row (multiple of 4)
    const int32_t *child_ptr, *child_slot;
    const int64_t *indptr;
    const int32_t *entry_slot, *entry_count;
    int32_t n_leaf, mode, n_samples, pad;
};
// tasks_xy: (job, sample) pairs for the scatter; (job, slot) pairs of one level for the gather.
hipError_t launch_scatter_batched(const PropJob *jobs, const int32_t *tasks_xy, int32_t n_tasks,
                                  hipStream_t st);
hipError_t launch_level_batched(const PropJob *jobs, const int32_t *tasks_xy, int32_t n_tasks,
                                int32_t max_vec, hipStream_t st);
// out[v][0..width) = src[slot_of_node[v]][0..width), for node-ordered output.
hipError_t launch_gather_rows_u32(const uint32_t *src, int64_t sstride, const int32_t *slot_of_node,
                                  int32_t n_nodes, int32_t width, uint32_t *out, hipStream_t st);

// Striped path.  Embedding rows: emb[e][x], x in [0, estride); x < n + S holds the sample
// x mod n (the wrap copy lets k + s + 1 run past n without a modulo); the rest is zero.
struct StripeGeom {
    int32_t n, S;            // samples, stripes
    int32_t tkw, tsw;        // work-group tile: samples x stripes
    int64_t sstride;         // row stride of num/den (multiple of tkw)
    int32_t spad;            // stripes rounded up to tsw
    int64_t estride;         // embedding row stride
    int32_t occ;             // work-groups per CU the striped kernels are compiled for
};
StripeGeom stripe_geometry(int32_t n, bool fp64, int32_t den_mode, int32_t tile = 0);

// Count rows are int32 (cw = 4) or uint16 (cw = 2, when every sample total fits in 16 bits).
hipError_t launch_transform(bool fp64, int32_t method, const void *C, int32_t cw, int64_t cstride,
                            int32_t slot0, int32_t E, const int32_t *totals, int32_t n, int32_t S,
                            void *emb, int64_t estride, hipStream_t st);
hipError_t launch_stripe(bool fp64, int32_t method, int32_t den_mode, const void *emb,
                         int64_t estride, const double *len, int32_t E, double *num, double *den,
                         const StripeGeom &g, bool first, hipStream_t st);
// Fused transform + striped accumulation over all B branches in one launch (batches of E
// accumulate in registers; the stripe state, cleared beforehand, is the cross-batch
// accumulator).  StripeArgs describes one job for the fused and queued kernels.
struct StripeArgs {
    const void *C;           // counts [n_nodes][cstride], branch slots first
    int32_t cw, pad;         // bytes per count: 4 (int32) or 2 (uint16)
    int64_t cstride;
    const double *inv_t;     // 1 / total per sample
    const double *len;       // branch length per slot
    int32_t B, E, n, S;      // branches, batch depth, samples, stripes
    double *num, *den;       // stripe state [spad][sstride]
    int64_t sstride;
    int32_t method, tiles_k, tiles_s, s_base;   // s_base: stripe held by state row 0
    int32_t kz;              // branch splits (grid z), each with its own state copy
    int32_t store_first;     // 1: the first batch of each split writes its state copy
                             // instead of adding into it, so the copies need no clearing
    int64_t zstride;         // elements between state copies
};
StripeArgs make_stripe_args(int32_t method, const void *C, int32_t cw, int64_t cstride,
                            const double *inv_t, const double *len, int32_t B, int32_t E,
                            double *num, double *den, const StripeGeom &g);
// items_xy: (job index, item) pairs, item = z * tiles_k * tiles_s + s_tile * tiles_k + k_tile
// for branch split z of the job's kz (state copy z at num + z * zstride); *counter == 0.
hipError_t launch_stripe_queue(bool fp64, int32_t method, int32_t cw, int32_t den_mode, int32_t tile,
                               const StripeArgs *jobs, const int32_t *items_xy, int32_t n_items,
                               int32_t *counter, int32_t n_groups, hipStream_t st);
hipError_t launch_inv_totals(const int32_t *totals, int32_t n, double *inv_t, hipStream_t st);
// Covers stripe tiles [tile_s0, tile_s1); state row 0 holds stripe tile_s0 * tsw.
hipError_t launch_stripe_fused(bool fp64, int32_t method, int32_t den_mode, int32_t tile,
                               const void *C, int32_t cw, int64_t cstride, const double *inv_t,
                               const double *len, int32_t B, int32_t E, double *num, double *den,
                               const StripeGeom &g, int32_t tile_s0, int32_t tile_s1,
                               int32_t kz, int64_t zstride, bool store_first, hipStream_t st);
// x[i] = sum over z of x[z * zstride + i] (z in order), for i < count.
hipError_t launch_reduce_z(double *x, int64_t zstride, int32_t kz, int64_t count, hipStream_t st);
// Writes the pairs of stripes [s_begin, s_end) (the state block's row 0 holds stripe
// s_base) in one of three layouts: 0 = into a full condensed output; 1 = a dense
// [s_end - s_begin][n] block; 2 = the range's pairs only, in condensed order, row i's
// pairs from row_off[i] (range_row_offsets).
hipError_t launch_condense_range(int32_t method, const double *num, const double *den, const double *D,
                                 int64_t sstride, int32_t n, int32_t S, int32_t s_base,
                                 int32_t s_begin, int32_t s_end, int32_t out_f32, void *out,
                                 hipStream_t st, int32_t layout = 0, const int64_t *row_off = nullptr);
// Scatter of a dense block (layout 1) into the condensed matrix.
hipError_t launch_merge_block(const void *block, int32_t n, int32_t s_begin, int32_t s_end, int32_t f32,
                              void *condensed, hipStream_t st);
// Pairs of stripes [s_begin, s_end) in condensed row i: a run at distances j - i in
// [s_begin + 1, min(s_end, S)] and a run at distances in [max(n - s_end, S + 1), n - 1 - s_begin],
// both clipped to j < n.  Fills len_a, len_b (n each) and off (n + 1, prefix sums).
void range_row_runs(int32_t n, int32_t s_begin, int32_t s_end, std::vector<int32_t> *len_a,
                    std::vector<int32_t> *len_b, std::vector<int64_t> *off);
// Per-sample sums D_k = sum_b L_b u_kb over a batch of E branches (separable denominator);
// `part` holds rowdot_scratch_elems(n, E) doubles of scratch.
size_t rowdot_scratch_elems(int32_t n, int32_t E);
hipError_t launch_rowdot(int32_t method, const void *C, int32_t cw, int64_t cstride, int32_t slot0,
                         int32_t E, const int32_t *totals, const double *len, int32_t n,
                         double *D, bool first, double *part, hipStream_t st);
hipError_t launch_condense(int32_t method, const double *num, const double *den, const double *D,
                           int64_t sstride, int32_t n, int32_t S, int32_t out_f32, void *out,
                           hipStream_t st);

// Count rows generated from the range tables (no propagation): out[e][k] = reads of sample
// k below slot slot0 + e, for e < E, k < n, as cw-byte counts in rows of ostride elements;
// tmp holds n * E counts (the sample-major rows before their transpose).
hipError_t launch_range_counts(const int64_t *indptr, const int32_t *spos, const int32_t *scum,
                               const int32_t *lo, const int32_t *hi, int32_t slot0, int32_t E,
                               int32_t n, void *out, int32_t cw, int64_t ostride, void *tmp, hipStream_t st);
// Presence bits of branch slots [slot0, slot0 + Bc) in the matrix-core layout: P[k][b / 8]
// bit b % 8 for k < n_pad (rows k >= n are zero), b < kpad (bits b >= Bc are zero).
hipError_t launch_range_bits(const int64_t *indptr, const int32_t *spos, const int32_t *scum,
                             const int32_t *lo, const int32_t *hi, int32_t slot0, int32_t Bc,
                             int64_t kpad, int32_t n, int32_t n_pad, uint8_t *P, hipStream_t st);

// Matrix-core path (unweighted).  Presence bits P[n_pad][k_pad / 8] (bit b % 8 of byte b / 8
// per branch slot b), bf16 length splits hi/lo[k_pad], upper-triangular GM x GM output tiles.
struct MfmaGeom {
    int32_t n, B;
    int32_t n_pad;      // samples rounded up to 256
    int64_t k_pad;      // branches rounded up to the K stage (128)
    int32_t tile, kstep;
    int32_t n_tiles;    // upper-triangular tiles including the diagonal
};
MfmaGeom mfma_geometry(int32_t n, int32_t n_branches);
void mfma_tile_list(int32_t n, std::vector<int32_t> *xy);   // (I, J) pairs, I <= J
hipError_t launch_split_lengths(const double *len, int32_t B, int64_t k_pad, uint16_t *hi,
                                uint16_t *lo, hipStream_t st);
hipError_t launch_bits_transpose(const uint32_t *bits, int64_t bstride, const MfmaGeom &g,
                                 uint8_t *Pb, hipStream_t st);
// accum != 0: the products of this launch are added into S and T (a later chunk of branches)
hipError_t launch_mfma_gemm(const uint8_t *P, const uint16_t *hi, const uint16_t *lo,
                            int32_t k_chunk, const int32_t *tiles_xy, const MfmaGeom &g,
                            double *S, double *T, int32_t variant, hipStream_t st, int32_t accum = 0);
hipError_t launch_mfma_normalize(const double *S, const double *T, int32_t n, int32_t out_f32,
                                 void *out, hipStream_t st);
// One job of the matrix-core path, for the single-job and queued kernels.
struct MfmaArgs {
    const uint8_t *P;           // presence bits [n_pad][k_pad / 8]
    int64_t k_pad;
    int32_t n_kstep, chunk_steps;
    const uint16_t *hi, *lo;    // bf16 splits [k_pad]
    int32_t n, n_tiles;
    int32_t accum, pad;         // accum != 0: add into S and T instead of storing first
    double *S, *T;              // condensed shared lengths, per-sample totals
    const int2 *tiles;          // (I, J) tile list of this job
};
MfmaArgs make_mfma_args(const uint8_t *P, const uint16_t *hi, const uint16_t *lo, int32_t k_chunk,
                        const int32_t *tiles_xy, const MfmaGeom &g, double *S, double *T);
// items_xy: (job index, tile index) pairs; *counter == 0 at launch.
hipError_t launch_mfma_queue(const MfmaArgs *jobs, const int32_t *items_xy, int32_t n_items,
                             int32_t *counter, int32_t n_groups, int32_t variant, hipStream_t st);

}  // namespace ufmi
