// C ABI: contexts, plans, and the orchestration of the device hot path.
//
// A plan validates and preprocesses the inputs once and keeps them resident in device
// memory; uf_plan_distance then runs every step of the path on the GPU:
//   (a)  embedding propagation: scatter tip reads, one launch per height level;
//   (a2) embedding transform of a batch of branches into wrap-padded rows;
//   (b)  striped accumulation of the batch into the numerator/denominator stripes;
//   (d)  normalize/condense into the caller's condensed output.
// The matrix-core form of the unweighted variant replaces (a2)-(b) by presence bits and a
// bf16 MFMA product (k_mfma.hip).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>

#include "uf_runtime.h"

namespace ufmi {
thread_local std::string g_tls_err;
}

using namespace ufmi;

namespace ufmi {

void range_row_runs(int32_t n, int32_t s_begin, int32_t s_end, std::vector<int32_t> *len_a,
                    std::vector<int32_t> *len_b, std::vector<int64_t> *off)
{
    const int32_t S = n / 2;
    len_a->assign(n, 0);
    len_b->assign(n, 0);
    off->assign((size_t)n + 1, 0);
    const int32_t a_hi = std::min(s_end, S), b_lo = std::max(n - s_end, S + 1), b_hi = n - 1 - s_begin;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t lim = n - 1 - i;   // largest distance j - i in row i
        (*len_a)[i] = std::max(0, std::min(a_hi, lim) - s_begin);
        (*len_b)[i] = std::max(0, std::min(b_hi, lim) - b_lo + 1);
        (*off)[i + 1] = (*off)[i] + (*len_a)[i] + (*len_b)[i];
    }
}

int32_t resolve_count_width(const HostPrep &hp, int32_t requested)
{
    int32_t max_total = 0;
    for (int32_t t : hp.totals) max_total = std::max(max_total, t);
    if (requested == 4) return 4;
    if (requested == 2) return max_total <= 65535 ? 2 : -1;
    return max_total <= 65535 ? 2 : 4;
}

// (a) embedding propagation, count form (int32 or packed uint16 rows).
uf_status propagate_counts(uf_plan *plan, hipStream_t st, int32_t cw)
{
    uf_context *ctx = plan->ctx;
    const HostPrep &hp = plan->hp;
    cw = resolve_count_width(hp, cw);
    if (cw < 0) return set_err(ctx, UF_E_ARG, "16-bit counts need every sample total <= 65535");
    plan->cw = cw;
    UF_TRY(plan->counts.ensure((size_t)hp.n_nodes * plan->cstride * cw), "allocating embedding counts");
    return propagate_counts_into(plan, plan->counts.p, cw, st);
}

// The same into caller-provided rows C ([n_nodes][cstride] counts of cw bytes); allocates
// nothing.
uf_status propagate_counts_into(uf_plan *plan, void *C, int32_t cw, hipStream_t st)
{
    uf_context *ctx = plan->ctx;
    const HostPrep &hp = plan->hp;
    const int64_t words = plan->cstride * cw / 4;   // uint32 words per row
    UF_TRY(launch_fill_u32(C, 0u, (size_t)hp.n_leaf * words, st), "clearing tip rows");
    UF_TRY(timed(plan, "propagate", st, [&] {
               hipError_t r = launch_scatter_counts(plan->indptr.as<int64_t>(),
                                                    plan->entry_slot.as<int32_t>(),
                                                    plan->entry_count.as<int32_t>(), C, cw,
                                                    plan->cstride, hp.n_samples, st);
               for (int32_t h = 1; h < plan->tail_level && r == hipSuccess; ++h) {
                   const int32_t b = hp.level_ptr[h], e = hp.level_ptr[h + 1];
                   r = launch_level_sum(C, words, b, e - b, hp.n_leaf,
                                        plan->child_ptr.as<int32_t>(),
                                        plan->child_slot.as<int32_t>(), st);
               }
               if (r == hipSuccess)
                   r = launch_level_tail(false, static_cast<uint32_t *>(C), words, plan->tail, st);
               return r;
           }), "propagating counts");
    return UF_OK;
}

// (a) embedding propagation, presence-bit form.
uf_status propagate_bits(uf_plan *plan, hipStream_t st)
{
    uf_context *ctx = plan->ctx;
    const HostPrep &hp = plan->hp;
    UF_TRY(plan->bits.ensure((size_t)hp.n_nodes * plan->bstride * sizeof(uint32_t)),
           "allocating presence bits");
    uint32_t *B = plan->bits.as<uint32_t>();
    UF_TRY(launch_fill_u32(B, 0u, (size_t)hp.n_leaf * plan->bstride, st), "clearing tip rows");
    UF_TRY(timed(plan, "propagate", st, [&] {
               hipError_t r = launch_scatter_bits(plan->indptr.as<int64_t>(),
                                                  plan->entry_slot.as<int32_t>(),
                                                  plan->entry_count.as<int32_t>(), B,
                                                  plan->bstride, hp.n_samples, st);
               for (int32_t h = 1; h < plan->tail_level && r == hipSuccess; ++h) {
                   const int32_t b = hp.level_ptr[h], e = hp.level_ptr[h + 1];
                   r = launch_level_or(B, plan->bstride, b, e - b, hp.n_leaf,
                                       plan->child_ptr.as<int32_t>(),
                                       plan->child_slot.as<int32_t>(), st);
               }
               if (r == hipSuccess)
                   r = launch_level_tail(true, B, plan->bstride, plan->tail, st);
               return r;
           }), "propagating presence");
    return UF_OK;
}

uf_status plan_prepare(uf_context *ctx, const uf_tree *tree, const uf_table *table,
                       hipStream_t st, uf_plan **out)
{
    *out = nullptr;
    uf_plan *plan = new (std::nothrow) uf_plan;
    if (!plan) return set_err(ctx, UF_E_OOM, "host allocation failed");
    plan->ctx = ctx;
    std::string err;
    uf_status s = validate_and_prepare(tree, table, &plan->hp, &err);
    if (s != UF_OK) {
        delete plan;
        return set_err(ctx, s, err);
    }
    hipError_t e = enter_device(ctx->device);
    if (e != hipSuccess) {
        delete plan;
        return hip_fail(ctx, e, "hipSetDevice");
    }
    const HostPrep &hp = plan->hp;
    plan->cstride = round_up(hp.n_samples, 64);
    plan->bstride = round_up((hp.n_samples + 31) / 32, 4);
    hipError_t r = hipSuccess;
    if (r == hipSuccess) r = upload(plan->indptr, hp.indptr, st);
    if (r == hipSuccess) r = upload(plan->entry_slot, hp.entry_slot, st);
    if (r == hipSuccess) r = upload(plan->entry_count, hp.entry_count, st);
    if (r == hipSuccess) r = upload(plan->totals, hp.totals, st);
    if (r == hipSuccess) r = upload(plan->child_ptr, hp.child_ptr, st);
    if (r == hipSuccess) r = upload(plan->child_slot, hp.child_slot, st);
    if (r == hipSuccess) r = upload(plan->len_slot, hp.length_slot, st);
    if (r == hipSuccess) r = upload(plan->slot_of_node, hp.slot_of_node, st);
    // the narrow top of a deep tree (levels of at most 64 nodes) runs as one launch; a short
    // narrow top (under eight levels) keeps one launch per level
    plan->tail_level = std::max(narrow_tail_level(hp, 64), 1);
    TailProgramHost tph;
    if (hp.n_levels - plan->tail_level < 8 || !tail_program(hp, plan->tail_level, &tph))
        plan->tail_level = hp.n_levels;
    if (plan->tail_level < hp.n_levels) {
        if (r == hipSuccess) r = upload(plan->tail_lvl, tph.lvl, st);
        if (r == hipSuccess) r = upload(plan->tail_rec, tph.rec, st);
        if (r == hipSuccess) r = upload(plan->tail_kid, tph.kid, st);
        if (r == hipSuccess) r = upload(plan->tail_chunks, tph.chunks, st);
        plan->tail.lvl = plan->tail_lvl.as<int32_t>();
        plan->tail.rec = plan->tail_rec.as<int4>();
        plan->tail.kid = plan->tail_kid.as<int32_t>();
        plan->tail.chunks = plan->tail_chunks.as<int2>();
        plan->tail.n_chunks = (int32_t)(tph.chunks.size() / 2);
    }
    if (r == hipSuccess) r = hipStreamSynchronize(st);
    if (r != hipSuccess) {
        uf_plan_destroy(plan);
        return hip_fail(ctx, r, "uploading inputs");
    }
    *out = plan;
    return UF_OK;
}

}  // namespace ufmi

namespace ufmi {

Knobs resolve_knobs(const uf_tuning *t, uf_precision prec, int32_t n_branches)
{
    Knobs k;
    // FP32 sums inside a batch: worst-case relative error ~ E * 2^-24 of the denominator,
    // so the FP32 default batch is kept at 128 (< 1e-5); FP64 batches only trade stripe
    // traffic against embedding-buffer size.
    k.emb_batch = (t && t->emb_batch > 0) ? t->emb_batch : (prec == UF_PREC_FP32 ? 128 : 1024);
    k.e_free = (t && t->emb_batch > 0) || prec != UF_PREC_FP64 ? 0 : 1;
    k.emb_batch = std::min(k.emb_batch, 4096);
    if (n_branches > 0) k.emb_batch = std::min(k.emb_batch, n_branches);
    k.emb_batch = std::max(k.emb_batch, 1);
    k.k_chunk = (t && t->k_chunk > 0) ? t->k_chunk : 4096;
    k.den_mode = (t ? t->den_mode : 0);
    k.variant = (t ? t->variant : 0);
    // without knobs, tile shape 2: the fastest measured for the default den_mode 0 in both
    // precisions (and for the FP32 per-sample denominator form)
    k.tile = (t ? t->tile : 2);
    k.count_width = (t ? t->count_width : 0);
    k.k_split = (t ? t->k_split : 0);
    return k;
}

// Branch splits of the fused striped kernel: enough work-groups for about twenty rounds of
// the device, so that the work-groups that finish last hold a small part of the run (two
// rounds left a measured 5 % behind; on 4,096 samples 32 splits beat 16 by 1-1.5 % in FP32
// and FP64 once the copies were no longer cleared), at most 32 splits, at least two batches
// per split, and the copies of the stripe state within 4 GB.  No split when the stripe tiles
// alone give twenty rounds.
int32_t auto_k_split(const uf_context *ctx, const StripeGeom &g, int64_t tiles, int32_t B, int32_t *E,
                     bool e_free, size_t state_bytes)
{
    const int64_t slots = (int64_t)std::max(ctx->n_cu, 1) * std::max(g.occ, 1);
    constexpr int64_t kRounds = 20;
    if (tiles <= 0 || tiles >= kRounds * slots) return 1;
    int64_t kz = (kRounds * slots + tiles - 1) / tiles;
    // up to 32 splits; up to 64 when even 16 would not give the device one round
    kz = std::min<int64_t>(kz, tiles * 16 < slots ? 64 : 32);
    // >= 2 batches per split; a batch depth the caller left free (FP64, where it only
    // trades state traffic) shrinks, down to 64 branches, to allow the splits
    if (e_free && B / std::max(2 * *E, 1) < kz) *E = (int32_t)std::max<int64_t>(64, std::min<int64_t>(*E, B / (2 * kz)));
    kz = std::min<int64_t>(kz, std::max<int64_t>(1, B / std::max(2 * *E, 1)));
    const size_t budget = (size_t)4 << 30;
    if (state_bytes > 0) kz = std::min<int64_t>(kz, std::max<int64_t>(1, (int64_t)(budget / state_bytes)));
    return (int32_t)std::max<int64_t>(kz, 1);
}

StripeGeom striped_geometry(const uf_plan *plan, uf_precision prec, const Knobs &kn)
{
    return stripe_geometry(plan->hp.n_samples, prec == UF_PREC_FP64, kn.den_mode, kn.variant == 0 ? kn.tile : 0);
}

// Stripe tiles [*t0, *t1) that cover stripes [s_begin, s_end) (-1, -1 = all) and the FP64
// bytes of one copy of their state.
size_t striped_state_bytes(const StripeGeom &g, int32_t s_begin, int32_t s_end, int32_t *t0, int32_t *t1)
{
    *t0 = 0;
    *t1 = g.spad / g.tsw;
    if (s_begin >= 0) {
        *t0 = s_begin / g.tsw;
        *t1 = (s_end + g.tsw - 1) / g.tsw;
    }
    return (size_t)(*t1 - *t0) * g.tsw * g.sstride * sizeof(double);
}

// Branch splits (and, when the caller left it free, the FP64 batch depth) of the fused
// kernel.  Both follow from the whole problem's stripe tiles, not the range being computed,
// so that stripe ranges repeat the per-element arithmetic of the full computation.
int32_t striped_k_split(const uf_plan *plan, Knobs &kn, const StripeGeom &g, size_t state)
{
    const int32_t B = plan->hp.n_nodes - 1;
    const int64_t tiles = (int64_t)(g.sstride / g.tkw) * (g.spad / g.tsw);
    return kn.variant != 0 ? 1
           : kn.k_split > 0 ? std::min(kn.k_split, std::max(B, 1))
                            : auto_k_split(plan->ctx, g, tiles, B, &kn.emb_batch, kn.e_free != 0,
                                           kn.den_mode == 0 ? 2 * state : state);
}

// (a)-(b) of the fused form on caller-provided buffers, allocating nothing: propagation into
// W.C, the fused striped kernel over stripe tiles [t0, t1) into kz state copies at W.num /
// W.den (each `state` bytes), their reduction, and the per-sample sums into W.D (den_mode 1).
uf_status striped_core(uf_plan *plan, uf_method method, uf_precision prec, const Knobs &kn,
                       const StripeGeom &g, int32_t t0, int32_t t1, int32_t kz, size_t state,
                       int32_t cw, const StripedWork &W, hipStream_t st)
{
    uf_context *ctx = plan->ctx;
    const HostPrep &hp = plan->hp;
    const bool fp64 = (prec == UF_PREC_FP64);
    // the unnormalized variant accumulates the weighted-normalized numerator only
    const bool unnorm = (method == UF_WEIGHTED_UNNORMALIZED);
    if (unnorm) method = UF_WEIGHTED_NORMALIZED;
    const int32_t B = hp.n_nodes - 1;
    double *num = W.num, *den = kn.den_mode == 0 ? W.den : nullptr;
    if (B == 0) {  // single-node tree: no branches, every distance is 0
        UF_TRY(launch_fill_u32(num, 0u, state / 4, st), "clearing stripes");
        if (den) UF_TRY(launch_fill_u32(den, 0u, state / 4, st), "clearing stripes");
        UF_TRY(launch_fill_u32(W.D, 0u, (size_t)hp.n_samples * 2, st), "clearing sums");
        return UF_OK;
    }
    uf_status s = propagate_counts_into(plan, W.C, cw, st);
    if (s != UF_OK) return s;
    // no clearing: the first batch of every split writes its state copy (every split has at
    // least one branch, kz <= B, and the tiles cover the copy)
    const double *len = plan->len_slot.as<double>();
    UF_TRY(launch_inv_totals(plan->totals.as<int32_t>(), hp.n_samples, W.inv_t, st), "reciprocal totals");
    UF_TRY(timed(plan, "stripe", st, [&] {
               return launch_stripe_fused(fp64, method, kn.den_mode, kn.tile, W.C, cw,
                                          plan->cstride, W.inv_t, len, B, kn.emb_batch, num, den, g,
                                          t0, t1, kz, (int64_t)(state / sizeof(double)), true, st);
           }), "striped accumulation");
    if (kz > 1)   // the split copies, summed in split order
        UF_TRY(timed(plan, "reduce", st, [&] {
                   hipError_t r = launch_reduce_z(num, (int64_t)(state / sizeof(double)), kz,
                                                  (int64_t)(state / sizeof(double)), st);
                   if (r == hipSuccess && den)
                       r = launch_reduce_z(den, (int64_t)(state / sizeof(double)), kz,
                                           (int64_t)(state / sizeof(double)), st);
                   return r;
               }), "summing branch splits");
    if (kn.den_mode != 0 && !unnorm)
        UF_TRY(timed(plan, "rowdot", st, [&] {
                   return launch_rowdot(method, W.C, cw, plan->cstride, 0, B, plan->totals.as<int32_t>(),
                                        len, g.n, W.D, true, W.part, st);
               }), "per-sample sums");
    return UF_OK;
}

}  // namespace ufmi

namespace {

// Device bytes of the plan's resident inputs.
size_t input_bytes(const uf_plan *plan)
{
    const HostPrep &hp = plan->hp;
    return (size_t)(hp.n_samples + 1) * 8 + (size_t)hp.nnz * 8 + (size_t)hp.n_samples * 4 +
           (size_t)hp.n_nodes * (4 + 4 + 8 + 4);
}

// The generated-rows tables (depth-first tip ranges, sorted entries), a second stream and
// its events, made once per plan.
uf_status gen_prepare(uf_plan *plan, hipStream_t st)
{
    uf_context *ctx = plan->ctx;
    if (plan->gen_ready) return UF_OK;
    RangeTables rt;
    range_tables(plan->hp, &rt);
    UF_TRY(upload(plan->gen_lo, rt.lo, st), "uploading tip ranges");
    UF_TRY(upload(plan->gen_hi, rt.hi, st), "uploading tip ranges");
    UF_TRY(upload(plan->gen_spos, rt.spos, st), "uploading sorted entries");
    UF_TRY(upload(plan->gen_scum, rt.scum, st), "uploading sorted entries");
    if (!plan->gen_stream)
        UF_TRY(hipStreamCreateWithFlags(&plan->gen_stream, hipStreamNonBlocking), "creating the row stream");
    for (hipEvent_t *e : {&plan->gen_start, &plan->gen_filled[0], &plan->gen_filled[1], &plan->gen_used[0],
                          &plan->gen_used[1]})
        if (!*e) UF_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming), "creating row events");
    UF_TRY(hipStreamSynchronize(st), "synchronizing");   // the host tables go out of scope
    plan->gen_ready = true;
    return UF_OK;
}

size_t gen_table_bytes(const uf_plan *plan)
{
    return (size_t)plan->hp.nnz * 8 + (size_t)plan->hp.n_nodes * 8;
}

// (a)-(b) with generated rows: batch i of E branches is computed into buffer i % 2 on the
// row stream while the striped kernel accumulates batch i - 1 from the other buffer; events
// order each buffer's fill after its previous use.  One state copy (no branch split).
uf_status striped_generated(uf_plan *plan, uf_method method, uf_precision prec, const Knobs &kn,
                            const StripeGeom &g, int32_t t0, int32_t t1, size_t state, int32_t cw,
                            hipStream_t st)
{
    uf_context *ctx = plan->ctx;
    const HostPrep &hp = plan->hp;
    const bool fp64 = (prec == UF_PREC_FP64);
    const bool unnorm = (method == UF_WEIGHTED_UNNORMALIZED);
    if (unnorm) method = UF_WEIGHTED_NORMALIZED;
    const int32_t B = hp.n_nodes - 1, E = kn.emb_batch, n = hp.n_samples;
    uf_status s = gen_prepare(plan, st);
    if (s != UF_OK) return s;
    const size_t rows = (size_t)E * plan->cstride * cw;
    UF_TRY(plan->num.ensure(state), "allocating numerator stripes");
    if (kn.den_mode == 0) UF_TRY(plan->den.ensure(state), "allocating denominator stripes");
    UF_TRY(plan->D.ensure((size_t)n * sizeof(double)), "allocating per-sample sums");
    UF_TRY(plan->inv_t.ensure((size_t)n * sizeof(double)), "allocating totals");
    UF_TRY(plan->rowdot_part.ensure(rowdot_scratch_elems(n, E) * sizeof(double)), "allocating sum scratch");
    UF_TRY(plan->gen_buf[0].ensure(rows), "allocating generated rows");
    UF_TRY(plan->gen_buf[1].ensure(rows), "allocating generated rows");
    UF_TRY(plan->gen_tmp.ensure((size_t)E * n * cw), "allocating generated rows");
    double *num = plan->num.as<double>();
    double *den = kn.den_mode == 0 ? plan->den.as<double>() : nullptr;
    UF_TRY(launch_fill_u32(num, 0u, state / 4, st), "clearing stripes");
    if (den) UF_TRY(launch_fill_u32(den, 0u, state / 4, st), "clearing stripes");
    UF_TRY(launch_inv_totals(plan->totals.as<int32_t>(), n, plan->inv_t.as<double>(), st), "reciprocal totals");
    const double *len = plan->len_slot.as<double>();
    hipStream_t gs = plan->gen_stream;
    UF_TRY(hipEventRecord(plan->gen_start, st), "ordering the row stream");
    UF_TRY(hipStreamWaitEvent(gs, plan->gen_start, 0), "ordering the row stream");
    int32_t i = 0;
    for (int32_t b0 = 0; b0 < B; b0 += E, ++i) {
        const int32_t eb = std::min(E, B - b0), x = i & 1;
        void *buf = plan->gen_buf[x].p;
        if (i >= 2) UF_TRY(hipStreamWaitEvent(gs, plan->gen_used[x], 0), "reusing a row buffer");
        UF_TRY(timed(plan, "generate", gs, [&] {
                   return launch_range_counts(plan->indptr.as<int64_t>(), plan->gen_spos.as<int32_t>(),
                                              plan->gen_scum.as<int32_t>(), plan->gen_lo.as<int32_t>(),
                                              plan->gen_hi.as<int32_t>(), b0, eb, n, buf, cw,
                                              plan->cstride, plan->gen_tmp.p, gs);
               }), "generating count rows");
        UF_TRY(hipEventRecord(plan->gen_filled[x], gs), "ordering generated rows");
        UF_TRY(hipStreamWaitEvent(st, plan->gen_filled[x], 0), "ordering generated rows");
        UF_TRY(timed(plan, "stripe", st, [&] {
                   return launch_stripe_fused(fp64, method, kn.den_mode, kn.tile, buf, cw, plan->cstride,
                                              plan->inv_t.as<double>(), len + b0, eb, eb, num, den, g, t0,
                                              t1, 1, (int64_t)(state / sizeof(double)), false, st);
               }), "striped accumulation");
        if (kn.den_mode != 0 && !unnorm)
            UF_TRY(timed(plan, "rowdot", st, [&] {
                       return launch_rowdot(method, buf, cw, plan->cstride, 0, eb, plan->totals.as<int32_t>(),
                                            len + b0, n, plan->D.as<double>(), b0 == 0,
                                            plan->rowdot_part.as<double>(), st);
                   }), "per-sample sums");
        UF_TRY(hipEventRecord(plan->gen_used[x], st), "releasing a row buffer");
    }
    return UF_OK;
}

// (a)-(b): fills plan->num / den (den_mode 0) or num / D (den_mode 1).
// Stripes [s_begin, s_end) (-1, -1 = all): the state block covers the stripe tiles that
// overlap the range and *s_base receives the stripe held by its first row.
uf_status run_striped(uf_plan *plan, uf_method method, uf_precision prec, Knobs kn,
                      StripeGeom *geom, hipStream_t st, int32_t s_begin = -1, int32_t s_end = -1,
                      int32_t *s_base = nullptr)
{
    uf_context *ctx = plan->ctx;
    const HostPrep &hp = plan->hp;
    const bool fp64 = (prec == UF_PREC_FP64);
    const StripeGeom g = striped_geometry(plan, prec, kn);
    *geom = g;
    int32_t tile_s0 = 0, tile_s1 = 0;
    const size_t state = striped_state_bytes(g, s_begin, s_end, &tile_s0, &tile_s1);
    if (s_base) *s_base = tile_s0 * g.tsw;
    const int32_t B = hp.n_nodes - 1;
    const size_t tsz = fp64 ? sizeof(double) : sizeof(float);
    const int32_t cw = resolve_count_width(hp, kn.count_width);
    if (cw < 0) return set_err(ctx, UF_E_ARG, "16-bit counts need every sample total <= 65535");
    int32_t kz = striped_k_split(plan, kn, g, state);
    if (kn.variant == 0 && B > 0) {
        // resident rows, or rows generated batch by batch when they would not fit
        const size_t sums = (size_t)hp.n_samples * 16 + rowdot_scratch_elems(g.n, B) * sizeof(double);
        const size_t resident = input_bytes(plan) + (size_t)hp.n_nodes * plan->cstride * cw +
                                state * kz * (kn.den_mode == 0 ? 2 : 1) + sums;
        bool gen = plan->mem_limit > 0 && resident > (size_t)plan->mem_limit;
        if (gen) {
            const size_t need = input_bytes(plan) + gen_table_bytes(plan) +
                                3 * (size_t)kn.emb_batch * plan->cstride * cw +
                                state * (kn.den_mode == 0 ? 2 : 1) + (size_t)hp.n_samples * 16 +
                                rowdot_scratch_elems(g.n, kn.emb_batch) * sizeof(double);
            if (need > (size_t)plan->mem_limit)
                return set_err(ctx, UF_E_OOM, "even generated count rows need " + std::to_string(need) +
                                                  " device bytes, above the plan's limit");
        } else {
            hipError_t e = plan->counts.ensure((size_t)hp.n_nodes * plan->cstride * cw);
            if (e == hipErrorOutOfMemory) {   // the full rows do not fit: generate them
                (void)hipGetLastError();
                gen = true;
            } else if (e != hipSuccess) {
                return hip_fail(ctx, e, "allocating embedding counts");
            }
        }
        if (gen) {
            plan->counts.release();
            return striped_generated(plan, method, prec, kn, g, tile_s0, tile_s1, state, cw, st);
        }
    }
    UF_TRY(plan->num.ensure(state * kz), "allocating numerator stripes");
    if (kn.den_mode == 0) UF_TRY(plan->den.ensure(state * kz), "allocating denominator stripes");
    UF_TRY(plan->D.ensure((size_t)hp.n_samples * sizeof(double)), "allocating per-sample sums");
    double *num = plan->num.as<double>();
    double *den = kn.den_mode == 0 ? plan->den.as<double>() : nullptr;
    double *D = plan->D.as<double>();
    if (kn.variant == 0) {
        StripedWork W{};
        W.num = num;
        W.den = den;
        W.D = D;
        if (B > 0) {
            UF_TRY(plan->counts.ensure((size_t)hp.n_nodes * plan->cstride * cw), "allocating embedding counts");
            UF_TRY(plan->inv_t.ensure((size_t)hp.n_samples * sizeof(double)), "allocating totals");
            if (kn.den_mode != 0 && method != UF_WEIGHTED_UNNORMALIZED)
                UF_TRY(plan->rowdot_part.ensure(rowdot_scratch_elems(g.n, B) * sizeof(double)),
                       "allocating per-sample sum scratch");
            W.C = plan->counts.p;
            plan->cw = cw;
            W.inv_t = plan->inv_t.as<double>();
            W.part = plan->rowdot_part.as<double>();
        }
        return striped_core(plan, method, prec, kn, g, tile_s0, tile_s1, kz, state, cw, W, st);
    }
    // the unnormalized variant accumulates the weighted-normalized numerator only
    const bool unnorm = (method == UF_WEIGHTED_UNNORMALIZED);
    if (unnorm) method = UF_WEIGHTED_NORMALIZED;
    if (B == 0) {  // single-node tree: no branches, every distance is 0
        UF_TRY(launch_fill_u32(num, 0u, state / 4, st), "clearing stripes");
        if (den) UF_TRY(launch_fill_u32(den, 0u, state / 4, st), "clearing stripes");
        UF_TRY(launch_fill_u32(D, 0u, (size_t)hp.n_samples * 2, st), "clearing sums");
        return UF_OK;
    }
    uf_status s = propagate_counts(plan, st, kn.count_width);
    if (s != UF_OK) return s;
    UF_TRY(launch_fill_u32(num, 0u, state * kz / 4, st), "clearing stripes");
    if (den) UF_TRY(launch_fill_u32(den, 0u, state * kz / 4, st), "clearing stripes");
    const int32_t E = kn.emb_batch;
    const void *C = plan->counts.p;
    const double *len = plan->len_slot.as<double>();
    UF_TRY(plan->emb.ensure((size_t)E * g.estride * tsz), "allocating embedding batch");
    if (kn.den_mode != 0 && !unnorm)
        UF_TRY(plan->rowdot_part.ensure(rowdot_scratch_elems(g.n, E) * sizeof(double)),
               "allocating per-sample sum scratch");
    for (int32_t b0 = 0; b0 < B; b0 += E) {
        const int32_t eb = std::min(E, B - b0);
        UF_TRY(timed(plan, "transform", st, [&] {
                   return launch_transform(fp64, method, C, cw, plan->cstride, b0, eb,
                                           plan->totals.as<int32_t>(), g.n, g.S, plan->emb.p,
                                           g.estride, st);
               }), "embedding transform");
        UF_TRY(timed(plan, "stripe", st, [&] {
                   return launch_stripe(fp64, method, kn.den_mode, plan->emb.p, g.estride,
                                        len + b0, eb, num, den, g, b0 == 0, st);
               }), "striped accumulation");
        if (kn.den_mode != 0 && !unnorm)
            UF_TRY(timed(plan, "rowdot", st, [&] {
                       return launch_rowdot(method, C, cw, plan->cstride, b0, eb,
                                            plan->totals.as<int32_t>(), len + b0, g.n, D,
                                            b0 == 0, plan->rowdot_part.as<double>(), st);
                   }), "per-sample sums");
    }
    return UF_OK;
}

}  // namespace

namespace ufmi {

uf_status check_enums(uf_context *ctx, uf_method method, uf_precision prec)
{
    if (method != UF_UNWEIGHTED && method != UF_WEIGHTED_NORMALIZED &&
        method != UF_WEIGHTED_UNNORMALIZED)
        return set_err(ctx, UF_E_ARG, "unknown method");
    if (prec != UF_PREC_FP64 && prec != UF_PREC_FP32 && prec != UF_PREC_MFMA_BF16X2)
        return set_err(ctx, UF_E_ARG, "unknown precision");
    if (prec == UF_PREC_MFMA_BF16X2 && method != UF_UNWEIGHTED)
        return set_err(ctx, UF_E_UNSUPPORTED,
                       "the matrix-core form exists for unweighted UniFrac only");
    return UF_OK;
}

}  // namespace ufmi

namespace {
// Matrix-core form of the unweighted variant: fills `out_dev` with condensed distances.
// Scratch: [0] presence bits, [1] hi/lo splits, [2] tile list, [3] T and (for FP32 or
// host output) the FP64 shared-length array S.
uf_status run_mfma_unweighted(uf_plan *plan, int32_t k_chunk, int32_t variant, int32_t out_f32, void *out_dev,
                              hipStream_t st)
{
    uf_context *ctx = plan->ctx;
    const HostPrep &hp = plan->hp;
    const int32_t n = hp.n_samples, B = hp.n_nodes - 1;
    const MfmaGeom g = mfma_geometry(n, B);
    const int64_t n_pairs = (int64_t)n * (n - 1) / 2;
    k_chunk = std::max(g.kstep, k_chunk / g.kstep * g.kstep);
    DevMem &Pm = plan->mfma_scratch[0], &HL = plan->mfma_scratch[1];
    DevMem &TL = plan->mfma_scratch[2], &TS = plan->mfma_scratch[3];
    std::vector<int32_t> xy;
    mfma_tile_list(n, &xy);
    const bool s_in_out = !out_f32;   // FP64 output doubles as the S array
    const size_t t_bytes = (size_t)g.n_pad * sizeof(double);
    const size_t ts_bytes = t_bytes + (s_in_out ? 0 : (size_t)n_pairs * sizeof(double));
    // resident presence bits, or bits generated chunk by chunk when they would not fit
    const size_t fixed = input_bytes(plan) + xy.size() * sizeof(int32_t) + ts_bytes;
    const size_t resident = fixed + (size_t)hp.n_nodes * plan->bstride * 4 + (size_t)g.n_pad * (g.k_pad / 8) +
                            (size_t)4 * g.k_pad;
    bool gen = plan->mem_limit > 0 && resident > (size_t)plan->mem_limit;
    if (!gen) {
        hipError_t e = plan->bits.ensure((size_t)hp.n_nodes * plan->bstride * sizeof(uint32_t));
        if (e == hipSuccess) e = Pm.ensure((size_t)g.n_pad * (g.k_pad / 8));
        if (e == hipErrorOutOfMemory) {   // the full bits do not fit: generate them
            (void)hipGetLastError();
            gen = true;
        } else if (e != hipSuccess) {
            return hip_fail(ctx, e, "allocating presence bits");
        }
    }
    UF_TRY(TL.ensure(xy.size() * sizeof(int32_t)), "allocating tile list");
    UF_TRY(hipMemcpyAsync(TL.p, xy.data(), xy.size() * sizeof(int32_t), hipMemcpyHostToDevice, st),
           "uploading tile list");
    UF_TRY(TS.ensure(ts_bytes), "allocating shared lengths");
    double *T = TS.as<double>();
    double *S = s_in_out ? static_cast<double *>(out_dev) : T + g.n_pad;
    if (!gen) {
        uf_status s = propagate_bits(plan, st);
        if (s != UF_OK) return s;
        UF_TRY(HL.ensure((size_t)2 * g.k_pad * sizeof(uint16_t)), "allocating length splits");
        uint16_t *hi = HL.as<uint16_t>(), *lo = hi + g.k_pad;
        UF_TRY(timed(plan, "bits_transpose", st, [&] {
                   hipError_t r = launch_split_lengths(plan->len_slot.as<double>(), B, g.k_pad, hi, lo, st);
                   if (r == hipSuccess)
                       r = launch_bits_transpose(plan->bits.as<uint32_t>(), plan->bstride, g,
                                                Pm.as<uint8_t>(), st);
                   return r;
               }), "presence transpose");
        UF_TRY(timed(plan, "mfma", st, [&] {
                   return launch_mfma_gemm(Pm.as<uint8_t>(), hi, lo, k_chunk, TL.as<int32_t>(), g, S,
                                           T, variant, st);
               }), "matrix-core product");
    } else {
        // chunks of Kc branches, a multiple of the FP64 flush group (four FP32 chains of the
        // kernel's chunk), so the sums come out in the same order as one launch over all
        plan->bits.release();
        Pm.release();
        uf_status s = gen_prepare(plan, st);
        if (s != UF_OK) return s;
        const int32_t cs = (std::max(1, k_chunk / g.kstep) + 1) & ~1;
        const int64_t group = (int64_t)4 * cs * g.kstep;
        const size_t row_bytes = (size_t)g.n_pad / 8;   // bytes per branch over all samples
        int64_t avail = plan->mem_limit > 0
                            ? (int64_t)plan->mem_limit - (int64_t)(fixed + gen_table_bytes(plan))
                            : (int64_t)1 << 31;
        int64_t Kc = avail / (int64_t)(2 * row_bytes + 4) / group * group;
        Kc = std::min<int64_t>(std::max<int64_t>(Kc, group), (g.k_pad + group - 1) / group * group);
        if (plan->mem_limit > 0 && (int64_t)(fixed + gen_table_bytes(plan) + Kc * (2 * row_bytes + 4)) > plan->mem_limit)
            return set_err(ctx, UF_E_OOM, "even generated presence bits exceed the plan's limit");
        UF_TRY(plan->gen_buf[0].ensure((size_t)Kc * row_bytes), "allocating generated bits");
        UF_TRY(plan->gen_buf[1].ensure((size_t)Kc * row_bytes), "allocating generated bits");
        UF_TRY(HL.ensure((size_t)2 * Kc * sizeof(uint16_t)), "allocating length splits");
        const double *len = plan->len_slot.as<double>();
        hipStream_t gs = plan->gen_stream;
        UF_TRY(hipEventRecord(plan->gen_start, st), "ordering the row stream");
        UF_TRY(hipStreamWaitEvent(gs, plan->gen_start, 0), "ordering the row stream");
        int32_t i = 0;
        for (int64_t c0 = 0; c0 < B; c0 += Kc, ++i) {
            const int32_t bc = (int32_t)std::min<int64_t>(Kc, B - c0), x = i & 1;
            const MfmaGeom gc = mfma_geometry(n, bc);
            uint8_t *P = plan->gen_buf[x].as<uint8_t>();
            if (i >= 2) UF_TRY(hipStreamWaitEvent(gs, plan->gen_used[x], 0), "reusing a bit buffer");
            UF_TRY(timed(plan, "generate", gs, [&] {
                       return launch_range_bits(plan->indptr.as<int64_t>(), plan->gen_spos.as<int32_t>(),
                                                plan->gen_scum.as<int32_t>(), plan->gen_lo.as<int32_t>(),
                                                plan->gen_hi.as<int32_t>(), (int32_t)c0, bc, gc.k_pad, n,
                                                gc.n_pad, P, gs);
                   }), "generating presence bits");
            UF_TRY(hipEventRecord(plan->gen_filled[x], gs), "ordering generated bits");
            UF_TRY(hipStreamWaitEvent(st, plan->gen_filled[x], 0), "ordering generated bits");
            uint16_t *hi = HL.as<uint16_t>(), *lo = hi + gc.k_pad;
            UF_TRY(launch_split_lengths(len + c0, bc, gc.k_pad, hi, lo, st), "length splits");
            UF_TRY(timed(plan, "mfma", st, [&] {
                       return launch_mfma_gemm(P, hi, lo, k_chunk, TL.as<int32_t>(), gc, S, T, variant, st,
                                               c0 > 0 ? 1 : 0);
                   }), "matrix-core product");
            UF_TRY(hipEventRecord(plan->gen_used[x], st), "releasing a bit buffer");
        }
    }
    UF_TRY(timed(plan, "normalize", st, [&] {
               return launch_mfma_normalize(S, T, n, out_f32, out_dev, st);
           }), "normalize");
    return UF_OK;
}
}  // namespace

extern "C" {

const char *uf_status_string(uf_status s)
{
    switch (s) {
    case UF_OK: return "UF_OK";
    case UF_E_ARG: return "UF_E_ARG";
    case UF_E_TREE: return "UF_E_TREE";
    case UF_E_TABLE: return "UF_E_TABLE";
    case UF_E_EMPTY_SAMPLE: return "UF_E_EMPTY_SAMPLE";
    case UF_E_DEVICE: return "UF_E_DEVICE";
    case UF_E_OOM: return "UF_E_OOM";
    case UF_E_UNSUPPORTED: return "UF_E_UNSUPPORTED";
    case UF_E_INTERNAL: return "UF_E_INTERNAL";
    }
    return "UF_E_UNKNOWN";
}

const char *uf_last_error(const uf_context *ctx)
{
    return ctx ? ctx->err.c_str() : g_tls_err.c_str();
}

uf_status uf_validate(const uf_tree *tree, const uf_table *table)
{
    HostPrep hp;
    std::string err;
    uf_status s = validate_and_prepare(tree, table, &hp, &err);
    g_tls_err = (s == UF_OK) ? std::string() : err;
    return s;
}

uf_status uf_context_create(int32_t device, uf_context **out)
{
    if (!out) return set_err(nullptr, UF_E_ARG, "out must not be NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0)
        return set_err(nullptr, UF_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= count) return set_err(nullptr, UF_E_ARG, "device out of range");
    e = hipSetDevice(device);
    if (e != hipSuccess) return set_err(nullptr, UF_E_DEVICE, hipGetErrorString(e));
    uf_context *ctx = new (std::nothrow) uf_context;
    if (!ctx) return set_err(nullptr, UF_E_OOM, "host allocation failed");
    ctx->device = device;
    e = noalloc_scratch_init(device);   // this device's copy of the fixed scratch array
    if (e != hipSuccess) {
        delete ctx;
        return set_err(nullptr, UF_E_DEVICE, std::string("resolving the device scratch: ") + hipGetErrorString(e));
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        ctx->n_cu = cus;
    *out = ctx;
    return UF_OK;
}

void uf_context_destroy(uf_context *ctx) { delete ctx; }

uf_status uf_plan_create(uf_context *ctx, const uf_tree *tree, const uf_table *table,
                         void *stream, uf_plan **out)
{
    if (!ctx || !out) return set_err(ctx, UF_E_ARG, "ctx and out must not be NULL");
    return plan_prepare(ctx, tree, table, static_cast<hipStream_t>(stream), out);
}

void uf_plan_destroy(uf_plan *plan)
{
    if (!plan) return;
    (void)enter_device(plan->ctx->device);
    for (DevMem *m : {&plan->indptr, &plan->entry_slot, &plan->entry_count, &plan->totals,
                      &plan->child_ptr, &plan->child_slot, &plan->len_slot, &plan->slot_of_node,
                      &plan->tail_lvl, &plan->tail_rec, &plan->tail_kid, &plan->tail_chunks,
                      &plan->counts, &plan->bits, &plan->emb, &plan->num, &plan->den, &plan->D,
                      &plan->inv_t, &plan->out_tmp, &plan->gather_tmp, &plan->rowdot_part})
        m->release();
    for (DevMem &m : plan->mfma_scratch) m.release();
    for (DevMem *m : {&plan->gen_spos, &plan->gen_scum, &plan->gen_lo, &plan->gen_hi, &plan->gen_buf[0],
                      &plan->gen_buf[1], &plan->gen_tmp})
        m->release();
    if (plan->gen_stream) (void)hipStreamDestroy(plan->gen_stream);
    for (hipEvent_t e : {plan->gen_start, plan->gen_filled[0], plan->gen_filled[1], plan->gen_used[0],
                         plan->gen_used[1]})
        if (e) (void)hipEventDestroy(e);
    plan->prof.release();
    delete plan;
    (void)hipGetLastError();   // leave no error of the release pending for the caller
}

uf_status uf_plan_set_memory_limit(uf_plan *plan, int64_t max_device_bytes)
{
    if (!plan) return set_err(nullptr, UF_E_ARG, "plan must not be NULL");
    if (max_device_bytes < 0) return set_err(plan->ctx, UF_E_ARG, "the memory limit must be >= 0");
    plan->mem_limit = max_device_bytes;
    return UF_OK;
}

uf_status uf_plan_trim(uf_plan *plan)
{
    if (!plan) return set_err(nullptr, UF_E_ARG, "plan must not be NULL");
    (void)enter_device(plan->ctx->device);
    for (DevMem *m : {&plan->counts, &plan->bits, &plan->emb, &plan->num, &plan->den, &plan->D,
                      &plan->inv_t, &plan->out_tmp, &plan->gather_tmp, &plan->rowdot_part,
                      &plan->gen_buf[0], &plan->gen_buf[1], &plan->gen_tmp})
        m->release();
    for (DevMem &m : plan->mfma_scratch) m.release();
    return UF_OK;
}

uf_status uf_plan_query(const uf_plan *plan, uf_plan_info *info)
{
    if (!plan || !info) return set_err(nullptr, UF_E_ARG, "plan and info must not be NULL");
    const HostPrep &hp = plan->hp;
    info->n_samples = hp.n_samples;
    info->n_nodes = hp.n_nodes;
    info->n_branches = hp.n_nodes - 1;
    info->n_leaves = hp.n_leaf;
    info->n_levels = hp.n_levels;
    info->n_stripes = hp.n_samples / 2;
    info->n_pairs = (int64_t)hp.n_samples * (hp.n_samples - 1) / 2;
    info->nnz = hp.nnz;
    return UF_OK;
}

static uf_status emit_rows(uf_plan *plan, const void *src, int64_t sstride, int32_t width,
                           void *out, int32_t out_on_device, hipStream_t st)
{
    uf_context *ctx = plan->ctx;
    const HostPrep &hp = plan->hp;
    const size_t bytes = (size_t)hp.n_nodes * width * sizeof(uint32_t);
    void *dst = out;
    if (!out_on_device) {
        UF_TRY(plan->gather_tmp.ensure(bytes), "allocating output staging");
        dst = plan->gather_tmp.p;
    }
    UF_TRY(launch_gather_rows_u32(static_cast<const uint32_t *>(src), sstride,
                                  plan->slot_of_node.as<int32_t>(), hp.n_nodes, width,
                                  static_cast<uint32_t *>(dst), st), "gathering rows");
    if (!out_on_device)
        UF_TRY(hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, st), "copying rows out");
    UF_TRY(hipStreamSynchronize(st), "synchronizing");
    return UF_OK;
}

uf_status uf_plan_embedding_counts(uf_plan *plan, int32_t *out, int32_t out_on_device,
                                   void *stream)
{
    if (!plan || !out) return set_err(plan ? plan->ctx : nullptr, UF_E_ARG, "NULL argument");
    uf_context *ctx = plan->ctx;
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    uf_status s = propagate_counts(plan, st, 4);
    if (s != UF_OK) return s;
    return emit_rows(plan, plan->counts.p, plan->cstride, plan->hp.n_samples, out, out_on_device, st);
}

uf_status uf_plan_embedding_counts16(uf_plan *plan, int32_t *out, int32_t out_on_device, void *stream)
{
    if (!plan || !out) return set_err(plan ? plan->ctx : nullptr, UF_E_ARG, "NULL argument");
    uf_context *ctx = plan->ctx;
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    uf_status s = propagate_counts(plan, st, 2);
    if (s != UF_OK) return s;
    const HostPrep &hp = plan->hp;
    const size_t bytes = (size_t)hp.n_nodes * hp.n_samples * sizeof(int32_t);
    void *dst = out;
    if (!out_on_device) {
        UF_TRY(plan->gather_tmp.ensure(bytes), "allocating output staging");
        dst = plan->gather_tmp.p;
    }
    UF_TRY(launch_gather_rows_u16(plan->counts.as<uint16_t>(), plan->cstride,
                                  plan->slot_of_node.as<int32_t>(), hp.n_nodes, hp.n_samples,
                                  static_cast<int32_t *>(dst), st), "gathering rows");
    if (!out_on_device)
        UF_TRY(hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, st), "copying rows out");
    UF_TRY(hipStreamSynchronize(st), "synchronizing");
    return UF_OK;
}

uf_status uf_plan_embedding_presence(uf_plan *plan, uint32_t *out, int32_t out_on_device,
                                     void *stream)
{
    if (!plan || !out) return set_err(plan ? plan->ctx : nullptr, UF_E_ARG, "NULL argument");
    uf_context *ctx = plan->ctx;
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    uf_status s = propagate_bits(plan, st);
    if (s != UF_OK) return s;
    return emit_rows(plan, plan->bits.p, plan->bstride, (plan->hp.n_samples + 31) / 32, out,
                     out_on_device, st);
}

uf_status uf_debug_embedding_counts(uf_context *ctx, const uf_tree *tree, const uf_table *table,
                                    int32_t *out_counts)
{
    if (!ctx || !out_counts) return set_err(ctx, UF_E_ARG, "ctx and out_counts must not be NULL");
    uf_plan *plan = nullptr;
    uf_status s = plan_prepare(ctx, tree, table, nullptr, &plan);
    if (s != UF_OK) return s;
    const HostPrep &hp = plan->hp;
    const int32_t nb = hp.n_nodes - 1, n = hp.n_samples;
    if (nb == 0) {
        uf_plan_destroy(plan);
        return UF_OK;
    }
    // slots of the non-root nodes in ascending node id
    std::vector<int32_t> slots;
    slots.reserve(nb);
    for (int32_t v = 0; v < hp.n_nodes; ++v)
        if (v != hp.root) slots.push_back(hp.slot_of_node[v]);
    const size_t bytes = (size_t)nb * n * sizeof(int32_t);
    DevMem sl;
    hipError_t e = upload(sl, slots, nullptr);
    if (e == hipSuccess) s = propagate_counts(plan, nullptr, 4);
    if (e == hipSuccess && s == UF_OK) e = plan->gather_tmp.ensure(bytes);
    if (e == hipSuccess && s == UF_OK)
        e = launch_gather_rows_u32(plan->counts.as<uint32_t>(), plan->cstride, sl.as<int32_t>(), nb, n,
                                   plan->gather_tmp.as<uint32_t>(), nullptr);
    if (e == hipSuccess && s == UF_OK) e = hipMemcpy(out_counts, plan->gather_tmp.p, bytes, hipMemcpyDeviceToHost);
    sl.release();
    uf_plan_destroy(plan);
    if (s != UF_OK) return s;
    if (e != hipSuccess) return hip_fail(ctx, e, "embedding counts");
    return UF_OK;
}

uf_status uf_plan_distance(uf_plan *plan, uf_method method, uf_precision prec,
                           const uf_tuning *tuning, uf_dtype out_dtype, void *out,
                           int32_t out_on_device, void *stream)
{
    if (!plan) return set_err(nullptr, UF_E_ARG, "plan must not be NULL");
    uf_context *ctx = plan->ctx;
    uf_status s = check_enums(ctx, method, prec);
    if (s != UF_OK) return s;
    if (out_dtype != UF_F64 && out_dtype != UF_F32) return set_err(ctx, UF_E_ARG, "unknown dtype");
    const HostPrep &hp = plan->hp;
    const int64_t n_pairs = (int64_t)hp.n_samples * (hp.n_samples - 1) / 2;
    if (n_pairs == 0) return UF_OK;
    if (!out) return set_err(ctx, UF_E_ARG, "out must not be NULL");
    if (!tuning) tuning = tuned_knobs(ctx, method, prec, hp.n_samples, hp.n_nodes);
    Knobs kn = resolve_knobs(tuning, prec, hp.n_nodes - 1);
    if (kn.den_mode != 0 && kn.den_mode != 1) return set_err(ctx, UF_E_ARG, "den_mode must be 0 or 1");
    if (kn.variant != 0 && kn.variant != 1) return set_err(ctx, UF_E_ARG, "variant must be 0 or 1");
    if (method == UF_WEIGHTED_UNNORMALIZED) kn.den_mode = 1;   // no denominator at all
    if (kn.tile < 0 || kn.tile > 2) return set_err(ctx, UF_E_ARG, "tile must be 0, 1 or 2");
    if (kn.k_split < 0 || kn.k_split > 64) return set_err(ctx, UF_E_ARG, "k_split must be in [0, 64]");
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t esz = out_dtype == UF_F32 ? sizeof(float) : sizeof(double);
    void *dst = out;
    if (!out_on_device) {
        UF_TRY(plan->out_tmp.ensure((size_t)n_pairs * esz), "allocating output staging");
        dst = plan->out_tmp.p;
    }
    if (prec == UF_PREC_MFMA_BF16X2) {
        s = run_mfma_unweighted(plan, kn.k_chunk, kn.variant, out_dtype == UF_F32, dst, st);
        if (s != UF_OK) return s;
    } else {
        StripeGeom g;
        s = run_striped(plan, method, prec, kn, &g, st);
        if (s != UF_OK) return s;
        UF_TRY(timed(plan, "condense", st, [&] {
                   return launch_condense(method, plan->num.as<double>(),
                                          kn.den_mode == 0 ? plan->den.as<double>() : nullptr,
                                          kn.den_mode == 0 ? nullptr : plan->D.as<double>(),
                                          g.sstride, g.n, g.S, out_dtype == UF_F32, dst, st);
               }), "condense");
    }
    if (!out_on_device)
        UF_TRY(hipMemcpyAsync(out, dst, (size_t)n_pairs * esz, hipMemcpyDeviceToHost, st),
               "copying distances out");
    UF_TRY(hipStreamSynchronize(st), "synchronizing");
    if (plan->prof.on) plan->prof.collect();
    return UF_OK;
}

// Checks and knobs shared by the stripe-range entry points.
static uf_status range_setup(uf_plan *plan, uf_method method, uf_precision prec, const uf_tuning *tuning,
                             int32_t s_begin, int32_t s_end, uf_dtype out_dtype, Knobs *kn)
{
    uf_context *ctx = plan->ctx;
    uf_status s = check_enums(ctx, method, prec);
    if (s != UF_OK) return s;
    if (prec == UF_PREC_MFMA_BF16X2)
        return set_err(ctx, UF_E_ARG, "stripe ranges exist for the striped precisions only");
    if (out_dtype != UF_F64 && out_dtype != UF_F32) return set_err(ctx, UF_E_ARG, "unknown dtype");
    const HostPrep &hp = plan->hp;
    if (s_begin < 0 || s_end > hp.n_samples / 2 || s_begin > s_end)
        return set_err(ctx, UF_E_ARG, "stripe range must satisfy 0 <= s_begin <= s_end <= n/2");
    if (!tuning) tuning = tuned_knobs(ctx, method, prec, hp.n_samples, hp.n_nodes);
    *kn = resolve_knobs(tuning, prec, hp.n_nodes - 1);
    if (kn->den_mode != 0 && kn->den_mode != 1) return set_err(ctx, UF_E_ARG, "den_mode must be 0 or 1");
    if (kn->tile < 0 || kn->tile > 2) return set_err(ctx, UF_E_ARG, "tile must be 0, 1 or 2");
    if (kn->k_split < 0 || kn->k_split > 64) return set_err(ctx, UF_E_ARG, "k_split must be in [0, 64]");
    kn->variant = 0;
    if (method == UF_WEIGHTED_UNNORMALIZED) kn->den_mode = 1;
    return UF_OK;
}

uf_status uf_plan_distance_stripes(uf_plan *plan, uf_method method, uf_precision prec,
                                   const uf_tuning *tuning, int32_t s_begin, int32_t s_end,
                                   uf_dtype out_dtype, void *out, int32_t out_on_device,
                                   void *stream)
{
    if (!plan) return set_err(nullptr, UF_E_ARG, "plan must not be NULL");
    uf_context *ctx = plan->ctx;
    Knobs kn;
    uf_status s = range_setup(plan, method, prec, tuning, s_begin, s_end, out_dtype, &kn);
    if (s != UF_OK) return s;
    if (s_begin == s_end) return UF_OK;
    if (!out) return set_err(ctx, UF_E_ARG, "out must not be NULL");
    const HostPrep &hp = plan->hp;
    const int32_t n = hp.n_samples;
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t esz = out_dtype == UF_F32 ? sizeof(float) : sizeof(double);
    // host output: the range's pairs are written compactly in condensed order on the
    // device, copied back once, and each row's (at most two) runs copied into place
    std::vector<int32_t> len_a, len_b;
    std::vector<int64_t> off;
    DevMem row_off;
    if (!out_on_device) {
        range_row_runs(n, s_begin, s_end, &len_a, &len_b, &off);
        UF_TRY(upload(row_off, off, st), "uploading row offsets");
        UF_TRY(plan->out_tmp.ensure((size_t)std::max<int64_t>(off[n], 1) * esz), "allocating output staging");
    }
    StripeGeom g;
    int32_t s_base = 0;
    s = run_striped(plan, method, prec, kn, &g, st, s_begin, s_end, &s_base);
    if (s != UF_OK) return s;
    UF_TRY(timed(plan, "condense", st, [&] {
               return launch_condense_range(method, plan->num.as<double>(),
                                            kn.den_mode == 0 ? plan->den.as<double>() : nullptr,
                                            kn.den_mode == 0 ? nullptr : plan->D.as<double>(), g.sstride, g.n,
                                            g.S, s_base, s_begin, s_end, out_dtype == UF_F32,
                                            out_on_device ? out : plan->out_tmp.p, st, out_on_device ? 0 : 2,
                                            out_on_device ? nullptr : row_off.as<int64_t>());
           }), "condense");
    if (!out_on_device) {
        std::vector<unsigned char> stage((size_t)off[n] * esz);
        if (off[n] > 0)
            UF_TRY(hipMemcpyAsync(stage.data(), plan->out_tmp.p, stage.size(), hipMemcpyDeviceToHost, st),
                   "copying distances out");
        UF_TRY(hipStreamSynchronize(st), "synchronizing");
        unsigned char *dst = static_cast<unsigned char *>(out);
        const int32_t S = n / 2, b_lo = std::max(n - s_end, S + 1);
        for (int32_t i = 0; i < n; ++i) {
            const int64_t row = (int64_t)n * i - (int64_t)i * (i + 1) / 2;   // condensed index of (i, i + 1)
            if (len_a[i] > 0)
                std::memcpy(dst + (size_t)(row + s_begin) * esz, stage.data() + (size_t)off[i] * esz,
                            (size_t)len_a[i] * esz);
            if (len_b[i] > 0)
                std::memcpy(dst + (size_t)(row + b_lo - 1) * esz,
                            stage.data() + (size_t)(off[i] + len_a[i]) * esz, (size_t)len_b[i] * esz);
        }
    }
    UF_TRY(hipStreamSynchronize(st), "synchronizing");
    if (plan->prof.on) plan->prof.collect();
    return UF_OK;
}

uf_status uf_plan_distance_block(uf_plan *plan, uf_method method, uf_precision prec,
                                 const uf_tuning *tuning, int32_t s_begin, int32_t s_end,
                                 uf_dtype out_dtype, void *out, int32_t out_on_device, void *stream)
{
    if (!plan) return set_err(nullptr, UF_E_ARG, "plan must not be NULL");
    uf_context *ctx = plan->ctx;
    Knobs kn;
    uf_status s = range_setup(plan, method, prec, tuning, s_begin, s_end, out_dtype, &kn);
    if (s != UF_OK) return s;
    const int32_t n = plan->hp.n_samples;
    if (s_begin == s_end || n < 2) return UF_OK;
    if (!out) return set_err(ctx, UF_E_ARG, "out must not be NULL");
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t bytes = (size_t)(s_end - s_begin) * n * (out_dtype == UF_F32 ? sizeof(float) : sizeof(double));
    void *dst = out;
    if (!out_on_device) {
        UF_TRY(plan->out_tmp.ensure(bytes), "allocating output staging");
        dst = plan->out_tmp.p;
    }
    StripeGeom g;
    int32_t s_base = 0;
    s = run_striped(plan, method, prec, kn, &g, st, s_begin, s_end, &s_base);
    if (s != UF_OK) return s;
    UF_TRY(timed(plan, "condense", st, [&] {
               return launch_condense_range(method, plan->num.as<double>(),
                                            kn.den_mode == 0 ? plan->den.as<double>() : nullptr,
                                            kn.den_mode == 0 ? nullptr : plan->D.as<double>(), g.sstride, g.n,
                                            g.S, s_base, s_begin, s_end, out_dtype == UF_F32, dst, st, 1);
           }), "condense");
    if (!out_on_device) UF_TRY(hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, st), "copying the block out");
    UF_TRY(hipStreamSynchronize(st), "synchronizing");
    if (plan->prof.on) plan->prof.collect();
    return UF_OK;
}

uf_status uf_merge_block(uf_context *ctx, int32_t n, int32_t s_begin, int32_t s_end, uf_dtype dtype,
                         const void *block, int32_t block_on_device, void *condensed, void *stream)
{
    if (!ctx) return set_err(nullptr, UF_E_ARG, "ctx must not be NULL");
    if (dtype != UF_F64 && dtype != UF_F32) return set_err(ctx, UF_E_ARG, "unknown dtype");
    if (n < 0 || s_begin < 0 || s_end > n / 2 || s_begin > s_end)
        return set_err(ctx, UF_E_ARG, "stripe range must satisfy 0 <= s_begin <= s_end <= n/2");
    if (s_begin == s_end || n < 2) return UF_OK;
    if (!block || !condensed) return set_err(ctx, UF_E_ARG, "block and condensed must not be NULL");
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t bytes = (size_t)(s_end - s_begin) * n * (dtype == UF_F32 ? sizeof(float) : sizeof(double));
    DevMem staged;
    const void *src = block;
    if (!block_on_device) {
        UF_TRY(staged.ensure(bytes), "allocating block staging");
        UF_TRY(hipMemcpyAsync(staged.p, block, bytes, hipMemcpyHostToDevice, st), "staging the block");
        src = staged.p;
    }
    UF_TRY(launch_merge_block(src, n, s_begin, s_end, dtype == UF_F32, condensed, st), "merging the block");
    UF_TRY(hipStreamSynchronize(st), "synchronizing");
    return UF_OK;
}

uf_status uf_plan_set_profiling(uf_plan *plan, int32_t enable)
{
    if (!plan) return set_err(nullptr, UF_E_ARG, "plan must not be NULL");
    (void)enter_device(plan->ctx->device);
    plan->prof.collect();
    plan->prof.totals.clear();
    plan->prof.on = enable != 0;
    return UF_OK;
}

uf_status uf_plan_get_profile(uf_plan *plan, uf_kernel_stat *out, int32_t cap, int32_t *n_out)
{
    if (!plan || !n_out || (cap > 0 && !out))
        return set_err(plan ? plan->ctx : nullptr, UF_E_ARG, "NULL argument");
    (void)enter_device(plan->ctx->device);
    plan->prof.collect();
    int32_t n = 0;
    for (const auto &kv : plan->prof.totals) {
        if (n >= cap) break;
        std::memset(out[n].name, 0, sizeof out[n].name);
        std::strncpy(out[n].name, kv.first.c_str(), sizeof out[n].name - 1);
        out[n].launches = kv.second.first;
        out[n].total_ms = kv.second.second;
        ++n;
    }
    *n_out = n;
    return UF_OK;
}

uf_status uf_plan_stripes(uf_plan *plan, uf_method method, uf_precision prec,
                          const uf_tuning *tuning, double *num, double *den, void *stream)
{
    if (!plan || !num || !den) return set_err(plan ? plan->ctx : nullptr, UF_E_ARG, "NULL argument");
    uf_context *ctx = plan->ctx;
    uf_status s = check_enums(ctx, method, prec);
    if (s != UF_OK) return s;
    if (prec == UF_PREC_MFMA_BF16X2)
        return set_err(ctx, UF_E_ARG, "stripes exist for the striped precisions only");
    const HostPrep &hp = plan->hp;
    Knobs kn = resolve_knobs(tuning, prec, hp.n_nodes - 1);
    if (kn.den_mode != 0) return set_err(ctx, UF_E_ARG, "stripes need den_mode 0");
    if (method == UF_WEIGHTED_UNNORMALIZED)
        return set_err(ctx, UF_E_ARG, "the unnormalized variant has no denominator stripes");
    if (hp.n_samples / 2 == 0) return UF_OK;
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    StripeGeom g;
    s = run_striped(plan, method, prec, kn, &g, st);
    if (s != UF_OK) return s;
    const size_t pitch = (size_t)g.sstride * sizeof(double);
    const size_t width = (size_t)hp.n_samples * sizeof(double);
    UF_TRY(hipMemcpy2DAsync(num, width, plan->num.p, pitch, width, g.S, hipMemcpyDeviceToHost, st),
           "copying numerator stripes");
    UF_TRY(hipMemcpy2DAsync(den, width, plan->den.p, pitch, width, g.S, hipMemcpyDeviceToHost, st),
           "copying denominator stripes");
    UF_TRY(hipStreamSynchronize(st), "synchronizing");
    return UF_OK;
}

uf_status uf_distance(uf_context *ctx, const uf_tree *tree, const uf_table *table,
                      uf_method method, uf_precision prec, uf_dtype out_dtype, void *out,
                      int32_t out_on_device, void *stream)
{
    uf_plan *plan = nullptr;
    uf_status s = uf_plan_create(ctx, tree, table, stream, &plan);
    if (s != UF_OK) return s;
    s = uf_plan_distance(plan, method, prec, nullptr, out_dtype, out, out_on_device, stream);
    uf_plan_destroy(plan);
    return s;
}

}  // extern "C"
