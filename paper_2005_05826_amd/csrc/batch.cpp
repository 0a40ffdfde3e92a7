// Batched execution of many independent UniFrac jobs of uneven size.
//
// Every job is validated and made resident like a single plan.  The batch then builds
// device tables so that the device work for all jobs is a short, fixed sequence of
// launches: one tip scatter and one gather per height level for all jobs together, one
// persistent queue-driven striped launch per precision, one persistent queue-driven MFMA
// launch for the matrix-core jobs, and per-job condense/normalize launches.  The queues are
// ordered largest job first, so idle work-groups always pick the most expensive remaining
// tile (a longest-processing-time-first schedule).  The whole sequence can be captured
// once into a HIP graph and replayed; it allocates nothing and uses fill kernels (not
// memset nodes) to clear counters and accumulators.
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>

#include "uf_runtime.h"

using namespace ufmi;

struct uf_batch {
    uf_context *ctx = nullptr;
    std::vector<uf_plan *> plans;
    std::vector<uf_job> jobs;
    int32_t emb_batch = 0, den_mode = 0, k_chunk = 4096, tile = 0, count_width = 0;
    int32_t mfma_variant = 0;             // uf_tuning.variant: matrix-core accumulation form
    int32_t n_groups = 512;   // persistent matrix-core work-groups (two per CU)
    int32_t n_cus = 256;
    // propagation tables
    DevMem prop_jobs, scatter_tasks, level_tasks;
    std::vector<int32_t> level_ptr;       // per height level, range of level_tasks
    std::vector<int32_t> level_max_vec;   // widest row (uint4 columns) of each level
    int32_t n_scatter = 0;
    // striped tables, one queue per (precision, method, count width):
    // q = 4 * (FP32) + 2 * (weighted) + (16-bit counts)
    static constexpr int kQueues = 8;
    DevMem stripe_jobs[kQueues], stripe_items[kQueues];
    int32_t n_stripe_items[kQueues] = {};
    // matrix-core tables
    DevMem mfma_jobs, mfma_items, mfma_tiles;
    int32_t n_mfma_items = 0;
    DevMem counters;                      // [0, kQueues) striped queues, [kQueues] MFMA queue
    // graph
    hipStream_t cap_stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Profiler prof;
};

namespace {

bool is_striped(const uf_job &j) { return j.prec == UF_PREC_FP64 || j.prec == UF_PREC_FP32; }

// Enqueue the whole batch on `st` (no allocation, no host synchronisation).
uf_status enqueue(uf_batch *b, hipStream_t st)
{
    uf_context *ctx = b->ctx;
    const int32_t nj = (int32_t)b->plans.size();
    // (a) propagation: clear tip rows, scatter every job's tips, gather level by level
    for (int32_t j = 0; j < nj; ++j) {
        uf_plan *p = b->plans[j];
        if (is_striped(b->jobs[j]))
            UF_TRY(launch_fill_u32(p->counts.p, 0u, (size_t)p->hp.n_leaf * p->cstride * p->cw / 4, st),
                   "clearing tips");
        else
            UF_TRY(launch_fill_u32(p->bits.p, 0u, (size_t)p->hp.n_leaf * p->bstride, st), "clearing tips");
    }
    UF_TRY(timed(b->prof, "propagate", st, [&] {
               hipError_t r = launch_scatter_batched(b->prop_jobs.as<PropJob>(),
                                                     b->scatter_tasks.as<int32_t>(), b->n_scatter, st);
               for (size_t h = 1; h + 1 < b->level_ptr.size() && r == hipSuccess; ++h) {
                   const int32_t t0 = b->level_ptr[h], t1 = b->level_ptr[h + 1];
                   r = launch_level_batched(b->prop_jobs.as<PropJob>(),
                                            b->level_tasks.as<int32_t>() + 2 * (size_t)t0, t1 - t0,
                                            b->level_max_vec[h], st);
               }
               return r;
           }), "batched propagation");

    // (b) striped jobs: clear state and queue counters, one persistent launch per queue
    UF_TRY(launch_fill_u32(b->counters.p, 0u, uf_batch::kQueues + 1, st), "clearing queue counters");
    for (int32_t j = 0; j < nj; ++j) {
        if (!is_striped(b->jobs[j])) continue;
        uf_plan *p = b->plans[j];
        const StripeGeom g = stripe_geometry(p->hp.n_samples, b->jobs[j].prec == UF_PREC_FP64, b->den_mode, b->tile);
        const size_t words = (size_t)g.spad * g.sstride * 2;
        UF_TRY(launch_fill_u32(p->num.p, 0u, words, st), "clearing stripes");
        if (b->den_mode == 0) UF_TRY(launch_fill_u32(p->den.p, 0u, words, st), "clearing stripes");
        UF_TRY(launch_inv_totals(p->totals.as<int32_t>(), p->hp.n_samples, p->inv_t.as<double>(), st),
               "reciprocal totals");
    }
    for (int q = 0; q < uf_batch::kQueues; ++q) {
        if (b->n_stripe_items[q] == 0) continue;
        // as many persistent work-groups as the tile shape keeps resident (2 or 3 per CU)
        const int32_t groups = b->n_cus * stripe_geometry(256, (q & 4) == 0, b->den_mode, b->tile).occ;
        UF_TRY(timed(b->prof, "stripe", st, [&] {
                   return launch_stripe_queue((q & 4) == 0, (q & 2) ? UF_WEIGHTED_NORMALIZED : UF_UNWEIGHTED,
                                              (q & 1) ? 2 : 4, b->den_mode, b->tile,
                                              b->stripe_jobs[q].as<StripeArgs>(),
                                              b->stripe_items[q].as<int32_t>(), b->n_stripe_items[q],
                                              b->counters.as<int32_t>() + q,
                                              std::min(groups, b->n_stripe_items[q]), st);
               }), "queued striped accumulation");
    }
    for (int32_t j = 0; j < nj; ++j) {
        if (!is_striped(b->jobs[j])) continue;
        uf_plan *p = b->plans[j];
        const uf_job &J = b->jobs[j];
        const StripeGeom g = stripe_geometry(p->hp.n_samples, J.prec == UF_PREC_FP64, b->den_mode, b->tile);
        if (b->den_mode != 0 && J.method != UF_WEIGHTED_UNNORMALIZED)
            UF_TRY(launch_rowdot(J.method, p->counts.p, p->cw, p->cstride, 0, p->hp.n_nodes - 1,
                                 p->totals.as<int32_t>(), p->len_slot.as<double>(), g.n,
                                 p->D.as<double>(), true, p->rowdot_part.as<double>(), st),
                   "per-sample sums");
        UF_TRY(timed(b->prof, "condense", st, [&] {
                   return launch_condense(J.method, p->num.as<double>(),
                                          b->den_mode == 0 ? p->den.as<double>() : nullptr,
                                          b->den_mode == 0 ? nullptr : p->D.as<double>(), g.sstride,
                                          g.n, g.S, J.out_dtype == UF_F32, J.out, st);
               }), "condense");
    }

    // (c) matrix-core jobs: presence bits, one persistent MFMA launch, normalize
    if (b->n_mfma_items > 0) {
        for (int32_t j = 0; j < nj; ++j) {
            if (is_striped(b->jobs[j])) continue;
            uf_plan *p = b->plans[j];
            const MfmaGeom g = mfma_geometry(p->hp.n_samples, p->hp.n_nodes - 1);
            uint16_t *hi = p->mfma_scratch[1].as<uint16_t>(), *lo = hi + g.k_pad;
            UF_TRY(timed(b->prof, "bits_transpose", st, [&] {
                       hipError_t r = launch_split_lengths(p->len_slot.as<double>(), g.B, g.k_pad, hi, lo, st);
                       if (r == hipSuccess)
                           r = launch_bits_transpose(p->bits.as<uint32_t>(), p->bstride, g,
                                                    p->mfma_scratch[0].as<uint8_t>(), st);
                       return r;
                   }), "presence transpose");
        }
        UF_TRY(timed(b->prof, "mfma", st, [&] {
                   return launch_mfma_queue(b->mfma_jobs.as<MfmaArgs>(), b->mfma_items.as<int32_t>(),
                                            b->n_mfma_items, b->counters.as<int32_t>() + uf_batch::kQueues,
                                            std::min(b->mfma_variant == 1 ? b->n_groups / 2 : b->n_groups,
                                                     b->n_mfma_items),
                                            b->mfma_variant, st);
               }), "queued matrix-core product");
        for (int32_t j = 0; j < nj; ++j) {
            if (is_striped(b->jobs[j])) continue;
            uf_plan *p = b->plans[j];
            const uf_job &J = b->jobs[j];
            const MfmaGeom g = mfma_geometry(p->hp.n_samples, p->hp.n_nodes - 1);
            double *T = p->mfma_scratch[3].as<double>();
            double *S = J.out_dtype == UF_F64 ? static_cast<double *>(J.out) : T + g.n_pad;
            UF_TRY(timed(b->prof, "normalize", st, [&] {
                       return launch_mfma_normalize(S, T, g.n, J.out_dtype == UF_F32, J.out, st);
                   }), "normalize");
        }
    }
    return UF_OK;
}

uf_status build_tables(uf_batch *b, hipStream_t st)
{
    uf_context *ctx = b->ctx;
    const int32_t nj = (int32_t)b->plans.size();
    int dev_cus = 256;
    (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    b->n_cus = std::max(dev_cus, 1);
    b->n_groups = 2 * b->n_cus;

    // propagation tables and per-job scratch
    std::vector<PropJob> pj(nj);
    std::vector<int32_t> scatter;
    int32_t max_levels = 1;
    for (int32_t j = 0; j < nj; ++j) max_levels = std::max(max_levels, b->plans[j]->hp.n_levels);
    std::vector<std::vector<int32_t>> lv(max_levels);
    b->level_max_vec.assign(max_levels, 0);
    for (int32_t j = 0; j < nj; ++j) {
        uf_plan *p = b->plans[j];
        const HostPrep &hp = p->hp;
        const bool striped = is_striped(b->jobs[j]);
        if (striped) {
            p->cw = resolve_count_width(hp, b->count_width);
            if (p->cw < 0) return set_err(ctx, UF_E_ARG, "16-bit counts need every sample total <= 65535");
            UF_TRY(p->counts.ensure((size_t)hp.n_nodes * p->cstride * p->cw), "allocating counts");
        } else
            UF_TRY(p->bits.ensure((size_t)hp.n_nodes * p->bstride * sizeof(uint32_t)), "allocating bits");
        PropJob &J = pj[j];
        J.X = striped ? p->counts.as<uint32_t>() : p->bits.as<uint32_t>();
        J.stride = striped ? p->cstride * p->cw / 4 : p->bstride;
        J.child_ptr = p->child_ptr.as<int32_t>();
        J.child_slot = p->child_slot.as<int32_t>();
        J.indptr = p->indptr.as<int64_t>();
        J.entry_slot = p->entry_slot.as<int32_t>();
        J.entry_count = p->entry_count.as<int32_t>();
        J.n_leaf = hp.n_leaf;
        J.mode = striped ? (p->cw == 2 ? 2 : 0) : 1;
        J.n_samples = hp.n_samples;
        J.pad = 0;
        for (int32_t k = 0; k < hp.n_samples; ++k) {
            scatter.push_back(j);
            scatter.push_back(k);
        }
        for (int32_t h = 1; h < hp.n_levels; ++h) {
            for (int32_t s = hp.level_ptr[h]; s < hp.level_ptr[h + 1]; ++s) {
                lv[h].push_back(j);
                lv[h].push_back(s);
            }
            b->level_max_vec[h] = std::max<int32_t>(b->level_max_vec[h], (int32_t)(J.stride / 4));
        }
    }
    std::vector<int32_t> levels;
    b->level_ptr.assign(max_levels + 1, 0);
    for (int32_t h = 0; h < max_levels; ++h) {
        b->level_ptr[h] = (int32_t)(levels.size() / 2);
        levels.insert(levels.end(), lv[h].begin(), lv[h].end());
    }
    b->level_ptr[max_levels] = (int32_t)(levels.size() / 2);
    b->n_scatter = (int32_t)(scatter.size() / 2);
    UF_TRY(upload(b->prop_jobs, pj, st), "uploading job table");
    UF_TRY(upload(b->scatter_tasks, scatter, st), "uploading scatter tasks");
    UF_TRY(upload(b->level_tasks, levels, st), "uploading level tasks");

    // striped tables, jobs ordered by branch count (largest first)
    std::vector<int32_t> order(nj);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return b->plans[x]->hp.n_nodes > b->plans[y]->hp.n_nodes;
    });
    for (int q = 0; q < uf_batch::kQueues; ++q) {
        const bool fp64 = (q & 4) == 0;
        std::vector<StripeArgs> sj;
        std::vector<int32_t> items;
        for (int32_t j : order) {
            const uf_job &J = b->jobs[j];
            if (!is_striped(J) || (J.prec == UF_PREC_FP64) != fp64) continue;
            // the unnormalized variant runs the weighted-normalized numerator
            const int32_t km = J.method == UF_WEIGHTED_UNNORMALIZED ? UF_WEIGHTED_NORMALIZED : J.method;
            uf_plan *p = b->plans[j];
            if ((km == UF_WEIGHTED_NORMALIZED) != ((q & 2) != 0) || (p->cw == 2) != ((q & 1) != 0)) continue;
            const HostPrep &hp = p->hp;
            const StripeGeom g = stripe_geometry(hp.n_samples, fp64, b->den_mode, b->tile);
            const size_t state = (size_t)g.spad * g.sstride * sizeof(double);
            UF_TRY(p->num.ensure(state), "allocating stripes");
            if (b->den_mode == 0) UF_TRY(p->den.ensure(state), "allocating stripes");
            UF_TRY(p->D.ensure((size_t)hp.n_samples * sizeof(double)), "allocating sums");
            if (b->den_mode != 0)
                UF_TRY(p->rowdot_part.ensure(rowdot_scratch_elems(hp.n_samples, hp.n_nodes - 1) * sizeof(double)),
                       "allocating sum scratch");
            UF_TRY(p->inv_t.ensure((size_t)hp.n_samples * sizeof(double)), "allocating totals");
            int32_t E = b->emb_batch > 0 ? b->emb_batch : (fp64 ? 1024 : 128);
            E = std::max(1, std::min(E, std::max(1, hp.n_nodes - 1)));
            const int32_t idx = (int32_t)sj.size();
            sj.push_back(make_stripe_args(km, p->counts.p, p->cw, p->cstride,
                                          p->inv_t.as<double>(), p->len_slot.as<double>(),
                                          hp.n_nodes - 1, E, p->num.as<double>(),
                                          b->den_mode == 0 ? p->den.as<double>() : nullptr, g));
            if (hp.n_nodes - 1 <= 0 || g.S == 0) continue;  // nothing to accumulate
            const int32_t n_tiles = sj.back().tiles_k * sj.back().tiles_s;
            for (int32_t t = 0; t < n_tiles; ++t) {
                items.push_back(idx);
                items.push_back(t);
            }
        }
        b->n_stripe_items[q] = (int32_t)(items.size() / 2);
        UF_TRY(upload(b->stripe_jobs[q], sj, st), "uploading striped jobs");
        UF_TRY(upload(b->stripe_items[q], items, st), "uploading striped items");
    }

    // matrix-core tables
    std::vector<MfmaArgs> mj;
    std::vector<int32_t> mitems, tiles_all;
    std::vector<std::pair<int32_t, size_t>> tile_off;   // (job, offset into tiles_all)
    std::vector<int32_t> morder;
    for (int32_t j : order)
        if (!is_striped(b->jobs[j])) morder.push_back(j);
    for (int32_t j : morder) {
        std::vector<int32_t> xy;
        mfma_tile_list(b->plans[j]->hp.n_samples, &xy);
        tile_off.push_back({j, tiles_all.size()});
        tiles_all.insert(tiles_all.end(), xy.begin(), xy.end());
    }
    UF_TRY(upload(b->mfma_tiles, tiles_all, st), "uploading tile lists");
    for (size_t m = 0; m < morder.size(); ++m) {
        const int32_t j = morder[m];
        uf_plan *p = b->plans[j];
        const uf_job &J = b->jobs[j];
        const MfmaGeom g = mfma_geometry(p->hp.n_samples, p->hp.n_nodes - 1);
        const int64_t n_pairs = (int64_t)g.n * (g.n - 1) / 2;
        UF_TRY(p->bits.ensure((size_t)p->hp.n_nodes * p->bstride * sizeof(uint32_t)), "allocating bits");
        UF_TRY(p->mfma_scratch[0].ensure((size_t)g.n_pad * (g.k_pad / 8)), "allocating presence bits");
        UF_TRY(p->mfma_scratch[1].ensure((size_t)2 * g.k_pad * sizeof(uint16_t)), "allocating splits");
        const bool s_in_out = J.out_dtype == UF_F64;
        UF_TRY(p->mfma_scratch[3].ensure((size_t)g.n_pad * sizeof(double) +
                                         (s_in_out ? 0 : (size_t)n_pairs * sizeof(double))),
               "allocating shared lengths");
        double *T = p->mfma_scratch[3].as<double>();
        double *S = s_in_out ? static_cast<double *>(J.out) : T + g.n_pad;
        uint16_t *hi = p->mfma_scratch[1].as<uint16_t>();
        mj.push_back(make_mfma_args(p->mfma_scratch[0].as<uint8_t>(), hi, hi + g.k_pad, b->k_chunk,
                                    b->mfma_tiles.as<int32_t>() + tile_off[m].second, g, S, T));
        for (int32_t t = 0; t < g.n_tiles; ++t) {
            mitems.push_back((int32_t)m);
            mitems.push_back(t);
        }
    }
    b->n_mfma_items = (int32_t)(mitems.size() / 2);
    UF_TRY(upload(b->mfma_jobs, mj, st), "uploading matrix-core jobs");
    UF_TRY(upload(b->mfma_items, mitems, st), "uploading matrix-core items");
    UF_TRY(b->counters.ensure((uf_batch::kQueues + 1) * sizeof(int32_t)), "allocating counters");
    UF_TRY(hipStreamSynchronize(st), "synchronizing");
    return UF_OK;
}

void destroy_graph(uf_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

}  // namespace

extern "C" {

uf_status uf_batch_create(uf_context *ctx, const uf_job *jobs, int32_t n_jobs,
                          const uf_tuning *tuning, void *stream, uf_batch **out)
{
    if (!ctx || !out || (n_jobs > 0 && !jobs) || n_jobs < 0)
        return set_err(ctx, UF_E_ARG, "invalid batch arguments");
    *out = nullptr;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const uf_job &J = jobs[j];
        if (J.method != UF_UNWEIGHTED && J.method != UF_WEIGHTED_NORMALIZED &&
            J.method != UF_WEIGHTED_UNNORMALIZED)
            return set_err(ctx, UF_E_ARG, "job has an unknown method");
        if (J.prec != UF_PREC_FP64 && J.prec != UF_PREC_FP32 && J.prec != UF_PREC_MFMA_BF16X2)
            return set_err(ctx, UF_E_ARG, "job has an unknown precision");
        if (J.prec == UF_PREC_MFMA_BF16X2 && J.method != UF_UNWEIGHTED)
            return set_err(ctx, UF_E_UNSUPPORTED, "matrix-core jobs must be unweighted");
        if (J.out_dtype != UF_F64 && J.out_dtype != UF_F32)
            return set_err(ctx, UF_E_ARG, "job has an unknown output dtype");
        if (!J.out && J.table.n_samples > 1) return set_err(ctx, UF_E_ARG, "job output is NULL");
    }
    uf_batch *b = new (std::nothrow) uf_batch;
    if (!b) return set_err(ctx, UF_E_OOM, "host allocation failed");
    b->ctx = ctx;
    b->tile = 2;   // without knobs, the fastest measured shape for den_mode 0
    if (tuning) {
        b->emb_batch = tuning->emb_batch;
        b->den_mode = tuning->den_mode;
        b->tile = tuning->tile;
        b->count_width = tuning->count_width;
        b->mfma_variant = tuning->variant;
        if (tuning->k_chunk > 0) b->k_chunk = tuning->k_chunk;
    }
    if ((b->den_mode != 0 && b->den_mode != 1) || (b->tile < 0 || b->tile > 2) ||
        (b->mfma_variant != 0 && b->mfma_variant != 1)) {
        delete b;
        return set_err(ctx, UF_E_ARG, "den_mode and variant must be 0 or 1, tile 0, 1 or 2");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    b->jobs.assign(jobs, jobs + n_jobs);
    for (int32_t j = 0; j < n_jobs; ++j) {
        uf_plan *p = nullptr;
        uf_status s = plan_prepare(ctx, &jobs[j].tree, &jobs[j].table, st, &p);
        if (s != UF_OK) {
            std::string msg = "job " + std::to_string(j) + ": " + ctx->err;
            uf_batch_destroy(b);
            return set_err(ctx, s, msg);
        }
        b->plans.push_back(p);
    }
    uf_status s = build_tables(b, st);
    if (s != UF_OK) {
        uf_batch_destroy(b);
        return s;
    }
    *out = b;
    return UF_OK;
}

uf_status uf_batch_run(uf_batch *b, void *stream)
{
    if (!b) return set_err(nullptr, UF_E_ARG, "batch must not be NULL");
    uf_context *ctx = b->ctx;
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (b->exec) {
        // the graph runs on the batch's own stream, ordered after the caller's stream work
        // and before anything the caller enqueues next
        hipStream_t gs = b->cap_stream;
        UF_TRY(hipEventRecord(b->ev_in, st), "recording order event");
        UF_TRY(hipStreamWaitEvent(gs, b->ev_in, 0), "ordering graph launch");
        UF_TRY(timed(b->prof, "graph", gs, [&] { return hipGraphLaunch(b->exec, gs); }), "graph launch");
        UF_TRY(hipEventRecord(b->ev_out, gs), "recording completion event");
        UF_TRY(hipStreamWaitEvent(st, b->ev_out, 0), "ordering caller stream");
        UF_TRY(hipStreamSynchronize(gs), "synchronizing");
    } else {
        uf_status s = enqueue(b, st);
        if (s != UF_OK) return s;
    }
    UF_TRY(hipStreamSynchronize(st), "synchronizing");
    if (b->prof.on) b->prof.collect();
    return UF_OK;
}

uf_status uf_batch_capture(uf_batch *b)
{
    if (!b) return set_err(nullptr, UF_E_ARG, "batch must not be NULL");
    uf_context *ctx = b->ctx;
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    destroy_graph(b);
    if (!b->cap_stream)
        UF_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "creating capture stream");
    if (!b->ev_in) UF_TRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming), "creating event");
    if (!b->ev_out) UF_TRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming), "creating event");
    const bool prof_on = b->prof.on;
    b->prof.on = false;   // no timing events inside the graph
    UF_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    uf_status s = enqueue(b, b->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    b->prof.on = prof_on;
    if (s != UF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "end capture");
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        destroy_graph(b);
        return hip_fail(ctx, e, "graph instantiate");
    }
    return UF_OK;
}

uf_status uf_batch_set_profiling(uf_batch *b, int32_t enable)
{
    if (!b) return set_err(nullptr, UF_E_ARG, "batch must not be NULL");
    b->prof.collect();
    b->prof.totals.clear();
    b->prof.on = enable != 0;
    return UF_OK;
}

uf_status uf_batch_get_profile(uf_batch *b, uf_kernel_stat *out, int32_t cap, int32_t *n_out)
{
    if (!b || !n_out || (cap > 0 && !out)) return set_err(b ? b->ctx : nullptr, UF_E_ARG, "NULL argument");
    b->prof.collect();
    int32_t n = 0;
    for (const auto &kv : b->prof.totals) {
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

void uf_batch_destroy(uf_batch *b)
{
    if (!b) return;
    (void)enter_device(b->ctx->device);
    destroy_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    for (uf_plan *p : b->plans) uf_plan_destroy(p);
    for (int q = 0; q < uf_batch::kQueues; ++q) {
        b->stripe_jobs[q].release();
        b->stripe_items[q].release();
    }
    for (DevMem *m : {&b->prop_jobs, &b->scatter_tasks, &b->level_tasks, &b->mfma_jobs,
                      &b->mfma_items, &b->mfma_tiles, &b->counters})
        m->release();
    b->prof.release();
    delete b;
}

uf_status uf_distance_batch(uf_context *ctx, const uf_job *jobs, int32_t n_jobs, void *stream)
{
    uf_batch *b = nullptr;
    uf_status s = uf_batch_create(ctx, jobs, n_jobs, nullptr, stream, &b);
    if (s != UF_OK) return s;
    s = uf_batch_run(b, stream);
    uf_batch_destroy(b);
    return s;
}

}  // extern "C"
