// Batched execution of many independent UniFrac jobs of uneven size.
//
// Every job is validated and made resident like a single plan.  The batch then builds
// device tables so that the device work for all jobs is a short, fixed sequence of
// launches: one tip scatter and one gather per height level for all jobs together, one
// persistent queue-driven striped launch per kernel form (precision, method, count width,
// denominator mode, tile shape), one persistent queue-driven MFMA launch per accumulation
// variant on a second stream beside them, and per-job condense/normalize launches.  Every
// job carries its own knobs (batch depth, MFMA chunk, branch splits), so one batch can mix
// tunings; a batch too small to fill the device splits its jobs' branches as single plans do.  The
// queues are ordered largest job first, so idle work-groups always pick the most expensive
// remaining tile (a longest-processing-time-first schedule).  The whole sequence can be captured
// once into a HIP graph and replayed; it allocates nothing and uses fill kernels (not
// memset nodes) to clear counters and accumulators.
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>

#include "uf_runtime.h"

using namespace ufmi;

// Knobs of one job: from the batch's tuning, else from the context's tune cache, else the
// library defaults.
struct JobKnobs {
    int32_t E, den_mode, tile, count_width, k_chunk, variant;
    int32_t k_split;   // striped branch splits: 0 automatic, else at most this many
    int32_t e_free;    // 1: E is the FP64 default and may shrink for branch splits
};

struct uf_batch {
    uf_context *ctx = nullptr;
    std::vector<uf_plan *> plans;
    std::vector<uf_job> jobs;
    std::vector<JobKnobs> knobs;
    std::vector<int32_t> kz;              // branch splits of every striped job (state copies)
    std::vector<void *> dev_out;          // device output of every job (its own or staging)
    int32_t n_cus = 256;
    // propagation tables
    DevMem prop_jobs, scatter_tasks, level_tasks;
    std::vector<int32_t> level_ptr;       // per height level, range of level_tasks
    std::vector<int32_t> level_max_vec;   // widest row (uint4 columns) of each level
    int32_t n_scatter = 0;
    // striped queues, one per kernel instantiation:
    // q = ((FP32 * 2 + weighted) * 2 + 16-bit counts) * 6 + den_mode * 3 + tile
    static constexpr int kQueues = 48;
    DevMem stripe_jobs[kQueues], stripe_items[kQueues];
    int32_t n_stripe_items[kQueues] = {};
    // matrix-core queues, one per accumulation variant
    DevMem mfma_jobs[2], mfma_items[2], mfma_tiles;
    int32_t n_mfma_items[2] = {};
    DevMem counters;                      // [0, kQueues) striped, then the two matrix-core queues
    // the matrix-core queue runs on a second stream beside the striped queues
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // graph
    hipStream_t cap_stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Profiler prof;
};

namespace {

bool is_striped(const uf_job &j) { return j.prec == UF_PREC_FP64 || j.prec == UF_PREC_FP32; }

int queue_of(bool fp32, bool weighted, bool c16, int32_t den_mode, int32_t tile)
{
    return ((((fp32 ? 1 : 0) * 2 + (weighted ? 1 : 0)) * 2 + (c16 ? 1 : 0)) * 6) + den_mode * 3 + tile;
}

// Enqueue the whole batch on `st` (no allocation, no host synchronisation).  The matrix-core
// jobs run on the batch's second stream, forked from and joined back into `st` with events,
// so that their persistent queue fills the device when the striped queues drain.
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
    UF_TRY(launch_fill_u32(b->counters.p, 0u, uf_batch::kQueues + 2, st), "clearing queue counters");

    // (c) matrix-core jobs on the second stream: presence bits, persistent MFMA queues,
    // normalize
    const bool has_mfma = b->n_mfma_items[0] + b->n_mfma_items[1] > 0;
    if (has_mfma) {
        hipStream_t ss = b->side;
        UF_TRY(hipEventRecord(b->ev_fork, st), "forking the matrix-core stream");
        UF_TRY(hipStreamWaitEvent(ss, b->ev_fork, 0), "forking the matrix-core stream");
        for (int32_t j = 0; j < nj; ++j) {
            if (is_striped(b->jobs[j])) continue;
            uf_plan *p = b->plans[j];
            const MfmaGeom g = mfma_geometry(p->hp.n_samples, p->hp.n_nodes - 1);
            uint16_t *hi = p->mfma_scratch[1].as<uint16_t>(), *lo = hi + g.k_pad;
            UF_TRY(timed(b->prof, "bits_transpose", ss, [&] {
                       hipError_t r = launch_split_lengths(p->len_slot.as<double>(), g.B, g.k_pad, hi, lo, ss);
                       if (r == hipSuccess)
                           r = launch_bits_transpose(p->bits.as<uint32_t>(), p->bstride, g,
                                                    p->mfma_scratch[0].as<uint8_t>(), ss);
                       return r;
                   }), "presence transpose");
        }
        for (int v = 0; v < 2; ++v) {
            if (b->n_mfma_items[v] == 0) continue;
            // persistent work-groups: two per CU (variant 0) or one (variant 1)
            const int32_t groups = std::min(b->n_cus * (v == 1 ? 1 : 2), b->n_mfma_items[v]);
            UF_TRY(timed(b->prof, "mfma", ss, [&] {
                       return launch_mfma_queue(b->mfma_jobs[v].as<MfmaArgs>(), b->mfma_items[v].as<int32_t>(),
                                                b->n_mfma_items[v],
                                                b->counters.as<int32_t>() + uf_batch::kQueues + v, groups, v, ss);
                   }), "queued matrix-core product");
        }
        for (int32_t j = 0; j < nj; ++j) {
            if (is_striped(b->jobs[j])) continue;
            uf_plan *p = b->plans[j];
            const uf_job &J = b->jobs[j];
            const MfmaGeom g = mfma_geometry(p->hp.n_samples, p->hp.n_nodes - 1);
            double *T = p->mfma_scratch[3].as<double>();
            double *S = J.out_dtype == UF_F64 ? static_cast<double *>(b->dev_out[j]) : T + g.n_pad;
            UF_TRY(timed(b->prof, "normalize", ss, [&] {
                       return launch_mfma_normalize(S, T, g.n, J.out_dtype == UF_F32, b->dev_out[j], ss);
                   }), "normalize");
        }
        UF_TRY(hipEventRecord(b->ev_join, ss), "joining the matrix-core stream");
    }

    // (b) striped jobs: clear state, one persistent launch per queue, then condense
    for (int32_t j = 0; j < nj; ++j) {
        if (!is_striped(b->jobs[j])) continue;
        uf_plan *p = b->plans[j];
        const JobKnobs &K = b->knobs[j];
        const StripeGeom g = stripe_geometry(p->hp.n_samples, b->jobs[j].prec == UF_PREC_FP64, K.den_mode, K.tile);
        // a job with branches needs no clearing: the first batch of each of its splits writes
        // that split's state copy; a single-node tree's zero state is cleared here
        if (p->hp.n_nodes - 1 <= 0) {
            const size_t words = (size_t)g.spad * g.sstride * 2;
            UF_TRY(launch_fill_u32(p->num.p, 0u, words, st), "clearing stripes");
            if (K.den_mode == 0) UF_TRY(launch_fill_u32(p->den.p, 0u, words, st), "clearing stripes");
        }
        UF_TRY(launch_inv_totals(p->totals.as<int32_t>(), p->hp.n_samples, p->inv_t.as<double>(), st),
               "reciprocal totals");
    }
    for (int q = 0; q < uf_batch::kQueues; ++q) {
        if (b->n_stripe_items[q] == 0) continue;
        const int32_t tile = q % 3, den_mode = (q / 3) % 2, c16 = (q / 6) % 2, wn = (q / 12) % 2;
        const bool fp64 = q < 24;
        // as many persistent work-groups as the tile shape keeps resident (2 to 4 per CU)
        const int32_t groups = b->n_cus * stripe_geometry(256, fp64, den_mode, tile).occ;
        UF_TRY(timed(b->prof, "stripe", st, [&] {
                   return launch_stripe_queue(fp64, wn ? UF_WEIGHTED_NORMALIZED : UF_UNWEIGHTED,
                                              c16 ? 2 : 4, den_mode, tile,
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
        const JobKnobs &K = b->knobs[j];
        const StripeGeom g = stripe_geometry(p->hp.n_samples, J.prec == UF_PREC_FP64, K.den_mode, K.tile);
        if (b->kz[j] > 1) {   // the branch splits' state copies, summed in split order
            const int64_t cnt = (int64_t)g.spad * g.sstride;
            UF_TRY(timed(b->prof, "reduce", st, [&] {
                       hipError_t r = launch_reduce_z(p->num.as<double>(), cnt, b->kz[j], cnt, st);
                       if (r == hipSuccess && K.den_mode == 0)
                           r = launch_reduce_z(p->den.as<double>(), cnt, b->kz[j], cnt, st);
                       return r;
                   }), "summing branch splits");
        }
        if (K.den_mode != 0 && J.method != UF_WEIGHTED_UNNORMALIZED)
            UF_TRY(launch_rowdot(J.method, p->counts.p, p->cw, p->cstride, 0, p->hp.n_nodes - 1,
                                 p->totals.as<int32_t>(), p->len_slot.as<double>(), g.n,
                                 p->D.as<double>(), true, p->rowdot_part.as<double>(), st),
                   "per-sample sums");
        UF_TRY(timed(b->prof, "condense", st, [&] {
                   return launch_condense(J.method, p->num.as<double>(),
                                          K.den_mode == 0 ? p->den.as<double>() : nullptr,
                                          K.den_mode == 0 ? nullptr : p->D.as<double>(), g.sstride,
                                          g.n, g.S, J.out_dtype == UF_F32, b->dev_out[j], st);
               }), "condense");
    }
    if (has_mfma) UF_TRY(hipStreamWaitEvent(st, b->ev_join, 0), "joining the matrix-core stream");
    return UF_OK;
}

uf_status build_tables(uf_batch *b, hipStream_t st)
{
    uf_context *ctx = b->ctx;
    const int32_t nj = (int32_t)b->plans.size();
    int dev_cus = 256;
    (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    b->n_cus = std::max(dev_cus, 1);

    // outputs: the job's device pointer, or a staging buffer for a host output
    b->dev_out.assign(nj, nullptr);
    for (int32_t j = 0; j < nj; ++j) {
        const uf_job &J = b->jobs[j];
        uf_plan *p = b->plans[j];
        const int64_t n_pairs = (int64_t)p->hp.n_samples * (p->hp.n_samples - 1) / 2;
        if (J.out_on_device) {
            b->dev_out[j] = J.out;
        } else if (n_pairs > 0) {
            UF_TRY(p->out_tmp.ensure((size_t)n_pairs * (J.out_dtype == UF_F32 ? 4 : 8)), "allocating output staging");
            b->dev_out[j] = p->out_tmp.p;
        }
    }

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
            p->cw = resolve_count_width(hp, b->knobs[j].count_width);
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
    std::vector<std::vector<StripeArgs>> sj(uf_batch::kQueues);
    std::vector<std::vector<int32_t>> items(uf_batch::kQueues);
    // Branch splits: a tuning's k_split, else the single plan's automatic rule while all the
    // batch's stripe tiles come to fewer than ten rounds of the device (a job then gets the
    // splits and batch depth, and so the results, it gets when run alone); none once the
    // tiles fill the device by themselves, or when the automatic splits' extra state copies
    // would pass kSplitStateBudget over the whole batch (many small jobs).
    constexpr size_t kSplitStateBudget = (size_t)16 << 30;
    double rounds = 0.0;
    for (int32_t j = 0; j < nj; ++j) {
        if (!is_striped(b->jobs[j])) continue;
        const StripeGeom g = stripe_geometry(b->plans[j]->hp.n_samples, b->jobs[j].prec == UF_PREC_FP64,
                                             b->knobs[j].den_mode, b->knobs[j].tile);
        rounds += (double)(g.sstride / g.tkw) * (g.spad / g.tsw) / ((double)b->n_cus * std::max(g.occ, 1));
    }
    const bool device_full = rounds >= 10.0;
    b->kz.assign(nj, 1);
    std::vector<int32_t> job_E(nj, 1);
    size_t auto_extra = 0;
    for (int32_t j = 0; j < nj; ++j) {
        if (!is_striped(b->jobs[j])) continue;
        const JobKnobs &K = b->knobs[j];
        uf_plan *p = b->plans[j];
        const StripeGeom g = stripe_geometry(p->hp.n_samples, b->jobs[j].prec == UF_PREC_FP64, K.den_mode, K.tile);
        const size_t state = (size_t)g.spad * g.sstride * sizeof(double);
        job_E[j] = std::max(1, std::min({K.E, 4096, std::max(1, p->hp.n_nodes - 1)}));
        if (K.k_split > 0 || !device_full) {
            Knobs kn{};
            kn.emb_batch = job_E[j];
            kn.k_chunk = K.k_chunk;
            kn.den_mode = K.den_mode;
            kn.variant = 0;   // the queues always run the fused form
            kn.tile = K.tile;
            kn.count_width = K.count_width;
            kn.k_split = K.k_split;
            kn.e_free = K.e_free;
            b->kz[j] = striped_k_split(p, kn, g, state);
            job_E[j] = kn.emb_batch;   // the rule may shrink an FP64 default batch depth
            if (K.k_split == 0) auto_extra += (size_t)(b->kz[j] - 1) * state * (K.den_mode == 0 ? 2 : 1);
        }
    }
    if (auto_extra > kSplitStateBudget)
        for (int32_t j = 0; j < nj; ++j)
            if (is_striped(b->jobs[j]) && b->knobs[j].k_split == 0) {
                b->kz[j] = 1;
                job_E[j] = std::max(1, std::min({b->knobs[j].E, 4096, std::max(1, b->plans[j]->hp.n_nodes - 1)}));
            }
    for (int32_t j : order) {
        const uf_job &J = b->jobs[j];
        if (!is_striped(J)) continue;
        const JobKnobs &K = b->knobs[j];
        const bool fp64 = J.prec == UF_PREC_FP64;
        // the unnormalized variant runs the weighted-normalized numerator
        const int32_t km = J.method == UF_WEIGHTED_UNNORMALIZED ? UF_WEIGHTED_NORMALIZED : J.method;
        uf_plan *p = b->plans[j];
        const HostPrep &hp = p->hp;
        const int q = queue_of(!fp64, km == UF_WEIGHTED_NORMALIZED, p->cw == 2, K.den_mode, K.tile);
        const StripeGeom g = stripe_geometry(hp.n_samples, fp64, K.den_mode, K.tile);
        const size_t state = (size_t)g.spad * g.sstride * sizeof(double);
        const int32_t E = job_E[j];
        const int32_t kz = b->kz[j];
        UF_TRY(p->num.ensure(state * kz), "allocating stripes");
        if (K.den_mode == 0) UF_TRY(p->den.ensure(state * kz), "allocating stripes");
        UF_TRY(p->D.ensure((size_t)hp.n_samples * sizeof(double)), "allocating sums");
        if (K.den_mode != 0)
            UF_TRY(p->rowdot_part.ensure(rowdot_scratch_elems(hp.n_samples, hp.n_nodes - 1) * sizeof(double)),
                   "allocating sum scratch");
        UF_TRY(p->inv_t.ensure((size_t)hp.n_samples * sizeof(double)), "allocating totals");
        const int32_t idx = (int32_t)sj[q].size();
        sj[q].push_back(make_stripe_args(km, p->counts.p, p->cw, p->cstride,
                                         p->inv_t.as<double>(), p->len_slot.as<double>(),
                                         hp.n_nodes - 1, E, p->num.as<double>(),
                                         K.den_mode == 0 ? p->den.as<double>() : nullptr, g));
        sj[q].back().kz = kz;
        sj[q].back().zstride = (int64_t)(state / sizeof(double));
        sj[q].back().store_first = 1;
        if (hp.n_nodes - 1 <= 0 || g.S == 0) continue;  // nothing to accumulate
        const int32_t n_tiles = sj[q].back().tiles_k * sj[q].back().tiles_s;
        for (int32_t z = 0; z < kz; ++z)
            for (int32_t t = 0; t < n_tiles; ++t) {
                items[q].push_back(idx);
                items[q].push_back(z * n_tiles + t);
            }
    }
    for (int q = 0; q < uf_batch::kQueues; ++q) {
        b->n_stripe_items[q] = (int32_t)(items[q].size() / 2);
        if (sj[q].empty()) continue;
        UF_TRY(upload(b->stripe_jobs[q], sj[q], st), "uploading striped jobs");
        UF_TRY(upload(b->stripe_items[q], items[q], st), "uploading striped items");
    }

    // matrix-core tables
    std::vector<int32_t> tiles_all;
    std::vector<size_t> tile_off(nj, 0);
    std::vector<int32_t> morder;
    for (int32_t j : order)
        if (!is_striped(b->jobs[j])) morder.push_back(j);
    for (int32_t j : morder) {
        std::vector<int32_t> xy;
        mfma_tile_list(b->plans[j]->hp.n_samples, &xy);
        tile_off[j] = tiles_all.size();
        tiles_all.insert(tiles_all.end(), xy.begin(), xy.end());
    }
    if (!tiles_all.empty()) UF_TRY(upload(b->mfma_tiles, tiles_all, st), "uploading tile lists");
    std::vector<MfmaArgs> mj[2];
    std::vector<int32_t> mitems[2];
    for (int32_t j : morder) {
        uf_plan *p = b->plans[j];
        const uf_job &J = b->jobs[j];
        const JobKnobs &K = b->knobs[j];
        const int v = K.variant;
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
        double *S = s_in_out ? static_cast<double *>(b->dev_out[j]) : T + g.n_pad;
        uint16_t *hi = p->mfma_scratch[1].as<uint16_t>();
        const int32_t m = (int32_t)mj[v].size();
        mj[v].push_back(make_mfma_args(p->mfma_scratch[0].as<uint8_t>(), hi, hi + g.k_pad, K.k_chunk,
                                       b->mfma_tiles.as<int32_t>() + tile_off[j], g, S, T));
        for (int32_t t = 0; t < g.n_tiles; ++t) {
            mitems[v].push_back(m);
            mitems[v].push_back(t);
        }
    }
    for (int v = 0; v < 2; ++v) {
        b->n_mfma_items[v] = (int32_t)(mitems[v].size() / 2);
        if (mj[v].empty()) continue;
        UF_TRY(upload(b->mfma_jobs[v], mj[v], st), "uploading matrix-core jobs");
        UF_TRY(upload(b->mfma_items[v], mitems[v], st), "uploading matrix-core items");
    }
    UF_TRY(b->counters.ensure((uf_batch::kQueues + 2) * sizeof(int32_t)), "allocating counters");
    if (!morder.empty()) {
        UF_TRY(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking), "creating the matrix-core stream");
        UF_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming), "creating event");
        UF_TRY(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming), "creating event");
    }
    UF_TRY(hipStreamSynchronize(st), "synchronizing");
    return UF_OK;
}

// Host outputs: copy every staged job output back after the device work on `st`.
uf_status copy_out(uf_batch *b, hipStream_t st)
{
    uf_context *ctx = b->ctx;
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        const uf_job &J = b->jobs[j];
        if (J.out_on_device || !b->dev_out[j]) continue;
        const int64_t n = b->plans[j]->hp.n_samples;
        const size_t bytes = (size_t)(n * (n - 1) / 2) * (J.out_dtype == UF_F32 ? 4 : 8);
        UF_TRY(hipMemcpyAsync(J.out, b->dev_out[j], bytes, hipMemcpyDeviceToHost, st), "copying distances out");
    }
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
        // knobs: the batch's tuning, else what uf_autotune stored for this kind of problem
        const uf_job &J = jobs[j];
        const uf_tuning *t = tuning ? tuning
                                    : tuned_knobs(ctx, J.method, J.prec, p->hp.n_samples, p->hp.n_nodes);
        JobKnobs K;
        K.E = (t && t->emb_batch > 0) ? t->emb_batch : (J.prec == UF_PREC_FP64 ? 1024 : 128);
        K.den_mode = t ? t->den_mode : 0;
        K.tile = t ? t->tile : 2;   // without knobs, the fastest measured shape for den_mode 0
        K.count_width = t ? t->count_width : 0;
        K.k_chunk = (t && t->k_chunk > 0) ? t->k_chunk : 4096;
        K.variant = t ? t->variant : 0;
        K.k_split = t ? t->k_split : 0;
        K.e_free = (t && t->emb_batch > 0) || J.prec != UF_PREC_FP64 ? 0 : 1;
        if ((K.den_mode != 0 && K.den_mode != 1) || K.tile < 0 || K.tile > 2 ||
            (K.variant != 0 && K.variant != 1)) {
            uf_batch_destroy(b);
            return set_err(ctx, UF_E_ARG, "den_mode and variant must be 0 or 1, tile 0, 1 or 2");
        }
        if (K.k_split < 0 || K.k_split > 64) {
            uf_batch_destroy(b);
            return set_err(ctx, UF_E_ARG, "k_split must be in [0, 64]");
        }
        if (J.method == UF_WEIGHTED_UNNORMALIZED) K.den_mode = 1;   // no denominator at all
        b->knobs.push_back(K);
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
    uf_status s = copy_out(b, st);
    if (s != UF_OK) return s;
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
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    for (uf_plan *p : b->plans) uf_plan_destroy(p);
    for (int q = 0; q < uf_batch::kQueues; ++q) {
        b->stripe_jobs[q].release();
        b->stripe_items[q].release();
    }
    for (int v = 0; v < 2; ++v) {
        b->mfma_jobs[v].release();
        b->mfma_items[v].release();
    }
    for (DevMem *m : {&b->prop_jobs, &b->scatter_tasks, &b->level_tasks, &b->mfma_tiles, &b->counters})
        m->release();
    b->prof.release();
    delete b;
    (void)hipGetLastError();   // leave no error of the release pending for the caller
}

uf_status uf_distance_batch(uf_context *ctx, const uf_job *jobs, int32_t n_jobs, void *stream)
{
    uf_batch *b = nullptr;
    uf_status s = uf_batch_create(ctx, jobs, n_jobs, nullptr, stream, &b);
    if (s != UF_OK) return s;
    s = uf_batch_run(b, stream);
    // the batch's buffers are released below: wait for the work that reads them
    if (s == UF_OK) {
        const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (e != hipSuccess) s = hip_fail(ctx, e, "synchronizing the batch");
    }
    uf_batch_destroy(b);
    return s;
}

}  // extern "C"
