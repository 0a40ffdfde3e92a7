// Autotuner for the knobs the paper calls grouping parameters (Section 3: the tile and
// batch sizes "can drastically affect the observed run time").
//
// For a plan and a (method, precision) it times candidate settings on the resident inputs
// with HIP events, rejects any candidate whose output differs from the reference candidate
// by more than the path's tolerance, and returns the fastest.  Two front ends:
//  - uf_plan_autotune tunes one plan; winners can be kept in a small text cache keyed by
//    device architecture, method, precision, denominator mode and problem-size bucket;
//  - uf_autotune tunes representative jobs and keeps the winners in the context, where the
//    distance entry points and batches find them for problems of the same kind and size.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "uf_runtime.h"

using namespace ufmi;

namespace {

int bucket(int64_t x)
{
    int b = 0;
    while ((int64_t(1) << b) < x) ++b;
    return b;
}

std::string make_key(uf_plan *plan, uf_method method, uf_precision prec, int32_t den_mode)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, plan->ctx->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    std::ostringstream os;
    os << arch << "|m" << (int)method << "|p" << (int)prec << "|d" << den_mode << "|n"
       << bucket(plan->hp.n_samples) << "|b" << bucket(plan->hp.n_nodes);
    return os.str();
}

bool cache_lookup(const char *path, const std::string &key, uf_tuning *t, double *ms)
{
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {   // the last entry for a key wins
        std::istringstream is(line);
        std::string k;
        uf_tuning c{};
        double m = 0;
        if (!(is >> k >> c.emb_batch >> c.k_chunk >> c.den_mode >> c.variant >> c.tile >> m)) continue;
        if (k == key) {
            *t = c;
            *ms = m;
            found = true;
        }
    }
    return found;
}

void cache_store(const char *path, const std::string &key, const uf_tuning &t, double ms)
{
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << ' ' << t.emb_batch << ' ' << t.k_chunk << ' ' << t.den_mode << ' ' << t.variant
      << ' ' << t.tile << ' ' << ms << '\n';
}

// Candidate knobs of one (method, precision).  The first candidate is the reference the
// others are compared with.  FP32 batch depths stop at 128: the in-batch FP32 sums of E
// positive terms carry at most (E - 1) * 2^-24 of the distance, below 1e-5 only up to there.
std::vector<uf_tuning> candidates(uf_method method, uf_precision prec, const std::vector<int32_t> &dens)
{
    std::vector<uf_tuning> c;
    if (prec == UF_PREC_MFMA_BF16X2) {
        for (int32_t v : {0, 1})
            for (int32_t kc : {4096, 16384}) c.push_back(uf_tuning{0, kc, 0, v, 0, 0, 0});
        return c;
    }
    const std::vector<int32_t> Es = prec == UF_PREC_FP32 ? std::vector<int32_t>{128, 64, 32}
                                                         : std::vector<int32_t>{1024, 256, 4096};
    for (int32_t d : dens) {
        if (method == UF_WEIGHTED_UNNORMALIZED && d == 0) continue;   // no denominator at all
        for (int32_t tile : {2, 0, 1})
            for (int32_t E : Es) c.push_back(uf_tuning{E, 0, d, 0, tile, 0, 0});
    }
    return c;
}

// Times every candidate on the plan (one checked call, then `reps` timed calls on the default
// stream) and returns the fastest eligible one.
uf_status tune_plan(uf_plan *plan, uf_method method, uf_precision prec,
                    const std::vector<uf_tuning> &cands, int32_t reps, uf_tuning *best, double *best_ms)
{
    uf_context *ctx = plan->ctx;
    const int64_t n = plan->hp.n_samples;
    const int64_t n_pairs = n * (n - 1) / 2;
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    DevMem ref, out, diff;
    UF_TRY(ref.ensure((size_t)std::max<int64_t>(n_pairs, 1) * sizeof(double)), "allocating tuner output");
    UF_TRY(out.ensure((size_t)std::max<int64_t>(n_pairs, 1) * sizeof(double)), "allocating tuner output");
    UF_TRY(diff.ensure(sizeof(double)), "allocating tuner scratch");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    UF_TRY(hipEventCreate(&e0), "event");
    UF_TRY(hipEventCreate(&e1), "event");
    const double tol = prec == UF_PREC_FP64 ? 1e-12 : 1e-5;
    double best_t = INFINITY;
    uf_status status = UF_OK;
    for (size_t c = 0; c < cands.size(); ++c) {
        DevMem &dst = c == 0 ? ref : out;
        uf_status s = uf_plan_distance(plan, method, prec, &cands[c], UF_F64, dst.p, 1, nullptr);
        if (s != UF_OK) {
            if (c == 0) { status = s; break; }
            continue;
        }
        if (c > 0 && n_pairs > 0) {
            double h = 0;
            if (launch_max_abs_diff(ref.as<double>(), out.as<double>(), n_pairs, diff.as<double>(), nullptr) != hipSuccess ||
                hipMemcpy(&h, diff.p, sizeof h, hipMemcpyDeviceToHost) != hipSuccess) {
                status = set_err(ctx, UF_E_DEVICE, "tuner comparison failed");
                break;
            }
            if (!(h <= tol)) continue;   // a candidate that changes the answer is not eligible
        }
        float t = 0.f;
        (void)hipEventRecord(e0, nullptr);
        for (int32_t r = 0; r < reps; ++r)
            (void)uf_plan_distance(plan, method, prec, &cands[c], UF_F64, dst.p, 1, nullptr);
        (void)hipEventRecord(e1, nullptr);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&t, e0, e1);
        const double per = (double)t / reps;
        if (per < best_t) {
            best_t = per;
            *best = cands[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ref.release();
    out.release();
    diff.release();
    if (status != UF_OK) return status;
    if (best_ms) *best_ms = best_t;
    return UF_OK;
}

}  // namespace

namespace ufmi {

std::string tune_key(uf_method method, uf_precision prec, int32_t n_samples, int32_t n_nodes)
{
    std::ostringstream os;
    os << "m" << (int)method << "|p" << (int)prec << "|n" << bucket(n_samples) << "|b" << bucket(n_nodes);
    return os.str();
}

const uf_tuning *tuned_knobs(const uf_context *ctx, uf_method method, uf_precision prec,
                             int32_t n_samples, int32_t n_nodes)
{
    if (!ctx || ctx->tune.empty()) return nullptr;
    auto it = ctx->tune.find(tune_key(method, prec, n_samples, n_nodes));
    return it == ctx->tune.end() ? nullptr : &it->second;
}

}  // namespace ufmi

extern "C" {

uf_status uf_plan_autotune(uf_plan *plan, uf_method method, uf_precision prec,
                           const uf_tuning *base, int32_t reps, const char *cache_path,
                           uf_tuning *best, double *best_ms)
{
    if (!plan || !best) return set_err(plan ? plan->ctx : nullptr, UF_E_ARG, "NULL argument");
    uf_context *ctx = plan->ctx;
    if (prec == UF_PREC_MFMA_BF16X2 && method != UF_UNWEIGHTED)
        return set_err(ctx, UF_E_UNSUPPORTED, "the matrix-core form exists for unweighted UniFrac only");
    const int32_t den_mode = base ? base->den_mode : 0;
    const std::string key = make_key(plan, method, prec, den_mode);
    double ms = 0;
    if (cache_lookup(cache_path, key, best, &ms)) {
        if (best_ms) *best_ms = ms;
        return UF_OK;
    }
    std::vector<uf_tuning> cands = candidates(method, prec, {den_mode});
    uf_status s = tune_plan(plan, method, prec, cands, reps > 0 ? reps : 3, best, &ms);
    if (s != UF_OK) return s;
    if (best_ms) *best_ms = ms;
    cache_store(cache_path, key, *best, ms);
    return UF_OK;
}

uf_status uf_autotune(uf_context *ctx, const uf_job *jobs, int32_t n)
{
    if (!ctx || n < 0 || (n > 0 && !jobs)) return set_err(ctx, UF_E_ARG, "invalid autotune arguments");
    for (int32_t j = 0; j < n; ++j) {
        const uf_job &J = jobs[j];
        if (J.method != UF_UNWEIGHTED && J.method != UF_WEIGHTED_NORMALIZED &&
            J.method != UF_WEIGHTED_UNNORMALIZED)
            return set_err(ctx, UF_E_ARG, "job has an unknown method");
        if (J.prec != UF_PREC_FP64 && J.prec != UF_PREC_FP32 && J.prec != UF_PREC_MFMA_BF16X2)
            return set_err(ctx, UF_E_ARG, "job has an unknown precision");
        if (J.prec == UF_PREC_MFMA_BF16X2 && J.method != UF_UNWEIGHTED)
            return set_err(ctx, UF_E_UNSUPPORTED, "matrix-core jobs must be unweighted");
        uf_plan *plan = nullptr;
        uf_status s = plan_prepare(ctx, &J.tree, &J.table, nullptr, &plan);
        if (s != UF_OK) return set_err(ctx, s, "job " + std::to_string(j) + ": " + ctx->err);
        if (plan->hp.n_samples < 2) {   // no pairs: nothing to time
            uf_plan_destroy(plan);
            continue;
        }
        uf_tuning best{};
        double ms = 0;
        s = tune_plan(plan, J.method, J.prec, candidates(J.method, J.prec, {0, 1}), 2, &best, &ms);
        const std::string key = tune_key(J.method, J.prec, plan->hp.n_samples, plan->hp.n_nodes);
        uf_plan_destroy(plan);
        if (s != UF_OK) return s;
        ctx->tune[key] = best;
    }
    return UF_OK;
}

uf_status uf_autotune_lookup(const uf_context *ctx, uf_method method, uf_precision prec,
                             int32_t n_samples, int32_t n_nodes, uf_tuning *out, int32_t *found)
{
    if (!ctx || !out || !found) return set_err(nullptr, UF_E_ARG, "NULL argument");
    const uf_tuning *t = tuned_knobs(ctx, method, prec, n_samples, n_nodes);
    *found = t ? 1 : 0;
    if (t) *out = *t;
    return UF_OK;
}

}  // extern "C"
