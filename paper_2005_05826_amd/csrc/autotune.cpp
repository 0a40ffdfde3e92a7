// Autotuner for the knobs the paper calls grouping parameters (Section 3: the tile and
// batch sizes "can drastically affect the observed run time").
//
// For a plan and a (method, precision) it times candidate settings on the resident inputs
// with HIP events, rejects any candidate whose output differs from the reference candidate
// by more than the path's tolerance, and returns the fastest.  Winners can be kept in a
// small text cache keyed by device architecture, method, precision, denominator mode and
// problem-size bucket, so later calls skip the timing.
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

}  // namespace

extern "C" uf_status uf_autotune(uf_plan *plan, uf_method method, uf_precision prec,
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
    const int64_t n = plan->hp.n_samples;
    const int64_t n_pairs = n * (n - 1) / 2;
    reps = reps > 0 ? reps : 3;

    std::vector<uf_tuning> cands;
    if (prec == UF_PREC_MFMA_BF16X2) {
        for (int32_t v : {0, 1})
            for (int32_t kc : {4096, 16384}) cands.push_back(uf_tuning{0, kc, 0, v, 0, 0});
    } else {
        // FP32 sums inside a batch carry up to ~E * 2^-24 relative error: deeper FP32 batches
        // are candidates too, and win only if their output stays within the tolerance of the
        // first (E = 128) candidate
        const std::vector<int32_t> Es = prec == UF_PREC_FP32 ? std::vector<int32_t>{128, 64, 256, 512}
                                                             : std::vector<int32_t>{1024, 256, 4096};
        for (int32_t tile : {0, 1, 2})
            for (int32_t E : Es) cands.push_back(uf_tuning{E, 0, den_mode, 0, tile});
    }

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
        if (c > 0) {
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
    cache_store(cache_path, key, *best, best_t);
    return UF_OK;
}
