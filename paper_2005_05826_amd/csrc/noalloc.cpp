// Distance entry point for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): the striped path of
// uf_plan_distance with every scratch buffer carved out of one fixed device array.
//
// The array is a file-scope __device__ variable, so every GPU the library runs on holds its
// own copy for the life of the process.  Host code never uses the variable's name as a
// device address: uf_context_create resolves the copy of its device with
// hipGetSymbolAddress (with that device current) and keeps the address per device, and
// only that address reaches kernels.
#include <mutex>

#include "uf_runtime.h"

using namespace ufmi;

namespace {

constexpr size_t kScratchBytes = size_t(UF_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace ufmi {

// Called by uf_context_create with `device` current.
hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

}  // namespace ufmi

extern "C" uf_status uf_plan_distance_noalloc(uf_plan *plan, uf_method method, uf_precision prec,
                                              const uf_tuning *tuning, uf_dtype out_dtype, void *out,
                                              void *stream)
{
    if (!plan) return set_err(nullptr, UF_E_ARG, "plan must not be NULL");
    uf_context *ctx = plan->ctx;
    uf_status s = check_enums(ctx, method, prec);
    if (s != UF_OK) return s;
    if (prec == UF_PREC_MFMA_BF16X2)
        return set_err(ctx, UF_E_UNSUPPORTED, "the no-allocation entry point runs the striped precisions only");
    if (out_dtype != UF_F64 && out_dtype != UF_F32) return set_err(ctx, UF_E_ARG, "unknown dtype");
    const HostPrep &hp = plan->hp;
    const int64_t n_pairs = (int64_t)hp.n_samples * (hp.n_samples - 1) / 2;
    if (n_pairs == 0) return UF_OK;
    if (!out) return set_err(ctx, UF_E_ARG, "out must not be NULL");
    if (!tuning) tuning = tuned_knobs(ctx, method, prec, hp.n_samples, hp.n_nodes);
    Knobs kn = resolve_knobs(tuning, prec, hp.n_nodes - 1);
    if (kn.den_mode != 0 && kn.den_mode != 1) return set_err(ctx, UF_E_ARG, "den_mode must be 0 or 1");
    if (kn.tile < 0 || kn.tile > 2) return set_err(ctx, UF_E_ARG, "tile must be 0, 1 or 2");
    if (kn.k_split < 0 || kn.k_split > 64) return set_err(ctx, UF_E_ARG, "k_split must be in [0, 64]");
    kn.variant = 0;   // the fused kernel: no embedding buffer
    if (method == UF_WEIGHTED_UNNORMALIZED) kn.den_mode = 1;
    const int32_t cw = resolve_count_width(hp, kn.count_width);
    if (cw < 0) return set_err(ctx, UF_E_ARG, "16-bit counts need every sample total <= 65535");
    if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_scratch_ptr[ctx->device])
        return set_err(ctx, UF_E_INTERNAL, "device scratch was not resolved for this device");
    unsigned char *base = static_cast<unsigned char *>(g_scratch_ptr[ctx->device]);

    // carve the scratch: count rows, reciprocal totals, per-sample sums and their partials,
    // then the stripe state copies (as many branch splits as asked for, or as fit)
    const StripeGeom g = striped_geometry(plan, prec, kn);
    int32_t t0 = 0, t1 = 0;
    const size_t state = striped_state_bytes(g, -1, -1, &t0, &t1);
    const int32_t B = hp.n_nodes - 1;
    const size_t c_bytes = align256((size_t)hp.n_nodes * plan->cstride * cw);
    const size_t v_bytes = align256((size_t)hp.n_samples * sizeof(double));
    const size_t part_bytes = align256(rowdot_scratch_elems(hp.n_samples, std::max(B, 1)) * sizeof(double));
    const size_t fixed = c_bytes + 2 * v_bytes + part_bytes;
    const size_t per_copy = align256(state) * (kn.den_mode == 0 ? 2 : 1);
    if (fixed + per_copy > kScratchBytes)
        return set_err(ctx, UF_E_ARG,
                       "problem needs " + std::to_string(fixed + per_copy) + " bytes of device scratch, more than the " +
                           std::to_string(kScratchBytes) + " the no-allocation entry point holds");
    int32_t kz = striped_k_split(plan, kn, g, state);
    kz = (int32_t)std::min<size_t>((size_t)kz, (kScratchBytes - fixed) / per_copy);
    StripedWork W{};
    size_t off = 0;
    W.C = base + off;
    off += c_bytes;
    W.inv_t = reinterpret_cast<double *>(base + off);
    off += v_bytes;
    W.D = reinterpret_cast<double *>(base + off);
    off += v_bytes;
    W.part = reinterpret_cast<double *>(base + off);
    off += part_bytes;
    W.num = reinterpret_cast<double *>(base + off);
    off += align256(state) * kz;
    W.den = kn.den_mode == 0 ? reinterpret_cast<double *>(base + off) : nullptr;

    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // no timing events either: the profiler would create them
    const bool prof_on = plan->prof.on;
    plan->prof.on = false;
    s = striped_core(plan, method, prec, kn, g, t0, t1, kz, state, cw, W, st);
    plan->prof.on = prof_on;
    if (s != UF_OK) return s;
    UF_TRY(launch_condense(method, W.num, W.den, kn.den_mode == 0 ? nullptr : W.D, g.sstride, g.n, g.S,
                           out_dtype == UF_F32, out, st),
           "condense");
    return UF_OK;
}
