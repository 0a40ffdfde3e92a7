// Host runtime objects shared by the C ABI files: device buffers, event profiler, the
// context and plan structures, and error helpers.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "uf_internal.h"

namespace ufmi {

extern thread_local std::string g_tls_err;

// A device allocation that only grows.
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t want)
    {
        if (want == 0) want = 256;
        if (bytes >= want) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// Event-pair timing of launches, grouped by kernel class.
struct Profiler {
    bool on = false;
    struct Pending {
        std::string cls;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Pending> pending;
    std::map<std::string, std::pair<int64_t, double>> totals;

    hipEvent_t take()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void collect()
    {
        for (Pending &p : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                auto &t = totals[p.cls];
                t.first += 1;
                t.second += ms;
            }
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
    void release()
    {
        collect();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};

}  // namespace ufmi

// Every entry point starts here: drops an error left pending by earlier, unrelated HIP calls
// on this thread (so that a later launch check does not report it) and selects the device.
inline hipError_t enter_device(int device)
{
    (void)hipGetLastError();
    return hipSetDevice(device);
}

struct uf_context {
    int32_t device = 0;
    int32_t n_cu = 256;      // compute units of the device
    std::string err;
    // knobs chosen by uf_autotune, by problem kind and size bucket (tune_key)
    std::map<std::string, uf_tuning> tune;
};

struct uf_plan {
    uf_context *ctx = nullptr;
    ufmi::HostPrep hp;
    // resident inputs
    ufmi::DevMem indptr, entry_slot, entry_count, totals, child_ptr, child_slot, len_slot,
        slot_of_node, tail_lvl, tail_rec, tail_kid, tail_chunks;
    ufmi::TailProgram tail{};   // the narrow top of the tree as one launch (n_chunks 0: none)
    int32_t tail_level = 0;     // first level of that top; lower levels run one launch each
    // scratch, allocated on first use
    ufmi::DevMem counts, bits, emb, num, den, D, inv_t, out_tmp, gather_tmp, rowdot_part;
    ufmi::DevMem mfma_scratch[4];
    ufmi::Profiler prof;
    int64_t cstride = 0;  // count elements per row (multiple of 64)
    int32_t cw = 4;       // bytes per count of the last propagation: 4 (int32) or 2 (uint16)
    int64_t bstride = 0;  // uint32 words per presence row (multiple of 4)
    // generated rows: when all count rows (or presence bits) would not fit, batches of them
    // are computed from depth-first tip ranges on a second stream, double-buffered
    int64_t mem_limit = 0;   // device bytes the plan may hold (0: whatever the device has)
    bool gen_ready = false;
    ufmi::DevMem gen_spos, gen_scum, gen_lo, gen_hi, gen_buf[2], gen_tmp;
    hipStream_t gen_stream = nullptr;
    hipEvent_t gen_start = nullptr, gen_filled[2] = {}, gen_used[2] = {};
};

namespace ufmi {

inline uf_status set_err(uf_context *ctx, uf_status code, const std::string &msg)
{
    if (ctx)
        ctx->err = msg;
    else
        g_tls_err = msg;
    return code;
}

inline uf_status hip_fail(uf_context *ctx, hipError_t e, const char *what)
{
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    return set_err(ctx, e == hipErrorOutOfMemory ? UF_E_OOM : UF_E_DEVICE, msg);
}

#define UF_TRY(expr, what)                                       \
    do {                                                         \
        hipError_t _e = (expr);                                  \
        if (_e != hipSuccess) return hip_fail(ctx, _e, (what));  \
    } while (0)

template <typename T>
hipError_t upload(DevMem &m, const std::vector<T> &v, hipStream_t st)
{
    hipError_t e = m.ensure(v.size() * sizeof(T));
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpyAsync(m.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Launch `fn` on `st`, bracketed by timing events when the profiler is on.
template <typename F>
hipError_t timed(Profiler &P, const char *cls, hipStream_t st, F &&fn)
{
    if (!P.on) return fn();
    hipEvent_t a = P.take(), b = P.take();
    if (!a || !b) return fn();
    hipError_t e = hipEventRecord(a, st);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, st);
    if (e == hipSuccess) P.pending.push_back({cls, a, b});
    return e;
}

template <typename F>
hipError_t timed(uf_plan *plan, const char *cls, hipStream_t st, F &&fn)
{
    return timed(plan->prof, cls, st, fn);
}

// Plan-level steps reused by the batch runner.
// cw: 4 = int32 counts, 2 = uint16 (needs every total <= 65535), 0 = uint16 when it fits
uf_status propagate_counts(uf_plan *plan, hipStream_t st, int32_t cw = 0);
int32_t resolve_count_width(const HostPrep &hp, int32_t requested);
uf_status propagate_bits(uf_plan *plan, hipStream_t st);
uf_status plan_prepare(uf_context *ctx, const uf_tree *tree, const uf_table *table,
                       hipStream_t st, uf_plan **out);

// Resolved knobs of one distance call (uf_tuning with the defaults filled in).
struct Knobs {
    int32_t emb_batch, k_chunk, den_mode, variant, tile, count_width, k_split;
    int32_t e_free;   // 1: emb_batch is the FP64 default and may shrink for branch splits
};
Knobs resolve_knobs(const uf_tuning *t, uf_precision prec, int32_t n_branches);
uf_status check_enums(uf_context *ctx, uf_method method, uf_precision prec);

// Device buffers of the fused striped path: count rows, reciprocal totals, stripe state
// copies, per-sample sums and their partial-sum scratch.
struct StripedWork {
    void *C;
    double *inv_t, *num, *den, *D, *part;
};
uf_status propagate_counts_into(uf_plan *plan, void *C, int32_t cw, hipStream_t st);
StripeGeom striped_geometry(const uf_plan *plan, uf_precision prec, const Knobs &kn);
size_t striped_state_bytes(const StripeGeom &g, int32_t s_begin, int32_t s_end, int32_t *t0, int32_t *t1);
int32_t striped_k_split(const uf_plan *plan, Knobs &kn, const StripeGeom &g, size_t state);
uf_status striped_core(uf_plan *plan, uf_method method, uf_precision prec, const Knobs &kn,
                       const StripeGeom &g, int32_t t0, int32_t t1, int32_t kz, size_t state,
                       int32_t cw, const StripedWork &W, hipStream_t st);

// Resolves this device's copy of the fixed scratch array of uf_plan_distance_noalloc
// (once per device; the device must be current).
hipError_t noalloc_scratch_init(int device);

// Context tune cache: key of a (method, precision) problem with n samples and n_nodes nodes
// (log2 buckets of both), and the stored knobs for it (nullptr when none).
std::string tune_key(uf_method method, uf_precision prec, int32_t n_samples, int32_t n_nodes);
const uf_tuning *tuned_knobs(const uf_context *ctx, uf_method method, uf_precision prec,
                             int32_t n_samples, int32_t n_nodes);

}  // namespace ufmi
