// (a2) embedding transform, (b) striped accumulation and (d) normalize/condense.
//
// Stripe layout (Section 2, Fig. 1): stripe s, column k accumulates the pair
// (k, (k + s + 1) mod n); with S = floor(n/2) stripes every unordered pair appears once,
// except that for even n the last stripe holds each of its pairs twice (both copies are
// equal and the condense step reads the first).  num and den are [spad][sstride] FP64.
//
// Batching (Section 3, Figs. 2-3): one launch folds a batch of E branch embeddings into the
// stripes.  Every work-group owns a tile of TSW stripes x TKW samples and keeps it in
// registers for the whole batch, so the stripe memory is read and written once per batch
// instead of once per branch.  For each group of EB branches the work-group stages, in
// LDS, the window of samples k (TKW values) and the window of samples k + s + 1
// (TKW + TSW - 1 values) with coalesced loads; every lane then owns TKT consecutive samples
// of TST consecutive stripes, which need only TKT + TKT + TST - 1 values per branch.
#include "uf_internal.h"

namespace ufmi {

namespace {

constexpr int kBlock = 256;  // 4 waves: wave w owns stripes [w*TST, (w+1)*TST) of the tile

template <typename T>
struct StripeCfg;
template <>
struct StripeCfg<double> {
    static constexpr int TKT = 4, TST = 8, EB = 16;
};
template <>
struct StripeCfg<float> {
    static constexpr int TKT = 8, TST = 4, EB = 16;
};

// emb[e][x] = f(C[slot0 + e][x mod n]) for x < n + S, else 0.
// Weighted normalized: f = count / total (FP64 division, then rounded to T).
// Unweighted: f = 1 if count > 0 else 0.
template <typename T, int METHOD>
__global__ void k_transform(const int32_t *__restrict__ C, int64_t cstride, int32_t slot0,
                            const int32_t *__restrict__ totals, int32_t n, int32_t S,
                            T *__restrict__ emb, int64_t estride)
{
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= estride) return;
    const int32_t e = blockIdx.y;
    T val = T(0);
    if (x < (int64_t)n + S) {
        const int32_t k = x < n ? (int32_t)x : (int32_t)(x - n);
        const int32_t c = C[(int64_t)(slot0 + e) * cstride + k];
        if (METHOD == UF_WEIGHTED_NORMALIZED)
            val = (T)((double)c / (double)totals[k]);
        else
            val = c > 0 ? T(1) : T(0);
    }
    emb[(int64_t)e * estride + x] = val;
}

template <typename T, int METHOD, int DEN>
__global__ __launch_bounds__(kBlock, 2) void k_stripe(
    const T *__restrict__ emb, int64_t estride, const double *__restrict__ len, int32_t E,
    double *__restrict__ num, double *__restrict__ den, int64_t sstride, int32_t first)
{
    constexpr int TKT = StripeCfg<T>::TKT, TST = StripeCfg<T>::TST, EB = StripeCfg<T>::EB;
    constexpr int TKW = 64 * TKT, TSW = 4 * TST, VW = TKW + TSW;
    constexpr int NV = TKT + TST - 1;
    __shared__ T su[EB * TKW];
    __shared__ T sv[EB * VW];

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t k0 = (int64_t)blockIdx.x * TKW;
    const int32_t s0 = blockIdx.y * TSW;
    const T *ubase = emb + k0;
    const T *vbase = emb + k0 + s0 + 1;

    T an[TST][TKT], ad[TST][TKT];
#pragma unroll
    for (int s = 0; s < TST; ++s)
#pragma unroll
        for (int r = 0; r < TKT; ++r) {
            an[s][r] = T(0);
            ad[s][r] = T(0);
        }

    for (int32_t e0 = 0; e0 < E; e0 += EB) {
        const int eb = (E - e0) < EB ? (E - e0) : EB;
        __syncthreads();
        for (int idx = threadIdx.x; idx < eb * TKW; idx += kBlock) {
            const int e = idx / TKW, x = idx - e * TKW;
            su[idx] = ubase[(int64_t)(e0 + e) * estride + x];
        }
        for (int idx = threadIdx.x; idx < eb * VW; idx += kBlock) {
            const int e = idx / VW, x = idx - e * VW;
            sv[idx] = vbase[(int64_t)(e0 + e) * estride + x];
        }
        __syncthreads();
        for (int e = 0; e < eb; ++e) {
            const T L = (T)len[e0 + e];
            T u[TKT], v[NV];
#pragma unroll
            for (int r = 0; r < TKT; ++r) u[r] = su[e * TKW + lane * TKT + r];
#pragma unroll
            for (int c = 0; c < NV; ++c) v[c] = sv[e * VW + lane * TKT + w * TST + c];
#pragma unroll
            for (int s = 0; s < TST; ++s)
#pragma unroll
                for (int r = 0; r < TKT; ++r) {
                    const T x = v[r + s];
                    an[s][r] = fma(fabs(u[r] - x), L, an[s][r]);
                    if (DEN == 0) {
                        if (METHOD == UF_WEIGHTED_NORMALIZED)
                            ad[s][r] = fma(u[r] + x, L, ad[s][r]);
                        else
                            ad[s][r] = fma(fmax(u[r], x), L, ad[s][r]);
                    }
                }
        }
    }

#pragma unroll
    for (int s = 0; s < TST; ++s) {
        const int64_t off = (int64_t)(s0 + w * TST + s) * sstride + k0 + lane * TKT;
#pragma unroll
        for (int r = 0; r < TKT; ++r) {
            const double a = first ? 0.0 : num[off + r];
            num[off + r] = a + (double)an[s][r];
            if (DEN == 0) {
                const double b = first ? 0.0 : den[off + r];
                den[off + r] = b + (double)ad[s][r];
            }
        }
    }
}

// D[k] (+)= sum over the batch of L_e * u_k,e in FP64, for the separable denominator.
template <int METHOD>
__global__ void k_rowdot(const int32_t *__restrict__ C, int64_t cstride, int32_t slot0,
                         int32_t E, const int32_t *__restrict__ totals,
                         const double *__restrict__ len, int32_t n, double *__restrict__ D,
                         int32_t first)
{
    const int32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const double t = (double)totals[k];
    double acc = first ? 0.0 : D[k];
    for (int32_t e = 0; e < E; ++e) {
        const int32_t c = C[(int64_t)(slot0 + e) * cstride + k];
        const double u = METHOD == UF_WEIGHTED_NORMALIZED ? (double)c / t : (c > 0 ? 1.0 : 0.0);
        acc = fma(len[e], u, acc);
    }
    D[k] = acc;
}

// One work-group per condensed row i; d = num / den in FP64 (0 when den == 0).
// With D != nullptr the denominator comes from per-sample sums:
//   weighted normalized  den = D_i + D_j
//   unweighted           den = (D_i + D_j + num) / 2      (or = (u + v + xor) / 2)
template <int METHOD, typename OUT>
__global__ void k_condense(const double *__restrict__ num, const double *__restrict__ den,
                           const double *__restrict__ D, int64_t sstride, int32_t n, int32_t S,
                           OUT *__restrict__ out)
{
    const int32_t i = blockIdx.x;
    const int64_t row0 = (int64_t)n * i - (int64_t)i * (i + 1) / 2 - i - 1;
    for (int32_t j = i + 1 + threadIdx.x; j < n; j += kBlock) {
        const int32_t diff = j - i;
        int32_t s, k;
        if (diff <= S) {
            s = diff - 1;
            k = i;
        } else {
            s = n - diff - 1;
            k = j;
        }
        const int64_t at = (int64_t)s * sstride + k;
        const double a = num[at];
        double b;
        if (D == nullptr)
            b = den[at];
        else if (METHOD == UF_WEIGHTED_NORMALIZED)
            b = D[i] + D[j];
        else
            b = 0.5 * (D[i] + D[j] + a);
        const double d = (b == 0.0) ? 0.0 : a / b;
        out[row0 + j] = (OUT)d;
    }
}

inline unsigned grid1(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

template <typename T>
hipError_t stripe_dispatch(int32_t method, int32_t den_mode, const void *emb, int64_t estride,
                           const double *len, int32_t E, double *num, double *den,
                           const StripeGeom &g, bool first, hipStream_t st)
{
    dim3 grid((unsigned)(g.sstride / g.tkw), (unsigned)(g.spad / g.tsw));
    const T *e = static_cast<const T *>(emb);
    const int f = first ? 1 : 0;
    if (method == UF_WEIGHTED_NORMALIZED) {
        if (den_mode == 0)
            k_stripe<T, UF_WEIGHTED_NORMALIZED, 0><<<grid, kBlock, 0, st>>>(e, estride, len, E, num, den, g.sstride, f);
        else
            k_stripe<T, UF_WEIGHTED_NORMALIZED, 1><<<grid, kBlock, 0, st>>>(e, estride, len, E, num, den, g.sstride, f);
    } else {
        if (den_mode == 0)
            k_stripe<T, UF_UNWEIGHTED, 0><<<grid, kBlock, 0, st>>>(e, estride, len, E, num, den, g.sstride, f);
        else
            k_stripe<T, UF_UNWEIGHTED, 1><<<grid, kBlock, 0, st>>>(e, estride, len, E, num, den, g.sstride, f);
    }
    return hipGetLastError();
}

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

}  // namespace

StripeGeom stripe_geometry(int32_t n, bool fp64)
{
    StripeGeom g;
    g.n = n;
    g.S = n / 2;
    g.tkw = fp64 ? 64 * StripeCfg<double>::TKT : 64 * StripeCfg<float>::TKT;
    g.tsw = fp64 ? 4 * StripeCfg<double>::TST : 4 * StripeCfg<float>::TST;
    g.sstride = round_up(n, g.tkw);
    g.spad = (int32_t)round_up(g.S > 0 ? g.S : 1, g.tsw);
    // largest embedding index read: (sstride - tkw) + (spad - tsw) + 1 + (tkw + tsw) - 1
    g.estride = round_up(g.sstride + g.spad + 1, 64);
    return g;
}

hipError_t launch_transform(bool fp64, int32_t method, const int32_t *C, int64_t cstride,
                            int32_t slot0, int32_t E, const int32_t *totals, int32_t n, int32_t S,
                            void *emb, int64_t estride, hipStream_t st)
{
    if (E <= 0) return hipSuccess;
    dim3 grid(grid1(estride, kBlock), (unsigned)E);
    if (fp64) {
        if (method == UF_WEIGHTED_NORMALIZED)
            k_transform<double, UF_WEIGHTED_NORMALIZED><<<grid, kBlock, 0, st>>>(C, cstride, slot0, totals, n, S, (double *)emb, estride);
        else
            k_transform<double, UF_UNWEIGHTED><<<grid, kBlock, 0, st>>>(C, cstride, slot0, totals, n, S, (double *)emb, estride);
    } else {
        if (method == UF_WEIGHTED_NORMALIZED)
            k_transform<float, UF_WEIGHTED_NORMALIZED><<<grid, kBlock, 0, st>>>(C, cstride, slot0, totals, n, S, (float *)emb, estride);
        else
            k_transform<float, UF_UNWEIGHTED><<<grid, kBlock, 0, st>>>(C, cstride, slot0, totals, n, S, (float *)emb, estride);
    }
    return hipGetLastError();
}

hipError_t launch_stripe(bool fp64, int32_t method, int32_t den_mode, const void *emb,
                         int64_t estride, const double *len, int32_t E, double *num, double *den,
                         const StripeGeom &g, bool first, hipStream_t st)
{
    if (E <= 0) return hipSuccess;
    if (fp64) return stripe_dispatch<double>(method, den_mode, emb, estride, len, E, num, den, g, first, st);
    return stripe_dispatch<float>(method, den_mode, emb, estride, len, E, num, den, g, first, st);
}

hipError_t launch_rowdot(int32_t method, const int32_t *C, int64_t cstride, int32_t slot0,
                         int32_t E, const int32_t *totals, const double *len, int32_t n,
                         double *D, bool first, hipStream_t st)
{
    const int f = first ? 1 : 0;
    if (method == UF_WEIGHTED_NORMALIZED)
        k_rowdot<UF_WEIGHTED_NORMALIZED><<<grid1(n, kBlock), kBlock, 0, st>>>(C, cstride, slot0, E, totals, len, n, D, f);
    else
        k_rowdot<UF_UNWEIGHTED><<<grid1(n, kBlock), kBlock, 0, st>>>(C, cstride, slot0, E, totals, len, n, D, f);
    return hipGetLastError();
}

hipError_t launch_condense(int32_t method, const double *num, const double *den, const double *D,
                           int64_t sstride, int32_t n, int32_t S, int32_t out_f32, void *out,
                           hipStream_t st)
{
    if (n < 2) return hipSuccess;
    if (method == UF_WEIGHTED_NORMALIZED) {
        if (out_f32)
            k_condense<UF_WEIGHTED_NORMALIZED, float><<<n - 1, kBlock, 0, st>>>(num, den, D, sstride, n, S, (float *)out);
        else
            k_condense<UF_WEIGHTED_NORMALIZED, double><<<n - 1, kBlock, 0, st>>>(num, den, D, sstride, n, S, (double *)out);
    } else {
        if (out_f32)
            k_condense<UF_UNWEIGHTED, float><<<n - 1, kBlock, 0, st>>>(num, den, D, sstride, n, S, (float *)out);
        else
            k_condense<UF_UNWEIGHTED, double><<<n - 1, kBlock, 0, st>>>(num, den, D, sstride, n, S, (double *)out);
    }
    return hipGetLastError();
}

}  // namespace ufmi
