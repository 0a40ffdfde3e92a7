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
#include <type_traits>

#include "uf_internal.h"

namespace ufmi {

namespace {

constexpr int kBlock = 256;  // 4 waves: wave w owns stripes [w*TST, (w+1)*TST) of the tile

// Per-lane micro-tile: TKT consecutive samples x TST consecutive stripes; EB branches per
// LDS stage.  The tile is sized so that accumulators stay near 128 VGPRs (two waves per
// SIMD) and the work-group covers enough stripes (4 * TST) to amortize the staging of its
// windows (2 * TKW + TSW values per branch for TKW * TSW updates).
template <typename T, int DEN, int TILE>
struct StripeCfg;
// EB: most branches per LDS stage.  OCC: work-groups per CU the fused and queued kernels
// are compiled for (tile 2 trades a smaller tile for three or four waves per SIMD; the FP32
// 4 x 16 shape takes shorter stages so that its staging registers fit four).
template <> struct StripeCfg<double, 0, 0> { static constexpr int TKT = 4, TST = 8, EB = 8, OCC = 2; };
template <> struct StripeCfg<double, 0, 1> { static constexpr int TKT = 2, TST = 12, EB = 8, OCC = 2; };
template <> struct StripeCfg<double, 0, 2> { static constexpr int TKT = 2, TST = 8, EB = 8, OCC = 3; };
template <> struct StripeCfg<double, 1, 0> { static constexpr int TKT = 4, TST = 16, EB = 8, OCC = 2; };
template <> struct StripeCfg<double, 1, 1> { static constexpr int TKT = 2, TST = 24, EB = 8, OCC = 2; };
template <> struct StripeCfg<double, 1, 2> { static constexpr int TKT = 4, TST = 8, EB = 8, OCC = 3; };
template <> struct StripeCfg<float, 0, 0> { static constexpr int TKT = 4, TST = 16, EB = 8, OCC = 2; };
template <> struct StripeCfg<float, 0, 1> { static constexpr int TKT = 8, TST = 8, EB = 8, OCC = 2; };
template <> struct StripeCfg<float, 0, 2> { static constexpr int TKT = 4, TST = 8, EB = 8, OCC = 3; };
template <> struct StripeCfg<float, 1, 0> { static constexpr int TKT = 4, TST = 24, EB = 8, OCC = 2; };
template <> struct StripeCfg<float, 1, 1> { static constexpr int TKT = 8, TST = 16, EB = 8, OCC = 2; };
template <> struct StripeCfg<float, 1, 2> { static constexpr int TKT = 4, TST = 16, EB = 6, OCC = 4; };

// Pins a register value at this point of the program: the conversions that follow cannot
// be hoisted above it, which keeps the FP64 copies of a tile from being live all at once.
template <typename T>
__device__ inline T pin(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Adds a lane's register tile (TST stripe rows of TKT consecutive samples) into the FP64
// stripe state, one row at a time; with `store` (the first batch of a branch range whose
// state was not cleared) writes it instead.  With the numerator alone the stored batch skips
// the reads; with both stripes the old values read are replaced by zero, because a branch
// around the reads made the compiler wait for each row before storing it instead of keeping
// the next read in flight (2.7 % slower where the state traffic dominates).
template <int TST, int TKT, int DEN, typename T>
__device__ inline void add_tile(const T (&an)[TST][TKT], const T (&ad)[TST][TKT],
                                double *__restrict__ num, double *__restrict__ den,
                                int64_t off, int64_t sstride, bool store)
{
    static_assert(TKT % 2 == 0, "rows are written as double2");
    if constexpr (DEN == 1) {
        if (store) {
#pragma unroll
            for (int s = 0; s < TST; ++s) {
                double2 *pn = reinterpret_cast<double2 *>(num + off + s * sstride);
#pragma unroll
                for (int r = 0; r < TKT; r += 2)
                    pn[r / 2] = make_double2((double)pin(an[s][r]), (double)pin(an[s][r + 1]));
            }
            return;
        }
    }
#pragma unroll
    for (int s = 0; s < TST; ++s) {
        double2 *pn = reinterpret_cast<double2 *>(num + off + s * sstride);
        double2 *pd = reinterpret_cast<double2 *>(den + off + s * sstride);
#pragma unroll
        for (int r = 0; r < TKT; r += 2) {
            double2 a = pn[r / 2];
            if (store) a = make_double2(0.0, 0.0);
            a.x += (double)pin(an[s][r]);
            a.y += (double)pin(an[s][r + 1]);
            pn[r / 2] = a;
            if (DEN == 0) {
                double2 b = pd[r / 2];
                if (store) b = make_double2(0.0, 0.0);
                b.x += (double)pin(ad[s][r]);
                b.y += (double)pin(ad[s][r + 1]);
                pd[r / 2] = b;
            }
        }
    }
}

// emb[e][x] = f(C[slot0 + e][x mod n]) for x < n + S, else 0.
// Weighted normalized: f = count / total (FP64 division, then rounded to T).
// Unweighted: f = 1 if count > 0 else 0.
template <typename T, int METHOD, typename CT>
__global__ void k_transform(const CT *__restrict__ C, int64_t cstride, int32_t slot0,
                            const int32_t *__restrict__ totals, int32_t n, int32_t S,
                            T *__restrict__ emb, int64_t estride)
{
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= estride) return;
    const int32_t e = blockIdx.y;
    T val = T(0);
    if (x < (int64_t)n + S) {
        const int32_t k = x < n ? (int32_t)x : (int32_t)(x - n);
        const int32_t c = (int32_t)C[(int64_t)(slot0 + e) * cstride + k];
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
    constexpr int TKT = StripeCfg<T, DEN, 0>::TKT, TST = StripeCfg<T, DEN, 0>::TST, EB = StripeCfg<T, DEN, 0>::EB;
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
#pragma unroll 1
        for (int e = 0; e < eb; ++e) {
            const T L = (T)len[e0 + e];
            T u[TKT], v[NV];
#pragma unroll
            for (int r = 0; r < TKT; ++r) u[r] = su[e * TKW + lane * TKT + r];
#pragma unroll
            for (int c = 0; c < NV; ++c) v[c] = sv[e * VW + lane * TKT + w * TST + c];
            // an += |u - v| L and, with the pair-wise denominator, ad += (u + v) L or max(u, v) L.
            // Where measured faster (interleaved runs on one GPU) the non-FMA operations of a
            // lane's samples are formed before their FMAs: FP32 with the numerator alone at
            // four samples per lane (1-1.5 %), FP64 with both stripes at two samples per lane
            // (1-1.4 %).  Grouping was slower for FP32 at eight samples per lane, for the FP32
            // num + den form and for FP64 at four samples per lane, which keep each operation
            // beside its FMA.
            if constexpr (DEN == 1 && std::is_same_v<T, float> && TKT == 4) {
#pragma unroll
                for (int s = 0; s < TST; ++s)
#pragma unroll
                    for (int r = 0; r < TKT; r += 4) {
                        T d[4];
#pragma unroll
                        for (int g = 0; g < 4; ++g) d[g] = u[r + g] - v[r + g + s];
#pragma unroll
                        for (int g = 0; g < 4; ++g) an[s][r + g] = fma(fabs(d[g]), L, an[s][r + g]);
                    }
            } else if constexpr (DEN == 0 && std::is_same_v<T, double> && TKT == 2) {
#pragma unroll
                for (int s = 0; s < TST; ++s) {
                    T d[2], q[2];
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        const T x = v[g + s];
                        d[g] = u[g] - x;
                        q[g] = METHOD == UF_WEIGHTED_NORMALIZED ? u[g] + x : fmax(u[g], x);
                    }
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        an[s][g] = fma(fabs(d[g]), L, an[s][g]);
                        ad[s][g] = fma(q[g], L, ad[s][g]);
                    }
                }
            } else {
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
    }

    add_tile<TST, TKT, DEN>(an, ad, num, den, (int64_t)(s0 + w * TST) * sstride + k0 + lane * TKT,
                            sstride, false);
}

// Fused form of (a2) + (b): one work-group tile covers every batch of branches.  The
// work-group stages the embedding windows straight from the int32 count rows (transforming
// while staging: proportion = count * (1 / total) or presence = count > 0), so no embedding
// buffer is written.  A thread stages fixed window positions for every branch, so the
// sample index (with the wrap k + s + 1 - n) and the reciprocal total of each position are
// computed once.  Batches of E branches accumulate in registers; between batches the tile
// is added into the FP64 stripe state (num/den, cleared beforehand), the cross-batch
// accumulator.
template <typename T, int DEN, int TILE>
struct StripeSmem {
    static constexpr int TKT = StripeCfg<T, DEN, TILE>::TKT, TST = StripeCfg<T, DEN, TILE>::TST;
    static constexpr int TKW = 64 * TKT, TSW = 4 * TST, VW = TKW + TSW;
    static constexpr int OCC = StripeCfg<T, DEN, TILE>::OCC;
    // branches per stage: two stages must fit the work-group's share of the 160 KB LDS (OCC
    // work-groups per CU), and the next stage's counts wait in registers (EB x 3 per thread)
    static constexpr int EBM = (163840 / OCC - 256) / (2 * (TKW + VW) * (int)sizeof(T));
    static constexpr int EBC = StripeCfg<T, DEN, TILE>::EB;
    static constexpr int EB = EBM < EBC ? EBM : EBC;
    __align__(16) T su[2][EB * TKW];
    __align__(16) T sv[2][EB * VW];
    __align__(16) T sl[2][EB];   // the stage's branch lengths
};

// Reads N consecutive values from 16-byte aligned LDS: whole 16-byte loads, then one
// narrower load for the remainder, so that every register a pending read writes is one the
// caller uses (a register left unused by a wider load could be handed out as a temporary
// while the load is in flight, which forces a wait for it).
template <typename T, int N>
__device__ inline void lds_read_vec(const T *src, T (&dst)[N])
{
    constexpr int CH = 16 / (int)sizeof(T);
    constexpr int NF = N / CH, RM = N % CH;
    typedef T vec __attribute__((ext_vector_type(CH)));
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        const vec x = *reinterpret_cast<const vec *>(src + q * CH);
#pragma unroll
        for (int c = 0; c < CH; ++c) dst[q * CH + c] = x[c];
    }
    if constexpr (RM == 3) {
        typedef T vec3 __attribute__((ext_vector_type(3)));
        const vec3 x = *reinterpret_cast<const vec3 *>(src + NF * CH);
        dst[NF * CH] = x[0];
        dst[NF * CH + 1] = x[1];
        dst[NF * CH + 2] = x[2];
    } else if constexpr (RM == 2) {
        typedef T vec2 __attribute__((ext_vector_type(2)));
        const vec2 x = *reinterpret_cast<const vec2 *>(src + NF * CH);
        dst[NF * CH] = x[0];
        dst[NF * CH + 1] = x[1];
    } else if constexpr (RM == 1) {
        dst[NF * CH] = src[NF * CH];
    }
}

// Branches [bb, be) of one tile, added into the state copy at num / den.
template <typename T, int METHOD, int DEN, int TILE, typename CT>
__device__ void stripe_tile(const StripeArgs &a, int32_t k0, int32_t s0, int32_t bb, int32_t be,
                            double *num, double *den, StripeSmem<T, DEN, TILE> &sm)
{
    using SM = StripeSmem<T, DEN, TILE>;
    constexpr int TKT = SM::TKT, TST = SM::TST, EB = SM::EB;
    constexpr int TKW = SM::TKW, VW = SM::VW;
    constexpr int NV = TKT + TST - 1;
    constexpr int NU_T = (TKW + kBlock - 1) / kBlock;   // u positions per thread
    constexpr int NV_T = (VW + kBlock - 1) / kBlock;    // v positions per thread
    const CT *__restrict__ C = static_cast<const CT *>(a.C);
    const double *__restrict__ len = a.len;
    const int64_t cstride = a.cstride, sstride = a.sstride;
    const int32_t n = a.n, S = a.S, E = a.E;
    if (be <= bb) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;

    // staging positions: clamped sample index, validity, and scale (1/total or 1)
    int32_t uk[NU_T], vk[NV_T];
    T us[NU_T], vs[NV_T];
#pragma unroll
    for (int q = 0; q < NU_T; ++q) {
        const int32_t g = k0 + tid + q * kBlock;
        const bool ok = g < n && tid + q * kBlock < TKW;
        uk[q] = ok ? g : 0;
        us[q] = ok ? (METHOD == UF_WEIGHTED_NORMALIZED ? (T)a.inv_t[g] : T(1)) : T(0);
    }
#pragma unroll
    for (int q = 0; q < NV_T; ++q) {
        const int32_t x = tid + q * kBlock;
        const int32_t g = k0 + s0 + 1 + x;
        int32_t k = -1;
        if (x < VW) k = g < n ? g : (g < n + S ? g - n : -1);
        vk[q] = k >= 0 ? k : 0;
        vs[q] = k >= 0 ? (METHOD == UF_WEIGHTED_NORMALIZED ? (T)a.inv_t[k] : T(1)) : T(0);
    }

    // Stage pipeline: the count rows of the next stage are loaded into registers while the
    // current stage computes from LDS, then written to the other LDS buffer; one barrier per
    // stage.  Rows past a stage's end re-read its last row and are never stored; padding
    // positions read sample 0 and are zeroed by their scale.
    int32_t cu[EB][NU_T], cv[EB][NV_T];
    double rl = 0.0;
    auto gload = [&](int32_t e0, int32_t eb) {
        rl = tid < eb ? len[e0 + tid] : 0.0;
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            const CT *row = C + (int64_t)(e0 + (e < eb ? e : eb - 1)) * cstride;
#pragma unroll
            for (int q = 0; q < NU_T; ++q) cu[e][q] = (int32_t)row[uk[q]];
#pragma unroll
            for (int q = 0; q < NV_T; ++q) cv[e][q] = (int32_t)row[vk[q]];
        }
    };
    auto lstore = [&](int buf, int32_t eb) {
        T *su = sm.su[buf], *sv = sm.sv[buf];
        if (tid < EB) sm.sl[buf][tid] = (T)rl;
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            if (e < eb) {
#pragma unroll
                for (int q = 0; q < NU_T; ++q) {
                    const int32_t x = tid + q * kBlock;
                    const int32_t c = cu[e][q];
                    if (x < TKW)
                        su[e * TKW + x] = METHOD == UF_WEIGHTED_NORMALIZED ? (T)c * us[q]
                                                                          : (c > 0 ? us[q] : T(0));
                }
#pragma unroll
                for (int q = 0; q < NV_T; ++q) {
                    const int32_t x = tid + q * kBlock;
                    const int32_t c = cv[e][q];
                    if (x < VW)
                        sv[e * VW + x] = METHOD == UF_WEIGHTED_NORMALIZED ? (T)c * vs[q]
                                                                         : (c > 0 ? vs[q] : T(0));
                }
            }
        }
    };

    T an[TST][TKT], ad[TST][TKT];
#pragma unroll
    for (int s = 0; s < TST; ++s)
#pragma unroll
        for (int r = 0; r < TKT; ++r) {
            an[s][r] = T(0);
            ad[s][r] = T(0);
        }
    // stages: windows of at most EB branches inside batches [b0, b1) of E branches
    bool store = a.store_first != 0;   // the range's first batch writes the state
    int32_t b1 = E < be - bb ? bb + E : be;
    int32_t e0 = bb;
    int32_t eb = (b1 - e0) < EB ? (b1 - e0) : EB;
    int buf = 0;
    gload(e0, eb);
    lstore(0, eb);
    __syncthreads();
    for (;;) {
        int32_t ne0 = e0 + eb, nb1 = b1;
        if (ne0 >= b1) nb1 = (be - b1) < E ? be : b1 + E;
        const bool more = ne0 < be;
        const int32_t neb = more ? ((nb1 - ne0) < EB ? (nb1 - ne0) : EB) : 0;
        if (more) gload(ne0, neb);
        const T *su = sm.su[buf], *sv = sm.sv[buf], *sl = sm.sl[buf];
        static_assert(NV <= TKT + TST, "reads of the v window stay inside the staged row");
#pragma unroll 1
        for (int e = 0; e < eb; ++e) {
            const T L = sl[e];
            T u[TKT], v[NV];
            lds_read_vec<T, TKT>(su + e * TKW + lane * TKT, u);
            lds_read_vec<T, NV>(sv + e * VW + lane * TKT + w * TST, v);
            // an += |u - v| L and, with the pair-wise denominator, ad += (u + v) L or max(u, v) L.
            // Where measured faster (interleaved runs on one GPU) the non-FMA operations of a
            // lane's samples are formed before their FMAs: FP32 with the numerator alone at
            // four samples per lane (1-1.5 %), FP64 with both stripes at two samples per lane
            // (1-1.4 %).  Grouping was slower for FP32 at eight samples per lane, for the FP32
            // num + den form and for FP64 at four samples per lane, which keep each operation
            // beside its FMA.
            if constexpr (DEN == 1 && std::is_same_v<T, float> && TKT == 4) {
#pragma unroll
                for (int s = 0; s < TST; ++s)
#pragma unroll
                    for (int r = 0; r < TKT; r += 4) {
                        T d[4];
#pragma unroll
                        for (int g = 0; g < 4; ++g) d[g] = u[r + g] - v[r + g + s];
#pragma unroll
                        for (int g = 0; g < 4; ++g) an[s][r + g] = fma(fabs(d[g]), L, an[s][r + g]);
                    }
            } else if constexpr (DEN == 0 && std::is_same_v<T, double> && TKT == 2) {
#pragma unroll
                for (int s = 0; s < TST; ++s) {
                    T d[2], q[2];
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        const T x = v[g + s];
                        d[g] = u[g] - x;
                        q[g] = METHOD == UF_WEIGHTED_NORMALIZED ? u[g] + x : fmax(u[g], x);
                    }
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        an[s][g] = fma(fabs(d[g]), L, an[s][g]);
                        ad[s][g] = fma(q[g], L, ad[s][g]);
                    }
                }
            } else {
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
        if (e0 + eb >= b1) {   // end of a batch: add the register tile into the FP64 state
            // the offset passes through an empty asm so that the row addresses are formed
            // here rather than hoisted out of the stage loop into live registers
            int64_t off = (int64_t)(s0 - a.s_base + w * TST) * sstride + k0 + lane * TKT;
            asm volatile("" : "+v"(off));
            add_tile<TST, TKT, DEN>(an, ad, num, den, off, sstride, store);
            store = false;
#pragma unroll
            for (int s = 0; s < TST; ++s)
#pragma unroll
                for (int r = 0; r < TKT; ++r) {
                    an[s][r] = T(0);
                    ad[s][r] = T(0);
                }
        }
        if (!more) break;
        lstore(buf ^ 1, neb);
        __syncthreads();
        buf ^= 1;
        e0 = ne0;
        eb = neb;
        b1 = nb1;
    }
}

template <typename T, int METHOD, int DEN, int TILE, typename CT>
__global__ __launch_bounds__(kBlock, (StripeCfg<T, DEN, TILE>::OCC)) void k_stripe_fused(StripeArgs a)
{
    using SM = StripeSmem<T, DEN, TILE>;
    __shared__ SM sm;
    // grid z: branch split z of kz, accumulated into its own state copy
    const int32_t z = blockIdx.z;
    const int32_t bb = (int32_t)((int64_t)a.B * z / a.kz), be = (int32_t)((int64_t)a.B * (z + 1) / a.kz);
    stripe_tile<T, METHOD, DEN, TILE, CT>(a, blockIdx.x * SM::TKW, a.s_base + blockIdx.y * SM::TSW, bb, be,
                                          a.num + z * a.zstride, a.den ? a.den + z * a.zstride : nullptr, sm);
}

// Persistent form for many jobs: every work-group takes items (job, tile) from a global
// counter until the list is exhausted.  Items are listed largest job first (cost of a tile
// is proportional to the job's branch count), so the dynamic queue is a longest-processing-
// time-first schedule over the machine.  The counter must be zero at launch; every
// work-group leaves the loop at its first fetch past the end.
template <typename T, int METHOD, int DEN, int TILE, typename CT>
__global__ __launch_bounds__(kBlock, (StripeCfg<T, DEN, TILE>::OCC)) void k_stripe_queue(
    const StripeArgs *__restrict__ jobs, const int2 *__restrict__ items, int32_t n_items,
    int32_t *__restrict__ counter)
{
    using SM = StripeSmem<T, DEN, TILE>;
    __shared__ SM sm;
    __shared__ int32_t s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t it = s_item;
        if (it >= n_items) break;
        const int2 item = items[it];
        const StripeArgs a = jobs[item.x];
        // item.y = z * (tiles of the job) + tile: branch split z of a.kz, into its own state copy
        const int32_t nt = a.tiles_k * a.tiles_s;
        const int32_t z = item.y / nt, t = item.y - z * nt;
        const int32_t kt = t % a.tiles_k, stile = t / a.tiles_k;
        const int32_t k0 = kt * SM::TKW, s0 = a.s_base + stile * SM::TSW;
        const int32_t bb = (int32_t)((int64_t)a.B * z / a.kz), be = (int32_t)((int64_t)a.B * (z + 1) / a.kz);
        stripe_tile<T, METHOD, DEN, TILE, CT>(a, k0, s0, bb, be, a.num + z * a.zstride,
                                              a.den ? a.den + z * a.zstride : nullptr, sm);
    }
}

// x[i] = sum_z x[z * zstride + i] over the branch splits, in split order.
__global__ void k_reduce_z(double *__restrict__ x, int64_t zstride, int32_t kz, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= count) return;
    double s = x[i];
    for (int32_t z = 1; z < kz; ++z) s += x[z * zstride + i];
    x[i] = s;
}

// 1 / total per sample (FP64), for the fused transform.
__global__ void k_inv_totals(const int32_t *__restrict__ totals, int32_t n, double *__restrict__ inv_t)
{
    const int32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k < n) inv_t[k] = 1.0 / (double)totals[k];
}

// Separable denominator, D[k] (+)= sum over a batch of branches of L_e * u_k,e in FP64.
// Pass 1: partial sums over chunks of branches, one thread per (sample, chunk), reading count
// rows coalesced; the weighted form sums L * count and divides by the total once in pass 2.
// Pass 2 adds the chunks of each sample in chunk order, so the result is deterministic.
template <int METHOD, typename CT>
__global__ void k_rowdot_part(const CT *__restrict__ C, int64_t cstride, int32_t slot0, int32_t E,
                              int32_t chunk, const double *__restrict__ len, int32_t n,
                              double *__restrict__ part)
{
    const int32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int32_t e0 = (int32_t)blockIdx.y * chunk;
    const int32_t e1 = (E - e0) < chunk ? E : e0 + chunk;
    double acc = 0.0;
#pragma unroll 8
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t x = (int32_t)C[(int64_t)(slot0 + e) * cstride + k];
        acc = fma(len[e], METHOD == UF_WEIGHTED_NORMALIZED ? (double)x : (x > 0 ? 1.0 : 0.0), acc);
    }
    part[(int64_t)blockIdx.y * n + k] = acc;
}

template <int METHOD>
__global__ void k_rowdot_sum(const double *__restrict__ part, int32_t n_chunks,
                             const int32_t *__restrict__ totals, int32_t n, double *__restrict__ D,
                             int32_t first)
{
    const int32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    double acc = 0.0;
    for (int32_t c = 0; c < n_chunks; ++c) acc += part[(int64_t)c * n + k];
    if (METHOD == UF_WEIGHTED_NORMALIZED) acc /= (double)totals[k];
    D[k] = first ? acc : D[k] + acc;
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
        double d;
        if (METHOD == UF_WEIGHTED_UNNORMALIZED) {
            d = a;
        } else {
            double b;
            if (D == nullptr)
                b = den[at];
            else if (METHOD == UF_WEIGHTED_NORMALIZED)
                b = D[i] + D[j];
            else
                b = 0.5 * (D[i] + D[j] + a);
            d = (b == 0.0) ? 0.0 : a / b;
        }
        out[row0 + j] = (OUT)d;
    }
}

// Condense of a stripe range [s_begin, s_end) held in a state block whose first row is
// stripe s_base: each (s, k) computes the distance of the pair (k, (k + s + 1) mod n) and
// writes it where the output layout puts it:
//   RANGE_CONDENSED  the full condensed matrix (for even n the last stripe writes only
//                    k < n/2, the first copy of each pair);
//   RANGE_BLOCK      a dense [s_end - s_begin][n] block, every k (the duplicated half of an
//                    even n's last stripe included);
//   RANGE_COMPACT    the range's pairs only, in condensed order: row i's pairs start at
//                    row_off[i], first those at distance j - i <= S (stripe j - i - 1), then
//                    those beyond (stripe n - (j - i) - 1).
enum { RANGE_CONDENSED = 0, RANGE_BLOCK = 1, RANGE_COMPACT = 2 };

template <int METHOD, typename OUT, int LAYOUT>
__global__ void k_condense_range(const double *__restrict__ num, const double *__restrict__ den,
                                 const double *__restrict__ D, int64_t sstride, int32_t n, int32_t S,
                                 int32_t s_base, int32_t s_begin, int32_t s_end,
                                 const int64_t *__restrict__ row_off, OUT *__restrict__ out)
{
    const int32_t s = s_begin + blockIdx.y;
    const int32_t k = blockIdx.x * kBlock + threadIdx.x;
    const int32_t kmax = (LAYOUT != RANGE_BLOCK && n % 2 == 0 && s == S - 1) ? n / 2 : n;
    if (k >= kmax) return;
    const int32_t j = (k + s + 1) % n;
    const int32_t lo = k < j ? k : j, hi = k < j ? j : k;
    const int64_t at = (int64_t)(s - s_base) * sstride + k;
    const double a = num[at];
    double d;
    if (METHOD == UF_WEIGHTED_UNNORMALIZED) {
        d = a;
    } else {
        double b;
        if (D == nullptr)
            b = den[at];
        else if (METHOD == UF_WEIGHTED_NORMALIZED)
            b = D[k] + D[j];
        else
            b = 0.5 * (D[k] + D[j] + a);
        d = (b == 0.0) ? 0.0 : a / b;
    }
    int64_t idx;
    if (LAYOUT == RANGE_CONDENSED) {
        idx = (int64_t)n * lo - (int64_t)lo * (lo + 1) / 2 + (hi - lo - 1);
    } else if (LAYOUT == RANGE_BLOCK) {
        idx = (int64_t)(s - s_begin) * n + k;
    } else {
        const int32_t dist = hi - lo;
        if (dist <= S) {
            idx = row_off[lo] + (dist - (s_begin + 1));
        } else {
            const int32_t a_end = (s_end < S ? s_end : S) < n - 1 - lo ? (s_end < S ? s_end : S) : n - 1 - lo;
            const int32_t len_a = a_end - s_begin > 0 ? a_end - s_begin : 0;
            const int32_t b0 = (n - s_end) > S + 1 ? (n - s_end) : S + 1;
            idx = row_off[lo] + len_a + (dist - b0);
        }
    }
    out[idx] = (OUT)d;
}

// Scatter of a dense stripe block (RANGE_BLOCK layout) into the condensed matrix.
template <typename T>
__global__ void k_merge_block(const T *__restrict__ block, int32_t n, int32_t S, int32_t s_begin,
                              T *__restrict__ out)
{
    const int32_t s = s_begin + blockIdx.y;
    const int32_t k = blockIdx.x * kBlock + threadIdx.x;
    const int32_t kmax = (n % 2 == 0 && s == S - 1) ? n / 2 : n;
    if (k >= kmax) return;
    const int32_t j = (k + s + 1) % n;
    const int32_t lo = k < j ? k : j, hi = k < j ? j : k;
    out[(int64_t)n * lo - (int64_t)lo * (lo + 1) / 2 + (hi - lo - 1)] = block[(int64_t)(s - s_begin) * n + k];
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

template <typename T, int DEN, int TILE>
static void tile_dims(StripeGeom *g)
{
    g->tkw = 64 * StripeCfg<T, DEN, TILE>::TKT;
    g->tsw = 4 * StripeCfg<T, DEN, TILE>::TST;
    g->occ = StripeCfg<T, DEN, TILE>::OCC;
}

StripeGeom stripe_geometry(int32_t n, bool fp64, int32_t den_mode, int32_t tile)
{
    StripeGeom g;
    g.n = n;
    g.S = n / 2;
    const int key = (fp64 ? 6 : 0) + (den_mode ? 3 : 0) + (tile == 1 ? 1 : tile == 2 ? 2 : 0);
    switch (key) {
    case 0: tile_dims<float, 0, 0>(&g); break;
    case 1: tile_dims<float, 0, 1>(&g); break;
    case 2: tile_dims<float, 0, 2>(&g); break;
    case 3: tile_dims<float, 1, 0>(&g); break;
    case 4: tile_dims<float, 1, 1>(&g); break;
    case 5: tile_dims<float, 1, 2>(&g); break;
    case 6: tile_dims<double, 0, 0>(&g); break;
    case 7: tile_dims<double, 0, 1>(&g); break;
    case 8: tile_dims<double, 0, 2>(&g); break;
    case 9: tile_dims<double, 1, 0>(&g); break;
    case 10: tile_dims<double, 1, 1>(&g); break;
    default: tile_dims<double, 1, 2>(&g); break;
    }
    g.sstride = round_up(n, g.tkw);
    g.spad = (int32_t)round_up(g.S > 0 ? g.S : 1, g.tsw);
    // largest embedding index read: (sstride - tkw) + (spad - tsw) + 1 + (tkw + tsw) - 1
    g.estride = round_up(g.sstride + g.spad + 1, 64);
    return g;
}

template <typename CT>
static hipError_t transform_dispatch(bool fp64, int32_t method, const CT *C, int64_t cstride,
                                     int32_t slot0, int32_t E, const int32_t *totals, int32_t n,
                                     int32_t S, void *emb, int64_t estride, hipStream_t st)
{
    dim3 grid(grid1(estride, kBlock), (unsigned)E);
    if (fp64) {
        if (method == UF_WEIGHTED_NORMALIZED)
            k_transform<double, UF_WEIGHTED_NORMALIZED, CT><<<grid, kBlock, 0, st>>>(C, cstride, slot0, totals, n, S, (double *)emb, estride);
        else
            k_transform<double, UF_UNWEIGHTED, CT><<<grid, kBlock, 0, st>>>(C, cstride, slot0, totals, n, S, (double *)emb, estride);
    } else {
        if (method == UF_WEIGHTED_NORMALIZED)
            k_transform<float, UF_WEIGHTED_NORMALIZED, CT><<<grid, kBlock, 0, st>>>(C, cstride, slot0, totals, n, S, (float *)emb, estride);
        else
            k_transform<float, UF_UNWEIGHTED, CT><<<grid, kBlock, 0, st>>>(C, cstride, slot0, totals, n, S, (float *)emb, estride);
    }
    return hipGetLastError();
}

hipError_t launch_transform(bool fp64, int32_t method, const void *C, int32_t cw, int64_t cstride,
                            int32_t slot0, int32_t E, const int32_t *totals, int32_t n, int32_t S,
                            void *emb, int64_t estride, hipStream_t st)
{
    if (E <= 0) return hipSuccess;
    if (cw == 2)
        return transform_dispatch(fp64, method, static_cast<const uint16_t *>(C), cstride, slot0, E,
                                  totals, n, S, emb, estride, st);
    return transform_dispatch(fp64, method, static_cast<const int32_t *>(C), cstride, slot0, E,
                              totals, n, S, emb, estride, st);
}

hipError_t launch_stripe(bool fp64, int32_t method, int32_t den_mode, const void *emb,
                         int64_t estride, const double *len, int32_t E, double *num, double *den,
                         const StripeGeom &g, bool first, hipStream_t st)
{
    if (E <= 0) return hipSuccess;
    if (fp64) return stripe_dispatch<double>(method, den_mode, emb, estride, len, E, num, den, g, first, st);
    return stripe_dispatch<float>(method, den_mode, emb, estride, len, E, num, den, g, first, st);
}

hipError_t launch_inv_totals(const int32_t *totals, int32_t n, double *inv_t, hipStream_t st)
{
    k_inv_totals<<<grid1(n, kBlock), kBlock, 0, st>>>(totals, n, inv_t);
    return hipGetLastError();
}

template <typename T, int TILE, typename CT>
static hipError_t fused_dispatch(const StripeArgs &a, int32_t den_mode, const StripeGeom &g,
                                 hipStream_t st)
{
    dim3 grid((unsigned)a.tiles_k, (unsigned)a.tiles_s, (unsigned)a.kz);
#define UF_FUSED(M, D) k_stripe_fused<T, M, D, TILE, CT><<<grid, kBlock, 0, st>>>(a)
    if (a.method == UF_WEIGHTED_NORMALIZED) {
        if (den_mode == 0) UF_FUSED(UF_WEIGHTED_NORMALIZED, 0); else UF_FUSED(UF_WEIGHTED_NORMALIZED, 1);
    } else {
        if (den_mode == 0) UF_FUSED(UF_UNWEIGHTED, 0); else UF_FUSED(UF_UNWEIGHTED, 1);
    }
#undef UF_FUSED
    return hipGetLastError();
}

hipError_t launch_stripe_fused(bool fp64, int32_t method, int32_t den_mode, int32_t tile,
                               const void *C, int32_t cw, int64_t cstride, const double *inv_t,
                               const double *len, int32_t B, int32_t E, double *num, double *den,
                               const StripeGeom &g, int32_t tile_s0, int32_t tile_s1,
                               int32_t kz, int64_t zstride, bool store_first, hipStream_t st)
{
    if (B <= 0 || tile_s1 <= tile_s0) return hipSuccess;
    StripeArgs a = make_stripe_args(method, C, cw, cstride, inv_t, len, B, E, num, den, g);
    a.s_base = tile_s0 * g.tsw;
    a.tiles_s = tile_s1 - tile_s0;
    a.kz = kz < 1 ? 1 : kz;
    a.zstride = zstride;
    a.store_first = store_first ? 1 : 0;
    const int key = (fp64 ? 6 : 0) + 2 * (tile == 1 ? 1 : tile == 2 ? 2 : 0) + (cw == 2 ? 1 : 0);
    switch (key) {
    case 0: return fused_dispatch<float, 0, int32_t>(a, den_mode, g, st);
    case 1: return fused_dispatch<float, 0, uint16_t>(a, den_mode, g, st);
    case 2: return fused_dispatch<float, 1, int32_t>(a, den_mode, g, st);
    case 3: return fused_dispatch<float, 1, uint16_t>(a, den_mode, g, st);
    case 4: return fused_dispatch<float, 2, int32_t>(a, den_mode, g, st);
    case 5: return fused_dispatch<float, 2, uint16_t>(a, den_mode, g, st);
    case 6: return fused_dispatch<double, 0, int32_t>(a, den_mode, g, st);
    case 7: return fused_dispatch<double, 0, uint16_t>(a, den_mode, g, st);
    case 8: return fused_dispatch<double, 1, int32_t>(a, den_mode, g, st);
    case 9: return fused_dispatch<double, 1, uint16_t>(a, den_mode, g, st);
    case 10: return fused_dispatch<double, 2, int32_t>(a, den_mode, g, st);
    default: return fused_dispatch<double, 2, uint16_t>(a, den_mode, g, st);
    }
}

StripeArgs make_stripe_args(int32_t method, const void *C, int32_t cw, int64_t cstride,
                            const double *inv_t, const double *len, int32_t B, int32_t E,
                            double *num, double *den, const StripeGeom &g)
{
    StripeArgs a;
    a.C = C;
    a.cw = cw;
    a.pad = 0;
    a.cstride = cstride;
    a.inv_t = inv_t;
    a.len = len;
    a.B = B;
    a.E = E;
    a.n = g.n;
    a.S = g.S;
    a.num = num;
    a.den = den;
    a.sstride = g.sstride;
    a.method = method;
    a.tiles_k = (int32_t)(g.sstride / g.tkw);
    a.tiles_s = g.spad / g.tsw;
    a.s_base = 0;
    a.kz = 1;
    a.store_first = 0;
    a.zstride = 0;
    return a;
}

hipError_t launch_stripe_queue(bool fp64, int32_t method, int32_t cw, int32_t den_mode, int32_t tile,
                               const StripeArgs *jobs, const int32_t *items_xy, int32_t n_items,
                               int32_t *counter, int32_t n_groups, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    const int2 *it = reinterpret_cast<const int2 *>(items_xy);
    const bool wn = (method == UF_WEIGHTED_NORMALIZED), c16 = (cw == 2);
#define UF_Q(T, M, D, TL, CT) k_stripe_queue<T, M, D, TL, CT><<<n_groups, kBlock, 0, st>>>(jobs, it, n_items, counter)
#define UF_QM(T, D, TL)                                                             \
    do {                                                                            \
        if (wn) {                                                                   \
            if (c16) UF_Q(T, UF_WEIGHTED_NORMALIZED, D, TL, uint16_t);              \
            else UF_Q(T, UF_WEIGHTED_NORMALIZED, D, TL, int32_t);                   \
        } else {                                                                    \
            if (c16) UF_Q(T, UF_UNWEIGHTED, D, TL, uint16_t);                       \
            else UF_Q(T, UF_UNWEIGHTED, D, TL, int32_t);                            \
        }                                                                           \
    } while (0)
    const int key = (fp64 ? 6 : 0) + (den_mode ? 3 : 0) + (tile == 1 ? 1 : tile == 2 ? 2 : 0);
    switch (key) {
    case 0: UF_QM(float, 0, 0); break;
    case 1: UF_QM(float, 0, 1); break;
    case 2: UF_QM(float, 0, 2); break;
    case 3: UF_QM(float, 1, 0); break;
    case 4: UF_QM(float, 1, 1); break;
    case 5: UF_QM(float, 1, 2); break;
    case 6: UF_QM(double, 0, 0); break;
    case 7: UF_QM(double, 0, 1); break;
    case 8: UF_QM(double, 0, 2); break;
    case 9: UF_QM(double, 1, 0); break;
    case 10: UF_QM(double, 1, 1); break;
    default: UF_QM(double, 1, 2); break;
    }
#undef UF_QM
#undef UF_Q
    return hipGetLastError();
}

hipError_t launch_reduce_z(double *x, int64_t zstride, int32_t kz, int64_t count, hipStream_t st)
{
    if (kz <= 1 || count <= 0) return hipSuccess;
    k_reduce_z<<<grid1(count, kBlock), kBlock, 0, st>>>(x, zstride, kz, count);
    return hipGetLastError();
}

int32_t rowdot_chunk_len(int32_t n, int32_t E)
{
    // about 2,048 work-groups, chunks of at least 64 branches
    const int64_t groups = (n + kBlock - 1) / kBlock;
    int64_t want = std::max<int64_t>(1, (2048 + groups - 1) / groups);
    want = std::min<int64_t>(want, std::max<int64_t>(1, ((int64_t)E + 63) / 64));
    return (int32_t)std::max<int64_t>(1, ((int64_t)E + want - 1) / want);
}

size_t rowdot_scratch_elems(int32_t n, int32_t E)
{
    if (n <= 0 || E <= 0) return 1;
    const int32_t ch = rowdot_chunk_len(n, E);
    return (size_t)((E + ch - 1) / ch) * (size_t)n;
}

hipError_t launch_rowdot(int32_t method, const void *C, int32_t cw, int64_t cstride, int32_t slot0,
                         int32_t E, const int32_t *totals, const double *len, int32_t n,
                         double *D, bool first, double *part, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int f = first ? 1 : 0;
    const int32_t ch = rowdot_chunk_len(n, E);
    const int32_t n_chunks = E > 0 ? (E + ch - 1) / ch : 0;
    const dim3 grid(grid1(n, kBlock), (unsigned)std::max(n_chunks, 1));
#define UF_RD(M, CT) k_rowdot_part<M, CT><<<grid, kBlock, 0, st>>>(static_cast<const CT *>(C), cstride, slot0, E, ch, len, n, part)
    if (n_chunks > 0) {
        if (method == UF_WEIGHTED_NORMALIZED) {
            if (cw == 2) UF_RD(UF_WEIGHTED_NORMALIZED, uint16_t); else UF_RD(UF_WEIGHTED_NORMALIZED, int32_t);
        } else {
            if (cw == 2) UF_RD(UF_UNWEIGHTED, uint16_t); else UF_RD(UF_UNWEIGHTED, int32_t);
        }
        const hipError_t r = hipGetLastError();
        if (r != hipSuccess) return r;
    }
#undef UF_RD
    if (method == UF_WEIGHTED_NORMALIZED)
        k_rowdot_sum<UF_WEIGHTED_NORMALIZED><<<grid1(n, kBlock), kBlock, 0, st>>>(part, n_chunks, totals, n, D, f);
    else
        k_rowdot_sum<UF_UNWEIGHTED><<<grid1(n, kBlock), kBlock, 0, st>>>(part, n_chunks, totals, n, D, f);
    return hipGetLastError();
}

hipError_t launch_condense(int32_t method, const double *num, const double *den, const double *D,
                           int64_t sstride, int32_t n, int32_t S, int32_t out_f32, void *out,
                           hipStream_t st)
{
    if (n < 2) return hipSuccess;
    if (method == UF_WEIGHTED_UNNORMALIZED) {
        if (out_f32)
            k_condense<UF_WEIGHTED_UNNORMALIZED, float><<<n - 1, kBlock, 0, st>>>(num, den, D, sstride, n, S, (float *)out);
        else
            k_condense<UF_WEIGHTED_UNNORMALIZED, double><<<n - 1, kBlock, 0, st>>>(num, den, D, sstride, n, S, (double *)out);
    } else if (method == UF_WEIGHTED_NORMALIZED) {
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

namespace ufmi {

hipError_t launch_condense_range(int32_t method, const double *num, const double *den, const double *D,
                                 int64_t sstride, int32_t n, int32_t S, int32_t s_base,
                                 int32_t s_begin, int32_t s_end, int32_t out_f32, void *out,
                                 hipStream_t st, int32_t layout, const int64_t *row_off)
{
    if (s_end <= s_begin || n < 2) return hipSuccess;
    dim3 grid(grid1(n, kBlock), (unsigned)(s_end - s_begin));
#define UF_CR(M, O, L) k_condense_range<M, O, L><<<grid, kBlock, 0, st>>>(num, den, D, sstride, n, S, s_base, s_begin, s_end, row_off, (O *)out)
#define UF_CRL(M, O)                                                   \
    do {                                                               \
        if (layout == RANGE_BLOCK) UF_CR(M, O, RANGE_BLOCK);           \
        else if (layout == RANGE_COMPACT) UF_CR(M, O, RANGE_COMPACT);  \
        else UF_CR(M, O, RANGE_CONDENSED);                             \
    } while (0)
    if (method == UF_WEIGHTED_UNNORMALIZED) {
        if (out_f32) UF_CRL(UF_WEIGHTED_UNNORMALIZED, float); else UF_CRL(UF_WEIGHTED_UNNORMALIZED, double);
    } else if (method == UF_WEIGHTED_NORMALIZED) {
        if (out_f32) UF_CRL(UF_WEIGHTED_NORMALIZED, float); else UF_CRL(UF_WEIGHTED_NORMALIZED, double);
    } else {
        if (out_f32) UF_CRL(UF_UNWEIGHTED, float); else UF_CRL(UF_UNWEIGHTED, double);
    }
#undef UF_CRL
#undef UF_CR
    return hipGetLastError();
}

hipError_t launch_merge_block(const void *block, int32_t n, int32_t s_begin, int32_t s_end, int32_t f32,
                              void *condensed, hipStream_t st)
{
    if (s_end <= s_begin || n < 2) return hipSuccess;
    dim3 grid(grid1(n, kBlock), (unsigned)(s_end - s_begin));
    if (f32)
        k_merge_block<float><<<grid, kBlock, 0, st>>>(static_cast<const float *>(block), n, n / 2, s_begin,
                                                     static_cast<float *>(condensed));
    else
        k_merge_block<double><<<grid, kBlock, 0, st>>>(static_cast<const double *>(block), n, n / 2, s_begin,
                                                      static_cast<double *>(condensed));
    return hipGetLastError();
}

}  // namespace ufmi
