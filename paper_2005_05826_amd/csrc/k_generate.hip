// (a) Embedding rows generated batch by batch, for problems whose full count rows do not fit
// in device memory.
//
// The paper's kernels take one batch of per-branch input buffers per invocation, produced
// outside the accumulation (Section 3, Fig. 2).  When all branch rows cannot be resident
// (the level propagation needs them all), a batch of rows is computed directly from the
// table: with tips numbered in depth-first order the tips below a node form one range
// [lo, hi), and a sample's reads below the node are the difference of two prefix sums over
// its entries sorted by tip position (two binary searches).  Rows come out exactly equal to
// the propagated ones (integer arithmetic).
#include <algorithm>

#include "uf_internal.h"

namespace ufmi {

namespace {

constexpr int kBlock = 256;
constexpr int kGenThreads = 128;     // threads per sample-staging work-group
constexpr int kGenCap = 2048;        // entries of one sample staged in LDS (16 KB: a work-group fits
                                     // beside the striped kernel's on a CU)
constexpr int kGenGroups = 4096;     // sample-staging work-groups (grid-stride over samples)

// Reads of one sample at tip positions < x: m entries of the sample sorted by position, with
// running sums cum.  Binary search for the first entry at or past x.
__device__ inline int32_t reads_below(const int32_t *__restrict__ pos, const int32_t *__restrict__ cum, int32_t m,
                                      int32_t x)
{
    int32_t lo = 0, hi = m;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (pos[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo > 0 ? cum[lo - 1] : 0;
}

// Stages sample k's entries into LDS when they fit (returns true), after a barrier that
// ends the previous sample's searches.
__device__ inline bool stage_sample(const int32_t *__restrict__ spos, const int32_t *__restrict__ scum,
                                    int64_t a, int32_t m, int32_t *s_pos, int32_t *s_cum)
{
    __syncthreads();
    const bool staged = m <= kGenCap;
    if (staged)
        for (int32_t i = threadIdx.x; i < m; i += kGenThreads) {
            s_pos[i] = spos[a + i];
            s_cum[i] = scum[a + i];
        }
    __syncthreads();
    return staged;
}

// Count rows, sample-major: work-groups take samples in turn, stage the sample's entries in
// LDS once and answer all 2 E searches of the batch from there (the searches of one sample
// share its few kilobytes instead of each touching its own cache lines in HBM); row k of tmp
// gets the sample's E counts.  A sample with more than kGenCap entries searches them in place.
template <typename CT>
__global__ __launch_bounds__(kGenThreads) void k_range_counts(const int64_t *__restrict__ indptr,
                                                              const int32_t *__restrict__ spos,
                                                              const int32_t *__restrict__ scum,
                                                              const int32_t *__restrict__ lo,
                                                              const int32_t *__restrict__ hi, int32_t slot0,
                                                              int32_t E, int32_t n, CT *__restrict__ tmp)
{
    __shared__ int32_t s_pos[kGenCap], s_cum[kGenCap];
    for (int32_t k = blockIdx.x; k < n; k += gridDim.x) {
        const int64_t a = indptr[k];
        const int32_t m = (int32_t)(indptr[k + 1] - a);
        const bool staged = stage_sample(spos, scum, a, m, s_pos, s_cum);
        const int32_t *pp = staged ? s_pos : spos + a;
        const int32_t *pc = staged ? s_cum : scum + a;
        for (int32_t e = threadIdx.x; e < E; e += kGenThreads) {
            const int32_t s = slot0 + e;
            const int32_t c = reads_below(pp, pc, m, hi[s]) - reads_below(pp, pc, m, lo[s]);
            tmp[(int64_t)k * E + e] = (CT)c;
        }
    }
}

// tmp [n][E] -> out [E][ostride] through 32 x 32 LDS tiles (coalesced on both sides).
template <typename CT>
__global__ void k_rows_transpose(const CT *__restrict__ tmp, int32_t n, int32_t E, CT *__restrict__ out,
                                 int64_t ostride)
{
    __shared__ CT t[32][33];
    const int32_t k0 = blockIdx.x * 32, e0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int r = ty; r < 32; r += kBlock / 32) {
        const int32_t k = k0 + r, e = e0 + tx;
        if (k < n && e < E) t[r][tx] = tmp[(int64_t)k * E + e];
    }
    __syncthreads();
#pragma unroll
    for (int r = ty; r < 32; r += kBlock / 32) {
        const int32_t e = e0 + r, k = k0 + tx;
        if (k < n && e < E) out[(int64_t)e * ostride + k] = t[tx][r];
    }
}

// Presence bits in the matrix-core layout, one sample row at a time as above: thread t
// computes dwords t, t + 128, ... of the row (32 branches each, bit b of byte q = branch
// slot0 + 8 q + b); rows k >= n are zero.
__global__ __launch_bounds__(kGenThreads) void k_range_bits(const int64_t *__restrict__ indptr,
                                                            const int32_t *__restrict__ spos,
                                                            const int32_t *__restrict__ scum,
                                                            const int32_t *__restrict__ lo,
                                                            const int32_t *__restrict__ hi, int32_t slot0,
                                                            int32_t Bc, int64_t kbytes, int32_t n, int32_t n_pad,
                                                            uint8_t *__restrict__ P)
{
    __shared__ int32_t s_pos[kGenCap], s_cum[kGenCap];
    const int64_t kwords = kbytes / 4;
    for (int32_t k = blockIdx.x; k < n_pad; k += gridDim.x) {
        uint32_t *row = reinterpret_cast<uint32_t *>(P + (int64_t)k * kbytes);
        if (k >= n) {   // uniform per work-group
            for (int64_t q = threadIdx.x; q < kwords; q += kGenThreads) row[q] = 0u;
            continue;
        }
        const int64_t a = indptr[k];
        const int32_t m = (int32_t)(indptr[k + 1] - a);
        const bool staged = stage_sample(spos, scum, a, m, s_pos, s_cum);
        const int32_t *pp = staged ? s_pos : spos + a;
        const int32_t *pc = staged ? s_cum : scum + a;
        for (int64_t q = threadIdx.x; q < kwords; q += kGenThreads) {
            uint32_t word = 0;
            for (int t = 0; t < 32; ++t) {
                const int64_t br = q * 32 + t;
                if (br >= Bc) break;
                const int32_t s = slot0 + (int32_t)br;
                if (reads_below(pp, pc, m, hi[s]) > reads_below(pp, pc, m, lo[s])) word |= 1u << t;
            }
            row[q] = word;
        }
    }
}

inline unsigned grid1(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_range_counts(const int64_t *indptr, const int32_t *spos, const int32_t *scum,
                               const int32_t *lo, const int32_t *hi, int32_t slot0, int32_t E,
                               int32_t n, void *out, int32_t cw, int64_t ostride, void *tmp, hipStream_t st)
{
    if (E <= 0 || n <= 0) return hipSuccess;
    const unsigned groups = (unsigned)std::min(n, kGenGroups);
    const dim3 tgrid(grid1(n, 32), grid1(E, 32));
    if (cw == 2) {
        k_range_counts<uint16_t><<<groups, kGenThreads, 0, st>>>(indptr, spos, scum, lo, hi, slot0, E, n,
                                                                  static_cast<uint16_t *>(tmp));
        k_rows_transpose<uint16_t><<<tgrid, kBlock, 0, st>>>(static_cast<const uint16_t *>(tmp), n, E,
                                                             static_cast<uint16_t *>(out), ostride);
    } else {
        k_range_counts<int32_t><<<groups, kGenThreads, 0, st>>>(indptr, spos, scum, lo, hi, slot0, E, n,
                                                                 static_cast<int32_t *>(tmp));
        k_rows_transpose<int32_t><<<tgrid, kBlock, 0, st>>>(static_cast<const int32_t *>(tmp), n, E,
                                                            static_cast<int32_t *>(out), ostride);
    }
    return hipGetLastError();
}

hipError_t launch_range_bits(const int64_t *indptr, const int32_t *spos, const int32_t *scum,
                             const int32_t *lo, const int32_t *hi, int32_t slot0, int32_t Bc,
                             int64_t kpad, int32_t n, int32_t n_pad, uint8_t *P, hipStream_t st)
{
    if (n_pad <= 0 || kpad <= 0) return hipSuccess;
    const unsigned groups = (unsigned)std::min(n_pad, kGenGroups);
    k_range_bits<<<groups, kGenThreads, 0, st>>>(indptr, spos, scum, lo, hi, slot0, Bc, kpad / 8, n, n_pad, P);
    return hipGetLastError();
}

}  // namespace ufmi
