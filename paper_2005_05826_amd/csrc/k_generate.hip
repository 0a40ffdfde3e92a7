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

// Reads of one sample at tip positions < x: entries [a, b) of the sample sorted by position,
// running sums scum.  Binary search for the first entry at or past x.
__device__ inline int32_t reads_below(const int32_t *__restrict__ spos, const int32_t *__restrict__ scum,
                                      int64_t a, int64_t b, int32_t x)
{
    int64_t lo = a, hi = b;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (spos[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo > a ? scum[lo - 1] : 0;
}

// Thread per sample (grid x), rows strided over grid y: writes of one row are coalesced and
// a thread's binary searches stay inside its own sample's entries.
template <typename CT>
__global__ void k_range_counts(const int64_t *__restrict__ indptr, const int32_t *__restrict__ spos,
                               const int32_t *__restrict__ scum, const int32_t *__restrict__ lo,
                               const int32_t *__restrict__ hi, int32_t slot0, int32_t E, int32_t n,
                               CT *__restrict__ out, int64_t ostride)
{
    const int32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t a = indptr[k], b = indptr[k + 1];
    for (int32_t e = blockIdx.y; e < E; e += gridDim.y) {
        const int32_t s = slot0 + e;
        const int32_t c = reads_below(spos, scum, a, b, hi[s]) - reads_below(spos, scum, a, b, lo[s]);
        out[(int64_t)e * ostride + k] = (CT)c;
    }
}

// Sample rows of the matrix-core presence layout strided over grid y, threads over a row's
// bytes (grid x): byte q holds branches slot0 + 8q .. slot0 + 8q + 7.
__global__ void k_range_bits(const int64_t *__restrict__ indptr, const int32_t *__restrict__ spos,
                             const int32_t *__restrict__ scum, const int32_t *__restrict__ lo,
                             const int32_t *__restrict__ hi, int32_t slot0, int32_t Bc, int64_t kbytes,
                             int32_t n, int32_t n_pad, uint8_t *__restrict__ P)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= kbytes) return;
    for (int32_t k = blockIdx.y; k < n_pad; k += gridDim.y) {
        uint32_t byte = 0;
        if (k < n) {
            const int64_t a = indptr[k], b = indptr[k + 1];
            for (int t = 0; t < 8; ++t) {
                const int64_t br = q * 8 + t;
                if (br >= Bc) break;
                const int32_t s = slot0 + (int32_t)br;
                const int32_t c = reads_below(spos, scum, a, b, hi[s]) - reads_below(spos, scum, a, b, lo[s]);
                if (c > 0) byte |= 1u << t;
            }
        }
        P[(int64_t)k * kbytes + q] = (uint8_t)byte;
    }
}

inline unsigned grid1(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_range_counts(const int64_t *indptr, const int32_t *spos, const int32_t *scum,
                               const int32_t *lo, const int32_t *hi, int32_t slot0, int32_t E,
                               int32_t n, void *out, int32_t cw, int64_t ostride, hipStream_t st)
{
    if (E <= 0 || n <= 0) return hipSuccess;
    dim3 grid(grid1(n, kBlock), (unsigned)std::min(E, 1024));
    if (cw == 2)
        k_range_counts<uint16_t><<<grid, kBlock, 0, st>>>(indptr, spos, scum, lo, hi, slot0, E, n,
                                                           static_cast<uint16_t *>(out), ostride);
    else
        k_range_counts<int32_t><<<grid, kBlock, 0, st>>>(indptr, spos, scum, lo, hi, slot0, E, n,
                                                          static_cast<int32_t *>(out), ostride);
    return hipGetLastError();
}

hipError_t launch_range_bits(const int64_t *indptr, const int32_t *spos, const int32_t *scum,
                             const int32_t *lo, const int32_t *hi, int32_t slot0, int32_t Bc,
                             int64_t kpad, int32_t n, int32_t n_pad, uint8_t *P, hipStream_t st)
{
    if (n_pad <= 0 || kpad <= 0) return hipSuccess;
    const int64_t kbytes = kpad / 8;
    dim3 grid(grid1(kbytes, kBlock), (unsigned)std::min(n_pad, 32768));
    k_range_bits<<<grid, kBlock, 0, st>>>(indptr, spos, scum, lo, hi, slot0, Bc, kbytes, n, n_pad, P);
    return hipGetLastError();
}

}  // namespace ufmi
