// Mantel test between two condensed distance matrices, the paper's precision criterion for
// the fp32 code path (Section 4: fp32 and fp64 matrices agree with Mantel R^2 0.99999).
//
// r is Pearson's correlation over all pairs.  For a permutation pi of the samples the
// second matrix is relabelled, y'_ij = y_{pi(i) pi(j)}; the sums of y and y^2 do not change,
// so each permutation needs only the cross sum sum_ij x_ij y'_ij.  One work-group per
// (row i, permutation) gathers that row's terms and writes a partial sum; a second pass adds
// the partials of each permutation in row order, so the result is deterministic.
#include <cmath>

#include "uf_runtime.h"

namespace ufmi {

namespace {

constexpr int kBlock = 256;

__device__ inline int64_t cidx(int64_t n, int64_t i, int64_t j)
{
    const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    return n * lo - lo * (lo + 1) / 2 + (hi - lo - 1);
}

// partial[p][i] = sum_{j > i} x_ij * y_{pi(i) pi(j)}; the identity when perms == nullptr.
__global__ void k_mantel_rows(const double *__restrict__ x, const double *__restrict__ y, int32_t n,
                              const int32_t *__restrict__ perms, double *__restrict__ partial)
{
    __shared__ double red[kBlock];
    const int32_t i = blockIdx.x;
    const int32_t p = blockIdx.y;
    const int32_t *pi = perms ? perms + (int64_t)p * n : nullptr;
    const int64_t row0 = (int64_t)n * i - (int64_t)i * (i + 1) / 2 - i - 1;
    const int32_t ii = pi ? pi[i] : i;
    double acc = 0.0;
    for (int32_t j = i + 1 + threadIdx.x; j < n; j += kBlock) {
        const int32_t jj = pi ? pi[j] : j;
        // permutations are validated before this launch; the guard keeps every access in
        // bounds regardless
        if (ii >= 0 && ii < n && jj >= 0 && jj < n && ii != jj)
            acc = fma(x[row0 + j], y[cidx(n, ii, jj)], acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)p * n + i] = red[0];
}

// sums[0..3] = sum x, sum y, sum x^2, sum y^2 (row partials, then added in order).
__global__ void k_mantel_moments(const double *__restrict__ x, const double *__restrict__ y,
                                 int32_t n, double *__restrict__ partial4)
{
    __shared__ double red[4][kBlock];
    const int32_t i = blockIdx.x;
    const int64_t row0 = (int64_t)n * i - (int64_t)i * (i + 1) / 2 - i - 1;
    double a = 0, b = 0, c = 0, d = 0;
    for (int32_t j = i + 1 + threadIdx.x; j < n; j += kBlock) {
        const double xv = x[row0 + j], yv = y[row0 + j];
        a += xv;
        b += yv;
        c = fma(xv, xv, c);
        d = fma(yv, yv, d);
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    red[2][threadIdx.x] = c;
    red[3][threadIdx.x] = d;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) partial4[(int64_t)q * n + i] = red[q][0];
}

// Flags (*bad = 1) any permutation with an entry outside [0, n) or a repeated entry.
// seen: n_perm * ceil(n/32) zeroed words.
__global__ void k_perm_check(const int32_t *__restrict__ perms, int32_t n, int32_t n_perm,
                             uint32_t *__restrict__ seen, int32_t *__restrict__ bad)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * n_perm) return;
    const int32_t p = (int32_t)(t / n);
    const int32_t v = perms[t];
    if (v < 0 || v >= n) {
        atomicOr(bad, 1);
        return;
    }
    const int64_t words = (n + 31) / 32;
    const uint32_t bit = 1u << (v & 31);
    if (atomicOr(seen + p * words + (v >> 5), bit) & bit) atomicOr(bad, 1);
}

// out[r] = sum_i partial[r][i] in row order, one thread per row of partials.
__global__ void k_rowsum(const double *__restrict__ partial, int32_t n, int32_t rows,
                         double *__restrict__ out)
{
    const int32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= rows) return;
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += partial[(int64_t)r * n + i];
    out[r] = s;
}

}  // namespace

}  // namespace ufmi

using namespace ufmi;

extern "C" uf_status uf_mantel(uf_context *ctx, const double *x, const double *y, int32_t n,
                               const int32_t *perms, int32_t n_perm, double *r_out,
                               double *r_perm_out, double *p_out, void *stream)
{
    if (!ctx || !x || !y || !r_out || n < 3 || n_perm < 0 || (n_perm > 0 && !perms))
        return set_err(ctx, UF_E_ARG, "invalid Mantel arguments (need n >= 3)");
    UF_TRY(enter_device(ctx->device), "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n_perm > 0) {
        const int64_t words = (int64_t)n_perm * ((n + 31) / 32);
        DevMem seen;
        UF_TRY(seen.ensure((size_t)(words + 1) * sizeof(uint32_t)), "allocating permutation check");
        UF_TRY(launch_fill_u32(seen.p, 0u, (size_t)(words + 1), st), "clearing permutation check");
        int32_t *bad = reinterpret_cast<int32_t *>(seen.as<uint32_t>() + words);
        const int64_t total = (int64_t)n * n_perm;
        k_perm_check<<<(unsigned)((total + kBlock - 1) / kBlock), kBlock, 0, st>>>(
            perms, n, n_perm, seen.as<uint32_t>(), bad);
        UF_TRY(hipGetLastError(), "permutation check");
        int32_t hbad = 0;
        UF_TRY(hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, st), "reading check");
        UF_TRY(hipStreamSynchronize(st), "synchronizing");
        if (hbad) return set_err(ctx, UF_E_ARG, "perms holds a row that is not a permutation of 0..n-1");
    }
    const int32_t rows = n_perm + 1 + 4;
    DevMem partial, sums;
    UF_TRY(partial.ensure((size_t)rows * n * sizeof(double)), "allocating Mantel partials");
    UF_TRY(sums.ensure((size_t)rows * sizeof(double)), "allocating Mantel sums");
    double *P = partial.as<double>();
    // row 0: the observed cross sum; rows 1..n_perm: permuted; last 4: moments
    UF_TRY(launch_fill_u32(P, 0u, (size_t)rows * n * 2, st), "clearing partials");
    k_mantel_rows<<<dim3(n - 1, 1), kBlock, 0, st>>>(x, y, n, nullptr, P);
    UF_TRY(hipGetLastError(), "Mantel rows");
    for (int32_t p0 = 0; p0 < n_perm; p0 += 65535) {
        const int32_t pc = std::min(65535, n_perm - p0);
        k_mantel_rows<<<dim3(n - 1, pc), kBlock, 0, st>>>(x, y, n, perms + (int64_t)p0 * n,
                                                          P + (int64_t)(1 + p0) * n);
        UF_TRY(hipGetLastError(), "Mantel permutations");
    }
    k_mantel_moments<<<n - 1, kBlock, 0, st>>>(x, y, n, P + (int64_t)(1 + n_perm) * n);
    UF_TRY(hipGetLastError(), "Mantel moments");
    k_rowsum<<<(rows + kBlock - 1) / kBlock, kBlock, 0, st>>>(P, n, rows, sums.as<double>());
    UF_TRY(hipGetLastError(), "Mantel sums");
    std::vector<double> h(rows);
    UF_TRY(hipMemcpyAsync(h.data(), sums.p, rows * sizeof(double), hipMemcpyDeviceToHost, st),
           "copying Mantel sums");
    UF_TRY(hipStreamSynchronize(st), "synchronizing");
    const double m = (double)n * (n - 1) / 2;
    const double sx = h[n_perm + 1], sy = h[n_perm + 2], sxx = h[n_perm + 3], syy = h[n_perm + 4];
    const double vx = sxx - sx * sx / m, vy = syy - sy * sy / m;
    const double denom = std::sqrt(vx * vy);
    auto corr = [&](double sxy) { return denom > 0 ? (sxy - sx * sy / m) / denom : 0.0; };
    const double r = corr(h[0]);
    *r_out = r;
    int64_t ge = 0;
    for (int32_t p = 0; p < n_perm; ++p) {
        const double rp = corr(h[1 + p]);
        if (r_perm_out) r_perm_out[p] = rp;
        if (std::fabs(rp) >= std::fabs(r)) ++ge;
    }
    if (p_out) *p_out = n_perm > 0 ? (double)(ge + 1) / (double)(n_perm + 1) : 1.0;
    return UF_OK;
}
