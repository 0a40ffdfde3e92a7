// (a) Level-synchronous embedding propagation.
//
// The paper's kernels consume one input buffer per branch, an embedding of how much of
// every sample sits below that branch, produced by a CPU section (Section 3).  Here the
// embeddings are built on the GPU: tip rows are scattered from the CSR table, then every
// height level of the tree is one launch in which each internal node gathers the sum of
// its children's rows.  Children always live in lower levels, so each level only reads
// finished rows and writes its own: no atomics between levels and a deterministic result.
// Rows are sample-contiguous, so every gather is a coalesced 16-byte-per-lane stream.
#include "uf_internal.h"

namespace ufmi {

namespace {

constexpr int kBlock = 256;

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t value, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = value;
}

// One wave per sample; its lanes stride over the sample's CSR entries.  Duplicate
// features in a row land on the same element, hence the (exact, integer) atomic add.
template <int CW>
__global__ void k_scatter_counts(const int64_t *__restrict__ indptr,
                                 const int32_t *__restrict__ entry_slot,
                                 const int32_t *__restrict__ entry_count,
                                 void *__restrict__ C, int64_t cstride, int32_t n_samples)
{
    const int32_t k = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (k >= n_samples) return;
    const int lane = threadIdx.x & 63;
    const int64_t e1 = indptr[k + 1];
    for (int64_t e = indptr[k] + lane; e < e1; e += 64) {
        const int64_t at = (int64_t)entry_slot[e] * cstride + k;
        if (CW == 4)
            atomicAdd(static_cast<int32_t *>(C) + at, entry_count[e]);
        else   // add into the half of the 32-bit word that holds element `at`
            atomicAdd(static_cast<uint32_t *>(C) + (at >> 1), (uint32_t)entry_count[e] << (16 * (at & 1)));
    }
}

__global__ void k_scatter_bits(const int64_t *__restrict__ indptr,
                               const int32_t *__restrict__ entry_slot,
                               const int32_t *__restrict__ entry_count,
                               uint32_t *__restrict__ B, int64_t bstride, int32_t n_samples)
{
    const int32_t k = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (k >= n_samples) return;
    const int lane = threadIdx.x & 63;
    const int64_t e1 = indptr[k + 1];
    const uint32_t bit = 1u << (k & 31);
    for (int64_t e = indptr[k] + lane; e < e1; e += 64)
        if (entry_count[e] > 0)
            atomicOr(B + (int64_t)entry_slot[e] * bstride + (k >> 5), bit);
}

// Rows [slot_begin, slot_begin + n_rows) are the internal nodes of one height level.
// blockIdx.x walks 16-byte columns of a row, blockIdx.y (strided) walks the rows.
template <bool OR>
__global__ void k_level(uint32_t *__restrict__ X, int64_t stride, int32_t n_vec,
                        int32_t slot_begin, int32_t n_rows, int32_t n_leaf,
                        const int32_t *__restrict__ child_ptr,
                        const int32_t *__restrict__ child_slot)
{
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= n_vec) return;
    for (int32_t r = blockIdx.y; r < n_rows; r += gridDim.y) {
        const int32_t slot = slot_begin + r;
        const int32_t i = slot - n_leaf;
        const int32_t q0 = child_ptr[i], q1 = child_ptr[i + 1];
        uint4 acc = make_uint4(0u, 0u, 0u, 0u);
        for (int32_t q = q0; q < q1; ++q) {
            const uint4 v = reinterpret_cast<const uint4 *>(X + (int64_t)child_slot[q] * stride)[c];
            if (OR) {
                acc.x |= v.x; acc.y |= v.y; acc.z |= v.z; acc.w |= v.w;
            } else {
                acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
            }
        }
        reinterpret_cast<uint4 *>(X + (int64_t)slot * stride)[c] = acc;
    }
}

// The narrow top of a deep tree in one launch: work-group g owns uint4 columns
// [g * kTailCols, (g + 1) * kTailCols) of every row and walks the tail's levels in order with
// a barrier between them.  A node's children sit in lower levels, computed either by earlier
// launches or by this same work-group for these same columns, so no other work-group is ever
// waited for; the barrier's workgroup-scope fence makes a level's stores visible to the next
// level's loads (one CU, one L1).  The tail's topology (TailProgram) is staged into LDS a
// chunk of levels at a time, so that a level waits only on its row loads.
constexpr int kTailCols = 16;
template <bool OR>
__global__ void k_level_tail(uint32_t *__restrict__ X, int64_t stride, int32_t n_vec, TailProgram tp)
{
    __shared__ int32_t s_lvl[kTailMaxLevels + 1];
    __shared__ int4 s_rec[kTailMaxNodes];     // (slot, first kid, end kid, 0), kids chunk-relative
    __shared__ int32_t s_kid[kTailMaxKids];
    const int32_t c = blockIdx.x * kTailCols + (int32_t)(threadIdx.x % kTailCols);
    const int32_t lane = (int32_t)(threadIdx.x / kTailCols);
    constexpr int32_t kLanes = kBlock / kTailCols;
    for (int32_t ch = 0; ch < tp.n_chunks; ++ch) {
        const int2 lv = tp.chunks[ch];                     // levels [lv.x, lv.y) of the tail
        const int32_t r0 = tp.lvl[lv.x], r1 = tp.lvl[lv.y];
        const int32_t k0 = tp.rec[r0].y, k1 = tp.rec[r1 - 1].z;
        for (int32_t i = threadIdx.x; i <= lv.y - lv.x; i += kBlock) s_lvl[i] = tp.lvl[lv.x + i] - r0;
        for (int32_t i = threadIdx.x; i < r1 - r0; i += kBlock) {
            int4 r = tp.rec[r0 + i];
            r.y -= k0;
            r.z -= k0;
            s_rec[i] = r;
        }
        for (int32_t i = threadIdx.x; i < k1 - k0; i += kBlock) s_kid[i] = tp.kid[k0 + i];
        __syncthreads();
        for (int32_t h = 0; h < lv.y - lv.x; ++h) {
            const int32_t b = s_lvl[h], e = s_lvl[h + 1];
            if (c < n_vec) {
                for (int32_t i = b + lane; i < e; i += kLanes) {
                    const int4 r = s_rec[i];
                    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
                    for (int32_t q = r.y; q < r.z; ++q) {
                        const uint4 v = reinterpret_cast<const uint4 *>(X + (int64_t)s_kid[q] * stride)[c];
                        if (OR) {
                            acc.x |= v.x; acc.y |= v.y; acc.z |= v.z; acc.w |= v.w;
                        } else {
                            acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
                        }
                    }
                    reinterpret_cast<uint4 *>(X + (int64_t)r.x * stride)[c] = acc;
                }
            }
            __syncthreads();
        }
    }
}

__global__ void k_gather_rows_u16(const uint16_t *__restrict__ src, int64_t sstride,
                                  const int32_t *__restrict__ slot_of_node, int32_t n_nodes,
                                  int32_t width, int32_t *__restrict__ out)
{
    const int32_t x = blockIdx.x * kBlock + threadIdx.x;
    if (x >= width) return;
    for (int32_t v = blockIdx.y; v < n_nodes; v += gridDim.y)
        out[(int64_t)v * width + x] = (int32_t)src[(int64_t)slot_of_node[v] * sstride + x];
}

__global__ void k_gather_rows(const uint32_t *__restrict__ src, int64_t sstride,
                              const int32_t *__restrict__ slot_of_node, int32_t n_nodes,
                              int32_t width, uint32_t *__restrict__ out)
{
    const int32_t x = blockIdx.x * kBlock + threadIdx.x;
    if (x >= width) return;
    for (int32_t v = blockIdx.y; v < n_nodes; v += gridDim.y)
        out[(int64_t)v * width + x] = src[(int64_t)slot_of_node[v] * sstride + x];
}

inline unsigned grid1(size_t n, size_t per) { return (unsigned)((n + per - 1) / per); }

// Many jobs at once: one launch scatters the tips of every job, and one launch per height
// level gathers that level of every job (tasks are (job, slot) pairs), so a batch of jobs
// costs max-height launches rather than the sum of the heights.
__global__ void k_scatter_batched(const PropJob *__restrict__ jobs, const int2 *__restrict__ tasks,
                                  int32_t n_tasks)
{
    const int32_t t = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (t >= n_tasks) return;
    const int2 task = tasks[t];
    const PropJob &J = jobs[task.x];
    const int32_t k = task.y;
    const int lane = threadIdx.x & 63;
    const int64_t e1 = J.indptr[k + 1];
    if (J.mode == 0) {
        int32_t *C = reinterpret_cast<int32_t *>(J.X);
        for (int64_t e = J.indptr[k] + lane; e < e1; e += 64)
            atomicAdd(C + (int64_t)J.entry_slot[e] * J.stride + k, J.entry_count[e]);
    } else if (J.mode == 2) {   // uint16 counts, 2 * stride elements per row
        for (int64_t e = J.indptr[k] + lane; e < e1; e += 64) {
            const int64_t at = (int64_t)J.entry_slot[e] * (2 * J.stride) + k;
            atomicAdd(J.X + (at >> 1), (uint32_t)J.entry_count[e] << (16 * (at & 1)));
        }
    } else {
        const uint32_t bit = 1u << (k & 31);
        for (int64_t e = J.indptr[k] + lane; e < e1; e += 64)
            if (J.entry_count[e] > 0) atomicOr(J.X + (int64_t)J.entry_slot[e] * J.stride + (k >> 5), bit);
    }
}

__global__ void k_level_batched(const PropJob *__restrict__ jobs, const int2 *__restrict__ tasks,
                                int32_t n_tasks)
{
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    for (int32_t r = blockIdx.y; r < n_tasks; r += gridDim.y) {
        const int2 task = tasks[r];
        const PropJob &J = jobs[task.x];
        if (c >= (int32_t)(J.stride / 4)) continue;
        const int32_t i = task.y - J.n_leaf;
        const int32_t q0 = J.child_ptr[i], q1 = J.child_ptr[i + 1];
        uint4 acc = make_uint4(0u, 0u, 0u, 0u);
        for (int32_t q = q0; q < q1; ++q) {
            const uint4 v = reinterpret_cast<const uint4 *>(J.X + (int64_t)J.child_slot[q] * J.stride)[c];
            if (J.mode == 1) {
                acc.x |= v.x; acc.y |= v.y; acc.z |= v.z; acc.w |= v.w;
            } else {
                acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
            }
        }
        reinterpret_cast<uint4 *>(J.X + (int64_t)task.y * J.stride)[c] = acc;
    }
}

// max |a - b| over n elements into *out (which the launcher clears first).  Non-negative
// doubles order like their bit patterns, so an integer atomicMax combines work-groups.
__global__ void k_max_abs_diff(const double *__restrict__ a, const double *__restrict__ b, int64_t n,
                               unsigned long long *__restrict__ out)
{
    __shared__ double red[kBlock];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double d = fabs(a[i] - b[i]);
        m = (d > m || d != d) ? (d != d ? INFINITY : d) : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

}  // namespace

hipError_t launch_max_abs_diff(const double *a, const double *b, int64_t n, double *out, hipStream_t st)
{
    hipError_t e = launch_fill_u32(out, 0u, 2, st);
    if (e != hipSuccess || n <= 0) return e;
    size_t blocks = grid1((size_t)n, kBlock * 16);
    if (blocks > 4096) blocks = 4096;
    k_max_abs_diff<<<(unsigned)blocks, kBlock, 0, st>>>(a, b, n, reinterpret_cast<unsigned long long *>(out));
    return hipGetLastError();
}

hipError_t launch_fill_u32(void *p, uint32_t value, size_t n_words, hipStream_t st)
{
    if (n_words == 0) return hipSuccess;
    size_t blocks = grid1(n_words, kBlock * 8);
    if (blocks > 65536) blocks = 65536;
    k_fill_u32<<<(unsigned)blocks, kBlock, 0, st>>>((uint32_t *)p, value, n_words);
    return hipGetLastError();
}

hipError_t launch_scatter_counts(const int64_t *indptr, const int32_t *entry_slot,
                                 const int32_t *entry_count, void *C, int32_t cw, int64_t cstride,
                                 int32_t n_samples, hipStream_t st)
{
    if (cw == 2)
        k_scatter_counts<2><<<grid1(n_samples, kBlock / 64), kBlock, 0, st>>>(
            indptr, entry_slot, entry_count, C, cstride, n_samples);
    else
        k_scatter_counts<4><<<grid1(n_samples, kBlock / 64), kBlock, 0, st>>>(
            indptr, entry_slot, entry_count, C, cstride, n_samples);
    return hipGetLastError();
}

hipError_t launch_gather_rows_u16(const uint16_t *src, int64_t sstride, const int32_t *slot_of_node,
                                  int32_t n_nodes, int32_t width, int32_t *out, hipStream_t st)
{
    if (n_nodes <= 0 || width <= 0) return hipSuccess;
    dim3 grid(grid1(width, kBlock), (unsigned)(n_nodes < 65535 ? n_nodes : 65535));
    k_gather_rows_u16<<<grid, kBlock, 0, st>>>(src, sstride, slot_of_node, n_nodes, width, out);
    return hipGetLastError();
}

hipError_t launch_scatter_bits(const int64_t *indptr, const int32_t *entry_slot,
                               const int32_t *entry_count, uint32_t *B, int64_t bstride,
                               int32_t n_samples, hipStream_t st)
{
    k_scatter_bits<<<grid1(n_samples, kBlock / 64), kBlock, 0, st>>>(
        indptr, entry_slot, entry_count, B, bstride, n_samples);
    return hipGetLastError();
}

static hipError_t launch_level(bool is_or, uint32_t *X, int64_t stride, int32_t slot_begin,
                               int32_t n_rows, int32_t n_leaf, const int32_t *child_ptr,
                               const int32_t *child_slot, hipStream_t st)
{
    if (n_rows <= 0) return hipSuccess;
    const int32_t n_vec = (int32_t)(stride / 4);
    dim3 grid(grid1(n_vec, kBlock), (unsigned)(n_rows < 65535 ? n_rows : 65535));
    if (is_or)
        k_level<true><<<grid, kBlock, 0, st>>>(X, stride, n_vec, slot_begin, n_rows, n_leaf,
                                               child_ptr, child_slot);
    else
        k_level<false><<<grid, kBlock, 0, st>>>(X, stride, n_vec, slot_begin, n_rows, n_leaf,
                                                child_ptr, child_slot);
    return hipGetLastError();
}

hipError_t launch_level_tail(bool is_or, uint32_t *X, int64_t stride_words, const TailProgram &tp,
                             hipStream_t st)
{
    if (tp.n_chunks <= 0) return hipSuccess;
    const int32_t n_vec = (int32_t)(stride_words / 4);
    const unsigned groups = grid1(n_vec, kTailCols);
    if (is_or)
        k_level_tail<true><<<groups, kBlock, 0, st>>>(X, stride_words, n_vec, tp);
    else
        k_level_tail<false><<<groups, kBlock, 0, st>>>(X, stride_words, n_vec, tp);
    return hipGetLastError();
}

hipError_t launch_level_sum(void *C, int64_t stride_words, int32_t slot_begin, int32_t n_rows,
                            int32_t n_leaf, const int32_t *child_ptr, const int32_t *child_slot,
                            hipStream_t st)
{
    return launch_level(false, static_cast<uint32_t *>(C), stride_words, slot_begin, n_rows,
                        n_leaf, child_ptr, child_slot, st);
}

hipError_t launch_level_or(uint32_t *B, int64_t bstride, int32_t slot_begin, int32_t n_rows,
                           int32_t n_leaf, const int32_t *child_ptr, const int32_t *child_slot,
                           hipStream_t st)
{
    return launch_level(true, B, bstride, slot_begin, n_rows, n_leaf, child_ptr, child_slot, st);
}

hipError_t launch_gather_rows_u32(const uint32_t *src, int64_t sstride, const int32_t *slot_of_node,
                                  int32_t n_nodes, int32_t width, uint32_t *out, hipStream_t st)
{
    if (n_nodes <= 0 || width <= 0) return hipSuccess;
    dim3 grid(grid1(width, kBlock), (unsigned)(n_nodes < 65535 ? n_nodes : 65535));
    k_gather_rows<<<grid, kBlock, 0, st>>>(src, sstride, slot_of_node, n_nodes, width, out);
    return hipGetLastError();
}

}  // namespace ufmi

namespace ufmi {

hipError_t launch_scatter_batched(const PropJob *jobs, const int32_t *tasks_xy, int32_t n_tasks,
                                  hipStream_t st)
{
    if (n_tasks <= 0) return hipSuccess;
    k_scatter_batched<<<grid1(n_tasks, kBlock / 64), kBlock, 0, st>>>(
        jobs, reinterpret_cast<const int2 *>(tasks_xy), n_tasks);
    return hipGetLastError();
}

hipError_t launch_level_batched(const PropJob *jobs, const int32_t *tasks_xy, int32_t n_tasks,
                                int32_t max_vec, hipStream_t st)
{
    if (n_tasks <= 0) return hipSuccess;
    dim3 grid(grid1(max_vec, kBlock), (unsigned)(n_tasks < 65535 ? n_tasks : 65535));
    k_level_batched<<<grid, kBlock, 0, st>>>(jobs, reinterpret_cast<const int2 *>(tasks_xy), n_tasks);
    return hipGetLastError();
}

}  // namespace ufmi
