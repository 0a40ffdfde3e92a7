// (c) Matrix-core form of unweighted UniFrac.
//
// For 0/1 presence P (samples x branches) and branch lengths L, the branch length shared by
// samples i and j is S_ij = sum_b L_b P_ib P_jb, the entries of P diag(L) P^T; the length
// observed in sample i alone is T_i = S_ii.  Then
//   unique(i, j)   = T_i + T_j - 2 S_ij         (numerator: length seen in exactly one)
//   observed(i, j) = T_i + T_j -   S_ij         (denominator: length seen in either)
// so the pairwise work is one symmetric product, run on bf16 MFMA.  Each length is split
// into two bf16 terms, hi = bf16(L) and lo = bf16(L - hi) (the subtraction is exact in
// FP32), so S = P diag(hi) P^T + P diag(lo) P^T with 0/1 operands exact in bf16.  Products
// accumulate in FP32 inside chunks of k_chunk branches and are added into the FP64 output
// between chunks; the final division is FP64.
//
// Layout: presence is stored once per sample as one bit per branch, [n_pad][k_pad / 8]
// bytes (bit t of byte q = branch 8q + t).  A work-group stages 128 branches of its row and
// column panels at a time and expands the bits to bytes on the way into LDS: 0x00 or 0xFF
// for the row panel, 0x00 or 0x3F for the column panel.  A row-panel byte pair becomes a
// pair of 16-bit masks with one byte permute, and a mask ANDed with the bf16 pattern of 2 hi
// or 2 lo is the row operand; a column-panel byte pair placed in the high bytes of two
// 16-bit halves by one byte permute is already the bf16 pair 0.5 / 0, the column operand.
// Every product (2 hi) * 0.5 equals hi exactly (and (2 lo) * 0.5 equals lo), so the sums are
// those of the operands hi, lo and 1.0.  Each presence byte is expanded through a 256-entry
// table in LDS, and the steps of a stage are software-pipelined: while the matrix
// instructions of one 16-branch step run, the LDS words of the step after next are read, the
// operands of the next one built and an eighth of the next stage expanded.  The lengths of a
// step are the same for the 32 lanes of each K half: a stage's length words are stored so that
// each lane reads its eight (one per step) at once, and each step takes the four hi and four lo
// words of its K half from lanes 0-7 of the lane's 16-lane row by DPP broadcast, folded into
// the ANDs that mask them.
#include "uf_internal.h"

namespace ufmi {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int GM = 128;            // work-group tile: GM x GM outputs, 4 waves of 64 x 64
constexpr int GK = 128;            // branches per LDS stage (16 bytes of presence bits per row)
constexpr int LDK = GK + 8;        // padded LDS row of expanded bytes (conflict-free operand reads)
constexpr uint32_t kRowByte = 0x0000FF00u;   // byte 1: the row-panel byte of a present branch
constexpr uint32_t kColByte = 0x00003F00u;   // byte 1: high byte of bf16 0.5

// round-to-nearest-even FP32 -> bf16 (finite, non-negative inputs)
__device__ inline uint16_t bf16_rne(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Writes 2 hi and 2 lo (the column operand carries the factor 0.5 back); doubling a bf16 is
// exact for every length below 2^127 (larger ones overflow, as lengths beyond the FP32 range
// did already).
__global__ void k_split_lengths(const double *__restrict__ len, int32_t B, int32_t k_pad,
                                uint16_t *__restrict__ hi, uint16_t *__restrict__ lo)
{
    const int32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= k_pad) return;
    uint16_t h = 0, l = 0;
    if (b < B) {
        const float L32 = (float)len[b];
        h = bf16_rne(L32);
        const float rest = L32 - __uint_as_float((uint32_t)h << 16);
        l = bf16_rne(rest < 0.f ? -rest : rest);
        if (rest < 0.f) l |= 0x8000u;
        // the doubling is exact in FP32, and its result is a bf16 value again
        h = bf16_rne(2.f * __uint_as_float((uint32_t)h << 16));
        l = (uint16_t)((l & 0x8000u) | bf16_rne(2.f * __uint_as_float((uint32_t)(l & 0x7FFFu) << 16)));
    }
    hi[b] = h;
    lo[b] = l;
}

// Presence bits [slot][bstride] (bit k%32 of word k/32 = sample k) -> per-sample rows
// Pb[k][b / 8] (bit b % 8 = sample k has a read below branch slot b), one 256-sample x
// 64-branch tile per work-group, transposed through LDS.
__global__ void k_bits_transpose(const uint32_t *__restrict__ bits, int64_t bstride, int32_t B,
                                 int32_t n_pad, int64_t kb, uint8_t *__restrict__ Pb)
{
    __shared__ uint32_t w[64][8];
    const int32_t b0 = blockIdx.x * 64;
    const int32_t k0 = blockIdx.y * 256;
    const int tid = threadIdx.x;
    {   // 64 branch rows x 8 words
        const int r = tid >> 2, c = (tid & 3) * 2;
        const int32_t b = b0 + r;
        for (int q = 0; q < 2; ++q) {
            const int64_t word = k0 / 32 + c + q;
            w[r][c + q] = (b < B && word < bstride) ? bits[(int64_t)b * bstride + word] : 0u;
        }
    }
    __syncthreads();
    const int32_t k = k0 + tid;
    if (k >= n_pad) return;
    const uint32_t sh = tid & 31, wc = tid >> 5;
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int t = 0; t < 32; ++t) {
        lo |= ((w[t][wc] >> sh) & 1u) << t;
        hi |= ((w[32 + t][wc] >> sh) & 1u) << t;
    }
    *reinterpret_cast<uint2 *>(Pb + (int64_t)k * kb + b0 / 8) = make_uint2(lo, hi);
}

// 32 presence bits -> 32 bytes (byte t of dword d <- bit 4d + t): byte 1 of `c` for a set
// bit, byte 0 of `c` (zero) for a clear one.  A nibble times 0x204081 puts its bit t at bit 8t
// (the other partial products land on bits that the mask clears), and the resulting 0 / 1
// selector bytes pick bytes of c.
__device__ inline void expand_bits(uint32_t x, uint32_t c, uint32_t (&out)[8])
{
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const uint32_t nib = (x >> (4 * d)) & 0xFu;
        out[d] = __builtin_amdgcn_perm(c, c, (nib * 0x204081u) & 0x01010101u);
    }
}

// x of lane N of the calling lane's 16-lane row (DPP row_newbcast)
template <int N>
__device__ inline uint32_t row_bcast(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x150 + N, 0xF, 0xF, false);
}

__device__ inline bf16x8 as_bf16x8(uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 v = {a, b, c, d};
    return __builtin_bit_cast(bf16x8, v);
}

// Two LDS stages: the next stage's global loads are in flight while this one computes.
// hl holds the stage's hi and lo split words (two branches each) in reading order: the word
// of step kk (16 branches), K half g and position p (0-3 hi, 4-7 lo) at (8 g + p) * 8 + kk.
// lut[p][v] holds the eight expanded bytes of presence byte v for panel p (0 rows, 1 columns).
struct MfmaSmem {
    __align__(16) uint8_t A[2][GM * LDK];
    __align__(16) uint8_t B[2][GM * LDK];
    __align__(16) uint16_t hl[2][2 * GK];
    __align__(16) uint2 lut[2][256];
};

// Fills both expansion tables (one entry of each per thread of a 256-thread group); the
// caller synchronizes before the first use.
__device__ inline void fill_lut(MfmaSmem &sm)
{
    const uint32_t v = threadIdx.x;
    uint32_t e[8];
    expand_bits(v, kRowByte, e);
    sm.lut[0][v] = make_uint2(e[0], e[1]);
    expand_bits(v, kColByte, e);
    sm.lut[1][v] = make_uint2(e[0], e[1]);
}

// One GM x GM tile of S = P diag(hi + lo) P^T (rows row0.., columns col0.., row0 <= col0):
// writes S_ij (i < j) into the condensed array and S_ii into T.  The FP32 chunk sums are
// added in FP64 either into the output itself after every chunk (REG64 = false, small
// register footprint, two work-groups per CU; the default) or into FP64 registers written
// once at the end (REG64 = true, one work-group per CU, no extra output traffic).
template <bool REG64>
__device__ void mfma_tile(const MfmaArgs &a, int32_t row0, int32_t col0, MfmaSmem &sm)
{
    const uint8_t *__restrict__ P = a.P;
    const int32_t n_kstep = a.n_kstep, chunk_steps = a.chunk_steps, n = a.n;
    double *__restrict__ S = a.S;
    double *__restrict__ T = a.T;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int lrow = lane & 31;
    const int kg = lane >> 5;
    // element (mb, nb, r) of the lane: row i, column j of S (32x32 accumulator layout: lane l,
    // register r holds row 8*(r/4) + 4*(l/32) + r%4 and column l%32 of the block)
    auto elem_row = [&](int mb, int r) { return row0 + wm * 64 + mb * 32 + 8 * (r >> 2) + 4 * kg + (r & 3); };
    auto elem_col = [&](int nb) { return col0 + wn * 64 + nb * 32 + lrow; };
    double acc64[REG64 ? 2 : 1][REG64 ? 2 : 1][REG64 ? 16 : 1];
    if (REG64) {
#pragma unroll
        for (int x = 0; x < (REG64 ? 2 : 1); ++x)
#pragma unroll
            for (int y = 0; y < (REG64 ? 2 : 1); ++y)
#pragma unroll
                for (int r = 0; r < (REG64 ? 16 : 1); ++r) acc64[x][y][r] = 0.0;
    }

    // each thread stages the 16 bytes of presence bits of one row (threads 0..127 the row
    // panel, 128..255 the column panel) and one dword of the hi or lo splits (threads 128..
    // repeat the dwords of threads 0..127, writing the same values): dword hd of the stage's
    // 64 holds branches 2 hd and 2 hd + 1, i.e. step hd / 8, K half (hd % 8) / 4, position
    // hd % 4 (+ 4 for lo)
    const int64_t kb = a.k_pad / 8;
    const uint8_t *prow = P + (int64_t)((tid < 128 ? row0 : col0) + (tid & 127)) * kb;
    uint8_t *srow = (tid < 128 ? &sm.A[0][0] : &sm.B[0][0]) + (tid & 127) * LDK;
    const uint32_t *phl = reinterpret_cast<const uint32_t *>((tid & 64) ? a.lo : a.hi) + (tid & 63);
    const int hd = tid & 63;
    const int hpos = (((hd & 7) >> 2) * 8 + (hd & 3) + ((tid & 64) ? 4 : 0)) * 8 + (hd >> 3);
    const uint2 *lut = sm.lut[tid < 128 ? 0 : 1];
    // Global loads run two stages ahead of the compute: stage ks + 2 is loaded into one
    // register set while stage ks + 1 (loaded one stage earlier) waits in the other and is
    // expanded into the free LDS buffer while stage ks computes.  chunk_steps is even, so
    // every chunk starts on an even stage and the two sets alternate with static names.
    struct Stage {
        uint4 bits;
        uint32_t hl;
    };
    Stage R0{}, R1{};
    auto gload = [&](Stage &R, int32_t ks) {
        const int64_t k0 = (int64_t)ks * GK;
        R.bits = *reinterpret_cast<const uint4 *>(prow + k0 / 8);
        R.hl = phl[k0 / 2];
    };
    // One eighth of a stage's expansion into LDS buffer buf: bytes 2h and 2h + 1 (h = part
    // % 2) of bits word part / 2, i.e. branches 16 part .. 16 part + 15 of this thread's row,
    // each byte looked up in the panel's table (rows are LDK = 136 bytes apart: 8-byte
    // aligned stores).
    auto store_part = [&](const Stage &R, int buf, int part) {
        uint2 *dst = reinterpret_cast<uint2 *>(srow + buf * (GM * LDK));
        const int q = part >> 1, h = part & 1;
        const uint32_t x = q == 0 ? R.bits.x : q == 1 ? R.bits.y : q == 2 ? R.bits.z : R.bits.w;
        const uint2 e0 = lut[(x >> (16 * h)) & 0xFFu];
        const uint2 e1 = lut[(x >> (16 * h + 8)) & 0xFFu];
        dst[4 * q + 2 * h] = e0;
        dst[4 * q + 2 * h + 1] = e1;
        if (part == 0) reinterpret_cast<uint32_t *>(sm.hl[buf])[hpos] = R.hl;
    };
    auto lstore = [&](const Stage &R, int buf) {
#pragma unroll
        for (int part = 0; part < GK / 16; ++part) store_part(R, buf, part);
    };
    // LDS words of one 16-branch step: the lane's two row-panel and two column-panel byte
    // runs; and the MFMA operands built from them and the step's length words
    struct Raw {
        uint2 a[2], b[2];
    };
    struct Ops {
        bf16x8 ahi[2], alo[2], bo[2];
    };
    // the lane's length word of every step of the stage (position lane % 8 of its K half)
    static_assert(GK / 16 == 8, "a lane's length words of one stage are two 16-byte reads");
    auto lds_hl = [&](int buf, uint32_t (&hl8)[GK / 16]) {
        const uint4 *src = reinterpret_cast<const uint4 *>(sm.hl[buf]) + (kg * 8 + (lane & 7)) * 2;
        const uint4 x = src[0], y = src[1];
        hl8[0] = x.x; hl8[1] = x.y; hl8[2] = x.z; hl8[3] = x.w;
        hl8[4] = y.x; hl8[5] = y.y; hl8[6] = y.z; hl8[7] = y.w;
    };
    auto lds_raw = [&](int buf, int kk, Raw &r) {
        const int koff = kk * 16 + kg * 8;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
            r.a[mb] = *reinterpret_cast<const uint2 *>(sm.A[buf] + (wm * 64 + mb * 32 + lrow) * LDK + koff);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
            r.b[nb] = *reinterpret_cast<const uint2 *>(sm.B[buf] + (wn * 64 + nb * 32 + lrow) * LDK + koff);
    };
    auto build = [&](const Raw &r, uint32_t hl, Ops &o) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const uint2 m = r.a[mb];
            const uint32_t m0 = __builtin_amdgcn_perm(m.x, m.x, 0x01010000u);
            const uint32_t m1 = __builtin_amdgcn_perm(m.x, m.x, 0x03030202u);
            const uint32_t m2 = __builtin_amdgcn_perm(m.y, m.y, 0x01010000u);
            const uint32_t m3 = __builtin_amdgcn_perm(m.y, m.y, 0x03030202u);
            o.ahi[mb] = as_bf16x8(m0 & row_bcast<0>(hl), m1 & row_bcast<1>(hl),
                                  m2 & row_bcast<2>(hl), m3 & row_bcast<3>(hl));
            o.alo[mb] = as_bf16x8(m0 & row_bcast<4>(hl), m1 & row_bcast<5>(hl),
                                  m2 & row_bcast<6>(hl), m3 & row_bcast<7>(hl));
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            // bytes b0 b1 -> 16-bit halves b0 << 8, b1 << 8 (selector 12 gives a zero byte)
            const uint2 m = r.b[nb];
            o.bo[nb] = as_bf16x8(__builtin_amdgcn_perm(m.x, m.x, 0x010C000Cu),
                                 __builtin_amdgcn_perm(m.x, m.x, 0x030C020Cu),
                                 __builtin_amdgcn_perm(m.y, m.y, 0x010C000Cu),
                                 __builtin_amdgcn_perm(m.y, m.y, 0x030C020Cu));
        }
    };
    f32x16 acc[2][2];
    // the four hi products first, then the four lo ones: no matrix instruction waits on the
    // accumulator of the one just issued (0.4 % faster than hi and lo of a block back to back)
    auto mfma8 = [&](const Ops &o) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ahi[mb], o.bo[nb], acc[mb][nb], 0, 0, 0);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.alo[mb], o.bo[nb], acc[mb][nb], 0, 0, 0);
    };
    // Stage ks from LDS buffer buf, software-pipelined: the LDS words of step kk + 2 are read
    // and the operands of step kk + 1 built while the matrix instructions of step kk run,
    // and an eighth of the next stage's expansion (set Rn, into buffer nbuf) is interleaved
    // with every step.  At the last stage Rn holds no stage and the writes land in a buffer
    // nothing reads.
    auto compute_store = [&](int buf, const Stage &Rn, int nbuf) {
        constexpr int NKK = GK / 16;
        uint32_t hl8[NKK];
        Raw r0, r1;
        Ops o;
        lds_hl(buf, hl8);
        lds_raw(buf, 0, r0);
        lds_raw(buf, 1, r1);
        build(r0, hl8[0], o);
#pragma unroll
        for (int kk = 0; kk < NKK; ++kk) {
            Raw r2;
            if (kk + 2 < NKK) lds_raw(buf, kk + 2, r2);
            mfma8(o);
            store_part(Rn, nbuf, kk);
            if (kk + 1 < NKK) build(r1, hl8[kk + 1], o);
            if (kk + 2 < NKK) r1 = r2;
            // each matrix instruction followed by the VALU work that runs beside it; the
            // LDS reads early, the LDS writes of the expansion mid-way
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x200, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);
            }
        }
    };
    // Rn holds stage ks + 1 (in flight), Rf is free
    auto step = [&](int32_t ks, Stage &Rn, Stage &Rf) {
        if (ks + 2 < n_kstep) gload(Rf, ks + 2);
        compute_store(ks & 1, Rn, (ks + 1) & 1);
        __syncthreads();
    };

    if (n_kstep > 0) {
        gload(R0, 0);
        lstore(R0, 0);
    }
    if (n_kstep > 1) gload(R1, 1);
    __syncthreads();
    // Variant 0 (REG64 = false): the FP32 sums of kGroupChunks consecutive chunks are added
    // in FP32 (a few roundings on top of each chunk's) before one FP64 read-modify-write of
    // the output, which cuts that traffic kGroupChunks-fold.
    constexpr int kGroupChunks = 4;
    float acc2[REG64 ? 1 : 2][REG64 ? 1 : 2][REG64 ? 1 : 16];
    if (!REG64) {
#pragma unroll
        for (int x = 0; x < (REG64 ? 1 : 2); ++x)
#pragma unroll
            for (int y = 0; y < (REG64 ? 1 : 2); ++y)
#pragma unroll
                for (int r = 0; r < (REG64 ? 1 : 16); ++r) acc2[x][y][r] = 0.f;
    }
    int32_t grouped = 0;
    bool flushed = a.accum != 0;   // accumulating launches add from their first flush on
    int32_t ks = 0;
    while (ks < n_kstep) {
        // FP32 accumulation inside a chunk of chunk_steps stages, then one FP64 flush
        const int32_t kend = (n_kstep - ks) < chunk_steps ? n_kstep : ks + chunk_steps;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[x][y][r] = 0.f;
        for (; ks + 1 < kend; ks += 2) {
            step(ks, R1, R0);
            step(ks + 1, R0, R1);
        }
        if (ks < kend) {   // odd-length last chunk
            step(ks, R1, R0);
            ++ks;
        }
        if (REG64) {
#pragma unroll
            for (int x = 0; x < (REG64 ? 2 : 1); ++x)
#pragma unroll
                for (int y = 0; y < (REG64 ? 2 : 1); ++y)
#pragma unroll
                    for (int r = 0; r < (REG64 ? 16 : 1); ++r) acc64[x][y][r] += (double)acc[x][y][r];
            continue;
        }
#pragma unroll
        for (int x = 0; x < (REG64 ? 1 : 2); ++x)
#pragma unroll
            for (int y = 0; y < (REG64 ? 1 : 2); ++y)
#pragma unroll
                for (int r = 0; r < (REG64 ? 1 : 16); ++r) acc2[x][y][r] += acc[REG64 ? 0 : x][REG64 ? 0 : y][REG64 ? 0 : r];
        if (++grouped < kGroupChunks && ks < n_kstep) continue;
        grouped = 0;
        // FP64 cross-chunk sum kept in the output itself: the first flush stores, later
        // flushes add (each element belongs to this work-group alone, chunks in K order).
        const bool first = !flushed;
        flushed = true;
        // the lane's row and column origins pass through an empty asm so that the element
        // addresses are computed here, per flush, instead of being hoisted out of the
        // chunk loop into 64 live pointer registers
        int32_t ib = row0 + wm * 64 + 4 * kg, jb = col0 + wn * 64 + lrow;
        asm volatile("" : "+v"(ib), "+v"(jb));
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                // one 32 x 32 block at a time keeps the flush's live registers small
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int32_t i = ib + mb * 32 + 8 * (r >> 2) + (r & 3);
                    const int32_t j = jb + nb * 32;
                    if (i < n && j < n && i <= j) {
                        double *dst = i < j ? S + ((int64_t)n * i - (int64_t)i * (i + 1) / 2 + (j - i - 1)) : T + i;
                        const double v = (double)acc2[REG64 ? 0 : mb][REG64 ? 0 : nb][REG64 ? 0 : r];
                        *dst = first ? v : *dst + v;
                    }
                }
            }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int x = 0; x < (REG64 ? 1 : 2); ++x)
#pragma unroll
            for (int y = 0; y < (REG64 ? 1 : 2); ++y)
#pragma unroll
                for (int r = 0; r < (REG64 ? 1 : 16); ++r) acc2[x][y][r] = 0.f;
    }
    if (REG64) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int32_t i = elem_row(mb, r);
                    const int32_t j = elem_col(nb);
                    if (i < n && j < n && i <= j) {
                        double *dst = i < j ? S + ((int64_t)n * i - (int64_t)i * (i + 1) / 2 + (j - i - 1)) : T + i;
                        const double v = acc64[REG64 ? mb : 0][REG64 ? nb : 0][REG64 ? r : 0];
                        *dst = a.accum ? *dst + v : v;
                    }
                }
        return;
    }
    if (n_kstep == 0 && !a.accum) {   // no branches: every shared length is 0
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int32_t i = elem_row(mb, r);
                    const int32_t j = elem_col(nb);
                    if (i < n && j < n && i <= j)
                        *(i < j ? S + ((int64_t)n * i - (int64_t)i * (i + 1) / 2 + (j - i - 1)) : T + i) = 0.0;
                }
    }
}

// Single job.  Work-group b takes tile (b % 8) * per + b / 8 of the upper-triangular list,
// so the 8 XCDs (which receive work-groups round-robin) each sweep a contiguous run of
// tiles that share A panels in their L2.
template <bool REG64>
__global__ __launch_bounds__(256, REG64 ? 1 : 2) void k_mfma_gemm(MfmaArgs a, const int2 *__restrict__ tiles,
                                                                 int32_t n_tiles)
{
    __shared__ MfmaSmem sm;
    const int32_t per = (n_tiles + 7) / 8;
    const int32_t t = (int32_t)(blockIdx.x % 8) * per + (int32_t)(blockIdx.x / 8);
    if (t >= n_tiles) return;
    fill_lut(sm);
    __syncthreads();
    const int2 tile = tiles[t];
    mfma_tile<REG64>(a, tile.x * GM, tile.y * GM, sm);
}

// Many jobs: work-groups take (job, tile) items from a global counter (items listed
// largest job first), leaving at the first fetch past the end.  *counter is zero at launch.
template <bool REG64>
__global__ __launch_bounds__(256, REG64 ? 1 : 2) void k_mfma_queue(const MfmaArgs *__restrict__ jobs,
                                                      const int2 *__restrict__ items,
                                                      int32_t n_items, int32_t *__restrict__ counter)
{
    __shared__ MfmaSmem sm;
    __shared__ int32_t s_item;
    fill_lut(sm);   // the loop's first barrier orders it before every use
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t it = s_item;
        if (it >= n_items) break;
        const int2 item = items[it];
        const MfmaArgs a = jobs[item.x];
        const int2 tile = a.tiles[item.y];
        mfma_tile<REG64>(a, tile.x * GM, tile.y * GM, sm);
    }
}

// d_ij = (T_i + T_j - 2 S_ij) / (T_i + T_j - S_ij), 0 when the denominator is 0.
// S may alias out (FP64 output): each element is read before it is written by one thread.
template <typename OUT>
__global__ void k_mfma_normalize(const double *S, const double *__restrict__ T, int32_t n,
                                 OUT *out)
{
    const int32_t i = blockIdx.x;
    const int64_t row0 = (int64_t)n * i - (int64_t)i * (i + 1) / 2 - i - 1;
    const double ti = T[i];
    for (int32_t j = i + 1 + threadIdx.x; j < n; j += 256) {
        const double s = S[row0 + j];
        const double tt = ti + T[j];
        const double u = tt - s;
        const double d = (u == 0.0) ? 0.0 : (tt - 2.0 * s) / u;
        out[row0 + j] = (OUT)d;
    }
}

inline unsigned grid1(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

MfmaGeom mfma_geometry(int32_t n, int32_t n_branches)
{
    MfmaGeom g;
    g.n = n;
    g.B = n_branches;
    g.n_pad = (int32_t)((n + 255) / 256 * 256);
    g.k_pad = (int64_t)(n_branches + GK - 1) / GK * GK;
    g.tile = GM;
    g.kstep = GK;
    const int32_t nb = (n + GM - 1) / GM;
    g.n_tiles = nb * (nb + 1) / 2;
    return g;
}

void mfma_tile_list(int32_t n, std::vector<int32_t> *xy)
{
    // Upper-triangular tiles in groups of kGroup x kGroup tiles: the work-groups resident on
    // one XCD at a time (2 per CU x 32 CUs) then cover one group, whose kGroup row panels and
    // kGroup column panels are each shared by kGroup tiles through that XCD's L2.
    constexpr int32_t kGroup = 8;
    const int32_t nb = (n + GM - 1) / GM;
    const int32_t ng = (nb + kGroup - 1) / kGroup;
    xy->clear();
    xy->reserve((size_t)nb * (nb + 1));
    for (int32_t gi = 0; gi < ng; ++gi)
        for (int32_t gj = gi; gj < ng; ++gj)
            for (int32_t I = gi * kGroup; I < std::min(nb, gi * kGroup + kGroup); ++I)
                for (int32_t J = std::max(I, gj * kGroup); J < std::min(nb, gj * kGroup + kGroup); ++J) {
                    xy->push_back(I);
                    xy->push_back(J);
                }
}

hipError_t launch_split_lengths(const double *len, int32_t B, int64_t k_pad, uint16_t *hi,
                                uint16_t *lo, hipStream_t st)
{
    if (k_pad <= 0) return hipSuccess;
    k_split_lengths<<<grid1(k_pad, 256), 256, 0, st>>>(len, B, (int32_t)k_pad, hi, lo);
    return hipGetLastError();
}

hipError_t launch_bits_transpose(const uint32_t *bits, int64_t bstride, const MfmaGeom &g,
                                 uint8_t *Pb, hipStream_t st)
{
    if (g.k_pad <= 0) return hipSuccess;
    const dim3 grid((unsigned)(g.k_pad / 64), (unsigned)(g.n_pad / 256));
    k_bits_transpose<<<grid, 256, 0, st>>>(bits, bstride, g.B, g.n_pad, g.k_pad / 8, Pb);
    return hipGetLastError();
}

MfmaArgs make_mfma_args(const uint8_t *P, const uint16_t *hi, const uint16_t *lo, int32_t k_chunk,
                        const int32_t *tiles_xy, const MfmaGeom &g, double *S, double *T)
{
    MfmaArgs a;
    a.P = P;
    a.k_pad = g.k_pad;
    a.n_kstep = (int32_t)(g.k_pad / GK);
    // whole stages, an even number of them (the tile loop alternates two register sets)
    const int32_t cs = k_chunk / GK < 1 ? 1 : k_chunk / GK;
    a.chunk_steps = (cs + 1) & ~1;
    a.hi = hi;
    a.lo = lo;
    a.n = g.n;
    a.n_tiles = g.n_tiles;
    a.accum = 0;
    a.pad = 0;
    a.S = S;
    a.T = T;
    a.tiles = reinterpret_cast<const int2 *>(tiles_xy);
    return a;
}

hipError_t launch_mfma_gemm(const uint8_t *P, const uint16_t *hi, const uint16_t *lo,
                            int32_t k_chunk, const int32_t *tiles_xy, const MfmaGeom &g,
                            double *S, double *T, int32_t variant, hipStream_t st, int32_t accum)
{
    MfmaArgs a = make_mfma_args(P, hi, lo, k_chunk, tiles_xy, g, S, T);
    a.accum = accum;
    const int32_t per = (g.n_tiles + 7) / 8;
    if (variant == 1)
        k_mfma_gemm<true><<<(unsigned)(8 * per), 256, 0, st>>>(a, a.tiles, g.n_tiles);
    else
        k_mfma_gemm<false><<<(unsigned)(8 * per), 256, 0, st>>>(a, a.tiles, g.n_tiles);
    return hipGetLastError();
}

hipError_t launch_mfma_queue(const MfmaArgs *jobs, const int32_t *items_xy, int32_t n_items,
                             int32_t *counter, int32_t n_groups, int32_t variant, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    const int2 *it = reinterpret_cast<const int2 *>(items_xy);
    if (variant == 1)
        k_mfma_queue<true><<<n_groups, 256, 0, st>>>(jobs, it, n_items, counter);
    else
        k_mfma_queue<false><<<n_groups, 256, 0, st>>>(jobs, it, n_items, counter);
    return hipGetLastError();
}

hipError_t launch_mfma_normalize(const double *S, const double *T, int32_t n, int32_t out_f32,
                                 void *out, hipStream_t st)
{
    if (n < 2) return hipSuccess;
    if (out_f32)
        k_mfma_normalize<float><<<n - 1, 256, 0, st>>>(S, T, n, (float *)out);
    else
        k_mfma_normalize<double><<<n - 1, 256, 0, st>>>(S, T, n, (double *)out);
    return hipGetLastError();
}

}  // namespace ufmi
