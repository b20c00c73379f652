// Exact-integer X-streaming products on the matrix cores (arXiv 1805.06604:
// the W^T X and X H^T terms of the HALS updates, section 1 and Remark 1).
//
// Number format. Every row i of Z (X or the resident X^T) carries a power of
// two 2^s_i chosen so that u = Z(i,:) 2^s_i lies in (-64, 64); u is stored as
// four int8 slices, u = d0 + d1/128 + d2/128^2 + d3/128^3 (+ at most
// 2^-22), each |d| <= 64, formed by repeated round-to-nearest. A factor column
// k is scaled the same way by 2^t_k (from the column's max |F|) and sliced on
// the fly. Then
//     sum_j u_ij v_jk = sum_{a,b} 128^-(a+b) sum_j d_a(i,j) e_b(j,k),
// and the inner sums are exact in int32 on v_mfma_i32_16x16x64_i8. The pairs
// with a + b <= 3 are kept (four int32 accumulators, one per weight a + b);
// the dropped pairs weigh at most 2^-28 of the leading one. At the end of the
// K-chunk the accumulators are combined in FP64 and scaled by 2^-(s_i+t_k):
// products accurate to about 2^-27 of the row and column maxima, with no
// rounding in the summation over K.
//
// Z layout (fragment order). The slices of Z are stored per 16-row block and
// 64-column tile as 4 slices x 64 lanes x 16 bytes, lane lr + 16 g holding
// row lr, columns 16 g .. 16 g + 15 of the tile: [row / 16][tile][slice]
// [lane][16]. One wave load of an MFMA operand is then 1 KB of contiguous
// memory, and a 16-row block streams its K-chunk front to back.
//
// Tiling. A workgroup is 8 waves (two per SIMD) over 128 rows x RP columns
// and one K-chunk; each wave owns 16 rows (one 16-row MFMA block) and all
// RP/16 column blocks, so that one wave's multiplies overlap the other's waits.
// K advances in tiles of 64 (one MFMA k-step). Each wave streams the slices of
// its own rows straight into registers, three tiles ahead of the multiply
// (four register buffers), with non-temporal loads: Z is read once per product.
// The factor is sliced once per product by its own kernel (in MFMA operand
// order); its tiles, which all 8 waves read, go through a 4-stage LDS ring
// filled by direct global-to-LDS loads in the same issue group as the Z tile,
// one barrier per tile. The K loop is unrolled by the four buffers, so every
// buffer and stage index is static, and every load is issued unconditionally
// (the tile index clamped to the K-chunk: the loop starts one round early and
// ends past the last tile with harmless reloads), so the wait counts are
// static and no load precedes the loop.
#pragma once

#include "nmf_internal.h"

namespace nmf {
namespace i8 {

typedef int int32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;
constexpr int kWM = 16;                 // rows per wave (one 16-row MFMA block)
constexpr int kBM = kWaves * kWM;       // rows per workgroup
constexpr int kKT = 64;                 // K per tile (one MFMA k-step)
constexpr int kSl = 4;                  // slices per value
constexpr int kMaxW = 3;                // kept pairs: a + b <= kMaxW

// Scale exponent s with |x| 2^s < 64 for |x| <= amax (0 for amax == 0).
__host__ __device__ inline int slice_exponent(double amax)
{
    if (!(amax > 0.0)) return 0;
    int e;
    frexp(amax, &e);            // amax = f 2^e, f in [0.5, 1)
    return 6 - e;               // amax 2^s = f 64 < 64
}

// Four int8 slices of u (|u| < 64): u ~ d0 + d1/128 + d2/128^2 + d3/128^3.
__device__ __forceinline__ void slice4(float u, int (&d)[kSl])
{
#pragma unroll
    for (int q = 0; q < kSl; ++q) {
        const float r = rintf(u);
        d[q] = (int)r;
        u = (u - r) * 128.0f;   // exact: u - rint(u) needs no rounding
    }
}

// Position of the 16-byte part `part` (columns 16 part .. 16 part + 15 of the
// tile) of factor column c in a sliced tile: parts are XOR-swizzled by
// (c / 4) mod 4, so that the 16 lanes reading one part of 16 consecutive
// columns hit distinct LDS banks.
__host__ __device__ constexpr int fpart(int c, int part) { return part ^ ((c >> 2) & 3); }

// Slices one 64-row tile of the factor F (K x RP, FP32) per workgroup into
// Fsl[tile][slice][column][4 parts of 16] (int8, MFMA operand order, parts
// swizzled by fpart, zero past K), with column exponents t_k from the column
// maxima; block 0 also stores t_k.
template <int RP>
__device__ __forceinline__ void slice_body(const ProdArgs &a, int bid)
{
    __shared__ int s_texp[RP];
    const DevState *st = a.st;
    int slot = 0;
    if (a.sel != SEL_SLOT0) {
        if (st->done) return;
        slot = (a.sel == SEL_W_Y) ? st->w_y : (st->hp == 1 ? st->h_n : st->h_yn);
    }
    const float *__restrict__ F = a.F_base + slot * a.slot_stride;
    const double *colmax = (a.sel == SEL_W_Y ? a.gram_base + (size_t)st->w_y * a.gram_slot_stride
                                             : a.gram_base) + RP * RP + RP;
    const int tid = threadIdx.x;
    if (tid < RP) {
        s_texp[tid] = slice_exponent(colmax[tid]);
        if (bid == 0) a.texp[tid] = s_texp[tid];
    }
    __syncthreads();
    const int64_t tile = bid;
    uint32_t *out = reinterpret_cast<uint32_t *>(a.Fsl + tile * (kSl * RP * kKT));
    // One item per thread (RP x 4 <= 256): column c, the 16 rows of part
    // `part`; all 16 loads are issued before any store.
    for (int item = tid; item < RP * 4; item += 256) {
        const int c = item % RP, part = item / RP;
        float f[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int64_t k = tile * kKT + 16 * part + e;
            f[e] = (k < a.K) ? F[k * RP + c] : 0.0f;
        }
        uint32_t w[kSl][4] = {};
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            int d[kSl];
            slice4(ldexpf(f[e], s_texp[c]), d);
#pragma unroll
            for (int p = 0; p < kSl; ++p) w[p][e / 4] |= ((uint32_t)(d[p] & 0xff)) << (8 * (e % 4));
        }
#pragma unroll
        for (int p = 0; p < kSl; ++p)
            *reinterpret_cast<uint4 *>(out + (p * RP + c) * (kKT / 4) + fpart(c, part) * 4) =
                make_uint4(w[p][0], w[p][1], w[p][2], w[p][3]);
    }
}

// s_waitcnt immediate: vmcnt(n) (bits 3:0 and 15:14), lgkmcnt(0), no expcnt wait.
__host__ __device__ constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x0070; }

constexpr int kDepth = 3;               // tiles in flight ahead of the multiply
constexpr int kBufs = kDepth + 1;       // register buffers = LDS stages = K-loop unroll

template <int RP>
__device__ __forceinline__ void prod_body(const ProdArgs &args, int bid)
{
    // A private copy: the grouped kernels read the arguments from global
    // memory, which the compiler would otherwise reload (and wait for) after
    // every direct-to-LDS load.
    const ProdArgs a = args;
    constexpr int NCB = RP / 16;
    constexpr int FT = kSl * RP * kKT;                // factor tile bytes (RP KB)
    constexpr int FTK = FT / 1024;
    // Every wave moves FOPS KB of each factor tile (the last KB again where the
    // tile does not split evenly: identical bytes to the same place), so all
    // waves issue the same number of loads per tile.
    constexpr int FOPS = (FTK + kWaves - 1) / kWaves;
    constexpr int GOPS = kSl + FOPS;                  // loads per wave per tile
    static_assert((kDepth - 1) * GOPS <= 63, "vmcnt range");
    __shared__ __attribute__((aligned(1024))) signed char ring[kBufs][FT];

    const DevState *st = a.st;
    if (a.sel != SEL_SLOT0 && st->done) return;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, lr = lane & 15;
    const int kc = bid % a.nsplit;
    const int64_t rb = bid / a.nsplit;
    const int64_t kbeg = (int64_t)kc * a.kchunk;
    int64_t kend = kbeg + a.kchunk;
    if (kend > a.ld) kend = a.ld;
    const int64_t row0 = rb * kBM + wave * kWM;
    const int64_t ntile = a.ld / kKT;
    // The wave's 16-row block of tile t starts at ((row0/16) ntile + t) 4 KB in
    // the fragment layout; this lane's 16 bytes of slice p at p KB + 16 lane.
    const signed char *zsrc = static_cast<const signed char *>(a.Z) +
                              (row0 / 16) * ntile * (kSl * 1024) + 16 * lane;
    // This lane's byte offset of part g of column 16 c + lr, slice j, within
    // the factor tile: ((j RP + 16 c + lr) 4 + fpart) 16.
    const int boff = (lr * 4 + fpart(lr, g)) * 16;

    int32x4 acc[NCB][kMaxW + 1];
#pragma unroll
    for (int c = 0; c < NCB; ++c)
#pragma unroll
        for (int w = 0; w <= kMaxW; ++w) acc[c][w] = int32x4{0, 0, 0, 0};

    const int64_t t0 = kbeg / kKT, t1 = (kend + kKT - 1) / kKT;   // tiles [t0, t1)
    if (t0 < t1) {
        int32x4 z[kBufs][kSl];
        // Issue group of tile `tile` (clamped to [t0, t1)): this wave's
        // share of the factor tile into stage `sg`, then its Z slices into zb.
        auto issue = [&](int64_t tile, int sg, int32x4 (&zb)[kSl]) {
            if (tile < t0) tile = t0;
            if (tile > t1 - 1) tile = t1 - 1;
            const signed char *fs = a.Fsl + tile * FT + 16 * lane;
#pragma unroll
            for (int q = 0; q < FOPS; ++q) {
                const int kb = (wave * FOPS + q < FTK) ? wave * FOPS + q : FTK - 1;
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(fs + kb * 1024),
                    (__attribute__((address_space(3))) void *)(ring[sg] + kb * 1024), 16, 0, 0);
            }
            const signed char *zp = zsrc + tile * (kSl * 1024);
#pragma unroll
            for (int p = 0; p < kSl; ++p)
                zb[p] = __builtin_nontemporal_load(reinterpret_cast<const int32x4 *>(zp + p * 1024));
        };
        // The loop starts kBufs tiles early: its first round only issues the
        // groups of tiles t0 .. t0 + kDepth - 1 (and a harmless load of tile
        // t0 into the buffer of t0 - 1), so that no load precedes the loop and
        // the register buffers need no copies at its head.
        for (int64_t tb = t0 - kBufs; tb < t1; tb += kBufs) {
            static_for<kBufs>([&](auto UU) {
                constexpr int u = decltype(UU)::value;          // tile tb + u: buffer and stage u
                constexpr int un = (u + kDepth) % kBufs;        // freed by tile tb + u - 1
                const int64_t t = tb + u;
                // Tile t's group has landed once at most the kDepth - 1 later
                // groups are in flight; after the barrier every wave's share of
                // the factor tile is visible, and every wave is done with the
                // stage read for tile t - 1. (The scheduling barriers keep the
                // wait, the barrier and the issue group in this order.)
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_waitcnt(vmcnt_imm((kDepth - 1) * GOPS));
                __builtin_amdgcn_s_barrier();
                __builtin_amdgcn_sched_barrier(0);
                issue(t + kDepth, un, z[un]);
                __builtin_amdgcn_sched_barrier(0);
                if (t >= t0 && t < t1) {                        // (uniform)
                    const signed char *ft = ring[u];
                    // Factor slice j against Z slices i <= kMaxW - j.
#pragma unroll
                    for (int j = 0; j < kSl; ++j) {
                        int32x4 bp[NCB];
#pragma unroll
                        for (int c = 0; c < NCB; ++c)
                            bp[c] = *reinterpret_cast<const int32x4 *>(ft + (j * RP + 16 * c) * 64 + boff);
#pragma unroll
                        for (int i = 0; i + j <= kMaxW; ++i)
#pragma unroll
                            for (int c = 0; c < NCB; ++c)
                                acc[c][i + j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                                    z[u][i], bp[c], acc[c][i + j], 0, 0, 0);
                    }
                }
            });
        }
        __builtin_amdgcn_s_waitcnt(0x0070);            // vmcnt(0): no load outlives the loop
    }

    // D layout: lane holds column lr of each block, rows 4g..4g+3.
    double *Y = a.Y + (size_t)kc * a.rows_pad * RP;
    int te[NCB];
#pragma unroll
    for (int c = 0; c < NCB; ++c) te[c] = a.texp[c * 16 + lr];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + 4 * g + i;
        const int se = a.zexp[row];
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            double v = 0.0;
#pragma unroll
            for (int w = kMaxW; w >= 0; --w) v = v * (1.0 / 128.0) + (double)acc[c][w][i];
            Y[row * RP + c * 16 + lr] = ldexp(v, -se - te[c]);
        }
    }
}

template <int RP>
__global__ __launch_bounds__(256) void slice_factor_kernel(ProdArgs a)
{
    slice_body<RP>(a, blockIdx.x);
}

template <int RP>
__global__ __launch_bounds__(kWaves * 64, 1) void prod_i8_kernel(ProdArgs a)
{
    prod_body<RP>(a, blockIdx.x);
}

// Grouped forms (one launch over several problems of one padded rank).
// Each workgroup takes the work blocks blockIdx.x, blockIdx.x + gridDim.x,
// ... in turn, with a barrier between two blocks (LDS reuse).
template <int RP>
__global__ __launch_bounds__(256) void slice_factor_group_kernel(Group g)
{
    const int total = group_total(g);
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        int lb, cnt;
        const int p = group_find(g, b, &lb, &cnt);
        slice_body<RP>(*reinterpret_cast<const ProdArgs *>(g.base + (size_t)p * g.stride), lb);
        __syncthreads();
    }
}

template <int RP>
__global__ __launch_bounds__(kWaves * 64, 1) void prod_i8_group_kernel(Group g)
{
    const int total = group_total(g);
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        int lb, cnt;
        const int p = group_find(g, b, &lb, &cnt);
        prod_body<RP>(*reinterpret_cast<const ProdArgs *>(g.base + (size_t)p * g.stride), lb);
        // The body ends with loads past its last tile still in flight (into
        // registers and, by direct loads, into the LDS ring): all of them
        // land before the next block reuses the ring.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
}

// Blocks of the two kernels of one product.
inline int slice_blocks(const ProdArgs &a) { return (int)(a.ld / kKT); }
inline int prod_blocks(const ProdArgs &a) { return (int)((a.rows_pad / kBM) * a.nsplit); }

template <int RP>
void launch_group(const Group &gs, int sblocks, const Group &gp, int pblocks, hipStream_t s)
{
    slice_factor_group_kernel<RP><<<sblocks, 256, 0, s>>>(gs);
    prod_i8_group_kernel<RP><<<pblocks, kWaves * 64, 0, s>>>(gp);
}

template <int RP>
void launch(const ProdArgs &a, hipStream_t s, hipEvent_t mid)
{
    slice_factor_kernel<RP><<<(unsigned)(a.ld / kKT), 256, 0, s>>>(a);
    if (mid) (void)hipEventRecord(mid, s);
    const int64_t blocks = (a.rows_pad / kBM) * a.nsplit;
    prod_i8_kernel<RP><<<(unsigned)blocks, kWaves * 64, 0, s>>>(a);
}

}  // namespace i8
}  // namespace nmf
