// X-streaming products for X stored in 16 bits (BF16 or FP16) on the 16-bit
// matrix cores (arXiv 1805.06604: the W^T X and X H^T terms of the HALS
// updates, section 1 and Remark 1).
//
// Precision. The factor is split once per product into two parts of the X
// type, f = f0 + f1 + (a rounding residue), round to nearest at each step:
// for BF16 X two BF16 parts (residue at most 2^-16 |f|); for FP16 X two FP16
// parts of f 2^t_k, with a power of two per column from the column maximum
// (the largest scaled value below 2^15, residue at most 2^-22 of it), taken
// out again when the sums are stored. X feeds the matrix cores as stored:
// two products per k-step (x f0 and x f1), accumulated in FP32 on
// v_mfma_f32_16x16x32_bf16 / _f16 within the K-chunk; the K-chunk partials
// are written in FP32 and summed in FP64 by the sweep kernels.
//
// Z layout (fragment order). The 16-bit copy of Z (X or the resident X^T) is
// stored per 16-row block and 64-column tile as 2 k-steps x 64 lanes x 16
// bytes, lane lr + 16 g holding row lr, columns 32 s + 8 g .. 32 s + 8 g + 7
// of the tile: [row / 16][tile][k-step][lane][8]. One wave load of an MFMA
// operand is then 1 KB of contiguous memory.
//
// Tiling (as in the exact-integer product, with two row blocks per wave so
// that each factor operand read from LDS serves 32 rows). A workgroup is 8
// waves (two per SIMD) over 256 rows x RP columns and one K-chunk; each wave
// owns two 16-row blocks and all RP/16 column blocks, streams its Z fragments
// straight into registers three steps (of kTPS tiles) ahead with non-temporal
// loads, and reads the split factor tiles from a 4-stage LDS ring filled by
// direct global-to-LDS loads in the same issue group; one barrier per step.
// The K loop is unrolled by the four buffers and every load is issued
// unconditionally (tile index clamped to the K-chunk: the loop starts one
// round early and ends past the last tile with harmless reloads), so the wait
// counts are static and no load precedes the loop.
#pragma once

#include "nmf_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace nmf {
namespace x16 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef int int32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;
constexpr int kBPW = 2;                 // 16-row MFMA blocks per wave
constexpr int kWM = 16 * kBPW;          // rows per wave
constexpr int kBM = kWaves * kWM;       // rows per workgroup
static_assert(kBM == kX16Rows, "row padding of the 16-bit path");
constexpr int kKT = 64;                 // K per tile (two MFMA k-steps)
constexpr int kFP = 2;                  // parts of the factor
constexpr int kTPS = 1;                 // tiles per step (one barrier per step)
constexpr int kDepth = 3;               // steps in flight ahead of the multiply
constexpr int kBufs = kDepth + 1;       // register buffers = LDS stages = K-loop unroll

// Position of the 16-byte group g (k = 8 g .. 8 g + 7 of a k-step) of factor
// column c in the split tile: XOR-swizzled by (c / 4) mod 4, so that the 16
// lanes reading one group of 16 consecutive columns hit distinct LDS banks.
__host__ __device__ constexpr int fgroup(int c, int g) { return g ^ ((c >> 2) & 3); }

// s_waitcnt immediate: vmcnt(n) (bits 3:0 and 15:14), lgkmcnt(0), no expcnt wait.
__host__ __device__ constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x0070; }

// Operand vectors of 8 16-bit values and the matrix-core product of the X
// type.
template <typename XT> struct Ops16;
template <> struct Ops16<__hip_bfloat16> {
    typedef bf16x8 vec;
    typedef __bf16 elem;
    static constexpr bool scaled = false;
    __device__ static floatx4 mfma(vec x, vec f, floatx4 acc)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, f, acc, 0, 0, 0);
    }
};
template <> struct Ops16<__half> {
    typedef half8 vec;
    typedef _Float16 elem;
    static constexpr bool scaled = true;
    __device__ static floatx4 mfma(vec x, vec f, floatx4 acc)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, f, acc, 0, 0, 0);
    }
};

// Column scale exponent t of the FP16 factor parts: |f| 2^t < 2^15 for
// |f| <= amax (0 for amax == 0).
__host__ __device__ inline int half_exponent(double amax)
{
    if (!(amax > 0.0)) return 0;
    int e;
    frexp(amax, &e);            // amax = m 2^e, m in [0.5, 1)
    return 15 - e;
}

// Splits one 64-row tile of the factor F (K x RP, FP32) per workgroup into
// Fsp[tile][k-step][part][column][4 groups of 16 B] (parts of the X type in
// B-operand order, groups swizzled by fgroup, zero past K); for FP16 parts
// the columns are scaled by 2^t_k first (t_k from the column maxima in the
// Gram buffer's tail; block 0 also stores t_k).
template <int RP, typename XT>
__device__ __forceinline__ void split_body(const ProdArgs &a, int bid)
{
    typedef typename Ops16<XT>::vec vec;
    typedef typename Ops16<XT>::elem elem;
    __shared__ int s_texp[RP];
    const DevState *st = a.st;
    int slot = 0;
    if (a.sel != SEL_SLOT0) {
        if (st->done) return;
        slot = (a.sel == SEL_W_Y) ? st->w_y : (st->hp == 1 ? st->h_n : st->h_yn);
    }
    const float *__restrict__ F = a.F_base + slot * a.slot_stride;
    if constexpr (Ops16<XT>::scaled) {
        const double *colmax = (a.sel == SEL_W_Y ? a.gram_base + (size_t)st->w_y * a.gram_slot_stride
                                                 : a.gram_base) + RP * RP + RP;
        if (threadIdx.x < RP) {
            s_texp[threadIdx.x] = half_exponent(colmax[threadIdx.x]);
            if (bid == 0) a.texp[threadIdx.x] = s_texp[threadIdx.x];
        }
        __syncthreads();
    }
    const int64_t tile = bid;
    signed char *out = a.Fsl + tile * (2 * kFP * RP * 64);
    // One item per (k-step s, column c, group g): 8 rows, both parts.
    for (int item = threadIdx.x; item < 2 * RP * 4; item += 256) {
        const int c = item % RP, g = (item / RP) % 4, s = item / (4 * RP);
        float f[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t k = tile * kKT + 32 * s + 8 * g + e;
            f[e] = (k < a.K) ? F[k * RP + c] : 0.0f;
            if constexpr (Ops16<XT>::scaled) f[e] = ldexpf(f[e], s_texp[c]);   // exact
        }
        vec p0, p1;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const elem h = (elem)f[e];
            p0[e] = h;
            p1[e] = (elem)(f[e] - (float)h);
        }
        *reinterpret_cast<vec *>(out + ((s * kFP + 0) * RP + c) * 64 + fgroup(c, g) * 16) = p0;
        *reinterpret_cast<vec *>(out + ((s * kFP + 1) * RP + c) * 64 + fgroup(c, g) * 16) = p1;
    }
}

template <int RP, typename XT>
__device__ __forceinline__ void prod_body(const ProdArgs &args, int bid)
{
    // A private copy: the grouped form would otherwise re-read the argument
    // record after every direct-to-LDS load.
    const ProdArgs a = args;
    typedef typename Ops16<XT>::vec vec;
    constexpr int NCB = RP / 16;
    constexpr int FT = 2 * kFP * RP * 64;             // split factor tile bytes (RP KB)
    constexpr int FTK = FT / 1024;
    constexpr int SFK = kTPS * FTK;                   // factor KB per step
    constexpr int FOPS = (SFK + kWaves - 1) / kWaves; // factor KB per wave per step
    constexpr int GOPS = 2 * kTPS * kBPW + FOPS;      // loads per wave per step
    static_assert((kDepth - 1) * GOPS <= 63, "vmcnt range");
    __shared__ __attribute__((aligned(1024))) signed char ring[kBufs][kTPS * FT];

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
    // The wave's 16-row block b of tile t starts at ((row0/16 + b) ntile + t)
    // 2 KB; this lane's 16 bytes of k-step s at s KB + 16 lane.
    const signed char *zsrc = static_cast<const signed char *>(a.Z) +
                              (row0 / 16) * ntile * 2048 + 16 * lane;
    const int boff = (lr * 4 + fgroup(lr, g)) * 16;

    floatx4 acc[kBPW][NCB];
#pragma unroll
    for (int b = 0; b < kBPW; ++b)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[b][c] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int64_t t0 = kbeg / kKT, t1 = (kend + kKT - 1) / kKT;   // tiles [t0, t1)
    const int64_t nstep = (t1 - t0 + kTPS - 1) / kTPS;            // kTPS tiles per step
    if (t0 < t1) {
        int32x4 z[kBufs][kTPS][kBPW][2];
        // Issue group of step j (tiles clamped to [t0, t1)): this wave's share
        // of the step's factor tiles into stage sg, then its Z fragments.
        auto issue = [&](int64_t j, int sg, int32x4 (&zb)[kTPS][kBPW][2]) {
#pragma unroll
            for (int q = 0; q < FOPS; ++q) {
                const int kb = (wave * FOPS + q < SFK) ? wave * FOPS + q : SFK - 1;
                int64_t tile = t0 + kTPS * j + kb / FTK;
                if (tile < t0) tile = t0;
                if (tile > t1 - 1) tile = t1 - 1;
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(a.Fsl + tile * FT +
                                                                     (kb % FTK) * 1024 + 16 * lane),
                    (__attribute__((address_space(3))) void *)(ring[sg] + kb * 1024), 16, 0, 0);
            }
#pragma unroll
            for (int h = 0; h < kTPS; ++h) {
                int64_t tile = t0 + kTPS * j + h;
                if (tile < t0) tile = t0;
                if (tile > t1 - 1) tile = t1 - 1;
#pragma unroll
                for (int b = 0; b < kBPW; ++b) {
                    const signed char *zp = zsrc + (b * ntile + tile) * 2048;
#pragma unroll
                    for (int s = 0; s < 2; ++s)
                        zb[h][b][s] = __builtin_nontemporal_load(
                            reinterpret_cast<const int32x4 *>(zp + s * 1024));
                }
            }
        };
        // The loop starts one round early (that round only issues the groups
        // of steps 0 .. kDepth - 1), so that no load precedes it.
        for (int64_t jb = -kBufs; jb < nstep; jb += kBufs) {
            static_for<kBufs>([&](auto UU) {
                constexpr int u = decltype(UU)::value;
                constexpr int un = (u + kDepth) % kBufs;
                const int64_t j = jb + u;
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_waitcnt(vmcnt_imm((kDepth - 1) * GOPS));
                __builtin_amdgcn_s_barrier();
                __builtin_amdgcn_sched_barrier(0);
                issue(j + kDepth, un, z[un]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int h = 0; h < kTPS; ++h) {
                    const int64_t t = t0 + kTPS * j + h;
                    if (j >= 0 && t < t1) {                     // (uniform)
                        const signed char *ft = ring[u] + h * FT;
#pragma unroll
                        for (int s = 0; s < 2; ++s) {
                            vec bp[NCB][kFP];
#pragma unroll
                            for (int c = 0; c < NCB; ++c)
#pragma unroll
                                for (int p = 0; p < kFP; ++p)
                                    bp[c][p] = *reinterpret_cast<const vec *>(
                                        ft + ((s * kFP + p) * RP + 16 * c) * 64 + boff);
#pragma unroll
                            for (int p = 0; p < kFP; ++p)
#pragma unroll
                                for (int b = 0; b < kBPW; ++b)
#pragma unroll
                                    for (int c = 0; c < NCB; ++c)
                                        acc[b][c] = Ops16<XT>::mfma(
                                            __builtin_bit_cast(vec, z[u][h][b][s]), bp[c][p],
                                            acc[b][c]);
                        }
                    }
                }
            });
        }
        __builtin_amdgcn_s_waitcnt(0x0070);            // vmcnt(0): no load outlives the loop
    }

    // D layout: lane holds column lr of each block, rows 4g..4g+3. The
    // K-chunk's FP32 sums are stored as they are (FP32 partials; the sweep
    // kernels add them in FP64), FP16 ones scaled back by 2^-t_k (exact).
    float *Y = reinterpret_cast<float *>(a.Y) + (size_t)kc * a.rows_pad * RP;
    int te[NCB] = {};
    if constexpr (Ops16<XT>::scaled) {
#pragma unroll
        for (int c = 0; c < NCB; ++c) te[c] = a.texp[c * 16 + lr];
    }
#pragma unroll
    for (int b = 0; b < kBPW; ++b)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = acc[b][c][i];
                if constexpr (Ops16<XT>::scaled) v = ldexpf(v, -te[c]);
                Y[(row0 + 16 * b + 4 * g + i) * RP + c * 16 + lr] = v;
            }
}

template <int RP, typename XT>
__global__ __launch_bounds__(256) void split_factor_kernel(ProdArgs a)
{
    split_body<RP, XT>(a, blockIdx.x);
}

template <int RP, typename XT>
__global__ __launch_bounds__(kWaves * 64, 1) void prod_x16_kernel(ProdArgs a)
{
    prod_body<RP, XT>(a, blockIdx.x);
}

template <int RP, typename XT>
void launch(const ProdArgs &a, hipStream_t s, hipEvent_t mid)
{
    split_factor_kernel<RP, XT><<<(unsigned)(a.ld / kKT), 256, 0, s>>>(a);
    if (mid) (void)hipEventRecord(mid, s);
    const int64_t blocks = (a.rows_pad / kBM) * a.nsplit;
    prod_x16_kernel<RP, XT><<<(unsigned)blocks, kWaves * 64, 0, s>>>(a);
}

}  // namespace x16
}  // namespace nmf
