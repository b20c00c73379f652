// X-streaming products on the matrix cores (arXiv 1805.06604: the W^T X and
// X H^T terms of the HALS updates, section 1 and Remark 1).
//
// Y_part[kc] = Z[:, K-chunk kc] * F[K-chunk kc, :] for a row-major Z (X or the
// resident X^T, rows padded to a multiple of 128, row length ld padded to a
// multiple of 64, zero-filled) and a row-major FP32 factor F (K x RP). The
// K-chunk partials are summed in FP64 by the consumer (the sweep kernels).
//
// Precision. An FP32 value is split exactly into BF16 parts p0 + p1 + p2 with
// 8 significant bits each (round to nearest at every step), so that part i
// carries the bits of weight about 2^(-8 i) relative to the value. The product
// of two values is the sum over part pairs (i, j); the kernel keeps the pairs
// with i + j <= L and accumulates them in FP32 on v_mfma_f32_16x16x32_bf16
// within the K-chunk (partials are written in FP64):
//   L = 2: every pair down to relative weight 2^-16 (FP32-equivalent products;
//          6 pairs for FP32 X, 3 for BF16 X, 5 for FP16 X);
//   L = 1: pairs down to 2^-8 (16-bit operands; 3, 2 and 3 pairs).
// BF16 X is exact in one part and FP16 X in two.
//
// Tiling. A workgroup is 4 waves and covers 128 rows x RP columns over one
// K-chunk; each wave owns 32 rows (two 16-row MFMA blocks) and all RP/16
// column blocks. K advances in tiles of 64 (two MFMA k-steps). X fragments go
// straight from HBM to registers, one tile ahead of use; the F tile is read as
// FP32, split once per workgroup and stored to LDS in MFMA operand order.
#pragma once

#include "nmf_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace nmf {
namespace mfma {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kWM = 32;                 // rows per wave
constexpr int kBM = kWaves * kWM;       // rows per workgroup
constexpr int kKT = 64;                 // K per tile
constexpr int kPad = 8;                 // LDS row padding (bf16 elements)


template <typename XT> struct XParts;
template <> struct XParts<float> { static constexpr int n = 3; };
template <> struct XParts<__half> { static constexpr int n = 2; };
template <> struct XParts<__hip_bfloat16> { static constexpr int n = 1; };

__device__ __forceinline__ float bf2f(__bf16 v) { return (float)v; }

// Exact split of 8 FP32 values into NP BF16 parts.
template <int NP>
__device__ __forceinline__ void split8(const float (&x)[8], bf16x8 (&p)[NP])
{
    float r[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = x[j];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const __bf16 h = (__bf16)r[j];
            p[q][j] = h;
            if (q + 1 < NP) r[j] = r[j] - bf2f(h);
        }
    }
}

// Position of k (0..31 within a k-step) in MFMA operand order, where lane
// group g holds positions 8g..8g+7. FP32 X is loaded as two 16-byte pieces per
// lane (k = 4g..4g+3 and 16+4g..16+4g+3) so that each load instruction reads
// 64 contiguous bytes of a row; 16-bit X takes k = 8g..8g+7 in one load.
template <typename XT>
__device__ __forceinline__ int kpos(int kq)
{
    if constexpr (sizeof(XT) == 4) {
        const int hi = kq >> 4, w = kq & 15;
        return ((w >> 2) << 3) + (hi << 2) + (w & 3);
    } else {
        return kq;
    }
}

// Loads the 8 X values of one lane for one k-step (row pointer already at
// the k-step's first column).
template <typename XT>
__device__ __forceinline__ void load_x(const XT *__restrict__ p, int g, float (&x)[8]);

template <>
__device__ __forceinline__ void load_x<float>(const float *__restrict__ p, int g, float (&x)[8])
{
    const float4 a = *reinterpret_cast<const float4 *>(p + 4 * g);
    const float4 b = *reinterpret_cast<const float4 *>(p + 16 + 4 * g);
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
}

template <>
__device__ __forceinline__ void load_x<__hip_bfloat16>(const __hip_bfloat16 *__restrict__ p, int g,
                                                       float (&x)[8])
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p + 8 * g);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        x[2 * j] = __uint_as_float(w[j] << 16);
        x[2 * j + 1] = __uint_as_float(w[j] & 0xffff0000u);
    }
}

template <>
__device__ __forceinline__ void load_x<__half>(const __half *__restrict__ p, int g, float (&x)[8])
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p + 8 * g);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        __half2 h = *reinterpret_cast<const __half2 *>(&w[j]);
        const float2 f = __half22float2(h);
        x[2 * j] = f.x;
        x[2 * j + 1] = f.y;
    }
}

template <int RP, typename XT, int L>
__global__ __launch_bounds__(kWaves * 64, 2) void prod_mfma_kernel(ProdArgs a)
{
    constexpr int NF = L + 1;
    constexpr int NX = (XParts<XT>::n < L + 1) ? XParts<XT>::n : L + 1;
    constexpr int NCB = RP / 16;
    constexpr int LDK = kKT + kPad;
    __shared__ __attribute__((aligned(16))) __bf16 Fs[NF][RP][LDK];

    const DevState *st = a.st;
    int slot = 0;
    if (a.sel != SEL_SLOT0) {
        if (st->done) return;
        slot = (a.sel == SEL_W_Y) ? st->w_y : (st->hp == 1 ? st->h_n : st->h_yn);
    }
    const float *__restrict__ F = a.F_base + slot * a.slot_stride;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, lr = lane & 15;
    const int kc = blockIdx.x % a.nsplit;
    const int64_t rb = blockIdx.x / a.nsplit;
    const int64_t kbeg = (int64_t)kc * a.kchunk;
    int64_t kend = kbeg + a.kchunk;
    if (kend > a.ld) kend = a.ld;
    const int64_t row0 = rb * kBM + wave * kWM;
    const XT *__restrict__ Z = static_cast<const XT *>(a.Z);
    const XT *zr0 = Z + (row0 + lr) * a.ld;
    const XT *zr1 = Z + (row0 + 16 + lr) * a.ld;

    floatx4 acc[2][NCB];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[b][c] = floatx4{0.f, 0.f, 0.f, 0.f};

    // F tile loader: KT x RP FP32 values as float4 chunks.
    constexpr int CHUNKS = kKT * RP / 4;
    constexpr int PER_T = (CHUNKS + kWaves * 64 - 1) / (kWaves * 64);
    float4 fpre[PER_T];
    auto load_f = [&](int64_t k0) {
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const int q = tid + i * kWaves * 64;
            const int kk = q / (RP / 4), c4 = (q % (RP / 4)) * 4;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (q < CHUNKS && k0 + kk < a.K)
                v = *reinterpret_cast<const float4 *>(F + (k0 + kk) * RP + c4);
            fpre[i] = v;
        }
    };
    auto store_f = [&]() {
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const int q = tid + i * kWaves * 64;
            if (q >= CHUNKS) continue;
            const int kk = q / (RP / 4), c4 = (q % (RP / 4)) * 4;
            const int pos = (kk & ~31) + kpos<XT>(kk & 31);
            const float v[4] = {fpre[i].x, fpre[i].y, fpre[i].z, fpre[i].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float r = v[e];
#pragma unroll
                for (int p = 0; p < NF; ++p) {
                    const __bf16 h = (__bf16)r;
                    Fs[p][c4 + e][pos] = h;
                    if (p + 1 < NF) r = r - bf2f(h);
                }
            }
        }
    };

    float xcur[2][2][8], xnext[2][2][8];
    auto load_tile_x = [&](int64_t k0, float (&x)[2][2][8]) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            load_x<XT>(zr0 + k0 + 32 * s, g, x[0][s]);
            load_x<XT>(zr1 + k0 + 32 * s, g, x[1][s]);
        }
    };

    if (kbeg < kend) {
        load_tile_x(kbeg, xcur);
        load_f(kbeg);
    }
    for (int64_t k0 = kbeg; k0 < kend; k0 += kKT) {
        __syncthreads();            // previous tile's LDS reads are done
        store_f();
        const bool more = k0 + kKT < kend;
        if (more) {
            load_tile_x(k0 + kKT, xnext);
            load_f(k0 + kKT);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            bf16x8 ap[2][NX];
            split8<NX>(xcur[0][s], ap[0]);
            split8<NX>(xcur[1][s], ap[1]);
            bf16x8 bp[NCB][NF];
#pragma unroll
            for (int c = 0; c < NCB; ++c)
#pragma unroll
                for (int p = 0; p < NF; ++p)
                    bp[c][p] = *reinterpret_cast<const bf16x8 *>(&Fs[p][c * 16 + lr][32 * s + 8 * g]);
            // Consecutive MFMAs cycle through the 2 x NCB accumulators.
#pragma unroll
            for (int i = 0; i < NX; ++i)
#pragma unroll
                for (int j = 0; j < NF; ++j)
                    if (i + j <= L)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
#pragma unroll
                            for (int c = 0; c < NCB; ++c)
                                acc[b][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    ap[b][i], bp[c][j], acc[b][c], 0, 0, 0);
        }
        if (more) {
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int j = 0; j < 8; ++j) xcur[b][s][j] = xnext[b][s][j];
        }
    }

    // D layout: lane holds column lr of each block, rows 4g..4g+3.
    double *Y = a.Y + (size_t)kc * a.rows_pad * RP;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                Y[(row0 + 16 * b + 4 * g + i) * RP + c * 16 + lr] = (double)acc[b][c][i];
}

template <int RP, typename XT, int L>
void launch_mfma(const ProdArgs &a, hipStream_t s)
{
    const int64_t blocks = (a.rows_pad / kBM) * a.nsplit;
    prod_mfma_kernel<RP, XT, L><<<(unsigned)blocks, kWaves * 64, 0, s>>>(a);
}

}  // namespace mfma
}  // namespace nmf
