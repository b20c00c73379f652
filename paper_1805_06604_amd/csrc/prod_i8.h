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
// Tiling. A workgroup is 4 waves over 128 rows x RP columns and one K-chunk;
// each wave owns 32 rows (two 16-row MFMA blocks) and all RP/16 column blocks.
// K advances in tiles of 64 (one MFMA k-step). The slices of Z go straight
// from HBM to registers, one tile ahead; the FP32 factor tile is sliced once
// per workgroup into LDS in MFMA operand order.
#pragma once

#include "nmf_internal.h"

namespace nmf {
namespace i8 {

typedef int int32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kWM = 32;                 // rows per wave
constexpr int kBM = kWaves * kWM;       // rows per workgroup
constexpr int kKT = 64;                 // K per tile (one MFMA k-step)
constexpr int kSl = 4;                  // slices per value
constexpr int kMaxW = 3;                // kept pairs: a + b <= kMaxW
constexpr int kLdsRow = kKT + 16;       // LDS bytes per factor column (padded)

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

template <int RP>
__global__ __launch_bounds__(kWaves * 64, 1) void prod_i8_kernel(ProdArgs a)
{
    constexpr int NCB = RP / 16;
    __shared__ __attribute__((aligned(16))) signed char Fs[kSl][RP][kLdsRow];
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

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, lr = lane & 15;
    if (tid < RP) s_texp[tid] = slice_exponent(colmax[tid]);

    const int kc = blockIdx.x % a.nsplit;
    const int64_t rb = blockIdx.x / a.nsplit;
    const int64_t kbeg = (int64_t)kc * a.kchunk;
    int64_t kend = kbeg + a.kchunk;
    if (kend > a.ld) kend = a.ld;
    const int64_t row0 = rb * kBM + wave * kWM;
    const int64_t ntile = a.ld / kKT;
    // Z slices: [row][tile][slice][64 bytes]; lane group g reads bytes 16g..16g+15.
    const signed char *Z = static_cast<const signed char *>(a.Z);
    const signed char *zr0 = Z + ((row0 + lr) * ntile) * (kSl * kKT) + 16 * g;
    const signed char *zr1 = Z + ((row0 + 16 + lr) * ntile) * (kSl * kKT) + 16 * g;

    int32x4 acc[2][NCB][kMaxW + 1];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
            for (int w = 0; w <= kMaxW; ++w) acc[b][c][w] = int32x4{0, 0, 0, 0};

    // Factor tile loader: KT x RP FP32 values as float4 chunks.
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
            const float v[4] = {fpre[i].x, fpre[i].y, fpre[i].z, fpre[i].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int d[kSl];
                slice4(ldexpf(v[e], s_texp[c4 + e]), d);
#pragma unroll
                for (int p = 0; p < kSl; ++p) Fs[p][c4 + e][kk] = (signed char)d[p];
            }
        }
    };

    int32x4 zcur[2][kSl], znext[2][kSl];
    auto load_z = [&](int64_t tile, int32x4 (&z)[2][kSl]) {
#pragma unroll
        for (int p = 0; p < kSl; ++p) {
            z[0][p] = *reinterpret_cast<const int32x4 *>(zr0 + tile * (kSl * kKT) + p * kKT);
            z[1][p] = *reinterpret_cast<const int32x4 *>(zr1 + tile * (kSl * kKT) + p * kKT);
        }
    };

    __syncthreads();   // s_texp
    if (kbeg < kend) {
        load_z(kbeg / kKT, zcur);
        load_f(kbeg);
    }
    for (int64_t k0 = kbeg; k0 < kend; k0 += kKT) {
        __syncthreads();            // the previous tile's LDS reads are done
        store_f();
        const bool more = k0 + kKT < kend;
        if (more) {
            load_z(k0 / kKT + 1, znext);
            load_f(k0 + kKT);
        }
        __syncthreads();
        int32x4 bp[NCB][kSl];
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
            for (int p = 0; p < kSl; ++p)
                bp[c][p] = *reinterpret_cast<const int32x4 *>(&Fs[p][c * 16 + lr][16 * g]);
        // Consecutive MFMAs cycle through the 2 x NCB output blocks.
#pragma unroll
        for (int i = 0; i < kSl; ++i)
#pragma unroll
            for (int j = 0; j < kSl; ++j)
                if (i + j <= kMaxW)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int c = 0; c < NCB; ++c)
                            acc[b][c][i + j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                                zcur[b][i], bp[c][j], acc[b][c][i + j], 0, 0, 0);
        if (more) {
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int p = 0; p < kSl; ++p) zcur[b][p] = znext[b][p];
        }
    }

    // D layout: lane holds column lr of each block, rows 4g..4g+3.
    double *Y = a.Y + (size_t)kc * a.rows_pad * RP;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = row0 + 16 * b + 4 * g + i;
            const int se = a.zexp[row];
#pragma unroll
            for (int c = 0; c < NCB; ++c) {
                double v = 0.0;
#pragma unroll
                for (int w = kMaxW; w >= 0; --w) v = v * (1.0 / 128.0) + (double)acc[b][c][w][i];
                Y[row * RP + c * 16 + lr] = ldexp(v, -se - s_texp[c * 16 + lr]);
            }
        }
    }
}

template <int RP>
void launch(const ProdArgs &a, hipStream_t s)
{
    const int64_t blocks = (a.rows_pad / kBM) * a.nsplit;
    prod_i8_kernel<RP><<<(unsigned)blocks, kWaves * 64, 0, s>>>(a);
}

}  // namespace i8
}  // namespace nmf
