// Dense X-streaming products and the set-up of X (arXiv 1805.06604: the
// W^T X and X H^T terms of the closed-form updates, section 1 and Remark 1).
//
// Both products of an outer iteration have one shape, Y = Z F with Z row-major
// (rows x K) and F row-major (K x RP): A = X H_w^T uses Z = X, F = H_w^T, and
// C^T = X^T W_y uses Z = X^T (kept resident as its own row-major copy), F = W_y.
// Each pass therefore reads Z exactly once, front to back.
#include "nmf_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>

namespace nmf {
namespace {

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(__hip_bfloat16 v) { return __bfloat162float(v); }
__device__ __forceinline__ float to_f32(__half v) { return __half2float(v); }

__device__ __forceinline__ const float *select_factor(const float *base, int64_t stride,
                                                      int sel, const DevState *st,
                                                      bool *skip)
{
    int slot = 0;
    *skip = false;
    if (sel != SEL_SLOT0) {
        if (st->done) { *skip = true; return nullptr; }
        slot = (sel == SEL_W_Y) ? st->w_y : (st->hp == 1 ? st->h_n : st->h_yn);
    }
    return base + slot * stride;
}

// Vector-ALU product in FP64: a 64-row tile per workgroup, K in steps of 32
// staged through LDS as FP32 (exact), 4 x RP/16 outputs per thread, products
// and sums in FP64 over the whole row. This is the reference-accuracy path.
template <int RP, typename XT>
__global__ __launch_bounds__(256) void prod_fp64_kernel(ProdArgs a)
{
    constexpr int BM = 64, BK = 32, TN = RP / 16;
    __shared__ __attribute__((aligned(16))) float Zs[BK][BM + 4];
    __shared__ float Fs[BK][RP];
    bool skip;
    const float *F = select_factor(a.F_base, a.slot_stride, a.sel, a.st, &skip);
    if (skip) return;
    const XT *__restrict__ Z = static_cast<const XT *>(a.Z);

    const int tid = threadIdx.x;
    const int tr = tid >> 4, tc = tid & 15;
    const int64_t row0 = (int64_t)blockIdx.x * BM;
    double acc[4][TN];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = 0.0;

    const int lr = tid >> 2, lc = (tid & 3) * 8;
    const int64_t grow = row0 + lr;
    for (int64_t k0 = 0; k0 < a.K; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t gk = k0 + lc + q;
            float v = 0.f;
            if (grow < a.rows && gk < a.K) v = to_f32(Z[grow * a.ld + gk]);
            Zs[lc + q][lr] = v;
        }
        for (int e = tid; e < BK * RP; e += 256) {
            const int kk = e / RP, c = e % RP;
            const int64_t gk = k0 + kk;
            Fs[kk][c] = (gk < a.K) ? F[gk * RP + c] : 0.f;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < BK; ++kk) {
            const float4 z = *reinterpret_cast<const float4 *>(&Zs[kk][tr * 4]);
            double f[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) f[j] = (double)Fs[kk][tc + 16 * j];
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                acc[0][j] = fma((double)z.x, f[j], acc[0][j]);
                acc[1][j] = fma((double)z.y, f[j], acc[1][j]);
                acc[2][j] = fma((double)z.z, f[j], acc[2][j]);
                acc[3][j] = fma((double)z.w, f[j], acc[3][j]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + tr * 4 + i;
        if (row < a.rows) {
#pragma unroll
            for (int j = 0; j < TN; ++j) a.Y[row * RP + tc + 16 * j] = acc[i][j];
        }
    }
}

template <int RP, typename XT>
void go_prod_fp64(const ProdArgs &a, hipStream_t s)
{
    const int blocks = (int)((a.rows + 63) / 64);
    prod_fp64_kernel<RP, XT><<<blocks, 256, 0, s>>>(a);
}

template <typename XT>
hipError_t prod_fp64_dispatch(int rp, const ProdArgs &a, hipStream_t s)
{
    switch (rp) {
    case 16: go_prod_fp64<16, XT>(a, s); break;
    case 32: go_prod_fp64<32, XT>(a, s); break;
    case 48: go_prod_fp64<48, XT>(a, s); break;
    case 64: go_prod_fp64<64, XT>(a, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ X set-up

__device__ __forceinline__ void store_as(float *p, float v) { *p = v; }
__device__ __forceinline__ void store_as(__hip_bfloat16 *p, float v) { *p = __float2bfloat16(v); }
__device__ __forceinline__ void store_as(__half *p, float v) { *p = __float2half(v); }

// Converts a 32 x 32 tile of the FP32 source into X and, transposed, X^T.
template <typename XT>
__global__ __launch_bounds__(256) void convert_x_kernel(const float *__restrict__ src,
                                                        int64_t m, int64_t n,
                                                        XT *__restrict__ X, int64_t ldx,
                                                        XT *__restrict__ Xt, int64_t ldxt)
{
    __shared__ float tile[32][33];
    const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int q = ty; q < 32; q += 8) {
        const int64_t i = i0 + q, j = j0 + tx;
        float v = 0.f;
        if (i < m && j < n) {
            v = src[i * n + j];
            store_as(&X[i * ldx + j], v);
        }
        tile[q][tx] = v;
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int64_t j = j0 + q, i = i0 + tx;
        if (i < m && j < n) store_as(&Xt[j * ldxt + i], tile[tx][q]);
    }
}

// Sum of squares in FP64 of the stored values (the objective uses ||X||^2 of
// exactly the matrix the products stream).
template <typename T>
__global__ __launch_bounds__(256) void sumsq_kernel(const T *__restrict__ v, int64_t count,
                                                    double *__restrict__ part)
{
    __shared__ double sh[4];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * 256) {
        const double x = (double)to_f32(v[e]);
        s += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void sum_parts_kernel(const double *__restrict__ part, int nblk, double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[b];
        *out = s;
    }
}

}  // namespace

namespace i8 {
void launch(int rp, const ProdArgs &a, hipStream_t s, hipEvent_t mid);
}
namespace x16 {
hipError_t launch(int rp, int xdtype, const ProdArgs &a, hipStream_t s, hipEvent_t mid);
}
namespace csr {
hipError_t launch(int rp, const ProdArgs &a, hipStream_t s);
}

hipError_t launch_product(int rp, int xdtype, int kernel, const ProdArgs &a, hipStream_t s,
                          hipEvent_t mid)
{
    if (rp != 16 && rp != 32 && rp != 48 && rp != 64) return hipErrorInvalidValue;
    if (kernel == PK_MFMA_I8) {
        i8::launch(rp, a, s, mid);
        return hipGetLastError();
    }
    if (kernel == PK_MFMA_X16) return x16::launch(rp, xdtype, a, s, mid);
    // No slicing step: the "between" mark goes before the product.
    if (mid) (void)hipEventRecord(mid, s);
    if (kernel == PK_CSR) return csr::launch(rp, a, s);
    if (kernel == PK_VALU) {
        switch (xdtype) {
        case 0: return prod_fp64_dispatch<float>(rp, a, s);
        case 1: return prod_fp64_dispatch<__hip_bfloat16>(rp, a, s);
        case 2: return prod_fp64_dispatch<__half>(rp, a, s);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_convert_x(const float *src, int64_t m, int64_t n, int xdtype, void *X,
                            int64_t ldx, void *Xt, int64_t ldxt, hipStream_t s)
{
    const dim3 grid((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32));
    switch (xdtype) {
    case 0:
        convert_x_kernel<float><<<grid, 256, 0, s>>>(src, m, n, (float *)X, ldx, (float *)Xt, ldxt);
        break;
    case 1:
        convert_x_kernel<__hip_bfloat16><<<grid, 256, 0, s>>>(src, m, n, (__hip_bfloat16 *)X, ldx,
                                                              (__hip_bfloat16 *)Xt, ldxt);
        break;
    case 2:
        convert_x_kernel<__half><<<grid, 256, 0, s>>>(src, m, n, (__half *)X, ldx, (__half *)Xt, ldxt);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sumsq_typed(const void *v, int xdtype, int64_t count, double *part, int nblk,
                              double *out, hipStream_t s)
{
    switch (xdtype) {
    case 0: sumsq_kernel<float><<<nblk, 256, 0, s>>>((const float *)v, count, part); break;
    case 1: sumsq_kernel<__hip_bfloat16><<<nblk, 256, 0, s>>>((const __hip_bfloat16 *)v, count, part); break;
    case 2: sumsq_kernel<__half><<<nblk, 256, 0, s>>>((const __half *)v, count, part); break;
    default: return hipErrorInvalidValue;
    }
    sum_parts_kernel<<<1, 64, 0, s>>>(part, nblk, out);
    return hipGetLastError();
}

hipError_t launch_sumsq(const float *src, int64_t count, double *part, int nblk, double *out,
                        hipStream_t s)
{
    return launch_sumsq_typed(src, 0, count, part, nblk, out, s);
}

}  // namespace nmf
