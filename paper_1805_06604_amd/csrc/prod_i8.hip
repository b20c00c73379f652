// Exact-integer product kernels (one instance per padded rank) and the
// one-time slicing of X and X^T into the int8 format they stream.
#include "prod_i8.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace nmf {
namespace i8 {
namespace {

__device__ __forceinline__ float as_f32(float v) { return v; }
__device__ __forceinline__ float as_f32(__hip_bfloat16 v) { return __bfloat162float(v); }
__device__ __forceinline__ float as_f32(__half v) { return __half2float(v); }

// One workgroup per row of Z: the row's max |z|, its scale exponent, then the
// four slices of every entry in fragment order ([row / 16][tile][slice][lane]
// [16], lane = row % 16 + 16 (column % 64) / 16). Entries past `cols` (row
// padding) are zero.
template <typename XT>
__global__ __launch_bounds__(256) void slice_rows_kernel(const XT *__restrict__ src, int64_t cols,
                                                         int64_t ld_src, int64_t ntile,
                                                         signed char *__restrict__ dst,
                                                         int *__restrict__ zexp)
{
    __shared__ double sh[4];
    const int64_t row = blockIdx.x;
    const XT *z = src + row * ld_src;
    double mx = 0.0;
    for (int64_t j = threadIdx.x; j < cols; j += 256) mx = fmax(mx, fabs((double)as_f32(z[j])));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    const int s = slice_exponent(mx);
    if (threadIdx.x == 0) zexp[row] = s;
    signed char *out = dst + (row / 16) * ntile * (kSl * 1024) + (row % 16) * 16;
    for (int64_t j = threadIdx.x; j < ntile * kKT; j += 256) {
        const float x = (j < cols) ? as_f32(z[j]) : 0.0f;
        int d[kSl];
        slice4(ldexpf(x, s), d);
        const int64_t t = j / kKT, kk = j % kKT;
#pragma unroll
        for (int p = 0; p < kSl; ++p)
            out[(t * kSl + p) * 1024 + (kk / 16) * 256 + (kk % 16)] = (signed char)d[p];
    }
}

}  // namespace

void launch(int rp, const ProdArgs &a, hipStream_t s, hipEvent_t mid)
{
    switch (rp) {
    case 16: launch<16>(a, s, mid); break;
    case 32: launch<32>(a, s, mid); break;
    case 48: launch<48>(a, s, mid); break;
    case 64: launch<64>(a, s, mid); break;
    default: break;
    }
}

hipError_t launch_group(int rp, const Group &gs, int sblocks, const Group &gp, int pblocks,
                        hipStream_t s)
{
    switch (rp) {
    case 16: launch_group<16>(gs, sblocks, gp, pblocks, s); break;
    case 32: launch_group<32>(gs, sblocks, gp, pblocks, s); break;
    case 48: launch_group<48>(gs, sblocks, gp, pblocks, s); break;
    case 64: launch_group<64>(gs, sblocks, gp, pblocks, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t slice_rows(const void *src, int xdtype, int64_t rows, int64_t cols, int64_t ld_src,
                      int64_t ld_dst, void *dst, int *zexp, hipStream_t s)
{
    const int64_t ntile = ld_dst / kKT;
    switch (xdtype) {
    case 0:
        slice_rows_kernel<float><<<(unsigned)rows, 256, 0, s>>>((const float *)src, cols, ld_src,
                                                               ntile, (signed char *)dst, zexp);
        break;
    case 1:
        slice_rows_kernel<__hip_bfloat16><<<(unsigned)rows, 256, 0, s>>>(
            (const __hip_bfloat16 *)src, cols, ld_src, ntile, (signed char *)dst, zexp);
        break;
    case 2:
        slice_rows_kernel<__half><<<(unsigned)rows, 256, 0, s>>>((const __half *)src, cols, ld_src,
                                                                ntile, (signed char *)dst, zexp);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace i8
}  // namespace nmf
