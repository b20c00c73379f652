// 16-bit X products on the 16-bit matrix cores (one instance per padded rank and
// storage type) and the one-time copy of X and X^T into their fragment order.
#include "prod_x16.h"

namespace nmf {
namespace x16 {
namespace {

// One 16-byte fragment per thread: lane lr + 16 g of k-step s of tile t of
// row block rb holds row 16 rb + lr, columns 64 t + 32 s + 8 g .. + 7.
__global__ __launch_bounds__(256) void frag16_kernel(const uint4 *__restrict__ src, int64_t rows_pad,
                                                     int64_t ld, uint4 *__restrict__ dst)
{
    const int64_t ntile = ld / kKT;
    const int64_t total = rows_pad * ld / 8;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(q & 63), s = (int)((q >> 6) & 1);
        const int64_t t = (q >> 7) % ntile, rb = (q >> 7) / ntile;
        const int64_t row = 16 * rb + (lane & 15);
        const int64_t col = kKT * t + 32 * s + 8 * (lane >> 4);
        dst[q] = src[(row * ld + col) / 8];
    }
}

}  // namespace

hipError_t to_fragments(const void *src, int64_t rows_pad, int64_t ld, void *dst, hipStream_t s)
{
    if (rows_pad % 16 != 0 || ld % kKT != 0) return hipErrorInvalidValue;
    frag16_kernel<<<4096, 256, 0, s>>>(static_cast<const uint4 *>(src), rows_pad, ld,
                                       static_cast<uint4 *>(dst));
    return hipGetLastError();
}

hipError_t launch(int rp, int xdtype, const ProdArgs &a, hipStream_t s, hipEvent_t mid)
{
#define NMF_X16(RPV)                                                        \
    if (xdtype == 1) x16::launch<RPV, __hip_bfloat16>(a, s, mid);           \
    else if (xdtype == 2) x16::launch<RPV, __half>(a, s, mid);              \
    else return hipErrorInvalidValue;
    switch (rp) {
    case 16: NMF_X16(16) break;
    case 32: NMF_X16(32) break;
    case 48: NMF_X16(48) break;
    case 64: NMF_X16(64) break;
    default: return hipErrorInvalidValue;
    }
#undef NMF_X16
    return hipGetLastError();
}

}  // namespace x16
}  // namespace nmf
