// Sparse X-streaming products (arXiv 1805.06604: the W^T X and X H^T terms
// of the HALS updates, section 1, for a sparse X as in the text-mining
// experiments of section 5): Y = S F for a CSR operand S (X, or the CSC copy
// of X read as the CSR form of X^T) and a dense FP32 factor F (K x RP).
//
// Work split. The rows of S are cut into items of at most csr_item_nnz(RP)
// nonzeros (built once on the host), one wave per item, so that a row with
// 20000 nonzeros and one with 11 take comparable work units. Within a wave,
// RP / 4 lanes cover the RP columns of one nonzero (a float4 gather of the
// factor row each) and 64 / (RP / 4) nonzeros go side by side. Products of
// FP32 values are exact in FP64 and all sums are FP64 in a fixed order
// (per lane, then over the lane groups, then over the items of a long row),
// so the result is deterministic.
#include "nmf_internal.h"

namespace nmf {
namespace csr {
namespace {

struct Args {
    CsrPlan p;
    const float *F_base;
    int64_t slot_stride;
    int sel;
    const DevState *st;
    double *Y;              // rows_pad x RP
};

__device__ __forceinline__ const float *factor(const Args &a, bool *skip)
{
    int slot = 0;
    *skip = false;
    if (a.sel != SEL_SLOT0) {
        if (a.st->done) {
            *skip = true;
            return nullptr;
        }
        slot = (a.sel == SEL_W_Y) ? a.st->w_y : (a.st->hp == 1 ? a.st->h_n : a.st->h_yn);
    }
    return a.F_base + slot * a.slot_stride;
}

template <int RP>
__global__ __launch_bounds__(256) void spmm_kernel(Args a)
{
    constexpr int W = RP / 4;          // lanes per nonzero
    constexpr int G = 64 / W;          // nonzeros per step
    __shared__ double red[4][G][RP];
    bool skip;
    const float *F = factor(a, &skip);
    if (skip) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int grp = lane / W, l = lane % W;
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;
    if (item >= a.p.nitems) return;            // whole waves only
    const bool active = grp < G;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (active) {
        const int64_t beg = a.p.item_beg[item], end = a.p.item_end[item];
        for (int64_t j = beg + grp; j < end; j += G) {
            const int64_t c = a.p.col[j];
            const double v = (double)a.p.val[j];
            const float4 f = *reinterpret_cast<const float4 *>(F + c * RP + 4 * l);
            acc[0] = fma(v, (double)f.x, acc[0]);
            acc[1] = fma(v, (double)f.y, acc[1]);
            acc[2] = fma(v, (double)f.z, acc[2]);
            acc[3] = fma(v, (double)f.w, acc[3]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wave][grp][4 * l + q] = acc[q];
    }
    __builtin_amdgcn_wave_barrier();           // LDS operations of a wave complete in order
    if (grp == 0) {
        const int32_t slot = a.p.item_slot[item];
        double *dst = (slot < 0) ? a.Y + (int64_t)a.p.item_row[item] * RP
                                 : a.p.partial + (int64_t)slot * RP;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double s = red[wave][0][4 * l + q];
#pragma unroll
            for (int gi = 1; gi < G; ++gi) s += red[wave][gi][4 * l + q];
            dst[4 * l + q] = s;
        }
    }
}

// Rows cut into several items: the sum of their partial rows, in item order.
template <int RP>
__global__ __launch_bounds__(256) void segsum_kernel(Args a)
{
    bool skip;
    (void)factor(a, &skip);
    if (skip) return;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t lr = idx / RP;
    const int c = (int)(idx % RP);
    if (lr >= a.p.nlong) return;
    const int64_t first = a.p.long_first[lr];
    const int cnt = a.p.long_count[lr];
    double s = 0.0;
    for (int q = 0; q < cnt; ++q) s += a.p.partial[(first + q) * RP + c];
    a.Y[(int64_t)a.p.long_row[lr] * RP + c] = s;
}

template <int RP>
void go(const Args &a, hipStream_t s)
{
    if (a.p.nitems > 0)
        spmm_kernel<RP><<<(unsigned)((a.p.nitems + 3) / 4), 256, 0, s>>>(a);
    if (a.p.nlong > 0)
        segsum_kernel<RP><<<(unsigned)((a.p.nlong * RP + 255) / 256), 256, 0, s>>>(a);
}

}  // namespace

hipError_t launch(int rp, const ProdArgs &pa, hipStream_t s)
{
    if (!pa.csr) return hipErrorInvalidValue;
    Args a;
    a.p = *pa.csr;
    a.F_base = pa.F_base;
    a.slot_stride = pa.slot_stride;
    a.sel = pa.sel;
    a.st = pa.st;
    a.Y = pa.Y;
    switch (rp) {
    case 16: go<16>(a, s); break;
    case 32: go<32>(a, s); break;
    case 48: go<48>(a, s); break;
    case 64: go<64>(a, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace csr
}  // namespace nmf
