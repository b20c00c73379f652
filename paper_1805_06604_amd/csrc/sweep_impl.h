// Templates of the HALS sweeps with fused epilogues, Gram reductions and the FP64 decision
// step of E-A-HALS (arXiv 1805.06604: section 1 closed form, Algorithm 2,
// Algorithm 3, Remark 1).
//
// Layout: one factor row per lane. W rows and H^T rows (columns of H) have the
// same shape (RP floats), so both blocks use the same code; the Gram matrix of
// the other factor is read with wave-uniform addresses (scalar loads).
#pragma once

#include "nmf_internal.h"

#include <algorithm>
#include <cmath>

namespace nmf {
namespace sweep {

constexpr int kThreads = kRowsPerBlock;

// ---------------------------------------------------------------- row I/O

template <int RP>
__device__ __forceinline__ void load_row(const float *__restrict__ p, float (&v)[RP])
{
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int i = 0; i < RP / 4; ++i) {
        const float4 t = q[i];
        v[4 * i] = t.x; v[4 * i + 1] = t.y; v[4 * i + 2] = t.z; v[4 * i + 3] = t.w;
    }
}

template <int RP>
__device__ __forceinline__ void store_row(float *__restrict__ p, const float (&v)[RP])
{
    float4 *q = reinterpret_cast<float4 *>(p);
#pragma unroll
    for (int i = 0; i < RP / 4; ++i)
        q[i] = make_float4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
}

// Linear term of one row: the product kernel's K-chunk partials are summed in
// FP64, in a fixed order, into the first partial slice (the row belongs to
// this thread alone); returns the row's address there.
template <int RP>
__device__ __forceinline__ const double *sum_lin(double *__restrict__ lin, int nsplit,
                                                 int64_t split_stride, int64_t row)
{
    double *dst = lin + row * RP;
    if (nsplit > 1) {
#pragma unroll
        for (int q = 0; q < RP / 2; ++q) {
            double2 acc = *reinterpret_cast<const double2 *>(dst + 2 * q);
            for (int sp = 1; sp < nsplit; ++sp) {
                const double2 v = *reinterpret_cast<const double2 *>(dst + sp * split_stride + 2 * q);
                acc.x += v.x;
                acc.y += v.y;
            }
            *reinterpret_cast<double2 *>(dst + 2 * q) = acc;
        }
    }
    return dst;
}

// <x, c> in FP64 for an FP32 row x and an FP64 row c in memory.
template <int RP>
__device__ __forceinline__ double dot_lin(const float (&x)[RP], const double *__restrict__ c)
{
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < RP / 2; ++q) {
        const double2 v = *reinterpret_cast<const double2 *>(c + 2 * q);
        s = fma((double)x[2 * q], v.x, s);
        s = fma((double)x[2 * q + 1], v.y, s);
    }
    return s;
}

// --------------------------------------------------------------- the sweep

// K sweeps of the HALS closed form over the coordinates of one row x, with
// linear term c (a row of X H^T, or a column of W^T X) and the symmetric Gram
// matrix G of the fixed factor (section 1):
//     x_k <- max(0, x_k + (c_k - G(k,:) x) / G(k,k)),   k ascending,
// each update used at once (Gauss-Seidel); this is the Sigma_{j != k} form of
// the paper written around the current x_k. The numerator is a difference of
// nearly equal terms once the iterate settles, so x, c, G and the sums are
// FP64. The coordinates go in blocks of 16: t = c_b - G(b,:) x is formed for
// the whole block with 16 independent accumulators (one uniform load of a
// Gram row segment feeds 16 FMAs), then the block is updated in order, each
// change of x_k corrected into the t of the later coordinates of the block. A
// zero inverse diagonal (k >= r, or a zero G(k,k)) leaves max(0, x_k).
typedef const __attribute__((address_space(4))) double *gram_ptr;

// Loads N consecutive Gram entries with wave-uniform (scalar) loads.
template <int N>
__device__ __forceinline__ void load_g(double (&g)[N], gram_ptr p)
{
#pragma unroll
    for (int q = 0; q < N; ++q) g[q] = p[q];
}

// Coordinates per Gauss-Seidel block of the sweep.
constexpr int kGS = 8;

// The block loop is a runtime loop and x rotates by kGS registers per block,
// so that the current block always sits in x[0..kGS): register indices stay
// static and the loop body stays small enough for the scheduler to keep the
// scalar Gram loads close to their use. x[j] holds coordinate (j + b) mod RP.
template <int RP>
__device__ __forceinline__ void hals_sweeps(double (&x)[RP], const double *crow,
                                            const double *__restrict__ G, int K)
{
    // The Gram matrix is read through the constant address space, so that
    // every access is a scalar (wave-uniform) load; no block of a sweep
    // kernel writes the Gram matrix it reads.
    const gram_ptr Gs = (gram_ptr)G;
    for (int s = 0; s < K; ++s) {
#pragma unroll 1
        for (int b = 0; b < RP; b += kGS) {
            double t[kGS];
#pragma unroll
            for (int q = 0; q < kGS; q += 2) {
                const double2 v = *reinterpret_cast<const double2 *>(crow + b + q);
                t[q] = v.x;
                t[q + 1] = v.y;
            }
            // t = c_b - G(b, :) x over the rows of G (= its columns).
#pragma unroll
            for (int j = 0; j < RP; ++j) {
                int l = j + b;
                if (l >= RP) l -= RP;
                double g[kGS];
                load_g<kGS>(g, Gs + l * RP + b);
#pragma unroll
                for (int q = 0; q < kGS; ++q) t[q] = fma(-g[q], x[j], t[q]);
            }
            // In-block Gauss-Seidel: x_k, then the later t of the block.
#pragma unroll
            for (int q = 0; q < kGS; ++q) {
                const int k = b + q;
                const double xn = fmax(fma(t[q], (double)Gs[RP * RP + k], x[q]), 0.0);
                const double d = xn - x[q];
                x[q] = xn;
#pragma unroll
                for (int q2 = q + 1; q2 < kGS; ++q2)
                    t[q2] = fma(-(double)Gs[k * RP + b + q2], d, t[q2]);
            }
            // Rotate: the next block moves to x[0..kGS).
            double keep[kGS];
#pragma unroll
            for (int q = 0; q < kGS; ++q) keep[q] = x[q];
#pragma unroll
            for (int j = 0; j < RP - kGS; ++j) x[j] = x[j + kGS];
#pragma unroll
            for (int q = 0; q < kGS; ++q) x[RP - kGS + q] = keep[q];
        }
    }
}

// ------------------------------------------------------------- reductions

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return t;
}

// Partial Gram v v^T of the block's 256 rows (FP32 values, FP64 products and
// sums), written to out (RP*RP), and the block's column maxima max |v_k|,
// written to out_max (RP). Each wave's 64 rows pass through an LDS tile in
// turn.
template <int RP>
__device__ void block_gram(const float (&v)[RP], double *__restrict__ out,
                           double *__restrict__ out_max, float (*tile)[RP + 1])
{
    constexpr int PER = RP * RP / kThreads;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    double acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] = 0.0;
    float cmax = 0.0f;
    for (int w = 0; w < kThreads / 64; ++w) {
        if (wave == w) {
#pragma unroll
            for (int k = 0; k < RP; ++k) tile[lane][k] = v[k];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + kThreads * q, k = e / RP, l = e % RP;
            double a = acc[q];
            for (int row = 0; row < 64; ++row)
                a = fma((double)tile[row][k], (double)tile[row][l], a);
            acc[q] = a;
        }
        if (tid < RP)
            for (int row = 0; row < 64; ++row) cmax = fmaxf(cmax, fabsf(tile[row][tid]));
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) out[tid + kThreads * q] = acc[q];
    if (tid < RP) out_max[tid] = cmax;
}

// Marks this block done; returns true in every thread of the last block to
// finish. Partials written before the call are visible to that block. The
// blocks of a grid run on all XCDs, whose L2 caches are not coherent with one
// another, so the counter is updated at system scope (coherent at memory);
// the fences write back and invalidate the L2 for the partials.
__device__ inline bool last_block(uint32_t *counter, int *s_flag)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t prev =
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_SYSTEM);
        *s_flag = (prev == gridDim.x - 1);
    }
    __syncthreads();
    const bool last = *s_flag != 0;
    if (last) __threadfence();
    return last;
}

// Re-arms a last-block counter for the next launch (system scope, like the
// increments).
__device__ inline void reset_counter(uint32_t *counter)
{
    __hip_atomic_store(counter, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Sum of the partial Grams `which` (0 or 1) over nblk blocks in FP64, fixed
// block order; writes the Gram, its inverse diagonal and the column maxima
// to G and keeps this thread's Gram entries in g64.
template <int RP>
__device__ void finish_gram(const double *__restrict__ part, const double *__restrict__ part_m,
                            int nblk, int which, double *__restrict__ G, int r,
                            double (&g64)[RP * RP / kThreads])
{
    if (threadIdx.x < RP) {
        double mx = 0.0;
        for (int b = 0; b < nblk; ++b) mx = fmax(mx, part_m[((size_t)b * 2 + which) * RP + threadIdx.x]);
        G[RP * RP + RP + threadIdx.x] = mx;
    }
    constexpr int PER = RP * RP / kThreads;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + kThreads * q;
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[((size_t)b * 2 + which) * RP * RP + e];
        g64[q] = s;
        G[e] = s;
        const int k = e / RP, l = e % RP;
        if (k == l) G[RP * RP + k] = (k < r && s > 0.0) ? 1.0 / s : 0.0;
    }
}

// ------------------------------------------------------ decision (a8 row)

// Error, accept/restart (Algorithm 2) and beta update (Algorithm 3), run by
// one thread after <W_n, A> (s1) and <W_n^T W_n, H_w H_w^T> (s2) are known.
__device__ inline void decide(DevState *st, double s1, double s2, double *trace,
                       uint8_t *accepted, double *beta_used)
{
    const double e2 = st->nx2 - 2.0 * s1 + s2;               // Remark 1
    const double e = sqrt(e2 > 0.0 ? e2 : 0.0);
    const int k = st->k + 1;
    trace[k] = e / sqrt(st->nx2);
    const double e_cmp = (st->flags & 2) ? st->e_acc : st->e_prev;
    const bool fin = isfinite(e);
    const bool dec = fin && !(e > e_cmp);                     // ties accept
    const double bk = st->beta;
    accepted[k - 1] = dec ? 1 : 0;
    beta_used[k - 1] = bk;
    double next;
    if (dec) {
        st->w_acc = st->w_n; st->w_y = st->w_yn;
        st->h_acc = st->h_n; st->h_y = st->h_yn;
        st->e_acc = e;
        next = fmin(st->betabar, st->gamma * bk);
        st->betabar = fmin(1.0, st->gamma_bar * st->betabar);
        st->beta_acc = bk;
    } else {
        st->w_y = st->w_acc;                                  // restart
        st->h_y = st->h_acc;
        next = bk / st->eta;
        st->betabar = (st->flags & 1) ? st->beta_acc : st->beta_prev;
    }
    st->beta_prev = bk;
    st->beta = next;
    if (fin) st->e_prev = e;
    st->k = k;
    plan_slots(st->w_acc, st->w_y, &st->w_n, &st->w_yn);
    plan_slots(st->h_acc, st->h_y, &st->h_n, &st->h_yn);
    bool stop = k >= st->max_iter;
    if (st->tol > 0.0 && dec && fabs(trace[k] - trace[k - 1]) < st->tol) stop = true;
    if (stop) st->done = 1;
}

// ------------------------------------------------------------- the kernels

struct SweepArgs {
    int64_t rows;
    int r, K, nblk;
    double *lin;           // nsplit x (rows_pad x RP) partials of the linear term
    int nsplit;
    int64_t split_stride;
    float *fac;            // factor slots
    int64_t slot_stride;
    const double *GW;      // Gram slots of W
    double *GWout;         // = GW (written by the W side)
    double *GH;            // Gram of H_w
    double *part_g;
    double *part_m;
    double *part_d;
    uint32_t *counter;
    DevState *st;
    double *trace;
    uint8_t *accepted;
    double *beta_used;
};

// Rounds the FP64 iterate to the FP32 values that are stored.
template <int RP>
__device__ __forceinline__ void to_f32(const double (&x)[RP], float (&xf)[RP])
{
#pragma unroll
    for (int k = 0; k < RP; ++k) xf[k] = (float)x[k];
}

// a3 + a4: H_n from H_y by K sweeps with W_y^T X and W_y^T W_y; H_y' =
// H_n + beta (H_n - H) (projected for hp = 3); Gram of H_w into GH.
template <int RP>
__global__ __launch_bounds__(kThreads) void sweep_h_kernel(SweepArgs a)
{
    __shared__ float tile[64][RP + 1];
    __shared__ int s_last;
    DevState *st = a.st;
    if (st->done) return;
    const int h_acc = st->h_acc, h_y = st->h_y, h_n = st->h_n, h_yn = st->h_yn;
    const int hp = st->hp;
    const double beta = st->beta;
    const double *G = a.GW + (size_t)st->w_y * gram_stride(RP);
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;

    float w[RP];
    if (j < a.rows) {
        double x[RP];
        {
            float x0[RP];
            load_row<RP>(a.fac + h_y * a.slot_stride + j * RP, x0);
#pragma unroll
            for (int k = 0; k < RP; ++k) x[k] = x0[k];
        }
        const double *c = sum_lin<RP>(a.lin, a.nsplit, a.split_stride, j);
        hals_sweeps<RP>(x, c, G, a.K);
        float xf[RP], h[RP];
        to_f32<RP>(x, xf);
        store_row<RP>(a.fac + h_n * a.slot_stride + j * RP, xf);
        load_row<RP>(a.fac + h_acc * a.slot_stride + j * RP, h);
#pragma unroll
        for (int k = 0; k < RP; ++k) {
            double y = fma(beta, (double)xf[k] - (double)h[k], (double)xf[k]);
            if (hp == 3) y = fmax(y, 0.0);
            h[k] = (float)y;
        }
        store_row<RP>(a.fac + h_yn * a.slot_stride + j * RP, h);
#pragma unroll
        for (int k = 0; k < RP; ++k) w[k] = (hp == 1) ? xf[k] : h[k];
    } else {
#pragma unroll
        for (int k = 0; k < RP; ++k) w[k] = 0.f;
    }
    block_gram<RP>(w, a.part_g + (size_t)blockIdx.x * 2 * RP * RP,
                   a.part_m + (size_t)blockIdx.x * 2 * RP, tile);
    if (!last_block(a.counter, &s_last)) return;
    double g64[RP * RP / kThreads];
    finish_gram<RP>(a.part_g, a.part_m, a.nblk, 0, a.GH, a.r, g64);
    if (threadIdx.x == 0) reset_counter(a.counter);
}

// a6 + a7 + a8: W_n from W_y by K sweeps with X H_w^T and H_w H_w^T;
// W_y' = W_n + beta (W_n - W); partial <W_n, A>, Gram(W_n), Gram(W_y'); the
// last block finishes them and takes the decision.
template <int RP>
__global__ __launch_bounds__(kThreads) void sweep_w_kernel(SweepArgs a)
{
    __shared__ float tile[64][RP + 1];
    __shared__ double shd[4];
    __shared__ int s_last;
    DevState *st = a.st;
    if (st->done) return;
    const int w_acc = st->w_acc, w_y = st->w_y, w_n = st->w_n, w_yn = st->w_yn;
    const double beta = st->beta;
    const double *G = a.GH;
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;

    float xf[RP], y[RP];
    double s1 = 0.0;
    if (i < a.rows) {
        double x[RP];
        {
            float x0[RP];
            load_row<RP>(a.fac + w_y * a.slot_stride + i * RP, x0);
#pragma unroll
            for (int k = 0; k < RP; ++k) x[k] = x0[k];
        }
        const double *c = sum_lin<RP>(a.lin, a.nsplit, a.split_stride, i);
        hals_sweeps<RP>(x, c, G, a.K);
        to_f32<RP>(x, xf);
        store_row<RP>(a.fac + w_n * a.slot_stride + i * RP, xf);
        s1 = dot_lin<RP>(xf, c);
        load_row<RP>(a.fac + w_acc * a.slot_stride + i * RP, y);
#pragma unroll
        for (int k = 0; k < RP; ++k)
            y[k] = (float)fma(beta, (double)xf[k] - (double)y[k], (double)xf[k]);
        store_row<RP>(a.fac + w_yn * a.slot_stride + i * RP, y);
    } else {
#pragma unroll
        for (int k = 0; k < RP; ++k) { xf[k] = 0.f; y[k] = 0.f; }
    }
    double *pb = a.part_g + (size_t)blockIdx.x * 2 * RP * RP;
    double *pm = a.part_m + (size_t)blockIdx.x * 2 * RP;
    block_gram<RP>(xf, pb, pm, tile);
    block_gram<RP>(y, pb + RP * RP, pm + RP, tile);
    s1 = block_sum(s1, shd);
    if (threadIdx.x == 0) a.part_d[blockIdx.x] = s1;
    if (!last_block(a.counter, &s_last)) return;

    double gn[RP * RP / kThreads], gy[RP * RP / kThreads];
    finish_gram<RP>(a.part_g, a.part_m, a.nblk, 0, a.GWout + (size_t)w_n * gram_stride(RP), a.r, gn);
    finish_gram<RP>(a.part_g, a.part_m, a.nblk, 1, a.GWout + (size_t)w_yn * gram_stride(RP), a.r, gy);
    double s2 = 0.0;
#pragma unroll
    for (int q = 0; q < RP * RP / kThreads; ++q)
        s2 = fma(gn[q], a.GH[threadIdx.x + kThreads * q], s2);
    s2 = block_sum(s2, shd);
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int b = 0; b < a.nblk; ++b) t += a.part_d[b];
        decide(st, t, s2, a.trace, a.accepted, a.beta_used);
        reset_counter(a.counter);
    }
}

// Set-up: Gram of the rows of slot 0 of `fac` into Gout. With `with_error`
// (W side) it also forms <W0, A> and, in the last block, e(0) (Alg. 2, first
// step, via Remark 1) and the initial state.
template <int RP>
__global__ __launch_bounds__(kThreads) void setup_gram_kernel(SweepArgs a, int with_error)
{
    __shared__ float tile[64][RP + 1];
    __shared__ double shd[4];
    __shared__ int s_last;
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    float x[RP];
    double s1 = 0.0;
    if (i < a.rows) {
        load_row<RP>(a.fac + i * RP, x);
        if (with_error) s1 = dot_lin<RP>(x, sum_lin<RP>(a.lin, a.nsplit, a.split_stride, i));
    } else {
#pragma unroll
        for (int k = 0; k < RP; ++k) x[k] = 0.f;
    }
    block_gram<RP>(x, a.part_g + (size_t)blockIdx.x * 2 * RP * RP,
                   a.part_m + (size_t)blockIdx.x * 2 * RP, tile);
    if (with_error) {
        s1 = block_sum(s1, shd);
        if (threadIdx.x == 0) a.part_d[blockIdx.x] = s1;
    }
    if (!last_block(a.counter, &s_last)) return;
    double g[RP * RP / kThreads];
    finish_gram<RP>(a.part_g, a.part_m, a.nblk, 0, a.GWout, a.r, g);
    if (with_error) {
        double s2 = 0.0;
#pragma unroll
        for (int q = 0; q < RP * RP / kThreads; ++q)
            s2 = fma(g[q], a.GH[threadIdx.x + kThreads * q], s2);
        s2 = block_sum(s2, shd);
        if (threadIdx.x == 0) {
            DevState *st = a.st;
            double t = 0.0;
            for (int b = 0; b < a.nblk; ++b) t += a.part_d[b];
            const double e2 = st->nx2 - 2.0 * t + s2;
            const double e = sqrt(e2 > 0.0 ? e2 : 0.0);
            a.trace[0] = e / sqrt(st->nx2);
            st->e0 = e;
            st->e_prev = e;
            st->e_acc = e;
            if (!isfinite(e) || st->max_iter == 0) st->done = 1;
        }
    }
    if (threadIdx.x == 0) reset_counter(a.counter);
}

template <int RP>
SweepArgs base_args(const Buffers &b, int64_t rows, int r, int K)
{
    SweepArgs a{};
    a.rows = rows;
    a.r = r;
    a.K = K;
    a.nblk = (int)((rows + kThreads - 1) / kThreads);
    a.part_g = b.part_g;
    a.part_m = b.part_m;
    a.part_d = b.part_d;
    a.st = b.st;
    a.trace = b.trace;
    a.accepted = b.accepted;
    a.beta_used = b.beta_used;
    a.GW = b.GW;
    a.GWout = b.GW;
    a.GH = b.GH;
    return a;
}

// Enqueues the sweep kernels of one padded rank (one translation unit each).
template <int RP>
struct Launch {
    static void sweep_h(int64_t n, int r, int K, const Buffers &b, hipStream_t s)
    {
        SweepArgs a = base_args<RP>(b, n, r, K);
        a.lin = b.Ct;
        a.nsplit = b.nsplit_c;
        a.split_stride = b.n_pad * RP;
        a.fac = b.Hf;
        a.slot_stride = n * RP;
        a.counter = b.counters + CNT_H;
        sweep_h_kernel<RP><<<a.nblk, kThreads, 0, s>>>(a);
    }
    static void sweep_w(int64_t m, int r, int K, const Buffers &b, hipStream_t s)
    {
        SweepArgs a = base_args<RP>(b, m, r, K);
        a.lin = b.A;
        a.nsplit = b.nsplit_a;
        a.split_stride = b.m_pad * RP;
        a.fac = b.Wf;
        a.slot_stride = m * RP;
        a.counter = b.counters + CNT_W;
        sweep_w_kernel<RP><<<a.nblk, kThreads, 0, s>>>(a);
    }
    static void setup_h(int64_t n, int r, const Buffers &b, hipStream_t s)
    {
        SweepArgs a = base_args<RP>(b, n, r, 0);
        a.fac = b.Hf;
        a.GWout = b.GH;
        a.counter = b.counters + CNT_G;
        setup_gram_kernel<RP><<<a.nblk, kThreads, 0, s>>>(a, 0);
    }
    static void setup_err(int64_t m, int r, const Buffers &b, hipStream_t s)
    {
        SweepArgs a = base_args<RP>(b, m, r, 0);
        a.fac = b.Wf;
        a.lin = b.A;
        a.nsplit = b.nsplit_a;
        a.split_stride = b.m_pad * RP;
        a.GWout = b.GW;   // slot 0
        a.counter = b.counters + CNT_G;
        setup_gram_kernel<RP><<<a.nblk, kThreads, 0, s>>>(a, 1);
    }
};

}  // namespace sweep
}  // namespace nmf
