// HALS sweeps with fused epilogues, Gram reductions and the FP64 decision step
// of E-A-HALS (arXiv 1805.06604: section 1 closed form, Algorithm 2,
// Algorithm 3, Remark 1).
//
// Each half-iteration is two launches:
//  * hals_kernel: a workgroup is 4 waves over 64 factor rows, each wave owns
//    16 rows. The K Gauss-Seidel sweeps of the closed form run in FP64 with
//    the coordinates in blocks of 16: the block's numerators t = c_b - x G_b
//    come from the FP64 matrix cores (v_mfma_f64_16x16x4f64, the Gram block in
//    registers in B-operand order), then the 16 coordinates of the block are
//    updated in order, lane q of each 16-lane row owning coordinate q and
//    passing its change to the other lanes with one 64-bit row broadcast
//    (DPP row_newbcast). The epilogue stores the new factor rows and the
//    extrapolated rows, and writes one record per workgroup: the partial Gram
//    matrices (FP64 matrix cores again), column maxima and <W_n, A>.
//  * finish_kernel: sums the records in a fixed order (deterministic) and
//    writes the Gram matrices with their inverse diagonals and column maxima;
//    on W sides a one-workgroup decide_kernel follows (the launch boundary
//    makes the sums visible), which forms the error of Remark 1 and takes the
//    decision.
//
// Register layout of the 16 x 16 tiles (16 rows of a wave, 16 coordinates):
// lane l = lr + 16 g holds, in its 4 values v, rows 4 v + g of coordinate lr
// ("D layout", the accumulator layout of the FP64 MFMA), and for the A operand
// of the sweep product x[row lr][coordinate 4 s + g] for k-step s.
#pragma once

#include "nmf_internal.h"

#include <cmath>
#include <utility>

namespace nmf {
namespace sweep {

typedef double double4v __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kRows = kRowsPerBlock;       // rows per workgroup (16 per wave)
constexpr int kThreads = kWaves * 64;
static_assert(kRows == kWaves * 16, "one 16-row tile per wave");

enum Mode { SETUP_H = 0, SETUP_W = 1, SWEEP_H = 2, SWEEP_W = 3 };

template <int M>
struct ModeInfo {
    static constexpr bool sweeps = (M == SWEEP_H || M == SWEEP_W);
    static constexpr bool lin = (M != SETUP_H);            // reads the linear term
    static constexpr bool s1 = (M == SETUP_W || M == SWEEP_W);
    static constexpr int ngram = (M == SWEEP_W) ? 2 : 1;
};

// Per-workgroup record: ngram x (the Gram's 16 x 16 blocks on and above the
// diagonal, block rows in order and each block row from its diagonal block
// on, 256 entries each in row-major order; then RP column maxima), then
// <x, c> and the numerator and denominator of the beta* diagnostic. The
// Gram is symmetric: the blocks below the diagonal are the transposes of
// those above and are written by the finish kernels from them.
constexpr int kRecTail = 3;
__host__ __device__ constexpr int gram_blocks(int rp) { return (rp / 16) * (rp / 16 + 1) / 2; }
__host__ __device__ constexpr int rec_gram_len(int rp) { return gram_blocks(rp) * 256 + rp; }
template <int RP>
__host__ __device__ constexpr int rec_len(int ngram) { return ngram * rec_gram_len(RP) + kRecTail; }
// Index of block (b1, b2), b1 <= b2, among the stored blocks.
__host__ __device__ constexpr int gram_block_index(int nb, int b1, int b2)
{
    return b1 * nb - b1 * (b1 - 1) / 2 + (b2 - b1);
}

// Solver flags read on the device (the NMF_FLAG_* values of the C ABI).
constexpr int kFlagBetaStar = 4;

// One coordinate step on the four rows a lane holds. Every lane forms the
// change its own coordinate would take, d = max(t, -x); the change of lane Q
// of the 16-lane row is then taken into t, t -= gq * d(lane Q). The broadcast
// rides on the multiply-add as its DPP source (v_fmac_f64 with row_newbcast:Q
// on the negated src0), which the compiler does not form by itself: 8
// instructions per step instead of 12 with a separate v_mov_b64_dpp per row.
// Rounding is that of fma(-gq, d, t). Each DPP source is written three
// instructions before it is read, more than the two wait states a DPP read
// of a VALU result needs; no memory is touched.
template <int Q>
__device__ __forceinline__ void step4(double &t0, double &t1, double &t2, double &t3, double x0,
                                      double x1, double x2, double x3, double gq)
{
    double d0, d1, d2, d3;
    asm("v_max_f64 %0, %4, -%8\n\t"
        "v_max_f64 %1, %5, -%9\n\t"
        "v_max_f64 %2, %6, -%10\n\t"
        "v_max_f64 %3, %7, -%11\n\t"
        "v_fmac_f64_dpp %4, -%0, %12 row_newbcast:%13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %5, -%1, %12 row_newbcast:%13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %6, -%2, %12 row_newbcast:%13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %7, -%3, %12 row_newbcast:%13 row_mask:0xf bank_mask:0xf"
        : "=&v"(d0), "=&v"(d1), "=&v"(d2), "=&v"(d3), "+v"(t0), "+v"(t1), "+v"(t2), "+v"(t3)
        : "v"(x0), "v"(x1), "v"(x2), "v"(x3), "v"(gq), "i"(Q));
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

// ------------------------------------------------------ decision (a8 row)

// Error, accept/restart (Algorithm 2) and beta update (Algorithm 3), run by
// one thread after <W_n, A> (s1) and <W_n^T W_n, H_w H_w^T> (s2) are known.
__device__ inline void decide(DevState *st, double s1, double s2, double *trace,
                              uint8_t *accepted, double *beta_used)
{
    const int k = st->k + 1;
    double e2 = st->nx2 - 2.0 * s1 + s2;                     // Remark 1
    if (k < st->e2_scale_n) e2 *= st->e2_scale[k];
    const double e = err_of_sq(e2);
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

struct HalsArgs {
    int64_t rows;          // factor rows (m for W, n for H^T)
    int r, K;
    const double *lin;     // nsplit x (rows_pad x RP) partials of the linear term
    const float *lin32;    // the same in FP32 (16-bit X products), used when non-null
    int nsplit;
    int64_t split_stride;
    float *fac;            // factor slots, rows x RP each
    int64_t slot_stride;
    const double *gram;    // Gram buffers of the fixed factor
    int64_t gram_slot_stride;   // > 0: slot chosen by w_y (H update)
    double *part;          // per-workgroup records
    DevState *st;
    // Sweep modes. src_mode: where x starts: 0 the extrapolated slot, 1 the
    // new-iterate slot (filled by the exact NNLS solve, used with K = 0), 2 the
    // FP64 buffer x64 (adaptive inner loop, epilogue with K = 0). step: 0 a
    // whole half-iteration (K sweeps and the epilogue); 1 / 2 sweep `sweep`
    // (1, 2, ...) of the adaptive loop from the extrapolated slot / from x64,
    // result to x64 and its squared change to part_n (two halves of one
    // value per block, by the sweep's parity). Sweep l >= 2 first sums the
    // changes of sweep l - 1 (every workgroup the same way) and takes the
    // loop's decision: sweep 2 sets the reference change, a later sweep stops
    // the loop (and returns) once the change is at most delta times it; a
    // stopped loop's later sweeps return at once. The epilogue after the
    // loop records the number of sweeps run in sweeps[2 k + side].
    int src_mode;
    int step;
    int sweep;
    double delta;
    double *x64;
    double *part_n;
    int32_t *sweeps;
    // Exact solve: the inverse of the Gram matrix (RP x RP, then a 1 / 0 flag)
    // computed beforehand, or null for an inversion in every workgroup.
    double *ginv;
};

// Linear term of one coordinate: its K-chunk partials summed in FP64 in
// split order.
__device__ __forceinline__ double lin_sum(const HalsArgs &a, int64_t off)
{
    if (a.lin32) {
        const float *p = a.lin32 + off;
        double c = p[0];
        for (int sp = 1; sp < a.nsplit; ++sp) c += (double)p[sp * a.split_stride];
        return c;
    }
    const double *p = a.lin + off;
    double c = p[0];
    for (int sp = 1; sp < a.nsplit; ++sp) c += p[sp * a.split_stride];
    return c;
}

// SETUP_H / SETUP_W: Gram (and for W, <W0, A>) of slot 0.
// SWEEP_H (a3 + a4): H_n from H_y by K sweeps with C^T = X^T W_y and
//   G = W_y^T W_y; H_y' = H_n + beta (H_n - H) (projected for hp = 3); Gram of
//   H_w (H_n for hp = 1, else H_y').
// SWEEP_W (a6 + a7): W_n from W_y by K sweeps with A = X H_w^T and
//   G = H_w H_w^T; W_y' = W_n + beta (W_n - W); <W_n, A>, Gram(W_n),
//   Gram(W_y').
// BS: the W epilogue holds the beta* diagnostic (computed when its flag is
// set); the single-problem launches use the instance without it unless the
// flag was given, which spares that epilogue the diagnostic's registers.
template <int RP, int MODE, bool BS = true>
__device__ __forceinline__ void hals_body(const HalsArgs &a, int bid)
{
    using MI = ModeInfo<MODE>;
    constexpr int NB = RP / 16, NS = RP / 4, NG = MI::ngram;
    constexpr int LREC = rec_len<RP>(NG);
    static_assert(LREC <= sweep_record(RP), "record fits");
    constexpr int XLD = RP + 1;                       // padded LDS row (doubles)
    constexpr int BUF = (kWaves * 16 * XLD > kWaves * NB * 256) ? kWaves * 16 * XLD
                                                                : kWaves * NB * 256;
    __shared__ double s_tri[MI::sweeps ? NB : 1][16][16];
    __shared__ double s_gb[MI::sweeps ? NS : 1][MI::sweeps ? NB : 1][64];
    __shared__ double s_buf[BUF];
    __shared__ double s_cm[kWaves][NG * RP];
    __shared__ double s_s1[kWaves][kRecTail];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, g = lane >> 4;
    const int64_t row0 = (int64_t)bid * kRows + wave * 16;

    DevState *st = a.st;
    int src = 0, dst_n = 0, dst_y = 0, acc_slot = 0, hp = 3;
    double beta = 0.0;
    const double *G = a.gram;
    if constexpr (MI::sweeps) {
        if (st->done) return;
        hp = st->hp;
        beta = st->beta;
        if constexpr (MODE == SWEEP_H) {
            src = st->h_y; dst_n = st->h_n; dst_y = st->h_yn; acc_slot = st->h_acc;
            G += (int64_t)st->w_y * a.gram_slot_stride;
        } else {
            src = st->w_y; dst_n = st->w_n; dst_y = st->w_yn; acc_slot = st->w_acc;
        }
        if (a.src_mode == 1) src = dst_n;
        if (a.step == 1 && bid == 0 && tid == 0) {
            st->in_stop = 0;
            st->in_count = 1;
        }
        if (a.step == 2) {
            if (st->in_stop) return;
            const int nblk = (int)((a.rows + kRows - 1) / kRows);
            const double *pn = a.part_n + ((a.sweep - 2) & 1) * (int64_t)nblk;
            double v = 0.0;
            for (int i = tid; i < nblk; i += kThreads) v += pn[i];
            v = block_sum(v, &s_s1[0][0]);
            const double d = sqrt(v);                 // change of sweep sweep - 1
            if (a.sweep > 2 && d <= a.delta * st->in_eps0) {
                if (bid == 0 && tid == 0) st->in_stop = 1;
                return;
            }
            if (bid == 0 && tid == 0) {
                if (a.sweep == 2) st->in_eps0 = d;
                st->in_count = a.sweep;
            }
        }
        if (a.step == 0 && a.src_mode == 2 && bid == 0 && tid == 0)
            a.sweeps[2 * st->k + (MODE == SWEEP_W ? 1 : 0)] = st->in_count;
    }
    const float *xsrc = a.fac + src * a.slot_stride;
    const double *x64 = (MI::sweeps && a.src_mode == 2) ? a.x64 : nullptr;

    // x and c in D layout: rows 4v+g of the wave's tile, coordinate 16b+lr.
    // The loop over the K-chunk partials of c runs outside the unrolled tile
    // loops, so that all loads of one partial are in flight together (the
    // sum per entry is still p0 + p1 + ... in split order).
    // Rows past the factor's end read the last row (in bounds, every load
    // unconditional so that they are all in flight together) and count as 0.
    double xd[NB][4], cd[NB][4];
    bool okv[4];
    int64_t rowc[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + 4 * v + g;
        okv[v] = row < a.rows;
        rowc[v] = okv[v] ? row : a.rows - 1;
    }
    auto load_x = [&](auto ld) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const double x = ld(rowc[v] * RP + 16 * b + lr);
                xd[b][v] = okv[v] ? x : 0.0;
                cd[b][v] = 0.0;
            }
    };
    if (x64) load_x([&](int64_t off) { return x64[off]; });
    else load_x([&](int64_t off) { return (double)xsrc[off]; });
    if constexpr (MI::lin) {
        auto add_split = [&](auto load, int sp) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const double c = load(sp * a.split_stride + rowc[v] * RP + 16 * b + lr);
                    const double nv = (sp == 0) ? c : cd[b][v] + c;
                    cd[b][v] = okv[v] ? nv : 0.0;
                }
        };
        if (a.lin32) {
            auto ld = [&](int64_t off) { return (double)a.lin32[off]; };
            for (int sp = 0; sp < a.nsplit; ++sp) add_split(ld, sp);
        } else {
            auto ld = [&](int64_t off) { return a.lin[off]; };
            for (int sp = 0; sp < a.nsplit; ++sp) add_split(ld, sp);
        }
    }

    double xa[NS];             // x in A layout (sweep modes)
    if constexpr (MI::sweeps) {
        // B operands: -G(4s+g, 16b+lr); inverse diagonal of coordinate 16b+lr;
        // strictly lower in-block Gram entries scaled by the inverse diagonal
        // of their row, tri[b][q][l] = G(16b+l, 16b+q) / G(16b+l, 16b+l) for
        // l > q (0 otherwise, and 0 for a zero diagonal), for the in-block
        // corrections of the scaled numerators.
        // B operands in LDS (shared by the four waves, read right before each
        // MFMA): s_gb[s][b][lane] = -G(4s+g, 16b+lr).
        // (All global loads of the staging first, then the LDS stores.)
        constexpr int NGB = NS * NB * 64 / kThreads, NTR = NB * 256 / kThreads;
        static_assert(NGB * kThreads == NS * NB * 64 && NTR * kThreads == NB * 256, "staging split");
        double inv[NB], gtmp[NGB], ttmp[NTR];
#pragma unroll
        for (int i = 0; i < NGB; ++i) {
            const int e = tid + i * kThreads, sb = e >> 6, ln = e & 63;
            const int ss = sb / NB, bb = sb % NB;
            gtmp[i] = -G[(4 * ss + (ln >> 4)) * RP + 16 * bb + (ln & 15)];
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) inv[b] = G[RP * RP + 16 * b + lr];
#pragma unroll
        for (int i = 0; i < NTR; ++i) {
            const int e = tid + i * kThreads, b = e >> 8, q = (e >> 4) & 15, l = e & 15;
            ttmp[i] = (l > q) ? G[(16 * b + l) * RP + 16 * b + q] * G[RP * RP + 16 * b + l] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < NGB; ++i) {
            const int e = tid + i * kThreads, sb = e >> 6, ln = e & 63;
            s_gb[sb / NB][sb % NB][ln] = gtmp[i];
        }
#pragma unroll
        for (int i = 0; i < NTR; ++i) {
            const int e = tid + i * kThreads;
            s_tri[e >> 8][(e >> 4) & 15][e & 15] = ttmp[i];
        }
        // x in A layout: row lr, coordinate 4s+g.
        {
            const int64_t row = row0 + lr;
            const bool ok = row < a.rows;
            const int64_t rc = ok ? row : a.rows - 1;
            auto load_xa = [&](auto ld) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const double x = ld(rc * RP + 4 * s + g);
                    xa[s] = ok ? x : 0.0;
                }
            };
            if (x64) load_xa([&](int64_t off) { return x64[off]; });
            else load_xa([&](int64_t off) { return (double)xsrc[off]; });
        }
        __syncthreads();
        double *xs = s_buf + wave * 16 * XLD;

        // The numerators of the next block start before the current block is
        // updated: its MFMAs over the k-steps outside the current block are
        // independent of the update and overlap it; the four k-steps inside
        // follow once the block's new values are in A layout.
        double4v tcur = {cd[0][0], cd[0][1], cd[0][2], cd[0][3]};
#pragma unroll
        for (int s = 0; s < NS; ++s)
            tcur = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[s], s_gb[s][0][lane], tcur, 0, 0, 0);
        for (int it = 0; it < a.K; ++it) {
            static_for<NB>([&](auto B) {
                constexpr int b = decltype(B)::value;
                constexpr int nb = (b + 1) % NB;
                // t of the next block over the k-steps outside block b, in two
                // chains.
                double4v tn0 = {cd[nb][0], cd[nb][1], cd[nb][2], cd[nb][3]};
                double4v tn1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (s / 4 == b) continue;
                    const double bo = s_gb[s][nb][lane];
                    if (s & 1) tn1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[s], bo, tn1, 0, 0, 0);
                    else tn0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[s], bo, tn0, 0, 0, 0);
                }
                // The numerators scaled by the inverse diagonal, tau = t / G_kk
                // (the step of the closed form before projection).
                double t0 = tcur[0] * inv[b], t1 = tcur[1] * inv[b];
                double t2 = tcur[2] * inv[b], t3 = tcur[3] * inv[b];
                // The block's in-block Gram column entries, all read before
                // the first step: the empty asm takes them as in/out operands,
                // so the compiler can neither sink each read to its step (and
                // wait on it there) nor read them again.
                double gqv[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) gqv[q] = s_tri[b][q][lr];
                asm volatile(""
                             : "+v"(gqv[0]), "+v"(gqv[1]), "+v"(gqv[2]), "+v"(gqv[3]),
                               "+v"(gqv[4]), "+v"(gqv[5]), "+v"(gqv[6]), "+v"(gqv[7]),
                               "+v"(gqv[8]), "+v"(gqv[9]), "+v"(gqv[10]), "+v"(gqv[11]),
                               "+v"(gqv[12]), "+v"(gqv[13]), "+v"(gqv[14]), "+v"(gqv[15]));
                // Coordinates 16b .. 16b+15 in order. Every lane forms the
                // change its coordinate would take; lane q's is the one used
                // at step q, and the later coordinates correct their tau. Lanes
                // l <= q get a zero correction, so each tau stops at the value
                // its own step used. Coordinates at or beyond r (rank padding,
                // only ever in the last block) have x = 0, a zero inverse
                // diagonal and hence no change: their steps are skipped (a
                // uniform branch).
                static_for<16>([&](auto Q) {
                    constexpr int q = decltype(Q)::value;
                    if (b + 1 < NB || 16 * b + q < a.r) {
                        // The change max(x + tau, 0) - x, formed as
                        // max(tau, -x): equal up to rounding, shorter. The
                        // four independent rows of the lane go stage by
                        // stage, so that their latencies overlap.
                        step4<q>(t0, t1, t2, t3, xd[b][0], xd[b][1], xd[b][2], xd[b][3], gqv[q]);
                    }
                });
                xd[b][0] = fmax(xd[b][0] + t0, 0.0);
                xd[b][1] = fmax(xd[b][1] + t1, 0.0);
                xd[b][2] = fmax(xd[b][2] + t2, 0.0);
                xd[b][3] = fmax(xd[b][3] + t3, 0.0);
                // The block's new values into A layout (wave-private LDS tile;
                // the LDS operations of a wave complete in order).
#pragma unroll
                for (int v = 0; v < 4; ++v) xs[(4 * v + g) * XLD + 16 * b + lr] = xd[b][v];
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int s = 0; s < 4; ++s) xa[4 * b + s] = xs[lr * XLD + 16 * b + 4 * s + g];
                __builtin_amdgcn_wave_barrier();
                // The k-steps inside block b complete the next block's t.
                tn0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[4 * b], s_gb[4 * b][nb][lane], tn0, 0, 0, 0);
                tn1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[4 * b + 1], s_gb[4 * b + 1][nb][lane], tn1, 0, 0, 0);
                tn0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[4 * b + 2], s_gb[4 * b + 2][nb][lane], tn0, 0, 0, 0);
                tn1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[4 * b + 3], s_gb[4 * b + 3][nb][lane], tn1, 0, 0, 0);
                tcur = tn0 + tn1;
            });
        }
    }

    // One sweep of the adaptive loop: x to the FP64 buffer, and the
    // workgroup's squared change (each entry is read and written by the lane
    // that owns it).
    if constexpr (MI::sweeps) {
        if (a.step != 0) {
            double d2 = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = row0 + 4 * v + g;
                if (row < a.rows) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const int64_t off = row * RP + 16 * b + lr;
                        const double old = (a.step == 1) ? (double)xsrc[off] : a.x64[off];
                        const double dx = xd[b][v] - old;
                        d2 = fma(dx, dx, d2);
                        a.x64[off] = xd[b][v];
                    }
                }
            }
            d2 = block_sum(d2, &s_s1[0][0]);
            if (tid == 0)
                a.part_n[((a.sweep - 1) & 1) * ((a.rows + kRows - 1) / kRows) + bid] = d2;
            return;
        }
    }

    // Epilogue: stored FP32 rows, extrapolation, Gram operands, <x, c>.
    double gw[NG][NB][4];
    double dw[NB][4];          // W_n - W (beta* diagnostic)
    double s1 = 0.0;
    // The accepted rows first, all loads in flight together (the accepted
    // slot is never written by this kernel).
    float prv[NB][4];
    if constexpr (MI::sweeps) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int b = 0; b < NB; ++b)
                prv[b][v] = a.fac[acc_slot * a.slot_stride + rowc[v] * RP + 16 * b + lr];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + 4 * v + g;
        const bool ok = row < a.rows;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int64_t off = row * RP + 16 * b + lr;
            const float xn = (float)xd[b][v];
            if constexpr (MI::sweeps) {
                float yf = 0.0f;
                dw[b][v] = 0.0;
                if (ok) {
                    a.fac[dst_n * a.slot_stride + off] = xn;
                    const float prev = prv[b][v];
                    dw[b][v] = xd[b][v] - (double)prev;
                    double y = fma(beta, (double)xn - (double)prev, (double)xn);
                    if (MODE == SWEEP_H && hp == 3) y = fmax(y, 0.0);
                    yf = (float)y;
                    a.fac[dst_y * a.slot_stride + off] = yf;
                }
                if constexpr (MODE == SWEEP_H) {
                    gw[0][b][v] = ok ? (double)(hp == 1 ? xn : yf) : 0.0;
                } else {
                    gw[0][b][v] = ok ? (double)xn : 0.0;
                    gw[NG - 1][b][v] = ok ? (double)yf : 0.0;
                }
            } else {
                gw[0][b][v] = ok ? (double)xn : 0.0;
            }
            if constexpr (MI::s1) s1 = fma((double)xn, cd[b][v], s1);
        }
    }

    // beta* of section 4 (W side, when enabled): per row, the numerator
    // <c - x G, dW> and the denominator <dW G, dW>, from the final x (A
    // layout, xa) and dW (moved into A layout through the wave's LDS tile).
    double bs_num = 0.0, bs_den = 0.0;
    if constexpr (MODE == SWEEP_W && BS) {
        if (st->flags & kFlagBetaStar) {
            double *xs = s_buf + wave * 16 * XLD;
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) xs[(4 * v + g) * XLD + 16 * b + lr] = dw[b][v];
            __builtin_amdgcn_wave_barrier();
            double da[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) da[q] = xs[lr * XLD + 4 * q + g];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                double4v t = {cd[b][0], cd[b][1], cd[b][2], cd[b][3]};
                double4v u = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const double bo = s_gb[q][b][lane];          // -G(4q+g, 16b+lr)
                    t = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[q], bo, t, 0, 0, 0);
                    u = __builtin_amdgcn_mfma_f64_16x16x4f64(da[q], bo, u, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    bs_num = fma(t[v], dw[b][v], bs_num);
                    bs_den = fma(-u[v], dw[b][v], bs_den);
                }
            }
        }
    }

    double *rec = a.part + (size_t)bid * LREC;
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        // Column maxima of the tile: over v, then over the 4 lane groups.
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            double mx = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) mx = fmax(mx, fabs(gw[gi][b][v]));
            mx = fmax(mx, __shfl_xor(mx, 16));
            mx = fmax(mx, __shfl_xor(mx, 32));
            if (g == 0) s_cm[wave][gi * RP + 16 * b + lr] = mx;
        }
        // Partial Gram, one block row b1 at a time, the blocks b2 >= b1 only:
        // G(16b1 + i, 16b2 + j) = sum over the wave's 16 rows of
        // w(row, 16b1+i) w(row, 16b2+j).
        double *rg = rec + gi * rec_gram_len(RP);
        static_for<NB>([&](auto B1) {
            constexpr int b1 = decltype(B1)::value;
            constexpr int NC = NB - b1;      // blocks b1 .. NB-1 of the row
            double4v acc[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                acc[c] = double4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(gw[gi][b1][v], gw[gi][b1 + c][v],
                                                                  acc[c], 0, 0, 0);
            }
            __syncthreads();                 // s_buf free (sweep tiles, previous row)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) s_buf[((wave * NB + c) * 4 + v) * 64 + lane] = acc[c][v];
            __syncthreads();
            // Entry e of the row's stored blocks: block b1 + (e >> 8), rows
            // 4v + (ln >> 4), column ln & 15, i.e. offset e from the row's
            // first stored block.
            double *rb = rg + gram_block_index(NB, b1, b1) * 256;
            for (int e = tid; e < NC * 256; e += kThreads) {
                const int c = e >> 8, v = (e >> 6) & 3, ln = e & 63;
                double sum = 0.0;
#pragma unroll
                for (int w = 0; w < kWaves; ++w) sum += s_buf[((w * NB + c) * 4 + v) * 64 + ln];
                rb[e] = sum;
            }
        });
    }
    if constexpr (MI::s1) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            s1 += __shfl_xor(s1, off);
            bs_num += __shfl_xor(bs_num, off);
            bs_den += __shfl_xor(bs_den, off);
        }
        if (lane == 0) {
            s_s1[wave][0] = s1;
            s_s1[wave][1] = bs_num;
            s_s1[wave][2] = bs_den;
        }
    }
    __syncthreads();
    for (int e = tid; e < NG * RP; e += kThreads) {
        double mx = s_cm[0][e];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) mx = fmax(mx, s_cm[w][e]);
        const int gi = e / RP, k = e % RP;
        rec[gi * rec_gram_len(RP) + gram_blocks(RP) * 256 + k] = mx;
    }
    if (tid < kRecTail) {
        double v = 0.0;
        if (MI::s1) v = (s_s1[0][tid] + s_s1[1][tid]) + (s_s1[2][tid] + s_s1[3][tid]);
        rec[LREC - kRecTail + tid] = v;
    }
}

struct FinArgs {
    const double *part;    // nblk records
    int nblk, r;
    double *gram;          // destination Gram buffers
    int64_t gram_slot_stride;
    const double *GH;      // Gram of H_w (W sides: s2)
    double *scratch;       // the summed <x, c>, beta* numerator and denominator
    DevState *st;
    double *trace;
    uint8_t *accepted;
    double *beta_used;
    double *beta_star;
};

// Sums the per-workgroup records (64 outputs per workgroup, each output over
// 16 interleaved strides of records, the 16 partial sums combined in a fixed
// order) into the Gram buffers: Gram (an entry above the diagonal blocks
// also into its mirror below), inverse diagonal (0 beyond r or for a zero
// diagonal) and column maxima. On W sides a second launch of one workgroup
// then forms e(k) and decides. A single problem's finish uses 1024-thread
// workgroups (a wave per stride: short load chains for its 256 records at
// 16384 rows); the grouped finish of the batch engine walks many small work
// blocks over a fixed grid and uses 256-thread workgroups (four strides per
// wave), which keeps more workgroups, and more work blocks, in flight. Both
// form the same sums, and so does the decision step.
constexpr int kFinOut = 64;
constexpr int kFinThreads = 1024;
constexpr int kFinGroupThreads = 256;

// Destination of output e of the records: the Gram entry (and the inverse
// diagonal beside a diagonal entry), a column maximum, or one of the scalars
// <x, c> and the beta* numerator and denominator.
template <int RP, int MODE>
__device__ __forceinline__ void fin_store(const FinArgs &a, const int *slot, int e, double s)
{
    constexpr int NG = ModeInfo<MODE>::ngram, NB = RP / 16;
    constexpr int GL = rec_gram_len(RP), GB = gram_blocks(RP) * 256;
    if (e < NG * GL) {
        const int gi = e / GL, w = e % GL;
        double *Gd = a.gram + slot[gi] * a.gram_slot_stride;
        if (w < GB) {
            int u = w >> 8, b1 = 0;
            while (u >= NB - b1) u -= NB - b1++;
            const int b2 = b1 + u;
            const int k = 16 * b1 + ((w >> 4) & 15), l = 16 * b2 + (w & 15);
            Gd[k * RP + l] = s;
            if (b1 != b2) Gd[l * RP + k] = s;
            if (k == l) Gd[RP * RP + k] = (k < a.r && s > 0.0) ? 1.0 / s : 0.0;
        } else {
            Gd[RP * RP + RP + (w - GB)] = s;
        }
    } else if (ModeInfo<MODE>::s1) {
        a.scratch[e - NG * GL] = s;        // <x, c>, beta* numerator, denominator
    }
}

// After every output is stored and visible to the calling workgroup: s2,
// then e(k) and the decision (W sweep), or e(0) (W set-up).
template <int RP, int MODE, int NT>
__device__ __forceinline__ void fin_decide(const FinArgs &a, const int *slot, double *shd)
{
    if constexpr (ModeInfo<MODE>::s1) {
        DevState *st = a.st;
        const double *Gn = a.gram + slot[0] * a.gram_slot_stride;
        // s2 = <Gn, GH> in the order of kFinThreads virtual threads, whatever
        // the workgroup size NT: virtual thread t sums entries t, t + 1024,
        // ... in order; each virtual wave is reduced across its lanes; the
        // 16 wave sums are added in a fixed tree. Thread tid plays the
        // virtual threads tid + k NT, which sit in the same lane of virtual
        // waves tid / 64 + k NT / 64.
        constexpr int NV = kFinThreads / NT, VW = kFinThreads / 64;
        double part[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            part[k] = 0.0;
            for (int q = threadIdx.x + k * NT; q < RP * RP; q += kFinThreads)
                part[k] = fma(Gn[q], a.GH[q], part[k]);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) part[k] += __shfl_xor(part[k], off);
            if ((threadIdx.x & 63) == 0) shd[(threadIdx.x >> 6) + k * (NT / 64)] = part[k];
        }
        __syncthreads();
        double t[VW];
#pragma unroll
        for (int w = 0; w < VW; ++w) t[w] = shd[w];
#pragma unroll
        for (int h = VW / 2; h > 0; h /= 2)
#pragma unroll
            for (int w = 0; w < h; ++w) t[w] = t[w] + t[w + h];
        const double s2 = t[0];
        if (threadIdx.x == 0) {
            const double s1 = a.scratch[0];
            if constexpr (MODE == SWEEP_W) {
                if (st->flags & kFlagBetaStar) {
                    const double den = a.scratch[2];
                    a.beta_star[st->k] = den > 0.0 ? a.scratch[1] / den : 0.0;
                }
                decide(st, s1, s2, a.trace, a.accepted, a.beta_used);
            } else {
                // e(0) of Algorithm 2 through Remark 1.
                double e2 = st->nx2 - 2.0 * s1 + s2;
                if (st->e2_scale_n > 0) e2 *= st->e2_scale[0];
                const double e0 = err_of_sq(e2);
                a.trace[0] = e0 / sqrt(st->nx2);
                st->e0 = e0;
                st->e_prev = e0;
                st->e_acc = e0;
                if (!isfinite(e0) || st->max_iter == 0) st->done = 1;
            }
        }
    }
}

template <int RP, int MODE>
__device__ __forceinline__ void fin_slots(const DevState *st, int *slot)
{
    constexpr int NG = ModeInfo<MODE>::ngram;
    if constexpr (MODE == SWEEP_W) {
        slot[0] = st->w_n;
        slot[NG - 1] = st->w_yn;
    } else {
        slot[0] = 0;
    }
}

// The summing step (kFinOut outputs per work block) and, in the next launch
// (whose boundary makes the sums visible), the decision step of one work
// block per problem; neither has a cross-workgroup fence.
template <int RP, int MODE, int NT>
__device__ __forceinline__ void finish_sum_body(const FinArgs &a, int bid)
{
    constexpr int NG = ModeInfo<MODE>::ngram;
    constexpr int GL = rec_gram_len(RP);
    constexpr int LREC = rec_len<RP>(NG);
    // 16 record strides per output whatever the workgroup size: wave w of
    // NT / 64 takes strides w, w + NT / 64, ... (the sums are the same for
    // every NT).
    constexpr int kFinSplit = kFinThreads / kFinOut, NW = NT / 64;
    __shared__ double sh[kFinSplit][kFinOut];
    DevState *st = a.st;
    int slot[NG];
    if constexpr (ModeInfo<MODE>::sweeps) {
        if (st->done) return;        // set-up launches always run
    }
    fin_slots<RP, MODE>(st, slot);
    const int o = threadIdx.x & (kFinOut - 1), w = threadIdx.x / kFinOut;
    const int e = bid * kFinOut + o;
    const bool is_max = e < NG * GL && (e % GL) >= gram_blocks(RP) * 256;
    const double *src = a.part + e;
#pragma unroll
    for (int j = w; j < kFinSplit; j += NW) {
        double v = 0.0;
        if (e < LREC) {
#pragma unroll 16
            for (int b = j; b < a.nblk; b += kFinSplit) {
                const double x = src[(size_t)b * LREC];
                v = is_max ? fmax(v, x) : v + x;
            }
        }
        sh[j][o] = v;
    }
    __syncthreads();
    if (w == 0 && e < LREC) {
        double s = sh[0][o];
#pragma unroll
        for (int q = 1; q < kFinSplit; ++q) s = is_max ? fmax(s, sh[q][o]) : s + sh[q][o];
        fin_store<RP, MODE>(a, slot, e, s);
    }
}

template <int RP, int MODE, int NT>
__device__ __forceinline__ void finish_decide_body(const FinArgs &a)
{
    constexpr int NG = ModeInfo<MODE>::ngram;
    __shared__ double shd[kFinThreads / 64];
    DevState *st = a.st;
    int slot[NG];
    if constexpr (ModeInfo<MODE>::sweeps) {
        if (st->done) return;        // set-up launches always run
    }
    fin_slots<RP, MODE>(st, slot);
    fin_decide<RP, MODE, NT>(a, slot, shd);
}

template <int RP, int MODE, bool BS = true>
__global__ __launch_bounds__(kThreads, 1) void hals_kernel(HalsArgs a)
{
    hals_body<RP, MODE, BS>(a, blockIdx.x);
}

template <int RP, int MODE>
__global__ __launch_bounds__(kFinThreads) void finish_kernel(FinArgs a)
{
    finish_sum_body<RP, MODE, kFinThreads>(a, blockIdx.x);
}

// One workgroup: s2, then e(k) and the decision (W sweep) or e(0) (W set-up).
template <int RP, int MODE>
__global__ __launch_bounds__(kFinThreads) void decide_kernel(FinArgs a)
{
    finish_decide_body<RP, MODE, kFinThreads>(a);
}

// Grouped forms: one launch over several problems of the same padded rank
// (argument records and block ranges in g), each workgroup taking the work
// blocks blockIdx.x, blockIdx.x + gridDim.x, ... in turn; the barrier between
// two blocks keeps one block's LDS reads ahead of the next block's writes.
template <int RP, int MODE>
__global__ __launch_bounds__(kThreads, 1) void hals_group_kernel(Group g)
{
    const int total = group_total(g);
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        int lb, cnt;
        const int p = group_find(g, b, &lb, &cnt);
        hals_body<RP, MODE>(*reinterpret_cast<const HalsArgs *>(g.base + (size_t)p * g.stride), lb);
        __syncthreads();
    }
}

template <int RP, int MODE>
__global__ __launch_bounds__(kFinGroupThreads) void finish_group_kernel(Group g)
{
    const int total = group_total(g);
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        int lb, cnt;
        const int p = group_find(g, b, &lb, &cnt);
        finish_sum_body<RP, MODE, kFinGroupThreads>(
            *reinterpret_cast<const FinArgs *>(g.base + (size_t)p * g.stride), lb);
        __syncthreads();
    }
}

// One work block per problem.
template <int RP, int MODE>
__global__ __launch_bounds__(kFinGroupThreads) void decide_group_kernel(Group g)
{
    const int total = group_total(g);
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        int lb, cnt;
        const int p = group_find(g, b, &lb, &cnt);
        finish_decide_body<RP, MODE, kFinGroupThreads>(
            *reinterpret_cast<const FinArgs *>(g.base + (size_t)p * g.stride));
        __syncthreads();
    }
}

// Exact NNLS solve of every factor row (E-ANLS), defined in nnls_exact.h:
// warm start from the extrapolated slot, solution into the new-iterate slot;
// kExactRows factor rows per workgroup of kThreads.
constexpr int kExactRows = 32;
template <int RP, int MODE>
__global__ __launch_bounds__(kThreads, 2) void exact_kernel(HalsArgs a);
template <int RP, int MODE>
__global__ __launch_bounds__(kThreads, 2) void exact_group_kernel(Group g);
template <int RP, int MODE>
__global__ __launch_bounds__(kThreads) void invert_kernel(HalsArgs a);
inline int exact_blocks(int64_t rows) { return (int)((rows + kExactRows - 1) / kExactRows); }

// Argument records of one half-iteration (or set-up step) of one problem.
inline HalsArgs hals_args(int rp, int64_t rows, int r, int K, const Buffers &b, bool w_side)
{
    HalsArgs h{};
    h.rows = rows;
    h.r = r;
    h.K = K;
    h.fac = w_side ? b.Wf : b.Hf;
    h.slot_stride = rows * rp;
    if (b.lin_f32) h.lin32 = reinterpret_cast<const float *>(w_side ? b.A : b.Ct);
    if (w_side) {
        h.lin = b.A;
        h.nsplit = b.nsplit_a;
        h.split_stride = b.m_pad * rp;
        h.gram = b.GH;
        h.gram_slot_stride = 0;
    } else {
        h.lin = b.Ct;
        h.nsplit = b.nsplit_c;
        h.split_stride = b.n_pad * rp;
        h.gram = b.GW;
        h.gram_slot_stride = gram_stride(rp);
    }
    h.part = b.part_g;
    h.st = b.st;
    h.ginv = w_side ? b.ginv_w : b.ginv_h;
    return h;
}

inline FinArgs fin_args(int rp, int64_t rows, int r, const Buffers &b, bool w_side)
{
    FinArgs f{};
    f.part = b.part_g;
    f.nblk = (int)((rows + kRows - 1) / kRows);
    f.r = r;
    f.gram = w_side ? b.GW : b.GH;
    f.gram_slot_stride = w_side ? gram_stride(rp) : 0;
    f.GH = b.GH;
    f.scratch = b.part_d;
    f.st = b.st;
    f.trace = b.trace;
    f.accepted = b.accepted;
    f.beta_used = b.beta_used;
    f.beta_star = b.beta_star;
    return f;
}

// Blocks of the two kernels of a half-iteration.
inline int hals_blocks(int64_t rows) { return (int)((rows + kRows - 1) / kRows); }
inline int fin_blocks(int rp, int ngram) { return (int)((ngram * rec_gram_len(rp) + kRecTail + kFinOut - 1) / kFinOut); }

// Enqueues one half-iteration (or a set-up step) of one padded rank.
template <int RP>
struct Launch {
    // exact (sweep modes): the exact NNLS solve, then the sweep kernel with
    // no sweeps for the epilogue.
    template <int MODE>
    static void run(int64_t rows, int r, int K, const Buffers &b, bool w_side, hipStream_t s,
                    hipEvent_t mid = nullptr, bool exact = false)
    {
        HalsArgs h = hals_args(RP, rows, r, K, b, w_side);
        if constexpr (ModeInfo<MODE>::sweeps) {
            if (exact) {
                exact_kernel<RP, MODE><<<exact_blocks(rows), kThreads, 0, s>>>(h);
                h.K = 0;
                h.src_mode = 1;
            }
        }
        sweep_kernel<MODE>(rows, b, h, s);
        if (mid) (void)hipEventRecord(mid, s);
        finish<MODE>(rows, r, b, w_side, s);
    }
    // The sweep kernel, on W sides without the beta* code unless asked for.
    template <int MODE>
    static void sweep_kernel(int64_t rows, const Buffers &b, const HalsArgs &h, hipStream_t s)
    {
        if constexpr (MODE == SWEEP_W) {
            if (!b.beta_star_on) {
                hals_kernel<RP, MODE, false><<<hals_blocks(rows), kThreads, 0, s>>>(h);
                return;
            }
        }
        hals_kernel<RP, MODE><<<hals_blocks(rows), kThreads, 0, s>>>(h);
    }
    // The finish launch of a half-iteration, and the decision launch of the
    // W sides.
    template <int MODE>
    static void finish(int64_t rows, int r, const Buffers &b, bool w_side, hipStream_t s)
    {
        constexpr int NG = ModeInfo<MODE>::ngram;
        const FinArgs f = fin_args(RP, rows, r, b, w_side);
        finish_kernel<RP, MODE><<<fin_blocks(RP, NG), kFinThreads, 0, s>>>(f);
        if constexpr (ModeInfo<MODE>::s1) decide_kernel<RP, MODE><<<1, kFinThreads, 0, s>>>(f);
    }
    // Grouped half-iteration: the sweep kernel over group gh, then the
    // summing finish kernel over group gf (and, W side, the decision).
    // Grouped exact NNLS solves (the problems of the group that use them).
    static void exact_group(bool w_side, const Group &g, int blocks, hipStream_t s)
    {
        if (w_side) exact_group_kernel<RP, SWEEP_W><<<blocks, kThreads, 0, s>>>(g);
        else exact_group_kernel<RP, SWEEP_H><<<blocks, kThreads, 0, s>>>(g);
    }
    // The W side adds the decision launch over group gd.
    static void group(bool w_side, const Group &gh, int hblocks, const Group &gf, int fblocks,
                      const Group &gd, int dblocks, hipStream_t s)
    {
        if (w_side) {
            hals_group_kernel<RP, SWEEP_W><<<hblocks, kThreads, 0, s>>>(gh);
            finish_group_kernel<RP, SWEEP_W><<<fblocks, kFinGroupThreads, 0, s>>>(gf);
            decide_group_kernel<RP, SWEEP_W><<<dblocks, kFinGroupThreads, 0, s>>>(gd);
        } else {
            hals_group_kernel<RP, SWEEP_H><<<hblocks, kThreads, 0, s>>>(gh);
            finish_group_kernel<RP, SWEEP_H><<<fblocks, kFinGroupThreads, 0, s>>>(gf);
        }
    }
    // Half-iteration with the adaptive inner loop: `cap` single-sweep launches
    // (each takes the loop's decision on the previous sweep; launches after
    // the stop are no-ops), then the sweep kernel with no sweeps from the FP64
    // buffer for the epilogue, and the finish kernel.
    template <int MODE>
    static void adaptive(int64_t rows, int r, int cap, double delta, const Buffers &b, bool w_side,
                         hipStream_t s, hipEvent_t mid)
    {
        HalsArgs h = hals_args(RP, rows, r, 1, b, w_side);
        h.x64 = b.x64;
        h.part_n = b.part_n;
        h.sweeps = b.sweeps;
        h.delta = delta;
        for (int l = 1; l <= cap; ++l) {
            h.step = (l == 1) ? 1 : 2;
            h.sweep = l;
            h.src_mode = (l == 1) ? 0 : 2;
            sweep_kernel<MODE>(rows, b, h, s);
        }
        h.step = 0;
        h.K = 0;
        h.src_mode = 2;
        sweep_kernel<MODE>(rows, b, h, s);
        if (mid) (void)hipEventRecord(mid, s);
        finish<MODE>(rows, r, b, w_side, s);
    }
    static void sweep_h_adaptive(int64_t n, int r, int cap, double delta, const Buffers &b,
                                 hipStream_t s, hipEvent_t mid)
    {
        adaptive<SWEEP_H>(n, r, cap, delta, b, false, s, mid);
    }
    static void sweep_w_adaptive(int64_t m, int r, int cap, double delta, const Buffers &b,
                                 hipStream_t s, hipEvent_t mid)
    {
        adaptive<SWEEP_W>(m, r, cap, delta, b, true, s, mid);
    }
    static void invert(bool w_side, int r, const Buffers &b, hipStream_t s)
    {
        const HalsArgs h = hals_args(RP, 0, r, 0, b, w_side);
        if (w_side) invert_kernel<RP, SWEEP_W><<<1, kThreads, 0, s>>>(h);
        else invert_kernel<RP, SWEEP_H><<<1, kThreads, 0, s>>>(h);
    }
    static void sweep_h(int64_t n, int r, int K, bool exact, const Buffers &b, hipStream_t s,
                        hipEvent_t mid)
    {
        run<SWEEP_H>(n, r, K, b, false, s, mid, exact);
    }
    static void sweep_w(int64_t m, int r, int K, bool exact, const Buffers &b, hipStream_t s,
                        hipEvent_t mid)
    {
        run<SWEEP_W>(m, r, K, b, true, s, mid, exact);
    }
    static void setup_h(int64_t n, int r, const Buffers &b, hipStream_t s)
    {
        run<SETUP_H>(n, r, 0, b, false, s);
    }
    static void setup_err(int64_t m, int r, const Buffers &b, hipStream_t s)
    {
        run<SETUP_W>(m, r, 0, b, true, s);
    }
};

}  // namespace sweep
}  // namespace nmf
