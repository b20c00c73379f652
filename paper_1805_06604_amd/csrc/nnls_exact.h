// Exact NNLS blocks of E-ANLS (arXiv 1805.06604, section 1: ANLS solves each
// block subproblem of Algorithm 1 exactly, with the active-set method of Kim
// and Park; Algorithm 2 extrapolates around it).
//
// Each factor row is one problem min 1/2 x^T G x - c^T x over x >= 0, with G
// the Gram matrix of the fixed factor (shared by all rows) and c the row of
// the linear term. Block principal pivoting: the passive set starts at the
// support of the warm start (the extrapolated iterate); each step solves the
// unconstrained problem on the passive set and exchanges the coordinates that
// violate x_F >= 0 on it or y = G x - c >= 0 off it: all of them while the
// number of violations drops (or up to three times without progress), else
// only the largest index.
//
// Layout: a row's problem lives in one segment of a wave (16, 32 or 64 lanes;
// lane k = coordinate k), lane k holding row k of the passive-set system in
// registers. The system is solved by symmetric Gaussian elimination (LDL^T,
// no square root): pivot p needs column p in the trailing rows, which by
// symmetry is register p of every lane, exchanged through LDS (one write,
// broadcast reads). A pivot that is passive in no segment of the wave is
// skipped. Back substitution goes row by row with one broadcast per step.
// G sits in LDS, shared by the four waves of a workgroup.
//
// Nearly full passive sets take a shorter exact route. With z = G^-1 c (once
// per row) and N the q coordinates off the passive set, the solution with
// x_N = 0 is x = z - G^-1(:,N) l with (G^-1)_NN l = z_N, and the dual
// variables on N are y_N = -l (those on the passive set are zero): a q x q
// solve and a rank-q correction per step instead of the elimination. Each
// workgroup inverts G once in LDS (in-place Gauss-Jordan on the coordinates
// with a positive diagonal); a pivot that shrinks below 1e-10 of its diagonal
// sends every row to the elimination. A step takes this route when q <=
// kQFast in every segment of the wave.
//
// A coordinate with a zero Gram diagonal does not enter the objective and
// keeps max(0, warm start); a singular passive-set system (a pivot <= 0) or
// the step cap 10 r + 20 ends the solve with the last complete iterate,
// projected onto x >= 0.
#pragma once

#include "sweep_impl.h"

namespace nmf {
namespace sweep {

constexpr int kQFast = 8;

template <int RP>
struct ExactShape {
    static constexpr int SEG = RP <= 16 ? 16 : RP <= 32 ? 32 : 64;   // lanes per problem
    static constexpr int NSEG = 64 / SEG;                             // problems per wave
};

// G^-1 of the r x r Gram matrix in s_g (RP x RP, read after a barrier the
// caller has passed) into s_ginv, *s_ok = 0 where a pivot fails; every thread
// of the workgroup takes part and the result is visible to all on return.
template <int RP>
__device__ __forceinline__ void invert_gram(int r, const double *s_g, double *s_ginv, double *s_rowp,
                                            double *s_colp, int *s_ok)
{
    // G^-1 on the coordinates with a positive diagonal (zero elsewhere), by
    // in-place Gauss-Jordan: pivot p maps a = A(p,p) to 1/a, row p to A(p,j)/a,
    // column p to -A(i,p)/a and the rest to A(i,j) - A(i,p) A(p,j)/a.
    auto posc = [&](int i) { return i < r && s_g[i * RP + i] > 0.0; };
    for (int e = threadIdx.x; e < RP * RP; e += kThreads) {
        const int i = e / RP, j = e % RP;
        s_ginv[e] = (posc(i) && posc(j)) ? s_g[e] : 0.0;
    }
    if (threadIdx.x == 0) *s_ok = 1;
    __syncthreads();
    for (int p = 0; p < RP; ++p) {
        if (!posc(p)) continue;
        const double piv = s_ginv[p * RP + p];
        if (!(piv > 1e-10 * s_g[p * RP + p])) {
            if (threadIdx.x == 0) *s_ok = 0;
            break;
        }
        const double inv = 1.0 / piv;
        if (threadIdx.x < RP) {
            s_rowp[threadIdx.x] = s_ginv[p * RP + threadIdx.x];
            s_colp[threadIdx.x] = s_ginv[threadIdx.x * RP + p];
        }
        __syncthreads();
        // A fixed number of entries per thread, unrolled, so that the LDS
        // reads of a pivot step are all in flight together.
        static_assert(RP * RP % kThreads == 0, "whole entries per thread");
        double v[RP * RP / kThreads];
        // Every operand is read and the case is a select: no branch keeps
        // the reads of one entry from overlapping the others'. When the
        // threads of a workgroup span whole rows, a thread's column (and so
        // A(p,j)/a) is the same for all its entries.
        constexpr bool kFixedCol = kThreads % RP == 0;
        const double rjs0 = kFixedCol ? s_rowp[threadIdx.x % RP] * inv : 0.0;
#pragma unroll
        for (int u = 0; u < RP * RP / kThreads; ++u) {
            const int e = u * kThreads + threadIdx.x, i = e / RP, j = e % RP;
            const double rjs = kFixedCol ? rjs0 : s_rowp[j] * inv;
            const double ci = s_colp[i], aij = s_ginv[e];
            double w = fma(-ci, rjs, aij);
            w = (j == p) ? -ci * inv : w;
            w = (i == p) ? rjs : w;
            v[u] = (i == p && j == p) ? inv : w;
        }
#pragma unroll
        for (int u = 0; u < RP * RP / kThreads; ++u) s_ginv[u * kThreads + threadIdx.x] = v[u];
        __syncthreads();
    }
    __syncthreads();
}

template <int RP, int MODE>
__device__ __forceinline__ void exact_body(const HalsArgs &a, int bid)
{
    constexpr int SEG = ExactShape<RP>::SEG, NSEG = ExactShape<RP>::NSEG;
    constexpr int PASSES = kExactRows / (kWaves * NSEG);
    static_assert(PASSES * kWaves * NSEG == kExactRows, "rows per workgroup");
    __shared__ double s_g[RP * RP];
    __shared__ double s_col[kWaves][64];
    __shared__ double s_b[kWaves][64];
    __shared__ double s_x[kWaves][64];
    __shared__ double s_d[kWaves][64];
    __shared__ double s_ginv[RP * RP];
    __shared__ double s_z[kWaves][64];
    __shared__ double s_rowp[RP], s_colp[RP];
    __shared__ int s_ginv_ok;

    DevState *st = a.st;
    if (st->done) return;
    int src, dst;
    const double *G = a.gram;
    if constexpr (MODE == SWEEP_H) {
        src = st->h_y; dst = st->h_n;
        G += (int64_t)st->w_y * a.gram_slot_stride;
    } else {
        src = st->w_y; dst = st->w_n;
    }
    for (int e = threadIdx.x; e < RP * RP; e += kThreads) s_g[e] = G[e];
    __syncthreads();

    if (a.ginv) {
        // Taken beforehand, once for all workgroups (invert_kernel).
        for (int e = threadIdx.x; e < RP * RP; e += kThreads) s_ginv[e] = a.ginv[e];
        if (threadIdx.x == 0) s_ginv_ok = a.ginv[RP * RP] != 0.0;
        __syncthreads();
    } else {
        invert_gram<RP>(a.r, s_g, s_ginv, s_rowp, s_colp, &s_ginv_ok);
    }
    const bool ginv_ok = s_ginv_ok != 0;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int seg = lane / SEG, k = lane % SEG, sb = seg * SEG;
    const int kk = k < RP ? k : RP - 1;          // LDS column of idle lanes (RP = 48)
    const uint64_t segmask = SEG == 64 ? ~0ull : ((1ull << SEG) - 1);
    const int cap = 10 * a.r + 20;
    const float *xsrc = a.fac + src * a.slot_stride;
    float *xdst = a.fac + dst * a.slot_stride;
    double *col = s_col[wave], *bb = s_b[wave], *xs = s_x[wave], *sd = s_d[wave];
    double *zs = s_z[wave];

    for (int pass = 0; pass < PASSES; ++pass) {
        const int64_t row = (int64_t)bid * kExactRows + (pass * kWaves + wave) * NSEG + seg;
        const bool valid = row < a.rows && k < RP;
        double c = 0.0, w = 0.0;
        if (valid) {
            c = lin_sum(a, row * RP + k);
            w = (double)xsrc[row * RP + k];
        }
        const bool pos = valid && k < a.r && s_g[kk * RP + kk] > 0.0;
        const uint64_t pm = (__ballot(pos) >> sb) & segmask;    // coordinates that enter
        // z = G^-1 c (fast route).
        if (ginv_ok) {
            xs[lane] = c;
            __builtin_amdgcn_wave_barrier();
            double z = 0.0;
            static_for<RP>([&](auto J) {
                constexpr int j = decltype(J)::value;
                z = fma(s_ginv[j * RP + kk], xs[sb + j], z);
            });
            __builtin_amdgcn_wave_barrier();
            zs[lane] = z;
            __builtin_amdgcn_wave_barrier();
        }
        const double x0 = fmax(w, 0.0);
        double x = x0;                           // last complete iterate
        bool F = pos && w > 0.0;                 // passive set
        bool done = !(row < a.rows);             // uniform over the segment
        int alpha = 3, best = RP + 1;
        for (int it = 0; it < cap; ++it) {
            if (__ballot(!done) == 0) break;
            // The lane's coordinate, opaque to the compiler, so that the
            // comparisons with the pivot below are formed where they are used
            // rather than kept live for every pivot across the whole loop.
            int kl = k;
            asm volatile("" : "+v"(kl));
            const uint64_t fw = __ballot(F);
            const uint64_t fm = (fw >> sb) & segmask;        // this segment's set
            uint64_t fu = 0;                                 // union over segments
#pragma unroll
            for (int q = 0; q < NSEG; ++q) fu |= (fw >> (q * SEG)) & segmask;

            const uint64_t nm = pm & ~fm;                  // off the passive set
            const int q = __popcll(nm);
            const bool fast = ginv_ok && __ballot(!done && q > kQFast) == 0;
            double xn, y = 0.0;
            bool fail = false;
            if (fast) {
                // The q <= kQFast coordinates of N in order, (G^-1)_NN and z_N
                // (the same in every lane of the segment).
                int ni[kQFast];
                uint64_t t = nm;
#pragma unroll
                for (int u = 0; u < kQFast; ++u) {
                    ni[u] = t ? __builtin_ctzll(t) : 0;
                    t &= t - 1;
                }
                double S[kQFast][kQFast], lz[kQFast];
#pragma unroll
                for (int u = 0; u < kQFast; ++u) {
                    lz[u] = u < q ? zs[sb + ni[u]] : 0.0;
#pragma unroll
                    for (int v = 0; v < kQFast; ++v)
                        S[u][v] = (u < q && v < q) ? s_ginv[ni[u] * RP + ni[v]] : (u == v ? 1.0 : 0.0);
                }
                // (G^-1)_NN l = z_N by symmetric elimination and back substitution
                // (the pivots' reciprocals kept for the latter).
                double rpiv[kQFast];
#pragma unroll
                for (int pp = 0; pp < kQFast; ++pp) {
                    if (pp < q && !(S[pp][pp] > 0.0)) fail = true;
                    const double inv = 1.0 / S[pp][pp];
                    rpiv[pp] = inv;
#pragma unroll
                    for (int i = pp + 1; i < kQFast; ++i) {
                        const double f = S[i][pp] * inv;
#pragma unroll
                        for (int j = pp + 1; j < kQFast; ++j) S[i][j] = fma(-f, S[pp][j], S[i][j]);
                        lz[i] = fma(-f, lz[pp], lz[i]);
                    }
                }
#pragma unroll
                for (int pp = kQFast - 1; pp >= 0; --pp) {
                    double v = lz[pp];
#pragma unroll
                    for (int j = pp + 1; j < kQFast; ++j) v = fma(-S[pp][j], lz[j], v);
                    lz[pp] = v * rpiv[pp];
                }
                // x = z - G^-1(:,N) l on the passive set; y_N = -l.
                double xf = zs[lane];
                int myidx = 0;
#pragma unroll
                for (int u = 0; u < kQFast; ++u) {
                    if (u < q) xf = fma(-s_ginv[ni[u] * RP + kk], lz[u], xf);
                    if (u < q && ni[u] == k) myidx = u;
                }
                xn = pos ? (F ? xf : 0.0) : x0;
#pragma unroll
                for (int u = 0; u < kQFast; ++u)
                    if (u == myidx) y = -lz[u];
            } else {
                // Row k of the system: G restricted to the passive set (rows and
                // columns off it are zero; their pivots are skipped and their
                // solution is 0).
                double M[RP];
                static_for<RP>([&](auto J) {
                    constexpr int j = decltype(J)::value;
                    const double gj = s_g[j * RP + kk];
                    M[j] = (F && ((fm >> j) & 1)) ? gj : 0.0;
                });
                double b = F ? c : 0.0;

                // Elimination: rows k > p lose f_k times row p, f_k = S(k,p) / S(p,p);
                // row p of the trailing matrix is column p by symmetry.
                static_for<RP>([&](auto P) {
                    constexpr int p = decltype(P)::value;
                    if ((fu >> p) & 1) {
                        col[lane] = M[p];
                        bb[lane] = b;
                        __builtin_amdgcn_wave_barrier();
                        const double d = col[sb + p], bp = bb[sb + p];
                        const bool pp = (fm >> p) & 1;
                        const bool ok = d > 0.0;
                        if (pp && !ok) fail = true;
                        const double f = (pp && ok && kl > p) ? M[p] / d : 0.0;
                        sd[sb + p] = d;
                        static_for<RP - p - 1>([&](auto J) {
                            constexpr int j = p + 1 + decltype(J)::value;
                            M[j] = fma(-f, col[sb + j], M[j]);
                        });
                        b = fma(-f, bp, b);
                        __builtin_amdgcn_wave_barrier();
                    }
                });

                // Back substitution: x_p = (b_p - sum_{j > p} S(p,j) x_j) / S(p,p),
                // the sum accumulated in lane p as the later x_j become known; a
                // lane's value is final once its own step is done.
                const double rdk = F ? 1.0 / sd[sb + kk] : 1.0;
                double acc = 0.0;
                static_for<RP>([&](auto P) {
                    constexpr int p = RP - 1 - decltype(P)::value;
                    if ((fu >> p) & 1) {
                        xs[lane] = (b - acc) * rdk;
                        __builtin_amdgcn_wave_barrier();
                        const double xp = xs[sb + p];
                        acc = fma(kl < p ? M[p] : 0.0, xp, acc);
                        __builtin_amdgcn_wave_barrier();
                    }
                });
                const double sol = (b - acc) * rdk;
                xn = pos ? (F ? sol : 0.0) : x0;

                // Dual variables y = G x - c and the infeasible coordinates.
                xs[lane] = xn;
                __builtin_amdgcn_wave_barrier();
                y = -c;
                static_for<RP>([&](auto J) {
                    constexpr int j = decltype(J)::value;
                    y = fma(s_g[j * RP + kk], xs[sb + j], y);
                });
                __builtin_amdgcn_wave_barrier();
            }
            const bool viol = pos && (F ? xn < 0.0 : y < 0.0);
            const uint64_t vm = (__ballot(viol) >> sb) & segmask;
            const int nv = __popcll(vm);
            if (!done) {
                if (fail) {
                    done = true;
                } else {
                    x = xn;
                    if (nv == 0) {
                        done = true;
                    } else if (nv < best || alpha > 0) {
                        if (nv < best) {
                            best = nv;
                            alpha = 3;
                        } else {
                            --alpha;
                        }
                        if (viol) F = !F;
                    } else if (k == 63 - __clzll(vm)) {
                        F = !F;
                    }
                }
            }
        }
        if (valid) xdst[row * RP + k] = (float)fmax(x, 0.0);
    }
}

template <int RP, int MODE>
__global__ __launch_bounds__(kThreads, 2) void exact_kernel(HalsArgs a)
{
    exact_body<RP, MODE>(a, blockIdx.x);
}

// The inverse for all workgroups of one exact solve, taken once (one
// workgroup) while the product that precedes the solve runs: RP x RP entries
// of G^-1, then 1.0 where every pivot held, 0.0 where one failed.
template <int RP, int MODE>
__global__ __launch_bounds__(kThreads) void invert_kernel(HalsArgs a)
{
    __shared__ double s_g[RP * RP];
    __shared__ double s_ginv[RP * RP];
    __shared__ double s_rowp[RP], s_colp[RP];
    __shared__ int s_ok;
    const DevState *st = a.st;
    if (st->done) return;
    const double *G = a.gram;
    if constexpr (MODE == SWEEP_H) G += (int64_t)st->w_y * a.gram_slot_stride;
    for (int e = threadIdx.x; e < RP * RP; e += kThreads) s_g[e] = G[e];
    __syncthreads();
    invert_gram<RP>(a.r, s_g, s_ginv, s_rowp, s_colp, &s_ok);
    for (int e = threadIdx.x; e < RP * RP; e += kThreads) a.ginv[e] = s_ginv[e];
    if (threadIdx.x == 0) a.ginv[RP * RP] = s_ok ? 1.0 : 0.0;
}

// Grouped form: one launch over the problems of a group that solve their
// blocks exactly (argument records and block ranges in g; the others have no
// blocks).
template <int RP, int MODE>
__global__ __launch_bounds__(kThreads, 2) void exact_group_kernel(Group g)
{
    const int total = group_total(g);
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        int lb, cnt;
        const int p = group_find(g, b, &lb, &cnt);
        exact_body<RP, MODE>(*reinterpret_cast<const HalsArgs *>(g.base + (size_t)p * g.stride), lb);
        __syncthreads();
    }
}

}  // namespace sweep
}  // namespace nmf
