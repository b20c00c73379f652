// Internal declarations shared by the kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

namespace nmf {

// f(integral_constant<int, 0>) .. f(integral_constant<int, N - 1>) in order,
// for loops whose index must be a compile-time constant (register arrays).
template <typename F, int... I>
__device__ __forceinline__ void static_for_(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_(f, std::make_integer_sequence<int, N>{});
}

// Three buffers per factor: the accepted iterate, the NNLS output and the
// extrapolated point. Which buffer plays which role lives in DevState, so an
// accept or a restart (Algorithm 2) is an index flip taken on the device.
constexpr int kSlots = 3;
// Rows of one workgroup of the 16-bit product: the row padding of X and X^T
// (and of the factors) when that product is used; 128 otherwise.
constexpr int kX16Rows = 256;

// Factor rows handled by one workgroup of the sweep kernels (16 per wave).
constexpr int kRowsPerBlock = 64;

// Per-workgroup record of the sweep kernels: up to two partial Gram matrices
// (their 16 x 16 blocks on and above the diagonal) with their column maxima,
// and three FP64 partial sums (<W, A>, and the numerator and denominator of
// the beta* diagnostic).
__host__ __device__ constexpr int64_t sweep_record(int rp)
{
    return 2 * ((rp / 16) * (rp / 16 + 1) / 2 * 256 + rp) + 3;
}

// Slot selectors for the product kernels.
enum FactorSel : int32_t {
    SEL_W_Y = 0,     // W_y: warm start of the coming W update, input of X^T W_y
    SEL_H_W = 1,     // H used by the W update: H_n (hp = 1) or H_y (hp >= 2)
    SEL_SLOT0 = 2,   // slot 0, unconditionally (set-up of e(0))
};

// Solver state kept in device memory and updated only by the decision step.
struct DevState {
    int32_t k;              // completed outer iterations
    int32_t done;           // 1: iterations are no-ops (max_iter or tol reached)
    int32_t bad_input;      // set by the packing kernels
    int32_t hp;
    int32_t w_acc, w_y, w_n, w_yn;   // W slots: accepted, warm start, new, new extrapolated
    int32_t h_acc, h_y, h_n, h_yn;   // H slots, same roles
    int32_t max_iter, flags, r, pad0;
    double beta, betabar, beta_prev, beta_acc;
    double e_prev, e_acc, nx2, tol;
    double gamma, gamma_bar, eta, e0;
    // Adaptive inner loop of the half-iteration in progress: ||x^(1) - x^(0)||_F,
    // stop flag and sweeps run so far.
    double in_eps0;
    int32_t in_stop, in_count;
    // Test hook of the restart branch: e(k)^2 is multiplied by e2_scale[k]
    // (device array) for k < e2_scale_n before the test of Algorithm 2; k = 0
    // is e(0). Null and 0 when unused.
    const double *e2_scale;
    int32_t e2_scale_n, pad1;
};

// e from e^2: the combination of Remark 1 can round slightly below zero,
// which is clamped to 0; a non-finite e^2 stays non-finite (NaN stays NaN,
// an infinite one gives +inf), so that Algorithm 2 restarts on it instead of
// accepting an error of 0.
__device__ inline double err_of_sq(double e2)
{
    if (!isfinite(e2)) return fabs(e2);
    return sqrt(e2 > 0.0 ? e2 : 0.0);
}

// Gram buffers (FP64) hold RP*RP entries, then RP inverse diagonal entries
// (0 where the coordinate is skipped: beyond r, or a zero diagonal), then the
// RP column maxima max |F(:,k)| of the factor (scales of the exact-integer
// products).
__host__ __device__ constexpr int gram_stride(int rp) { return rp * rp + 2 * rp; }

// Slots written by the coming iteration, given the accepted and warm-start
// slots: the NNLS output goes to a slot that is neither, and the new
// extrapolated point overwrites the warm start (each row is read before it is
// written, by the same thread) unless the warm start is the accepted iterate.
__host__ __device__ inline void plan_slots(int acc, int y, int32_t *n, int32_t *yn)
{
    if (acc == y) {
        *n = (acc + 1) % kSlots;
        *yn = (acc + 2) % kSlots;
    } else {
        *n = kSlots - acc - y;
        *yn = y;
    }
}

// A sparse operand (X, or X^T built from it) in CSR form on the device, with
// the work split of its product: rows cut into items of at most a fixed
// number of nonzeros. An item of a row that has a single item writes the
// result row; the items of a longer row write partial rows into `partial`
// (slots item_slot), which a second kernel sums in slot order.
struct CsrPlan {
    int64_t rows = 0;
    const int64_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
    const float *val = nullptr;
    int64_t nitems = 0;
    const int32_t *item_row = nullptr;
    const int64_t *item_beg = nullptr;
    const int64_t *item_end = nullptr;
    const int32_t *item_slot = nullptr;   // -1: the item is its row
    int64_t nlong = 0;
    const int32_t *long_row = nullptr;
    const int32_t *long_first = nullptr;
    const int32_t *long_count = nullptr;
    double *partial = nullptr;            // slots x RP
};

// Nonzeros per item of a sparse product at padded rank rp: 32 steps of the
// wave, which takes 64 / (rp / 4) nonzeros per step.
__host__ __device__ constexpr int64_t csr_item_nnz(int rp) { return 32 * (64 / (rp / 4)); }

// One X-streaming product Y = Z F (see the product kernels). Z is X or the
// resident X^T with rows padded to a multiple of 128 and rows of length ld (a
// multiple of 64), zero-filled; Y holds nsplit partial sums over K-chunks.
struct ProdArgs {
    const void *Z;          // rows_pad x ld, storage dtype
    int64_t ld;             // row length of Z
    int64_t K;              // contraction length (rows of F)
    int64_t rows;           // true rows of Z
    int64_t rows_pad;       // multiple of 128
    const float *F_base;    // factor slots, K x RP each
    int64_t slot_stride;
    int sel;                // FactorSel
    const DevState *st;
    double *Y;              // nsplit x rows_pad x RP partial sums (FP64; FP32 for the
                            // 16-bit X product, whose sums within a K-chunk are FP32)
    int64_t kchunk;         // K per split, multiple of 64
    int nsplit;
    // Exact-integer kernel only: per-row scale exponents of Z, and the Gram
    // buffers whose tail holds the column maxima of each factor slot.
    const int *zexp;
    const double *gram_base;
    int64_t gram_slot_stride;
    signed char *Fsl;       // the factor in int8 slices: (ld / 64) x 4 x RP x 64, or
                            // (16-bit X) in two parts of X's type: (ld / 64) x 2 x 2 x RP x 64 B
    int *texp;              // its column scale exponents (RP)
    // Sparse kernel only: the CSR operand (host pointer to its plan).
    const CsrPlan *csr;
};

// Product kernels: VALU FP64 FMA over the stored values (products exact, sums
// in FP64); the exact-integer matrix-core product (X and the factor in int8
// slices, int32 sums); the sparse product; and the 16-bit X product on the
// 16-bit matrix cores (X in fragment order, the factor split into two 16-bit
// parts once per product, FP32 sums within a K-chunk).
enum ProdKernel { PK_VALU = 0, PK_MFMA_I8 = 3, PK_CSR = 4, PK_MFMA_X16 = 5 };

// Device buffers of one context. Factors are FP32, row-major with RP columns
// (r rounded up to a multiple of 16; the padding stays zero):
//   W slots: m x RP each, H slots hold H^T: n x RP each.
// Everything that enters the HALS numerator c_k - G(k,:) x (linear terms,
// Grams) is FP64.
struct Buffers {
    float *Wf = nullptr;     // kSlots * m * RP
    float *Hf = nullptr;     // kSlots * n * RP
    double *GW = nullptr;    // kSlots * gram_stride: Gram of each W slot
    double *GH = nullptr;    // gram_stride: Gram of H_w
    double *A = nullptr;     // nsplit_a x m_pad x RP : partials of X H_w^T
    double *Ct = nullptr;    // nsplit_c x n_pad x RP : partials of X^T W_y
    int nsplit_a = 1, nsplit_c = 1;
    bool lin_f32 = false;    // A and Ct hold FP32 partials (the 16-bit X product)
    bool beta_star_on = false; // the W sweeps form the beta* diagnostic (its flag set)
    int64_t m_pad = 0, n_pad = 0;
    double *part_g = nullptr;// per-workgroup records of the sweep kernels
    double *part_d = nullptr;// FP64 scratch: reduction partials, the summed <W, A>
    DevState *st = nullptr;
    double *trace = nullptr; // max_iter + 1
    uint8_t *accepted = nullptr;
    double *beta_used = nullptr;
    double *beta_star = nullptr; // max_iter + 1: the beta* diagnostic (when enabled)
    float *stage = nullptr;  // staging of W0 / H0 / outputs: (m + n) * r
    signed char *fsl = nullptr; // exact-integer / 16-bit products: the sliced or split factor (shared)
    int *texp = nullptr;     // and its column exponents
    // Adaptive inner loop: the factor being updated in FP64 between its
    // sweeps (max(m, n) x RP), the per-workgroup squared changes of a sweep,
    // and the sweeps run per iteration (H, W).
    double *x64 = nullptr;
    // E-ANLS: the inverses of G_W (H solve) and G_H (W solve), RP x RP and a
    // 1 / 0 flag each, computed once per side beside the preceding product.
    double *ginv_h = nullptr, *ginv_w = nullptr;
    double *part_n = nullptr;
    int32_t *sweeps = nullptr;
};

// A grouped launch runs one kernel over several problems at once: problem p
// owns the work blocks prefix[p] .. prefix[p + 1] - 1 and reads its argument
// record at base + p * stride. The tables and the problem count *np live in
// device memory, so that a launch (and a graph of launches) stays valid while
// the host rewrites them between batch iterations; a fixed grid walks the
// prefix[*np] work blocks with a grid stride.
struct Group {
    const char *base = nullptr;
    int stride = 0;
    const int *prefix = nullptr;
    const int *np = nullptr;
};

// Work blocks of a grouped launch.
__device__ inline int group_total(const Group &g) { return g.prefix[*g.np]; }

// Problem of work block b of a grouped launch, and the block's index within it.
__device__ inline int group_find(const Group &g, int b, int *local, int *count)
{
    int lo = 0, hi = *g.np;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (g.prefix[mid] <= b) lo = mid;
        else hi = mid;
    }
    *local = b - g.prefix[lo];
    *count = g.prefix[lo + 1] - g.prefix[lo];
    return lo;
}

// ------------------------------------------------------------ launchers
// All return hipGetLastError() after enqueueing on `s`. A non-null `mid` is
// recorded on `s` between the two kernels of the step (after the factor
// slicing of a product, after the sweep kernel of a half-iteration).
hipError_t launch_product(int rp, int xdtype, int kernel, const ProdArgs &a, hipStream_t s,
                          hipEvent_t mid = nullptr);

// A half-iteration: the factor update (inner_k HALS sweeps, or with `exact`
// the exact NNLS solve of every row), its epilogue and its finish step.
hipError_t launch_sweep_h(int rp, int64_t n, int r, int inner_k, bool exact, const Buffers &b,
                          hipStream_t s, hipEvent_t mid = nullptr);
hipError_t launch_sweep_w(int rp, int64_t m, int r, int inner_k, bool exact, const Buffers &b,
                          hipStream_t s, hipEvent_t mid = nullptr);
// The same with the adaptive inner loop: up to `cap` single sweeps, stopping
// once a sweep changes the factor by at most delta times the first one.
hipError_t launch_sweep_h_adaptive(int rp, int64_t n, int r, int cap, double delta,
                                   const Buffers &b, hipStream_t s, hipEvent_t mid = nullptr);
hipError_t launch_sweep_w_adaptive(int rp, int64_t m, int r, int cap, double delta,
                                   const Buffers &b, hipStream_t s, hipEvent_t mid = nullptr);

// Set-up of e(0): Gram of H0 (slot 0) into GH, then Gram of W0 (slot 0) into
// GW[0] together with <W0, A>, and the initial error into the state.
hipError_t launch_setup_gram_h(int rp, int64_t n, int r, const Buffers &b, hipStream_t s);
hipError_t launch_setup_error(int rp, int64_t m, int r, const Buffers &b, hipStream_t s);

// Packing: W0 (m x r) -> W slot 0 (m x RP); H0 (r x n) -> H slot 0 (n x RP),
// flagging negative or non-finite entries in st->bad_input.
hipError_t launch_pack(int rp, int64_t m, int64_t n, int r, const float *W0,
                       const float *H0, const Buffers &b, hipStream_t s);
// Unpacking of the accepted slots into W (m x r) and H (r x n).
hipError_t launch_unpack(int rp, int64_t m, int64_t n, int r, const Buffers &b,
                         float *W, float *H, hipStream_t s);

// Exact-integer path: slices the rows of a typed row-major matrix (rows x cols,
// rows of length ld_src) into int8 slices with rows of ld_dst entries.
namespace i8 {
hipError_t slice_rows(const void *src, int xdtype, int64_t rows, int64_t cols, int64_t ld_src,
                      int64_t ld_dst, void *dst, int *zexp, hipStream_t s);
}

// 16-bit path: copies a row-major 16-bit matrix (rows_pad x ld, ld a multiple
// of 64) into the fragment order of the 16-bit product (same size).
namespace x16 {
hipError_t to_fragments(const void *src, int64_t rows_pad, int64_t ld, void *dst, hipStream_t s);
}

// X conversion at create: source FP32 (m x n) -> X (rows of length ldx) and
// X^T (rows of length ldxt) in the storage type; padding must be zero already.
hipError_t launch_convert_x(const float *src, int64_t m, int64_t n, int xdtype,
                            void *X, int64_t ldx, void *Xt, int64_t ldxt, hipStream_t s);
// ||X||^2 in FP64 (deterministic two-pass reduction) of FP32 values, or of
// values stored as xdtype.
hipError_t launch_sumsq(const float *src, int64_t count, double *part, int nblk,
                        double *out, hipStream_t s);
hipError_t launch_sumsq_typed(const void *v, int xdtype, int64_t count, double *part,
                              int nblk, double *out, hipStream_t s);

// Grouped launches (one launch per kernel over several problems of one
// padded rank): the exact-integer product (factor slicing, then product) and
// a half-iteration of sweeps (sweep kernel, then finish kernel).
namespace i8 {
hipError_t launch_group(int rp, const Group &gs, int sblocks, const Group &gp, int pblocks,
                        hipStream_t s);
}
hipError_t launch_group_exact(int rp, bool w_side, const Group &g, int blocks, hipStream_t s);
// E-ANLS: the inverse of the Gram matrix the H (w_side false) or W solve uses,
// into b.ginv_h / b.ginv_w (one workgroup).
hipError_t launch_invert(int rp, bool w_side, int r, const Buffers &b, hipStream_t s);
hipError_t launch_group_sweep(int rp, bool w_side, const Group &gh, int hblocks, const Group &gf,
                              int fblocks, const Group &gd, int dblocks, hipStream_t s);

}  // namespace nmf
