// Host engine and C ABI (include/nmf.h): validation, device buffers, the
// hipGraph of one outer iteration of Algorithm 2, and the entry points.
#include "nmf.h"
#include "nmf_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <thread>
#include <new>
#include <string>
#include <vector>

using nmf::Buffers;
using nmf::DevState;

struct nmf_ctx {
    int device = 0;
    nmf_params p{};
    int64_t m = 0, n = 0;
    int r = 0, rp = 0;
    int fmt = NMF_DENSE_ROWMAJOR;
    void *X = nullptr;   // m_pad x ldx, storage dtype, zero padding
    void *Xt = nullptr;  // n_pad x ldxt
    int64_t ldx = 0, ldxt = 0;
    int *zexp_x = nullptr;   // exact-integer path: row scale exponents of X
    int *zexp_xt = nullptr;  // and of X^T
    int prod_kernel = nmf::PK_MFMA_I8;
    nmf::ProdArgs pa{};  // A = X H_w^T
    nmf::ProdArgs pc{};  // C^T = X^T W_y
    nmf::CsrPlan csr_x{};    // sparse X: CSR of X (for A) and of X^T (for C^T)
    nmf::CsrPlan csr_xt{};
    std::vector<void *> extra;   // device arrays of the sparse plans
    double nx2 = 0.0;
    Buffers b;
    hipStream_t own = nullptr;
    // E-ANLS: a second stream on which the Gram inversions run beside the
    // products (fork and join events per side).
    hipStream_t side = nullptr;
    hipEvent_t fork[2] = {nullptr, nullptr}, join[2] = {nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool started = false;
    int32_t launched = 0;
    int cap_h = 0, cap_w = 0;    // adaptive inner loop: sweep caps of the two sides
    DevState hs{};       // host copy of the device state
    double *e2_scale = nullptr;  // test hook of the restart branch (device)
    int32_t e2_scale_n = 0;
    std::string err;
};

namespace {

thread_local std::string g_err;

nmf_status fail(nmf_ctx *ctx, nmf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_err = buf;
    return st;
}

#define HIP_TRY(ctx, call)                                                          \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            return fail(ctx, NMF_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

size_t xbytes(int xdtype) { return xdtype == NMF_X_F32 ? 4 : 2; }

int round_rank(int r) { return ((r + 15) / 16) * 16; }

int64_t round_up(int64_t v, int64_t q) { return ((v + q - 1) / q) * q; }

int choose_kernel(const nmf_params *p, int fmt)
{
    if (fmt == NMF_CSR) return nmf::PK_CSR;
    switch (p->prod) {
    case NMF_PROD_VALU: return nmf::PK_VALU;
    case NMF_PROD_MFMA_EXACT: return nmf::PK_MFMA_I8;
    case NMF_PROD_MFMA_FAST: return nmf::PK_MFMA_X16;
    default: return p->x_dtype == NMF_X_F32 ? nmf::PK_MFMA_I8 : nmf::PK_MFMA_X16;
    }
}

// Split-K plan of one product: enough workgroups of 128 rows (256 for the
// 16-bit kernel) to fill the chip (about 512 for the kernels that run two per
// CU, 256 for the exact-integer and 16-bit kernels, whose 8-wave workgroups
// take a whole CU), K-chunks of whole 64-column tiles.
void plan_product(nmf::ProdArgs &a, int kernel, int64_t rows, int64_t rows_pad, int64_t K,
                  int64_t ld, int64_t target_wg = 0)
{
    a.rows = rows;
    a.rows_pad = rows_pad;
    a.K = K;
    a.ld = ld;
    if (kernel == nmf::PK_VALU || kernel == nmf::PK_CSR) {
        a.nsplit = 1;
        a.kchunk = ld;
        return;
    }
    const int64_t rb = rows_pad / (kernel == nmf::PK_MFMA_X16 ? nmf::kX16Rows : 128), tiles = ld / 64;
    const bool whole_cu = kernel == nmf::PK_MFMA_I8 || kernel == nmf::PK_MFMA_X16;
    const int64_t target = target_wg > 0 ? target_wg : whole_cu ? 256 : 512;
    int64_t want = (target + rb - 1) / rb;
    // The exact-integer sums stay below 2^31 for chunks of at most 65536.
    if (kernel == nmf::PK_MFMA_I8) want = std::max<int64_t>(want, (tiles + 1023) / 1024);
    want = std::max<int64_t>(1, std::min<int64_t>({want, tiles, 64}));
    a.kchunk = ((tiles + want - 1) / want) * 64;
    a.nsplit = (int)((ld + a.kchunk - 1) / a.kchunk);
}

nmf_status check_params(const nmf_params *p)
{
    if (!p) return fail(nullptr, NMF_E_INVAL, "params is NULL");
    if (p->r < 1) return fail(nullptr, NMF_E_INVAL, "r = %d must be >= 1", p->r);
    if (p->r > 64) return fail(nullptr, NMF_E_UNSUPPORTED, "r = %d: ranks above 64 are not provided", p->r);
    if (p->hp < 1 || p->hp > 3) return fail(nullptr, NMF_E_INVAL, "hp = %d must be 1, 2 or 3", p->hp);
    if (!(p->beta0 >= 0.0 && p->beta0 < 1.0))
        return fail(nullptr, NMF_E_INVAL, "beta0 = %g must lie in [0, 1)", p->beta0);
    if (!(1.0 < p->gamma_bar && p->gamma_bar < p->gamma && p->gamma < p->eta) ||
        !std::isfinite(p->eta))
        return fail(nullptr, NMF_E_INVAL,
                    "need 1 < gamma_bar < gamma < eta (got %g, %g, %g)", p->gamma_bar,
                    p->gamma, p->eta);
    if (p->inner_rule != NMF_INNER_FIXED && p->inner_rule != NMF_INNER_EXACT &&
        p->inner_rule != NMF_INNER_ADAPTIVE)
        return fail(nullptr, NMF_E_UNSUPPORTED, "inner_rule %d is not provided", p->inner_rule);
    if (p->inner_rule == NMF_INNER_ADAPTIVE &&
        !(p->inner_alpha >= 0.0 && std::isfinite(p->inner_alpha) && p->inner_delta >= 0.0 &&
          std::isfinite(p->inner_delta)))
        return fail(nullptr, NMF_E_INVAL, "inner_alpha = %g and inner_delta = %g must be finite and >= 0",
                    p->inner_alpha, p->inner_delta);
    if (p->inner_rule == NMF_INNER_ADAPTIVE &&
        !(p->inner_rho_h >= 0.0 && std::isfinite(p->inner_rho_h) && p->inner_rho_w >= 0.0 &&
          std::isfinite(p->inner_rho_w)))
        return fail(nullptr, NMF_E_INVAL, "inner_rho_h = %g and inner_rho_w = %g must be finite and >= 0",
                    p->inner_rho_h, p->inner_rho_w);
    if (p->inner_k < 1 || p->inner_k > 1000)
        return fail(nullptr, NMF_E_INVAL, "inner_k = %d must lie in 1..1000", p->inner_k);
    if (p->max_iter < 0 || p->max_iter > (1 << 28))
        return fail(nullptr, NMF_E_INVAL, "max_iter = %d out of range", p->max_iter);
    if (!(p->tol >= 0.0) || !std::isfinite(p->tol))
        return fail(nullptr, NMF_E_INVAL, "tol = %g must be finite and >= 0", p->tol);
    if (p->x_dtype < NMF_X_F32 || p->x_dtype > NMF_X_F16)
        return fail(nullptr, NMF_E_INVAL, "x_dtype = %d unknown", p->x_dtype);
    if (p->prod < NMF_PROD_AUTO || p->prod > NMF_PROD_MFMA_FAST)
        return fail(nullptr, NMF_E_INVAL, "prod = %d unknown", p->prod);
    if (p->flags & ~(NMF_FLAG_BETABAR_LAST_ACCEPTED | NMF_FLAG_CMP_LAST_ACCEPTED | NMF_FLAG_BETA_STAR))
        return fail(nullptr, NMF_E_INVAL, "unknown flags 0x%x", p->flags);
    return NMF_OK;
}

// Index of the first non-finite value of v[0..cnt), or -1. Blocks are scanned
// without an exit inside (so the scan vectorizes); only a block that holds a
// non-finite value is searched again.
int64_t first_nonfinite(const float *v, int64_t cnt)
{
    constexpr int64_t kBlock = 4096;
    for (int64_t b = 0; b < cnt; b += kBlock) {
        const int64_t e = std::min(cnt, b + kBlock);
        uint32_t bad = 0;
        for (int64_t i = b; i < e; ++i) {
            uint32_t u;
            std::memcpy(&u, v + i, sizeof(u));
            bad |= (uint32_t)((u & 0x7f800000u) == 0x7f800000u);   // exponent all ones: inf or NaN
        }
        if (bad)
            for (int64_t i = b; i < e; ++i)
                if (!std::isfinite(v[i])) return i;
    }
    return -1;
}

int64_t copy_checked_serial(const float *src, float *dst, int64_t cnt, bool *nonzero)
{
    constexpr int64_t kBlock = 4096;
    uint32_t any = 0;
    for (int64_t b = 0; b < cnt; b += kBlock) {
        const int64_t e = std::min(cnt, b + kBlock);
        uint32_t bad = 0;
        for (int64_t i = b; i < e; ++i) {
            uint32_t u;
            std::memcpy(&u, src + i, sizeof(u));
            std::memcpy(dst + i, &u, sizeof(u));
            bad |= (uint32_t)((u & 0x7f800000u) == 0x7f800000u);
            any |= u & 0x7fffffffu;
        }
        if (bad) return first_nonfinite(src + b, e - b) + b;
    }
    *nonzero = any != 0;
    return -1;
}

// copy_checked_serial over up to 4 threads for large arrays (one host core
// copies far below the memory bandwidth).
int64_t copy_checked(const float *src, float *dst, int64_t cnt, bool *nonzero)
{
    constexpr int64_t kPerThread = int64_t(1) << 18;     // 1 MB of floats
    const int nt = (int)std::min<int64_t>(4, cnt / kPerThread);
    if (nt < 2) return copy_checked_serial(src, dst, cnt, nonzero);
    const int64_t chunk = (cnt + nt - 1) / nt;
    int64_t bad[4] = {-1, -1, -1, -1};
    bool nz[4] = {false, false, false, false};
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) {
        const int64_t b = t * chunk, e = std::min(cnt, b + chunk);
        th.emplace_back([=, &bad, &nz] {
            const int64_t i = copy_checked_serial(src + b, dst + b, e - b, &nz[t]);
            bad[t] = i < 0 ? -1 : b + i;
        });
    }
    bad[0] = copy_checked_serial(src, dst, std::min(cnt, chunk), &nz[0]);
    for (auto &x : th) x.join();
    bool any = false;
    for (int t = 0; t < nt; ++t) {
        if (bad[t] >= 0) return bad[t];                    // the first slice with one
        any = any || nz[t];
    }
    *nonzero = any;
    return -1;
}

nmf_status check_matrix(const nmf_matrix *X, bool scan_dense = true)
{
    if (!X) return fail(nullptr, NMF_E_INVAL, "X is NULL");
    if (X->m < 1 || X->n < 1)
        return fail(nullptr, NMF_E_INVAL, "X is %lld x %lld; both must be >= 1",
                    (long long)X->m, (long long)X->n);
    if (X->m > (int64_t)1 << 31 || X->n > (int64_t)1 << 31)
        return fail(nullptr, NMF_E_UNSUPPORTED, "X dimensions above 2^31 are not provided");
    if (X->fmt == NMF_DENSE_ROWMAJOR) {
        if (!X->dense) return fail(nullptr, NMF_E_INVAL, "dense X has a NULL pointer");
        const int64_t bad = scan_dense ? first_nonfinite(X->dense, X->m * X->n) : -1;
        if (bad >= 0)
            return fail(nullptr, NMF_E_INVAL, "X has a non-finite entry at %lld", (long long)bad);
        return NMF_OK;
    }
    if (X->fmt == NMF_CSR) {
        if (X->nnz < 0) return fail(nullptr, NMF_E_INVAL, "nnz = %lld < 0", (long long)X->nnz);
        if (!X->row_ptr || (X->nnz > 0 && (!X->col_idx || !X->val)))
            return fail(nullptr, NMF_E_INVAL, "CSR X has a NULL array");
        if (X->nnz >= ((int64_t)1 << 40))
            return fail(nullptr, NMF_E_UNSUPPORTED, "nnz above 2^40 is not provided");
        if (X->row_ptr[0] != 0 || X->row_ptr[X->m] != X->nnz)
            return fail(nullptr, NMF_E_INVAL, "CSR row_ptr must start at 0 and end at nnz");
        for (int64_t i = 0; i < X->m; ++i) {
            const int64_t b = X->row_ptr[i], e = X->row_ptr[i + 1];
            if (e < b) return fail(nullptr, NMF_E_INVAL, "CSR row_ptr decreases at row %lld", (long long)i);
            for (int64_t j = b; j < e; ++j) {
                const int32_t c = X->col_idx[j];
                if (c < 0 || c >= X->n)
                    return fail(nullptr, NMF_E_INVAL, "CSR column %d out of range at %lld", c, (long long)j);
                if (j > b && c <= X->col_idx[j - 1])
                    return fail(nullptr, NMF_E_INVAL,
                                "CSR columns must increase strictly within a row (row %lld)", (long long)i);
                if (!std::isfinite(X->val[j]))
                    return fail(nullptr, NMF_E_INVAL, "X has a non-finite entry at %lld", (long long)j);
            }
        }
        return NMF_OK;
    }
    return fail(nullptr, NMF_E_INVAL, "fmt = %d unknown", X->fmt);
}

void free_all(nmf_ctx *c)
{
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (void *p : c->extra)
        if (p) (void)hipFree(p);
    void *ptrs[] = {c->X, c->Xt, c->zexp_x, c->zexp_xt, c->b.Wf, c->b.Hf, c->b.GW, c->b.GH,
                    c->b.A, c->b.Ct, c->b.part_g, c->b.part_d, c->b.st, c->b.trace,
                    c->b.accepted, c->b.beta_used, c->b.beta_star, c->b.stage, c->b.fsl, c->b.texp,
                    c->b.x64, c->b.part_n, c->b.sweeps, c->b.ginv_h, c->b.ginv_w,
                    c->e2_scale};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (int i = 0; i < 2; ++i) {
        if (c->fork[i]) (void)hipEventDestroy(c->fork[i]);
        if (c->join[i]) (void)hipEventDestroy(c->join[i]);
    }
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->own) (void)hipStreamDestroy(c->own);
}

template <typename T>
hipError_t dalloc(T **p, size_t count)
{
    return hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(count, 1) * sizeof(T));
}

nmf_status alloc_buffers(nmf_ctx *c)
{
    const int rp = c->rp;
    const int64_t m = c->m, n = c->n;
    const int gs = nmf::gram_stride(rp);
    const int64_t nblk = (std::max(m, n) + nmf::kRowsPerBlock - 1) / nmf::kRowsPerBlock;
    const int64_t rec = nmf::sweep_record(rp);
    Buffers &b = c->b;
    HIP_TRY(c, dalloc(&b.Wf, (size_t)nmf::kSlots * m * rp));
    HIP_TRY(c, dalloc(&b.Hf, (size_t)nmf::kSlots * n * rp));
    HIP_TRY(c, dalloc(&b.GW, (size_t)nmf::kSlots * gs));
    HIP_TRY(c, dalloc(&b.GH, (size_t)gs));
    HIP_TRY(c, dalloc(&b.A, (size_t)c->pa.nsplit * b.m_pad * rp));
    HIP_TRY(c, dalloc(&b.Ct, (size_t)c->pc.nsplit * b.n_pad * rp));
    // Rows that no product writes (padding; empty rows of a sparse X) read as 0.
    HIP_TRY(c, hipMemsetAsync(b.A, 0, sizeof(double) * c->pa.nsplit * b.m_pad * rp, c->own));
    HIP_TRY(c, hipMemsetAsync(b.Ct, 0, sizeof(double) * c->pc.nsplit * b.n_pad * rp, c->own));
    c->pa.Y = b.A;
    c->pc.Y = b.Ct;
    HIP_TRY(c, dalloc(&b.part_g, (size_t)(nblk * rec)));
    HIP_TRY(c, dalloc(&b.part_d, (size_t)1024));
    HIP_TRY(c, dalloc(&b.st, 1));
    HIP_TRY(c, dalloc(&b.trace, (size_t)c->p.max_iter + 1));
    HIP_TRY(c, dalloc(&b.accepted, (size_t)c->p.max_iter));
    HIP_TRY(c, dalloc(&b.beta_used, (size_t)c->p.max_iter));
    HIP_TRY(c, dalloc(&b.beta_star, (size_t)c->p.max_iter + 1));
    HIP_TRY(c, hipMemsetAsync(b.beta_star, 0, sizeof(double) * (c->p.max_iter + 1), c->own));
    HIP_TRY(c, dalloc(&b.stage, (size_t)(m + n) * c->r));
    if (c->p.inner_rule == NMF_INNER_ADAPTIVE) {
        HIP_TRY(c, dalloc(&b.x64, (size_t)std::max(m, n) * rp));
        HIP_TRY(c, dalloc(&b.part_n, 2 * (size_t)nblk));   // by sweep parity
        HIP_TRY(c, dalloc(&b.sweeps, (size_t)2 * std::max(c->p.max_iter, 1)));
        HIP_TRY(c, hipMemsetAsync(b.sweeps, 0, sizeof(int32_t) * 2 * std::max(c->p.max_iter, 1), c->own));
    }
    if (c->p.inner_rule == NMF_INNER_EXACT) {
        HIP_TRY(c, dalloc(&b.ginv_h, (size_t)rp * rp + 1));
        HIP_TRY(c, dalloc(&b.ginv_w, (size_t)rp * rp + 1));
    }
    if (c->prod_kernel == nmf::PK_MFMA_I8 || c->prod_kernel == nmf::PK_MFMA_X16) {
        // Both products slice their factor into one shared buffer (they run in
        // stream order): (ld / 64) tiles of 4 slices x RP columns x 64 rows
        // (int8), or of 2 k-steps x 2 BF16 parts x RP columns x 32 rows.
        HIP_TRY(c, dalloc(&b.fsl, (size_t)std::max(c->ldx, c->ldxt) * 4 * rp));
        HIP_TRY(c, dalloc(&b.texp, (size_t)rp));
    }
    // Zero the factor slots once so that no slot ever holds garbage padding.
    HIP_TRY(c, hipMemsetAsync(b.Wf, 0, sizeof(float) * nmf::kSlots * m * rp, c->own));
    HIP_TRY(c, hipMemsetAsync(b.Hf, 0, sizeof(float) * nmf::kSlots * n * rp, c->own));
    return NMF_OK;
}

nmf_status upload_dense(nmf_ctx *c, const nmf_matrix *X)
{
    const int64_t cnt = c->m * c->n;
    const int xd = c->p.x_dtype;
    const size_t xsz = (size_t)c->b.m_pad * c->ldx * xbytes(xd);
    const size_t xtsz = (size_t)c->b.n_pad * c->ldxt * xbytes(xd);
    HIP_TRY(c, hipMalloc(&c->X, xsz));
    HIP_TRY(c, hipMalloc(&c->Xt, xtsz));
    HIP_TRY(c, hipMemsetAsync(c->X, 0, xsz, c->own));
    HIP_TRY(c, hipMemsetAsync(c->Xt, 0, xtsz, c->own));
    float *src = nullptr;
    HIP_TRY(c, dalloc(&src, (size_t)cnt));
    hipError_t e = hipMemcpyAsync(src, X->dense, sizeof(float) * cnt, hipMemcpyHostToDevice, c->own);
    if (e == hipSuccess)
        e = nmf::launch_convert_x(src, c->m, c->n, xd, c->X, c->ldx, c->Xt, c->ldxt, c->own);
    double *nx2 = nullptr;
    if (e == hipSuccess) e = dalloc(&nx2, 1);
    if (e == hipSuccess)
        e = nmf::launch_sumsq_typed(c->X, xd, (int64_t)(xsz / xbytes(xd)), c->b.part_d, 1024, nx2,
                                    c->own);
    if (e == hipSuccess) e = hipStreamSynchronize(c->own);
    if (e == hipSuccess) e = hipMemcpy(&c->nx2, nx2, sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(src);
    if (nx2) (void)hipFree(nx2);
    if (e != hipSuccess)
        return fail(c, NMF_E_DEVICE, "uploading X failed: %s", hipGetErrorString(e));
    // Replaces X and X^T by the copies the product streams, made by `fill`
    // into new buffers of xs_bytes and xts_bytes; the new buffers are freed
    // again if any step fails.
    auto replace_x = [&](size_t xs_bytes, size_t xts_bytes, auto fill) -> nmf_status {
        void *xs = nullptr, *xts = nullptr;
        hipError_t e2 = hipMalloc(&xs, xs_bytes);
        if (e2 == hipSuccess) e2 = hipMalloc(&xts, xts_bytes);
        if (e2 == hipSuccess) e2 = fill(xs, xts);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->own);
        if (e2 != hipSuccess) {
            if (xs) (void)hipFree(xs);
            if (xts) (void)hipFree(xts);
            return fail(c, NMF_E_DEVICE, "preparing X for the product failed: %s",
                        hipGetErrorString(e2));
        }
        (void)hipFree(c->X);
        (void)hipFree(c->Xt);
        c->X = xs;
        c->Xt = xts;
        return NMF_OK;
    };
    if (c->prod_kernel == nmf::PK_MFMA_I8) {
        // Keep only the int8 slices of X and X^T (4 bytes per entry).
        HIP_TRY(c, dalloc(&c->zexp_x, (size_t)c->b.m_pad));
        HIP_TRY(c, dalloc(&c->zexp_xt, (size_t)c->b.n_pad));
        HIP_TRY(c, hipMemsetAsync(c->zexp_x, 0, sizeof(int) * c->b.m_pad, c->own));
        HIP_TRY(c, hipMemsetAsync(c->zexp_xt, 0, sizeof(int) * c->b.n_pad, c->own));
        const size_t sb = (size_t)c->b.m_pad * c->ldx * 4, stb = (size_t)c->b.n_pad * c->ldxt * 4;
        const nmf_status st = replace_x(sb, stb, [&](void *xs, void *xts) {
            hipError_t e3 = hipMemsetAsync(xs, 0, sb, c->own);
            if (e3 == hipSuccess) e3 = hipMemsetAsync(xts, 0, stb, c->own);
            if (e3 == hipSuccess)
                e3 = nmf::i8::slice_rows(c->X, xd, c->m, c->n, c->ldx, c->ldx, xs, c->zexp_x, c->own);
            if (e3 == hipSuccess)
                e3 = nmf::i8::slice_rows(c->Xt, xd, c->n, c->m, c->ldxt, c->ldxt, xts, c->zexp_xt,
                                         c->own);
            return e3;
        });
        if (st != NMF_OK) return st;
    }
    if (c->prod_kernel == nmf::PK_MFMA_X16) {
        // Keep X and X^T in 16 bits, in the fragment order the product streams.
        const nmf_status st = replace_x(xsz, xtsz, [&](void *xf, void *xtf) {
            hipError_t e3 = nmf::x16::to_fragments(c->X, c->b.m_pad, c->ldx, xf, c->own);
            if (e3 == hipSuccess) e3 = nmf::x16::to_fragments(c->Xt, c->b.n_pad, c->ldxt, xtf, c->own);
            return e3;
        });
        if (st != NMF_OK) return st;
    }
    return NMF_OK;
}

// Copies a host array to a new device array owned by the context.
template <typename T>
hipError_t to_device(nmf_ctx *c, const T *h, size_t count, const T **out)
{
    T *d = nullptr;
    hipError_t e = dalloc(&d, count);
    if (e != hipSuccess) return e;
    c->extra.push_back(d);
    if (count) e = hipMemcpyAsync(d, h, sizeof(T) * count, hipMemcpyHostToDevice, c->own);
    *out = d;
    return e;
}

// Work items of a sparse product (see CsrPlan) and their device copies.
hipError_t build_plan(nmf_ctx *c, int64_t rows, const int64_t *rp, const int32_t *col,
                      const float *val, nmf::CsrPlan *P)
{
    const int64_t T = nmf::csr_item_nnz(c->rp);
    std::vector<int32_t> irow, islot, lrow, lfirst, lcount;
    std::vector<int64_t> ibeg, iend;
    int32_t slots = 0;
    for (int64_t i = 0; i < rows; ++i) {
        const int64_t b = rp[i], e = rp[i + 1];
        if (e == b) continue;
        const int64_t parts = (e - b + T - 1) / T;
        if (parts > 1) {
            lrow.push_back((int32_t)i);
            lfirst.push_back(slots);
            lcount.push_back((int32_t)parts);
        }
        for (int64_t q = 0; q < parts; ++q) {
            irow.push_back((int32_t)i);
            ibeg.push_back(b + q * T);
            iend.push_back(std::min(e, b + (q + 1) * T));
            islot.push_back(parts > 1 ? slots++ : -1);
        }
    }
    const int64_t nnz = rp[rows];
    P->rows = rows;
    P->nitems = (int64_t)irow.size();
    P->nlong = (int64_t)lrow.size();
    hipError_t e = to_device(c, rp, (size_t)rows + 1, &P->row_ptr);
    if (e == hipSuccess) e = to_device(c, col, (size_t)nnz, &P->col);
    if (e == hipSuccess) e = to_device(c, val, (size_t)nnz, &P->val);
    if (e == hipSuccess) e = to_device(c, irow.data(), irow.size(), &P->item_row);
    if (e == hipSuccess) e = to_device(c, ibeg.data(), ibeg.size(), &P->item_beg);
    if (e == hipSuccess) e = to_device(c, iend.data(), iend.size(), &P->item_end);
    if (e == hipSuccess) e = to_device(c, islot.data(), islot.size(), &P->item_slot);
    if (e == hipSuccess) e = to_device(c, lrow.data(), lrow.size(), &P->long_row);
    if (e == hipSuccess) e = to_device(c, lfirst.data(), lfirst.size(), &P->long_first);
    if (e == hipSuccess) e = to_device(c, lcount.data(), lcount.size(), &P->long_count);
    if (e == hipSuccess) {
        double *part = nullptr;
        e = dalloc(&part, (size_t)std::max<int32_t>(slots, 1) * c->rp);
        if (e == hipSuccess) c->extra.push_back(part);
        P->partial = part;
    }
    return e;
}

// Sparse X: the CSR as given, its transpose (CSC of X, columns in row order)
// built here, the work items of both products, and ||X||^2 from the values.
nmf_status upload_csr(nmf_ctx *c, const nmf_matrix *X)
{
    const int64_t m = c->m, n = c->n, nnz = X->nnz;
    std::vector<int64_t> cp((size_t)n + 1, 0);
    for (int64_t j = 0; j < nnz; ++j) ++cp[(size_t)X->col_idx[j] + 1];
    for (int64_t k = 0; k < n; ++k) cp[k + 1] += cp[k];
    std::vector<int64_t> next(cp.begin(), cp.end() - 1);
    std::vector<int32_t> ri((size_t)nnz);
    std::vector<float> rv((size_t)nnz);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = X->row_ptr[i]; j < X->row_ptr[i + 1]; ++j) {
            const int64_t pos = next[X->col_idx[j]]++;
            ri[pos] = (int32_t)i;
            rv[pos] = X->val[j];
        }
    HIP_TRY(c, build_plan(c, m, X->row_ptr, X->col_idx, X->val, &c->csr_x));
    HIP_TRY(c, build_plan(c, n, cp.data(), ri.data(), rv.data(), &c->csr_xt));
    double *nx2 = nullptr;
    HIP_TRY(c, dalloc(&nx2, 1));
    c->extra.push_back(nx2);
    HIP_TRY(c, nmf::launch_sumsq(c->csr_x.val, nnz, c->b.part_d, 1024, nx2, c->own));
    HIP_TRY(c, hipStreamSynchronize(c->own));
    HIP_TRY(c, hipMemcpy(&c->nx2, nx2, sizeof(double), hipMemcpyDeviceToHost));
    return NMF_OK;
}

// One outer iteration (nine kernels in eight phases). With `ev`
// non-null, ev[i] is recorded before kernel i (enum nmf_phase) and
// ev[NMF_PHASE_COUNT] after the last one.
nmf_status enqueue_iteration(nmf_ctx *c, hipStream_t s, hipEvent_t *ev = nullptr)
{
    const int rp = c->rp, xd = c->p.x_dtype, pk = c->prod_kernel;
    const bool exact = c->p.inner_rule == NMF_INNER_EXACT;
    const bool adaptive = c->p.inner_rule == NMF_INNER_ADAPTIVE;
    Buffers &b = c->b;
    auto e = [&](int i) { return ev ? ev[i] : nullptr; };
    // a1: C^T = X^T W_y ; a2-a4: H sweeps + epilogue ; a5: A = X H_w^T ;
    // a6-a8: W sweeps + epilogue + decision. Exact solves: the inverse of
    // each Gram matrix is taken on the side stream while the product that
    // precedes its solve runs (fork after the Gram is final, join before the
    // solve).
    auto fork = [&](int side) -> nmf_status {
        HIP_TRY(c, hipEventRecord(c->fork[side], s));
        HIP_TRY(c, hipStreamWaitEvent(c->side, c->fork[side], 0));
        HIP_TRY(c, nmf::launch_invert(rp, side == 1, c->r, b, c->side));
        HIP_TRY(c, hipEventRecord(c->join[side], c->side));
        return NMF_OK;
    };
    if (exact) {
        const nmf_status fs = fork(0);
        if (fs != NMF_OK) return fs;
    }
    if (ev) HIP_TRY(c, hipEventRecord(ev[NMF_PHASE_SLICE_W], s));
    HIP_TRY(c, nmf::launch_product(rp, xd, pk, c->pc, s, e(NMF_PHASE_PROD_CT)));
    if (exact) HIP_TRY(c, hipStreamWaitEvent(s, c->join[0], 0));
    if (ev) HIP_TRY(c, hipEventRecord(ev[NMF_PHASE_SWEEP_H], s));
    if (adaptive)
        HIP_TRY(c, nmf::launch_sweep_h_adaptive(rp, c->n, c->r, c->cap_h, c->p.inner_delta, b, s,
                                                e(NMF_PHASE_FINISH_H)));
    else
        HIP_TRY(c, nmf::launch_sweep_h(rp, c->n, c->r, c->p.inner_k, exact, b, s, e(NMF_PHASE_FINISH_H)));
    if (exact) {
        const nmf_status fs = fork(1);
        if (fs != NMF_OK) return fs;
    }
    if (ev) HIP_TRY(c, hipEventRecord(ev[NMF_PHASE_SLICE_H], s));
    HIP_TRY(c, nmf::launch_product(rp, xd, pk, c->pa, s, e(NMF_PHASE_PROD_A)));
    if (exact) HIP_TRY(c, hipStreamWaitEvent(s, c->join[1], 0));
    if (ev) HIP_TRY(c, hipEventRecord(ev[NMF_PHASE_SWEEP_W], s));
    if (adaptive)
        HIP_TRY(c, nmf::launch_sweep_w_adaptive(rp, c->m, c->r, c->cap_w, c->p.inner_delta, b, s,
                                                e(NMF_PHASE_FINISH_W)));
    else
        HIP_TRY(c, nmf::launch_sweep_w(rp, c->m, c->r, c->p.inner_k, exact, b, s, e(NMF_PHASE_FINISH_W)));
    if (ev) HIP_TRY(c, hipEventRecord(ev[NMF_PHASE_COUNT], s));
    return NMF_OK;
}

nmf_status build_graph(nmf_ctx *c)
{
    HIP_TRY(c, hipStreamBeginCapture(c->own, hipStreamCaptureModeThreadLocal));
    nmf_status st = enqueue_iteration(c, c->own);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->own, &g);
    if (st != NMF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(c, NMF_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    c->graph = g;
    HIP_TRY(c, hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0));
    return NMF_OK;
}

}  // namespace

namespace nmf {
namespace host {
void set_error(const std::string &msg) { g_err = msg; }
nmf_status check_params(const nmf_params *p) { return ::check_params(p); }
nmf_status check_matrix(const nmf_matrix *X) { return ::check_matrix(X, true); }
nmf_status check_matrix_shape(const nmf_matrix *X) { return ::check_matrix(X, false); }
int64_t copy_checked(const float *src, float *dst, int64_t cnt, bool *nonzero)
{
    return ::copy_checked(src, dst, cnt, nonzero);
}
int round_rank(int r) { return ::round_rank(r); }
int64_t round_up(int64_t v, int64_t q) { return ::round_up(v, q); }
void plan_product(ProdArgs &a, int kernel, int64_t rows, int64_t rows_pad, int64_t K, int64_t ld,
                  int64_t target_wg)
{
    ::plan_product(a, kernel, rows, rows_pad, K, ld, target_wg);
}
}  // namespace host
}  // namespace nmf

extern "C" {

void nmf_params_default(nmf_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->r = 10;
    p->hp = 3;
    p->beta0 = 0.5;
    p->gamma = 1.01;
    p->gamma_bar = 1.005;
    p->eta = 1.5;
    p->inner_rule = NMF_INNER_FIXED;
    p->inner_k = 10;
    p->max_iter = 100;
    p->tol = 0.0;
    p->x_dtype = NMF_X_F32;
    p->prod = NMF_PROD_AUTO;
    p->flags = 0;
    p->inner_alpha = 0.5;
    p->inner_delta = 0.1;
    p->inner_rho_h = 0.0;
    p->inner_rho_w = 0.0;
}

nmf_status nmf_create(const nmf_matrix *X, const nmf_params *p, nmf_ctx **out)
{
    if (!out) return fail(nullptr, NMF_E_INVAL, "out is NULL");
    *out = nullptr;
    nmf_status st = check_params(p);
    if (st != NMF_OK) return st;
    st = check_matrix(X);
    if (st != NMF_OK) return st;
    if (X->fmt == NMF_CSR && (p->x_dtype != NMF_X_F32 || p->prod == NMF_PROD_MFMA_FAST))
        return fail(nullptr, NMF_E_UNSUPPORTED,
                    "sparse X is kept in FP32 with FP64 sums: x_dtype must be F32 and prod not MFMA_FAST");
    if (X->fmt != NMF_CSR && p->x_dtype == NMF_X_F32 && p->prod == NMF_PROD_MFMA_FAST)
        return fail(nullptr, NMF_E_UNSUPPORTED,
                    "MFMA_FAST streams X in 16 bits: it needs x_dtype BF16 or F16 "
                    "(FP32 X uses MFMA_EXACT or VALU)");

    nmf_ctx *c = new (std::nothrow) nmf_ctx();
    if (!c) return fail(nullptr, NMF_E_NOMEM, "host allocation failed");
    c->p = *p;
    c->m = X->m;
    c->n = X->n;
    c->r = p->r;
    c->rp = round_rank(p->r);
    c->fmt = X->fmt;
    c->prod_kernel = choose_kernel(p, X->fmt);
    const int64_t row_q = (c->prod_kernel == nmf::PK_MFMA_X16) ? nmf::kX16Rows : 128;
    c->b.m_pad = round_up(c->m, row_q);
    c->b.n_pad = round_up(c->n, row_q);
    c->ldx = round_up(c->n, 64);
    c->ldxt = round_up(c->m, 64);
    plan_product(c->pa, c->prod_kernel, c->m, c->b.m_pad, c->n, c->ldx);
    plan_product(c->pc, c->prod_kernel, c->n, c->b.n_pad, c->m, c->ldxt);
    c->b.nsplit_a = c->pa.nsplit;
    c->b.nsplit_c = c->pc.nsplit;
    c->b.lin_f32 = c->prod_kernel == nmf::PK_MFMA_X16;
    c->b.beta_star_on = (c->p.flags & NMF_FLAG_BETA_STAR) != 0;
    if (p->inner_rule == NMF_INNER_ADAPTIVE) {
        // Sweep caps floor(1 + alpha rho), rho = 1 + (mn + K r) / (R (r + 1)) for
        // R rows updated against K fixed ones (nnz for mn when X is sparse), or
        // the caller's cost ratio of the side when it is positive.
        const double mn = X->fmt == NMF_CSR ? (double)X->nnz : (double)c->m * (double)c->n;
        auto cap = [&](double rows, double fixed, double given) {
            const double rho = given > 0.0 ? given : 1.0 + (mn + fixed * c->r) / (rows * (c->r + 1.0));
            const double k = std::floor(1.0 + p->inner_alpha * rho);
            return (int)std::max(1.0, std::min(k, (double)p->inner_k));
        };
        c->cap_h = cap((double)c->n, (double)c->m, p->inner_rho_h);
        c->cap_w = cap((double)c->m, (double)c->n, p->inner_rho_w);
    }
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking);
    if (e == hipSuccess && p->inner_rule == NMF_INNER_EXACT) {
        e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
        for (int i = 0; i < 2 && e == hipSuccess; ++i) {
            e = hipEventCreateWithFlags(&c->fork[i], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming);
        }
    }
    if (e != hipSuccess) {
        fail(nullptr, NMF_E_DEVICE, "no usable HIP device: %s", hipGetErrorString(e));
        free_all(c);
        delete c;
        return NMF_E_DEVICE;
    }
    st = alloc_buffers(c);
    if (st == NMF_OK) st = (X->fmt == NMF_CSR) ? upload_csr(c, X) : upload_dense(c, X);
    if (st == NMF_OK) {
        // A = X H_w^T reads X and the H slots; C^T = X^T W_y reads X^T and the W slots.
        c->pa.Z = c->X;
        c->pa.F_base = c->b.Hf;
        c->pa.slot_stride = c->n * c->rp;
        c->pa.sel = nmf::SEL_H_W;
        c->pa.st = c->b.st;
        c->pa.zexp = c->zexp_x;
        c->pa.gram_base = c->b.GH;
        c->pa.gram_slot_stride = 0;
        c->pa.Fsl = c->b.fsl;
        c->pa.texp = c->b.texp;
        c->pc.Z = c->Xt;
        c->pc.F_base = c->b.Wf;
        c->pc.slot_stride = c->m * c->rp;
        c->pc.sel = nmf::SEL_W_Y;
        c->pc.st = c->b.st;
        c->pc.zexp = c->zexp_xt;
        c->pc.gram_base = c->b.GW;
        c->pc.gram_slot_stride = nmf::gram_stride(c->rp);
        c->pc.Fsl = c->b.fsl;
        c->pc.texp = c->b.texp;
        c->pa.csr = &c->csr_x;
        c->pc.csr = &c->csr_xt;
    }
    if (st == NMF_OK && !(c->nx2 > 0.0))
        st = fail(c, NMF_E_INVAL, "X is zero: the relative error is undefined");
    if (st == NMF_OK) st = build_graph(c);
    // Every set-up step ran on the context's stream; finish them before any
    // other stream may touch the buffers.
    if (st == NMF_OK && hipStreamSynchronize(c->own) != hipSuccess)
        st = fail(c, NMF_E_DEVICE, "set-up on the device failed");
    if (st != NMF_OK) {
        g_err = c->err;
        free_all(c);
        delete c;
        return st;
    }
    *out = c;
    return NMF_OK;
}

nmf_status nmf_start(nmf_ctx *c, const float *W0, const float *H0, int32_t on_device,
                     void *stream)
{
    if (!c) return fail(nullptr, NMF_E_INVAL, "ctx is NULL");
    if (!W0 || !H0) return fail(c, NMF_E_INVAL, "W0 and H0 must not be NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t m = c->m, n = c->n;
    const int r = c->r;
    HIP_TRY(c, hipSetDevice(c->device));
    const float *w0 = W0, *h0 = H0;
    if (!on_device) {
        for (int64_t i = 0; i < m * r; ++i)
            if (!(W0[i] >= 0.0f) || !std::isfinite(W0[i]))
                return fail(c, NMF_E_INVAL, "W0 has a negative or non-finite entry at %lld", (long long)i);
        for (int64_t i = 0; i < (int64_t)r * n; ++i)
            if (!(H0[i] >= 0.0f) || !std::isfinite(H0[i]))
                return fail(c, NMF_E_INVAL, "H0 has a negative or non-finite entry at %lld", (long long)i);
        HIP_TRY(c, hipMemcpyAsync(c->b.stage, W0, sizeof(float) * m * r, hipMemcpyHostToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(c->b.stage + m * r, H0, sizeof(float) * r * n,
                                  hipMemcpyHostToDevice, s));
        w0 = c->b.stage;
        h0 = c->b.stage + m * r;
    }
    DevState &h = c->hs;
    std::memset(&h, 0, sizeof(h));
    h.hp = c->p.hp;
    h.w_acc = h.w_y = 0;
    h.h_acc = h.h_y = 0;
    nmf::plan_slots(0, 0, &h.w_n, &h.w_yn);
    nmf::plan_slots(0, 0, &h.h_n, &h.h_yn);
    h.max_iter = c->p.max_iter;
    h.flags = c->p.flags;
    h.r = r;
    h.beta = c->p.beta0;        // beta of iteration 1
    h.betabar = 1.0;            // upper bound, once per solve
    h.beta_prev = c->p.beta0;
    h.beta_acc = c->p.beta0;
    h.nx2 = c->nx2;
    h.tol = c->p.tol;
    h.gamma = c->p.gamma;
    h.gamma_bar = c->p.gamma_bar;
    h.eta = c->p.eta;
    h.e2_scale = c->e2_scale;
    h.e2_scale_n = c->e2_scale_n;
    const int rp = c->rp;
    Buffers &b = c->b;
    HIP_TRY(c, hipMemcpyAsync(b.st, &h, sizeof(h), hipMemcpyHostToDevice, s));
    HIP_TRY(c, nmf::launch_pack(rp, m, n, r, w0, h0, b, s));
    HIP_TRY(c, nmf::launch_setup_gram_h(rp, n, r, b, s));
    nmf::ProdArgs a0 = c->pa;
    a0.sel = nmf::SEL_SLOT0;   // A = X H0^T for e(0)
    HIP_TRY(c, nmf::launch_product(rp, c->p.x_dtype, c->prod_kernel, a0, s));
    HIP_TRY(c, nmf::launch_setup_error(rp, m, r, b, s));
    HIP_TRY(c, hipMemcpyAsync(&h, b.st, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    c->started = false;
    if (h.bad_input) return fail(c, NMF_E_INVAL, "W0 or H0 has a negative or non-finite entry");
    if (!std::isfinite(h.e0)) return fail(c, NMF_E_NUMERIC, "the initial error e(0) is not finite");
    c->started = true;
    c->launched = 0;
    return NMF_OK;
}

nmf_status nmf_set_error_scale(nmf_ctx *c, const double *scale, int32_t count)
{
    if (!c) return fail(nullptr, NMF_E_INVAL, "ctx is NULL");
    if (count < 0 || (count > 0 && !scale))
        return fail(c, NMF_E_INVAL, "need count >= 0 and a scale array when count > 0");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());     // no running iteration reads the old array
    if (c->e2_scale) HIP_TRY(c, hipFree(c->e2_scale));
    c->e2_scale = nullptr;
    c->e2_scale_n = 0;
    if (count == 0) return NMF_OK;
    HIP_TRY(c, hipMalloc(reinterpret_cast<void **>(&c->e2_scale), sizeof(double) * count));
    HIP_TRY(c, hipMemcpy(c->e2_scale, scale, sizeof(double) * count, hipMemcpyHostToDevice));
    c->e2_scale_n = count;
    return NMF_OK;
}

nmf_status nmf_iterate(nmf_ctx *c, int32_t iters, void *stream)
{
    if (!c) return fail(nullptr, NMF_E_INVAL, "ctx is NULL");
    if (!c->started) return fail(c, NMF_E_STATE, "nmf_iterate before a successful nmf_start");
    if (iters < 0) return fail(c, NMF_E_INVAL, "iters = %d must be >= 0", iters);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t todo = std::min<int32_t>(iters, c->p.max_iter - c->launched);
    for (int32_t i = 0; i < todo; ++i) HIP_TRY(c, hipGraphLaunch(c->exec, s));
    c->launched += std::max(todo, 0);
    return NMF_OK;
}

nmf_status nmf_read(nmf_ctx *c, float *W, float *H, int32_t on_device, double *trace,
                    int32_t trace_cap, int32_t *n_iter, uint8_t *accepted, double *beta,
                    void *stream)
{
    if (!c) return fail(nullptr, NMF_E_INVAL, "ctx is NULL");
    if (!c->started) return fail(c, NMF_E_STATE, "nmf_read before a successful nmf_start");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(c, hipStreamSynchronize(s));
    DevState &h = c->hs;
    HIP_TRY(c, hipMemcpy(&h, c->b.st, sizeof(h), hipMemcpyDeviceToHost));
    const int32_t k = h.k;
    if (trace && trace_cap < k + 1)
        return fail(c, NMF_E_INVAL, "trace_cap = %d < %d", trace_cap, k + 1);
    const int64_t m = c->m, n = c->n;
    const int r = c->r;
    if (W || H) {
        float *dw = on_device ? W : c->b.stage;
        float *dh = on_device ? H : c->b.stage + m * r;
        if (on_device && (!W || !H)) return fail(c, NMF_E_INVAL, "device W and H must both be given");
        HIP_TRY(c, nmf::launch_unpack(c->rp, m, n, r, c->b, dw, dh, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        if (!on_device) {
            if (W) HIP_TRY(c, hipMemcpy(W, dw, sizeof(float) * m * r, hipMemcpyDeviceToHost));
            if (H) HIP_TRY(c, hipMemcpy(H, dh, sizeof(float) * r * n, hipMemcpyDeviceToHost));
        }
    }
    if (trace) HIP_TRY(c, hipMemcpy(trace, c->b.trace, sizeof(double) * (k + 1), hipMemcpyDeviceToHost));
    if (accepted && k > 0)
        HIP_TRY(c, hipMemcpy(accepted, c->b.accepted, (size_t)k, hipMemcpyDeviceToHost));
    if (beta && k > 0)
        HIP_TRY(c, hipMemcpy(beta, c->b.beta_used, sizeof(double) * k, hipMemcpyDeviceToHost));
    if (n_iter) *n_iter = k;
    return NMF_OK;
}

}  // extern "C"

namespace {

// Header of a saved state: what it was saved from, so that a load into a
// context of another problem or other parameters is refused.
struct StateHeader {
    char magic[8];
    int32_t version, r, hp, inner_rule, inner_k, x_dtype, prod, flags, max_iter, stopped;
    int64_t m, n;
    double beta0, gamma, gamma_bar, eta, tol, inner_alpha, inner_delta, inner_rho_h, inner_rho_w, nx2;
    uint64_t bytes;
};
constexpr char kStateMagic[8] = {'N', 'M', 'F', 'S', 'T', 'A', 'T', 'E'};
constexpr int32_t kStateVersion = 2;

// The device buffers that carry a solve from one iteration to the next: the
// factor slots, the Gram buffers of the slots (with their inverse diagonals
// and column maxima), the per-iteration records, and the adaptive loop's
// sweep counts. Everything else is recomputed within an iteration.
struct StatePart {
    void *dev;
    size_t bytes;
};

std::vector<StatePart> state_parts(nmf_ctx *c)
{
    const int64_t m = c->m, n = c->n, rp = c->rp;
    const size_t iters = (size_t)std::max(c->p.max_iter, 1);
    const size_t gs = (size_t)nmf::gram_stride(c->rp);
    std::vector<StatePart> v = {
        {c->b.Wf, sizeof(float) * nmf::kSlots * m * rp},
        {c->b.Hf, sizeof(float) * nmf::kSlots * n * rp},
        {c->b.GW, sizeof(double) * nmf::kSlots * gs},
        {c->b.GH, sizeof(double) * gs},
        {c->b.trace, sizeof(double) * (c->p.max_iter + 1)},
        {c->b.accepted, iters},
        {c->b.beta_used, sizeof(double) * iters},
        {c->b.beta_star, sizeof(double) * (c->p.max_iter + 1)}};
    if (c->p.inner_rule == NMF_INNER_ADAPTIVE) v.push_back({c->b.sweeps, sizeof(int32_t) * 2 * iters});
    return v;
}

size_t state_bytes(nmf_ctx *c)
{
    size_t total = sizeof(StateHeader) + sizeof(DevState);
    for (const StatePart &q : state_parts(c)) total += q.bytes;
    return total;
}

}  // namespace

extern "C" {

nmf_status nmf_state_size(nmf_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return fail(c, NMF_E_INVAL, "ctx and bytes must not be NULL");
    *bytes = state_bytes(c);
    return NMF_OK;
}

nmf_status nmf_save_state(nmf_ctx *c, void *buf, size_t cap, void *stream)
{
    if (!c) return fail(nullptr, NMF_E_INVAL, "ctx is NULL");
    if (!c->started) return fail(c, NMF_E_STATE, "nmf_save_state before a successful nmf_start");
    const size_t need = state_bytes(c);
    if (!buf || cap < need) return fail(c, NMF_E_INVAL, "need a buffer of %zu bytes", need);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    HIP_TRY(c, hipDeviceSynchronize());
    char *out = static_cast<char *>(buf);
    DevState h{};
    HIP_TRY(c, hipMemcpy(&h, c->b.st, sizeof(h), hipMemcpyDeviceToHost));
    StateHeader hd{};
    std::memcpy(hd.magic, kStateMagic, sizeof(hd.magic));
    hd.version = kStateVersion;
    hd.r = c->r;
    hd.hp = c->p.hp;
    hd.inner_rule = c->p.inner_rule;
    hd.inner_k = c->p.inner_k;
    hd.x_dtype = c->p.x_dtype;
    hd.prod = c->p.prod;
    hd.flags = c->p.flags;
    hd.max_iter = c->p.max_iter;
    hd.stopped = (h.done && h.k < c->p.max_iter) ? 1 : 0;   // by the tol rule
    hd.m = c->m;
    hd.n = c->n;
    hd.beta0 = c->p.beta0;
    hd.gamma = c->p.gamma;
    hd.gamma_bar = c->p.gamma_bar;
    hd.eta = c->p.eta;
    hd.tol = c->p.tol;
    hd.inner_alpha = c->p.inner_alpha;
    hd.inner_delta = c->p.inner_delta;
    hd.inner_rho_h = c->p.inner_rho_h;
    hd.inner_rho_w = c->p.inner_rho_w;
    hd.nx2 = c->nx2;
    hd.bytes = need;
    std::memcpy(out, &hd, sizeof(hd));
    std::memcpy(out + sizeof(hd), &h, sizeof(h));
    size_t off = sizeof(hd) + sizeof(h);
    for (const StatePart &q : state_parts(c)) {
        HIP_TRY(c, hipMemcpy(out + off, q.dev, q.bytes, hipMemcpyDeviceToHost));
        off += q.bytes;
    }
    return NMF_OK;
}

nmf_status nmf_load_state(nmf_ctx *c, const void *buf, size_t len, void *stream)
{
    if (!c) return fail(nullptr, NMF_E_INVAL, "ctx is NULL");
    if (!buf || len < sizeof(StateHeader)) return fail(c, NMF_E_INVAL, "not a saved state");
    const char *in = static_cast<const char *>(buf);
    StateHeader hd;
    std::memcpy(&hd, in, sizeof(hd));
    if (std::memcmp(hd.magic, kStateMagic, sizeof(hd.magic)) != 0 || hd.version != kStateVersion)
        return fail(c, NMF_E_INVAL, "not a saved state of this library version");
    const nmf_params &p = c->p;
    if (hd.m != c->m || hd.n != c->n || hd.r != c->r)
        return fail(c, NMF_E_INVAL, "the state is of a %lld x %lld, r = %d problem",
                    (long long)hd.m, (long long)hd.n, hd.r);
    if (hd.nx2 != c->nx2) return fail(c, NMF_E_INVAL, "the state was saved for another X");
    if (hd.hp != p.hp || hd.inner_rule != p.inner_rule || hd.inner_k != p.inner_k ||
        hd.x_dtype != p.x_dtype || hd.prod != p.prod || hd.flags != p.flags ||
        hd.beta0 != p.beta0 || hd.gamma != p.gamma || hd.gamma_bar != p.gamma_bar ||
        hd.eta != p.eta || hd.tol != p.tol || hd.inner_alpha != p.inner_alpha ||
        hd.inner_delta != p.inner_delta || hd.inner_rho_h != p.inner_rho_h ||
        hd.inner_rho_w != p.inner_rho_w)
        return fail(c, NMF_E_INVAL, "the state was saved with other parameters");
    DevState h;
    std::memcpy(&h, in + sizeof(hd), sizeof(h));
    if (h.k < 0 || h.k > p.max_iter)
        return fail(c, NMF_E_INVAL, "the state has %d iterations, beyond max_iter = %d", h.k, p.max_iter);
    if (hd.max_iter != p.max_iter) {
        // The per-iteration records are sized by max_iter: only equal sizes load.
        return fail(c, NMF_E_INVAL, "the state was saved with max_iter = %d", hd.max_iter);
    }
    const size_t need = state_bytes(c);
    if (len < need || hd.bytes != need) return fail(c, NMF_E_INVAL, "the state is truncated");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // This context's own device pointers and stop rule.
    h.e2_scale = c->e2_scale;
    h.e2_scale_n = c->e2_scale_n;
    h.max_iter = p.max_iter;
    h.done = (hd.stopped || h.k >= p.max_iter) ? 1 : 0;
    c->hs = h;
    size_t off = sizeof(hd) + sizeof(h);
    for (const StatePart &q : state_parts(c)) {
        HIP_TRY(c, hipMemcpyAsync(q.dev, in + off, q.bytes, hipMemcpyHostToDevice, s));
        off += q.bytes;
    }
    HIP_TRY(c, hipMemcpyAsync(c->b.st, &c->hs, sizeof(h), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    c->started = true;
    c->launched = h.k;
    return NMF_OK;
}

nmf_status nmf_read_sweeps(nmf_ctx *c, int32_t *sweeps, int32_t cap, int32_t *n_iter)
{
    if (!c) return fail(nullptr, NMF_E_INVAL, "ctx is NULL");
    if (!c->started) return fail(c, NMF_E_STATE, "nmf_read_sweeps before a successful nmf_start");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    DevState h{};
    HIP_TRY(c, hipMemcpy(&h, c->b.st, sizeof(h), hipMemcpyDeviceToHost));
    if (sweeps && cap < h.k) return fail(c, NMF_E_INVAL, "cap = %d < %d", cap, h.k);
    if (sweeps && h.k > 0) {
        if (c->p.inner_rule == NMF_INNER_ADAPTIVE) {
            HIP_TRY(c, hipMemcpy(sweeps, c->b.sweeps, sizeof(int32_t) * 2 * h.k, hipMemcpyDeviceToHost));
        } else {
            const int32_t v = c->p.inner_rule == NMF_INNER_EXACT ? 0 : c->p.inner_k;
            for (int32_t i = 0; i < 2 * h.k; ++i) sweeps[i] = v;
        }
    }
    if (n_iter) *n_iter = h.k;
    return NMF_OK;
}

nmf_status nmf_read_beta_star(nmf_ctx *c, double *beta_star, int32_t cap, int32_t *n_iter)
{
    if (!c) return fail(nullptr, NMF_E_INVAL, "ctx is NULL");
    if (!(c->p.flags & NMF_FLAG_BETA_STAR))
        return fail(c, NMF_E_STATE, "the context was created without NMF_FLAG_BETA_STAR");
    if (!c->started) return fail(c, NMF_E_STATE, "nmf_read_beta_star before a successful nmf_start");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    DevState h{};
    HIP_TRY(c, hipMemcpy(&h, c->b.st, sizeof(h), hipMemcpyDeviceToHost));
    if (beta_star && cap < h.k) return fail(c, NMF_E_INVAL, "cap = %d < %d", cap, h.k);
    if (beta_star && h.k > 0)
        HIP_TRY(c, hipMemcpy(beta_star, c->b.beta_star, sizeof(double) * h.k, hipMemcpyDeviceToHost));
    if (n_iter) *n_iter = h.k;
    return NMF_OK;
}

nmf_status nmf_solve(nmf_ctx *c, const float *W0, const float *H0, float *W, float *H,
                     double *trace, int32_t trace_cap, int32_t *n_iter, uint8_t *accepted,
                     double *beta)
{
    if (!c) return fail(nullptr, NMF_E_INVAL, "ctx is NULL");
    if (!W || !H || !trace || !n_iter) return fail(c, NMF_E_INVAL, "W, H, trace and n_iter are required");
    if (trace_cap < c->p.max_iter + 1)
        return fail(c, NMF_E_INVAL, "trace_cap = %d < max_iter + 1 = %d", trace_cap, c->p.max_iter + 1);
    nmf_status st = nmf_start(c, W0, H0, 0, c->own);
    if (st != NMF_OK) return st;
    st = nmf_iterate(c, c->p.max_iter, c->own);
    if (st != NMF_OK) return st;
    return nmf_read(c, W, H, 0, trace, trace_cap, n_iter, accepted, beta, c->own);
}

nmf_status nmf_profile(nmf_ctx *c, int32_t iters, void *stream, double *ms)
{
    if (!c) return fail(nullptr, NMF_E_INVAL, "ctx is NULL");
    if (!c->started) return fail(c, NMF_E_STATE, "nmf_profile before a successful nmf_start");
    if (iters < 1 || !ms) return fail(c, NMF_E_INVAL, "need iters >= 1 and ms != NULL");
    if (c->launched + iters > c->p.max_iter)
        return fail(c, NMF_E_INVAL, "only %d iterations left before max_iter",
                    c->p.max_iter - c->launched);
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(c, hipSetDevice(c->device));
    constexpr int NE = NMF_PHASE_COUNT + 1;
    std::vector<hipEvent_t> ev((size_t)iters * NE, nullptr);
    nmf_status st = NMF_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            st = fail(c, NMF_E_DEVICE, "hipEventCreate failed");
            break;
        }
    for (int32_t i = 0; st == NMF_OK && i < iters; ++i) st = enqueue_iteration(c, s, &ev[(size_t)i * NE]);
    if (st == NMF_OK) {
        c->launched += iters;
        double acc[NMF_PHASE_COUNT] = {};
        hipError_t e = hipEventSynchronize(ev.back());
        for (int32_t i = 0; e == hipSuccess && i < iters; ++i)
            for (int ph = 0; ph < NMF_PHASE_COUNT && e == hipSuccess; ++ph) {
                float t = 0.f;
                e = hipEventElapsedTime(&t, ev[(size_t)i * NE + ph], ev[(size_t)i * NE + ph + 1]);
                acc[ph] += t;
            }
        if (e != hipSuccess) st = fail(c, NMF_E_DEVICE, "event timing failed: %s", hipGetErrorString(e));
        for (int ph = 0; ph < NMF_PHASE_COUNT; ++ph) ms[ph] = acc[ph] / iters;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return st;
}

void nmf_destroy(nmf_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    free_all(c);
    delete c;
}

const char *nmf_last_error(const nmf_ctx *c)
{
    if (c) return c->err.c_str();
    return g_err.c_str();
}

}  // extern "C"
