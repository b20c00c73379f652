// nmf_solve_noalloc: the dense FP32 solve of nmf_create + nmf_solve for
// callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid hipMalloc). Every buffer the solve
// needs besides the caller's inputs and outputs is carved from one
// file-scope device array, `scratch`, of kScratchBytes; every step is
// enqueued on the caller's stream with the same kernels, launch plans and
// arguments as a context with the exact-integer products, so the results are
// those of nmf_solve, bit for bit.
//
// The array lives in the library's code object: each GPU the library runs
// on holds its own copy until the process ends, at its own address, which
// the first call on a device looks up with hipGetSymbolAddress. Host code
// uses only that address (the symbol's name on the host is a stand-in, not a
// device address). All calls on one GPU share the array and it keeps the
// last call's contents, so each call clears what must start at zero; two
// calls that overlap on one GPU (different streams, or threads) race.
#include "host_util.h"
#include "nmf.h"
#include "nmf_internal.h"

#include <algorithm>
#include <mutex>
#include <string>

namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per device).
hipError_t scratch_base(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Zero fill of [p, p + bytes), bytes a multiple of 16 (a kernel, not a
// memset node, so that a captured call replays correctly).
__global__ void zero_kernel(uint4 *p, size_t n16)
{
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = z;
}

// The initial device state, passed by value.
__global__ void init_state_kernel(nmf::DevState *st, nmf::DevState v) { *st = v; }

// After e(0): inputs that nmf_create / nmf_start would have refused on the
// host (a zero or non-finite X, a negative or non-finite W0 or H0, a
// non-finite e(0)) stop the solve before its first iteration and are
// reported in info[0]; info[1] receives the completed iterations at the end.
__global__ void gate_kernel(nmf::DevState *st, int32_t *info)
{
    int32_t status = NMF_OK;
    if (!(st->nx2 > 0.0) || !isfinite(st->nx2) || st->bad_input) status = NMF_E_INVAL;
    else if (!isfinite(st->e0)) status = NMF_E_NUMERIC;
    if (status != NMF_OK) st->done = 1;
    info[0] = status;
    info[1] = 0;
}

__global__ void info_kernel(const nmf::DevState *st, int32_t *info) { info[1] = st->k; }

// The buffers of one solve, carved in order from `base` (sizes only when
// base is null); returns the bytes used.
struct Plan {
    int64_t m = 0, n = 0, m_pad = 0, n_pad = 0, ldx = 0, ldxt = 0;
    int r = 0, rp = 0;
    nmf::Buffers b;
    nmf::ProdArgs pa{}, pc{};
    void *Xs = nullptr, *Xts = nullptr;
    int *zx = nullptr, *zxt = nullptr;
    float *Xf = nullptr, *Xtf = nullptr;
};

size_t carve(Plan &q, const nmf_params &p, char *base, uint8_t *accepted, double *beta)
{
    size_t cur = 0;
    auto take = [&](size_t bytes) -> char * {
        char *ptr = base ? base + cur : nullptr;
        cur += align_up(std::max<size_t>(bytes, 1));
        return ptr;
    };
    const int64_t m = q.m, n = q.n, rp = q.rp;
    const size_t gs = (size_t)nmf::gram_stride(q.rp);
    const int64_t nblk = (std::max(m, n) + nmf::kRowsPerBlock - 1) / nmf::kRowsPerBlock;
    const size_t iters = (size_t)std::max(p.max_iter, 1);
    nmf::Buffers &b = q.b;
    b.Wf = (float *)take(sizeof(float) * nmf::kSlots * m * rp);
    b.Hf = (float *)take(sizeof(float) * nmf::kSlots * n * rp);
    b.GW = (double *)take(sizeof(double) * nmf::kSlots * gs);
    b.GH = (double *)take(sizeof(double) * gs);
    b.A = (double *)take(sizeof(double) * q.pa.nsplit * q.m_pad * rp);
    b.Ct = (double *)take(sizeof(double) * q.pc.nsplit * q.n_pad * rp);
    b.part_g = (double *)take(sizeof(double) * nblk * nmf::sweep_record(q.rp));
    b.part_d = (double *)take(sizeof(double) * 1024);
    b.st = (nmf::DevState *)take(sizeof(nmf::DevState));
    b.accepted = accepted ? accepted : (uint8_t *)take(iters);
    b.beta_used = beta ? beta : (double *)take(sizeof(double) * iters);
    b.beta_star = (double *)take(sizeof(double) * (iters + 1));
    b.fsl = (signed char *)take((size_t)std::max(q.ldx, q.ldxt) * 4 * rp);
    b.texp = (int *)take(sizeof(int) * rp);
    q.Xs = take((size_t)q.m_pad * q.ldx * 4);
    q.Xts = take((size_t)q.n_pad * q.ldxt * 4);
    q.zx = (int *)take(sizeof(int) * q.m_pad);
    q.zxt = (int *)take(sizeof(int) * q.n_pad);
    q.Xf = (float *)take(sizeof(float) * q.m_pad * q.ldx);
    q.Xtf = (float *)take(sizeof(float) * q.n_pad * q.ldxt);
    b.nsplit_a = q.pa.nsplit;
    b.nsplit_c = q.pc.nsplit;
    b.m_pad = q.m_pad;
    b.n_pad = q.n_pad;
    return cur;
}

nmf_status err(nmf_status st, const std::string &msg)
{
    nmf::host::set_error(msg);
    return st;
}

#define NHIP(call)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return err(NMF_E_DEVICE, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

extern "C" nmf_status nmf_solve_noalloc(const float *X, int64_t m, int64_t n,
                                        const nmf_params *p, const float *W0, const float *H0,
                                        float *W, float *H, double *trace, uint8_t *accepted,
                                        double *beta, int32_t *info, void *stream)
{
    nmf_status st = nmf::host::check_params(p);
    if (st != NMF_OK) return st;
    if (m < 1 || n < 1) return err(NMF_E_INVAL, "m and n must be >= 1");
    if (!X || !W0 || !H0 || !W || !H || !trace || !info)
        return err(NMF_E_INVAL, "X, W0, H0, W, H, trace and info must not be NULL");
    if (p->x_dtype != NMF_X_F32 || (p->prod != NMF_PROD_AUTO && p->prod != NMF_PROD_MFMA_EXACT))
        return err(NMF_E_UNSUPPORTED, "nmf_solve_noalloc takes FP32 X with the exact-integer products");
    if (p->inner_rule != NMF_INNER_FIXED)
        return err(NMF_E_UNSUPPORTED, "nmf_solve_noalloc runs the fixed inner rule");
    if (p->flags & ~(NMF_FLAG_BETABAR_LAST_ACCEPTED | NMF_FLAG_CMP_LAST_ACCEPTED))
        return err(NMF_E_UNSUPPORTED, "nmf_solve_noalloc takes the reading flags only");
    Plan q;
    q.m = m;
    q.n = n;
    q.r = p->r;
    q.rp = nmf::host::round_rank(p->r);
    q.m_pad = nmf::host::round_up(m, 128);
    q.n_pad = nmf::host::round_up(n, 128);
    q.ldx = nmf::host::round_up(n, 64);
    q.ldxt = nmf::host::round_up(m, 64);
    nmf::host::plan_product(q.pa, nmf::PK_MFMA_I8, m, q.m_pad, n, q.ldx, 0);
    nmf::host::plan_product(q.pc, nmf::PK_MFMA_I8, n, q.n_pad, m, q.ldxt, 0);
    const size_t need = carve(q, *p, nullptr, accepted, beta);
    if (need > kScratchBytes)
        return err(NMF_E_NOMEM, "the solve needs " + std::to_string(need) +
                                    " bytes of scratch; nmf_solve_noalloc holds " +
                                    std::to_string(kScratchBytes));
    int dev = 0;
    NHIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return err(NMF_E_UNSUPPORTED, "device index out of range");
    void *base = nullptr;
    NHIP(scratch_base(dev, &base));
    carve(q, *p, static_cast<char *>(base), accepted, beta);
    nmf::Buffers &b = q.b;
    b.trace = trace;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int rp = q.rp, r = q.r;

    // Everything carved starts at zero (padding of X, of the factor slots
    // and of the products).
    const size_t n16 = need / 16;
    zero_kernel<<<(unsigned)std::min<size_t>((n16 + 255) / 256, 8192), 256, 0, s>>>(
        static_cast<uint4 *>(base), n16);
    NHIP(hipGetLastError());
    // The state nmf_start sets; ||X||^2 goes into it on the device.
    nmf::DevState h{};
    h.hp = p->hp;
    nmf::plan_slots(0, 0, &h.w_n, &h.w_yn);
    nmf::plan_slots(0, 0, &h.h_n, &h.h_yn);
    h.max_iter = p->max_iter;
    h.flags = p->flags;
    h.r = r;
    h.beta = p->beta0;
    h.betabar = 1.0;
    h.beta_prev = p->beta0;
    h.beta_acc = p->beta0;
    h.tol = p->tol;
    h.gamma = p->gamma;
    h.gamma_bar = p->gamma_bar;
    h.eta = p->eta;
    init_state_kernel<<<1, 1, 0, s>>>(b.st, h);
    NHIP(hipGetLastError());
    // X as a context prepares it: padded FP32 copies of X and X^T, ||X||^2
    // from the padded X, then the int8 slices and row exponents of both.
    NHIP(nmf::launch_convert_x(X, m, n, NMF_X_F32, q.Xf, q.ldx, q.Xtf, q.ldxt, s));
    NHIP(nmf::launch_sumsq_typed(q.Xf, NMF_X_F32, q.m_pad * q.ldx, b.part_d, 1024, &b.st->nx2, s));
    NHIP(nmf::i8::slice_rows(q.Xf, NMF_X_F32, m, n, q.ldx, q.ldx, q.Xs, q.zx, s));
    NHIP(nmf::i8::slice_rows(q.Xtf, NMF_X_F32, n, m, q.ldxt, q.ldxt, q.Xts, q.zxt, s));
    auto fill = [&](nmf::ProdArgs &a, bool w_side) {
        a.st = b.st;
        a.Fsl = b.fsl;
        a.texp = b.texp;
        a.csr = nullptr;
        if (w_side) {   // A = X H_w^T
            a.Z = q.Xs;
            a.F_base = b.Hf;
            a.slot_stride = n * rp;
            a.sel = nmf::SEL_H_W;
            a.zexp = q.zx;
            a.gram_base = b.GH;
            a.gram_slot_stride = 0;
            a.Y = b.A;
        } else {        // C^T = X^T W_y
            a.Z = q.Xts;
            a.F_base = b.Wf;
            a.slot_stride = m * rp;
            a.sel = nmf::SEL_W_Y;
            a.zexp = q.zxt;
            a.gram_base = b.GW;
            a.gram_slot_stride = nmf::gram_stride(rp);
            a.Y = b.Ct;
        }
    };
    fill(q.pa, true);
    fill(q.pc, false);
    // Algorithm 2, first step: W0, H0 into slot 0 and e(0).
    NHIP(nmf::launch_pack(rp, m, n, r, W0, H0, b, s));
    NHIP(nmf::launch_setup_gram_h(rp, n, r, b, s));
    nmf::ProdArgs a0 = q.pa;
    a0.sel = nmf::SEL_SLOT0;
    NHIP(nmf::launch_product(rp, NMF_X_F32, nmf::PK_MFMA_I8, a0, s));
    NHIP(nmf::launch_setup_error(rp, m, r, b, s));
    gate_kernel<<<1, 1, 0, s>>>(b.st, info);
    NHIP(hipGetLastError());
    // The outer iterations; past max_iter or the tol stop every kernel
    // returns at entry.
    for (int32_t it = 0; it < p->max_iter; ++it) {
        NHIP(nmf::launch_product(rp, NMF_X_F32, nmf::PK_MFMA_I8, q.pc, s));
        NHIP(nmf::launch_sweep_h(rp, n, r, p->inner_k, false, b, s));
        NHIP(nmf::launch_product(rp, NMF_X_F32, nmf::PK_MFMA_I8, q.pa, s));
        NHIP(nmf::launch_sweep_w(rp, m, r, p->inner_k, false, b, s));
    }
    NHIP(nmf::launch_unpack(rp, m, n, r, b, W, H, s));
    info_kernel<<<1, 1, 0, s>>>(b.st, info);
    NHIP(hipGetLastError());
    return NMF_OK;
}
