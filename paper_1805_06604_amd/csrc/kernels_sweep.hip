// Set-up and read-out kernels of the factor slots, and the dispatch of the
// sweep kernels over the padded rank (each rank is its own translation unit).
#include "sweep_impl.h"

namespace nmf {

// Explicit instantiations live in sweep_rp{16,32,48,64}.hip.
extern template struct sweep::Launch<16>;
extern template struct sweep::Launch<32>;
extern template struct sweep::Launch<48>;
extern template struct sweep::Launch<64>;

namespace {

// W0 (m x r) -> W slot 0 (m x RP); H0 (r x n) -> H^T slot 0 (n x RP).
__global__ void pack_kernel(int rp, int64_t m, int64_t n, int r,
                            const float *__restrict__ W0, const float *__restrict__ H0,
                            float *__restrict__ Wf, float *__restrict__ Hf,
                            DevState *st)
{
    const int64_t total = (m + n) * rp;
    bool bad = false;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        if (e < m * rp) {
            const int64_t i = e / rp;
            const int k = (int)(e % rp);
            if (k < r) v = W0[i * r + k];
            Wf[e] = v;
        } else {
            const int64_t f = e - m * rp;
            const int64_t j = f / rp;
            const int k = (int)(f % rp);
            if (k < r) v = H0[(int64_t)k * n + j];
            Hf[f] = v;
        }
        if (!(v >= 0.0f) || !isfinite(v)) bad = true;
    }
    if (bad) __hip_atomic_fetch_or(&st->bad_input, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void unpack_kernel(int rp, int64_t m, int64_t n, int r,
                              const float *__restrict__ Wf, const float *__restrict__ Hf,
                              int64_t wstride, int64_t hstride, const DevState *st,
                              float *__restrict__ W, float *__restrict__ H)
{
    const float *Ws = Wf + st->w_acc * wstride;
    const float *Hs = Hf + st->h_acc * hstride;
    const int64_t total = (m + n) * r;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < m * r) {
            const int64_t i = e / r;
            const int k = (int)(e % r);
            W[e] = Ws[i * rp + k];
        } else {
            const int64_t f = e - m * r;
            const int k = (int)(f / n);
            const int64_t j = f % n;
            H[f] = Hs[j * rp + k];
        }
    }
}

}  // namespace

#define NMF_RP_CALL(rp, FN, ...)                                  \
    switch (rp) {                                                 \
    case 16: sweep::Launch<16>::FN(__VA_ARGS__); break;           \
    case 32: sweep::Launch<32>::FN(__VA_ARGS__); break;           \
    case 48: sweep::Launch<48>::FN(__VA_ARGS__); break;           \
    case 64: sweep::Launch<64>::FN(__VA_ARGS__); break;           \
    default: return hipErrorInvalidValue;                         \
    }

hipError_t launch_sweep_h(int rp, int64_t n, int r, int inner_k, bool exact, const Buffers &b,
                          hipStream_t s, hipEvent_t mid)
{
    NMF_RP_CALL(rp, sweep_h, n, r, inner_k, exact, b, s, mid);
    return hipGetLastError();
}

hipError_t launch_sweep_w(int rp, int64_t m, int r, int inner_k, bool exact, const Buffers &b,
                          hipStream_t s, hipEvent_t mid)
{
    NMF_RP_CALL(rp, sweep_w, m, r, inner_k, exact, b, s, mid);
    return hipGetLastError();
}

hipError_t launch_sweep_h_adaptive(int rp, int64_t n, int r, int cap, double delta,
                                   const Buffers &b, hipStream_t s, hipEvent_t mid)
{
    NMF_RP_CALL(rp, sweep_h_adaptive, n, r, cap, delta, b, s, mid);
    return hipGetLastError();
}

hipError_t launch_sweep_w_adaptive(int rp, int64_t m, int r, int cap, double delta,
                                   const Buffers &b, hipStream_t s, hipEvent_t mid)
{
    NMF_RP_CALL(rp, sweep_w_adaptive, m, r, cap, delta, b, s, mid);
    return hipGetLastError();
}

hipError_t launch_invert(int rp, bool w_side, int r, const Buffers &b, hipStream_t s)
{
    NMF_RP_CALL(rp, invert, w_side, r, b, s);
    return hipGetLastError();
}

hipError_t launch_group_exact(int rp, bool w_side, const Group &g, int blocks, hipStream_t s)
{
    NMF_RP_CALL(rp, exact_group, w_side, g, blocks, s);
    return hipGetLastError();
}

hipError_t launch_group_sweep(int rp, bool w_side, const Group &gh, int hblocks, const Group &gf,
                              int fblocks, const Group &gd, int dblocks, hipStream_t s)
{
    NMF_RP_CALL(rp, group, w_side, gh, hblocks, gf, fblocks, gd, dblocks, s);
    return hipGetLastError();
}

hipError_t launch_setup_gram_h(int rp, int64_t n, int r, const Buffers &b, hipStream_t s)
{
    NMF_RP_CALL(rp, setup_h, n, r, b, s);
    return hipGetLastError();
}

hipError_t launch_setup_error(int rp, int64_t m, int r, const Buffers &b, hipStream_t s)
{
    NMF_RP_CALL(rp, setup_err, m, r, b, s);
    return hipGetLastError();
}

hipError_t launch_pack(int rp, int64_t m, int64_t n, int r, const float *W0,
                       const float *H0, const Buffers &b, hipStream_t s)
{
    const int64_t total = (m + n) * rp;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    pack_kernel<<<blocks, 256, 0, s>>>(rp, m, n, r, W0, H0, b.Wf, b.Hf, b.st);
    return hipGetLastError();
}

hipError_t launch_unpack(int rp, int64_t m, int64_t n, int r, const Buffers &b,
                         float *W, float *H, hipStream_t s)
{
    const int64_t total = (m + n) * r;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    unpack_kernel<<<blocks, 256, 0, s>>>(rp, m, n, r, b.Wf, b.Hf, m * rp, n * rp, b.st, W, H);
    return hipGetLastError();
}

}  // namespace nmf
