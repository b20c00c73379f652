// Continuous batching of many independent small E-A-HALS problems on one GPU
// (the batched-solve entry points of include/nmf.h).
//
// Every admitted problem lives in one device arena (first-fit, 256-byte
// aligned blocks) with the same buffers as a single-problem context. A batch
// iteration runs one outer iteration of Algorithm 2 for every active problem:
// per padded rank, eleven grouped launches (factor slicing, Xᵀ W_y, the
// exact NNLS solves of the E-ANLS problems, H sweeps, H finish, factor
// slicing, X H_wᵀ, exact solves, W sweeps, W finish, the decision), each covering the work blocks of
// all problems of that rank with a fixed grid, so that small problems share
// the chip instead of each paying its own launch latency. The launches of a
// rank read their tables from device memory, so one batch iteration (and
// check_every of them) is captured once as a graph per rank and replayed. A problem that stopped
// (its device state says done) returns at the entry of every kernel until
// the host retires it at the next completion check.
#include "host_util.h"
#include "nmf.h"
#include "nmf_internal.h"
#include "sweep_impl.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using nmf::Buffers;
using nmf::DevState;
using nmf::Group;
using nmf::ProdArgs;

namespace {

constexpr size_t kAlign = 256;
constexpr int kClasses = 4;          // padded ranks 16, 32, 48, 64
constexpr int kKinds = 11;           // grouped kernels of one iteration (8, the exact
                                     // NNLS solves of E-ANLS problems, H and W, and
                                     // the decision after the W finish)
// Split-K of a problem's products: K is split only while the problem has
// fewer than 2 row blocks. The grouped kernels draw their parallelism from the
// many problems of a class; longer K ranges per work block keep each block's
// load pipeline full (on a saturated stream of m, n in 64..2048 this gave
// 1727 solves/s against 1198 with up to 64 blocks per product).
constexpr int64_t kBatchTargetWG = 2;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing of free neighbours.
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length

    void init(char *b, size_t n)
    {
        base = b;
        size = n;
        free_.clear();
        free_[0] = n;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Prob {
    int64_t ticket = 0;
    nmf_params p{};
    int64_t m = 0, n = 0;
    int r = 0, rp = 0;
    int64_t m_pad = 0, n_pad = 0, ldx = 0, ldxt = 0;
    std::unique_ptr<float[]> X;        // inputs until admitted (pageable), or
    float *Xpin = nullptr;             // in the batch's pinned pool at pin_off
    size_t pin_off = 0;
    const float *xsrc() const { return Xpin ? Xpin : X.get(); }
    std::vector<float> W0, H0;
    size_t off = 0, bytes = 0;         // persistent block
    size_t toff = 0, tbytes = 0;       // admission temporaries
    bool has_tmp = false;
    Buffers b;
    ProdArgs pa{}, pc{};
    void *Xs = nullptr, *Xts = nullptr;
    int *zx = nullptr, *zxt = nullptr;
    float *src = nullptr, *Xf = nullptr, *Xtf = nullptr;
    DevState hs{};                     // initial device state (outlives its upload)
    bool retired = false;
    std::vector<float> W, H;
    std::vector<double> trace, beta;
    std::vector<uint8_t> accepted;
    int32_t n_iter = 0;
};

// Persistent buffers of a problem, laid out from `base` (sizes only when
// base is null); returns the bytes used.
size_t layout(Prob &q, char *base)
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
    Buffers &b = q.b;
    b.Wf = (float *)take(sizeof(float) * nmf::kSlots * m * rp);
    b.Hf = (float *)take(sizeof(float) * nmf::kSlots * n * rp);
    b.GW = (double *)take(sizeof(double) * nmf::kSlots * gs);
    b.GH = (double *)take(sizeof(double) * gs);
    b.A = (double *)take(sizeof(double) * q.pa.nsplit * q.m_pad * rp);
    b.Ct = (double *)take(sizeof(double) * q.pc.nsplit * q.n_pad * rp);
    b.part_g = (double *)take(sizeof(double) * nblk * nmf::sweep_record(q.rp));
    b.part_d = (double *)take(sizeof(double) * 1024);
    b.st = (DevState *)take(sizeof(DevState));
    b.beta_star = (double *)take(sizeof(double) * (q.p.max_iter + 1));
    // The results, contiguous so that one copy reads them back: W and H
    // (unpacked into the staging area), trace, beta used, accepted flags.
    b.stage = (float *)take(sizeof(float) * (m + n) * q.r);
    b.trace = (double *)take(sizeof(double) * (q.p.max_iter + 1));
    b.beta_used = (double *)take(sizeof(double) * (q.p.max_iter + 1));
    b.accepted = (uint8_t *)take((size_t)q.p.max_iter + 1);
    b.fsl = (signed char *)take((size_t)std::max(q.ldx, q.ldxt) * 4 * rp);
    b.texp = (int *)take(sizeof(int) * rp);
    q.Xs = take((size_t)q.m_pad * q.ldx * 4);
    q.Xts = take((size_t)q.n_pad * q.ldxt * 4);
    q.zx = (int *)take(sizeof(int) * q.m_pad);
    q.zxt = (int *)take(sizeof(int) * q.n_pad);
    b.nsplit_a = q.pa.nsplit;
    b.nsplit_c = q.pc.nsplit;
    b.m_pad = q.m_pad;
    b.n_pad = q.n_pad;
    return cur;
}

// Admission temporaries: the FP32 source and the padded X and X^T that the
// slicing reads.
size_t layout_tmp(Prob &q, char *base)
{
    size_t cur = 0;
    auto take = [&](size_t bytes) -> char * {
        char *ptr = base ? base + cur : nullptr;
        cur += align_up(std::max<size_t>(bytes, 1));
        return ptr;
    };
    q.src = (float *)take(sizeof(float) * q.m * q.n);
    q.Xf = (float *)take(sizeof(float) * q.m_pad * q.ldx);
    q.Xtf = (float *)take(sizeof(float) * q.n_pad * q.ldxt);
    return cur;
}

// One record of a grouped launch per problem: the arguments of all eight
// kernels of an iteration.
struct Entry {
    ProdArgs pc, pa;
    nmf::sweep::HalsArgs hh, hw;
    nmf::sweep::FinArgs fh, fw;
};

__global__ void gather_state(const DevState *const *st, int np, int32_t *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) {
        out[2 * i] = st[i]->done;
        out[2 * i + 1] = st[i]->k;
    }
}

int rank_class(int rp) { return rp / 16 - 1; }

}  // namespace

struct nmf_batch {
    nmf_batch_params bp{};
    int device = 0;
    hipStream_t s = nullptr;             // admission, tables, read-back
    hipStream_t cs[kClasses] = {};       // batch iterations, one stream per padded rank
    char *pool = nullptr;
    Arena arena;
    std::deque<Prob *> queue;
    std::vector<Prob *> pending;         // admitted (set-up enqueued), not yet in the tables
    std::vector<Prob *> active;
    std::map<int64_t, std::unique_ptr<Prob>> all;
    int64_t next_ticket = 1;
    int32_t retired_unread = 0;
    // Guards what submissions and results share with the stepping thread:
    // queue, all, next_ticket, retired_unread, pin_arena and the retired
    // flags and results of the problems.
    std::mutex mu;
    // grouped-launch tables (device), rebuilt when the active set changes
    bool dirty = true;
    Entry *d_entries = nullptr;          // kClasses x max_active
    int *d_prefix = nullptr;             // kClasses x kKinds x (max_active + 1)
    int *d_np = nullptr;                 // kClasses: problems of each padded rank
    char *pin = nullptr;                 // pinned host pool for submitted X
    Arena pin_arena;
    // One batch iteration of a padded rank, and check_every of them, captured
    // once as graphs on the class streams (their launches read the tables
    // above, so they stay valid while the active set changes).
    hipGraphExec_t exec_one[kClasses] = {};
    hipGraphExec_t exec_chunk[kClasses] = {};
    bool need_exact[kClasses] = {};      // a member of the class runs exact NNLS solves
    bool cap_exact[kClasses] = {};       // the class's graphs hold the exact launches
    const DevState **d_states = nullptr; // max_active
    int32_t *d_flags = nullptr;          // 2 x max_active
    int32_t *h_flags = nullptr;          // pinned
    char *h_res = nullptr;               // pinned read-back area of retiring problems
    size_t h_res_cap = 0;
    std::vector<Prob *> members[kClasses];
    bool inflight = false;               // a chunk left running by the last step call
};

namespace {

nmf_status berr(nmf_status st, const std::string &msg)
{
    nmf::host::set_error(msg);
    return st;
}

#define BHIP(call)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return berr(NMF_E_DEVICE, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    } while (0)

// Places q in the arena and enqueues its set-up (upload, slicing, packing,
// e(0)); false if it does not fit now.
bool admit(nmf_batch *B, Prob &q, nmf_status *err)
{
    *err = NMF_OK;
    const size_t need = layout(q, nullptr), tneed = layout_tmp(q, nullptr);
    size_t off = 0, toff = 0;
    if (!B->arena.alloc(need, &off)) return false;
    if (!B->arena.alloc(tneed, &toff)) {
        B->arena.release(off, need);
        return false;
    }
    q.off = off;
    q.bytes = need;
    q.toff = toff;
    q.tbytes = tneed;
    q.has_tmp = true;
    layout(q, B->arena.base + off);
    layout_tmp(q, B->arena.base + toff);
    hipStream_t s = B->s;
    const int rp = q.rp;
    Buffers &b = q.b;
    // DevState as nmf_start sets it; ||X||^2 is written into it on the device.
    DevState &h = q.hs;
    h = DevState{};
    h.hp = q.p.hp;
    nmf::plan_slots(0, 0, &h.w_n, &h.w_yn);
    nmf::plan_slots(0, 0, &h.h_n, &h.h_yn);
    h.max_iter = q.p.max_iter;
    h.flags = q.p.flags;
    h.r = q.r;
    h.beta = q.p.beta0;
    h.betabar = 1.0;
    h.beta_prev = q.p.beta0;
    h.beta_acc = q.p.beta0;
    h.tol = q.p.tol;
    h.gamma = q.p.gamma;
    h.gamma_bar = q.p.gamma_bar;
    h.eta = q.p.eta;
    hipError_t e = hipMemsetAsync(B->arena.base + off, 0, need, s);
    if (e == hipSuccess) e = hipMemsetAsync(B->arena.base + toff, 0, tneed, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b.st, &h, sizeof(h), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(q.src, q.xsrc(), sizeof(float) * q.m * q.n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.stage, q.W0.data(), sizeof(float) * q.m * q.r, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.stage + q.m * q.r, q.H0.data(), sizeof(float) * q.r * q.n,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = nmf::launch_convert_x(q.src, q.m, q.n, NMF_X_F32, q.Xf, q.ldx, q.Xtf, q.ldxt, s);
    if (e == hipSuccess) e = nmf::launch_sumsq(q.src, q.m * q.n, b.part_d, 256, &b.st->nx2, s);
    if (e == hipSuccess) e = nmf::i8::slice_rows(q.Xf, NMF_X_F32, q.m, q.n, q.ldx, q.ldx, q.Xs, q.zx, s);
    if (e == hipSuccess)
        e = nmf::i8::slice_rows(q.Xtf, NMF_X_F32, q.n, q.m, q.ldxt, q.ldxt, q.Xts, q.zxt, s);
    if (e == hipSuccess) e = nmf::launch_pack(rp, q.m, q.n, q.r, b.stage, b.stage + q.m * q.r, b, s);
    // Products of this problem.
    auto fill = [&](ProdArgs &a, bool w_side) {
        a.st = b.st;
        a.Fsl = b.fsl;
        a.texp = b.texp;
        a.csr = nullptr;
        if (w_side) {   // A = X H_w^T
            a.Z = q.Xs;
            a.F_base = b.Hf;
            a.slot_stride = q.n * rp;
            a.sel = nmf::SEL_H_W;
            a.zexp = q.zx;
            a.gram_base = b.GH;
            a.gram_slot_stride = 0;
            a.Y = b.A;
        } else {        // C^T = X^T W_y
            a.Z = q.Xts;
            a.F_base = b.Wf;
            a.slot_stride = q.m * rp;
            a.sel = nmf::SEL_W_Y;
            a.zexp = q.zxt;
            a.gram_base = b.GW;
            a.gram_slot_stride = nmf::gram_stride(rp);
            a.Y = b.Ct;
        }
    };
    fill(q.pa, true);
    fill(q.pc, false);
    if (e == hipSuccess) e = nmf::launch_setup_gram_h(rp, q.n, q.r, b, s);
    ProdArgs a0 = q.pa;
    a0.sel = nmf::SEL_SLOT0;
    if (e == hipSuccess) e = nmf::launch_product(rp, NMF_X_F32, nmf::PK_MFMA_I8, a0, s);
    if (e == hipSuccess) e = nmf::launch_setup_error(rp, q.m, q.r, b, s);
    if (e != hipSuccess) {
        *err = berr(NMF_E_DEVICE, std::string("batch admission failed: ") + hipGetErrorString(e));
        return false;
    }
    return true;
}

// Rebuilds the grouped-launch tables of the active set (the stream is idle).
nmf_status rebuild(nmf_batch *B)
{
    const int cap = B->bp.max_active;
    std::vector<Entry> ent((size_t)kClasses * cap);
    std::vector<int> pre((size_t)kClasses * kKinds * (cap + 1), 0);
    std::vector<const DevState *> sts(B->active.size());
    for (auto &mem : B->members) mem.clear();
    for (size_t i = 0; i < B->active.size(); ++i) {
        Prob *q = B->active[i];
        B->members[rank_class(q->rp)].push_back(q);
        sts[i] = q->b.st;
    }
    for (int c = 0; c < kClasses; ++c) {
        const int rp = 16 * (c + 1);
        auto &mem = B->members[c];
        B->need_exact[c] = false;
        for (size_t i = 0; i < mem.size(); ++i) {
            Prob &q = *mem[i];
            Entry &E = ent[(size_t)c * cap + i];
            E.pc = q.pc;
            E.pa = q.pa;
            E.hh = nmf::sweep::hals_args(rp, q.n, q.r, q.p.inner_k, q.b, false);
            E.hw = nmf::sweep::hals_args(rp, q.m, q.r, q.p.inner_k, q.b, true);
            const bool exact = q.p.inner_rule == NMF_INNER_EXACT;
            B->need_exact[c] = B->need_exact[c] || exact;
            if (exact) {        // the exact solve fills the new slot; no sweeps after it
                E.hh.K = E.hw.K = 0;
                E.hh.src_mode = E.hw.src_mode = 1;
            }
            E.fh = nmf::sweep::fin_args(rp, q.n, q.r, q.b, false);
            E.fw = nmf::sweep::fin_args(rp, q.m, q.r, q.b, true);
            const int nb[kKinds] = {(int)(q.pc.ld / 64), (int)(q.pc.rows_pad / 128 * q.pc.nsplit),
                                    nmf::sweep::hals_blocks(q.n), nmf::sweep::fin_blocks(rp, 1),
                                    (int)(q.pa.ld / 64), (int)(q.pa.rows_pad / 128 * q.pa.nsplit),
                                    nmf::sweep::hals_blocks(q.m), nmf::sweep::fin_blocks(rp, 2),
                                    exact ? nmf::sweep::exact_blocks(q.n) : 0,
                                    exact ? nmf::sweep::exact_blocks(q.m) : 0, 1};
            for (int k = 0; k < kKinds; ++k) {
                int *P = &pre[((size_t)c * kKinds + k) * (cap + 1)];
                P[i + 1] = P[i] + nb[k];
            }
        }
    }
    // On the batch stream, complete before any grouped launch reads the tables
    // (the class streams do not order with the legacy default stream).
    BHIP(hipMemcpyAsync(B->d_entries, ent.data(), sizeof(Entry) * ent.size(), hipMemcpyHostToDevice,
                        B->s));
    BHIP(hipMemcpyAsync(B->d_prefix, pre.data(), sizeof(int) * pre.size(), hipMemcpyHostToDevice, B->s));
    int np[kClasses];
    for (int c = 0; c < kClasses; ++c) np[c] = (int)B->members[c].size();
    BHIP(hipMemcpyAsync(B->d_np, np, sizeof(np), hipMemcpyHostToDevice, B->s));
    if (!sts.empty())
        BHIP(hipMemcpyAsync(B->d_states, sts.data(), sizeof(DevState *) * sts.size(),
                            hipMemcpyHostToDevice, B->s));
    BHIP(hipStreamSynchronize(B->s));
    // A class's graphs hold the exact launches only while a member needs
    // them; they are captured again when that changes (the class streams are
    // idle here).
    for (int c = 0; c < kClasses; ++c) {
        if (!B->exec_one[c] || B->cap_exact[c] == B->need_exact[c]) continue;
        BHIP(hipGraphExecDestroy(B->exec_one[c]));
        B->exec_one[c] = nullptr;
        if (B->exec_chunk[c]) BHIP(hipGraphExecDestroy(B->exec_chunk[c]));
        B->exec_chunk[c] = nullptr;
    }
    B->dirty = false;
    return NMF_OK;
}

Group group_of(nmf_batch *B, int c, int kind, size_t member_offset)
{
    Group g;
    g.base = reinterpret_cast<const char *>(B->d_entries + (size_t)c * B->bp.max_active) + member_offset;
    g.stride = sizeof(Entry);
    g.prefix = B->d_prefix + ((size_t)c * kKinds + kind) * (B->bp.max_active + 1);
    g.np = B->d_np + c;
    return g;
}

// Fixed grids of the grouped kernels (workgroups walk the work blocks with a
// grid stride): about one resident round of the chip per kernel kind.
constexpr int kGrid[kKinds] = {1024, 256, 512, 1024, 1024, 256, 512, 1024, 512, 512, 512};

// One batch iteration of padded-rank class c on stream cs: both products,
// the exact solves (when a member of the class is an E-ANLS problem) and both
// sweep steps.
nmf_status enqueue_class_iteration(nmf_batch *B, int c, hipStream_t cs)
{
    const int rp = 16 * (c + 1);
    BHIP(nmf::i8::launch_group(rp, group_of(B, c, 0, offsetof(Entry, pc)), kGrid[0],
                               group_of(B, c, 1, offsetof(Entry, pc)), kGrid[1], cs));
    if (B->need_exact[c])
        BHIP(nmf::launch_group_exact(rp, false, group_of(B, c, 8, offsetof(Entry, hh)), kGrid[8], cs));
    BHIP(nmf::launch_group_sweep(rp, false, group_of(B, c, 2, offsetof(Entry, hh)), kGrid[2],
                                 group_of(B, c, 3, offsetof(Entry, fh)), kGrid[3], Group{}, 0, cs));
    BHIP(nmf::i8::launch_group(rp, group_of(B, c, 4, offsetof(Entry, pa)), kGrid[4],
                               group_of(B, c, 5, offsetof(Entry, pa)), kGrid[5], cs));
    if (B->need_exact[c])
        BHIP(nmf::launch_group_exact(rp, true, group_of(B, c, 9, offsetof(Entry, hw)), kGrid[9], cs));
    BHIP(nmf::launch_group_sweep(rp, true, group_of(B, c, 6, offsetof(Entry, hw)), kGrid[6],
                                 group_of(B, c, 7, offsetof(Entry, fw)), kGrid[7],
                                 group_of(B, c, 10, offsetof(Entry, fw)), kGrid[10], cs));
    return NMF_OK;
}

// Captures `iters` batch iterations of class c into an executable graph.
nmf_status capture_class(nmf_batch *B, int c, int iters, hipGraphExec_t *out)
{
    hipStream_t cs = B->cs[c];
    BHIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    nmf_status st = NMF_OK;
    for (int it = 0; it < iters && st == NMF_OK; ++it) st = enqueue_class_iteration(B, c, cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (st != NMF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return berr(NMF_E_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess)
        return berr(NMF_E_DEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(ei));
    return NMF_OK;
}

// Runs `iters` batch iterations of every non-empty class on its stream, as
// graph launches (check_every iterations per launch, single ones for the rest).
nmf_status run_iterations(nmf_batch *B, int iters)
{
    for (int c = 0; c < kClasses; ++c) {
        if (B->members[c].empty()) continue;
        if (!B->exec_one[c]) {
            B->cap_exact[c] = B->need_exact[c];
            nmf_status st = capture_class(B, c, 1, &B->exec_one[c]);
            if (st == NMF_OK && B->bp.check_every > 1)
                st = capture_class(B, c, B->bp.check_every, &B->exec_chunk[c]);
            if (st != NMF_OK) return st;
        }
        int left = iters;
        for (; B->exec_chunk[c] && left >= B->bp.check_every; left -= B->bp.check_every)
            BHIP(hipGraphLaunch(B->exec_chunk[c], B->cs[c]));
        for (; left > 0; --left) BHIP(hipGraphLaunch(B->exec_one[c], B->cs[c]));
    }
    return NMF_OK;
}

// Reads back the problems whose device state says done and frees their
// memory. The stream is idle.
nmf_status retire(nmf_batch *B)
{
    const int np = (int)B->active.size();
    for (int c = 0; c < kClasses; ++c) BHIP(hipStreamSynchronize(B->cs[c]));
    if (np == 0) return NMF_OK;
    gather_state<<<(np + 255) / 256, 256, 0, B->s>>>(B->d_states, np, B->d_flags);
    BHIP(hipGetLastError());
    BHIP(hipMemcpyAsync(B->h_flags, B->d_flags, sizeof(int32_t) * 2 * np, hipMemcpyDeviceToHost, B->s));
    BHIP(hipStreamSynchronize(B->s));
    // Every finished problem: W and H unpacked into its staging area, then
    // one copy of its contiguous results span into the pinned read-back
    // area; one wait for all of them; then the host copies.
    std::vector<Prob *> keep, done;
    std::vector<size_t> at;
    size_t total = 0;
    auto span = [](const Prob *q) {
        return (size_t)(reinterpret_cast<const char *>(q->b.accepted) + q->p.max_iter + 1 -
                        reinterpret_cast<const char *>(q->b.stage));
    };
    for (int i = 0; i < np; ++i) {
        Prob *q = B->active[i];
        if (!B->h_flags[2 * i]) {
            keep.push_back(q);
            continue;
        }
        q->n_iter = B->h_flags[2 * i + 1];
        done.push_back(q);
        at.push_back(total);
        total += (span(q) + 255) / 256 * 256;
    }
    if (done.empty()) return NMF_OK;
    if (total > B->h_res_cap) {      // grows; no copy into it is in flight here
        const size_t cap = std::max(total, 2 * B->h_res_cap + (size_t(1) << 20));
        if (B->h_res) BHIP(hipHostFree(B->h_res));
        B->h_res = nullptr;
        B->h_res_cap = 0;
        BHIP(hipHostMalloc(reinterpret_cast<void **>(&B->h_res), cap));
        B->h_res_cap = cap;
    }
    for (size_t j = 0; j < done.size(); ++j) {
        Prob *q = done[j];
        BHIP(nmf::launch_unpack(q->rp, q->m, q->n, q->r, q->b, q->b.stage, q->b.stage + q->m * q->r, B->s));
        BHIP(hipMemcpyAsync(B->h_res + at[j], q->b.stage, span(q), hipMemcpyDeviceToHost, B->s));
    }
    BHIP(hipStreamSynchronize(B->s));
    for (size_t j = 0; j < done.size(); ++j) {
        Prob *q = done[j];
        const char *h = B->h_res + at[j];
        auto host = [&](const void *dev) {
            return h + (reinterpret_cast<const char *>(dev) - reinterpret_cast<const char *>(q->b.stage));
        };
        const int32_t k = q->n_iter;
        q->W.resize((size_t)q->m * q->r);
        q->H.resize((size_t)q->r * q->n);
        q->trace.resize((size_t)k + 1);
        q->accepted.resize((size_t)k);
        q->beta.resize((size_t)k);
        std::memcpy(q->W.data(), h, sizeof(float) * q->W.size());
        std::memcpy(q->H.data(), h + sizeof(float) * q->W.size(), sizeof(float) * q->H.size());
        std::memcpy(q->trace.data(), host(q->b.trace), sizeof(double) * q->trace.size());
        std::memcpy(q->beta.data(), host(q->b.beta_used), sizeof(double) * (size_t)k);
        std::memcpy(q->accepted.data(), host(q->b.accepted), (size_t)k);
        B->arena.release(q->off, q->bytes);
        std::lock_guard<std::mutex> lk(B->mu);
        q->retired = true;
        ++B->retired_unread;
        B->dirty = true;
    }
    B->active.swap(keep);
    return NMF_OK;
}

// Admits queued problems in submission order while the arena and max_active
// allow, enqueueing their set-up on the batch stream (see admit).
nmf_status admit_queued(nmf_batch *B)
{
    std::lock_guard<std::mutex> lk(B->mu);
    while (!B->queue.empty() &&
           (int)(B->active.size() + B->pending.size()) < B->bp.max_active) {
        Prob *q = B->queue.front();
        nmf_status err;
        if (!admit(B, *q, &err)) {
            if (err != NMF_OK) return err;
            break;
        }
        B->queue.pop_front();
        B->pending.push_back(q);
    }
    return NMF_OK;
}

// Waits for the set-up of the pending problems, frees their temporaries and
// host copies, and moves them to the active set (the tables then need a
// rebuild).
nmf_status finish_admissions(nmf_batch *B)
{
    BHIP(hipStreamSynchronize(B->s));
    for (Prob *q : B->pending) {
        B->arena.release(q->toff, q->tbytes);
        q->has_tmp = false;
        q->X.reset();
        if (q->Xpin) {
            std::lock_guard<std::mutex> lk(B->mu);
            B->pin_arena.release(q->pin_off, sizeof(float) * q->m * q->n);
            q->Xpin = nullptr;
        }
        std::vector<float>().swap(q->W0);
        std::vector<float>().swap(q->H0);
        B->active.push_back(q);
    }
    B->pending.clear();
    B->dirty = true;
    return NMF_OK;
}

// Finishes the pending admissions, refreshes the tables, enqueues `chunk`
// batch iterations of every active problem, then the set-up of newly
// admitted problems on the batch stream beside them (uploads, slicing, e(0)).
// *ran is false when no problem is active.
nmf_status launch_chunk(nmf_batch *B, int chunk, bool *ran)
{
    *ran = false;
    if (B->active.empty() && B->pending.empty()) {
        nmf_status st = admit_queued(B);
        if (st != NMF_OK) return st;
    }
    if (!B->pending.empty()) {
        nmf_status st = finish_admissions(B);
        if (st != NMF_OK) return st;
    }
    if (B->active.empty()) return NMF_OK;
    if (B->dirty) {
        nmf_status st = rebuild(B);
        if (st != NMF_OK) return st;
    }
    nmf_status st = run_iterations(B, chunk);
    if (st != NMF_OK) return st;
    st = admit_queued(B);
    if (st != NMF_OK) return st;
    *ran = true;
    return NMF_OK;
}

}  // namespace

extern "C" {

nmf_status nmf_batch_create(const nmf_batch_params *bp, nmf_batch **out)
{
    if (!out) return berr(NMF_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!bp) return berr(NMF_E_INVAL, "params is NULL");
    if (bp->hbm_budget <= 0) return berr(NMF_E_INVAL, "hbm_budget must be > 0");
    if (bp->max_active < 1 || bp->max_active > 4096)
        return berr(NMF_E_INVAL, "max_active must lie in 1..4096");
    if (bp->check_every < 1) return berr(NMF_E_INVAL, "check_every must be >= 1");
    nmf_batch *B = new (std::nothrow) nmf_batch();
    if (!B) return berr(NMF_E_NOMEM, "host allocation failed");
    B->bp = *bp;
    auto cleanup = [&](nmf_status st) {
        nmf_batch_destroy(B);
        return st;
    };
    // The class streams are created first: the runtime maps streams onto a
    // few hardware queues (4 by default) and, once they are all taken, lets
    // new streams share the least used one. Created first, the classes take
    // queues of their own and the batch stream (admissions, read-back) is the
    // one that shares. Created after the batch stream, the saturated rate
    // varied by 30% from one batch object to the next in a process.
    if (hipGetDevice(&B->device) != hipSuccess)
        return cleanup(berr(NMF_E_DEVICE, "no usable HIP device"));
    for (int c = 0; c < kClasses; ++c)
        if (hipStreamCreateWithFlags(&B->cs[c], hipStreamNonBlocking) != hipSuccess)
            return cleanup(berr(NMF_E_DEVICE, "stream creation failed"));
    if (hipStreamCreateWithFlags(&B->s, hipStreamNonBlocking) != hipSuccess)
        return cleanup(berr(NMF_E_DEVICE, "stream creation failed"));
    if (hipMalloc(&B->pool, (size_t)bp->hbm_budget) != hipSuccess)
        return cleanup(berr(NMF_E_NOMEM, "the batch arena does not fit on the device"));
    B->arena.init(B->pool, (size_t)bp->hbm_budget);
    // Pinned staging of submitted X (1 GiB at most; without it, X is kept in
    // pageable memory).
    const size_t pin_bytes = std::min<size_t>((size_t)bp->hbm_budget, size_t(1) << 30);
    if (hipHostMalloc(reinterpret_cast<void **>(&B->pin), pin_bytes) == hipSuccess)
        B->pin_arena.init(B->pin, pin_bytes);
    else
        B->pin = nullptr;
    const size_t cap = (size_t)bp->max_active;
    if (hipMalloc(&B->d_entries, sizeof(Entry) * kClasses * cap) != hipSuccess ||
        hipMalloc(&B->d_prefix, sizeof(int) * kClasses * kKinds * (cap + 1)) != hipSuccess ||
        hipMalloc(&B->d_np, sizeof(int) * kClasses) != hipSuccess ||
        hipMalloc(&B->d_states, sizeof(DevState *) * cap) != hipSuccess ||
        hipMalloc(&B->d_flags, sizeof(int32_t) * 2 * cap) != hipSuccess ||
        hipHostMalloc(&B->h_flags, sizeof(int32_t) * 2 * cap) != hipSuccess)
        return cleanup(berr(NMF_E_NOMEM, "batch tables do not fit"));
    *out = B;
    return NMF_OK;
}

nmf_status nmf_batch_submit(nmf_batch *B, const nmf_matrix *X, const nmf_params *p,
                            const float *W0, const float *H0, int64_t *ticket)
{
    if (!B || !ticket) return berr(NMF_E_INVAL, "batch and ticket must not be NULL");
    nmf_status st = nmf::host::check_params(p);
    if (st != NMF_OK) return st;
    st = nmf::host::check_matrix_shape(X);     // the values are checked while copied below
    if (st != NMF_OK) return st;
    if (X->fmt != NMF_DENSE_ROWMAJOR)
        return berr(NMF_E_UNSUPPORTED, "batched solves take dense X");
    if (p->x_dtype != NMF_X_F32)
        return berr(NMF_E_UNSUPPORTED, "batched solves keep X in FP32 (exact-integer products)");
    if (p->inner_rule == NMF_INNER_ADAPTIVE)
        return berr(NMF_E_UNSUPPORTED, "batched solves run the fixed or the exact inner rule");
    if (!W0 || !H0) return berr(NMF_E_INVAL, "W0 and H0 must not be NULL");
    const int64_t m = X->m, n = X->n;
    const int r = p->r;
    for (int64_t i = 0; i < m * r; ++i)
        if (!(W0[i] >= 0.0f) || !std::isfinite(W0[i]))
            return berr(NMF_E_INVAL, "W0 has a negative or non-finite entry");
    for (int64_t i = 0; i < (int64_t)r * n; ++i)
        if (!(H0[i] >= 0.0f) || !std::isfinite(H0[i]))
            return berr(NMF_E_INVAL, "H0 has a negative or non-finite entry");
    auto q = std::make_unique<Prob>();
    q->p = *p;
    q->p.prod = NMF_PROD_MFMA_EXACT;
    q->m = m;
    q->n = n;
    q->r = r;
    q->rp = nmf::host::round_rank(r);
    q->m_pad = nmf::host::round_up(m, 128);
    q->n_pad = nmf::host::round_up(n, 128);
    q->ldx = nmf::host::round_up(n, 64);
    q->ldxt = nmf::host::round_up(m, 64);
    nmf::host::plan_product(q->pa, nmf::PK_MFMA_I8, m, q->m_pad, n, q->ldx, kBatchTargetWG);
    nmf::host::plan_product(q->pc, nmf::PK_MFMA_I8, n, q->n_pad, m, q->ldxt, kBatchTargetWG);
    if (layout(*q, nullptr) + layout_tmp(*q, nullptr) > (size_t)B->bp.hbm_budget)
        return berr(NMF_E_NOMEM, "the problem alone exceeds the batch arena");
    // X is kept until admission in the pinned pool when it fits (its upload is
    // then an asynchronous DMA that overlaps the running iterations), else in
    // pageable memory.
    float *dst = nullptr;
    size_t poff = 0;
    bool pinned = false;
    if (B->pin) {
        std::lock_guard<std::mutex> lk(B->mu);
        pinned = B->pin_arena.alloc(sizeof(float) * m * n, &poff);
    }
    if (pinned) {
        q->Xpin = reinterpret_cast<float *>(B->pin + poff);
        q->pin_off = poff;
        dst = q->Xpin;
    } else {
        q->X.reset(new (std::nothrow) float[(size_t)(m * n)]);
        if (!q->X) return berr(NMF_E_NOMEM, "host allocation failed");
        dst = q->X.get();
    }
    bool nonzero = false;
    const int64_t bad = nmf::host::copy_checked(X->dense, dst, m * n, &nonzero);
    if (bad >= 0 || !nonzero) {
        if (q->Xpin) {
            std::lock_guard<std::mutex> lk(B->mu);
            B->pin_arena.release(poff, sizeof(float) * m * n);
        }
        if (bad >= 0) return berr(NMF_E_INVAL, "X has a non-finite entry at " + std::to_string(bad));
        return berr(NMF_E_INVAL, "X is zero: the relative error is undefined");
    }
    q->W0.assign(W0, W0 + m * r);
    q->H0.assign(H0, H0 + (int64_t)r * n);
    std::lock_guard<std::mutex> lk(B->mu);
    q->ticket = B->next_ticket++;
    *ticket = q->ticket;
    B->queue.push_back(q.get());
    B->all[q->ticket] = std::move(q);
    return NMF_OK;
}

nmf_status nmf_batch_step(nmf_batch *B, int32_t iters, int32_t *active, int32_t *queued,
                          int32_t *retired)
{
    if (!B) return berr(NMF_E_INVAL, "batch is NULL");
    if (iters < 1) return berr(NMF_E_INVAL, "iters must be >= 1");
    BHIP(hipSetDevice(B->device));
    // The chunk the previous call left running.
    if (B->inflight) {
        B->inflight = false;
        nmf_status st = retire(B);
        if (st != NMF_OK) return st;
    }
    int done_iters = 0;
    while (done_iters < iters) {
        const int chunk = std::min(B->bp.check_every, iters - done_iters);
        bool ran = false;
        nmf_status st = launch_chunk(B, chunk, &ran);
        if (st != NMF_OK) return st;
        if (!ran) break;
        done_iters += chunk;
        if (done_iters >= iters) {
            // Left running: the caller's work (submissions, results) overlaps it.
            B->inflight = true;
            break;
        }
        st = retire(B);
        if (st != NMF_OK) return st;
    }
    std::lock_guard<std::mutex> lk(B->mu);
    if (active) *active = (int32_t)(B->active.size() + B->pending.size());
    if (queued) *queued = (int32_t)B->queue.size();
    if (retired) *retired = B->retired_unread;
    return NMF_OK;
}

nmf_status nmf_batch_result(nmf_batch *B, int64_t ticket, float *W, float *H, double *trace,
                            int32_t trace_cap, int32_t *n_iter, uint8_t *accepted, double *beta)
{
    if (!B) return berr(NMF_E_INVAL, "batch is NULL");
    std::lock_guard<std::mutex> lk(B->mu);
    auto it = B->all.find(ticket);
    if (it == B->all.end()) return berr(NMF_E_INVAL, "unknown ticket");
    Prob &q = *it->second;
    if (!q.retired) return NMF_PENDING;
    if (trace && trace_cap < q.n_iter + 1) return berr(NMF_E_INVAL, "trace_cap too small");
    if (W) std::memcpy(W, q.W.data(), sizeof(float) * q.W.size());
    if (H) std::memcpy(H, q.H.data(), sizeof(float) * q.H.size());
    if (trace) std::memcpy(trace, q.trace.data(), sizeof(double) * q.trace.size());
    if (n_iter) *n_iter = q.n_iter;
    if (accepted && q.n_iter > 0) std::memcpy(accepted, q.accepted.data(), q.accepted.size());
    if (beta && q.n_iter > 0) std::memcpy(beta, q.beta.data(), sizeof(double) * q.beta.size());
    --B->retired_unread;
    B->all.erase(it);
    return NMF_OK;
}

void nmf_batch_destroy(nmf_batch *B)
{
    if (!B) return;
    (void)hipSetDevice(B->device);
    for (int c = 0; c < kClasses; ++c)
        if (B->cs[c]) (void)hipStreamSynchronize(B->cs[c]);
    if (B->s) (void)hipStreamSynchronize(B->s);
    if (B->pool) (void)hipFree(B->pool);
    if (B->d_entries) (void)hipFree(B->d_entries);
    if (B->d_prefix) (void)hipFree(B->d_prefix);
    if (B->d_np) (void)hipFree(B->d_np);
    for (int c = 0; c < kClasses; ++c) {
        if (B->exec_one[c]) (void)hipGraphExecDestroy(B->exec_one[c]);
        if (B->exec_chunk[c]) (void)hipGraphExecDestroy(B->exec_chunk[c]);
    }
    if (B->d_states) (void)hipFree(B->d_states);
    if (B->d_flags) (void)hipFree(B->d_flags);
    if (B->h_flags) (void)hipHostFree(B->h_flags);
    if (B->h_res) (void)hipHostFree(B->h_res);
    if (B->pin) (void)hipHostFree(B->pin);
    if (B->s) (void)hipStreamDestroy(B->s);
    for (int c = 0; c < kClasses; ++c)
        if (B->cs[c]) (void)hipStreamDestroy(B->cs[c]);
    delete B;
}

}  // extern "C"
