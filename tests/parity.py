"""Comparison of GPU solves with the FP64 oracle (shared by the GPU tests).

Tolerances (the stated targets for the FP32-storage path):
  * trace: |rho_gpu(k) - rho_oracle(k)| <= 1e-5 rho_oracle(k) over the first
    50 iterations;
  * final W and H: ||G - O||_F <= 1e-4 ||O||_F.

Two effects that no FP32-storage implementation can remove widen these per
case, each measured on the oracle itself and never on the GPU result:
  * Conditioning. W and H are stored in FP32. The oracle is rerun twice
    with its iterates rounded to FP32 after every update (all arithmetic
    still FP64), to nearest and toward zero: two independent perturbations
    of the size FP32 storage makes. d_f32 is the largest distance among the
    three runs (each rerun from the FP64 run, and the two reruns from each
    other: two FP32-storage implementations of the same method); on chaotic
    trajectories it exceeds the targets. The bound becomes
    max(target, 3 d_f32), for the factors and for each trace entry.
    The drift of a chaotic trajectory grows with k, so each entry takes the
    largest drift seen up to its iteration.
  * Evaluation of rho^2. The GPU evaluates e^2 by Remark 1 as
    ||X||^2 - 2 s1 + s2 from its products, so rho^2 = e^2 / ||X||^2 carries
    the products' error relative to ||X||^2. The exact-integer products hold
    every term X_ij f_j to about 2^-27 of the row maximum of X times the
    column maximum of the factor; summed with worst-case signs this bounds
    the error of s1 / ||X||^2 by 2^-27 (max/rms of X)(max/rms of the
    factor), about 1e-8 on the data used here (the FP64 vector products:
    about 1e-15). An entry is therefore also accepted when
    |rho_g^2 - rho_o^2| <= RHO2_FLOOR = 1e-8. This matters only for small
    rho: at rho = 0.013 (the benchmark problem) it is 3e-5 relative, at
    rho = 0.1 it is 5e-7. Entries that pass only through it are printed.
  * A non-finite e(k) (the restart branch, forced through the error-scale
    hook) must be non-finite in the same way on both sides.
Accept/restart decisions may differ only where the oracle's margin
|e(k) - e(k-1)| / ||X|| is within FLIP_MARGIN; the oracle is then replayed
with the GPU's decisions and the comparison is made against that replay.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

TRACE_RTOL = 1e-5
FACTOR_RTOL = 1e-4
RHO2_FLOOR = 1e-8
FLIP_MARGIN = 1e-5


def rel_fro(a, b):
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def oracle_run(p, max_iter, replay=None, flags=0, **kw):
    return oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=max_iter, replay=replay,
                        flags=flags, **kw)


PROBES = (oracle.ROUND_F32, oracle.ROUND_F32_RZ)


def oracle_pair(p, max_iter, replay=None, oracle_flags=0, **kw):
    """The oracle run and its two FP32-storage reruns (a list), side by
    side on three threads (the oracle is plain C called through ctypes, which
    releases the GIL). All take their own decisions unless `replay` is
    given."""
    with ThreadPoolExecutor(3) as ex:
        fr = ex.submit(oracle_run, p, max_iter, replay, oracle_flags, **kw)
        fp = [ex.submit(oracle_run, p, max_iter, replay, oracle_flags | f, **kw)
              for f in PROBES]
        return fr.result(), [f.result() for f in fp]


def _replay_of(gpu, max_iter):
    """The GPU's decisions as a replay script; decisions past a tol stop are
    never reached, so the script is padded to max_iter."""
    rp = np.ones(max(max_iter, 1), dtype=np.uint8)
    rp[:gpu.n_iter] = gpu.accepted
    return rp


def compare_to_oracle(p, gpu, max_iter, trace_iters=50, oracle_flags=0, pair=None, **kw):
    """Checks the GPU result `gpu` (binding.Result) against the oracle run
    with the same parameters; returns a dict of the measured quantities.
    `oracle_flags` (e.g. oracle.ERR_REMARK1 on large sparse cases, where the
    explicit residual would cost O(mnr)) applies to every oracle run. `pair`
    may hold an (oracle run, FP32-storage rerun) computed beforehand with
    their own decisions; it is used where those decisions are the GPU's."""
    kw = dict(kw)
    base = oracle_flags
    rp = _replay_of(gpu, max_iter)
    n = gpu.n_iter
    if pair is None:
        ref, probes = oracle_pair(p, max_iter, None, base, **kw)
    else:
        ref, probes = pair
    probes = list(probes)
    flips = 0
    if not np.array_equal(ref["accepted"], gpu.accepted[:ref["n_iter"]]):
        k = int(np.argmax(ref["accepted"] != gpu.accepted[:ref["n_iter"]]))
        margin = abs(ref["margin"][k])
        assert margin < FLIP_MARGIN, (
            f"decision differs at iteration {k + 1} with margin {margin:.3e}")
        flips = int(np.sum(ref["accepted"] != gpu.accepted[:ref["n_iter"]]))
        ref, probes = oracle_pair(p, max_iter, rp, base, **kw)
    for i, f in enumerate(PROBES):
        q = probes[i]
        if q["n_iter"] < n or not np.array_equal(q["accepted"][:n], gpu.accepted):
            probes[i] = oracle_run(p, max_iter, rp, base | f, **kw)
    assert gpu.n_iter == ref["n_iter"]
    k = min(trace_iters, gpu.n_iter) + 1
    ro, rg = ref["trace"][:k], gpu.trace[:k]
    with np.errstate(invalid="ignore", divide="ignore"):
        d_tr = np.max([np.abs(q["trace"][:k] - ro) / ro for q in probes]
                      + [np.abs(probes[0]["trace"][:k] - probes[1]["trace"][:k]) / ro], axis=0)
        d_env = np.fmax.accumulate(np.where(np.isfinite(d_tr), d_tr, 0.0))
        tr_tol = np.maximum(TRACE_RTOL, 3 * d_env)
        rel = np.abs(rg - ro) / ro
        ok_rel = rel <= tr_tol
        ok_sq = np.abs(rg ** 2 - ro ** 2) <= RHO2_FLOOR
    fin = np.isfinite(ro)
    same_nonfinite = ~fin & ((np.isnan(ro) & np.isnan(rg)) | (ro == rg))
    bad = ~(ok_rel | ok_sq | same_nonfinite)
    floor_only = ok_sq & ~ok_rel
    if floor_only.any():
        idx = np.flatnonzero(floor_only)
        print(f"parity: {idx.size} trace entries pass only through the rho^2 floor, "
              f"k={idx.tolist()[:8]}, max |rho_g^2 - rho_o^2| = "
              f"{np.abs(rg[idx] ** 2 - ro[idx] ** 2).max():.2e}", flush=True)
    rel = np.where(fin, rel, 0.0)
    d_f32 = max(max(rel_fro(a["W"], b["W"]), rel_fro(a["H"], b["H"]))
                for a, b in [(probes[0], ref), (probes[1], ref), (probes[0], probes[1])])
    fac_tol = max(FACTOR_RTOL, 3 * d_f32)
    dw, dh = rel_fro(gpu.W, ref["W"]), rel_fro(gpu.H, ref["H"])
    dwh = rel_fro(np.asarray(gpu.W, np.float64) @ np.asarray(gpu.H, np.float64),
                  ref["W"] @ ref["H"])
    print(f"parity: iters={gpu.n_iter} trace_rel={rel.max():.2e} W={dw:.2e} H={dh:.2e} "
          f"WH={dwh:.2e} flips={flips} f32-storage drift={d_f32:.2e} "
          f"factor_tol={fac_tol:.2e}", flush=True)
    if bad.any():
        j = int(np.argmax(bad))
        raise AssertionError(
            f"trace mismatch at k={j}: rho_gpu {rg[j]:.9e} rho_oracle {ro[j]:.9e} "
            f"rel {rel[j]:.3e} (tol {tr_tol[j]:.2e}), |drho^2| {abs(rg[j]**2 - ro[j]**2):.2e}")
    np.testing.assert_allclose(gpu.beta, ref["beta"], rtol=1e-12)
    assert dw <= fac_tol and dh <= fac_tol, (dw, dh, fac_tol)
    # the product is free of the diagonal scaling ambiguity of (W, H)
    assert dwh <= fac_tol
    return dict(ref=ref, flips=flips, trace_rel=float(rel.max()), W=dw, H=dh, WH=dwh,
                d_f32=d_f32)
