"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each one checks it
against an independent route to the same number (brute-force enumeration, a
derivative-free 1-D search, numpy's own linear algebra, hand-computed
scripts of Algorithm 3, values printed in the paper's tables, or invariants
that any correct implementation must satisfy).
"""
import itertools
import json
import os

import numpy as np
import pytest

import nmf_synth as S
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- helpers

def brute_force_nnls(W, x):
    """min_{h >= 0} ||x - W h||_2 by enumerating all 2^r passive sets and
    solving the unconstrained least squares on each (numpy lstsq)."""
    r = W.shape[1]
    best, best_h = np.inf, None
    for mask in itertools.product([0, 1], repeat=r):
        P = [k for k in range(r) if mask[k]]
        h = np.zeros(r)
        if P:
            sol, *_ = np.linalg.lstsq(W[:, P], x, rcond=None)
            if np.any(sol < 0):
                continue
            h[P] = sol
        f = float(np.sum((x - W @ h) ** 2))
        if f < best:
            best, best_h = f, h
    return best_h


def ternary_min(f, lo, hi, iters=300):
    """Derivative-free minimizer of a convex function on [lo, hi]."""
    for _ in range(iters):
        a = lo + (hi - lo) / 3.0
        b = hi - (hi - lo) / 3.0
        if f(a) <= f(b):
            hi = b
        else:
            lo = a
    return 0.5 * (lo + hi)


def kkt_residual(X, W, H):
    """||min(W, grad_W)||_F + ||min(H, grad_H)||_F for f = 1/2 ||X - WH||^2."""
    gW = W @ (H @ H.T) - X @ H.T
    gH = (W.T @ W) @ H - W.T @ X
    return (np.linalg.norm(np.minimum(W, gW)) + np.linalg.norm(np.minimum(H, gH)))


# ------------------------------------------- the HALS closed form (section 1)

@pytest.mark.parametrize("seed", range(5))
def test_single_sweep_is_exact_coordinate_minimization(seed):
    """One HALS sweep replaces each row of H, in ascending order, by the
    exact minimizer of the objective over that row with the others fixed
    (section 1, the closed form and its sequential use). Checked against a
    derivative-free 1-D search of the objective itself."""
    rng = np.random.default_rng(seed)
    m, r, n = 7, 3, 4
    W = rng.random((m, r))
    X = rng.random((m, n)) - 0.2          # some coordinates must clamp at 0
    H0 = rng.random((r, n))
    got = oracle.nnls_h(X, W, H0, sweeps=1)
    want = H0.copy()
    for k in range(r):
        for c in range(n):
            def f(t, k=k, c=c):
                h = want[:, c].copy()
                h[k] = t
                return float(np.sum((X[:, c] - W @ h) ** 2))
            want[k, c] = ternary_min(f, 0.0, 50.0)
            # a quadratic is flat near its minimum: comparisons of f only
            # resolve the argmin to about sqrt(machine eps)
            assert abs(got[k, c] - want[k, c]) < 1e-7
            want[k, c] = got[k, c]


@pytest.mark.parametrize("seed", range(4))
def test_w_side_single_sweep_is_exact_coordinate_minimization(seed):
    """The W update by the symmetry ||X - WH|| = ||X^T - H^T W^T||
    (section 1): each column of W, in ascending order, is the exact
    minimizer with the other columns fixed."""
    rng = np.random.default_rng(100 + seed)
    m, r, n = 3, 3, 6
    H = rng.random((r, n))
    X = rng.random((m, n)) - 0.2
    W0 = rng.random((m, r))
    got = oracle.nnls_w(X, H, W0, sweeps=1)
    want = W0.copy()
    for k in range(r):
        for i in range(m):
            def f(t, k=k, i=i):
                w = want[i, :].copy()
                w[k] = t
                return float(np.sum((X[i, :] - w @ H) ** 2))
            want[i, k] = ternary_min(f, 0.0, 50.0)
            assert abs(got[i, k] - want[i, k]) < 1e-7
            want[i, k] = got[i, k]


@pytest.mark.parametrize("seed", range(6))
def test_sweeps_converge_to_brute_force_nnls_h(seed):
    """Repeated sweeps (A-HALS, section 1) solve the NNLS subproblem (nnls):
    on tiny inputs they match brute-force active-set enumeration."""
    rng = np.random.default_rng(seed)
    m = int(rng.integers(4, 9))
    r = int(rng.integers(2, min(m, 5) + 1))
    n = 5
    W = rng.random((m, r))
    X = rng.random((m, n)) * 2 - 0.5
    H = oracle.nnls_h(X, W, rng.random((r, n)), sweeps=4000)
    for c in range(n):
        np.testing.assert_allclose(H[:, c], brute_force_nnls(W, X[:, c]),
                                   atol=1e-9, rtol=0)


@pytest.mark.parametrize("seed", range(6))
def test_sweeps_converge_to_brute_force_nnls_w(seed):
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(4, 9))
    r = int(rng.integers(2, min(n, 5) + 1))
    m = 4
    H = rng.random((r, n))
    X = rng.random((m, n)) * 2 - 0.5
    W = oracle.nnls_w(X, H, rng.random((m, r)), sweeps=4000)
    for i in range(m):
        np.testing.assert_allclose(W[i, :], brute_force_nnls(H.T, X[i, :]),
                                   atol=1e-9, rtol=0)


def test_zero_denominator_keeps_the_coordinate():
    """A zero column of W makes ||W(:,k)||^2 = 0; that row of H does not
    enter the objective, so any nonnegative value minimizes: it is kept where
    nonnegative and projected to 0 where the warm start was negative."""
    rng = np.random.default_rng(3)
    W = rng.random((6, 3))
    W[:, 1] = 0.0
    X = rng.random((6, 4))
    H0 = rng.random((3, 4))
    H0[1, 2] = -0.5
    H = oracle.nnls_h(X, W, H0, sweeps=50)
    np.testing.assert_array_equal(H[1], np.maximum(H0[1], 0.0))
    Wk = W[:, [0, 2]]
    for c in range(4):
        np.testing.assert_allclose(H[[0, 2], c], brute_force_nnls(Wk, X[:, c]),
                                   atol=1e-9)


# ------------------------------------------------- Remark 1 and the error

@pytest.mark.parametrize("csr", [False, True])
def test_remark1_matches_explicit_residual(csr):
    """Remark 1's identity equals the explicit Frobenius residual, and both
    equal numpy's norm of X - WH."""
    rng = np.random.default_rng(7)
    m, n, r = 30, 25, 4
    Xd = rng.random((m, n)) * (rng.random((m, n)) < 0.4)
    W = rng.random((m, r))
    H = rng.random((r, n))
    X = S.dense_to_csr(Xd.astype(np.float32)) if csr else Xd
    Xref = S.csr_to_dense(X).astype(np.float64) if csr else Xd
    want = np.linalg.norm(Xref - W @ H) / np.linalg.norm(Xref)
    assert oracle.rel_error(X, W, H) == pytest.approx(want, rel=1e-13)
    assert oracle.rel_error_remark1(X, W, H) == pytest.approx(want, rel=1e-12)


# -------------------------------------------------------- Algorithm 3

def _golden_beta():
    with open(os.path.join(GOLDEN, "beta_script.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("idx", [0, 1])
def test_beta_controller_hand_computed_script(idx):
    g = _golden_beta()
    p = g["params"]
    s = g["scripts"][idx]
    for flags, key in [(0, "betabar_after_literal"),
                       (oracle.BETABAR_LAST_ACCEPTED, "betabar_after_last_accepted")]:
        bu, bb = oracle.beta_script(s["decreased"], p["beta0"], p["gamma"],
                                    p["gamma_bar"], p["eta"], flags)
        np.testing.assert_allclose(bu, s["beta_used"], rtol=1e-15)
        np.testing.assert_allclose(bb, s[key], rtol=1e-15)


def test_solve_follows_beta_controller():
    """The beta used by a full solve at each iteration is Algorithm 3 fed
    with that solve's own accept/restart outcomes."""
    p = S.fullrank(1, m=40, n=30, r=5)
    out = oracle.solve(p.X, p.r, p.W0, p.H0, hp=2, beta0=0.9, gamma=1.1,
                       gamma_bar=1.05, eta=1.5, max_iter=80)
    assert (~out["accepted"]).sum() >= 2, "the script needs restarts"
    bu, _ = oracle.beta_script(out["accepted"], 0.9, 1.1, 1.05, 1.5)
    np.testing.assert_array_equal(out["beta"], bu)


# ------------------------------------------------ Algorithm 2 end to end

def _alg2_brute(X, W0, H0, hp, betas, decisions):
    """Algorithm 2 with exact NNLS (brute-force enumeration) and explicit
    numpy residuals, driven by given betas and accept/restart decisions."""
    W, H = W0.copy(), H0.copy()
    Wy, Hy = W.copy(), H.copy()
    trace = []
    for beta, acc in zip(betas, decisions):
        Hn = np.stack([brute_force_nnls(Wy, X[:, c]) for c in range(X.shape[1])], 1)
        Hyn = Hn + beta * (Hn - H)
        if hp == 3:
            Hyn = np.maximum(Hyn, 0.0)
        Hw = Hn if hp == 1 else Hyn
        Wn = np.stack([brute_force_nnls(Hw.T, X[i, :]) for i in range(X.shape[0])], 0)
        Wyn = Wn + beta * (Wn - W)
        trace.append(np.linalg.norm(X - Wn @ Hw) / np.linalg.norm(X))
        if acc:
            W, H, Wy, Hy = Wn, Hn, Wyn, Hyn
        else:
            Wy, Hy = W.copy(), H.copy()
    return np.array(trace), W, H


@pytest.mark.parametrize("hp", [1, 2, 3])
def test_alg2_pipeline_against_brute_force(hp):
    """Four outer iterations on a tiny problem, with enough sweeps that the
    inner NNLS is exact, against an independent pipeline built from
    brute-force NNLS; decisions are forced (replay) to include a restart,
    and the betas are the hand-computed Algorithm 3 values for them."""
    rng = np.random.default_rng(11)
    m, n, r = 6, 5, 2
    X = rng.random((m, n))
    W0 = rng.random((m, r))
    H0 = rng.random((r, n))
    decisions = [1, 0, 1, 1]
    betas = [0.5, 0.525, 0.35, 0.3675]      # Alg. 3: accept, reject, accept
    out = oracle.solve(X, r, W0, H0, hp=hp, beta0=0.5, gamma=1.05,
                       gamma_bar=1.01, eta=1.5, inner_k=3000, max_iter=4,
                       replay=decisions)
    np.testing.assert_allclose(out["beta"], betas, rtol=1e-15)
    tr, W, H = _alg2_brute(X, W0, H0, hp, betas, decisions)
    np.testing.assert_allclose(out["trace"][1:], tr, rtol=1e-8)
    np.testing.assert_allclose(out["W"], W, atol=1e-8)
    np.testing.assert_allclose(out["H"], H, atol=1e-8)


def _alg2_brute_deciding(X, W0, H0, hp, e2_scale, beta0=0.5, gamma=1.05,
                        gamma_bar=1.01, eta=1.5):
    """The brute-force pipeline of _alg2_brute taking its own decisions, as
    Algorithm 2 states them: restart when e(k) is not finite or exceeds the
    previous finite error (R7, R9), accept otherwise (ties accept, R8).
    e(k)^2 is multiplied by e2_scale[k] first (the oracle's test hook). The
    beta of each iteration comes from the pinned Algorithm 3 script fed with
    the decisions taken so far."""
    W, H = W0.copy(), H0.copy()
    Wy, Hy = W.copy(), H.copy()
    nx = np.linalg.norm(X)
    e_prev = np.sqrt(np.sum((X - W @ H) ** 2) * e2_scale[0])
    trace, decisions = [e_prev / nx], []
    for k in range(1, len(e2_scale)):
        bu, _ = oracle.beta_script(decisions + [1], beta0, gamma, gamma_bar, eta)
        beta = bu[-1]
        Hn = np.stack([brute_force_nnls(Wy, X[:, c]) for c in range(X.shape[1])], 1)
        Hyn = Hn + beta * (Hn - H)
        if hp == 3:
            Hyn = np.maximum(Hyn, 0.0)
        Hw = Hn if hp == 1 else Hyn
        Wn = np.stack([brute_force_nnls(Hw.T, X[i, :]) for i in range(X.shape[0])], 0)
        Wyn = Wn + beta * (Wn - W)
        e2 = np.sum((X - Wn @ Hw) ** 2) * e2_scale[k]
        e = np.sqrt(e2) if np.isfinite(e2) else abs(e2)
        trace.append(e / nx)
        acc = bool(np.isfinite(e) and e <= e_prev)
        decisions.append(int(acc))
        if acc:
            W, H, Wy, Hy = Wn, Hn, Wyn, Hyn
        else:
            Wy, Hy = W.copy(), H.copy()
        if np.isfinite(e):
            e_prev = e
    return np.array(trace), np.array(decisions, dtype=bool), W, H


@pytest.mark.parametrize("flags", [0, oracle.ERR_REMARK1])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_error_restarts_and_keeps_the_previous_error(flags, bad):
    """R9 against the brute-force pipeline deciding for itself: a non-finite
    e(2) must be a restart, and must not become the error that e(3) is
    compared with. e(3)^2 is inflated a millionfold, so it exceeds e(1) and
    must restart too; had e(2) replaced e(1), nothing would exceed it and
    iteration 3 would be accepted. The error by Remark 1 (which clamps a
    slightly negative e^2 at zero) must not turn a NaN into an error of 0."""
    rng = np.random.default_rng(11)
    m, n, r = 6, 5, 2
    X = rng.random((m, n))
    W0 = rng.random((m, r))
    H0 = rng.random((r, n))
    scale = np.array([1.0, 1.0, bad, 1e6, 1.0, 1.0])
    out = oracle.solve(X, r, W0, H0, hp=3, beta0=0.5, gamma=1.05, gamma_bar=1.01,
                       eta=1.5, inner_k=3000, max_iter=5, flags=flags, e2_scale=scale)
    tr, dec, W, H = _alg2_brute_deciding(X, W0, H0, 3, scale)
    assert list(dec[:3]) == [True, False, False]
    np.testing.assert_array_equal(out["accepted"], dec)
    assert not np.isfinite(out["trace"][2]) and not np.isfinite(tr[2])
    if bad == np.inf:
        assert out["trace"][2] == np.inf
    else:
        assert np.isnan(out["trace"][2])
    fin = np.isfinite(tr)
    np.testing.assert_allclose(out["trace"][fin], tr[fin], rtol=1e-8)
    # Alg. 3 for accept, restart, restart, then the pipeline's outcomes.
    np.testing.assert_allclose(out["beta"][:4], [0.5, 0.525, 0.35, 0.35 / 1.5], rtol=1e-15)
    np.testing.assert_allclose(out["W"], W, atol=1e-8)
    np.testing.assert_allclose(out["H"], H, atol=1e-8)


@pytest.mark.parametrize("flags", [0, oracle.ERR_REMARK1])
def test_nonfinite_initial_error_is_a_numeric_error(flags):
    """R9: a non-finite e(0) is reported (status ORACLE_ENUMERIC), not
    taken as an error of 0."""
    p = S.fullrank(2, m=20, n=15, r=3)
    for bad in (np.nan, np.inf):
        with pytest.raises(RuntimeError, match="status 2"):
            oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=3, flags=flags, e2_scale=[bad])


def test_all_restarts_keep_the_initial_iterate():
    p = S.fullrank(2, m=20, n=15, r=3)
    out = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=5, replay=[0] * 5)
    np.testing.assert_array_equal(out["W"], p.W0.astype(np.float64))
    np.testing.assert_array_equal(out["H"], p.H0.astype(np.float64))


def test_replay_of_own_decisions_is_identical():
    p = S.fullrank(3, m=50, n=40, r=6)
    a = oracle.solve(p.X, p.r, p.W0, p.H0, hp=2, beta0=0.8, max_iter=60)
    b = oracle.solve(p.X, p.r, p.W0, p.H0, hp=2, beta0=0.8, max_iter=60,
                     replay=a["accepted"])
    np.testing.assert_array_equal(a["trace"], b["trace"])
    np.testing.assert_array_equal(a["W"], b["W"])


# ---------------------------------------------------------- special cases

@pytest.mark.parametrize("hp", [1, 2, 3])
def test_beta_zero_is_monotone_a_hals(hp):
    """beta = 0 gives back the base algorithm (section 2): exact block
    coordinate descent never increases the objective, so the trace is
    non-increasing and no restart fires (ties accept)."""
    p = S.fullrank(4, m=60, n=50, r=8)
    out = oracle.solve(p.X, p.r, p.W0, p.H0, hp=hp, beta0=0.0, max_iter=150)
    t = out["trace"]
    assert np.all(np.diff(t) <= 1e-15 * t[:-1])
    assert out["accepted"].all()
    assert np.all(out["beta"] == 0.0)


@pytest.mark.parametrize("seed", range(3))
def test_trace_above_svd_lower_bound(seed):
    """Eckart-Young: no rank-r product beats the truncated SVD, so every
    rho(k), feasible or not, is at least the SVD bound."""
    p = S.fullrank(seed)
    sv = np.linalg.svd(p.X.astype(np.float64), compute_uv=False)
    bound = np.sqrt(np.sum(sv[p.r:] ** 2) / np.sum(sv ** 2))
    for hp in (1, 2, 3):
        out = oracle.solve(p.X, p.r, p.W0, p.H0, hp=hp, max_iter=60)
        assert np.all(out["trace"] >= bound * (1 - 1e-12))


def test_hp3_iterates_feasible_and_trace_is_their_residual():
    """hp = 3 projects H_y, so (W_n, H_y) is feasible; the reported error of
    the last accepted iteration of an all-accept run with beta = 0 is then
    the residual of the returned pair."""
    p = S.fullrank(5, m=40, n=30, r=4)
    out = oracle.solve(p.X, p.r, p.W0, p.H0, hp=3, beta0=0.0, max_iter=30)
    assert out["W"].min() >= 0 and out["H"].min() >= 0
    Xd = p.X.astype(np.float64)
    want = np.linalg.norm(Xd - out["W"] @ out["H"]) / np.linalg.norm(Xd)
    assert out["trace"][-1] == pytest.approx(want, rel=1e-12)
    out2 = oracle.solve(p.X, p.r, p.W0, p.H0, hp=3, beta0=0.7, max_iter=30)
    assert out2["W"].min() >= 0 and out2["H"].min() >= 0


def test_planted_exact_6x5_rank2_recovered():
    """X = W* H* exactly (6 x 5, r = 2): E-A-HALS reaches an exact
    factorization (explicit residual below 1e-10) from most random starts;
    NMF is nonconvex, so 8 of 10 seeds are required."""
    ok = 0
    for seed in range(10):
        rng = np.random.default_rng(seed)
        X = rng.random((6, 2)) @ rng.random((2, 5))
        W0 = rng.random((6, 2))
        H0 = rng.random((2, 5))
        out = oracle.solve(X, 2, W0, H0, hp=3, max_iter=3000)
        res = np.linalg.norm(X - out["W"] @ out["H"]) / np.linalg.norm(X)
        ok += res < 1e-10
    assert ok >= 8


@pytest.mark.parametrize("beta0,hp", [(0.0, 3), (0.5, 3), (0.5, 1)])
def test_kkt_residual_vanishes_at_convergence(beta0, hp):
    rng = np.random.default_rng(21)
    X = rng.random((10, 8))
    W0 = rng.random((10, 3))
    H0 = rng.random((3, 8))
    one = oracle.solve(X, 3, W0, H0, hp=hp, beta0=beta0, max_iter=1)
    out = oracle.solve(X, 3, W0, H0, hp=hp, beta0=beta0, max_iter=4000)
    k1 = kkt_residual(X, one["W"], one["H"])
    kn = kkt_residual(X, out["W"], out["H"])
    assert kn <= 1e-8 * k1


def test_dense_and_csr_give_identical_traces():
    rng = np.random.default_rng(9)
    Xd = (rng.random((40, 35)) * (rng.random((40, 35)) < 0.3)).astype(np.float32)
    W0, H0 = S.init_factors(40, 35, 5, 9)
    a = oracle.solve(Xd, 5, W0, H0, max_iter=40)
    b = oracle.solve(S.dense_to_csr(Xd), 5, W0, H0, max_iter=40)
    np.testing.assert_allclose(a["trace"], b["trace"], rtol=1e-14, atol=0)
    np.testing.assert_allclose(a["W"], b["W"], rtol=1e-12, atol=1e-14)


def test_tol_stops_after_small_accepted_change():
    p = S.lowrank(0, m=30, n=30, r=3)
    out = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=5000, tol=1e-6)
    k = out["n_iter"]
    assert k < 5000
    assert out["accepted"][-1]
    assert abs(out["trace"][-1] - out["trace"][-2]) < 1e-6


def test_invalid_inputs_rejected():
    X = np.ones((3, 3))
    with pytest.raises(RuntimeError):
        oracle.solve(X, 1, np.ones((3, 1)), np.ones((1, 3)), hp=4)
    with pytest.raises(RuntimeError):
        oracle.solve(np.zeros((3, 3)), 1, np.ones((3, 1)), np.ones((1, 3)))


# ------------------------------------------------ statistics of the tables

def test_fullrank_final_error_matches_table4():
    """Table 4 prints E-A-HALS final rho = 0.423817 +- 1.184e-3 (hp = 3) on
    200 x 200 U[0,1] data with r = 20 and the final parameters of section
    5.3.2 (beta0 0.5, eta 1.5, gamma 1.01, gamma_bar 1.005). The mean of 10
    seeded data sets must lie within 3 standard errors of it."""
    fin = []
    for s in range(10):
        p = S.fullrank(s)
        out = oracle.solve(p.X, p.r, p.W0, p.H0, hp=3, beta0=0.5, gamma=1.01,
                           gamma_bar=1.005, eta=1.5, max_iter=300)
        fin.append(out["trace"][-1])
    assert abs(np.mean(fin) - 0.423817) < 3 * 1.184e-3 / np.sqrt(10)


def test_lowrank_extrapolation_beats_plain_ahals():
    """Table 3: on low-rank 200 x 200 r = 20 data, E-A-HALS (hp = 3) ends
    far below A-HALS in mean relative error. Same iteration budget here."""
    ext, plain = [], []
    for s in range(4):
        p = S.lowrank(s, r=20)
        kw = dict(hp=3, gamma=1.01, gamma_bar=1.005, eta=1.5, max_iter=300)
        ext.append(oracle.solve(p.X, 20, p.W0, p.H0, beta0=0.5, **kw)["trace"][-1])
        plain.append(oracle.solve(p.X, 20, p.W0, p.H0, beta0=0.0, **kw)["trace"][-1])
    assert np.mean(ext) < 0.5 * np.mean(plain)


# ------------------------------------------------------------ beta* (section 4)

def test_beta_star_is_the_minimizer_of_the_extrapolated_error():
    """beta* against a dense scan of ||X - (Wn + b (Wn - W)) Hw||_F^2 over b
    and against the direct form <X - Wn Hw, dW Hw> / ||dW Hw||^2 (numpy)."""
    rng = np.random.default_rng(11)
    for trial in range(5):
        m, n, r = 9, 7, 3
        X = rng.random((m, n))
        Wn, W, Hw = rng.random((m, r)), rng.random((m, r)), rng.random((r, n))
        b = oracle.beta_star(X, Wn, W, Hw)
        dWH = (Wn - W) @ Hw
        R = X - Wn @ Hw
        assert abs(b - np.sum(R * dWH) / np.sum(dWH * dWH)) < 1e-12 * max(1.0, abs(b))
        grid = np.linspace(b - 2.0, b + 2.0, 4001)
        f = [np.sum((X - (Wn + g * (Wn - W)) @ Hw) ** 2) for g in grid]
        assert abs(grid[int(np.argmin(f))] - b) <= 1e-3


def test_beta_star_without_direction_is_zero():
    """R16: W_n = W leaves no direction; beta* is reported as 0."""
    rng = np.random.default_rng(3)
    X = rng.random((6, 5))
    W = rng.random((6, 2))
    assert oracle.beta_star(X, W, W, rng.random((2, 5))) == 0.0


def test_beta_star_of_the_first_iteration():
    """The solve's beta*(1) equals beta* recomputed from its own first
    iterate: after an accepted first iteration W = W_n, H = H_n, and for
    hp = 3 the W update used H_w = max(0, H_n + beta0 (H_n - H0))."""
    p = S.fullrank(4, m=40, n=30, r=4)
    out = oracle.solve(p.X, p.r, p.W0, p.H0, hp=3, beta0=0.5, max_iter=1)
    assert out["accepted"][0]
    H0 = p.H0.astype(np.float64)
    Hw = np.maximum(out["H"] + 0.5 * (out["H"] - H0), 0.0)
    b = oracle.beta_star(p.X, out["W"], p.W0.astype(np.float64), Hw)
    assert abs(out["beta_star"][0] - b) < 1e-12 * max(1.0, abs(b))


# ------------------------------------------- exact NNLS and E-ANLS (section 1)

def nnls_kkt(G, c, x):
    """Largest violation of the NNLS optimality conditions x >= 0, y = Gx - c
    >= 0, x * y = 0, each relative to the size of x and of y."""
    y = G @ x - c
    xs = max(np.abs(x).max(), 1e-300)
    ys = np.abs(c).max() + np.abs(G).max() * xs
    return max(-x.min() / xs, -y.min() / ys, np.abs(x * y).max() / (xs * ys))


@pytest.mark.parametrize("seed", range(6))
def test_exact_nnls_matches_brute_force(seed):
    """The block principal pivoting solve of every column of H (and every row
    of W) equals brute-force enumeration of the 2^r passive sets, from a warm
    start that is far from the answer (negative entries included)."""
    rng = np.random.default_rng(100 + seed)
    m, n, r = 9, 7, 2 + seed % 4
    X = rng.random((m, n))
    W = rng.random((m, r)) - 0.3
    H0 = rng.standard_normal((r, n))
    H = oracle.nnls_exact_h(X, W, H0)
    for c in range(n):
        np.testing.assert_allclose(H[:, c], brute_force_nnls(W, X[:, c]), atol=1e-10)
    Hf = rng.random((r, n)) - 0.3
    W0 = rng.standard_normal((m, r))
    Wx = oracle.nnls_exact_w(X, Hf, W0)
    for i in range(m):
        np.testing.assert_allclose(Wx[i], brute_force_nnls(Hf.T, X[i, :]), atol=1e-10)


@pytest.mark.parametrize("seed", range(3))
def test_exact_nnls_satisfies_kkt_at_rank_20(seed):
    """At r = 20 enumeration is out of reach; the solution must satisfy the
    optimality conditions of the convex problem, which fix it uniquely when W
    has full column rank, and repeated warm starts must not move it."""
    rng = np.random.default_rng(200 + seed)
    m, n, r = 60, 40, 20
    X = rng.random((m, n))
    W = rng.random((m, r))
    H = oracle.nnls_exact_h(X, W, rng.standard_normal((r, n)))
    G, C = W.T @ W, W.T @ X
    for c in range(n):
        assert nnls_kkt(G, C[:, c], H[:, c]) < 1e-12
    assert (H == 0).sum() > 0, "no active constraint: the test would not exercise pivoting"
    H2 = oracle.nnls_exact_h(X, W, np.zeros((r, n)))
    np.testing.assert_allclose(H2, H, atol=1e-12)


def test_exact_nnls_zero_diagonal_keeps_the_coordinate():
    """A zero column of W: that row of H does not enter the objective; the
    exact solve keeps the warm start projected to the orthant, the others are
    the brute-force solution of the reduced problem."""
    rng = np.random.default_rng(5)
    W = rng.random((6, 3))
    W[:, 1] = 0.0
    X = rng.random((6, 4))
    H0 = rng.random((3, 4))
    H0[1, 2] = -0.5
    H = oracle.nnls_exact_h(X, W, H0)
    np.testing.assert_array_equal(H[1], np.maximum(H0[1], 0.0))
    for c in range(4):
        np.testing.assert_allclose(H[[0, 2], c], brute_force_nnls(W[:, [0, 2]], X[:, c]),
                                   atol=1e-10)


@pytest.mark.parametrize("hp", [1, 2, 3])
def test_eanls_pipeline_against_brute_force(hp):
    """E-ANLS (Algorithm 2 with each NNLS block solved exactly, section 1)
    against the independent brute-force pipeline, on forced decisions that
    include a restart, with r = 3 so that pivoting has work to do."""
    rng = np.random.default_rng(12)
    m, n, r = 7, 6, 3
    X = rng.random((m, n))
    W0 = rng.random((m, r))
    H0 = rng.random((r, n))
    decisions = [1, 0, 1, 1]
    betas = [0.5, 0.525, 0.35, 0.3675]
    out = oracle.solve(X, r, W0, H0, hp=hp, beta0=0.5, gamma=1.05, gamma_bar=1.01,
                       eta=1.5, max_iter=4, replay=decisions, flags=oracle.EXACT_NNLS)
    tr, W, H = _alg2_brute(X, W0, H0, hp, betas, decisions)
    np.testing.assert_allclose(out["trace"][1:], tr, rtol=1e-10)
    np.testing.assert_allclose(out["W"], W, atol=1e-10)
    np.testing.assert_allclose(out["H"], H, atol=1e-10)


def test_anls_is_monotone_and_ignores_inner_k():
    """beta = 0 gives ANLS: exact two-block descent never increases the
    error, and the inner sweep count has no effect on an exact solve."""
    p = S.fullrank(4, m=60, n=50, r=8)
    a = oracle.solve(p.X, p.r, p.W0, p.H0, hp=1, beta0=0.0, max_iter=60,
                     flags=oracle.EXACT_NNLS)
    b = oracle.solve(p.X, p.r, p.W0, p.H0, hp=1, beta0=0.0, max_iter=60, inner_k=1,
                     flags=oracle.EXACT_NNLS)
    t = a["trace"]
    assert np.all(np.diff(t) <= 1e-15 * t[:-1]) and a["accepted"].all()
    np.testing.assert_array_equal(a["trace"], b["trace"])


def test_eanls_fullrank_final_error_matches_table4():
    """Table 4 prints E-ANLS (hp = 1) final rho = 0.423795 +- 1.161e-3 on
    200 x 200 U[0,1] data with r = 20, using the E-ANLS parameters chosen in
    section 5.3.1 (beta0 0.5, eta 1.5, gamma 1.1, gamma_bar 1.05). The mean
    over 10 seeded data sets lies within 3 standard errors of it."""
    fin = []
    for s in range(10):
        p = S.fullrank(s)
        out = oracle.solve(p.X, p.r, p.W0, p.H0, hp=1, beta0=0.5, gamma=1.1, gamma_bar=1.05,
                           eta=1.5, max_iter=150, flags=oracle.EXACT_NNLS)
        fin.append(out["trace"][-1])
    assert abs(np.mean(fin) - 0.423795) < 3 * 1.161e-3 / np.sqrt(10)


def test_eanls_lowrank_beats_anls():
    """Table 3: on low-rank data E-ANLS (hp = 1) ends far below ANLS in mean
    error (2.6e-8 against 5.6e-5 there). Same iteration budget for both here."""
    ext, plain = [], []
    for s in range(4):
        p = S.lowrank(s, r=20)
        kw = dict(hp=1, gamma=1.1, gamma_bar=1.05, eta=1.5, max_iter=150,
                  flags=oracle.EXACT_NNLS)
        ext.append(oracle.solve(p.X, 20, p.W0, p.H0, beta0=0.5, **kw)["trace"][-1])
        plain.append(oracle.solve(p.X, 20, p.W0, p.H0, beta0=0.0, **kw)["trace"][-1])
    assert np.mean(ext) < 0.1 * np.mean(plain)


# ------------------------------------- adaptive inner loop (R18, recalled)

def test_adaptive_with_zero_delta_is_fixed_at_the_cap():
    """With delta = 0 the early stop never fires, so the adaptive loop is the
    fixed loop at its cap: 200 x 200, r = 10 gives rho = 1 + (40000 + 2000) /
    (200 * 11) = 20.09 and floor(1 + 0.5 rho) = 11 sweeps on either side."""
    p = S.lowrank(0)
    a = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=15, inner_k=50, inner_delta=0.0,
                     flags=oracle.ADAPTIVE_INNER)
    b = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=15, inner_k=11)
    assert np.all(a["sweeps"] == 11)
    np.testing.assert_array_equal(a["trace"], b["trace"])
    np.testing.assert_array_equal(a["W"], b["W"])


@pytest.mark.parametrize("r,inner_k,alpha,cap", [(20, 50, 0.5, 6), (20, 4, 0.5, 4),
                                                 (10, 50, 0.0, 1), (10, 50, 1.0, 21)])
def test_adaptive_sweep_cap(r, inner_k, alpha, cap):
    """The cap floor(1 + alpha rho), at most inner_k: for 200 x 200, r = 20,
    rho = 1 + 44000 / 4200 = 11.48 (cap 6 at alpha 0.5); r = 10 gives 20.09
    (cap 21 at alpha 1, 1 at alpha 0)."""
    p = S.fullrank(1, r=r)
    a = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=6, inner_k=inner_k, inner_alpha=alpha,
                     inner_delta=0.0, flags=oracle.ADAPTIVE_INNER)
    assert np.all(a["sweeps"] == cap)


def test_adaptive_caps_from_given_cost_ratios():
    """Cost ratios given per side replace the flop ratio: rho_H = 7 and
    rho_W = 3 at alpha 0.5 cap the H loop at floor(4.5) = 4 and the W loop at
    floor(2.5) = 2 sweeps; equal ratios of 7 on both sides, with delta = 0,
    give the fixed loop of 4 sweeps bit for bit."""
    p = S.lowrank(3)
    a = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=8, inner_k=50, inner_delta=0.0,
                     inner_rho_h=7.0, inner_rho_w=3.0, flags=oracle.ADAPTIVE_INNER)
    assert np.all(a["sweeps"][:, 0] == 4) and np.all(a["sweeps"][:, 1] == 2)
    b = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=8, inner_k=50, inner_delta=0.0,
                     inner_rho_h=7.0, inner_rho_w=7.0, flags=oracle.ADAPTIVE_INNER)
    c = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=8, inner_k=4)
    assert np.all(b["sweeps"] == 4)
    np.testing.assert_array_equal(b["trace"], c["trace"])
    np.testing.assert_array_equal(b["W"], c["W"])


def test_adaptive_refuses_a_negative_cost_ratio():
    p = S.lowrank(3)
    with pytest.raises(RuntimeError):
        oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=2, inner_rho_w=-1.0,
                     flags=oracle.ADAPTIVE_INNER)


def test_adaptive_with_huge_delta_stops_after_the_second_sweep():
    """The stopping test applies from the second sweep on: with a delta no
    change can exceed, every loop runs exactly two sweeps."""
    p = S.fullrank(2)
    a = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=10, inner_k=50, inner_delta=1e300,
                     flags=oracle.ADAPTIVE_INNER)
    b = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=10, inner_k=2)
    assert np.all(a["sweeps"] == 2)
    np.testing.assert_array_equal(a["trace"], b["trace"])


def test_adaptive_stop_follows_the_sweep_changes():
    """First H update of a solve: the sweep count equals the first l >= 2
    whose change ||H^(l) - H^(l-1)||_F is at most delta ||H^(1) - H^(0)||_F,
    from sweeps run one at a time by the pinned HALS routine."""
    p = S.lowrank(1)
    delta = 0.3
    a = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=1, inner_k=50, inner_delta=delta,
                     flags=oracle.ADAPTIVE_INNER)
    H = p.H0.astype(np.float64)
    d = []
    for _ in range(11):
        Hn = oracle.nnls_h(p.X, p.W0, H, 1)
        d.append(np.linalg.norm(Hn - H))
        H = Hn
    stop = next((l for l in range(2, 12) if d[l - 1] <= delta * d[0]), 11)
    assert 2 < stop < 11, "the case should stop strictly inside the cap"
    assert a["sweeps"][0, 0] == stop


def test_adaptive_replay_of_own_sweep_counts_is_identical():
    """Forcing the adaptive loop to the counts it chose reproduces the run,
    and the recorded closest calls are positive where a test was made."""
    p = S.lowrank(2, r=12)
    a = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=25, inner_k=50, flags=oracle.ADAPTIVE_INNER)
    b = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=25, inner_k=50, flags=oracle.ADAPTIVE_INNER,
                     sweeps_replay=a["sweeps"])
    np.testing.assert_array_equal(a["trace"], b["trace"])
    np.testing.assert_array_equal(a["sweeps"], b["sweeps"])
    assert np.all(a["sweep_margin"][a["sweeps"] >= 2] > 0)


@pytest.mark.parametrize("flag", [oracle.ROUND_F32, oracle.ROUND_F32_RZ])
def test_fp32_storage_probes_store_fp32_values_near_the_fp64_run(flag):
    """The conditioning probes of the parity protocol: every stored iterate
    is an FP32 value, and over a few iterations the run stays within a few
    FP32 units of the FP64 run (they perturb, they do not change the method)."""
    p = S.fullrank(6, m=30, n=25, r=4)
    a = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=5)
    b = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=5, flags=flag, replay=a["accepted"])
    for key in ("W", "H"):
        np.testing.assert_array_equal(b[key], b[key].astype(np.float32).astype(np.float64))
        assert 0 < np.abs(b[key] - a[key]).max() < 1e-4 * np.abs(a[key]).max()
    np.testing.assert_allclose(b["trace"], a["trace"], rtol=1e-5)


@pytest.mark.parametrize("hp,kw", [(3, {}), (1, {}), (2, dict(beta0=0.9, gamma=1.1)),
                                   (3, dict(flags=oracle.EXACT_NNLS)),
                                   (3, dict(flags=oracle.ADAPTIVE_INNER, inner_k=8))])
def test_resume_from_a_saved_state_is_bitwise_uninterrupted(hp, kw):
    """Checkpoint / resume: a solve stopped after 17 iterations and resumed
    from its saved state reproduces the uninterrupted solve bit for bit
    (iterates, trace, decisions, betas), restarts included."""
    p = S.fullrank(7, m=45, n=38, r=6)
    kw = dict(dict(hp=hp, max_iter=40), **kw)
    full = oracle.solve(p.X, p.r, p.W0, p.H0, **kw)
    first = oracle.solve(p.X, p.r, p.W0, p.H0, save=True, **dict(kw, max_iter=17))
    st = first["state"]
    assert st["k"] == 17
    rest = oracle.solve(p.X, p.r, p.W0, p.H0, resume=st, **kw)
    assert rest["n_iter"] == full["n_iter"] == 40
    assert (~full["accepted"]).any() or hp == 1, "the case should include restarts"
    np.testing.assert_array_equal(rest["W"], full["W"])
    np.testing.assert_array_equal(rest["H"], full["H"])
    np.testing.assert_array_equal(rest["trace"][17:], full["trace"][17:])
    np.testing.assert_array_equal(first["trace"], full["trace"][:18])
    np.testing.assert_array_equal(rest["accepted"][17:], full["accepted"][17:])
    np.testing.assert_array_equal(rest["beta"][17:], full["beta"][17:])


def test_resume_keeps_the_tol_rule():
    p = S.lowrank(0, m=30, n=30, r=3)
    full = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=5000, tol=1e-6)
    k = full["n_iter"]
    first = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=k - 1, tol=1e-6, save=True)
    rest = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=5000, tol=1e-6, resume=first["state"])
    assert rest["n_iter"] == k
    np.testing.assert_array_equal(rest["W"], full["W"])
