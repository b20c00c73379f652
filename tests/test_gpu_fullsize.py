"""Full-size GPU checks on the configurations the benchmark times: planted
dense 16384 x 16384, r = 64 (FP32 X, the benchmark's parameters), and the
image-like 10000 x 2000, r = 49. The oracle cannot run these whole, so the
first outer iteration is checked on outputs it computes one by one: the
update of sampled columns of H (K HALS sweeps, or the exact NNLS) from the
initial iterate, and of sampled rows of W from the GPU's own H_w; and the
error trace against the explicit FP64 residual of the iterates.
"""
import numpy as np
import pytest

import nmf_synth as S
import oracle
from parity import FACTOR_RTOL, TRACE_RTOL, rel_fro

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1805_06604_amd")

BENCH = dict(beta0=0.5, gamma=1.01, gamma_bar=1.005, eta=1.5)
EXACT = dict(beta0=0.5, gamma=1.1, gamma_bar=1.05, eta=1.5)
SAMPLES = 24


def residual(X, W, H, block=2048):
    """||X - W H||_F / ||X||_F in FP64, a block of rows at a time."""
    W = np.asarray(W, np.float64)
    H = np.asarray(H, np.float64)
    num = den = 0.0
    for i in range(0, X.shape[0], block):
        Xb = X[i:i + block].astype(np.float64)
        R = Xb - W[i:i + block] @ H
        num += float(np.einsum("ij,ij->", R, R))
        den += float(np.einsum("ij,ij->", Xb, Xb))
    return np.sqrt(num / den)


def check_first_iteration(p, hp, K, exact, alg):
    rule = P.Inner.EXACT if exact else P.Inner.FIXED
    print(f"case full-size {p.name} m={p.m} n={p.n} r={p.r} hp={hp} K={K} "
          f"rule={rule.name} {alg}", flush=True)
    with P.Solver(p.X, p.r, max_iter=1, hp=hp, inner_k=K, inner_rule=rule, **alg) as s:
        g = s.solve(p.W0, p.H0)
    assert g.n_iter == 1 and g.accepted[0]
    rng = np.random.default_rng(7)
    cols = np.sort(rng.choice(p.n, SAMPLES, replace=False))
    rows = np.sort(rng.choice(p.m, SAMPLES, replace=False))
    W0 = p.W0.astype(np.float64)
    H0 = p.H0.astype(np.float64)

    # H_n: sampled columns from H_0 with W_y = W_0.
    Xc = np.ascontiguousarray(p.X[:, cols], dtype=np.float64)
    if exact:
        Hs = oracle.nnls_exact_h(Xc, W0, H0[:, cols])
    else:
        Hs = oracle.nnls_h(Xc, W0, H0[:, cols], K)
    dh = rel_fro(g.H[:, cols], Hs)

    # H_w from the GPU's H_n as stored (FP32), then sampled rows of W_n.
    Hn = g.H.astype(np.float64)
    if hp == 1:
        Hw = Hn
    else:
        Hy = Hn + alg["beta0"] * (Hn - H0)
        if hp == 3:
            Hy = np.maximum(Hy, 0.0)
        Hw = Hy.astype(np.float32).astype(np.float64)
    Xr = np.ascontiguousarray(p.X[rows], dtype=np.float64)
    if exact:
        Ws = oracle.nnls_exact_w(Xr, Hw, W0[rows])
    else:
        Ws = oracle.nnls_w(Xr, Hw, W0[rows], K)
    dw = rel_fro(g.W[rows], Ws)

    rho0 = residual(p.X, W0, H0)
    rho1 = residual(p.X, g.W, Hw)
    t0 = abs(g.trace[0] - rho0) / rho0
    t1 = abs(g.trace[1] - rho1) / rho1
    print(f"full-size: H cols {dh:.2e} W rows {dw:.2e} rho0 {rho0:.6e} ({t0:.1e}) "
          f"rho1 {rho1:.6e} ({t1:.1e})", flush=True)
    assert dh <= FACTOR_RTOL and dw <= FACTOR_RTOL, (dh, dw)
    assert t0 <= TRACE_RTOL and t1 <= TRACE_RTOL, (t0, t1)


@pytest.fixture(scope="module")
def planted():
    return S.planted(0)


def test_planted_16384_r64_bench_configuration(planted):
    check_first_iteration(planted, 3, 10, False, BENCH)


def test_planted_16384_r64_exact_nnls(planted):
    check_first_iteration(planted, 1, 10, True, EXACT)


@pytest.mark.parametrize("exact", [False, True])
def test_imagelike_10000x2000_r49(exact):
    p = S.imagelike(0)
    check_first_iteration(p, 3 if not exact else 1, 10, exact, EXACT if exact else BENCH)


@pytest.mark.parametrize("xd", ["BF16", "F16"])
def test_planted_16384_r64_16bit_x(planted, xd):
    """The benchmark configuration with X stored in 16 bits (16-bit matrix-core
    products): after 30 iterations the final error, evaluated in FP64 against
    the FP32 X, is within 1e-3 absolute of the FP32 path's at the same
    iteration (the FP32 path being the one checked against the oracle
    above)."""
    p = planted
    kw = dict(max_iter=30, hp=3, inner_k=10, **BENCH)
    print(f"case full-size {p.name} m={p.m} n={p.n} r={p.r} x_dtype={xd} {kw}", flush=True)
    with P.Solver(p.X, p.r, x_dtype=P.XDtype[xd], prod=P.Prod.MFMA_FAST, **kw) as s:
        a = s.solve(p.W0, p.H0)
    with P.Solver(p.X, p.r, **kw) as s:
        b = s.solve(p.W0, p.H0)
    ra = residual(p.X, a.W, a.H)
    rb = residual(p.X, b.W, b.H)
    print(f"full-size {xd}: rho {ra:.6e} FP32 path {rb:.6e}", flush=True)
    assert abs(ra - rb) < 1e-3
