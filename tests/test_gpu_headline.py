"""Fifty outer iterations against the oracle on the benchmark's workloads at
sizes the oracle finishes in about a minute:

  * the planted dense problem (X = W H + 1e-3 |N(0,1)|, W, H ~ U[0,1]) at
    2048 x 2048, r = 64, with the benchmark's parameters (hp 3, beta0 0.5,
    gamma 1.01, gamma_bar 1.005, eta 1.5, K = 10): the exact-integer
    product path by the full parity protocol, and X stored in BF16 and FP16
    (16-bit matrix-core products) by the final error against the FP32 X,
    within 1e-3 absolute of the oracle's on the FP32 X;
  * the image-like 10000 x 2000, r = 49 set at its full size (the stand-in
    for the face-image sets), by the full parity protocol.

The oracle evaluates e(k) by Remark 1 here (its plain definition, the
explicit residual, costs another O(mnr) per iteration; the two agree to
about 1e-12 relative, which an oracle pin checks).
"""
import numpy as np
import pytest

import nmf_synth as S
import oracle
from parity import compare_to_oracle, oracle_pair

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1805_06604_amd")

BENCH = dict(hp=3, beta0=0.5, gamma=1.01, gamma_bar=1.005, eta=1.5, inner_k=10)
ITERS = 50


def _run(p, **kw):
    print(f"case {p.name} seed={p.seed} m={p.m} n={p.n} r={p.r} {kw}", flush=True)
    with P.Solver(p.X, p.r, max_iter=ITERS, **kw) as s:
        return s.solve(p.W0, p.H0)


def residual(X, W, H):
    """||X - W H||_F / ||X||_F in FP64 (numpy, on the host)."""
    Xd = X.astype(np.float64)
    R = Xd - np.asarray(W, np.float64) @ np.asarray(H, np.float64)
    return float(np.linalg.norm(R) / np.linalg.norm(Xd))


@pytest.fixture(scope="module")
def planted2048():
    p = S.planted(0, m=2048, n=2048, r=64)
    print("oracle: planted 2048 x 2048, r = 64, 50 iterations (and its FP32-storage "
          "rerun)", flush=True)
    pair = oracle_pair(p, ITERS, None, oracle.ERR_REMARK1, **BENCH)
    return p, pair


def test_planted_2048_r64_exact_integer_products(planted2048):
    p, pair = planted2048
    g = _run(p, prod=P.Prod.MFMA_EXACT, **BENCH)
    compare_to_oracle(p, g, ITERS, oracle_flags=oracle.ERR_REMARK1, pair=pair, **BENCH)


@pytest.mark.parametrize("xd", ["BF16", "F16"])
def test_planted_2048_r64_16bit_x(planted2048, xd):
    """X stored in 16 bits changes the problem (X_q != X); the result is
    judged by its error against the FP32 X, evaluated in FP64 on the host,
    which must be within 1e-3 of the oracle's final error on the FP32 X."""
    p, (ref, _) = planted2048
    g = _run(p, x_dtype=P.XDtype[xd], prod=P.Prod.MFMA_FAST, **BENCH)
    got = residual(p.X, g.W, g.H)
    want = oracle.rel_error(p.X, ref["W"], ref["H"])
    print(f"  {xd}: rho(W, H) vs FP32 X {got:.6e}, oracle {want:.6e}, "
          f"gap {abs(got - want):.2e}", flush=True)
    assert g.n_iter == ITERS
    assert abs(got - want) < 1e-3


def test_imagelike_full_size_50_iterations():
    p = S.imagelike(0)
    alg = dict(hp=3, beta0=0.5, gamma=1.05, gamma_bar=1.01, eta=1.5, inner_k=10)
    g = _run(p, prod=P.Prod.MFMA_EXACT, **alg)
    print("oracle: image-like 10000 x 2000, r = 49, 50 iterations", flush=True)
    compare_to_oracle(p, g, ITERS, oracle_flags=oracle.ERR_REMARK1, **alg)
