"""X stored in 16 bits (BF16, FP16) with the 16-bit matrix-core product: the
final error against the FP64 oracle on the FP32 X at the stated accuracy
(1e-3 absolute), over every padded rank class and ragged shapes (partial
256-row workgroups, partial K-chunks, a single row or column); and the
product itself against the FP64 vector product over the same 16-bit X.
"""
import numpy as np
import pytest

import nmf_synth as S
import oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1805_06604_amd")

ALG = dict(hp=3, beta0=0.5, gamma=1.05, gamma_bar=1.01, eta=1.5, inner_k=10)


def quantized(X, xd):
    """X rounded to the 16-bit storage type (round to nearest even)."""
    X = np.ascontiguousarray(X, np.float32)
    if xd == "F16":
        return X.astype(np.float16).astype(np.float32)
    u = X.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _run(p, max_iter, **kw):
    print(f"case {p.name} seed={p.seed} m={p.m} n={p.n} r={p.r} {kw}", flush=True)
    with P.Solver(p.X, p.r, max_iter=max_iter, **kw) as s:
        return s.solve(p.W0, p.H0)


@pytest.mark.parametrize("xd", ["BF16", "F16"])
@pytest.mark.parametrize("m,n,r", [(301, 157, 13), (157, 301, 33), (520, 260, 48),
                                   (700, 390, 64), (1, 40, 1), (40, 1, 1)])
def test_final_error_ragged(xd, m, n, r):
    """Final error within 1e-3 absolute of the oracle's. Only where the
    rank reaches min(m, n) (the single row and column), so that the oracle
    fits X exactly, is the bound widened by the storage rounding itself,
    q = ||X - X_q||_F / ||X||_F: the 16-bit X_q is then fitted exactly
    instead, which leaves an error of about q against X."""
    p = S.planted(7, m=m, n=n, r=r)
    g = _run(p, 40, x_dtype=P.XDtype[xd], prod=P.Prod.MFMA_FAST, **ALG)
    ref = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=40, **ALG)
    got = oracle.rel_error(p.X, g.W, g.H)
    X = p.X.astype(np.float64)
    q = np.linalg.norm(X - quantized(p.X, xd)) / np.linalg.norm(X)
    exact_fit = p.r >= min(p.m, p.n)
    print(f"  rho gpu {got:.6e} oracle {ref['trace'][-1]:.6e} q {q:.2e} "
          f"exact fit {exact_fit}", flush=True)
    assert abs(got - ref["trace"][-1]) < 1e-3 + (q if exact_fit else 0.0)


@pytest.mark.parametrize("xd", ["BF16", "F16"])
def test_product_against_fp64_products(xd):
    """Same 16-bit X, products on the 16-bit matrix cores (factor carried to 16
    significant bits for BF16, 22 for FP16; FP32 sums) against exact FP64
    products: over the first iterations the traces agree to within the
    product's accuracy."""
    p = S.planted(8, m=900, n=700, r=40)
    kw = dict(x_dtype=P.XDtype[xd], **ALG)
    a = _run(p, 8, prod=P.Prod.MFMA_FAST, **kw)
    b = _run(p, 8, prod=P.Prod.VALU, **kw)
    print("  trace dev", np.max(np.abs(a.trace - b.trace) / b.trace), flush=True)
    np.testing.assert_allclose(a.trace, b.trace, rtol=1e-4)


def test_bf16_runs_are_bitwise_deterministic():
    p = S.planted(9, m=600, n=500, r=24)
    kw = dict(x_dtype=P.XDtype.BF16, prod=P.Prod.MFMA_FAST, **ALG)
    a = _run(p, 10, **kw)
    b = _run(p, 10, **kw)
    np.testing.assert_array_equal(a.trace, b.trace)
    np.testing.assert_array_equal(a.W, b.W)
    np.testing.assert_array_equal(a.H, b.H)


@pytest.mark.parametrize("xd", ["BF16", "F16"])
def test_factor_columns_of_very_different_scales(xd):
    """Factor columns scaled by 2^-24 .. 2^12 (and the rows of H0 by the
    inverse, so that W0 H0 is unchanged), X already representable in the
    16-bit type: after one outer iteration every row of H and every column of
    W matches the FP64 oracle on the same X to 1e-3 relative. FP16 factor
    parts without their per-column scale would underflow to zero on the small
    columns and overflow on the large rows."""
    p = S.planted(9, m=300, n=260, r=16)
    Xq = quantized(p.X, xd)
    s = np.exp2(np.linspace(-24, 12, p.r)).astype(np.float32)
    W0 = (p.W0 * s[None, :]).astype(np.float32)
    H0 = (p.H0 / s[:, None]).astype(np.float32)
    print(f"case {xd} m={p.m} n={p.n} r={p.r} column scales 2^-24..2^12", flush=True)
    with P.Solver(Xq, p.r, max_iter=1, x_dtype=P.XDtype[xd], prod=P.Prod.MFMA_FAST, **ALG) as sv:
        g = sv.solve(W0, H0)
    ref = oracle.solve(Xq, p.r, W0, H0, max_iter=1, **ALG)
    assert np.array_equal(g.accepted, ref["accepted"])
    dh = np.linalg.norm(g.H - ref["H"], axis=1) / np.linalg.norm(ref["H"], axis=1)
    dw = np.linalg.norm(g.W - ref["W"], axis=0) / np.linalg.norm(ref["W"], axis=0)
    print(f"  max relative deviation: rows of H {dh.max():.2e}, columns of W {dw.max():.2e}",
          flush=True)
    assert np.all(np.isfinite(g.W)) and np.all(np.isfinite(g.H))
    assert dh.max() < 1e-3 and dw.max() < 1e-3
