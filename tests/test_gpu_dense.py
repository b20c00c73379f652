"""GPU parity of the dense E-A-HALS path against the FP64 oracle.

Every case is seeded and prints its name before running, so that a failing
case can be identified from the log alone.
"""
import numpy as np
import pytest

import nmf_synth as S
import oracle
from parity import compare_to_oracle, rel_fro

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1805_06604_amd")


def _run(p, max_iter, **kw):
    print(f"case {p.name} seed={p.seed} m={p.m} n={p.n} r={p.r} {kw}", flush=True)
    with P.Solver(p.X, p.r, max_iter=max_iter, **kw) as s:
        return s.solve(p.W0, p.H0)


ALG = dict(beta0=0.5, gamma=1.05, gamma_bar=1.01, eta=1.5, inner_k=10)

# Product paths held to the full parity bound: FP64 vector products and the
# exact-integer matrix-core products.
PRODS = ["VALU", "MFMA_EXACT"]


@pytest.mark.parametrize("prod", PRODS)
@pytest.mark.parametrize("hp", [1, 2, 3])
def test_fullrank_200(hp, prod):
    """Full-rank synthetic (section 5.1): 200 x 200 U[0,1], r = 20, 50
    iterations (for hp = 2 the extrapolated H turns negative at the first
    step and the method collapses to W = 0, in the oracle as well)."""
    p = S.fullrank(0)
    g = _run(p, 50, hp=hp, prod=P.Prod[prod], **ALG)
    compare_to_oracle(p, g, 50, hp=hp, **ALG)


@pytest.mark.parametrize("prod", PRODS)
@pytest.mark.parametrize("seed", [0, 1])
def test_lowrank_200_r10(seed, prod):
    """Low-rank synthetic 200 x 200, r = 10: rho falls towards 0."""
    p = S.lowrank(seed)
    g = _run(p, 50, hp=3, prod=P.Prod[prod], **ALG)
    compare_to_oracle(p, g, 50, hp=3, **ALG)


@pytest.mark.parametrize("prod", PRODS)
def test_hp2_lowrank(prod):
    """hp = 2 (H extrapolated, not projected) on low-rank data whose initial
    scale matches X."""
    p = S.lowrank(1, r=12)
    g = _run(p, 50, hp=2, prod=P.Prod[prod], **ALG)
    compare_to_oracle(p, g, 50, hp=2, **ALG)


@pytest.mark.parametrize("prod", PRODS)
@pytest.mark.parametrize("m,n,r", [(301, 157, 13), (157, 301, 33), (97, 413, 48),
                                   (520, 260, 64), (1, 40, 1), (40, 1, 1), (64, 64, 16)])
def test_ragged_shapes(m, n, r, prod):
    """Shapes that leave partial tiles and partial row blocks, every padded
    rank class (16, 32, 48, 64), and the degenerate single row / column
    (exactly factorable: rho reaches the FP64 floor)."""
    p = S.fullrank(3, m=m, n=n, r=r)
    g = _run(p, 50, hp=3, prod=P.Prod[prod], **ALG)
    compare_to_oracle(p, g, 50, hp=3, **ALG)


@pytest.mark.parametrize("prod", PRODS)
def test_imagelike(prod):
    """Image-like dense data (the stand-in for the face sets), r = 49: a
    chaotic trajectory, where FP32 storage alone moves the oracle by ~4e-4
    after 50 iterations."""
    p = S.imagelike(0, m=1000, n=300, r=49)
    g = _run(p, 50, hp=3, prod=P.Prod[prod], **ALG)
    compare_to_oracle(p, g, 50, hp=3, **ALG)


@pytest.mark.parametrize("xd", ["BF16", "F16"])
def test_16bit_x_final_error(xd):
    """X stored in BF16 / FP16 (products FP32-accumulated): the final
    relative error, evaluated in FP64 against the FP32 X, is within 1e-3
    absolute of the oracle's on the FP32 X."""
    p = S.planted(4, m=640, n=480, r=24)
    kw = dict(hp=3, **ALG)
    g = _run(p, 60, x_dtype=P.XDtype[xd], **kw)
    ref = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=60, **kw)
    got = oracle.rel_error(p.X, g.W, g.H)
    print(f"16-bit X {xd}: rho gpu {got:.6e} oracle {ref['trace'][-1]:.6e}", flush=True)
    assert abs(got - ref["trace"][-1]) < 1e-3


def test_beta_zero_is_monotone():
    p = S.fullrank(5, m=250, n=180, r=12)
    g = _run(p, 40, hp=3, beta0=0.0, gamma=1.05, gamma_bar=1.01, eta=1.5, prod=P.Prod.VALU)
    assert g.accepted.all()
    assert np.all(np.diff(g.trace) <= 1e-6 * g.trace[:-1])


def test_max_iter_zero_reports_initial_error():
    p = S.fullrank(6, m=50, n=40, r=4)
    g = _run(p, 0)
    want = oracle.rel_error(p.X, p.W0, p.H0)
    assert g.n_iter == 0
    assert g.trace[0] == pytest.approx(want, rel=1e-6)
    np.testing.assert_array_equal(g.W, p.W0)
    np.testing.assert_array_equal(g.H, p.H0)


def test_trace_is_residual_of_returned_iterate():
    """hp = 3 with beta = 0: every iterate is feasible and the last trace
    entry is the residual of the returned pair, which the oracle evaluates
    explicitly in FP64."""
    p = S.fullrank(7, m=180, n=220, r=20)
    g = _run(p, 20, hp=3, beta0=0.0, gamma=1.05, gamma_bar=1.01, eta=1.5, prod=P.Prod.VALU)
    assert g.W.min() >= 0 and g.H.min() >= 0
    want = oracle.rel_error(p.X, g.W, g.H)
    assert g.trace[-1] == pytest.approx(want, rel=1e-5)


def test_runs_are_bitwise_deterministic():
    p = S.fullrank(8, m=300, n=260, r=24)
    with P.Solver(p.X, p.r, max_iter=20, hp=3, **ALG) as s:
        a = s.solve(p.W0, p.H0)
        b = s.solve(p.W0, p.H0)
    np.testing.assert_array_equal(a.trace, b.trace)
    np.testing.assert_array_equal(a.W, b.W)
    np.testing.assert_array_equal(a.H, b.H)


def test_many_block_reductions_are_deterministic():
    """The Gram and objective partials of many workgroups (here 12 and 10 per
    sweep) are finished by whichever workgroup arrives last, on any XCD; the
    result must not depend on that order: repeated solves agree bitwise and
    stay at parity with the oracle."""
    p = S.fullrank(11, m=3000, n=2500, r=16)
    kw = dict(hp=3, prod=P.Prod.MFMA_EXACT, **ALG)
    runs = []
    with P.Solver(p.X, p.r, max_iter=15, **kw) as s:
        for _ in range(4):
            runs.append(s.solve(p.W0, p.H0))
    for g in runs[1:]:
        np.testing.assert_array_equal(g.trace, runs[0].trace)
        np.testing.assert_array_equal(g.W, runs[0].W)
    compare_to_oracle(p, runs[0], 15, hp=3, **ALG)


def test_tol_stop_matches_oracle():
    p = S.lowrank(2, m=120, n=90, r=6)
    kw = dict(hp=3, tol=1e-4, **ALG)
    g = _run(p, 500, prod=P.Prod.VALU, **kw)
    ref = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=500, **kw)
    assert g.n_iter == ref["n_iter"]
    assert g.n_iter < 500


def test_invalid_initial_iterate_rejected():
    p = S.fullrank(9, m=20, n=30, r=3)
    W0 = p.W0.copy()
    W0[3, 1] = -1.0
    with P.Solver(p.X, p.r, max_iter=5) as s:
        with pytest.raises(P.NMFError) as e:
            s.solve(W0, p.H0)
        assert e.value.status == P.Status.E_INVAL
        # the context stays usable after a rejected call
        g = s.solve(p.W0, p.H0)
        assert g.n_iter == 5


def test_device_pointer_interface_matches_host():
    torch = pytest.importorskip("torch")
    p = S.fullrank(10, m=210, n=190, r=17)
    with P.Solver(p.X, p.r, max_iter=15, hp=3, **ALG) as s:
        host = s.solve(p.W0, p.H0)
        dev = torch.device("cuda:0")
        W0 = torch.from_numpy(p.W0).to(dev)
        H0 = torch.from_numpy(p.H0).to(dev)
        stream = torch.cuda.current_stream()
        s.start(W0, H0, stream=stream)
        s.iterate(7, stream=stream)
        s.iterate(100, stream=stream)       # clamped at max_iter
        W = torch.empty((p.m, p.r), device=dev)
        H = torch.empty((p.r, p.n), device=dev)
        out = s.read(W, H, stream=stream)
    assert out.n_iter == 15
    np.testing.assert_array_equal(out.trace, host.trace)
    np.testing.assert_array_equal(W.cpu().numpy(), host.W)
    np.testing.assert_array_equal(H.cpu().numpy(), host.H)


@pytest.mark.parametrize("prod", PRODS)
@pytest.mark.parametrize("which", ["fullrank", "lowrank"])
def test_beta_star_diagnostic(which, prod):
    """The beta* of section 4 per iteration against the oracle's, and the
    diagnostic leaves the iterates unchanged. Tolerance per iteration: the
    larger of 1e-6 (1 + |beta*|) and 3x the move of the oracle's beta* when
    its iterates are rounded to FP32 (beta* divides by ||dW H_w||^2, which
    shrinks as the iterates settle)."""
    p = S.fullrank(0) if which == "fullrank" else S.lowrank(0)
    kw = dict(hp=3, **ALG)
    print(f"case beta* {which} {prod}", flush=True)
    with P.Solver(p.X, p.r, max_iter=30, prod=P.Prod[prod], flags=P.FLAG_BETA_STAR, **kw) as s:
        g = s.solve(p.W0, p.H0)
        bs = s.read_beta_star()
    g0 = _run(p, 30, prod=P.Prod[prod], **kw)
    assert np.array_equal(g.trace, g0.trace) and np.array_equal(g.W, g0.W)
    ref = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=30, replay=g.accepted, **kw)
    f32 = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=30, replay=g.accepted,
                       flags=oracle.ROUND_F32, **kw)
    bo, bf = ref["beta_star"], f32["beta_star"]
    tol = np.maximum(1e-6 * (1 + np.abs(bo)), 3 * np.abs(bf - bo))
    print("beta*", np.round(bo[:8], 4), "max dev", np.max(np.abs(bs - bo)), flush=True)
    assert bs.shape == bo.shape
    assert np.all(np.abs(bs - bo) <= tol), np.max(np.abs(bs - bo) / tol)
