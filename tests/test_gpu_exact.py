"""GPU parity of E-ANLS (Algorithm 2 with every block NNLS solved exactly,
section 1) against the FP64 oracle run with its exact NNLS: every padded
rank class, shapes with ragged row blocks, the plain ANLS special case, a
zero Gram diagonal, and sparse X.
"""
import numpy as np
import pytest

import nmf_synth as S
import oracle
from parity import compare_to_oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1805_06604_amd")

# The E-ANLS parameters chosen in section 5.3.1.
ALG = dict(beta0=0.5, gamma=1.1, gamma_bar=1.05, eta=1.5)


def _run(p, max_iter, **kw):
    print(f"case E-ANLS {p.name} seed={p.seed} m={p.m} n={p.n} r={p.r} {kw}", flush=True)
    with P.Solver(p.X, p.r, max_iter=max_iter, inner_rule=P.Inner.EXACT, **kw) as s:
        return s.solve(p.W0, p.H0)


def _compare(p, g, max_iter, **kw):
    return compare_to_oracle(p, g, max_iter, oracle_flags=oracle.EXACT_NNLS, **kw)


@pytest.mark.parametrize("hp", [1, 3])
def test_fullrank_200(hp):
    """Full-rank synthetic 200 x 200, r = 20 (padded rank 32)."""
    p = S.fullrank(0)
    g = _run(p, 50, hp=hp, **ALG)
    _compare(p, g, 50, hp=hp, **ALG)


def test_lowrank_200_r10():
    """Low-rank synthetic, r = 10 (padded rank 16, four problems per wave)."""
    p = S.lowrank(0)
    g = _run(p, 50, hp=1, **ALG)
    _compare(p, g, 50, hp=1, **ALG)


@pytest.mark.parametrize("m,n,r", [(301, 157, 13), (157, 301, 33), (97, 413, 48),
                                   (520, 260, 64), (1, 40, 1), (40, 1, 1)])
def test_ragged_shapes(m, n, r):
    """Partial row blocks of the exact solve (32 rows per workgroup) and of
    the epilogue, every padded rank class, and a single row or column."""
    p = S.fullrank(3, m=m, n=n, r=r)
    g = _run(p, 30, hp=3, **ALG)
    _compare(p, g, 30, hp=3, **ALG)


def test_plain_anls_is_monotone():
    """beta = 0 is ANLS: exact block descent never increases the error."""
    p = S.fullrank(5, m=250, n=180, r=12)
    g = _run(p, 40, hp=1, beta0=0.0, gamma=1.1, gamma_bar=1.05, eta=1.5)
    assert g.accepted.all()
    assert np.all(np.diff(g.trace) <= 1e-6 * g.trace[:-1])
    _compare(p, g, 40, hp=1, beta0=0.0, gamma=1.1, gamma_bar=1.05, eta=1.5)


def test_zero_gram_diagonal():
    """A zero column of W0: its coordinate of every H row has a zero Gram
    diagonal at the first H update and keeps its warm start."""
    p = S.fullrank(6, m=120, n=90, r=8)
    p.W0[:, 2] = 0.0
    g = _run(p, 20, hp=1, **ALG)
    _compare(p, g, 20, hp=1, **ALG)


def test_sparse_x():
    p = S.doclike(1, m=1500, n=1100, r=20, nnz=16000)
    g = _run(p, 30, hp=1, **ALG)
    _compare(p, g, 30, hp=1, **ALG)


def test_exact_runs_are_bitwise_deterministic():
    p = S.fullrank(8, m=300, n=260, r=24)
    with P.Solver(p.X, p.r, max_iter=15, hp=1, inner_rule=P.Inner.EXACT, **ALG) as s:
        a = s.solve(p.W0, p.H0)
        b = s.solve(p.W0, p.H0)
    np.testing.assert_array_equal(a.trace, b.trace)
    np.testing.assert_array_equal(a.W, b.W)
    np.testing.assert_array_equal(a.H, b.H)


def test_table4_eanls_full_rank_row():
    """Table 4's E-ANLS (hp = 1) row on the GPU: the mean final error over 10
    seeded 200 x 200, r = 20 full-rank data sets is within 3 standard errors
    of the printed 0.423795 (std 1.161e-3)."""
    fin = []
    for s in range(10):
        p = S.fullrank(s)
        fin.append(_run(p, 150, hp=1, **ALG).trace[-1])
    print(f"E-ANLS full-rank mean final rho {np.mean(fin):.6f}", flush=True)
    assert abs(np.mean(fin) - 0.423795) < 3 * 1.161e-3 / np.sqrt(10)


def test_table3_eanls_beats_anls_on_low_rank():
    """Table 3: on low-rank data E-ANLS (hp = 1) ends far below plain ANLS."""
    ext, plain = [], []
    for s in range(6):
        p = S.lowrank(s, r=20)
        ext.append(_run(p, 150, hp=1, **ALG).trace[-1])
        plain.append(_run(p, 150, hp=1, beta0=0.0, gamma=1.1, gamma_bar=1.05, eta=1.5).trace[-1])
    print(f"low-rank mean final rho: E-ANLS {np.mean(ext):.3e}, ANLS {np.mean(plain):.3e}", flush=True)
    assert np.mean(ext) < 0.1 * np.mean(plain)


def test_rank_one():
    """r = 1: every NNLS is one coordinate (max(0, c / g))."""
    p = S.fullrank(9, m=90, n=70, r=1)
    g = _run(p, 20, hp=1, **ALG)
    _compare(p, g, 20, hp=1, **ALG)


def test_tol_stop():
    """The tol stop (R12) ends E-ANLS at the oracle's iteration, with the
    oracle's trace up to there."""
    p = S.fullrank(10, m=150, n=120, r=10)
    g = _run(p, 200, hp=1, tol=1e-7, **ALG)
    ref = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=200, tol=1e-7, hp=1,
                       flags=oracle.EXACT_NNLS, **ALG)
    assert g.n_iter == ref["n_iter"] and g.n_iter < 200
    np.testing.assert_allclose(g.trace, ref["trace"], rtol=1e-5)


def test_beta_star_with_exact_blocks():
    """The beta* diagnostic of section 4 in E-ANLS, where W_n is an exact
    NNLS solution, against the oracle in its exact mode."""
    p = S.lowrank(0)
    kw = dict(hp=1, **ALG)
    with P.Solver(p.X, p.r, max_iter=30, inner_rule=P.Inner.EXACT, flags=P.FLAG_BETA_STAR, **kw) as s:
        g = s.solve(p.W0, p.H0)
        bs = s.read_beta_star()
    ref = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=30, replay=g.accepted,
                       flags=oracle.EXACT_NNLS, **kw)
    f32 = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=30, replay=g.accepted,
                       flags=oracle.EXACT_NNLS | oracle.ROUND_F32, **kw)
    bo, bf = ref["beta_star"], f32["beta_star"]
    tol = np.maximum(1e-6 * (1 + np.abs(bo)), 3 * np.abs(bf - bo))
    print("beta* (E-ANLS)", np.round(bo[:8], 4), "max dev", np.max(np.abs(bs - bo)), flush=True)
    assert np.all(np.abs(bs - bo) <= tol), np.max(np.abs(bs - bo) / tol)


def test_device_pointer_interface():
    """nmf_start / nmf_iterate / nmf_read on torch tensors give the host
    interface's result bit for bit."""
    torch = pytest.importorskip("torch")
    p = S.fullrank(11, m=160, n=140, r=12)
    kw = dict(hp=1, inner_rule=P.Inner.EXACT, **ALG)
    with P.Solver(p.X, p.r, max_iter=15, **kw) as s:
        a = s.solve(p.W0, p.H0)
        st = torch.cuda.current_stream()
        s.start(torch.from_numpy(p.W0).cuda(), torch.from_numpy(p.H0).cuda(), stream=st)
        s.iterate(15, stream=st)
        W = torch.empty((p.m, p.r), dtype=torch.float32, device="cuda")
        H = torch.empty((p.r, p.n), dtype=torch.float32, device="cuda")
        b = s.read(W, H, stream=st)
    np.testing.assert_array_equal(a.trace, b.trace)
    np.testing.assert_array_equal(a.W, W.cpu().numpy())
    np.testing.assert_array_equal(a.H, H.cpu().numpy())


@pytest.mark.parametrize("m,n,r", [(180, 150, 7), (200, 170, 20), (150, 260, 40), (240, 210, 64)])
def test_inverse_beside_product_matches_inverse_per_workgroup(m, n, r):
    """A single context takes G^-1 once per side on a second stream, beside the
    product before the solve; the batch engine's grouped solves invert G in
    every workgroup with the same code. Both therefore solve with the same
    inverse, and the runs agree to the products' rounding."""
    p = S.planted(11, m=m, n=n, r=r)
    print(f"case inverse placement m={m} n={n} r={r}", flush=True)
    kw = dict(hp=1, inner_rule=P.Inner.EXACT, **ALG)
    with P.Solver(p.X, p.r, max_iter=30, prod=P.Prod.MFMA_EXACT, **kw) as s:
        single = s.solve(p.W0, p.H0)
    res = None
    with P.Batch(1 << 28, max_active=4, check_every=5) as B:
        t = B.submit(p.X, p.r, p.W0, p.H0, max_iter=30, **kw)
        for _ in range(50):
            B.step(30)
            res = B.result(t)
            if res is not None:
                break
    assert res is not None and res.n_iter == single.n_iter
    np.testing.assert_allclose(res.trace, single.trace, rtol=1e-6)
    for a, b in ((res.W, single.W), (res.H, single.H)):
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b)


@pytest.mark.parametrize("rule", ["FIXED", "EXACT"])
def test_profiled_iterations_match_graph_iterations(rule):
    """Iterations launched one kernel at a time (nmf_profile; with exact
    solves, the inversions forked to the context's second stream and joined
    back outside any graph) interleaved with graph iterations reproduce a
    plain solve bitwise."""
    p = S.planted(12, m=300, n=260, r=24)
    kw = dict(hp=1, inner_rule=P.Inner[rule], inner_k=10, **ALG)
    print(f"case profiled/graph interleave rule={rule}", flush=True)
    with P.Solver(p.X, p.r, max_iter=20, **kw) as s:
        plain = s.solve(p.W0, p.H0)
    with P.Solver(p.X, p.r, max_iter=20, **kw) as s:
        s.start(p.W0, p.H0)
        s.iterate(5)
        ms = s.profile(5)
        s.iterate(10)
        mixed = s.read()
    assert all(v >= 0.0 for v in ms.values())
    assert mixed.n_iter == plain.n_iter == 20
    np.testing.assert_array_equal(mixed.trace, plain.trace)
    np.testing.assert_array_equal(mixed.W, plain.W)
    np.testing.assert_array_equal(mixed.H, plain.H)
