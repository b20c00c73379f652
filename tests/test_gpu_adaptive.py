"""GPU parity of the adaptive inner loop (the A-HALS rule the paper refers to
for updating the rows several times; recalled from the cited work, so the
rule itself is pinned only by its reductions to the fixed loop) against the
oracle in the same mode: the error trace, the factors and the number of
sweeps taken on each side in every iteration.
"""
import numpy as np
import pytest

import nmf_synth as S
import oracle
from parity import compare_to_oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1805_06604_amd")

ALG = dict(beta0=0.5, gamma=1.01, gamma_bar=1.005, eta=1.5)


def _run(p, max_iter, inner_k=50, inner_alpha=0.5, inner_delta=0.1, **kw):
    print(f"case adaptive {p.name} seed={p.seed} m={p.m} n={p.n} r={p.r} K<={inner_k} "
          f"alpha={inner_alpha} delta={inner_delta} {kw}", flush=True)
    with P.Solver(p.X, p.r, max_iter=max_iter, inner_rule=P.Inner.ADAPTIVE, inner_k=inner_k,
                  inner_alpha=inner_alpha, inner_delta=inner_delta, **kw) as s:
        g = s.solve(p.W0, p.H0)
        sw = s.read_sweeps()
    return g, sw


# A sweep count may differ from the oracle's only where the oracle's own
# stopping test was a near tie (relative margin below this).
SWEEP_FLIP = 1e-4


def _check(p, max_iter, inner_k=50, inner_alpha=0.5, inner_delta=0.1, prod=None, **kw):
    gkw = dict(kw) if prod is None else dict(kw, prod=prod)
    g, sw = _run(p, max_iter, inner_k, inner_alpha, inner_delta, **gkw)
    okw = dict(kw, inner_k=inner_k, inner_alpha=inner_alpha, inner_delta=inner_delta)
    own = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=max_iter, replay=g.accepted,
                       flags=oracle.ADAPTIVE_INNER, **okw)
    diff = np.argwhere(sw != own["sweeps"][:len(sw)])
    print("sweeps gpu", sw[:8].tolist(), "oracle", own["sweeps"][:8].tolist(),
          f"differing (iteration, side): {diff[:4].tolist()}", flush=True)
    if len(diff):
        k, side = diff[0]
        mg = own["sweep_margin"][k, side]
        assert mg < SWEEP_FLIP, f"sweep count differs at iteration {k + 1} with margin {mg:.2e}"
    # The rest against the oracle forced to the GPU's counts.
    compare_to_oracle(p, g, max_iter, oracle_flags=oracle.ADAPTIVE_INNER, sweeps_replay=sw, **okw)
    return sw


@pytest.mark.parametrize("hp", [1, 3])
def test_lowrank_200_r10(hp):
    """Cap 11 on both sides; the early stop ends most loops sooner."""
    sw = _check(S.lowrank(0), 50, hp=hp, **ALG)
    assert sw.min() >= 1 and sw.max() <= 11 and sw.min() < 11


def test_fullrank_200_r20():
    _check(S.fullrank(0), 50, hp=3, **ALG)


def test_lowrank_exact_integer_products():
    """The benchmark's product kernel with the adaptive loop."""
    _check(S.lowrank(2, m=300, n=250, r=16), 40, hp=3, prod=P.Prod.MFMA_EXACT, **ALG)


@pytest.mark.parametrize("m,n,r", [(301, 157, 13), (157, 301, 33), (97, 413, 48), (520, 260, 64)])
def test_ragged_shapes(m, n, r):
    """Every padded rank class and unequal caps on the two sides. The
    products are the FP64 ones: on these trajectories a loop stopped after
    two or three sweeps amplifies input perturbations about 20-fold (the
    oracle's own FP32-storage rerun moves W by 1.4e-6 after one iteration,
    against 6e-8 with four fixed sweeps), and the exact-integer products'
    2^-27 scale error then grows past the factor bound within 30
    iterations while the trace still agrees to 1e-7. The adaptive loop does
    not touch the products; they have their own parity tests."""
    _check(S.fullrank(3, m=m, n=n, r=r), 30, hp=3, prod=P.Prod.VALU, **ALG)


def test_zero_delta_runs_the_cap():
    p = S.lowrank(1, r=12)
    sw = _check(p, 20, inner_delta=0.0, hp=3, **ALG)
    assert np.all(sw == sw[0, 0])


def test_sparse_x():
    _check(S.doclike(1, m=1500, n=1100, r=20, nnz=16000), 30, hp=3, **ALG)


def test_fixed_rule_reports_inner_k():
    p = S.fullrank(4, m=120, n=90, r=8)
    with P.Solver(p.X, p.r, max_iter=5, inner_k=7, hp=3, **ALG) as s:
        s.solve(p.W0, p.H0)
        assert np.all(s.read_sweeps() == 7)


def test_beta_star_with_the_adaptive_loop():
    """beta* with the adaptive loop against the oracle forced to the GPU's
    sweep counts."""
    p = S.lowrank(3)
    kw = dict(hp=3, **ALG)
    with P.Solver(p.X, p.r, max_iter=25, inner_rule=P.Inner.ADAPTIVE, inner_k=50,
                  flags=P.FLAG_BETA_STAR, **kw) as s:
        g = s.solve(p.W0, p.H0)
        bs = s.read_beta_star()
        sw = s.read_sweeps()
    okw = dict(kw, inner_k=50, replay=g.accepted, sweeps_replay=sw)
    ref = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=25, flags=oracle.ADAPTIVE_INNER, **okw)
    f32 = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=25,
                       flags=oracle.ADAPTIVE_INNER | oracle.ROUND_F32, **okw)
    bo, bf = ref["beta_star"], f32["beta_star"]
    tol = np.maximum(1e-6 * (1 + np.abs(bo)), 3 * np.abs(bf - bo))
    print("beta* (adaptive)", np.round(bo[:8], 4), "max dev", np.max(np.abs(bs - bo)), flush=True)
    assert np.all(np.abs(bs - bo) <= tol), np.max(np.abs(bs - bo) / tol)


def test_given_cost_ratios_set_the_caps():
    """Cost ratios given per side (as measured on the device, instead of the
    flop ratio): rho_H = 7 and rho_W = 3 cap the loops at 4 and 2 sweeps, and
    with delta = 0 every iteration runs exactly those counts, against the
    oracle with the same ratios."""
    sw = _check(S.lowrank(3, m=260, n=300, r=12), 30, hp=3, inner_delta=0.0,
                inner_rho_h=7.0, inner_rho_w=3.0, **ALG)
    assert np.all(sw[:, 0] == 4) and np.all(sw[:, 1] == 2)


def test_given_cost_ratios_with_the_early_stop():
    """The same ratios at delta = 0.1: the caps bound the counts and the
    early stop decides below them, as the oracle's."""
    sw = _check(S.lowrank(4, m=260, n=300, r=12), 30, hp=3, inner_rho_h=7.0,
                inner_rho_w=3.0, **ALG)
    assert sw[:, 0].max() <= 4 and sw[:, 1].max() <= 2
