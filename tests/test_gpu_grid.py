"""GPU checks of the batched multi-start / parameter-grid runner (the tuning
protocol of section 5.3): grid runs against the FP64 oracle, the full-rank
rows of Table 4 and the low-rank ordering of Table 3, and the whole grid at
scale."""
import numpy as np
import pytest

import nmf_synth as S
from parity import compare_to_oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1805_06604_amd")
from paper_1805_06604_amd import grid as G  # noqa: E402


def test_grid_runs_match_oracle():
    probs = [S.fullrank(s) for s in range(2)]
    vs = [G.PLAIN, G.Variant(1, 0.75, 2.0, 1.05, 1.01), G.Variant(2, 0.25, 3.0, 1.1, 1.05),
          G.Variant(3, 0.5, 1.5, 1.01, 1.005), G.Variant(3, 0.75, 1.5, 1.005, 1.001)]
    print("grid parity: 5 variants x 2 data sets, 40 iterations", flush=True)
    res = G.run(probs, vs, 40)
    for v, row in zip(vs, res):
        for p, g in zip(probs, row):
            print(v.label(), f"seed={p.seed}", flush=True)
            compare_to_oracle(p, g, 40, inner_k=10, **v.params())


def test_table4_full_rank_rows():
    """Table 4 prints A-HALS 0.423815 +- 1.171e-3 and E-A-HALS (hp = 3,
    beta0 0.5, eta 1.5, gamma 1.01, gamma_bar 1.005) 0.423817 +- 1.184e-3 on
    200 x 200 U[0,1] data with r = 20: the means over 10 seeded data sets lie
    within 3 standard errors."""
    probs = [S.fullrank(s) for s in range(10)]
    vs = [G.PLAIN, G.Variant(3, 0.5, 1.5, 1.01, 1.005)]
    print("table 4 rows: 2 variants x 10 data sets, 300 iterations", flush=True)
    summ = G.summarize(vs, G.run(probs, vs, 300))
    plain, ext = summ["rows"]
    print(plain, ext, flush=True)
    assert abs(plain["rho_mean"] - 0.423815) < 3 * 1.171e-3 / np.sqrt(10)
    assert abs(ext["rho_mean"] - 0.423817) < 3 * 1.184e-3 / np.sqrt(10)


def test_table3_low_rank_ordering():
    """Table 3 (low-rank data, e_min = 0): E-A-HALS hp = 3 ends below hp = 1,
    which ends below plain A-HALS (same parameters, same iteration budget)."""
    probs = [S.lowrank(s, r=20) for s in range(6)]
    vs = [G.PLAIN, G.Variant(1, 0.5, 1.5, 1.01, 1.005), G.Variant(3, 0.5, 1.5, 1.01, 1.005)]
    print("table 3 ordering: 3 variants x 6 data sets, 300 iterations", flush=True)
    summ = G.summarize(vs, G.run(probs, vs, 300), e_min=[0.0] * len(probs))
    plain, hp1, hp3 = (r["E_mean"] for r in summ["rows"])
    print(plain, hp1, hp3, flush=True)
    assert hp3 < hp1 < plain


def test_whole_grid_at_scale():
    """All 109 parameter sets on 3 data sets (327 runs in one batch): every
    run completes its iterations with a finite, nonincreasing-on-accept trace,
    and a sample of runs matches the oracle."""
    probs = [S.fullrank(s) for s in range(3)]
    vs = G.grid_variants()
    assert len(vs) == 109
    print("whole grid: 109 variants x 3 data sets, 30 iterations", flush=True)
    res = G.run(probs, vs, 30)
    for row in res:
        for g in row:
            assert g.n_iter == 30 and np.all(np.isfinite(g.trace))
            acc = np.flatnonzero(g.accepted) + 1
            # accepted iterates never increase the error over the previous one
            assert np.all(g.trace[acc] <= g.trace[acc - 1] + 1e-12)
    summ = G.summarize(vs, res)
    assert set(summ["best_worst"]) == {1, 2, 3}
    rng = np.random.default_rng(0)
    for vi in rng.choice(len(vs), size=6, replace=False):
        v = vs[vi]
        for pi, p in enumerate(probs[:1]):
            print(v.label(), flush=True)
            compare_to_oracle(p, res[vi][pi], 30, inner_k=10, **v.params())


def test_eanls_grid_runs_match_oracle_and_table4():
    """E-ANLS through the batch (grouped exact NNLS solves): a sample of the
    82-variant grid of section 5.3 matches the oracle in its exact mode, and
    the chosen E-ANLS parameters (hp = 1, beta0 0.5, eta 1.5, gamma 1.1,
    gamma_bar 1.05) reproduce Table 4's full-rank mean 0.423795 +- 1.161e-3
    over 10 data sets within 3 standard errors."""
    import oracle
    vs = G.grid_variants(gammas=G.GAMMAS_ANLS)
    assert len(vs) == 82
    probs = [S.fullrank(s) for s in range(10)]
    chosen = G.Variant(1, 0.5, 1.5, 1.1, 1.05)
    sample = [G.PLAIN, chosen, G.Variant(3, 0.75, 2.0, 1.01, 1.005), G.Variant(2, 0.25, 3.0, 1.05, 1.01)]
    print("E-ANLS grid: 4 variants x 10 data sets, 150 iterations", flush=True)
    res = G.run(probs, sample, 150, inner_rule=P.Inner.EXACT)
    for v, row in zip(sample, res):
        for p, g in list(zip(probs, row))[:2]:
            print(v.label(), f"seed={p.seed}", flush=True)
            compare_to_oracle(p, g, 150, trace_iters=50, oracle_flags=oracle.EXACT_NNLS, **v.params())
    summ = G.summarize(sample, res)
    ext = summ["rows"][1]
    print(ext, flush=True)
    assert abs(ext["rho_mean"] - 0.423795) < 3 * 1.161e-3 / np.sqrt(10)


def test_mixed_rules_in_one_batch():
    """E-A-HALS and E-ANLS problems of the same padded rank share the grouped
    launches; each result is that of its own rule (against the oracle)."""
    import oracle
    probs = [S.fullrank(s, m=180, n=150, r=12) for s in range(4)]
    v = G.Variant(1, 0.5, 1.5, 1.1, 1.05)
    print("mixed batch: 2 fixed + 2 exact problems, 40 iterations", flush=True)
    out = {}
    with P.Batch(1 << 28, max_active=8, check_every=10) as B:
        t = [B.submit(p.X, p.r, p.W0, p.H0, max_iter=40, inner_k=10,
                      inner_rule=P.Inner.EXACT if i % 2 else P.Inner.FIXED, **v.params())
             for i, p in enumerate(probs)]
        while len(out) < len(t):
            B.step(10)
            for i, ti in enumerate(t):
                if i not in out:
                    g = B.result(ti)
                    if g is not None:
                        out[i] = g
    for i, p in enumerate(probs):
        print(f"problem {i} rule {'EXACT' if i % 2 else 'FIXED'}", flush=True)
        compare_to_oracle(p, out[i], 40, oracle_flags=oracle.EXACT_NNLS if i % 2 else 0,
                          inner_k=10, **v.params())


def test_class_gains_and_loses_exact_members():
    """One padded rank, at most two problems on the GPU at a time, E-A-HALS
    and E-ANLS problems of different lengths: the class's graphs drop the
    exact launches when its last E-ANLS problem retires and take them again
    when the next one is admitted. Each result equals the same problem run
    alone in a batch, bit for bit, and matches the oracle."""
    import oracle
    probs = [S.fullrank(10 + s, m=170, n=140, r=12) for s in range(5)]
    v = G.Variant(1, 0.5, 1.5, 1.1, 1.05)
    spec = [(False, 30), (True, 10), (False, 20), (False, 20), (True, 20)]
    print("admission order: fixed 30, exact 10, fixed 20, fixed 20, exact 20; "
          "max_active 2", flush=True)

    def kw(i):
        exact, n_it = spec[i]
        return dict(max_iter=n_it, inner_k=10, inner_rule=P.Inner.EXACT if exact else P.Inner.FIXED,
                    **v.params())

    def run(idx, max_active):
        out = {}
        with P.Batch(1 << 28, max_active=max_active, check_every=5) as B:
            t = {i: B.submit(probs[i].X, probs[i].r, probs[i].W0, probs[i].H0, **kw(i)) for i in idx}
            while len(out) < len(t):
                B.step(5)
                for i, ti in t.items():
                    if i not in out:
                        g = B.result(ti)
                        if g is not None:
                            out[i] = g
        return out

    mixed = run(range(5), 2)
    for i, p in enumerate(probs):
        exact, n_it = spec[i]
        print(f"problem {i} rule {'EXACT' if exact else 'FIXED'} iterations {n_it}", flush=True)
        alone = run([i], 1)[i]
        assert np.array_equal(alone.trace, mixed[i].trace)
        assert np.array_equal(alone.W, mixed[i].W) and np.array_equal(alone.H, mixed[i].H)
        compare_to_oracle(p, mixed[i], n_it, oracle_flags=oracle.EXACT_NNLS if exact else 0,
                          inner_k=10, **v.params())
