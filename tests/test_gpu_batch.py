"""GPU checks of batched solves (continuous batching of independent
problems, grouped launches): every batched problem against the FP64 oracle,
admission under a tight memory budget, problems that stop at different
iterations, and the pending state."""
import numpy as np
import pytest

import nmf_synth as S
from parity import compare_to_oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1805_06604_amd")

ALG = dict(beta0=0.5, gamma=1.05, gamma_bar=1.01, eta=1.5, inner_k=10)


def _problems():
    """Mixed shapes and every padded rank class (r = 5, 10 -> 16; 20 -> 32;
    40 -> 48; 64 -> 64), all with r < min(m, n) (with r >= min(m, n) the
    factors of an exact fit are not unique and only W H is comparable)."""
    specs = [(150, 120, 5, 0), (200, 200, 10, 1), (97, 333, 20, 2), (260, 190, 40, 3),
             (300, 180, 64, 4), (310, 77, 20, 5)]
    out = []
    for m, n, r, seed in specs:
        p = S.request_problem(S.Request(seed, 0.0, m, n, r, 1000 + seed))
        out.append(p)
    return out


def _run_batch(problems, budget, max_iter, max_active=64, check_every=5, **kw):
    print(f"batch of {len(problems)} budget={budget} max_iter={max_iter} {kw}", flush=True)
    res = {}
    with P.Batch(budget, max_active=max_active, check_every=check_every) as B:
        tickets = [B.submit(p.X, p.r, p.W0, p.H0, max_iter=max_iter, hp=3, **ALG, **kw)
                   for p in problems]
        assert B.result(tickets[0]) is None            # nothing has run yet
        for _ in range(200):
            a, q, d = B.step(max_iter)
            for i, t in enumerate(tickets):
                if i not in res:
                    g = B.result(t)
                    if g is not None:
                        res[i] = g
            if len(res) == len(problems):
                break
    assert len(res) == len(problems)
    return [res[i] for i in range(len(problems))]


def test_batch_matches_oracle():
    probs = _problems()
    got = _run_batch(probs, 1 << 30, 40)
    for p, g in zip(probs, got):
        print(f"problem m={p.m} n={p.n} r={p.r}", flush=True)
        compare_to_oracle(p, g, 40, hp=3, **ALG)


def test_batch_tight_budget_is_bitwise_identical():
    """A budget that holds only a few problems at a time: admission waits for
    retirements, and every result equals the unconstrained run bit for bit
    (the same per-problem work decomposition)."""
    probs = _problems()
    free = _run_batch(probs, 1 << 30, 30)
    tight = _run_batch(probs, 24 << 20, 30, check_every=3)
    for a, b in zip(free, tight):
        assert np.array_equal(a.trace, b.trace)
        assert np.array_equal(a.W, b.W) and np.array_equal(a.H, b.H)


def test_batch_problems_stop_independently():
    """Different max_iter per problem and the tol rule: each problem stops at
    its own iteration while the others go on."""
    probs = _problems()[:4]
    res = {}
    with P.Batch(1 << 30, max_active=8, check_every=4) as B:
        tk = [B.submit(p.X, p.r, p.W0, p.H0, max_iter=mi, hp=3, **ALG)
              for p, mi in zip(probs, (7, 13, 29, 50))]
        tk.append(B.submit(probs[0].X, probs[0].r, probs[0].W0, probs[0].H0, max_iter=300,
                           tol=1e-5, hp=3, **ALG))
        for _ in range(100):
            B.step(8)
            for i, t in enumerate(tk):
                if i not in res:
                    g = B.result(t)
                    if g is not None:
                        res[i] = g
            if len(res) == len(tk):
                break
    assert [res[i].n_iter for i in range(4)] == [7, 13, 29, 50]
    g = res[4]
    assert g.n_iter < 300 and g.accepted[-1]
    assert abs(g.trace[-1] - g.trace[-2]) < 1e-5
    with P.Solver(probs[0].X, probs[0].r, max_iter=300, tol=1e-5, hp=3,
                  prod=P.Prod.MFMA_EXACT, **ALG) as s:
        single = s.solve(probs[0].W0, probs[0].H0)
    assert single.n_iter == g.n_iter
    np.testing.assert_allclose(g.trace, single.trace, rtol=1e-6)


def test_batch_rejects_the_adaptive_inner_rule():
    p = _problems()[0]
    with P.Batch(1 << 24, max_active=4, check_every=1) as B:
        with pytest.raises(P.NMFError) as e:
            B.submit(p.X, p.r, p.W0, p.H0, inner_rule=P.Inner.ADAPTIVE)
    assert e.value.status == P.Status.E_UNSUPPORTED


def test_each_problem_is_the_same_alone_and_in_the_mix():
    """Continuous batching does not change a problem's result: each problem
    run alone in a batch equals the same problem run among the others bit for
    bit (its work blocks, K-chunks and reductions do not depend on the other
    problems), and equals the single-problem solve (whose product kernels
    split K differently) within the parity tolerances on the trace, W and H."""
    from parity import rel_fro
    probs = _problems()
    mix = _run_batch(probs, 1 << 30, 30, check_every=5)
    for p, g in zip(probs, mix):
        print(f"problem m={p.m} n={p.n} r={p.r}", flush=True)
        alone = _run_batch([p], 1 << 30, 30, check_every=5)[0]
        assert np.array_equal(alone.trace, g.trace)
        assert np.array_equal(alone.W, g.W) and np.array_equal(alone.H, g.H)
        with P.Solver(p.X, p.r, max_iter=30, hp=3, prod=P.Prod.MFMA_EXACT, **ALG) as s:
            single = s.solve(p.W0, p.H0)
        assert np.array_equal(single.accepted, g.accepted)
        np.testing.assert_allclose(g.trace, single.trace, rtol=1e-5)
        assert rel_fro(g.W, single.W) < 1e-4 and rel_fro(g.H, single.H) < 1e-4


def test_submissions_from_another_thread_while_stepping():
    """A serving loop: one thread steps the batch and collects results while
    another submits problems over time. Every result equals the same problem
    run alone, bit for bit."""
    import threading
    import time
    probs = _problems() * 3
    got = {}
    with P.Batch(1 << 30, max_active=64, check_every=5) as B:
        tickets = []
        done = threading.Event()

        def step():
            while not done.is_set() or len(got) < len(probs):
                B.step(5)
                for i, t in enumerate(list(tickets)):
                    if i not in got:
                        g = B.result(t)
                        if g is not None:
                            got[i] = g
                if done.is_set() and len(got) == len(tickets):
                    break
                time.sleep(0.0005)

        th = threading.Thread(target=step)
        th.start()
        for p in probs:
            tickets.append(B.submit(p.X, p.r, p.W0, p.H0, max_iter=25, hp=3, **ALG))
            time.sleep(0.002)
        done.set()
        th.join(timeout=120)
        assert not th.is_alive()
    assert len(got) == len(probs)
    for i, p in enumerate(probs[:len(_problems())]):
        alone = _run_batch([p], 1 << 30, 25, check_every=5)[0]
        for j in (i, i + len(_problems()), i + 2 * len(_problems())):
            assert np.array_equal(got[j].trace, alone.trace)
            assert np.array_equal(got[j].W, alone.W) and np.array_equal(got[j].H, alone.H)
