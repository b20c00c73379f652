"""GPU checkpoint / resume: a solve saved after some iterations and loaded
into a fresh context of the same problem continues bit for bit like the
uninterrupted solve (iterates, the whole trace, decisions, betas), for the
fixed, exact and adaptive inner rules; the resumed result also matches the
oracle resumed from its own saved state; states of other problems or
parameters are refused."""
import numpy as np
import pytest

import nmf_synth as S
import oracle
from parity import compare_to_oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1805_06604_amd")

ALG = dict(hp=3, beta0=0.5, gamma=1.05, gamma_bar=1.01, eta=1.5, inner_k=10)


def _full(p, **kw):
    with P.Solver(p.X, p.r, **kw) as s:
        s.start(p.W0, p.H0)
        s.iterate(kw["max_iter"])
        return s.read()


def _split(p, at, **kw):
    with P.Solver(p.X, p.r, **kw) as s:
        s.start(p.W0, p.H0)
        s.iterate(at)
        blob = s.save_state()
    with P.Solver(p.X, p.r, **kw) as s:
        s.load_state(blob)
        s.iterate(kw["max_iter"] - at)
        return s.read(), blob


@pytest.mark.parametrize("rule,extra", [("FIXED", dict(prod="MFMA_EXACT")), ("FIXED", dict(prod="VALU")),
                                        ("EXACT", {}), ("ADAPTIVE", dict(inner_k=8))])
def test_resume_is_bitwise_the_uninterrupted_solve(rule, extra):
    p = S.fullrank(5, m=301, n=157, r=13)
    kw = dict(ALG, max_iter=40, inner_rule=P.Inner[rule])
    kw.update({k: (P.Prod[v] if k == "prod" else v) for k, v in extra.items()})
    print(f"case {p.name} m={p.m} n={p.n} r={p.r} {kw}", flush=True)
    a = _full(p, **kw)
    b, _ = _split(p, 17, **kw)
    assert a.n_iter == b.n_iter == 40
    np.testing.assert_array_equal(b.trace, a.trace)
    np.testing.assert_array_equal(b.accepted, a.accepted)
    np.testing.assert_array_equal(b.beta, a.beta)
    np.testing.assert_array_equal(b.W, a.W)
    np.testing.assert_array_equal(b.H, a.H)


def test_resumed_solve_against_the_resumed_oracle():
    """The GPU solve interrupted after 20 iterations and resumed meets the
    parity protocol against the oracle's uninterrupted solve (which the
    oracle's own resume reproduces bit for bit, a CPU pin)."""
    p = S.fullrank(0)
    kw = dict(ALG, max_iter=50, prod=P.Prod.MFMA_EXACT)
    g, _ = _split(p, 20, **kw)
    compare_to_oracle(p, g, 50, **ALG)


def test_tol_stop_survives_the_checkpoint():
    p = S.lowrank(0, m=120, n=110, r=6)
    kw = dict(ALG, max_iter=600, tol=1e-6)
    a = _full(p, **kw)
    assert a.n_iter < 600
    b, _ = _split(p, a.n_iter, **kw)      # saved at the stop: nothing more runs
    assert b.n_iter == a.n_iter
    np.testing.assert_array_equal(b.W, a.W)
    c, _ = _split(p, a.n_iter - 3, **kw)
    assert c.n_iter == a.n_iter
    np.testing.assert_array_equal(c.trace, a.trace)


def test_states_of_other_problems_are_refused():
    p = S.fullrank(1, m=90, n=70, r=5)
    q = S.fullrank(2, m=90, n=70, r=5)
    kw = dict(ALG, max_iter=10)
    with P.Solver(p.X, p.r, **kw) as s:
        s.start(p.W0, p.H0)
        s.iterate(4)
        blob = s.save_state()
    for X, r, kw2, what in [(q.X, 5, kw, "another X"), (p.X, 5, dict(kw, hp=1), "other parameters"),
                            (p.X, 5, dict(kw, max_iter=20), "max_iter"),
                            (p.X[:, :60], 5, kw, "problem")]:
        with P.Solver(X, r, **kw2) as s:
            with pytest.raises(P.NMFError) as e:
                s.load_state(blob)
            assert e.value.status == P.Status.E_INVAL and what in str(e.value)
    with P.Solver(p.X, p.r, **kw) as s:
        with pytest.raises(P.NMFError):
            s.load_state(blob[:-8])
