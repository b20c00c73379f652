"""GPU: the restart branch of Algorithm 2 for a non-finite error.

A non-finite e(k) must restart (from the last accepted iterate, with
beta <- beta / eta and the upper bound <- the previous beta) and must not
replace the error that the next iteration is compared with; a non-finite
e(0) is NMF_E_NUMERIC. The condition is forced from the host through the
library's error-scale hook (e(k)^2 times a given factor before the test), so
every kernel runs normally, and the oracle runs under the same factors.
"""
import numpy as np
import pytest

import nmf_synth as S
import oracle
from parity import compare_to_oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1805_06604_amd")

ALG = dict(beta0=0.5, gamma=1.05, gamma_bar=1.01, eta=1.5, inner_k=10)


def _scale(max_iter, at):
    s = np.ones(max_iter + 1)
    for k, v in at.items():
        s[k] = v
    return s


def _run(p, max_iter, scale, **kw):
    print(f"case {p.name} seed={p.seed} m={p.m} n={p.n} r={p.r} "
          f"scale at {np.flatnonzero(scale != 1.0).tolist()} {kw}", flush=True)
    with P.Solver(p.X, p.r, max_iter=max_iter, **kw) as s:
        s.set_error_scale(scale)
        return s.solve(p.W0, p.H0)


# NaN at 5; a millionfold increase at 6, which must restart because e(6)
# is compared with e(4), not with the NaN; +inf at 12.
INJECT = {5: np.nan, 6: 1e6, 12: np.inf}


@pytest.mark.parametrize("prod", ["VALU", "MFMA_EXACT"])
@pytest.mark.parametrize("hp", [1, 3])
def test_nonfinite_error_restarts_like_the_oracle(hp, prod):
    p = S.fullrank(0)
    sc = _scale(30, INJECT)
    g = _run(p, 30, sc, hp=hp, prod=P.Prod[prod], **ALG)
    assert not g.accepted[4] and not g.accepted[5] and not g.accepted[11]
    assert np.isnan(g.trace[5]) and g.trace[12] == np.inf
    compare_to_oracle(p, g, 30, hp=hp, e2_scale=sc, **ALG)


def test_nonfinite_error_restarts_with_exact_nnls():
    p = S.fullrank(1)
    sc = _scale(20, INJECT)
    g = _run(p, 20, sc, hp=1, inner_rule=P.Inner.EXACT, **ALG)
    assert not g.accepted[4] and not g.accepted[5]
    compare_to_oracle(p, g, 20, oracle_flags=oracle.EXACT_NNLS, hp=1, e2_scale=sc, **ALG)


def test_nonfinite_error_with_tol_stop_and_remark1_trace():
    """A NaN right before the tolerance would stop the solve: the stop test
    compares with a NaN and cannot fire there; both sides continue alike."""
    p = S.lowrank(0)
    sc = _scale(60, {3: np.nan, 4: np.nan})
    g = _run(p, 60, sc, hp=3, prod=P.Prod.MFMA_EXACT, tol=1e-4, **ALG)
    compare_to_oracle(p, g, 60, oracle_flags=oracle.ERR_REMARK1, hp=3, tol=1e-4,
                      e2_scale=sc, **ALG)


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_initial_error_is_numeric_error(bad):
    p = S.fullrank(2, m=60, n=50, r=5)
    with pytest.raises(P.NMFError) as ei:
        _run(p, 5, np.array([bad]), hp=3, **ALG)
    assert ei.value.status == P.Status.E_NUMERIC
    # Removing the hook makes the same context usable again.
    with P.Solver(p.X, p.r, max_iter=5, hp=3, **ALG) as s:
        s.set_error_scale(np.array([bad]))
        with pytest.raises(P.NMFError):
            s.solve(p.W0, p.H0)
        s.set_error_scale(None)
        g = s.solve(p.W0, p.H0)
    assert g.n_iter == 5 and np.all(np.isfinite(g.trace))
