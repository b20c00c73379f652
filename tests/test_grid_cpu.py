"""CPU checks of the parameter grid of section 5.3 (no device work)."""
from paper_1805_06604_amd import grid as G


def test_grid_is_the_papers():
    vs = G.grid_variants()
    assert len(vs) == 1 + 3 * 3 * 3 * 4
    assert vs[0].plain and vs[0].label() == "plain"
    assert {v.beta0 for v in vs[1:]} == {0.25, 0.5, 0.75}
    assert {v.eta for v in vs[1:]} == {1.5, 2.0, 3.0}
    assert {(v.gamma, v.gamma_bar) for v in vs[1:]} == {(1.005, 1.001), (1.01, 1.005),
                                                        (1.05, 1.01), (1.1, 1.05)}
    assert all(1 < v.gamma_bar < v.gamma < v.eta for v in vs)


class _R:
    def __init__(self, trace):
        self.trace = trace


def test_summary_best_and_worst():
    vs = [G.PLAIN, G.Variant(1, 0.5, 1.5, 1.01, 1.005), G.Variant(1, 0.75, 2.0, 1.05, 1.01)]
    res = [[_R([1.0, 0.5]), _R([1.0, 0.6])], [_R([1.0, 0.4]), _R([1.0, 0.45])],
           [_R([1.0, 0.3]), _R([1.0, 0.7])]]
    s = G.summarize(vs, res)
    assert s["e_min"] == [0.3, 0.45]
    assert s["best_worst"][1]["best"]["variant"] == vs[1].label()
    assert s["best_worst"][1]["worst"]["variant"] == vs[2].label()
