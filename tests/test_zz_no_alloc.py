"""nmf_solve_noalloc (no device allocation: its buffers live in a static
device array of the library) against nmf_create + nmf_solve, the entry point
it is a variant of: the same kernels on the same inputs give the same
results bit for bit. Two calls in a row, the second on a smaller problem of
another rank class, so that the second call runs over what the first left
in the static array; then the error reports of the device-only interface."""
import numpy as np
import pytest

import nmf_synth as S

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1805_06604_amd")
torch = pytest.importorskip("torch")

ALG = dict(hp=3, beta0=0.5, gamma=1.05, gamma_bar=1.01, eta=1.5, inner_k=10)


def _context(p, **kw):
    with P.Solver(p.X, p.r, prod=P.Prod.MFMA_EXACT, **kw) as s:
        return s.solve(p.W0, p.H0)


def _noalloc(p, W0=None, **kw):
    dev = torch.device("cuda", torch.cuda.current_device())
    max_iter = kw["max_iter"]
    X = torch.from_numpy(np.ascontiguousarray(p.X)).to(dev)
    W0 = torch.from_numpy(np.ascontiguousarray(p.W0 if W0 is None else W0)).to(dev)
    H0 = torch.from_numpy(np.ascontiguousarray(p.H0)).to(dev)
    W = torch.full((p.m, p.r), -1.0, device=dev)
    H = torch.full((p.r, p.n), -1.0, device=dev)
    trace = torch.full((max_iter + 1,), float("nan"), dtype=torch.float64, device=dev)
    acc = torch.zeros(max(max_iter, 1), dtype=torch.uint8, device=dev)
    beta = torch.zeros(max(max_iter, 1), dtype=torch.float64, device=dev)
    info = torch.full((2,), -1, dtype=torch.int32, device=dev)
    P.solve_noalloc(X, p.r, W0, H0, W, H, trace, info, acc, beta,
                    stream=torch.cuda.current_stream(), **kw)
    torch.cuda.synchronize()
    status, k = (int(v) for v in info.cpu().numpy())
    res = P.Result(W.cpu().numpy(), H.cpu().numpy(), trace.cpu().numpy()[:k + 1],
                   acc.cpu().numpy()[:k].astype(bool), beta.cpu().numpy()[:k], k)
    return res, status


def _same(a, b):
    assert a.n_iter == b.n_iter
    np.testing.assert_array_equal(a.trace, b.trace)
    np.testing.assert_array_equal(a.accepted, b.accepted)
    np.testing.assert_array_equal(a.beta, b.beta)
    np.testing.assert_array_equal(a.W, b.W)
    np.testing.assert_array_equal(a.H, b.H)


def test_noalloc_equals_solve_on_two_calls_in_a_row():
    big = S.fullrank(3, m=700, n=390, r=48)
    small = S.lowrank(1, m=150, n=97, r=10)
    for p in (big, small):
        print(f"case {p.name} seed={p.seed} m={p.m} n={p.n} r={p.r}", flush=True)
        a = _context(p, max_iter=30, **ALG)
        b, status = _noalloc(p, max_iter=30, **ALG)
        assert status == P.Status.OK
        _same(a, b)


def test_noalloc_tol_stop_and_zero_iterations():
    p = S.lowrank(2, m=120, n=130, r=6)
    print(f"case {p.name} tol stop", flush=True)
    a = _context(p, max_iter=400, tol=1e-5, **ALG)
    b, status = _noalloc(p, max_iter=400, tol=1e-5, **ALG)
    assert status == P.Status.OK and a.n_iter < 400
    _same(a, b)
    a = _context(p, max_iter=0, **ALG)
    b, status = _noalloc(p, max_iter=0, **ALG)
    assert status == P.Status.OK and b.n_iter == 0
    _same(a, b)


def test_noalloc_reports_bad_inputs_on_the_device():
    p = S.fullrank(4, m=64, n=80, r=5)
    W0 = p.W0.copy()
    W0[3, 2] = -1.0
    print("case negative W0", flush=True)
    b, status = _noalloc(p, W0=W0, max_iter=5, **ALG)
    assert status == P.Status.E_INVAL and b.n_iter == 0


def test_noalloc_refuses_what_the_static_array_cannot_hold():
    dev = torch.device("cuda", torch.cuda.current_device())
    m = n = 4096
    X = torch.ones(m, n, device=dev)
    W0 = torch.ones(m, 4, device=dev)
    H0 = torch.ones(4, n, device=dev)
    W = torch.empty(m, 4, device=dev)
    H = torch.empty(4, n, device=dev)
    trace = torch.zeros(11, dtype=torch.float64, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    with pytest.raises(P.NMFError) as e:
        P.solve_noalloc(X, 4, W0, H0, W, H, trace, info, max_iter=10)
    assert e.value.status == P.Status.E_NOMEM
