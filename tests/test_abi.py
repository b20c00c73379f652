"""CPU checks of the C ABI: the library loads, exports every function that
include/nmf.h declares, and validates arguments before any device work."""
import os
import re

import numpy as np
import pytest

import paper_1805_06604_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "nmf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nmf_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    names = declared_functions()
    assert names, "no declarations found"
    assert sorted(P.EXPORTS) == names


def test_phase_names_follow_the_header_enum():
    text = open(os.path.join(ROOT, "include", "nmf.h")).read()
    found = re.findall(r"NMF_PHASE_([A-Z_]+) = (\d+)", text)
    names = [n.lower() for n, v in sorted(found, key=lambda t: int(t[1])) if n != "COUNT"]
    count = dict(found)["COUNT"]
    assert tuple(names) == P.PHASES and int(count) == len(P.PHASES)


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_defaults_are_the_papers_final_parameters():
    prm = P.make_params(20)
    assert (prm.hp, prm.beta0, prm.eta, prm.gamma, prm.gamma_bar) == (3, 0.5, 1.5, 1.01, 1.005)
    assert (prm.inner_rule, prm.inner_k, prm.inner_alpha, prm.inner_delta) == (P.Inner.FIXED, 10, 0.5, 0.1)
    assert (prm.inner_rho_h, prm.inner_rho_w) == (0.0, 0.0)


@pytest.mark.parametrize("kw,status", [
    (dict(hp=0), P.Status.E_INVAL),
    (dict(hp=4), P.Status.E_INVAL),
    (dict(beta0=-0.1), P.Status.E_INVAL),
    (dict(beta0=1.0), P.Status.E_INVAL),
    (dict(gamma=1.004), P.Status.E_INVAL),          # gamma <= gamma_bar
    (dict(eta=1.0), P.Status.E_INVAL),              # eta <= gamma
    (dict(gamma_bar=1.0), P.Status.E_INVAL),
    (dict(inner_k=0), P.Status.E_INVAL),
    (dict(max_iter=-1), P.Status.E_INVAL),
    (dict(tol=-1.0), P.Status.E_INVAL),
    (dict(x_dtype=7), P.Status.E_INVAL),
    (dict(prod=9), P.Status.E_INVAL),
    (dict(flags=8), P.Status.E_INVAL),
    (dict(inner_rule=3), P.Status.E_UNSUPPORTED),
    (dict(inner_rule=P.Inner.EXACT, inner_k=0), P.Status.E_INVAL),
    (dict(inner_rule=P.Inner.ADAPTIVE, inner_alpha=-0.5), P.Status.E_INVAL),
    (dict(inner_rule=P.Inner.ADAPTIVE, inner_delta=float("nan")), P.Status.E_INVAL),
    (dict(inner_rule=P.Inner.ADAPTIVE, inner_rho_h=-1.0), P.Status.E_INVAL),
    (dict(inner_rule=P.Inner.ADAPTIVE, inner_rho_w=float("inf")), P.Status.E_INVAL),
])
def test_parameter_validation(kw, status):
    with pytest.raises(P.NMFError) as e:
        P.Solver(np.ones((4, 3), np.float32), 2, **kw)
    assert e.value.status == status


@pytest.mark.parametrize("r,status", [(0, P.Status.E_INVAL), (65, P.Status.E_UNSUPPORTED)])
def test_rank_validation(r, status):
    with pytest.raises(P.NMFError) as e:
        P.Solver(np.ones((4, 3), np.float32), r)
    assert e.value.status == status


def test_nonfinite_matrix_rejected():
    X = np.ones((5, 4), np.float32)
    X[2, 1] = np.nan
    with pytest.raises(P.NMFError) as e:
        P.Solver(X, 2)
    assert e.value.status == P.Status.E_INVAL
    assert "non-finite" in str(e.value)


def test_empty_matrix_rejected():
    with pytest.raises(P.NMFError) as e:
        P.Solver(np.ones((0, 3), np.float32), 1)
    assert e.value.status == P.Status.E_INVAL


class _Csr:
    def __init__(self, m, n, row_ptr, col_idx, val):
        self.m, self.n = m, n
        self.row_ptr = np.asarray(row_ptr, np.int64)
        self.col_idx = np.asarray(col_idx, np.int32)
        self.val = np.asarray(val, np.float32)


@pytest.mark.parametrize("rp,ci,va,what", [
    ([1, 2, 3], [0, 1], [1.0, 1.0], "start at 0"),             # row_ptr[0] != 0
    ([0, 2, 1], [0, 1], [1.0, 1.0], "decreases"),              # row_ptr not monotone
    ([0, 2, 2], [0, 5], [1.0, 1.0], "out of range"),           # column >= n
    ([0, 2, 2], [1, 1], [1.0, 1.0], "strictly"),               # duplicate column
    ([0, 2, 2], [2, 1], [1.0, 1.0], "strictly"),               # unsorted
    ([0, 1, 2], [0, 1], [1.0, np.inf], "non-finite"),
])
def test_malformed_csr_rejected(rp, ci, va, what):
    with pytest.raises(P.NMFError) as e:
        P.Solver(_Csr(2, 3, rp, ci, va), 1)
    assert e.value.status == P.Status.E_INVAL
    assert what in str(e.value)


def test_csr_needs_fp32_storage():
    X = _Csr(2, 3, [0, 1, 2], [0, 2], [1.0, 2.0])
    for kw in (dict(x_dtype=P.XDtype.BF16), dict(prod=P.Prod.MFMA_FAST)):
        with pytest.raises(P.NMFError) as e:
            P.Solver(X, 1, **kw)
        assert e.value.status == P.Status.E_UNSUPPORTED


@pytest.mark.parametrize("kw", [dict(hbm_budget=0), dict(max_active=0), dict(max_active=5000),
                                dict(check_every=0)])
def test_batch_parameter_validation(kw):
    args = dict(hbm_budget=1 << 20, max_active=4, check_every=1)
    args.update(kw)
    with pytest.raises(P.NMFError) as e:
        P.Batch(**args)
    assert e.value.status == P.Status.E_INVAL



def test_error_scale_hook_validates_before_device_work():
    import ctypes as C
    lib = P.lib()
    sc = np.array([1.0, np.nan])
    assert lib.nmf_set_error_scale(None, sc.ctypes.data, 2) == P.Status.E_INVAL


@pytest.mark.parametrize("bad,what", [
    ("f16", "float32"), ("bf16", "float32"), ("shape", "shape"), ("small", "shape"),
    ("strided", "contiguous"), ("cpu", "cuda"), ("numpy", "torch tensor")])
def test_device_tensor_checks_reject_before_any_launch(bad, what):
    """Raw device pointers go to the kernels as m x r and r x n FP32 arrays:
    the binding must refuse anything that is not exactly that."""
    torch = pytest.importorskip("torch")
    from paper_1805_06604_amd.binding import _check_device_tensor
    m, r = 6, 3
    t = {"f16": torch.zeros(m, r, dtype=torch.float16),
         "bf16": torch.zeros(m, r, dtype=torch.bfloat16),
         "shape": torch.zeros(r, m),
         "small": torch.zeros(m - 1, r),
         "strided": torch.zeros(r, m).t(),
         "cpu": torch.zeros(m, r),
         "numpy": np.zeros((m, r), np.float32)}[bad]
    with pytest.raises(ValueError, match=what):
        _check_device_tensor(t, (m, r), "W0", 0)


def test_fast_product_needs_16bit_storage():
    X = np.ones((4, 3), np.float32)
    with pytest.raises(P.NMFError) as e:
        P.Solver(X, 1, prod=P.Prod.MFMA_FAST)
    assert e.value.status == P.Status.E_UNSUPPORTED
    assert "16 bits" in str(e.value)
