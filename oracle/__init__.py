"""ctypes front end of the FP64 E-A-HALS oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark use this package. The GPU library neither imports nor links it.
Inputs are promoted to float64 here; outputs are float64 numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

OK, EINVAL, ENUMERIC, ENOMEM = 0, 1, 2, 3
BETABAR_LAST_ACCEPTED = 1
CMP_LAST_ACCEPTED = 2
ERR_REMARK1 = 4
ROUND_F32 = 8
EXACT_NNLS = 16
ADAPTIVE_INNER = 32
ROUND_F32_RZ = 64

_lib = None


class _Matrix(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64),
                ("dense", C.c_void_p), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p)]


class _State(C.Structure):
    _fields_ = [("k", C.c_int), ("W", C.c_void_p), ("H", C.c_void_p),
                ("Wy", C.c_void_p), ("Hy", C.c_void_p), ("beta", C.c_double),
                ("betabar", C.c_double), ("beta_prev", C.c_double),
                ("beta_acc", C.c_double), ("e_prev", C.c_double), ("e_acc", C.c_double),
                ("rho", C.c_double)]


STATE_SCALARS = ("beta", "betabar", "beta_prev", "beta_acc", "e_prev", "e_acc", "rho")


class _Params(C.Structure):
    _fields_ = [("hp", C.c_int), ("beta0", C.c_double), ("gamma", C.c_double),
                ("gamma_bar", C.c_double), ("eta", C.c_double),
                ("inner_k", C.c_int), ("max_iter", C.c_int),
                ("tol", C.c_double), ("flags", C.c_int),
                ("replay", C.c_void_p), ("inner_alpha", C.c_double),
                ("inner_delta", C.c_double), ("sweeps_replay", C.c_void_p),
                ("e2_scale", C.c_void_p), ("e2_scale_n", C.c_int),
                ("resume", C.c_void_p), ("save", C.c_void_p),
                ("inner_rho_h", C.c_double), ("inner_rho_w", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        d, i, p = C.c_double, C.c_int, C.c_void_p
        _lib.oracle_eahals.argtypes = [p, i, p, p, p, p, p, p, p, p, p, p, p, p, p]
        _lib.oracle_eahals.restype = i
        _lib.oracle_nnls_h.argtypes = [p, i, p, p, i]
        _lib.oracle_nnls_w.argtypes = [p, i, p, p, i]
        _lib.oracle_beta_script.argtypes = [i, p, d, d, d, d, i, p, p]
        _lib.oracle_beta_script.restype = None
        _lib.oracle_rel_error.argtypes = [p, i, p, p]
        _lib.oracle_rel_error.restype = d
        _lib.oracle_rel_error_remark1.argtypes = [p, i, p, p]
        _lib.oracle_rel_error_remark1.restype = d
        _lib.oracle_nnls_exact_h.argtypes = [p, i, p, p]
        _lib.oracle_nnls_exact_w.argtypes = [p, i, p, p]
        _lib.oracle_beta_star.argtypes = [p, i, p, p, p]
        _lib.oracle_beta_star.restype = d
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class _Held:
    """Keeps the float64 copies alive while C holds pointers to them."""

    def __init__(self, X):
        if hasattr(X, "row_ptr"):
            self.row_ptr = np.ascontiguousarray(X.row_ptr, dtype=np.int64)
            self.col_idx = np.ascontiguousarray(X.col_idx, dtype=np.int32)
            self.val = np.ascontiguousarray(X.val, dtype=np.float64)
            self.s = _Matrix(X.m, X.n, None, _ptr(self.row_ptr).value,
                             _ptr(self.col_idx).value, _ptr(self.val).value)
        else:
            self.dense = np.ascontiguousarray(X, dtype=np.float64)
            m, n = self.dense.shape
            self.s = _Matrix(m, n, _ptr(self.dense).value, None, None, None)
        self.m, self.n = self.s.m, self.s.n


def solve(X, r, W0, H0, *, hp=3, beta0=0.5, gamma=1.05, gamma_bar=1.01,
          eta=1.5, inner_k=10, max_iter=100, tol=0.0, flags=0, replay=None,
          inner_alpha=0.5, inner_delta=0.1, sweeps_replay=None, e2_scale=None,
          resume=None, save=False, inner_rho_h=0.0, inner_rho_w=0.0):
    """Run Alg. 2 with Alg. 3 and return a dict with W, H (last accepted),
    trace (rho(0..n_iter)), accepted, beta, margin, beta_star (section 4,
    per iteration), sweeps (HALS sweeps on H and on W per iteration),
    sweep_margin (closest call of each adaptive stop decision) and n_iter.
    sweeps_replay forces the adaptive sweep counts ((max_iter, 2) array).
    inner_rho_h, inner_rho_w > 0 replace the flop ratios of the adaptive
    sweep caps (R18) by the caller's cost ratios of the two sides.
    e2_scale (test hook): factors applied to e(k)^2 for k = 0, 1, ... before
    the test of Algorithm 2 (NaN or inf drive its non-finite branch).
    save=True adds out["state"], the state after the last iteration (a dict:
    k, W, H, Wy, Hy and the scalars of STATE_SCALARS); resume=<such a dict>
    continues that solve (trace entries 0..k are then rho(k) at index k and
    zeros before it)."""
    h = _Held(X)
    W0 = np.ascontiguousarray(W0, dtype=np.float64).reshape(h.m, r)
    H0 = np.ascontiguousarray(H0, dtype=np.float64).reshape(r, h.n)
    W = np.empty_like(W0)
    H = np.empty_like(H0)
    trace = np.zeros(max_iter + 1)
    acc = np.zeros(max(max_iter, 1), dtype=np.uint8)
    beta = np.zeros(max(max_iter, 1))
    margin = np.zeros(max(max_iter, 1))
    bstar = np.zeros(max(max_iter, 1))
    sweeps = np.zeros((max(max_iter, 1), 2), dtype=np.int32)
    smargin = np.zeros((max(max_iter, 1), 2))
    sr = None
    if sweeps_replay is not None:
        sr = np.ascontiguousarray(sweeps_replay, dtype=np.int32).reshape(-1, 2)
        if sr.shape[0] < max_iter:
            raise ValueError("sweeps_replay needs max_iter rows")
    rp = None
    if replay is not None:
        rp = np.ascontiguousarray(replay, dtype=np.uint8)
        if rp.size < max_iter:
            raise ValueError("replay needs max_iter decisions")
    es = None
    if e2_scale is not None:
        es = np.ascontiguousarray(e2_scale, dtype=np.float64).ravel()
    rs = sv = None
    keep = []
    if resume is not None:
        arrs = [np.ascontiguousarray(resume[key], dtype=np.float64) for key in ("W", "H", "Wy", "Hy")]
        keep += arrs
        rs = _State(int(resume["k"]), *[_ptr(a).value for a in arrs],
                    *[float(resume[key]) for key in STATE_SCALARS])
    if save:
        sarr = dict(W=np.empty((h.m, r)), H=np.empty((r, h.n)), Wy=np.empty((h.m, r)),
                    Hy=np.empty((r, h.n)))
        sv = _State(0, *[_ptr(sarr[key]).value for key in ("W", "H", "Wy", "Hy")])
    prm = _Params(hp, beta0, gamma, gamma_bar, eta, inner_k, max_iter, tol,
                  flags, None if rp is None else _ptr(rp).value, inner_alpha, inner_delta,
                  None if sr is None else _ptr(sr).value,
                  None if es is None else _ptr(es).value, 0 if es is None else es.size,
                  None if rs is None else C.addressof(rs), None if sv is None else C.addressof(sv),
                  inner_rho_h, inner_rho_w)
    nit = C.c_int(0)
    st = lib().oracle_eahals(C.byref(h.s), r, _ptr(W0), _ptr(H0), C.byref(prm),
                             _ptr(W), _ptr(H), _ptr(trace), _ptr(acc),
                             _ptr(beta), _ptr(margin), C.byref(nit), _ptr(bstar),
                             _ptr(sweeps), _ptr(smargin))
    if st != OK:
        raise RuntimeError(f"oracle_eahals failed with status {st}")
    k = nit.value
    out = dict(W=W, H=H, trace=trace[:k + 1], accepted=acc[:k].astype(bool),
               beta=beta[:k], margin=margin[:k], beta_star=bstar[:k], sweeps=sweeps[:k],
               sweep_margin=smargin[:k], n_iter=k)
    if save:
        out["state"] = dict(k=sv.k, **sarr, **{key: getattr(sv, key) for key in STATE_SCALARS})
    return out


def beta_star(X, Wn, W, Hw):
    """Section 4: the beta minimizing ||X - (Wn + beta (Wn - W)) Hw||_F."""
    h = _Held(X)
    r = Hw.shape[0]
    Wn = np.ascontiguousarray(Wn, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    Hw = np.ascontiguousarray(Hw, dtype=np.float64)
    return lib().oracle_beta_star(C.byref(h.s), r, _ptr(Wn), _ptr(W), _ptr(Hw))


def nnls_h(X, W, H0, sweeps):
    h = _Held(X)
    r = W.shape[1]
    W = np.ascontiguousarray(W, dtype=np.float64)
    H = np.array(H0, dtype=np.float64, order="C", copy=True)
    if lib().oracle_nnls_h(C.byref(h.s), r, _ptr(W), _ptr(H), sweeps) != OK:
        raise RuntimeError("oracle_nnls_h failed")
    return H


def nnls_exact_h(X, W, H0):
    """Exact NNLS of every column of H (warm start H0) given W."""
    h = _Held(X)
    r = W.shape[1]
    W = np.ascontiguousarray(W, dtype=np.float64)
    H = np.array(H0, dtype=np.float64, order="C", copy=True)
    if lib().oracle_nnls_exact_h(C.byref(h.s), r, _ptr(W), _ptr(H)) != OK:
        raise RuntimeError("oracle_nnls_exact_h failed")
    return H


def nnls_exact_w(X, H, W0):
    """Exact NNLS of every row of W (warm start W0) given H."""
    h = _Held(X)
    r = H.shape[0]
    H = np.ascontiguousarray(H, dtype=np.float64)
    W = np.array(W0, dtype=np.float64, order="C", copy=True)
    if lib().oracle_nnls_exact_w(C.byref(h.s), r, _ptr(H), _ptr(W)) != OK:
        raise RuntimeError("oracle_nnls_exact_w failed")
    return W


def nnls_w(X, H, W0, sweeps):
    h = _Held(X)
    r = H.shape[0]
    H = np.ascontiguousarray(H, dtype=np.float64)
    W = np.array(W0, dtype=np.float64, order="C", copy=True)
    if lib().oracle_nnls_w(C.byref(h.s), r, _ptr(H), _ptr(W), sweeps) != OK:
        raise RuntimeError("oracle_nnls_w failed")
    return W


def beta_script(decreased, beta0, gamma, gamma_bar, eta, flags=0):
    d = np.ascontiguousarray(decreased, dtype=np.uint8)
    bu = np.zeros(d.size)
    bb = np.zeros(d.size)
    lib().oracle_beta_script(d.size, _ptr(d), beta0, gamma, gamma_bar, eta,
                             flags, _ptr(bu), _ptr(bb))
    return bu, bb


def rel_error(X, W, H):
    h = _Held(X)
    W = np.ascontiguousarray(W, dtype=np.float64)
    H = np.ascontiguousarray(H, dtype=np.float64)
    return lib().oracle_rel_error(C.byref(h.s), W.shape[1], _ptr(W), _ptr(H))


def rel_error_remark1(X, W, H):
    h = _Held(X)
    W = np.ascontiguousarray(W, dtype=np.float64)
    H = np.ascontiguousarray(H, dtype=np.float64)
    return lib().oracle_rel_error_remark1(C.byref(h.s), W.shape[1], _ptr(W),
                                          _ptr(H))
