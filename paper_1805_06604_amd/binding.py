"""ctypes binding of libnmf.so (the C ABI declared in include/nmf.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Host arrays are numpy; device arrays are torch CUDA tensors (torch supplies
device memory and streams, nothing else). The library must be built
(``__graft_entry__.build()``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import enum
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmf.so")

EXPORTS = ("nmf_params_default", "nmf_create", "nmf_solve", "nmf_start",
           "nmf_iterate", "nmf_read", "nmf_profile", "nmf_destroy",
           "nmf_last_error", "nmf_read_beta_star", "nmf_read_sweeps", "nmf_set_error_scale",
           "nmf_solve_noalloc", "nmf_state_size", "nmf_save_state", "nmf_load_state",
           "nmf_batch_create", "nmf_batch_submit", "nmf_batch_step",
           "nmf_batch_result", "nmf_batch_destroy")


class Status(enum.IntEnum):
    OK = 0
    E_INVAL = 1
    E_UNSUPPORTED = 2
    E_NOMEM = 3
    E_DEVICE = 4
    E_NUMERIC = 5
    E_STATE = 6
    PENDING = 7


class Format(enum.IntEnum):
    DENSE = 0
    CSR = 1


class XDtype(enum.IntEnum):
    F32 = 0
    BF16 = 1
    F16 = 2


class Inner(enum.IntEnum):
    FIXED = 0      # inner_k HALS sweeps per block (E-A-HALS)
    EXACT = 1      # exact NNLS per row by block principal pivoting (E-ANLS)
    ADAPTIVE = 2   # A-HALS inner loop with the cost-ratio cap and early stop


class Prod(enum.IntEnum):
    AUTO = 0
    VALU = 1
    MFMA_EXACT = 2
    MFMA_FAST = 3


# Kernels of one outer iteration in launch order (enum nmf_phase).
PHASES = ("slice_w", "prod_ct", "sweep_h", "finish_h", "slice_h", "prod_a", "sweep_w",
          "finish_w")

FLAG_BETABAR_LAST_ACCEPTED = 1
FLAG_CMP_LAST_ACCEPTED = 2
FLAG_BETA_STAR = 4


class NMFError(RuntimeError):
    def __init__(self, status, message):
        self.status = Status(status)
        super().__init__(f"{self.status.name}: {message}")


class _Matrix(C.Structure):
    _fields_ = [("fmt", C.c_int32), ("m", C.c_int64), ("n", C.c_int64),
                ("dense", C.c_void_p), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("nnz", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("r", C.c_int32), ("hp", C.c_int32), ("beta0", C.c_double),
                ("gamma", C.c_double), ("gamma_bar", C.c_double),
                ("eta", C.c_double), ("inner_rule", C.c_int32),
                ("inner_k", C.c_int32), ("max_iter", C.c_int32),
                ("tol", C.c_double), ("x_dtype", C.c_int32),
                ("prod", C.c_int32), ("flags", C.c_int32),
                ("inner_alpha", C.c_double), ("inner_delta", C.c_double),
                ("inner_rho_h", C.c_double), ("inner_rho_w", C.c_double)]


_lib = None


def lib():
    """Loads libnmf.so once; raises if it has not been built.

    torch is imported first when it is installed: libnmf.so then binds to the
    HIP runtime torch brings (one runtime per process), so that torch tensors
    and streams handed to the library belong to the same runtime."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build()")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        p, i32 = C.c_void_p, C.c_int32
        L.nmf_params_default.argtypes = [p]
        L.nmf_params_default.restype = None
        L.nmf_create.argtypes = [p, p, p]
        L.nmf_create.restype = i32
        L.nmf_solve.argtypes = [p, p, p, p, p, p, i32, p, p, p]
        L.nmf_solve.restype = i32
        L.nmf_start.argtypes = [p, p, p, i32, p]
        L.nmf_start.restype = i32
        L.nmf_iterate.argtypes = [p, i32, p]
        L.nmf_iterate.restype = i32
        L.nmf_read.argtypes = [p, p, p, i32, p, i32, p, p, p, p]
        L.nmf_read.restype = i32
        L.nmf_profile.argtypes = [p, i32, p, p]
        L.nmf_profile.restype = i32
        L.nmf_destroy.argtypes = [p]
        L.nmf_destroy.restype = None
        L.nmf_last_error.argtypes = [p]
        L.nmf_last_error.restype = C.c_char_p
        L.nmf_read_beta_star.argtypes = [p, p, i32, p]
        L.nmf_read_beta_star.restype = i32
        L.nmf_read_sweeps.argtypes = [p, p, i32, p]
        L.nmf_read_sweeps.restype = i32
        L.nmf_set_error_scale.argtypes = [p, p, i32]
        L.nmf_set_error_scale.restype = i32
        L.nmf_solve_noalloc.argtypes = [p, C.c_int64, C.c_int64, p, p, p, p, p, p, p, p, p, p]
        L.nmf_solve_noalloc.restype = i32
        L.nmf_state_size.argtypes = [p, p]
        L.nmf_state_size.restype = i32
        L.nmf_save_state.argtypes = [p, p, C.c_size_t, p]
        L.nmf_save_state.restype = i32
        L.nmf_load_state.argtypes = [p, p, C.c_size_t, p]
        L.nmf_load_state.restype = i32
        L.nmf_batch_create.argtypes = [p, p]
        L.nmf_batch_create.restype = i32
        L.nmf_batch_submit.argtypes = [p, p, p, p, p, p]
        L.nmf_batch_submit.restype = i32
        L.nmf_batch_step.argtypes = [p, i32, p, p, p]
        L.nmf_batch_step.restype = i32
        L.nmf_batch_result.argtypes = [p, C.c_int64, p, p, p, i32, p, p, p]
        L.nmf_batch_result.restype = i32
        L.nmf_batch_destroy.argtypes = [p]
        L.nmf_batch_destroy.restype = None
        _lib = L
    return _lib


def make_params(r, **kw) -> Params:
    prm = Params()
    lib().nmf_params_default(C.byref(prm))
    prm.r = r
    for k, v in kw.items():
        if not hasattr(prm, k):
            raise TypeError(f"unknown parameter {k!r}")
        setattr(prm, k, int(v) if isinstance(v, (enum.IntEnum, bool)) else v)
    return prm


def _ptr(a):
    return C.c_void_p(a.ctypes.data)


def _current_device():
    """Index of the current HIP device as torch sees it (the device a new
    context binds to), or None without a usable torch."""
    try:
        import torch
        return torch.cuda.current_device() if torch.cuda.is_available() else None
    except ImportError:
        return None


def _check_device_tensor(t, shape, name, device):
    """A torch tensor handed to the library as a raw device pointer must be a
    contiguous float32 tensor of exactly `shape` on the context's device;
    anything else would make the kernels read or write past it."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor like the others")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not t.is_cuda or (device is not None and t.device.index != device):
        raise ValueError(f"{name} must live on cuda:{device}, got {t.device}")


def _stream(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


@dataclasses.dataclass
class Result:
    W: np.ndarray
    H: np.ndarray
    trace: np.ndarray
    accepted: np.ndarray
    beta: np.ndarray
    n_iter: int


class Solver:
    """One context: X resident on the current GPU, reusable for many solves.

    ``X`` is a float32 (m, n) numpy array, or an object with ``m, n,
    row_ptr, col_idx, val`` (CSR). Keyword arguments set nmf_params fields
    (hp, beta0, gamma, gamma_bar, eta, inner_rule, inner_k, inner_alpha,
    inner_delta, inner_rho_h, inner_rho_w, max_iter, tol, x_dtype, prod,
    flags)."""

    def __init__(self, X, r, **params):
        self._ctx = C.c_void_p()
        self.params = make_params(r, **params)
        mat = _Matrix()
        keep = []
        if hasattr(X, "row_ptr"):
            rp = np.ascontiguousarray(X.row_ptr, dtype=np.int64)
            ci = np.ascontiguousarray(X.col_idx, dtype=np.int32)
            va = np.ascontiguousarray(X.val, dtype=np.float32)
            keep += [rp, ci, va]
            mat.fmt, mat.m, mat.n = Format.CSR, X.m, X.n
            mat.row_ptr, mat.col_idx, mat.val = rp.ctypes.data, ci.ctypes.data, va.ctypes.data
            mat.nnz = int(rp[-1])
        else:
            Xd = np.ascontiguousarray(X, dtype=np.float32)
            keep.append(Xd)
            mat.fmt, (mat.m, mat.n) = Format.DENSE, Xd.shape
            mat.dense = Xd.ctypes.data
        self.m, self.n, self.r = int(mat.m), int(mat.n), int(r)
        self.device = _current_device()
        st = lib().nmf_create(C.byref(mat), C.byref(self.params), C.byref(self._ctx))
        if st != Status.OK:
            raise NMFError(st, lib().nmf_last_error(None).decode())

    # ------------------------------------------------------------ helpers
    def _check(self, st):
        if st != Status.OK:
            raise NMFError(st, lib().nmf_last_error(self._ctx).decode())

    def close(self):
        if self._ctx:
            lib().nmf_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---------------------------------------------------------- entry points
    def solve(self, W0, H0) -> Result:
        """nmf_solve: host in, host out, synchronous."""
        W0 = np.ascontiguousarray(W0, dtype=np.float32)
        H0 = np.ascontiguousarray(H0, dtype=np.float32)
        if W0.shape != (self.m, self.r) or H0.shape != (self.r, self.n):
            raise ValueError("W0 must be (m, r) and H0 (r, n)")
        cap = self.params.max_iter + 1
        W = np.empty((self.m, self.r), np.float32)
        H = np.empty((self.r, self.n), np.float32)
        trace = np.zeros(cap)
        acc = np.zeros(max(cap - 1, 1), np.uint8)
        beta = np.zeros(max(cap - 1, 1))
        nit = C.c_int32()
        self._check(lib().nmf_solve(self._ctx, _ptr(W0), _ptr(H0), _ptr(W), _ptr(H),
                                    _ptr(trace), cap, C.byref(nit), _ptr(acc),
                                    _ptr(beta)))
        k = nit.value
        return Result(W, H, trace[:k + 1], acc[:k].astype(bool), beta[:k], k)

    def start(self, W0, H0, stream=None):
        """nmf_start from numpy (host) or torch CUDA tensors (device)."""
        if hasattr(W0, "data_ptr"):
            _check_device_tensor(W0, (self.m, self.r), "W0", self.device)
            _check_device_tensor(H0, (self.r, self.n), "H0", self.device)
            self._check(lib().nmf_start(self._ctx, C.c_void_p(W0.data_ptr()),
                                        C.c_void_p(H0.data_ptr()), 1, _stream(stream)))
        else:
            W0 = np.ascontiguousarray(W0, dtype=np.float32)
            H0 = np.ascontiguousarray(H0, dtype=np.float32)
            if W0.shape != (self.m, self.r) or H0.shape != (self.r, self.n):
                raise ValueError("W0 must be (m, r) and H0 (r, n)")
            self._check(lib().nmf_start(self._ctx, _ptr(W0), _ptr(H0), 0, _stream(stream)))

    def set_error_scale(self, scale=None):
        """nmf_set_error_scale (test hook): factors applied to e(k)^2 for
        k = 0, 1, ... from the next start on; None removes them."""
        if scale is None:
            self._check(lib().nmf_set_error_scale(self._ctx, None, 0))
            return
        sc = np.ascontiguousarray(scale, dtype=np.float64).ravel()
        self._check(lib().nmf_set_error_scale(self._ctx, _ptr(sc), sc.size))

    def save_state(self, stream=None) -> bytes:
        """nmf_save_state: the solver state after the last completed iteration."""
        size = C.c_size_t()
        self._check(lib().nmf_state_size(self._ctx, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        self._check(lib().nmf_save_state(self._ctx, buf, size.value, _stream(stream)))
        return buf.raw

    def load_state(self, state: bytes, stream=None):
        """nmf_load_state: continue a solve from a saved state."""
        buf = C.create_string_buffer(bytes(state), len(state))
        self._check(lib().nmf_load_state(self._ctx, buf, len(state), _stream(stream)))

    def iterate(self, iters, stream=None):
        self._check(lib().nmf_iterate(self._ctx, int(iters), _stream(stream)))

    def profile(self, iters, stream=None):
        """nmf_profile: average ms of each kernel of an outer iteration over
        `iters` eager iterations, keyed by PHASES."""
        ms = np.zeros(len(PHASES))
        self._check(lib().nmf_profile(self._ctx, int(iters), _stream(stream), _ptr(ms)))
        return {name: float(v) for name, v in zip(PHASES, ms)}

    def read_beta_star(self):
        """nmf_read_beta_star: the beta* diagnostic of section 4 for each
        completed iteration (the context must have FLAG_BETA_STAR)."""
        cap = max(self.params.max_iter, 1)
        out = np.zeros(cap)
        nit = C.c_int32()
        self._check(lib().nmf_read_beta_star(self._ctx, _ptr(out), cap, C.byref(nit)))
        return out[:nit.value]

    def read_sweeps(self):
        """nmf_read_sweeps: HALS sweeps run on H and on W in each completed
        iteration, as an (n_iter, 2) array."""
        cap = max(self.params.max_iter, 1)
        out = np.zeros((cap, 2), dtype=np.int32)
        nit = C.c_int32()
        self._check(lib().nmf_read_sweeps(self._ctx, _ptr(out), cap, C.byref(nit)))
        return out[:nit.value]

    def read(self, W=None, H=None, stream=None) -> Result:
        """nmf_read into host arrays, or into given torch CUDA tensors."""
        cap = self.params.max_iter + 1
        trace = np.zeros(cap)
        acc = np.zeros(max(cap - 1, 1), np.uint8)
        beta = np.zeros(max(cap - 1, 1))
        nit = C.c_int32()
        if W is not None and hasattr(W, "data_ptr"):
            _check_device_tensor(W, (self.m, self.r), "W", self.device)
            _check_device_tensor(H, (self.r, self.n), "H", self.device)
            self._check(lib().nmf_read(self._ctx, C.c_void_p(W.data_ptr()),
                                       C.c_void_p(H.data_ptr()), 1, _ptr(trace), cap,
                                       C.byref(nit), _ptr(acc), _ptr(beta), _stream(stream)))
            Wout, Hout = W, H
        else:
            Wout = np.empty((self.m, self.r), np.float32)
            Hout = np.empty((self.r, self.n), np.float32)
            self._check(lib().nmf_read(self._ctx, _ptr(Wout), _ptr(Hout), 0, _ptr(trace),
                                       cap, C.byref(nit), _ptr(acc), _ptr(beta),
                                       _stream(stream)))
        k = nit.value
        return Result(Wout, Hout, trace[:k + 1], acc[:k].astype(bool), beta[:k], k)


def solve(X, r, W0, H0, **params) -> Result:
    """One-shot solve: create a context, run nmf_solve, destroy it."""
    with Solver(X, r, **params) as s:
        return s.solve(W0, H0)


def solve_noalloc(X, r, W0, H0, W, H, trace, info, accepted=None, beta=None, stream=None,
                  **params):
    """nmf_solve_noalloc on torch CUDA tensors: X (m, n), W0 (m, r), H0 (r, n)
    float32 inputs; W (m, r), H (r, n) float32, trace (>= max_iter + 1)
    float64, info (2,) int32 and the optional accepted (uint8) and beta
    (float64, >= max_iter each) outputs, all on the current device. Enqueues
    the solve on `stream` and returns without waiting."""
    import torch
    prm = make_params(r, **params)
    m, n = int(X.shape[0]), int(X.shape[1])
    dev = _current_device()
    _check_device_tensor(X, (m, n), "X", dev)
    for t, shape, name in ((W0, (m, r), "W0"), (H0, (r, n), "H0"), (W, (m, r), "W"),
                           (H, (r, n), "H")):
        _check_device_tensor(t, shape, name, dev)
    iters = max(prm.max_iter, 1)
    for t, dt, size, name in ((trace, torch.float64, prm.max_iter + 1, "trace"),
                              (info, torch.int32, 2, "info"),
                              (accepted, torch.uint8, iters, "accepted"),
                              (beta, torch.float64, iters, "beta")):
        if t is None and name in ("accepted", "beta"):
            continue
        if (t is None or t.dtype != dt or not t.is_cuda or t.device.index != dev
                or not t.is_contiguous() or t.numel() < size):
            raise ValueError(f"{name} must be a contiguous {dt} tensor of at least {size} "
                             f"entries on cuda:{dev}")
    ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
    st = lib().nmf_solve_noalloc(ptr(X), m, n, C.byref(prm), ptr(W0), ptr(H0), ptr(W), ptr(H),
                                 ptr(trace), ptr(accepted), ptr(beta), ptr(info),
                                 _stream(stream))
    if st != Status.OK:
        raise NMFError(st, lib().nmf_last_error(None).decode())


class _BatchParams(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_active", C.c_int32),
                ("check_every", C.c_int32)]


class Batch:
    """Batched solves (nmf_batch_*): many independent small dense problems
    advanced together on the current GPU, inside a device arena of
    ``hbm_budget`` bytes."""

    def __init__(self, hbm_budget, max_active=256, check_every=10):
        self._b = C.c_void_p()
        bp = _BatchParams(int(hbm_budget), int(max_active), int(check_every))
        st = lib().nmf_batch_create(C.byref(bp), C.byref(self._b))
        if st != Status.OK:
            raise NMFError(st, lib().nmf_last_error(None).decode())
        self._shapes = {}

    def _check(self, st):
        if st != Status.OK:
            raise NMFError(st, lib().nmf_last_error(None).decode())

    def submit(self, X, r, W0, H0, **params):
        """Queues one problem; returns its ticket."""
        Xd = np.ascontiguousarray(X, dtype=np.float32)
        W0 = np.ascontiguousarray(W0, dtype=np.float32)
        H0 = np.ascontiguousarray(H0, dtype=np.float32)
        m, n = Xd.shape
        if W0.shape != (m, r) or H0.shape != (r, n):
            raise ValueError("W0 must be (m, r) and H0 (r, n)")
        mat = _Matrix()
        mat.fmt, mat.m, mat.n = Format.DENSE, m, n
        mat.dense = Xd.ctypes.data
        prm = make_params(r, **params)
        t = C.c_int64()
        self._check(lib().nmf_batch_submit(self._b, C.byref(mat), C.byref(prm), _ptr(W0),
                                           _ptr(H0), C.byref(t)))
        self._shapes[t.value] = (m, n, r, prm.max_iter)
        return t.value

    def step(self, iters=1):
        """Advances the batch; returns (active, queued, retired-unread)."""
        a, q, d = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(lib().nmf_batch_step(self._b, int(iters), C.byref(a), C.byref(q), C.byref(d)))
        return a.value, q.value, d.value

    def result(self, ticket):
        """The Result of a retired problem, or None while it is pending."""
        m, n, r, max_iter = self._shapes[ticket]
        W = np.empty((m, r), np.float32)
        H = np.empty((r, n), np.float32)
        trace = np.zeros(max_iter + 1)
        acc = np.zeros(max(max_iter, 1), np.uint8)
        beta = np.zeros(max(max_iter, 1))
        nit = C.c_int32()
        st = lib().nmf_batch_result(self._b, int(ticket), _ptr(W), _ptr(H), _ptr(trace),
                                    max_iter + 1, C.byref(nit), _ptr(acc), _ptr(beta))
        if st == Status.PENDING:
            return None
        self._check(st)
        del self._shapes[ticket]
        k = nit.value
        return Result(W, H, trace[:k + 1], acc[:k].astype(bool), beta[:k], k)

    def close(self):
        if self._b:
            lib().nmf_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
