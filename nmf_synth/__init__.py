"""Seeded synthetic workloads for NMF (inputs only, no NMF arithmetic).

This module is shared by the FP64 oracle tests and the GPU path. It draws
random matrices and nothing else: it never factorizes, updates or evaluates
an NMF. Every workload is reproducible from its seed (numpy PCG64).

Conventions (the experimental set-up of Ang & Gillis, section 5.2):
  * data seed ``s``; the initial iterate uses seed ``s + 1000``, with the
    entries of W0 and H0 drawn uniformly in [0, 1];
  * matrices are drawn in float64 and rounded once to float32, and both the
    oracle and the GPU receive those float32 values.

Workloads (the sizes and structures of the paper's experiments, section 5.1):
  ``lowrank``   X = W0 H0 with W0, H0 ~ U[0,1] (the low-rank synthetic set)
  ``fullrank``  X ~ U[0,1] (the full-rank synthetic set)
  ``imagelike`` dense stand-in for the face-image sets of Table 1
  ``doclike``   CSR stand-in for the text-mining sets of Table 2
  ``planted``   X = W0 H0 + noise * |N(0,1)|, the large dense case
  ``requests``  a Poisson stream of independent small NMF problems
None of the paper's real data sets is reproduced: their shapes, densities and
value distributions are imitated by random draws.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem", "Csr", "init_factors", "lowrank", "fullrank", "imagelike",
    "doclike", "planted", "csr_to_dense", "dense_to_csr", "Request",
    "requests", "request_problem",
]


@dataclasses.dataclass
class Csr:
    """Compressed sparse rows: int64 row_ptr, int32 col_idx (sorted per row,
    no duplicates), float32 values."""
    m: int
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


@dataclasses.dataclass
class Problem:
    """One NMF instance: X (dense float32 array or Csr), rank r, initial
    iterate W0 (m x r) and H0 (r x n), both float32 and nonnegative."""
    name: str
    X: object
    r: int
    W0: np.ndarray
    H0: np.ndarray
    seed: int

    @property
    def m(self) -> int:
        return self.X.m if isinstance(self.X, Csr) else self.X.shape[0]

    @property
    def n(self) -> int:
        return self.X.n if isinstance(self.X, Csr) else self.X.shape[1]


def init_factors(m: int, n: int, r: int, seed: int):
    """W0 ~ U[0,1]^{m x r}, H0 ~ U[0,1]^{r x n} from seed ``seed + 1000``."""
    rng = np.random.default_rng(seed + 1000)
    W0 = rng.random((m, r)).astype(np.float32)
    H0 = rng.random((r, n)).astype(np.float32)
    return W0, H0


def lowrank(seed: int, m: int = 200, n: int = 200, r: int = 10) -> Problem:
    """Low-rank synthetic set: X = W H with W, H ~ U[0,1] (section 5.1)."""
    rng = np.random.default_rng(seed)
    Wt = rng.random((m, r))
    Ht = rng.random((r, n))
    X = (Wt @ Ht).astype(np.float32)
    W0, H0 = init_factors(m, n, r, seed)
    return Problem("lowrank", X, r, W0, H0, seed)


def fullrank(seed: int, m: int = 200, n: int = 200, r: int = 20) -> Problem:
    """Full-rank synthetic set: X ~ U[0,1] entrywise (section 5.1)."""
    rng = np.random.default_rng(seed)
    X = rng.random((m, n)).astype(np.float32)
    W0, H0 = init_factors(m, n, r, seed)
    return Problem("fullrank", X, r, W0, H0, seed)


def imagelike(seed: int, m: int = 10000, n: int = 2000, r: int = 49,
              density: float = 0.3, noise: float = 0.01) -> Problem:
    """Dense image-like data: X = relu(W H + noise N(0,1)) / max, with W
    sparse-uniform (``density`` nonzeros) and H ~ U[0,1]. Pixels (rows) by
    images (columns), values in [0, 1], like the face sets of Table 1."""
    rng = np.random.default_rng(seed)
    Wt = (rng.random((m, r)) < density) * rng.random((m, r))
    Ht = rng.random((r, n))
    X = Wt @ Ht
    X += noise * rng.standard_normal((m, n))
    np.maximum(X, 0.0, out=X)
    mx = X.max()
    if mx > 0:
        X /= mx
    X = X.astype(np.float32)
    W0, H0 = init_factors(m, n, r, seed)
    return Problem("imagelike", X, r, W0, H0, seed)


def _zipf_ranks(rng, count: int, nranks: int, s: float) -> np.ndarray:
    p = np.arange(1, nranks + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    u = rng.random(count)
    return np.minimum(np.searchsorted(cdf, u, side="right"), nranks - 1)


def doclike(seed: int, m: int = 30000, n: int = 20000, r: int = 20,
            nnz: int = 1_800_000, zipf_s: float = 1.1) -> Problem:
    """Sparse term-document data in CSR (rows = terms, columns = documents).

    (term, doc) pairs are drawn with term ~ truncated Zipf(``zipf_s``) over
    ranks 1..m (row = rank - 1) and doc ~ U{0..n-1}; duplicates are dropped
    and more pairs drawn until at least ``nnz`` distinct pairs exist, then a
    random subset of exactly ``nnz`` is kept. Values ~ lognormal(0, 1); every
    nonempty column is scaled to unit Euclidean norm (tf-idf-like, as for
    the text-mining sets of Table 2)."""
    rng = np.random.default_rng(seed)
    keys = np.empty(0, dtype=np.int64)
    while keys.size < nnz:
        need = nnz - keys.size
        draw = max(int(need * 1.5), 1024)
        t = _zipf_ranks(rng, draw, m, zipf_s).astype(np.int64)
        d = rng.integers(0, n, size=draw, dtype=np.int64)
        keys = np.unique(np.concatenate([keys, t * n + d]))
    if keys.size > nnz:
        keep = rng.choice(keys.size, size=nnz, replace=False)
        keys = np.sort(keys[keep])
    rows = keys // n
    cols = (keys % n).astype(np.int32)
    vals = rng.lognormal(0.0, 1.0, size=nnz)
    colsq = np.bincount(cols, weights=vals * vals, minlength=n)
    scale = np.zeros(n)
    nzc = colsq > 0
    scale[nzc] = 1.0 / np.sqrt(colsq[nzc])
    vals = (vals * scale[cols]).astype(np.float32)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    X = Csr(m, n, row_ptr, cols, vals)
    W0, H0 = init_factors(m, n, r, seed)
    return Problem("doclike", X, r, W0, H0, seed)


def planted(seed: int, m: int = 16384, n: int = 16384, r: int = 64,
            noise: float = 1e-3, block: int = 1024) -> Problem:
    """Planted nonnegative rank-r data: X = W H + noise |N(0,1)| with W, H ~
    U[0,1]. Rows are produced in blocks of ``block`` (float64, then float32)
    so that the largest case never holds X in float64."""
    rng = np.random.default_rng(seed)
    Wt = rng.random((m, r))
    Ht = rng.random((r, n))
    X = np.empty((m, n), dtype=np.float32)
    for i0 in range(0, m, block):
        i1 = min(m, i0 + block)
        blk = Wt[i0:i1] @ Ht
        blk += noise * np.abs(rng.standard_normal((i1 - i0, n)))
        X[i0:i1] = blk
    W0, H0 = init_factors(m, n, r, seed)
    return Problem("planted", X, r, W0, H0, seed)


def csr_to_dense(A: Csr) -> np.ndarray:
    D = np.zeros((A.m, A.n), dtype=np.float32)
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    D[rows, A.col_idx] = A.val
    return D


def dense_to_csr(D: np.ndarray) -> Csr:
    D = np.asarray(D, dtype=np.float32)
    m, n = D.shape
    rows, cols = np.nonzero(D)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    return Csr(m, n, row_ptr, cols.astype(np.int32), D[rows, cols].copy())


@dataclasses.dataclass
class Request:
    """One request of the serving stream: arrival time (s), shape, seed."""
    rid: int
    t_arrive: float
    m: int
    n: int
    r: int
    seed: int


def requests(count: int = 4096, qps: float = 100.0, seed: int = 0,
             mn_range=(64, 2048), ranks=(5, 10, 20, 40)):
    """A Poisson request stream: exponential inter-arrival gaps at rate
    ``qps``, m and n ~ U{lo..hi}, r uniform over ``ranks``."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps) - gaps[0]
    lo, hi = mn_range
    ms = rng.integers(lo, hi + 1, size=count)
    ns = rng.integers(lo, hi + 1, size=count)
    rs = rng.choice(np.asarray(ranks), size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return [Request(i, float(t[i]), int(ms[i]), int(ns[i]), int(rs[i]),
                    int(seeds[i])) for i in range(count)]


def request_problem(req: Request, noise_frac: float = 0.01) -> Problem:
    """The data of one request: X = max(0, W H + noise_frac * RMS(W H) *
    N(0,1)) with planted W, H ~ U[0,1] (nonnegative low rank plus 1% noise)."""
    rng = np.random.default_rng(req.seed)
    Wt = rng.random((req.m, req.r))
    Ht = rng.random((req.r, req.n))
    X = Wt @ Ht
    rms = math.sqrt(float(np.mean(X * X)))
    X += noise_frac * rms * rng.standard_normal(X.shape)
    np.maximum(X, 0.0, out=X)
    W0, H0 = init_factors(req.m, req.n, req.r, req.seed)
    return Problem("request", X.astype(np.float32), req.r, W0, H0, req.seed)
