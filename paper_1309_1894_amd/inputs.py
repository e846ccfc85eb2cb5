"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module only draws numbers and builds sparsity patterns; it contains none
of the arithmetic of the kernels it feeds (no product, sum, WAXPY or dot).
It depends on numpy alone and never loads the HIP library or the oracle.

Random numbers come from one counter-based generator: the SplitMix64 output
function of Steele, Lea and Flood ("Fast splittable pseudorandom number
generators", OOPSLA 2014).  The i-th draw of stream ``s`` under seed ``seed``
is ``mix64(key(seed, s) + (i + 1) * GAMMA)`` (all arithmetic mod 2**64), which
is exactly the i-th output of a SplitMix64 generator whose state starts at
``key(seed, s)``.  numpy's distribution methods are avoided because their
output is not stable across numpy versions.

Workloads (the abstract names no matrices; these follow the problem sizes the
library is specified against):

* ``lap2d(N)``  -- 5-point Laplacian on an N x N grid, Dirichlet boundary
  (out-of-grid couplings dropped), diagonal 4, off-diagonals -1, row
  r = i*N + j, columns sorted.  nnz = 5 N^2 - 4 N.
* ``lap3d(N)``  -- 7-point analogue on N^3, diagonal 6, off-diagonals -1,
  r = (i*N + j)*N + k.  nnz = 7 N^3 - 6 N^2.
* ``zipf(m, ...)`` -- row lengths i.i.d. truncated Zipf P(L=k) ~ k^-s on
  1..min(kmax, n); one seed-chosen row forced to the maximum length; columns
  uniform without replacement, sorted; values uniform[-1, 1).
* ``spd_zipf(m)`` -- the zipf pattern made symmetric (each unordered pair
  {i, j} of an entry gets one value uniform[-1, 1)), plus a diagonal of
  1 + (off-diagonal entries in the row): strictly diagonally dominant,
  hence symmetric positive definite (the conjugate-gradient input with
  irregular rows).
* ``banded(m, b, fill)`` -- every position with |r - c| <= b kept
  independently with probability ``fill``; values uniform[-1, 1).
* ``batch_banded(count, ...)`` -- ``count`` banded instances with row counts
  floor(64 * 256**u) (log-uniform in [64, 16384)) and half-bandwidths uniform
  in [1, 32], concatenated with per-instance offsets.
* ``poisson_arrivals(n, rate)`` -- exponential inter-arrival gaps.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_S30 = np.uint64(30)
_S27 = np.uint64(27)
_S31 = np.uint64(31)
_S11 = np.uint64(11)
_S40 = np.uint64(40)

# Exponent of the truncated Zipf law whose mean on 1..4096 is 16.0.
ZIPF_S_MEAN16 = 1.729570


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output mixing function on a uint64 array (wraps mod 2**64)."""
    z = np.asarray(z, dtype=np.uint64)
    z = (z ^ (z >> _S30)) * _M1
    z = (z ^ (z >> _S27)) * _M2
    return z ^ (z >> _S31)


def stream_key(seed: int, stream: int) -> np.uint64:
    """Starting state of stream ``stream`` under ``seed``."""
    with np.errstate(over="ignore"):
        a = mix64(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))
        b = a + np.uint64(stream & 0xFFFFFFFFFFFFFFFF) * GAMMA
        return mix64(b)[0]


def u64(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Draws ``start .. start+count-1`` of one stream as uint64."""
    key = stream_key(seed, stream)
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + idx * GAMMA)


def u64_at(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Draws at arbitrary counter positions ``idx`` (uint64/int64 array)."""
    key = stream_key(seed, stream)
    with np.errstate(over="ignore"):
        return mix64(key + (np.asarray(idx, dtype=np.uint64) + np.uint64(1)) * GAMMA)


def splitmix64_sequence(state: int, count: int) -> list[int]:
    """The plain SplitMix64 sequence from a raw 64-bit state (for pinning)."""
    idx = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        out = mix64(np.uint64(state) + idx * GAMMA)
    return [int(v) for v in out]


def unit_from_u64(u: np.ndarray) -> np.ndarray:
    """uint64 -> float64 in [0, 1) on the 2^-53 grid."""
    return (u >> _S11).astype(np.float64) * (2.0 ** -53)


def sym_f64(u: np.ndarray) -> np.ndarray:
    """uint64 -> float64 uniform in [-1, 1); exact, never subnormal."""
    return unit_from_u64(u) * 2.0 - 1.0


def sym_f32(u: np.ndarray) -> np.ndarray:
    """uint64 -> float32 uniform in [-1, 1) on the 2^-23 grid (exact)."""
    k = (u >> _S40).astype(np.float32)
    return (k * np.float32(2.0 ** -24)) * np.float32(2.0) - np.float32(1.0)


def uniform(seed: int, stream: int, n: int, dtype=np.float64, start: int = 0) -> np.ndarray:
    """n values uniform in [-1, 1) of the given dtype (float64 or float32)."""
    u = u64(seed, stream, start, n)
    if np.dtype(dtype) == np.float64:
        return sym_f64(u)
    if np.dtype(dtype) == np.float32:
        return sym_f32(u)
    raise ValueError(f"unsupported dtype {dtype}")


@dataclasses.dataclass
class CSR:
    """Host CSR matrix: int32 indices, float64 or float32 values."""

    nrows: int
    ncols: int
    row_ptr: np.ndarray  # int32[nrows + 1]
    col_idx: np.ndarray  # int32[nnz]
    val: np.ndarray      # float64|float32[nnz]

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def dtype(self):
        return self.val.dtype

    def astype(self, dtype) -> "CSR":
        return CSR(self.nrows, self.ncols, self.row_ptr, self.col_idx, self.val.astype(dtype))

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def _csr_from_sorted(nrows: int, ncols: int, rows: np.ndarray, cols: np.ndarray, val: np.ndarray) -> CSR:
    counts = np.bincount(rows, minlength=nrows) if rows.size else np.zeros(nrows, np.int64)
    rp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    if rp[-1] >= 2 ** 31:
        raise ValueError("nnz exceeds int32 indexing")
    return CSR(nrows, ncols, rp.astype(np.int32), cols.astype(np.int32), val)


def lap2d(N: int, dtype=np.float64) -> CSR:
    """5-point Laplacian, Dirichlet, diag 4 / off -1, sorted columns."""
    n = N * N
    r = np.arange(n, dtype=np.int64)
    i, j = r // N, r % N
    # candidate offsets in ascending column order: -N, -1, 0, +1, +N
    offs = np.array([-N, -1, 0, 1, N], dtype=np.int64)
    vals = np.array([-1, -1, 4, -1, -1], dtype=dtype)
    ok = np.stack([i > 0, j > 0, np.ones(n, bool), j < N - 1, i < N - 1], axis=1)
    cols = r[:, None] + offs[None, :]
    rows = np.broadcast_to(r[:, None], cols.shape)
    v = np.broadcast_to(vals[None, :], cols.shape)
    return _csr_from_sorted(n, n, rows[ok], cols[ok], np.ascontiguousarray(v[ok]))


def lap3d(N: int, dtype=np.float64) -> CSR:
    """7-point Laplacian, Dirichlet, diag 6 / off -1, sorted columns."""
    n = N * N * N
    r = np.arange(n, dtype=np.int64)
    i, j, k = r // (N * N), (r // N) % N, r % N
    offs = np.array([-N * N, -N, -1, 0, 1, N, N * N], dtype=np.int64)
    vals = np.array([-1, -1, -1, 6, -1, -1, -1], dtype=dtype)
    ok = np.stack([i > 0, j > 0, k > 0, np.ones(n, bool), k < N - 1, j < N - 1, i < N - 1], axis=1)
    cols = r[:, None] + offs[None, :]
    rows = np.broadcast_to(r[:, None], cols.shape)
    v = np.broadcast_to(vals[None, :], cols.shape)
    return _csr_from_sorted(n, n, rows[ok], cols[ok], np.ascontiguousarray(v[ok]))


def zipf_lengths(m: int, kmax: int, s: float, seed: int, stream: int) -> np.ndarray:
    """m i.i.d. truncated-Zipf row lengths on 1..kmax; one row forced to kmax."""
    k = np.arange(1, kmax + 1, dtype=np.float64)
    pmf = k ** (-s)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    u = unit_from_u64(u64(seed, stream, 0, m))
    lengths = np.searchsorted(cdf, u, side="right").astype(np.int64) + 1
    np.minimum(lengths, kmax, out=lengths)
    if m > 0:
        forced = int(u64(seed, stream + 1, 0, 1)[0] % np.uint64(m))
        lengths[forced] = kmax
    return lengths


def _distinct_sorted_cols(rows: np.ndarray, ncols: int, seed: int, stream: int) -> np.ndarray:
    """Uniform column per slot, redrawn until every row is duplicate-free; sorted within rows."""
    nnz = rows.size
    cols = np.floor(unit_from_u64(u64(seed, stream, 0, nnz)) * ncols).astype(np.int64)
    rnd = 1
    while True:
        key = rows * ncols + cols
        order = np.argsort(key, kind="stable")
        rows, cols, key = rows[order], cols[order], key[order]
        dup = np.zeros(nnz, dtype=bool)
        if nnz > 1:
            dup[1:] = key[1:] == key[:-1]
        nd = int(dup.sum())
        if nd == 0:
            return cols
        where = np.nonzero(dup)[0]
        cols[where] = np.floor(unit_from_u64(u64_at(seed, stream + rnd, where)) * ncols).astype(np.int64)
        rnd += 1


def zipf(m: int, n: int | None = None, mean_target_s: float = ZIPF_S_MEAN16, kmax: int = 4096,
         seed_struct: int = 32, seed_val: int = 33, dtype=np.float64) -> CSR:
    """Random matrix with truncated-Zipf row lengths (mean 16 at s=1.72957, max 4096)."""
    n = m if n is None else n
    kcap = max(1, min(kmax, n))
    lengths = zipf_lengths(m, kcap, mean_target_s, seed_struct, 0) if n > 0 else np.zeros(m, np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), lengths)
    cols = _distinct_sorted_cols(rows, n, seed_struct, 100) if rows.size else rows
    val = uniform(seed_val, 0, rows.size, dtype)
    return _csr_from_sorted(m, n, rows, cols, val)


def spd_zipf(m: int, kmax: int = 4096, s: float = ZIPF_S_MEAN16, seed_struct: int = 34,
             seed_val: int = 35) -> CSR:
    """Symmetric positive definite matrix on the symmetrized zipf pattern.

    Off-diagonal values |v| < 1 and diagonal 1 + (off-diagonal count of the
    row) make every row strictly diagonally dominant."""
    Z = zipf(m, m, s, kmax, seed_struct, seed_val)
    rows = np.repeat(np.arange(m, dtype=np.int64), Z.row_lengths())
    cols = Z.col_idx.astype(np.int64)
    off = rows != cols
    lo, hi = np.minimum(rows[off], cols[off]), np.maximum(rows[off], cols[off])
    key = np.unique(lo * m + hi)
    lo, hi = key // m, key % m
    v = sym_f64(u64_at(seed_val, 1, key.astype(np.uint64)))
    diag = np.arange(m, dtype=np.int64)
    r = np.concatenate([lo, hi, diag])
    c = np.concatenate([hi, lo, diag])
    deg = np.bincount(np.concatenate([lo, hi]), minlength=m).astype(np.float64)
    vals = np.concatenate([v, v, 1.0 + deg])
    order = np.lexsort((c, r))
    return _csr_from_sorted(m, m, r[order], c[order], np.ascontiguousarray(vals[order]))


def banded(m: int, b: int, fill: float = 0.6, seed_struct: int = 41, seed_val: int = 42,
           stream: int = 0, dtype=np.float64) -> CSR:
    """Square banded matrix: positions |r-c| <= b kept independently with probability fill."""
    b = max(0, min(b, m - 1))
    w = 2 * b + 1
    r = np.arange(m, dtype=np.int64)
    c = r[:, None] + np.arange(-b, b + 1, dtype=np.int64)[None, :]
    cand = np.arange(m * w, dtype=np.int64).reshape(m, w)
    keep = unit_from_u64(u64_at(seed_struct, 1000 + stream, cand)) < fill
    keep &= (c >= 0) & (c < m)
    rows = np.broadcast_to(r[:, None], c.shape)[keep]
    cols = c[keep]
    val = uniform(seed_val, stream, rows.size, dtype)
    return _csr_from_sorted(m, m, rows, cols, val)


@dataclasses.dataclass
class Batch:
    """Concatenated independent square CSR instances.

    Instance i has ``m[i]`` rows; its row_ptr occupies
    ``row_ptr[rp_off[i] : rp_off[i] + m[i] + 1]`` with values local to the
    instance (starting at 0), its entries occupy ``col_idx/val[nz_off[i] :
    nz_off[i] + nnz[i]]`` with column indices local to the instance, and its
    vectors occupy ``[vec_off[i] : vec_off[i] + m[i]]`` of x, y and w.
    """

    m: np.ndarray        # int64[count]
    nnz: np.ndarray      # int64[count]
    band: np.ndarray     # int64[count] half-bandwidths
    rp_off: np.ndarray   # int64[count]
    nz_off: np.ndarray   # int64[count]
    vec_off: np.ndarray  # int64[count]
    row_ptr: np.ndarray  # int32
    col_idx: np.ndarray  # int32
    val: np.ndarray

    @property
    def count(self) -> int:
        return int(self.m.shape[0])

    def instance(self, i: int) -> CSR:
        m, ro, zo = int(self.m[i]), int(self.rp_off[i]), int(self.nz_off[i])
        nz = int(self.nnz[i])
        return CSR(m, m, self.row_ptr[ro:ro + m + 1], self.col_idx[zo:zo + nz], self.val[zo:zo + nz])


def batch_sizes(count: int, seed: int = 41, mmin: int = 64, ratio: float = 256.0, bmax: int = 32):
    """Row counts floor(mmin * ratio**u) and half-bandwidths uniform in [1, bmax]."""
    u = unit_from_u64(u64(seed, 0, 0, count))
    m = np.floor(mmin * np.power(ratio, u)).astype(np.int64)
    ub = unit_from_u64(u64(seed, 1, 0, count))
    b = 1 + np.floor(ub * bmax).astype(np.int64)
    return m, b


def batch_from_instances(insts: list[CSR], band: np.ndarray | None = None) -> Batch:
    count = len(insts)
    m = np.array([a.nrows for a in insts], dtype=np.int64)
    nnz = np.array([a.nnz for a in insts], dtype=np.int64)
    rp_off = np.zeros(count, dtype=np.int64)
    nz_off = np.zeros(count, dtype=np.int64)
    vec_off = np.zeros(count, dtype=np.int64)
    if count:
        rp_off[1:] = np.cumsum(m[:-1] + 1)
        nz_off[1:] = np.cumsum(nnz[:-1])
        vec_off[1:] = np.cumsum(m[:-1])
    dtype = insts[0].val.dtype if count else np.float64
    row_ptr = np.concatenate([a.row_ptr for a in insts]) if count else np.zeros(0, np.int32)
    col_idx = np.concatenate([a.col_idx for a in insts]) if count else np.zeros(0, np.int32)
    val = np.concatenate([a.val for a in insts]) if count else np.zeros(0, dtype)
    return Batch(m, nnz, band if band is not None else np.zeros(count, np.int64),
                 rp_off, nz_off, vec_off, row_ptr, col_idx, val)


def batch_banded(count: int = 4096, fill: float = 0.6, seed_struct: int = 41, seed_val: int = 42,
                 mmin: int = 64, ratio: float = 256.0, bmax: int = 32, dtype=np.float64) -> Batch:
    """``count`` random banded instances with log-uniform sizes (the batched workload)."""
    m, b = batch_sizes(count, seed_struct, mmin, ratio, bmax)
    insts = [banded(int(m[i]), int(b[i]), fill, seed_struct, seed_val, stream=i, dtype=dtype)
             for i in range(count)]
    return batch_from_instances(insts, b)


def block_diagonal(batch: Batch) -> CSR:
    """The batch as one square block-diagonal CSR matrix: instance i's rows
    become rows vec_off[i].., its columns shifted by vec_off[i] (instances
    stored back to back, as batch_from_instances lays them out)."""
    nv = int(batch.m.sum())
    nz = int(batch.nnz.sum())
    rp = np.empty(nv + 1, dtype=np.int64)
    rp[nv] = nz
    keep = np.ones(batch.row_ptr.shape[0], dtype=bool)
    keep[(batch.rp_off + batch.m).astype(np.int64)] = False          # each instance's closing row_ptr entry
    local = batch.row_ptr[keep].astype(np.int64)
    rp[:nv] = local + np.repeat(batch.nz_off, batch.m)
    if nz >= 2 ** 31:
        raise ValueError("block-diagonal form needs nnz < 2^31")
    ci = batch.col_idx + np.repeat(batch.vec_off, batch.nnz).astype(np.int32)
    return CSR(nv, nv, rp.astype(np.int32), ci.astype(np.int32, copy=False), batch.val)


def batch_vector(batch: Batch, seed: int = 43, dtype=np.float64) -> np.ndarray:
    """Concatenated x for a batch: instance i draws from stream i."""
    parts = [uniform(seed, i, int(batch.m[i]), dtype) for i in range(batch.count)]
    return np.concatenate(parts) if parts else np.zeros(0, dtype)


def poisson_arrivals(n: int, rate: float, seed: int = 51, stream: int = 7) -> np.ndarray:
    """Arrival times (s) of an open-loop Poisson process with ``rate`` requests/s."""
    u = unit_from_u64(u64(seed, stream, 0, n))
    gaps = -np.log1p(-u) / rate
    return np.cumsum(gaps)


def log_uniform_int(lo: float, hi: float, seed: int, stream: int, n: int) -> np.ndarray:
    """n integers floor(lo * (hi/lo)**u)."""
    u = unit_from_u64(u64(seed, stream, 0, n))
    return np.floor(lo * np.power(hi / lo, u)).astype(np.int64)


def zipf_mean(s: float, kmax: int = 4096) -> float:
    k = np.arange(1, kmax + 1, dtype=np.float64)
    p = k ** (-s)
    return float((k * p).sum() / p.sum())


def expected_lap_nnz(N: int, dim: int) -> int:
    return 5 * N * N - 4 * N if dim == 2 else 7 * N ** 3 - 6 * N * N


__all__ = [name for name in dir() if not name.startswith("_") and name not in ("annotations", "math")]
