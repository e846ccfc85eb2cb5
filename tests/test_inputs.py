"""Pins of the seeded input generators (CPU only)."""
import os

import numpy as np
import pytest

from paper_1309_1894_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_vector():
    want = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_state1234567.txt")) if l.strip() and l[0] != "#"]
    assert I.splitmix64_sequence(1234567, len(want)) == want


def test_counter_streams_are_reproducible_and_distinct():
    a = I.u64(5, 0, 0, 1000)
    assert np.array_equal(a, I.u64(5, 0, 0, 1000))
    assert np.array_equal(a[100:200], I.u64(5, 0, 100, 100))
    assert np.array_equal(a[[3, 999]], I.u64_at(5, 0, np.array([3, 999])))
    assert not np.array_equal(a, I.u64(5, 1, 0, 1000))
    assert not np.array_equal(a, I.u64(6, 0, 0, 1000))


def test_uniform_ranges_exact_grid():
    x = I.uniform(1, 0, 200000)
    assert x.min() >= -1.0 and x.max() < 1.0
    assert abs(x.mean()) < 0.01
    assert np.all((np.abs(x) >= 2.0 ** -52) | (x == 0))   # never subnormal
    f = I.uniform(1, 0, 200000, np.float32)
    assert f.dtype == np.float32 and f.min() >= -1 and f.max() < 1
    assert np.all((f.astype(np.float64) * 2 ** 23) == np.round(f.astype(np.float64) * 2 ** 23))


@pytest.mark.parametrize("N", [1, 2, 3, 64, 256])
def test_lap2d_structure(N):
    A = I.lap2d(N)
    assert A.nnz == I.expected_lap_nnz(N, 2) == 5 * N * N - 4 * N
    assert A.row_ptr[0] == 0 and A.row_ptr[-1] == A.nnz
    for r in range(A.nrows):
        c = A.col_idx[A.row_ptr[r]:A.row_ptr[r + 1]]
        assert np.all(np.diff(c) > 0)
        v = A.val[A.row_ptr[r]:A.row_ptr[r + 1]]
        assert v[c == r] == 4 and np.all(v[c != r] == -1)
        if N > 8:
            break


def test_lap3d_nnz_matches_dirichlet_count():
    A = I.lap3d(128)
    assert A.nrows == 2097152 and A.nnz == 14581760
    assert A.nnz == 7 * 128 ** 3 - 6 * 128 ** 2   # periodic would be 7*128^3


def test_zipf_statistics():
    assert abs(I.zipf_mean(I.ZIPF_S_MEAN16) - 16.0) < 1e-3
    A = I.zipf(200000)
    L = A.row_lengths()
    assert L.max() == 4096 and L.min() >= 1
    assert abs((L == 1).mean() - 0.501) < 0.01
    assert 12 < L.mean() < 21
    for r in np.nonzero(L > 1)[0][:2000]:
        c = A.col_idx[A.row_ptr[r]:A.row_ptr[r + 1]]
        assert np.all(np.diff(c) > 0) and c.min() >= 0 and c.max() < A.ncols


def test_zipf_small_n_caps_lengths():
    A = I.zipf(1000, n=1000)
    assert A.row_lengths().max() == 1000


def test_banded_fill_and_band():
    A = I.banded(4000, 10, 0.6, stream=3)
    r = np.repeat(np.arange(A.nrows), A.row_lengths())
    assert np.all(np.abs(A.col_idx - r) <= 10)
    interior = 4000 * 21 - 2 * sum(range(1, 11))
    assert abs(A.nnz / interior - 0.6) < 0.01


def test_batch_layout_and_sizes():
    B = I.batch_banded(64, seed_struct=41, seed_val=42)
    assert B.count == 64
    assert B.m.min() >= 64 and B.m.max() < 16384
    assert B.band.min() >= 1 and B.band.max() <= 32
    for i in range(B.count):
        A = B.instance(i)
        assert A.row_ptr[0] == 0 and A.row_ptr[-1] == A.nnz == B.nnz[i]
    assert B.row_ptr.size == int((B.m + 1).sum())
    assert B.val.size == int(B.nnz.sum())


def test_poisson_arrivals_rate():
    t = I.poisson_arrivals(100000, 1000.0)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 100000 - 1e-3) < 2e-5


def test_spd_zipf_symmetric_dominant_sorted():
    A = I.spd_zipf(2000, seed_struct=5, seed_val=6)
    rp, ci, v = A.row_ptr.astype(np.int64), A.col_idx.astype(np.int64), A.val
    r = np.repeat(np.arange(A.nrows), A.row_lengths())
    # sorted, distinct columns in every row
    same = r[1:] == r[:-1]
    assert np.all(ci[1:][same] > ci[:-1][same])
    # symmetric: the transposed entry list is the same list
    fwd = sorted(zip(r.tolist(), ci.tolist(), v.tolist()))
    bwd = sorted(zip(ci.tolist(), r.tolist(), v.tolist()))
    assert fwd == bwd
    # strictly diagonally dominant with a positive diagonal (hence SPD)
    diag = r == ci
    assert np.array_equal(r[diag], np.arange(A.nrows))
    off_abs = np.bincount(r[~diag], weights=np.abs(v[~diag]), minlength=A.nrows)
    assert np.all(v[diag] > off_abs)
    # the zipf hub row survives symmetrization
    assert A.row_lengths().max() >= 2000
    B = I.spd_zipf(2000, seed_struct=5, seed_val=6)
    assert np.array_equal(A.val, B.val) and np.array_equal(A.col_idx, B.col_idx)


def test_block_diagonal_equals_per_instance():
    """The batch as one block-diagonal matrix (the plain baseline's operand)
    gives, row for row, each instance's own product, bit for bit (same entry
    order per row); structure: square, sorted row_ptr, shifted columns."""
    import oracle as O
    insts = [I.banded(50, 3, 0.6, stream=1), I.banded(7, 2, 0.1, stream=2), I.lap2d(5),
             I.banded(1, 1, 1.0, stream=4), I.zipf(300, seed_struct=5, seed_val=6)]
    B = I.batch_from_instances(insts)
    D = I.block_diagonal(B)
    assert D.nrows == D.ncols == int(B.m.sum()) and D.nnz == int(B.nnz.sum())
    assert np.all(np.diff(D.row_ptr) >= 0) and D.row_ptr[0] == 0 and D.row_ptr[-1] == D.nnz
    x = I.batch_vector(B, seed=3)
    y, _ = O.spmv(D, x)
    for i in range(B.count):
        o, m = int(B.vec_off[i]), int(B.m[i])
        A = B.instance(i)
        assert np.array_equal(y[o:o + m], O.spmv(A, x[o:o + m])[0]), i
        ro = D.row_ptr[o:o + m + 1]
        assert np.array_equal(ro - ro[0], A.row_ptr)
        assert np.all((D.col_idx[ro[0]:ro[-1]] >= o) & (D.col_idx[ro[0]:ro[-1]] < o + m))
