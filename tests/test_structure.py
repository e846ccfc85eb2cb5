"""Structure detection behind the DIA and stencil SpMV formats, on the host
(spk_csr_structure needs no GPU): Laplacians in 1-, 2- and 3-D are found as
stencils with their grids and coefficients; anything that breaks exactness
(a changed value, an extra or missing entry, a duplicate) demotes a matrix
to DIA or to plain CSR."""
import numpy as np
import pytest

from paper_1309_1894_amd import inputs as I

SCALAR, VECTOR, SELL, ADAPTIVE, DIA, STENCIL = 1, 2, 3, 4, 5, 6
CSR_ONLY = (1 << SCALAR) | (1 << VECTOR) | (1 << SELL) | (1 << ADAPTIVE)


@pytest.fixture(scope="module")
def spk():
    from paper_1309_1894_amd import spk as _spk
    return _spk


def _csr(m, n, rows, cols, vals, dtype=np.float64):
    order = np.lexsort((cols, rows))
    rows, cols, vals = np.asarray(rows)[order], np.asarray(cols)[order], np.asarray(vals, dtype)[order]
    rp = np.zeros(m + 1, np.int64)
    np.add.at(rp, np.asarray(rows) + 1, 1)
    return I.CSR(m, n, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), vals)


def _entries(A):
    r = np.repeat(np.arange(A.nrows), A.row_lengths())
    return r, A.col_idx.astype(np.int64), A.val.copy()


@pytest.mark.parametrize("N", [2, 5, 33])
def test_lap2d_is_a_2d_stencil(spk, N):
    s = spk.spk_csr_structure(I.lap2d(N))
    assert s["formats"] == CSR_ONLY | (1 << DIA) | (1 << STENCIL)
    assert s["offsets"] == [-N, -1, 0, 1, N]
    assert s["dim"] == 2 and s["grid"] == (1, N, N)
    assert s["coef"] == [0.0, -1.0, -1.0, 4.0, -1.0, -1.0, 0.0]


@pytest.mark.parametrize("N", [2, 3, 12])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_lap3d_is_a_3d_stencil(spk, N, dtype):
    s = spk.spk_csr_structure(I.lap3d(N, dtype))
    assert s["formats"] & (1 << STENCIL)
    assert s["offsets"] == [-N * N, -N, -1, 0, 1, N, N * N]
    assert s["dim"] == 3 and s["grid"] == (N, N, N)
    assert s["coef"] == [-1.0, -1.0, -1.0, 6.0, -1.0, -1.0, -1.0]


def test_tridiagonal_is_a_1d_stencil(spk):
    n = 50
    r = np.concatenate([np.arange(n), np.arange(1, n), np.arange(n - 1)])
    c = np.concatenate([np.arange(n), np.arange(n - 1), np.arange(1, n)])
    v = np.concatenate([np.full(n, 2.5), np.full(n - 1, -1.25), np.full(n - 1, 0.5)])
    s = spk.spk_csr_structure(_csr(n, n, r, c, v))
    assert s["dim"] == 1 and s["grid"] == (1, 1, n)
    assert s["coef"] == [0.0, 0.0, -1.25, 2.5, 0.5, 0.0, 0.0]


def test_one_changed_value_leaves_dia_only(spk):
    A = I.lap2d(9)
    A.val[17] = -1.0000000000000002
    s = spk.spk_csr_structure(A)
    assert s["formats"] == CSR_ONLY | (1 << DIA) and s["dim"] == 0


def test_entry_across_a_grid_row_edge_is_not_a_stencil(spk):
    N = 6
    r, c, v = _entries(I.lap2d(N))
    # row (0, N-1) gets a "+1" neighbour that is really (1, 0): periodic-like wrap
    row = N - 1
    s = spk.spk_csr_structure(_csr(N * N, N * N, np.append(r, row), np.append(c, row + 1), np.append(v, -1.0)))
    assert s["formats"] == CSR_ONLY | (1 << DIA)


def test_missing_neighbour_is_not_a_stencil(spk):
    r, c, v = _entries(I.lap3d(4))
    keep = np.ones(r.size, bool)
    keep[np.nonzero((r == 21) & (c == 22))[0]] = False
    s = spk.spk_csr_structure(_csr(64, 64, r[keep], c[keep], v[keep]))
    assert s["formats"] == CSR_ONLY | (1 << DIA)


def test_duplicates_rule_out_dia(spk):
    r, c, v = _entries(I.lap2d(5))
    s = spk.spk_csr_structure(_csr(25, 25, np.append(r, 7), np.append(c, 7), np.append(v, 0.5)))
    assert s["formats"] == CSR_ONLY


def test_unsorted_rows_are_still_detected(spk):
    A = I.lap2d(7)
    rng = np.random.default_rng(3)
    ci, val = A.col_idx.copy(), A.val.copy()
    for i in range(A.nrows):
        a, b = A.row_ptr[i], A.row_ptr[i + 1]
        p = rng.permutation(b - a) + a
        ci[a:b], val[a:b] = ci[p], val[p]
    s = spk.spk_csr_structure(I.CSR(A.nrows, A.ncols, A.row_ptr, ci, val))
    assert s["dim"] == 2 and s["coef"][3] == 4.0


def test_banded_few_diagonals_is_dia(spk):
    A = I.banded(1000, 5, 1.0, stream=4)
    s = spk.spk_csr_structure(A)
    assert s["formats"] == CSR_ONLY | (1 << DIA)
    assert s["offsets"] == list(range(-5, 6))


def test_too_many_diagonals_or_random_columns_is_csr_only(spk):
    assert spk.spk_csr_structure(I.banded(1000, 10, 1.0, stream=5))["formats"] == CSR_ONLY   # 21 diagonals
    assert spk.spk_csr_structure(I.zipf(1000, seed_struct=6, seed_val=7))["formats"] == CSR_ONLY


def test_rectangular_and_empty(spk):
    m, n = 30, 40
    r = np.concatenate([np.arange(m), np.arange(m)])
    c = np.concatenate([np.arange(m), np.arange(m) + 10])
    s = spk.spk_csr_structure(_csr(m, n, r, c, np.ones(2 * m)))
    assert s["formats"] == CSR_ONLY | (1 << DIA) and s["offsets"] == [0, 10]
    e = I.CSR(5, 5, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert spk.spk_csr_structure(e)["formats"] == CSR_ONLY
