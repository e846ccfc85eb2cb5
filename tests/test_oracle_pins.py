"""Pins of the oracle to facts outside itself (CPU only).

The abstract prints no worked example, so every pin is a closed form, exact
rational arithmetic, an invariant, or a special case with a textbook answer:

* SpMV vs exact rational row sums on tiny matrices covering every structural
  edge case (empty rows, duplicates, unsorted, rectangular, explicit zeros);
* identity and diagonal matrices;
* 2-D and 3-D Laplacians applied to integer polynomials, where the centred
  second difference is exact (closed form: -Laplacian(p) plus the
  out-of-grid neighbour values), including a hand-checkable golden fixture;
* WAXPY/AXPY vs the correctly rounded exact result;
* dot vs exact rational sums and integer closed forms;
* metamorphic relations (scaling, row permutation, dot as a 1-row SpMV);
* the ulp metric and the per-row acceptance test;
* mutation checks: a dropped term, a transposed operand or a flipped sign,
  planted on the CPU side, fail these pins.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_1309_1894_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64 = 2.0 ** -53


def csr_from_entries(m, n, entries, dtype=np.float64):
    """CSR in the given storage order; entries = list of (row, col, val)."""
    entries = sorted(entries, key=lambda e: e[0])  # stable: keeps in-row order
    rp = np.zeros(m + 1, np.int32)
    for r, _, _ in entries:
        rp[r + 1] += 1
    rp = np.cumsum(rp).astype(np.int32)
    ci = np.array([c for _, c, _ in entries], np.int32)
    val = np.array([v for _, _, v in entries], dtype)
    return I.CSR(m, n, rp, ci, val)


def exact_rows(A, x):
    """Exact rational y_i = sum_k a_k x[col_k]."""
    out = []
    for i in range(A.nrows):
        s = Fraction(0)
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            s += Fraction(float(A.val[k])) * Fraction(float(x[A.col_idx[k]]))
        out.append(s)
    return out


def assert_rows_close_to_exact(A, x, y, unit=U64):
    ex = exact_rows(A, x)
    lens = np.diff(A.row_ptr)
    for i in range(A.nrows):
        mag = sum(abs(float(A.val[k]) * float(x[A.col_idx[k]])) for k in range(A.row_ptr[i], A.row_ptr[i + 1]))
        bound = (lens[i] + 1) * unit * mag
        assert abs(Fraction(float(y[i])) - ex[i]) <= Fraction(bound), (i, y[i], float(ex[i]))
        if lens[i] == 0:
            assert y[i] == 0.0


def tiny_cases():
    rng = np.random.default_rng(5)
    cases = {}
    cases["1x1"] = csr_from_entries(1, 1, [(0, 0, 2.5)])
    cases["empty_rows"] = csr_from_entries(4, 3, [(1, 0, 1.25), (1, 2, -3.0), (3, 1, 0.5)])
    cases["all_empty"] = csr_from_entries(5, 5, [])
    cases["n0"] = csr_from_entries(3, 0, [])
    cases["m0"] = csr_from_entries(0, 4, [])
    cases["dense_row"] = csr_from_entries(2, 64, [(0, c, float(rng.uniform(-1, 1))) for c in range(64)])
    cases["rect_wide"] = csr_from_entries(3, 40, [(r, int(c), float(rng.uniform(-1, 1)))
                                                  for r in range(3) for c in rng.choice(40, 9, replace=False)])
    cases["rect_tall"] = csr_from_entries(40, 3, [(r, int(r % 3), float(rng.uniform(-1, 1))) for r in range(40)])
    cases["duplicates"] = csr_from_entries(3, 4, [(0, 1, 0.5), (0, 1, 0.25), (0, 1, -2.0), (2, 3, 1.5), (2, 3, 1.5)])
    cases["unsorted"] = csr_from_entries(2, 6, [(0, 5, 1.0), (0, 0, -0.75), (0, 3, 0.1), (1, 4, 3.0), (1, 1, -0.3)])
    cases["explicit_zeros"] = csr_from_entries(3, 3, [(0, 0, 0.0), (1, 1, 0.0), (1, 2, 2.0), (2, 0, 0.0)])
    ents = []
    for r in range(64):
        for c in rng.choice(64, int(rng.integers(0, 20)), replace=False):
            ents.append((r, int(c), float(rng.uniform(-1, 1))))
    cases["random64"] = csr_from_entries(64, 64, ents)
    return cases


@pytest.mark.parametrize("name", list(tiny_cases().keys()))
def test_spmv_matches_exact_rational(name):
    A = tiny_cases()[name]
    x = I.uniform(7, 0, A.ncols)
    y, absum = O.spmv(A, x)
    assert y.shape == (A.nrows,)
    assert_rows_close_to_exact(A, x, y)
    # absum is the scale sum |a x| (each term rounded once, summed in order)
    for i in range(A.nrows):
        mag = sum(abs(float(A.val[k]) * float(x[A.col_idx[k]])) for k in range(A.row_ptr[i], A.row_ptr[i + 1]))
        assert absum[i] == pytest.approx(mag, rel=1e-14, abs=0)


@pytest.mark.parametrize("name", ["random64", "duplicates", "unsorted", "rect_wide", "dense_row"])
def test_spmv_f32_promotes_exactly(name):
    A = tiny_cases()[name].astype(np.float32)
    x = I.uniform(8, 0, A.ncols, np.float32)
    y, _ = O.spmv(A, x)
    assert y.dtype == np.float64
    assert_rows_close_to_exact(A, x, y)  # double accumulation: double-precision bound


def test_spmv_integer_values_bit_exact():
    rng = np.random.default_rng(3)
    ents = [(r, int(c), float(rng.integers(-9, 10))) for r in range(50) for c in rng.choice(70, 12, replace=False)]
    A = csr_from_entries(50, 70, ents)
    x = rng.integers(-100, 100, 70).astype(np.float64)
    y, _ = O.spmv(A, x)
    ex = exact_rows(A, x)
    assert all(Fraction(float(y[i])) == ex[i] for i in range(50))


def test_spmv_nan_inf_propagation():
    A = csr_from_entries(4, 3, [(0, 0, 1.0), (0, 1, 2.0), (1, 1, 0.0), (2, 2, 1.0), (3, 0, 1.0)])
    x = np.array([np.inf, np.nan, -np.inf])
    y, _ = O.spmv(A, x)
    assert np.isnan(y[0])          # inf + 2*nan
    assert np.isnan(y[1])          # 0 * nan
    assert y[2] == -np.inf
    assert y[3] == np.inf


def test_identity_and_diagonal():
    n = 1000
    x = I.uniform(1, 0, n)
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    Aid = I.CSR(n, n, rp, ci, np.ones(n))
    y, _ = O.spmv(Aid, x)
    assert np.array_equal(y, x)
    d = I.uniform(2, 0, n)
    Ad = I.CSR(n, n, rp, ci, d)
    y, _ = O.spmv(Ad, x)
    assert np.array_equal(y, d * x)   # a single rounded product


def _grid_closed_form_2d(N, p, lap):
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    i = i.astype(np.float64).ravel()
    j = j.astype(np.float64).ravel()
    y = -lap(i, j)
    for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        a, b = i + di, j + dj
        out = (a < 0) | (a >= N) | (b < 0) | (b >= N)
        y = y + np.where(out, p(a, b), 0.0)
    return p(i, j), y


POLYS_2D = [
    (lambda i, j: np.ones_like(i), lambda i, j: np.zeros_like(i)),
    (lambda i, j: i * i + j * j, lambda i, j: np.full_like(i, 4.0)),
    (lambda i, j: i ** 3 - 2 * i * j * j + 7, lambda i, j: 6 * i - 4 * i),
    (lambda i, j: 3 * j ** 3 + i * j - 5 * i, lambda i, j: 18 * j),
]


@pytest.mark.parametrize("N", [1, 2, 3, 17, 256])
@pytest.mark.parametrize("k", range(len(POLYS_2D)))
def test_lap2d_polynomial_closed_form(N, k):
    p, lap = POLYS_2D[k]
    A = I.lap2d(N)
    x, expected = _grid_closed_form_2d(N, p, lap)
    y, _ = O.spmv(A, x)
    assert np.array_equal(y, expected)


def test_lap2d_golden_fixture():
    rows = np.loadtxt(os.path.join(GOLDEN, "lap2d_N4_quadratic.txt"), comments="#")
    A = I.lap2d(4)
    x = np.zeros(16)
    for i, j, xv, _ in rows:
        x[int(i) * 4 + int(j)] = xv
    y, _ = O.spmv(A, x)
    for i, j, _, yv in rows:
        assert y[int(i) * 4 + int(j)] == yv


def _grid_closed_form_3d(N, p, lap):
    i, j, k = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    i, j, k = (v.astype(np.float64).ravel() for v in (i, j, k))
    y = -lap(i, j, k)
    for d in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
        a, b, c = i + d[0], j + d[1], k + d[2]
        out = (a < 0) | (a >= N) | (b < 0) | (b >= N) | (c < 0) | (c >= N)
        y = y + np.where(out, p(a, b, c), 0.0)
    return p(i, j, k), y


POLYS_3D = [
    (lambda i, j, k: np.ones_like(i), lambda i, j, k: np.zeros_like(i)),
    (lambda i, j, k: i * i + 2 * j * j - k * k, lambda i, j, k: np.full_like(i, 2.0 + 4.0 - 2.0)),
    (lambda i, j, k: k ** 3 + i * j * k - j ** 3, lambda i, j, k: 6 * k - 6 * j),
]


@pytest.mark.parametrize("N", [1, 2, 5, 32, 128])
@pytest.mark.parametrize("q", range(len(POLYS_3D)))
def test_lap3d_polynomial_closed_form(N, q):
    p, lap = POLYS_3D[q]
    A = I.lap3d(N)
    x, expected = _grid_closed_form_3d(N, p, lap)
    y, _ = O.spmv(A, x)
    assert np.array_equal(y, expected)


def test_lap_ones_counts_missing_neighbours():
    A = I.lap2d(9)
    y, _ = O.spmv(A, np.ones(81))
    g = y.reshape(9, 9)
    assert g[0, 0] == 2 and g[0, 4] == 1 and g[4, 4] == 0 and g[8, 8] == 2


def _round_exact(fr):
    return float(fr)  # CPython rounds a Fraction to the nearest double


@pytest.mark.parametrize("alpha", [1.5, 0.5, -0.3333333333333333, 1e-300, 7.25e10])
def test_waxpy_correctly_rounded(alpha):
    n = 3000
    x = I.uniform(21, 0, n)
    y = I.uniform(22, 0, n)
    w = O.waxpy(alpha, x, y)
    a = Fraction(alpha)
    for i in range(n):
        assert w[i] == _round_exact(a * Fraction(float(x[i])) + Fraction(float(y[i]))), i


def test_waxpy_f32_rounds_from_exact():
    n = 3000
    x = I.uniform(21, 0, n, np.float32)
    y = I.uniform(22, 0, n, np.float32)
    alpha = 1.5
    w = O.waxpy(alpha, x, y)
    assert w.dtype == np.float32
    for i in range(n):
        ex = Fraction(alpha) * Fraction(float(x[i])) + Fraction(float(y[i]))
        # the exact value rounded to double (exactly what fma gives), then to float
        assert w[i] == np.float32(_round_exact(ex)), i
        # and within one float ulp of the exact value
        assert abs(Fraction(float(w[i])) - ex) <= Fraction(float(np.spacing(np.float32(abs(float(ex))))))


def test_waxpy_alpha_not_special_cased():
    x = np.array([np.inf, 1.0, np.nan])
    y = np.array([1.0, 2.0, 3.0])
    w = O.waxpy(0.0, x, y)
    assert np.isnan(w[0]) and w[1] == 2.0 and np.isnan(w[2])


def test_axpy_is_waxpy_in_place():
    x = I.uniform(3, 0, 5000)
    y = I.uniform(4, 0, 5000)
    assert np.array_equal(O.axpy(1.5, x, y), O.waxpy(1.5, x, y))
    assert np.array_equal(O.axpy(1.5, x.astype(np.float32), y.astype(np.float32)),
                          O.waxpy(1.5, x.astype(np.float32), y.astype(np.float32)))


def test_waxpy_small_integers_exact():
    x = np.arange(-500, 500, dtype=np.float64)
    y = np.arange(1000, dtype=np.float64) * 3
    assert np.array_equal(O.waxpy(2.0, x, y), 2 * x + y)


@pytest.mark.parametrize("n", [0, 1, 7, 4095, 4096, 4097, 10000])
def test_dot_vs_exact_rational(n):
    x = I.uniform(21, 0, n)
    y = I.uniform(22, 0, n)
    d = O.dot(x, y)
    ex = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
    mag = float(np.sum(np.abs(x * y)))
    assert abs(Fraction(d) - ex) <= Fraction(3 * U64 * mag + 1e-300)


def test_dot_f32_vs_exact():
    n = 9000
    x = I.uniform(21, 0, n, np.float32)
    y = I.uniform(22, 0, n, np.float32)
    ex = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
    d = O.dot(x, y)
    assert abs(Fraction(d) - ex) <= Fraction(2 * U64 * float(np.sum(np.abs(x.astype(np.float64) * y))))


@pytest.mark.parametrize("n", [1, 1000, 1 << 20, (1 << 24) + 3])
def test_dot_integer_closed_forms(n):
    ones = np.ones(n)
    idx = np.arange(n, dtype=np.float64)
    assert O.dot(ones, ones) == n
    assert O.dot(idx, ones) == n * (n - 1) // 2
    if n <= (1 << 17):  # every partial sum of squares stays below 2**53
        assert O.dot(idx, idx) == float((n - 1) * n * (2 * n - 1) // 6)


def test_dot_thread_count_independent():
    x = I.uniform(21, 0, 300001)
    y = I.uniform(22, 0, 300001)
    t0 = O.num_threads()
    try:
        O.set_threads(1)
        a = O.dot(x, y)
        O.set_threads(max(2, t0))
        b = O.dot(x, y)
    finally:
        O.set_threads(t0)
    assert a == b


def test_metamorphic_scaling_and_permutation():
    A = I.zipf(3000, seed_struct=5, seed_val=6)
    x = I.uniform(9, 0, 3000)
    y, _ = O.spmv(A, x)
    y2, _ = O.spmv(A, 2.0 * x)
    assert np.array_equal(y2, 2.0 * y)
    perm = np.argsort(I.u64(1, 2, 0, 3000))
    lens = A.row_lengths()
    rp = np.zeros(3001, np.int64)
    rp[1:] = np.cumsum(lens[perm])
    ci = np.concatenate([A.col_idx[A.row_ptr[r]:A.row_ptr[r + 1]] for r in perm])
    va = np.concatenate([A.val[A.row_ptr[r]:A.row_ptr[r + 1]] for r in perm])
    P = I.CSR(3000, 3000, rp.astype(np.int32), ci, va)
    yp, _ = O.spmv(P, x)
    assert np.array_equal(yp, y[perm])
    assert np.array_equal(O.waxpy(1.5, 2 * x, 2 * y), 2 * O.waxpy(1.5, x, y))


def test_dot_equals_one_row_spmv():
    n = 5000
    x = I.uniform(1, 0, n)
    v = I.uniform(2, 0, n)
    A = I.CSR(1, n, np.array([0, n], np.int32), np.arange(n, dtype=np.int32), v)
    y, absum = O.spmv(A, x)
    assert abs(y[0] - O.dot(v, x)) <= 1e-13 * absum[0]


def test_spmv_waxpy_step_definition():
    A = I.lap2d(64)
    x = I.uniform(11, 0, A.nrows)
    y, w, absum = O.spmv_waxpy(A, x, 0.5)
    y1, a1 = O.spmv(A, x)
    assert np.array_equal(y, y1) and np.array_equal(absum, a1)
    assert np.array_equal(w, O.waxpy(0.5, y1, x))
    # alpha = 0.5 is exact, so w is the correctly rounded y/2 + x
    for i in range(0, A.nrows, 97):
        assert w[i] == _round_exact(Fraction(float(y[i])) / 2 + Fraction(float(x[i])))


def test_batch_oracle_is_per_instance():
    B = I.batch_banded(12, seed_struct=3, seed_val=4)
    x = I.batch_vector(B, seed=5)
    y, w, absum = O.batch_spmv_waxpy(B, x, 0.5)
    for b in range(B.count):
        A = B.instance(b)
        o = int(B.vec_off[b])
        yi, wi, ai = O.spmv_waxpy(A, x[o:o + A.nrows], 0.5)
        assert np.array_equal(y[o:o + A.nrows], yi)
        assert np.array_equal(w[o:o + A.nrows], wi)


def test_ulp_metric():
    a = np.array([1.0, 0.0, -0.0, 1.0, np.nan, np.nan, -1.0])
    b = np.array([np.nextafter(1.0, 2.0), -0.0, 5e-324, 1.0, np.nan, 1.0, np.nextafter(np.nextafter(-1.0, 0), 0)])
    assert O.max_ulp(a[:1], b[:1])[0] == 1
    assert O.max_ulp(a[1:2], b[1:2])[0] == 0      # +0 == -0
    assert O.max_ulp(a[2:3], b[2:3])[0] == 1      # -0 to the smallest subnormal
    assert O.max_ulp(a[3:5], b[3:5])[0] == 0      # equal, and NaN == NaN
    assert O.max_ulp(a[5:6], b[5:6])[0] == 2 ** 63 - 1
    assert O.max_ulp(a[6:7], b[6:7])[0] == 2
    f = np.array([1.0, -2.0], np.float32)
    g = np.array([np.nextafter(np.float32(1.0), np.float32(2.0)), np.float32(-2.0)], np.float32)
    assert O.max_ulp(f, g) == (1, 0)
    # across zero: -tiny to +tiny is two steps
    t = np.array([-5e-324]), np.array([5e-324])
    assert O.max_ulp(*t)[0] == 2


def test_check_rows_semantics():
    ref = np.array([1.0, 0.0, np.nan, np.inf, 2.0])
    absum = np.array([1.0, 0.0, 1.0, 1.0, 4.0])
    ok = np.array([1.0 + 5e-13, 0.0, np.nan, np.inf, 2.0])
    assert O.check_rows(ok, ref, absum, 1e-12)[0] == 0
    bad = ok.copy(); bad[0] = 1.0 + 2e-12
    assert O.check_rows(bad, ref, absum, 1e-12)[:1] == (1,)
    bad = ok.copy(); bad[1] = 1e-300        # empty row must be exactly zero
    assert O.check_rows(bad, ref, absum, 1e-12)[0] == 1
    bad = ok.copy(); bad[2] = 0.0
    assert O.check_rows(bad, ref, absum, 1e-12)[0] == 1
    bad = ok.copy(); bad[3] = -np.inf
    assert O.check_rows(bad, ref, absum, 1e-12)[0] == 1
    bad = ok.copy(); bad[4] = np.nan
    assert O.check_rows(bad, ref, absum, 1e-12)[0] == 1


# --- mutation checks: plausible mistakes, planted on the CPU, fail the pins ---

def test_dropped_term_fails_closed_form():
    A = I.lap2d(17)
    p, lap = POLYS_2D[1]
    x, expected = _grid_closed_form_2d(17, p, lap)
    rp = A.row_ptr.copy()
    rp[1:] = rp[1:] - 1                      # every row loses its last entry
    rp[0] = 0
    rp[1:] = np.maximum(rp[1:], 0)
    broken = I.CSR(A.nrows, A.ncols, rp, A.col_idx, A.val)
    y, _ = O.spmv(broken, x)
    assert not np.array_equal(y, expected)


def test_transposed_operand_fails_brute_force():
    A = tiny_cases()["random64"]
    x = I.uniform(7, 0, 64)
    dense = np.zeros((64, 64))
    for i in range(64):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            dense[i, A.col_idx[k]] += A.val[k]
    T = dense.T
    rows, cols = np.nonzero(T)
    At = I.CSR(64, 64, np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=64))]).astype(np.int32),
               cols.astype(np.int32), T[rows, cols].copy())
    y, _ = O.spmv(At, x)
    with pytest.raises(AssertionError):
        assert_rows_close_to_exact(A, x, y)


def test_wrong_sign_fails_exact_waxpy():
    x = I.uniform(21, 0, 100)
    y = I.uniform(22, 0, 100)
    w = O.waxpy(-1.5, x, y)
    ex = [_round_exact(Fraction(1.5) * Fraction(float(a)) + Fraction(float(b))) for a, b in zip(x, y)]
    assert not np.array_equal(w, np.array(ex))


# --- the Krylov iteration (CG) built on the kernels -------------------------

def test_cg_terminates_on_k_distinct_eigenvalues():
    """In exact arithmetic CG on a matrix with k distinct eigenvalues reaches
    the solution in k iterations (a textbook property); in FP64 the residual
    is then at rounding level."""
    n = 500
    d = np.array([1.0, 2.0, 3.5, 7.0, 11.0])[np.arange(n) % 5]
    A = I.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = I.uniform(3, 0, n)
    x, hist = O.cg(A, b, 5)
    assert np.sqrt(hist[5]) <= 1e-12 * np.sqrt(hist[0])
    assert np.max(np.abs(x - b / d)) <= 1e-12 * np.max(np.abs(b / d))


def test_cg_matches_direct_solve_on_laplacian():
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    A = I.lap2d(24)
    b = I.uniform(4, 0, A.nrows)
    x, hist = O.cg(A, b, 400)
    S = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.nrows, A.ncols))
    xd = spla.spsolve(S.tocsc(), b)
    assert np.max(np.abs(x - xd)) <= 1e-9 * np.max(np.abs(xd))
    # the recurrence residual tracks the true residual
    assert abs(np.sqrt(hist[-1]) - np.linalg.norm(b - S @ x)) <= 1e-9 * np.linalg.norm(b)


def test_cg_first_step_closed_form():
    """One iteration from x0 = 0: x1 = (b.b / b.Ab) b."""
    A = I.lap2d(10)
    b = I.uniform(5, 0, A.nrows)
    x, hist = O.cg(A, b, 1)
    Ab, _ = O.spmv(A, b)
    alpha = Fraction(float(np.dot(b, b))) / Fraction(float(np.dot(b, Ab)))
    assert np.max(np.abs(x - float(alpha) * b)) <= 1e-14 * np.max(np.abs(b))
    assert hist[0] == O.dot(b, b)


def test_cg_exact_solution_stays_put():
    """Starting from the exact solution the residual is zero and the guarded
    step sizes keep the iterate unchanged (no 0/0)."""
    n = 64
    d = np.full(n, 2.0)
    A = I.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    x0 = I.uniform(6, 0, n)
    b = 2.0 * x0
    x, hist = O.cg(A, b, 3, x0=x0)
    assert np.array_equal(x, x0) and np.all(hist == 0.0)


# --- the scale of the dot tolerance: sum_i |x_i*y_i| -------------------------
# Every dot parity test accepts |d - ref| <= tau * dot_absum(x, y), so a scale
# that came out too large would loosen them silently.  The scale is pinned to
# the exact rational magnitude sum; each of the n products is rounded once
# (exact for FP32 operands) and the n - 1 additions once each.

def _absum_exact(x, y):
    return sum((abs(Fraction(float(a)) * Fraction(float(b))) for a, b in zip(x, y)), Fraction(0))


def _absum_pinned(s, x, y, unit):
    """Is s the sum of |x_i y_i| within (n+1)*unit of it?"""
    ex = _absum_exact(x, y)
    return abs(Fraction(s) - ex) <= Fraction(len(x) + 1) * Fraction(unit) * ex


@pytest.mark.parametrize("n", [0, 1, 2, 7, 4096, 10001])
def test_dot_absum_vs_exact_rational(n):
    x = I.uniform(21, 0, n)
    y = I.uniform(22, 0, n)
    s = O.dot_absum(x, y)
    assert s >= 0.0
    assert _absum_pinned(s, x, y, U64)
    if n == 0:
        assert s == 0.0


def test_dot_absum_f32_widens_exactly():
    n = 9000
    x = I.uniform(21, 0, n, np.float32)
    y = I.uniform(22, 0, n, np.float32)
    s = O.dot_absum(x, y)
    # FP32 products are exact in double: only the additions round
    assert _absum_pinned(s, x, y, U64)
    # and the FP32 value itself would not do: the products are formed in double
    xs = x.astype(np.float64) * y.astype(np.float64)
    assert np.any(xs != (x * y).astype(np.float64))


@pytest.mark.parametrize("n", [1, 2, 1000, 4097, (1 << 20) + 1])
def test_dot_absum_integer_closed_forms(n):
    # alternating signs: sum |(-1)^i i * 1| = n(n-1)/2 although the dot itself
    # is -(n//2) or (n-1)/2, so the absolute value must be taken per product
    i = np.arange(n, dtype=np.float64)
    alt = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    assert O.dot_absum(alt * i, np.ones(n)) == n * (n - 1) // 2
    assert O.dot_absum(i, -alt) == n * (n - 1) // 2
    assert O.dot(alt * i, np.ones(n)) == ((n - 1) // 2 if n % 2 else -(n // 2))
    assert O.dot_absum(-np.ones(n), np.ones(n)) == n
    # FP32 operands: exact integers, widened before the product
    f = (alt * np.minimum(i, 4000)).astype(np.float32)
    exact = int(np.sum(np.minimum(np.arange(n), 4000)))
    assert O.dot_absum(f, np.full(n, -3, np.float32)) == 3 * exact


def test_dot_absum_bounds_the_dot_error():
    # the scale must be at least |sum x_i y_i| (triangle inequality) and is
    # what the compensated dot's own error is measured against
    x = I.uniform(31, 0, 50000)
    y = I.uniform(32, 0, 50000)
    s = O.dot_absum(x, y)
    assert s >= abs(O.dot(x, y))
    assert s == pytest.approx(float(np.sum(np.abs(x) * np.abs(y))), rel=1e-13)


def test_dot_absum_mutations_fail_the_pin():
    # plausible wrong scales, planted here on the CPU, fail the same pin
    x = I.uniform(21, 0, 257)
    y = I.uniform(22, 0, 257)
    assert _absum_pinned(O.dot_absum(x, y), x, y, U64)
    wrong_abs_of_sum = abs(O.dot(x, y))                              # |sum x y|
    wrong_product_of_sums = float(np.sum(np.abs(x)) * np.sum(np.abs(y)))  # sum|x| * sum|y|
    wrong_dropped_last = O.dot_absum(x[:-1], y[:-1])                 # one term short
    wrong_signed_x = float(np.sum(np.abs(x) * y))                    # |.| on one operand only
    for bad in (wrong_abs_of_sum, wrong_product_of_sums, wrong_dropped_last, wrong_signed_x):
        assert not _absum_pinned(bad, x, y, U64), bad


# Every function the oracle exports, and the tests above that pin it.
PINNED_BY = {
    "orc_num_threads": ["test_dot_thread_count_independent"],
    "orc_set_num_threads": ["test_dot_thread_count_independent"],
    "orc_waxpy_f64": ["test_waxpy_correctly_rounded", "test_waxpy_alpha_not_special_cased"],
    "orc_waxpy_f32": ["test_waxpy_f32_rounds_from_exact"],
    "orc_axpy_f64": ["test_axpy_is_waxpy_in_place"],
    "orc_axpy_f32": ["test_axpy_is_waxpy_in_place"],
    "orc_dot_f64": ["test_dot_vs_exact_rational", "test_dot_integer_closed_forms"],
    "orc_dot_f32": ["test_dot_f32_vs_exact"],
    "orc_dot_absum_f64": ["test_dot_absum_vs_exact_rational", "test_dot_absum_integer_closed_forms",
                          "test_dot_absum_mutations_fail_the_pin"],
    "orc_dot_absum_f32": ["test_dot_absum_f32_widens_exactly", "test_dot_absum_integer_closed_forms"],
    "orc_spmv_csr_f64": ["test_spmv_matches_exact_rational", "test_lap2d_polynomial_closed_form",
                         "test_lap3d_polynomial_closed_form", "test_identity_and_diagonal"],
    "orc_spmv_csr_f32": ["test_spmv_f32_promotes_exactly"],
    "orc_spmv_waxpy_f64": ["test_spmv_waxpy_step_definition"],
    "orc_batch_spmv_waxpy_f64": ["test_batch_oracle_is_per_instance"],
    "orc_max_ulp_f64": ["test_ulp_metric"],
    "orc_max_ulp_f32": ["test_ulp_metric"],
    "orc_check_rows": ["test_check_rows_semantics"],
    "orc_cg_f64": ["test_cg_terminates_on_k_distinct_eigenvalues", "test_cg_matches_direct_solve_on_laplacian",
                   "test_cg_first_step_closed_form", "test_cg_exact_solution_stays_put"],
}


def test_every_exported_oracle_function_is_pinned():
    import re
    src = open(O.SRC_PATH).read()
    exported = set(re.findall(r"ORC_API\s+[\w\s\*]+?\b(orc_\w+)\s*\(", src))
    assert exported == set(PINNED_BY), exported ^ set(PINNED_BY)
    here = globals()
    for name, tests in PINNED_BY.items():
        for t in tests:
            assert callable(here.get(t)), (name, t)
