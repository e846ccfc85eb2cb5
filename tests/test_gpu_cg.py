"""GPU parity of the conjugate-gradient solve (spk_cg) against the oracle's
CG, on Laplacians, an irregular SPD matrix (rows up to thousands of entries)
and the degenerate cases, for every compiled wavefront-tile shape.

Tolerance.  Both sides run the same recurrence in FP64 with different
summation orders (products summed per row in LDS vs. in storage order,
tree vs. compensated dots), so they differ by rounding, amplified by the
iteration.  For the matrices and iteration counts below an independent
CPU CG (numpy) stays within 4e-15 of the oracle on r_k.r_k and within 3e-13
on x (relative to max |x|): the bound 1e-10 leaves two to four orders of
headroom and still fails on any wrong step size, sign or index, which change
results at O(1).  Once CG has lost orthogonality (after an isolated
eigenvalue converges) the trajectories of two correct implementations
separate at a rate set by the spectrum -- on the irregular matrix the x
difference grows about tenfold per iteration after the sixth -- so that
matrix is compared over its first 8 iterations only."""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def _vecs(A, seed, x0_scale=0.1):
    n = A.nrows
    return I.uniform(seed, 0, n), I.uniform(seed, 1, n) * x0_scale


def _run(spk, M, b, x0, iters, dev, stream=None):
    bd = torch.from_numpy(b).to(dev)
    xd = torch.from_numpy(x0).to(dev)
    hist = spk.spk_cg(M, bd, xd, iters, stream=stream)
    torch.cuda.synchronize()
    return xd.cpu().numpy(), hist.cpu().numpy()


def _compare(x, hist, xo, ho):
    assert hist.shape == ho.shape
    assert np.all(np.isfinite(hist)) and np.all(np.isfinite(x))
    rel_h = np.abs(hist - ho) / np.maximum(ho, np.finfo(float).tiny)
    k = int(np.argmax(rel_h))
    assert rel_h[k] <= RTOL, f"r.r at iteration {k}: {hist[k]!r} vs oracle {ho[k]!r}"
    scale = max(np.abs(xo).max(), np.finfo(float).tiny)
    i = int(np.argmax(np.abs(x - xo)))
    assert abs(x[i] - xo[i]) <= RTOL * scale, f"x[{i}] = {x[i]!r} vs oracle {xo[i]!r}"


CASES = {
    "lap2d_33": (lambda: I.lap2d(33), 60),      # 1089 rows: ragged tail of the vector kernels
    "lap3d_20": (lambda: I.lap3d(20), 40),
    "spd_zipf_3000": (lambda: I.spd_zipf(3000), 8),   # one row of 3000 entries
    "lap2d_1": (lambda: I.lap2d(1), 3),         # 1x1
}


@pytest.mark.parametrize("name", list(CASES))
def test_cg_matches_oracle(spk, dev, name):
    make, iters = CASES[name]
    A = make()
    b, x0 = _vecs(A, 7)
    say("cg", name, "n", A.nrows, "nnz", A.nnz, "iters", iters)
    M = spk.Matrix(A)
    x, hist = _run(spk, M, b, x0, iters, dev)
    xo, ho = O.cg(A, b, iters, x0)
    _compare(x, hist, xo, ho)
    M.release()


def test_cg_every_tile_shape(spk, dev):
    """Each compiled (threads, entries per wavefront) shape, selected by the
    CG plan recorded for the matrix's class."""
    A = I.spd_zipf(2500, seed_struct=36, seed_val=37)
    b, x0 = _vecs(A, 8)
    xo, ho = O.cg(A, b, 8, x0)
    H = spk.Handle()
    try:
        M = spk.Matrix(A, handle=H)
        key = "cg:" + spk.spk_class_key(spk.problem(spk.SPK_OP_SPMV, A=M), handle=H)
        shapes = [(bs, e, 0) for bs in (128, 256, 512) for e in (256, 512, 1024)]
        shapes += [(bs, e, 2) for bs in (256, 512) for e in (256, 512, 1024)]   # two-byte columns
        got = {}
        for bs, e, vec in shapes:
            say("cg tile shape", bs, e, vec)
            v = spk.make_variant(format=spk.SPK_FMT_ADAPTIVE, block=bs, group=1, unroll=1, lds=e, streams=1,
                                 vec=vec)
            spk.spk_plan_put(key, v, handle=H)
            x, hist = _run(spk, M, b, x0, 8, dev)
            _compare(x, hist, xo, ho)
            got[(bs, e, vec)] = (x, hist)
            if vec == 2:   # the same arithmetic as the shape's four-byte kernel: the same bits
                assert np.array_equal(x, got[(bs, e, 0)][0]) and np.array_equal(hist, got[(bs, e, 0)][1])
        M.release()
    finally:
        H.close()


def test_cg_tune_records_a_validated_shape(spk, dev):
    """spk_cg_tune times every shape that reproduces the default shape's
    solve and files the winner under the CG class key; the tuned solve
    still matches the oracle."""
    A = I.lap3d(24)
    b, x0 = _vecs(A, 13)
    H = spk.Handle()
    try:
        M = spk.Matrix(A, handle=H)
        bd = torch.from_numpy(b).to(dev)
        say("cg tune lap3d 24")
        rep = spk.spk_cg_tune(M, bd, 10, reps=3, warmup=1)
        # nine tile shapes, six more with two-byte columns, and ten
        # matrix-free stencil kernels (four of them staging p through LDS)
        assert rep.tried == 25 and rep.rejected == 0
        assert rep.best.format in (spk.SPK_FMT_ADAPTIVE, spk.SPK_FMT_STENCIL)
        assert rep.best_us > 0 and rep.plain_us > 0
        tiles = spk.spk_cg_tune(M, bd, 10, reps=2, warmup=1, record=False, formats=1 << spk.SPK_FMT_ADAPTIVE)
        assert tiles.tried == 15 and tiles.best.format == spk.SPK_FMT_ADAPTIVE
        key = "cg:" + spk.spk_class_key(spk.problem(spk.SPK_OP_SPMV, A=M), handle=H)
        assert rep.class_key.decode() == key
        got = spk.spk_plan_get(key, handle=H)
        assert got is not None and (got.block, got.lds) == (rep.best.block, rep.best.lds)
        xd = torch.from_numpy(x0).to(dev)
        hist = spk.spk_cg(M, bd, xd, 30)
        torch.cuda.synchronize()
        xo, ho = O.cg(A, b, 30, x0)
        _compare(xd.cpu().numpy(), hist.cpu().numpy(), xo, ho)
        M.release()
    finally:
        H.close()


@pytest.mark.parametrize("name", ["lap3d_20", "lap2d_33"])
def test_cg_matrix_free_stencil(spk, dev, name):
    """The matrix-free SpMV+dot (a CG plan naming SPK_FMT_STENCIL) against
    the oracle, both block sizes, and on a matrix that is not a stencil the
    plan is ignored."""
    A = I.lap3d(20) if name == "lap3d_20" else I.lap2d(33)
    iters = 40
    b, x0 = _vecs(A, 14)
    xo, ho = O.cg(A, b, iters, x0)
    H = spk.Handle()
    try:
        M = spk.Matrix(A, handle=H)
        key = "cg:" + spk.spk_class_key(spk.problem(spk.SPK_OP_SPMV, A=M), handle=H)
        shapes = [(bs, r, 0) for bs in (256, 512) for r in (1, 2, 4)] + [(bs, r, 1) for bs in (256, 512)
                                                                         for r in (2, 4)]
        for bs, rows, lds in shapes:
            say("cg stencil", name, bs, rows, lds)
            spk.spk_plan_put(key, spk.make_variant(format=spk.SPK_FMT_STENCIL, block=bs, group=1, unroll=rows,
                                                   streams=1, lds=lds), handle=H)
            bd = torch.from_numpy(b).to(dev)
            xd = torch.from_numpy(x0).to(dev)
            hist = spk.spk_cg(M, bd, xd, iters)
            torch.cuda.synchronize()
            _compare(xd.cpu().numpy(), hist.cpu().numpy(), xo, ho)
        M.release()
        Z = I.spd_zipf(500, seed_struct=38, seed_val=39)
        Mz = spk.Matrix(Z, handle=H)
        kz = "cg:" + spk.spk_class_key(spk.problem(spk.SPK_OP_SPMV, A=Mz), handle=H)
        spk.spk_plan_put(kz, spk.make_variant(format=spk.SPK_FMT_STENCIL, block=256, group=1, unroll=1, streams=1),
                         handle=H)
        bz, xz = _vecs(Z, 15)
        xd = torch.from_numpy(xz).to(dev)
        hist = spk.spk_cg(Mz, torch.from_numpy(bz).to(dev), xd, 6)
        torch.cuda.synchronize()
        xo, ho = O.cg(Z, bz, 6, xz)
        _compare(xd.cpu().numpy(), hist.cpu().numpy(), xo, ho)
        Mz.release()
    finally:
        H.close()


def test_cg_zero_rhs_stays_zero(spk, dev):
    """b = 0, x0 = 0: r = 0, both step sizes are taken as zero, x stays 0."""
    A = I.lap2d(20)
    say("cg zero rhs")
    M = spk.Matrix(A)
    z = np.zeros(A.nrows)
    x, hist = _run(spk, M, z, z, 5, dev)
    assert np.all(hist == 0.0) and np.all(x == 0.0)
    xo, ho = O.cg(A, z, 5, z)
    assert np.all(ho == 0.0) and np.all(xo == 0.0)
    M.release()


def test_cg_zero_iterations(spk, dev):
    A = I.lap2d(17)
    b, x0 = _vecs(A, 9)
    say("cg iters=0")
    M = spk.Matrix(A)
    x, hist = _run(spk, M, b, x0, 0, dev)
    assert hist.shape == (1,)
    assert np.array_equal(x, x0)
    _, ho = O.cg(A, b, 0, x0)
    assert abs(hist[0] - ho[0]) <= RTOL * ho[0]
    M.release()


def test_cg_empty_matrix(spk, dev):
    A = I.CSR(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    say("cg empty")
    M = spk.Matrix(A)
    hist = torch.full((4,), 7.0, dtype=torch.float64, device=dev)
    e = torch.empty(0, dtype=torch.float64, device=dev)
    spk.spk_cg(M, e, e, 3, hist=hist)
    torch.cuda.synchronize()
    assert torch.all(hist == 0).item()
    M.release()


def test_cg_unaligned_x_and_determinism(spk, dev):
    """x at an 8-byte (not 16-byte) offset is iterated in an aligned copy:
    same bits as the aligned run, neighbours untouched; repeated solves are
    bit-identical."""
    A = I.lap3d(12)
    b, x0 = _vecs(A, 10)
    say("cg unaligned x")
    M = spk.Matrix(A)
    xa, ha = _run(spk, M, b, x0, 25, dev)
    xb, hb = _run(spk, M, b, x0, 25, dev)
    assert np.array_equal(xa, xb) and np.array_equal(ha, hb)
    buf = torch.full((A.nrows + 2,), -5.0, dtype=torch.float64, device=dev)
    buf[1:-1] = torch.from_numpy(x0).to(dev)
    xv = buf[1:-1]
    assert xv.data_ptr() % 16 == 8
    hist = spk.spk_cg(M, torch.from_numpy(b).to(dev), xv, 25)
    torch.cuda.synchronize()
    assert np.array_equal(xv.cpu().numpy(), xa) and np.array_equal(hist.cpu().numpy(), ha)
    assert buf[0].item() == -5.0 and buf[-1].item() == -5.0
    M.release()


def test_cg_streams_and_repeat_on_new_sizes(spk, dev):
    """Scratch grows per stream: a larger system after a smaller one, on a
    side stream, then the small one again."""
    s = torch.cuda.Stream()
    for A, it in ((I.lap2d(9), 8), (I.lap3d(16), 8), (I.lap2d(9), 8)):
        b, x0 = _vecs(A, 11)
        say("cg side stream n", A.nrows)
        M = spk.Matrix(A)
        with torch.cuda.stream(s):
            x, hist = _run(spk, M, b, x0, it, dev, stream=s)
        xo, ho = O.cg(A, b, it, x0)
        _compare(x, hist, xo, ho)
        M.release()


def test_cg_errors(spk, dev):
    say("cg error paths")
    A = I.lap2d(8)
    M = spk.Matrix(A)
    b = torch.ones(A.nrows, dtype=torch.float64, device=dev)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=dev)
    with pytest.raises(spk.SpkError, match="SPK_ERR_SHAPE"):
        spk.spk_cg(M, b, x, -1, hist=torch.empty(1, dtype=torch.float64, device=dev))
    with pytest.raises(spk.SpkError, match="SPK_ERR_ALIAS"):
        spk.spk_cg(M, b, b, 2)
    h = torch.empty(A.nrows + 8, dtype=torch.float64, device=dev)
    with pytest.raises(spk.SpkError, match="SPK_ERR_ALIAS"):
        spk.spk_cg(M, b, h[:A.nrows], 2, hist=h[4:7])
    M32 = spk.Matrix(A.astype(np.float32))
    with pytest.raises(spk.SpkError, match="SPK_ERR_DTYPE"):
        spk.spk_cg(M32, b.float(), x.float(), 2)
    R = spk.Matrix(I.zipf(40, 50, seed_struct=3, seed_val=4))
    with pytest.raises(spk.SpkError, match="SPK_ERR_SHAPE"):
        spk.spk_cg(R, torch.ones(40, dtype=torch.float64, device=dev), torch.zeros(50, dtype=torch.float64,
                                                                                  device=dev), 2)
    for m in (M, M32, R):
        m.release()


def test_cg_full_size_lap3d_128(spk, dev):
    """The benchmark system: 7-point Laplacian on 128^3 (2,097,152 rows),
    50 iterations, against the oracle at full size: with the default tile
    shape, then as the bench runs it -- the CSR tile shape tuned by
    spk_cg_tune, and the matrix-free stencil form tuned the same way."""
    A = I.lap3d(128)
    b, x0 = _vecs(A, 12)
    say("cg lap3d 128, 50 iterations")
    h = spk.Handle(0)
    M = spk.Matrix(A, handle=h)
    try:
        xo, ho = O.cg(A, b, 50, x0)
        x, hist = _run(spk, M, b, x0, 50, dev)
        _compare(x, hist, xo, ho)
        bd = torch.from_numpy(b).to(dev)
        for fmt in (spk.SPK_FMT_ADAPTIVE, spk.SPK_FMT_STENCIL):
            rep = spk.spk_cg_tune(M, bd, 10, reps=5, warmup=1, formats=1 << fmt)
            say(f"cg lap3d 128 tuned: {rep.best}")
            assert rep.best.format == fmt and rep.rejected == 0
            x, hist = _run(spk, M, b, x0, 50, dev)
            _compare(x, hist, xo, ho)
    finally:
        M.release()
        h.close()


def test_cg_irregular_spd_long_run(spk, dev):
    """Past the first iterations two correct CGs on the irregular SPD matrix
    part ways in their iterates (rounding amplified once orthogonality is
    lost), so that matrix is compared with the oracle over 8 iterations
    above; over a long run both must still reach the solution. After 250
    iterations the GPU's x equals a direct sparse solve (an independent
    method) and the oracle's x within 1e-12 of max|x|, its true residual
    b - Ax is at rounding level, and its recurrence r.r fell by 1e-30 (the
    oracle reaches these levels by 200 iterations on the same inputs)."""
    import scipy.sparse as sps
    import scipy.sparse.linalg as spla
    A = I.spd_zipf(3000)
    b, x0 = _vecs(A, 7)
    iters = 250
    say("cg long run spd_zipf_3000", iters)
    M = spk.Matrix(A)
    try:
        x, hist = _run(spk, M, b, x0, iters, dev)
    finally:
        M.release()
    xo, ho = O.cg(A, b, iters, x0)
    S = sps.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.nrows, A.ncols))
    xd = spla.spsolve(S.tocsc(), b)
    scale = np.abs(xd).max()
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(hist))
    assert np.abs(x - xd).max() <= 1e-12 * scale
    assert np.abs(x - xo).max() <= 1e-12 * scale
    assert np.linalg.norm(b - S @ x) <= 1e-12 * np.linalg.norm(b)
    assert hist[-1] <= 1e-30 * hist[0] and ho[-1] <= 1e-30 * ho[0]
