"""GPU parity of the x-window SpMV form (SPK_FMT_XWIN): the entries regrouped
into (row, column-window) pairs, each window of x staged in LDS by the
workgroups that use it, one FP64 partial per pair, then one pass adding a
row's partials in window order.  Every compiled kernel and chunking against
the oracle, FP64 and FP32, plain and fused, on the structural edge cases and
on matrices spanning many windows (empty windows, pairs long enough for the
one-pair-per-wavefront path, a row across every window), canaries after the
outputs, bit-exact single-entry rows, NaN/Inf, two streams at once, and the
tuner's search."""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I
from test_gpu_spmv import CASES, NP, _check, csr_from_entries

pytestmark = pytest.mark.gpu

KERNELS = [(512, 128, 256), (1024, 128, 128), (768, 128, 256), (256, 64, 256), (512, 64, 256)]


def _variants(spk):
    return [spk.make_variant(format=spk.SPK_FMT_XWIN, block=bs, group=kib, lds=e, grid=g, unroll=1, streams=1)
            for bs, kib, e in KERNELS for g in (1, 2)]


def wide_cases():
    rng = np.random.default_rng(5)
    out = {}
    # 300 rows over 70,000 columns: several windows in both precisions
    ents = [(r, int(c), float(rng.uniform(-1, 1))) for r in range(300)
            for c in rng.choice(70000, int(rng.integers(0, 40)), replace=False)]
    out["rand_wide"] = csr_from_entries(300, 70000, ents)
    # only columns of the first and the last window are used
    ents = [(r, int(c), float(rng.uniform(-1, 1))) for r in range(200)
            for c in np.concatenate([rng.choice(1000, 3, replace=False), 69000 + rng.choice(1000, 3, replace=False)])]
    out["gap_windows"] = csr_from_entries(200, 70000, ents)
    # one row over every window (pairs of thousands of entries: one wavefront
    # per pair), among short rows; a row with 200 entries inside one window
    ents = [(0, c, float(rng.uniform(-1, 1))) for c in range(0, 60000, 2)]
    ents += [(r, int(rng.integers(0, 60000)), float(rng.uniform(-1, 1))) for r in range(1, 400)]
    ents += [(7, c, 0.5) for c in range(30000, 30200)]
    out["long_pairs"] = csr_from_entries(400, 60000, ents)
    out["zipf_200k"] = I.zipf(200000, seed_struct=31, seed_val=32)
    return out


WIDE = wide_cases()
ALL = {**CASES, **WIDE}


def _run_all(spk, A, x, dt, variants):
    M = spk.Matrix(A)
    try:
        xd = torch.from_numpy(x).to(dev_of())
        pad = 64
        ybuf = torch.full((A.nrows + pad,), 7.0, dtype=M.torch_dtype, device=dev_of())
        wbuf = torch.full((A.nrows + pad,), 7.0, dtype=M.torch_dtype, device=dev_of())
        y, w = ybuf[:A.nrows], wbuf[:A.nrows]
        for v in variants:
            y.fill_(float("nan"))
            spk.spk_run(spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y), v)
            try:
                _check(A, x, y, dt=dt)
                if A.nrows == A.ncols:
                    y.fill_(float("nan"))
                    w.fill_(float("nan"))
                    spk.spk_run(spk.problem(spk.SPK_OP_SPMV_WAXPY, A=M, x=xd, y=y, w=w, alpha=0.5), v)
                    _check(A, x, y, w, 0.5, dt)
            except AssertionError as e:
                raise AssertionError(f"{v}: {e}")
            assert torch.all(ybuf[A.nrows:] == 7.0) and torch.all(wbuf[A.nrows:] == 7.0), v
    finally:
        M.release()


def dev_of():
    return torch.device("cuda:0")


@pytest.mark.parametrize("dt", [1, 0])
@pytest.mark.parametrize("name", list(ALL))
def test_xwin_every_variant(spk, dev, name, dt):
    A = ALL[name].astype(NP[dt])
    x = I.uniform(7, 0, A.ncols, NP[dt])
    say(f"x-window {name} dtype={dt}: m={A.nrows} n={A.ncols} nnz={A.nnz}")
    _run_all(spk, A, x, dt, _variants(spk))


def test_xwin_single_entry_rows_bit_exact(spk, dev):
    """A permutation times a diagonal over 100,003 columns: one product per
    row, so every kernel and window size gives it exactly."""
    n = 100003
    perm = np.argsort(I.uniform(3, 0, n)).astype(np.int32)
    d = I.uniform(4, 0, n)
    A = I.CSR(n, n, np.arange(n + 1, dtype=np.int32), perm, d)
    x = I.uniform(5, 0, n)
    M = spk.Matrix(A)
    try:
        xd = torch.from_numpy(x).to(dev)
        y = torch.empty(n, dtype=torch.float64, device=dev)
        for v in _variants(spk):
            y.fill_(float("nan"))
            spk.spk_run(spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y), v)
            assert np.array_equal(y.cpu().numpy(), d * x[perm]), v
    finally:
        M.release()


@pytest.mark.parametrize("dt", [1, 0])
def test_xwin_nan_inf(spk, dev, dt):
    A = WIDE["rand_wide"].astype(NP[dt])
    x = I.uniform(9, 0, A.ncols, NP[dt])
    used = np.unique(A.col_idx)
    x[used[[3, len(used) // 2, -1]]] = [np.nan, np.inf, -np.inf]
    say(f"x-window NaN/Inf dtype={dt}")
    _run_all(spk, A, x, dt, _variants(spk)[:2])


def test_xwin_two_streams_and_tuner(spk, dev):
    """A random-column matrix whose x (4.8 MB) exceeds an XCD's L2: the tuner
    searches the x-window form (every candidate validated first); two streams
    running it at once each use their own partials, with the same bits."""
    A = I.zipf(600000, seed_struct=21, seed_val=22)
    x = I.uniform(23, 0, A.ncols)
    say(f"x-window zipf(600000): {A.nnz} nnz")
    h = spk.Handle(0)
    M = spk.Matrix(A, handle=h)
    try:
        xd = torch.from_numpy(x).to(dev)
        y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
        p = spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y)
        before = M.bytes()
        rep = spk.spk_tune(p, reps=3, warmup=1, formats=1 << spk.SPK_FMT_XWIN, record=False, handle=h)
        say(f"x-window tuned: {rep.best} {rep.best_us:.1f} us")
        assert rep.best.format == spk.SPK_FMT_XWIN and rep.rejected == 0 and rep.tried == len(_variants(spk))
        # the regrouped entries, plans and partials are counted with the matrix
        assert M.bytes() >= before + A.nnz * 10
        _check(A, x, y)
        y2 = torch.empty_like(y)
        side = torch.cuda.Stream()
        for _ in range(2):
            y.fill_(float("nan"))
            y2.fill_(float("nan"))
            side.wait_stream(torch.cuda.current_stream())
            spk.spk_run(p, rep.best, handle=h)
            with torch.cuda.stream(side):
                spk.spk_run(spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y2), rep.best, handle=h)
            torch.cuda.synchronize()
            _check(A, x, y)
            assert torch.equal(y, y2)
    finally:
        M.release()
        h.close()


def test_xwin_rejects_bad_variants(spk, dev):
    A = I.lap2d(8)
    M = spk.Matrix(A)
    try:
        xd = torch.from_numpy(I.uniform(1, 0, A.ncols)).to(dev)
        y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
        p = spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y)
        for kw in ({"block": 512, "group": 96, "lds": 256, "grid": 1, "streams": 1},    # no such window
                   {"block": 512, "group": 128, "lds": 256, "grid": 0, "streams": 1},   # chunks per CU
                   {"block": 512, "group": 128, "lds": 256, "grid": 1, "streams": 2}):  # one stream only
            with pytest.raises(spk.SpkError):
                spk.spk_run(p, spk.make_variant(format=spk.SPK_FMT_XWIN, unroll=1, **kw))
    finally:
        M.release()
