"""GPU parity of the column-blocked SpMV form (SPK_FMT_COLBLOCK): the matrix
split by column ranges into sub-matrices of all rows, one row-block pass per
block into FP64 partials, then one pass adding them in block order.  Every
block count and per-block kernel against the oracle on the structural edge
cases (plain and fused), canaries after the outputs, two streams at once,
the FP32 refusal, and the tuner's search on a matrix whose x exceeds an
XCD's L2."""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I
from test_gpu_spmv import CASES, _check

pytestmark = pytest.mark.gpu

SHAPES = [(512, 256), (128, 256), (256, 1024)]


def _variants(spk):
    return [spk.make_variant(format=spk.SPK_FMT_COLBLOCK, block=bs, group=nb, unroll=1, streams=1, lds=lds)
            for nb in (2, 4) for bs, lds in SHAPES]


@pytest.mark.parametrize("name", list(CASES))
def test_column_blocks_every_variant(spk, dev, name):
    A = CASES[name]
    x = I.uniform(7, 0, A.ncols)
    M = spk.Matrix(A)
    try:
        xd = torch.from_numpy(x).to(dev)
        pad = 64
        ybuf = torch.full((A.nrows + pad,), 7.0, dtype=torch.float64, device=dev)
        wbuf = torch.full((A.nrows + pad,), 7.0, dtype=torch.float64, device=dev)
        y, w = ybuf[:A.nrows], wbuf[:A.nrows]
        for v in _variants(spk):
            say(f"column blocks {name}: {v}")
            y.fill_(float("nan"))
            spk.spk_run(spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y), v)
            _check(A, x, y)
            if A.nrows == A.ncols:
                y.fill_(float("nan"))
                w.fill_(float("nan"))
                spk.spk_run(spk.problem(spk.SPK_OP_SPMV_WAXPY, A=M, x=xd, y=y, w=w, alpha=0.5), v)
                _check(A, x, y, w, 0.5)
            assert torch.all(ybuf[A.nrows:] == 7.0) and torch.all(wbuf[A.nrows:] == 7.0), v
    finally:
        M.release()


def test_column_blocks_fp32_refused(spk, dev):
    A = I.lap2d(8, dtype=np.float32)
    M = spk.Matrix(A)
    try:
        assert not M.formats() & (1 << spk.SPK_FMT_COLBLOCK)
        xd = torch.from_numpy(I.uniform(1, 0, A.ncols, np.float32)).to(dev)
        y = torch.empty(A.nrows, dtype=torch.float32, device=dev)
        with pytest.raises(spk.SpkError):
            spk.spk_run(spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y), _variants(spk)[0])
    finally:
        M.release()


def test_column_blocks_two_streams_and_tuner(spk, dev):
    """A random-column matrix whose x (4.8 MB) exceeds an XCD's L2: the
    tuner searches the column-blocked form; two streams running it at once
    each use their own partials."""
    A = I.zipf(600000, seed_struct=21, seed_val=22)
    x = I.uniform(23, 0, A.ncols)
    say(f"column blocks zipf(600000): {A.nnz} nnz")
    h = spk.Handle(0)
    M = spk.Matrix(A, handle=h)
    try:
        xd = torch.from_numpy(x).to(dev)
        y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
        p = spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y)
        before = M.bytes()
        rep = spk.spk_tune(p, reps=3, warmup=1, formats=1 << spk.SPK_FMT_COLBLOCK, record=False, handle=h)
        # the sub-matrices and partials are counted with the matrix
        assert M.bytes() >= before + A.nnz * 12 + 2 * 8 * A.nrows
        assert rep.best.format == spk.SPK_FMT_COLBLOCK and rep.rejected == 0 and rep.tried >= 6
        _check(A, x, y)
        v2, v4 = _variants(spk)[0], _variants(spk)[3]
        y2 = torch.empty_like(y)
        side = torch.cuda.Stream()
        for _ in range(2):   # the second round reuses both streams' partials
            y.fill_(float("nan"))
            y2.fill_(float("nan"))
            side.wait_stream(torch.cuda.current_stream())
            spk.spk_run(p, v2, handle=h)
            with torch.cuda.stream(side):
                spk.spk_run(spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y2), v2, handle=h)
            torch.cuda.synchronize()
            _check(A, x, y)
            _check(A, x, y2)
            assert torch.equal(y, y2)
        spk.spk_run(p, v4, handle=h)
        _check(A, x, y)
    finally:
        M.release()
        h.close()
