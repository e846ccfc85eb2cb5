"""SpMV over more rows than one launch covers with G lanes per row: 2^25 + 4099
rows, so the 32- and 64-lane forms need more than 2^30 work-items and run as
consecutive launches over row ranges.  Integer-valued data make every row's
exact sum representable, so each row is checked bit for bit against its
closed form (FP64 and FP32, plain and fused step), rows sampled across the
2^24 and 2^25 boundaries also against the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I

pytestmark = pytest.mark.gpu

M = (1 << 25) + 4099


def _matrix(dtype):
    """Row i holds columns i and (i + M/2) mod M, except every 1000th row,
    which is empty; values and x are small integers."""
    i = np.arange(M, dtype=np.int64)
    j = (i + M // 2) % M
    empty = (i % 1000) == 999
    lens = np.where(empty, 0, 2)
    rp = np.zeros(M + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    v1 = (i % 7 - 3).astype(dtype)
    v2 = (i % 5 + 1).astype(dtype)
    lo = i < j
    cols = np.stack([np.where(lo, i, j), np.where(lo, j, i)], 1)[~empty].ravel()
    vals = np.stack([np.where(lo, v1, v2), np.where(lo, v2, v1)], 1)[~empty].ravel()
    x = (i % 11 - 5).astype(dtype)
    y = np.where(empty, 0, v1.astype(np.float64) * x[i] + v2.astype(np.float64) * x[j]).astype(dtype)
    return I.CSR(M, M, rp.astype(np.int32), cols.astype(np.int32), vals), x, y


def _sample_rows(A, rows):
    """The sampled rows as their own CSR (all columns kept)."""
    rp = A.row_ptr.astype(np.int64)
    lens = rp[rows + 1] - rp[rows]
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
    srp = np.zeros(rows.size + 1, np.int64)
    srp[1:] = np.cumsum(lens)
    return I.CSR(rows.size, A.ncols, srp.astype(np.int32), A.col_idx[idx], A.val[idx])


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_spmv_more_rows_than_one_launch(spk, dev, dtype):
    dt = 1 if dtype == np.float64 else 0
    say(f"huge spmv: {M} rows, dtype={dtype.__name__}")
    A, x, y_exact = _matrix(dtype)
    w_exact = (0.5 * y_exact.astype(np.float64) + x).astype(dtype)
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([np.arange(0, 8), np.arange((1 << 24) - 8, (1 << 24) + 8),
                                     np.arange((1 << 25) - 8, (1 << 25) + 8), np.arange(M - 8, M),
                                     rng.integers(0, M, 1000)]))
    ref, absum = O.spmv(_sample_rows(A, rows), x)
    assert np.array_equal(ref, y_exact[rows].astype(np.float64))
    Mx = spk.Matrix(A)
    try:
        xd = torch.from_numpy(x).to(dev)
        y = torch.empty(M, dtype=Mx.torch_dtype, device=dev)
        w = torch.empty_like(y)
        vs = [v for v in spk.variants(spk.SPK_OP_SPMV, dt) if v.format == spk.SPK_FMT_VECTOR and v.group >= 32]
        two = spk.make_variant(**{**vs[-1].as_dict(), "streams": 2})
        vs += [two, spk.spk_plain_variant(spk.SPK_OP_SPMV, 0), spk.spk_plain_variant(spk.SPK_OP_SPMV, 1), None]
        for v in vs:
            say(f"huge spmv variant {v}")
            y.fill_(float("nan"))
            spk.spk_run(spk.problem(spk.SPK_OP_SPMV, A=Mx, x=xd, y=y), v)
            yg = y.cpu().numpy()
            assert np.array_equal(yg, y_exact), (v, int(np.flatnonzero(yg != y_exact)[0]))
            assert O.check_rows(yg[rows].astype(np.float64), ref, absum, O.tau_for(dtype))[0] == 0, v
            if v is None or v.group == 64:
                y.fill_(float("nan"))
                w.fill_(float("nan"))
                spk.spk_run(spk.problem(spk.SPK_OP_SPMV_WAXPY, A=Mx, x=xd, y=y, w=w, alpha=0.5), v)
                assert np.array_equal(y.cpu().numpy(), y_exact), v
                assert np.array_equal(w.cpu().numpy(), w_exact), v
    finally:
        Mx.release()
        torch.cuda.empty_cache()
