"""Seeded random matrices through every compiled SpMV variant: runs of empty
rows, rows longer than any tile, very short and very long rows side by side,
tall and wide shapes, in FP64 and FP32; each variant against the oracle
(plain and, for square matrices, the fused step)."""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I

pytestmark = pytest.mark.gpu

NP = {0: np.float32, 1: np.float64}


def random_matrix(seed, dtype):
    rng = np.random.default_rng(2000 + seed)
    m = int(rng.integers(1, 20000))
    n = m if seed % 2 == 0 else int(rng.integers(1, 20000))
    # row lengths: mostly short, runs of empty rows, a few long ones
    lens = rng.integers(0, 9, m)
    for _ in range(int(rng.integers(0, 4))):
        a = int(rng.integers(0, m))
        lens[a:a + int(rng.integers(1, 300))] = 0
    for _ in range(int(rng.integers(0, 4))):
        lens[int(rng.integers(0, m))] = int(rng.integers(64, min(n, 9000) + 1)) if n >= 64 else n
    lens = np.minimum(lens, n)
    rows = np.repeat(np.arange(m), lens)
    cols = np.concatenate([np.sort(rng.choice(n, int(k), replace=False)) for k in lens if k > 0]) \
        if lens.sum() else np.zeros(0, np.int64)
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    val = rng.uniform(-1, 1, rows.size).astype(dtype)
    return I.CSR(m, n, rp.astype(np.int32), cols.astype(np.int32), val)


@pytest.mark.parametrize("seed", range(8))
def test_random_matrices_every_variant(spk, dev, seed):
    dt = 1 if seed % 4 < 2 else 0
    A = random_matrix(seed, NP[dt])
    x = I.uniform(90 + seed, 0, A.ncols, NP[dt])
    ref, absum = O.spmv(A, x)
    M = spk.Matrix(A)
    try:
        xd = torch.from_numpy(x).to(dev)
        y = torch.empty(A.nrows, dtype=M.torch_dtype, device=dev)
        w = torch.empty_like(y)
        vs = spk.variants(spk.SPK_OP_SPMV, dt)
        say(f"spmv fuzz seed={seed}: {A.nrows}x{A.ncols}, {A.nnz} nnz, dtype={dt}, {len(vs)} variants")
        for v in vs:
            y.fill_(float("nan"))
            spk.spk_run(spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y), v)
            yg = y.cpu().numpy()
            bad, worst, at = O.check_rows(yg.astype(np.float64), ref, absum, O.tau_for(NP[dt]))
            assert bad == 0, (seed, v, bad, worst, at)
            if A.nrows == A.ncols:
                y.fill_(float("nan"))
                w.fill_(float("nan"))
                spk.spk_run(spk.problem(spk.SPK_OP_SPMV_WAXPY, A=M, x=xd, y=y, w=w, alpha=0.5), v)
                yg = y.cpu().numpy()
                assert O.check_rows(yg.astype(np.float64), ref, absum, O.tau_for(NP[dt]))[0] == 0, (seed, v)
                d, at = O.max_ulp(w.cpu().numpy(), O.waxpy(0.5, yg, x))
                assert d <= (0 if dt == 1 else 1), (seed, v, d, at)
    finally:
        M.release()
