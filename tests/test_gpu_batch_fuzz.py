"""Seeded random batches through the batched tile kernel: instance shapes the
workload generator never makes (empty matrices, empty rows, a single row,
rows longer than a wavefront tile, dense bands, Zipf rows) in random mixes,
both dtypes and every launch kind, each instance checked against the oracle
and, with graph replay, the replay equal to the first launch bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I

pytestmark = pytest.mark.gpu


def _long_row(m, rng, dtype):
    """Diagonal plus one row holding every column."""
    r = int(rng.integers(0, m))
    rows = np.concatenate([np.arange(m), np.full(m, r)])
    cols = np.concatenate([np.arange(m), np.arange(m)])
    keep = ~((rows == r) & (np.arange(2 * m) < m))   # the long row carries its own diagonal
    rows, cols = rows[keep], cols[keep]
    order = np.lexsort((cols, rows))
    rp = np.zeros(m + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    val = rng.uniform(-1, 1, rows.size).astype(dtype)
    return I.CSR(m, m, np.cumsum(rp).astype(np.int32), cols[order].astype(np.int32), val)


def _empty(m, dtype):
    return I.CSR(m, m, np.zeros(m + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, dtype))


def random_batch(seed):
    rng = np.random.default_rng(1000 + seed)
    dtype = np.float64 if seed % 3 else np.float32
    insts = []
    for i in range(int(rng.integers(1, 20))):
        kind = int(rng.integers(0, 5))
        if kind == 0:
            insts.append(_empty(int(rng.integers(0, 40)), dtype))
        elif kind == 1:
            insts.append(I.banded(int(rng.integers(1, 4000)), int(rng.integers(0, 40)), float(rng.uniform(0.05, 1.0)),
                                  seed_struct=80 + seed, seed_val=81, stream=i, dtype=dtype))
        elif kind == 2:
            m = int(rng.integers(1, 3000))
            insts.append(I.zipf(m, kmax=max(1, min(4096, m)), seed_struct=82 + seed * 31 + i, seed_val=83,
                                dtype=dtype))
        elif kind == 3:
            insts.append(_long_row(int(rng.integers(100, 6000)), rng, dtype))
        else:
            insts.append(I.banded(1, 0, 1.0, seed_struct=84, seed_val=85, stream=i, dtype=dtype))   # 1x1
    return insts, dtype


@pytest.mark.parametrize("seed", range(12))
def test_random_batches(spk, dev, seed):
    insts, dtype = random_batch(seed)
    B = I.batch_from_instances(insts)
    nv = int(B.m.sum())
    x = I.batch_vector(B, seed=86 + seed, dtype=dtype)
    arrays = (torch.from_numpy(B.row_ptr).to(dev), torch.from_numpy(B.col_idx).to(dev),
              torch.from_numpy(B.val).to(dev))
    xd = torch.from_numpy(x).to(dev)
    persistent, graph = (seed // 2) % 2, seed % 2
    say(f"fuzz batch seed={seed}: {B.count} instances, {nv} rows, {int(B.nnz.sum())} nnz, dtype={dtype.__name__}, "
        f"persistent={persistent} graph={graph}")
    b = spk.Batch(B, arrays, persistent=bool(persistent), use_graph=bool(graph))
    try:
        y = torch.full((max(nv, 1),), float("nan"), dtype=xd.dtype, device=dev)[:nv]
        w = torch.full((max(nv, 1),), float("nan"), dtype=xd.dtype, device=dev)[:nv]
        b.run(0.5, xd, y, w)
        torch.cuda.synchronize()
        yg, wg = y.cpu().numpy().copy(), w.cpu().numpy().copy()
        for i in range(B.count):
            A = B.instance(i)
            o = int(B.vec_off[i])
            xi = x[o:o + A.nrows]
            ref, absum = O.spmv(A, xi)
            bad, worst, at = O.check_rows(yg[o:o + A.nrows].astype(np.float64), ref, absum, O.tau_for(dtype))
            assert bad == 0, f"seed {seed} instance {i}: {bad} rows (worst {worst:g} at {at})"
            d, at = O.max_ulp(wg[o:o + A.nrows], O.waxpy(0.5, yg[o:o + A.nrows], xi))
            assert d <= (0 if dtype == np.float64 else 1), (seed, i, d, at)
        # a second launch (with use_graph: the replay) gives the same bits
        y.fill_(float("nan"))
        w.fill_(float("nan"))
        b.run(0.5, xd, y, w)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), yg) and np.array_equal(w.cpu().numpy(), wg)
    finally:
        b.free()


@pytest.mark.parametrize("seed", range(6))
def test_random_batches_compact_columns(spk, dev, seed):
    """The random batches with every class planned to compact columns (mode
    3) on kernels with room for x, one to four wavefronts per workgroup:
    each instance against the oracle, and bit for bit the result of the
    plain row stream (mode 0) on the same batch."""
    insts, dtype = random_batch(seed)
    B = I.batch_from_instances(insts)
    nv = int(B.m.sum())
    x = I.batch_vector(B, seed=86 + seed, dtype=dtype)
    arrays = (torch.from_numpy(B.row_ptr).to(dev), torch.from_numpy(B.col_idx).to(dev),
              torch.from_numpy(B.val).to(dev))
    xd = torch.from_numpy(x).to(dev)
    block = (64, 128, 256)[seed % 3]
    persistent = seed % 2
    dname = "f64" if dtype == np.float64 else "f32"
    outs = {}
    for mode, xw in ((0, 256), (3, 256)):
        h = spk.Handle(0)
        for c in range(21):
            spk.spk_plan_put(f"batch:{dname}:c{c}",
                             spk.make_variant(format=spk.SPK_FMT_ADAPTIVE, block=block, group=mode, unroll=1,
                                              streams=1, lds=2048), handle=h)
        b = spk.Batch(B, arrays, handle=h, block=block, x_window=xw, persistent=bool(persistent))
        say(f"fuzz compact seed={seed}: {B.count} instances, {nv} rows, mode {mode}, block {block}, "
            f"persistent={persistent}, dtype={dname}, tiles per mode {b.tile_modes()}")
        try:
            y = torch.full((max(nv, 1),), float("nan"), dtype=xd.dtype, device=dev)[:nv]
            w = torch.full((max(nv, 1),), float("nan"), dtype=xd.dtype, device=dev)[:nv]
            b.run(0.5, xd, y, w)
            torch.cuda.synchronize()
            outs[mode] = (y.cpu().numpy().copy(), w.cpu().numpy().copy())
        finally:
            b.free()
            h.close()
    yg, wg = outs[3]
    for i in range(B.count):
        A = B.instance(i)
        o = int(B.vec_off[i])
        xi = x[o:o + A.nrows]
        ref, absum = O.spmv(A, xi)
        bad, worst, at = O.check_rows(yg[o:o + A.nrows].astype(np.float64), ref, absum, O.tau_for(dtype))
        assert bad == 0, f"seed {seed} instance {i}: {bad} rows (worst {worst:g} at {at})"
        d, at = O.max_ulp(wg[o:o + A.nrows], O.waxpy(0.5, yg[o:o + A.nrows], xi))
        assert d <= (0 if dtype == np.float64 else 1), (seed, i, d, at)
    assert np.array_equal(outs[0][0], yg) and np.array_equal(outs[0][1], wg)
