"""Vector operations past 2^32 elements (FP32, three 17 GB arrays): 64-bit
indexing in the kernels and launch grids capped below the 32-bit work-item
limit (the kernels then loop over the grid).  Inputs are periodic patterns
with prime periods, so every sampled result and the dot product have exact
closed forms: WAXPY/AXPY at indices across the 2^31 and 2^32 boundaries, the
ends and random positions; dot equal to the exact integer sum."""
import numpy as np
import pytest
import torch

from conftest import say

pytestmark = pytest.mark.gpu

N = (1 << 32) + 7
PX, PY = 1021, 509


def _pattern(period, n, scale, dev):
    base = torch.arange(period, dtype=torch.float32, device=dev) * scale
    return base.repeat((n + period - 1) // period)[:n]


def _indices(n):
    rng = np.random.default_rng(7)
    fixed = [0, 1, 2, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, (1 << 32) - 1, 1 << 32, (1 << 32) + 1, n - 2, n - 1]
    return np.unique(np.concatenate([np.array(fixed, np.int64), rng.integers(0, n, 4096)]))


def _expected_waxpy(idx, alpha):
    return (alpha * (idx % PX) + 0.5 * (idx % PY)).astype(np.float32)


def test_vector_ops_past_2_pow_32(spk, dev):
    free, total = torch.cuda.mem_get_info()
    if free < 80 * (1 << 30):
        pytest.skip(f"needs about 75 GB of free device memory ({free >> 30} GB free)")
    say(f"huge vectors: n = {N} FP32")
    x = _pattern(PX, N, 1.0, dev)
    y = _pattern(PY, N, 0.5, dev)
    w = torch.empty(N, dtype=torch.float32, device=dev)
    idx = _indices(N)
    idx_d = torch.from_numpy(idx).to(dev)
    try:
        variants = [spk.make_variant(block=256, vec=1, unroll=1, grid=0),    # one pass, grid capped
                    spk.make_variant(block=64, vec=1, unroll=1, grid=0),
                    spk.make_variant(block=256, vec=4, unroll=4, grid=0),
                    spk.make_variant(block=512, vec=2, unroll=2, grid=2)]    # grid-stride
        for v in variants:
            say(f"huge waxpy block={v.block} vec={v.vec} unroll={v.unroll} grid={v.grid}")
            w.fill_(float("nan"))
            spk.spk_run(spk.problem(spk.SPK_OP_WAXPY, x=x, y=y, w=w, alpha=1.5), v)
            got = w[idx_d].cpu().numpy()
            assert np.array_equal(got, _expected_waxpy(idx, 1.5)), v
            assert not torch.isnan(w).any().item(), v   # every element written
        say("huge axpy")
        spk.spk_run(spk.problem(spk.SPK_OP_AXPY, x=x, y=y, alpha=1.5), variants[2])
        assert np.array_equal(y[idx_d].cpu().numpy(), _expected_waxpy(idx, 1.5))
        y.copy_(_pattern(PY, N, 0.5, dev))
        # dot: sum (i mod PX) * 0.5 (i mod PY), an exact FP64 sum
        L = PX * PY
        i = np.arange(L, dtype=np.int64)
        per = int(((i % PX) * (i % PY)).sum())
        q, r = divmod(N, L)
        j = np.arange(r, dtype=np.int64)
        exact = 0.5 * (q * per + int(((j % PX) * (j % PY)).sum()))
        out = torch.empty(1, dtype=torch.float64, device=dev)
        for v in (spk.make_variant(block=256, vec=1, unroll=1, grid=0), spk.make_variant(block=512, vec=1, unroll=4,
                                                                                          grid=2)):
            say(f"huge dot block={v.block} grid={v.grid}")
            out.fill_(float("nan"))
            spk.spk_run(spk.problem(spk.SPK_OP_DOT, x=x, y=y, d_result=out), v)
            assert out.item() == exact, (v, out.item(), exact)
    finally:
        del x, y, w
        torch.cuda.empty_cache()
