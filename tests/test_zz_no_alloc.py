"""spk_dot_noalloc: the dot on the library's fixed per-GPU scratch gives the
same bits as spk_dot (same variant, same reduction order) on consecutive
calls that shrink, and stays within the oracle's dot tolerance; a dot whose
variant needs more partials than the scratch holds is refused before any
launch."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I

pytestmark = pytest.mark.gpu


def _bits(t):
    return t.cpu().numpy().view(np.uint64)[0]


def _pair(n, dt, dev, seed):
    x = I.uniform(seed, 0, n, dt)
    y = I.uniform(seed, 1, n, dt)
    return x, y, torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_dot_noalloc_equals_dot(spk, dev, dt):
    h = spk.Handle(0)   # no plans: the default dot variant on both paths
    try:
        # a large dot (partials added by a second launch), then smaller ones:
        # one workgroup (ticket), none, and a mid-sized grid again
        for k, n in enumerate((3_000_001, 1000, 0, 70_000)):
            x, y, xd, yd = _pair(n, dt, dev, 60 + k)
            say(f"dot_noalloc dtype={np.dtype(dt).name} n={n}")
            ref = spk.spk_dot(xd, yd, handle=h)
            out = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
            st = spk.lib.spk_dot_noalloc(h.ptr, spk.SPK_F64 if dt == np.float64 else spk.SPK_F32, n,
                                         xd.data_ptr() if n else None, yd.data_ptr() if n else None,
                                         out.data_ptr(), torch.cuda.current_stream().cuda_stream)
            assert st == 0, spk.spk_status_str(st)
            torch.cuda.synchronize()
            assert _bits(out) == _bits(ref), (n, out.item(), ref.item())
            tau = O.tau_for(dt)
            assert abs(out.item() - O.dot(x, y)) <= tau * O.dot_absum(x, y), n
    finally:
        h.close()


def test_dot_noalloc_two_calls_in_a_row_and_size_limit(spk, dev):
    """Back-to-back calls on one stream (the second smaller) through the
    binding, and the one-pass plain variant: 2^24 elements need exactly the
    65,536 partials the scratch holds, one more element is refused."""
    h = spk.Handle(0)
    try:
        outs = []
        for k, n in enumerate((1_000_003, 4_097)):
            x, y, xd, yd = _pair(n, np.float64, dev, 70 + k)
            out = torch.empty(1, dtype=torch.float64, device=dev)
            spk.spk_dot_noalloc(xd, yd, out, handle=h)
            outs.append((x, y, xd, yd, out))
        torch.cuda.synchronize()
        for x, y, xd, yd, out in outs:
            assert _bits(out) == _bits(spk.spk_dot(xd, yd, handle=h))
        h.set_plain(True)
        n = 1 << 24
        x, y, xd, yd = _pair(n + 1, np.float64, dev, 80)
        out = torch.empty(1, dtype=torch.float64, device=dev)
        say("dot_noalloc plain variant at 2^24 elements")
        spk.spk_dot_noalloc(xd[:n], yd[:n], out, handle=h)
        ref = spk.spk_dot(xd[:n], yd[:n], handle=h)
        torch.cuda.synchronize()
        assert _bits(out) == _bits(ref)
        assert abs(out.item() - O.dot(x[:n], y[:n])) <= O.TAU_F64 * O.dot_absum(x[:n], y[:n])
        with pytest.raises(spk.SpkError, match="SPK_ERR_SHAPE"):
            spk.spk_dot_noalloc(xd, yd, out, handle=h)
    finally:
        h.close()
