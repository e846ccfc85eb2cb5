"""GPU parity of WAXPY, AXPY and dot against the oracle, for every compiled
variant (block, vector width, unroll, grid), FP64 and FP32."""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I

pytestmark = pytest.mark.gpu

NP = {0: np.float32, 1: np.float64}


def _vec(n, seed, stream, dt, dev):
    a = I.uniform(seed, stream, n, NP[dt])
    return a, torch.from_numpy(a).to(dev)


@pytest.mark.parametrize("dt", [1, 0])
def test_waxpy_every_variant(spk, dev, dt):
    n = 100003  # ragged against every block size
    x, xd = _vec(n, 21, 0, dt, dev)
    y, yd = _vec(n, 22, 0, dt, dev)
    ref = O.waxpy(1.5, x, y)
    wd = torch.empty_like(xd)
    vs = spk.variants(spk.SPK_OP_WAXPY, dt)
    say(f"waxpy dtype={dt}: {len(vs)} variants, n={n}")
    for v in vs:
        wd.fill_(float("nan"))
        spk.spk_run(spk.problem(spk.SPK_OP_WAXPY, x=xd, y=yd, w=wd, alpha=1.5), v)
        got = wd.cpu().numpy()
        d, at = O.max_ulp(got, ref)
        limit = 0 if dt == 1 else 1   # FP64: both sides one fma; FP32: oracle rounds twice
        assert d <= limit, (v, d, at)


@pytest.mark.parametrize("dt", [1, 0])
def test_dot_every_variant(spk, dev, dt):
    n = 100003
    x, xd = _vec(n, 21, 0, dt, dev)
    y, yd = _vec(n, 22, 0, dt, dev)
    ref = O.dot(x, y)
    tol = O.tau_for(NP[dt]) * O.dot_absum(x, y)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    vs = spk.variants(spk.SPK_OP_DOT, dt)
    say(f"dot dtype={dt}: {len(vs)} variants")
    for v in vs:
        out.fill_(float("nan"))
        p = spk.problem(spk.SPK_OP_DOT, x=xd, y=yd, d_result=out)
        spk.spk_run(p, v)
        a = out.item()
        spk.spk_run(p, v)
        b = out.item()
        assert a == b, (v, "not reproducible")
        assert abs(a - ref) <= tol, (v, a, ref)


@pytest.mark.parametrize("dt", [1, 0])
@pytest.mark.parametrize("n", [0, 1, 2, 63, 64, 65, 255, 257, 4097, 1 << 20, (1 << 20) + 7])
def test_vector_ops_sizes(spk, dev, dt, n):
    say(f"vector ops dtype={dt} n={n}")
    x, xd = _vec(n, 1, 0, dt, dev)
    y, yd = _vec(n, 2, 0, dt, dev)
    lim = 0 if dt == 1 else 1
    w = spk.spk_waxpy(1.5, xd, yd)
    assert O.max_ulp(w.cpu().numpy(), O.waxpy(1.5, x, y))[0] <= lim
    y2 = yd.clone()
    spk.spk_axpy(-0.75, xd, y2)
    assert O.max_ulp(y2.cpu().numpy(), O.axpy(-0.75, x, y))[0] <= lim
    d = spk.spk_dot(xd, yd).item()
    assert abs(d - O.dot(x, y)) <= O.tau_for(NP[dt]) * O.dot_absum(x, y)
    if n == 0:
        assert d == 0.0


def test_waxpy_misaligned_and_aliased(spk, dev):
    n = 5001
    x, xd = _vec(n + 1, 3, 0, 1, dev)
    y, yd = _vec(n + 1, 4, 0, 1, dev)
    # offset by one element: 8-byte aligned only, vector loads must fall back
    w = spk.spk_waxpy(1.5, xd[1:], yd[1:])
    assert O.max_ulp(w.cpu().numpy(), O.waxpy(1.5, x[1:], y[1:]))[0] == 0
    # w == x and w == y are allowed
    a = xd.clone()
    spk.spk_waxpy(1.5, a, yd, w=a)
    assert O.max_ulp(a.cpu().numpy(), O.waxpy(1.5, x, y))[0] == 0
    b = yd.clone()
    spk.spk_axpy(2.0, b, b)   # y <- 2y + y
    assert np.array_equal(b.cpu().numpy(), O.axpy(2.0, y, y))
    with pytest.raises(spk.SpkError) as e:
        spk.spk_waxpy(1.5, xd[:-1], yd[:-1], w=xd[1:])
    assert e.value.name == "SPK_ERR_ALIAS"


def test_special_values_and_alpha_zero(spk, dev):
    x = np.array([np.inf, -np.inf, np.nan, 1.0, 0.0, -0.0, 5e-324, 1e308])
    y = np.array([1.0, np.inf, 2.0, np.nan, -0.0, -0.0, 5e-324, 1e308])
    for alpha in (0.0, 1.5, -2.0):
        w = spk.spk_waxpy(alpha, torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev))
        assert O.max_ulp(w.cpu().numpy(), O.waxpy(alpha, x, y))[0] == 0


def test_integer_dot_closed_form(spk, dev):
    n = (1 << 22) + 5
    ones = torch.ones(n, dtype=torch.float64, device=dev)
    idx = torch.arange(n, dtype=torch.float64, device=dev)
    assert spk.spk_dot(ones, ones).item() == n
    assert spk.spk_dot(idx, ones).item() == n * (n - 1) // 2
    f = torch.ones(n, dtype=torch.float32, device=dev)
    assert spk.spk_dot(f, f).item() == n   # FP64 accumulation of FP32 data


def test_plain_mode_and_tuned_dispatch(spk, dev):
    h = spk.Handle(0)
    try:
        n = 300001
        x, xd = _vec(n, 5, 0, 1, dev)
        y, yd = _vec(n, 6, 0, 1, dev)
        h.set_plain(True)
        w1 = spk.spk_waxpy(1.5, xd, yd, handle=h)
        h.set_plain(False)
        w2 = spk.spk_waxpy(1.5, xd, yd, handle=h)
        assert torch.equal(w1, w2)
        assert O.max_ulp(w2.cpu().numpy(), O.waxpy(1.5, x, y))[0] == 0
    finally:
        h.close()


@pytest.mark.parametrize("dt", [1, 0])
def test_vector_ops_at_2_pow_27_as_benched(spk, dev, dt):
    """WAXPY, AXPY and dot at n = 2^27 on the bench's inputs, tuned as the
    bench tunes them; the winners and the default dispatch (which follows
    the recorded plan) against the oracle."""
    n = 1 << 27
    npdt = np.float64 if dt == 1 else np.float32
    say(f"vector ops n=2^27 dtype={npdt.__name__}")
    xh, yh = I.uniform(21, 0, n, npdt), I.uniform(22, 0, n, npdt)
    x, y = torch.from_numpy(xh).to(dev), torch.from_numpy(yh).to(dev)
    w = torch.empty_like(x)
    d = torch.empty(1, dtype=torch.float64, device=dev)
    h = spk.Handle(0)
    ulp = 0 if dt == 1 else 1
    try:
        ref_w = O.waxpy(1.5, xh, yh)
        ref_d = O.dot(xh, yh)
        scale = O.dot_absum(xh, yh)
        for op in (spk.SPK_OP_WAXPY, spk.SPK_OP_AXPY, spk.SPK_OP_DOT):
            p = spk.problem(op, x=x, y=y, w=w if op == spk.SPK_OP_WAXPY else None,
                            d_result=d if op == spk.SPK_OP_DOT else None, alpha=1.5)
            rep = spk.spk_tune(p, reps=5, warmup=1, flush=False, record=True, handle=h)
            assert rep.rejected == 0
            for v in (rep.best, None):
                if op == spk.SPK_OP_WAXPY:
                    w.fill_(float("nan"))
                    spk.spk_run(p, v, handle=h)
                    assert O.max_ulp(w.cpu().numpy(), ref_w)[0] <= ulp, (op, v)
                elif op == spk.SPK_OP_AXPY:
                    y.copy_(torch.from_numpy(yh))   # in place: start from the input again
                    spk.spk_run(p, v, handle=h)
                    assert O.max_ulp(y.cpu().numpy(), ref_w)[0] <= ulp, (op, v)
                    y.copy_(torch.from_numpy(yh))
                else:
                    d.fill_(float("nan"))
                    spk.spk_run(p, v, handle=h)
                    assert abs(d.item() - ref_d) <= O.tau_for(npdt) * scale, (op, v, d.item(), ref_d)
    finally:
        h.close()
