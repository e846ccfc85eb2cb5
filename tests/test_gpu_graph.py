"""Library calls captured in a HIP graph (torch.cuda.graph) and replayed.

Every captured call must be capture-safe in its steady state: derived
formats (sliced ELL, row blocks, DIA) and the per-stream dot partials and CG
scratch are built by an eager call on the capture stream first, and the
launches themselves neither allocate, synchronise nor record memset nodes.  Each replay runs after eager work that
changes x, with the outputs poisoned, and must reproduce an eager run of the
same calls on the new x bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I

pytestmark = pytest.mark.gpu

DIA, STENCIL = 5, 6


def _variants(spk):
    """One compiled variant of every SpMV format (fused step), as (name, variant)."""
    out = {}
    for v in spk.variants(spk.SPK_OP_SPMV_WAXPY, spk.SPK_F64):
        name = {1: "scalar", 2: "vector", 3: "sell", 4: "adaptive"}.get(v.format)
        if name and name not in out:
            out[name] = v
    out["dia"] = spk.make_variant(format=DIA, block=256, group=1, unroll=1, streams=1)
    out["stencil"] = spk.make_variant(format=STENCIL, block=256, group=1, unroll=2, streams=1)
    out["stencil_lds"] = spk.make_variant(format=STENCIL, block=256, group=1, unroll=2, streams=1, lds=1)
    return out


def test_graph_replays_match_eager(spk, dev):
    A = I.lap2d(96)
    n = A.nrows
    H = spk.Handle()   # a private plan database: the recorded plan stays local to this test
    M = spk.Matrix(A, handle=H)
    try:
        assert M.formats() & (1 << DIA) and M.formats() & (1 << STENCIL)
        xd = torch.from_numpy(I.uniform(11, 0, n)).to(dev)
        vd = torch.from_numpy(I.uniform(12, 0, n)).to(dev)
        b = torch.from_numpy(I.uniform(13, 0, n)).to(dev)
        # the tuned plan (recorded) drives the plain call
        spk.spk_tune(spk.problem(spk.SPK_OP_SPMV_WAXPY, A=M, x=xd, y=torch.empty_like(xd), w=torch.empty_like(xd),
                                 alpha=0.5), reps=2, warmup=1, formats=spk.CSR_FORMATS, handle=H)
        vs = _variants(spk)
        assert set(vs) == {"scalar", "vector", "sell", "adaptive", "dia", "stencil", "stencil_lds"}
        outs = {k: (torch.empty_like(xd), torch.empty_like(xd)) for k in list(vs) + ["tuned"]}
        wx = torch.empty_like(xd)
        d = torch.empty(1, dtype=torch.float64, device=dev)
        xc = torch.zeros_like(xd)
        hist = torch.empty(11, dtype=torch.float64, device=dev)   # r.r for k = 0..10

        def calls():
            for k, v in vs.items():
                y, w = outs[k]
                spk.spk_run(spk.problem(spk.SPK_OP_SPMV_WAXPY, A=M, x=xd, y=y, w=w, alpha=0.5), v, handle=H)
            spk.spk_spmv_waxpy(M, 0.5, xd, *outs["tuned"])
            spk.spk_waxpy(1.5, xd, vd, wx, handle=H)
            spk.spk_dot(xd, vd, out=d, handle=H)
            xc.zero_()
            spk.spk_cg(M, b, xc, 10, hist)

        def snapshot():
            return [t.cpu().numpy().copy() for k in outs for t in outs[k]] + [wx.cpu().numpy(), d.cpu().numpy(),
                                                                                xc.cpu().numpy(), hist.cpu().numpy()]

        def poison():
            for k in outs:
                for t in outs[k]:
                    t.fill_(float("nan"))
            for t in (wx, d, xc, hist):
                t.fill_(float("nan"))

        # dot partials and CG scratch are kept per stream: the warm-up runs on
        # the stream the capture then uses
        cs = torch.cuda.Stream()
        cs.wait_stream(torch.cuda.current_stream())
        say("graph: eager warm-up of every captured call on the capture stream")
        with torch.cuda.stream(cs):
            calls()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        say("graph: capture")
        with torch.cuda.graph(g, stream=cs):
            calls()
        torch.cuda.synchronize()
        for r in range(3):
            x = I.uniform(100 + r, 0, n)
            xd.copy_(torch.from_numpy(x))
            poison()
            calls()                      # eager reference on the new x
            torch.cuda.synchronize()
            ref = snapshot()
            poison()
            torch.cuda.synchronize()
            say(f"graph: replay {r}")
            g.replay()
            torch.cuda.synchronize()
            got = snapshot()
            for i, (a, e) in enumerate(zip(got, ref)):
                assert np.array_equal(a, e), (r, i)
            # and the replay computed this x, not a stale one
            yref, absum = O.spmv(A, x)
            y_tuned = outs["tuned"][0].cpu().numpy()
            assert O.check_rows(y_tuned, yref, absum, O.TAU_F64)[0] == 0
        del g
    finally:
        M.release()
        H.close()
