"""Canary guards around every output buffer: each kernel variant writes its
output and nothing before or after it.

Outputs are views into larger buffers whose head and tail hold a signalling
NaN bit pattern; after every call the guards must hold the same bits, and
the output itself must hold no canary (every element was written)."""
import numpy as np
import pytest
import torch

from conftest import say
from paper_1309_1894_amd import inputs as I

pytestmark = pytest.mark.gpu

GUARD = 1024
CANARY = {1: (torch.int64, 0x7FF4DEADBEEF0001), 0: (torch.int32, 0x7FA0BEEF)}
FLOAT = {1: torch.float64, 0: torch.float32}
NP = {0: np.float32, 1: np.float64}
DIA, STENCIL = 5, 6


def guarded(n, dt, dev):
    it, bits = CANARY[dt]
    buf = torch.full((n + 2 * GUARD,), bits, dtype=it, device=dev)
    return buf, buf.view(FLOAT[dt])[GUARD:GUARD + n]


def assert_intact(buf, n, what):
    it, bits = CANARY[1 if buf.dtype == torch.int64 else 0]
    b = buf.cpu().numpy()
    head, body, tail = b[:GUARD], b[GUARD:GUARD + n], b[GUARD + n:]
    assert np.all(head == bits), f"{what}: write before the output ({np.count_nonzero(head != bits)} elements)"
    assert np.all(tail == bits), f"{what}: write past the output ({np.count_nonzero(tail != bits)} elements)"
    assert not np.any(body == bits), f"{what}: {np.count_nonzero(body == bits)} output elements never written"


def _square(dt):
    return {"lap2d_33": I.lap2d(33, dtype=NP[dt]),
            "zipf_3000": I.zipf(3000, kmax=3000, seed_struct=9, seed_val=10, dtype=NP[dt])}


@pytest.mark.parametrize("dt", [1, 0])
def test_spmv_variants_stay_inside_outputs(spk, dev, dt):
    mats = dict(_square(dt))
    mats["rect_700x3"] = I.CSR(700, 3, np.arange(701, dtype=np.int32), (np.arange(700) % 3).astype(np.int32),
                               I.uniform(5, 0, 700, NP[dt]))
    vs = spk.variants(spk.SPK_OP_SPMV, dt)
    structured = [spk.make_variant(format=DIA, block=bs, group=1, unroll=r, streams=1) for bs in (128, 512)
                  for r in (1, 2)]
    structured += [spk.make_variant(format=STENCIL, block=bs, group=1, unroll=r, streams=1, lds=l)
                   for bs, r, l in ((128, 8, 0), (512, 4, 0), (256, 2, 1), (512, 4, 1))]
    for name, A in mats.items():
        M = spk.Matrix(A)
        try:
            xd = torch.from_numpy(I.uniform(7, 0, A.ncols, NP[dt])).to(dev)
            todo = vs + ([s for s in structured if M.formats() & (1 << s.format)] if name == "lap2d_33" else [])
            say(f"guards: spmv {name} dtype={dt}, {len(todo)} variants")
            for v in todo:
                yb, y = guarded(A.nrows, dt, dev)
                spk.spk_run(spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y), v)
                assert_intact(yb, A.nrows, f"spmv {name} {v}")
                if A.nrows == A.ncols:
                    yb, y = guarded(A.nrows, dt, dev)
                    wb, w = guarded(A.nrows, dt, dev)
                    spk.spk_run(spk.problem(spk.SPK_OP_SPMV_WAXPY, A=M, x=xd, y=y, w=w, alpha=0.5), v)
                    assert_intact(yb, A.nrows, f"fused y {name} {v}")
                    assert_intact(wb, A.nrows, f"fused w {name} {v}")
        finally:
            M.release()


@pytest.mark.parametrize("dt", [1, 0])
def test_vector_variants_stay_inside_outputs(spk, dev, dt):
    n = 10007
    xd = torch.from_numpy(I.uniform(21, 0, n, NP[dt])).to(dev)
    yd = torch.from_numpy(I.uniform(22, 0, n, NP[dt])).to(dev)
    say(f"guards: waxpy/axpy/dot dtype={dt}")
    for v in spk.variants(spk.SPK_OP_WAXPY, dt):
        wb, w = guarded(n, dt, dev)
        spk.spk_run(spk.problem(spk.SPK_OP_WAXPY, x=xd, y=yd, w=w, alpha=1.5), v)
        assert_intact(wb, n, f"waxpy {v}")
    for v in spk.variants(spk.SPK_OP_AXPY, dt):
        yb, y = guarded(n, dt, dev)
        y.copy_(yd)
        spk.spk_run(spk.problem(spk.SPK_OP_AXPY, x=xd, y=y, alpha=1.5), v)
        assert_intact(yb, n, f"axpy {v}")
    for v in spk.variants(spk.SPK_OP_DOT, dt):
        ob, out = guarded(1, 1, dev)   # the result is FP64 for both dtypes
        spk.spk_run(spk.problem(spk.SPK_OP_DOT, x=xd, y=yd, d_result=out), v)
        assert_intact(ob, 1, f"dot {v}")


def test_batch_stays_inside_outputs(spk, dev):
    insts = [I.banded(int(m), int(b), 0.6, seed_struct=7, seed_val=8, stream=i)
             for i, (m, b) in enumerate(zip(*I.batch_sizes(24, seed=7, mmin=64, ratio=64.0, bmax=32)))]
    insts.append(I.zipf(3000, kmax=3000, seed_struct=9, seed_val=10))
    B = I.batch_from_instances(insts)
    arrays = (torch.from_numpy(B.row_ptr).to(dev), torch.from_numpy(B.col_idx).to(dev),
              torch.from_numpy(B.val).to(dev))
    nv = int(B.m.sum())
    xd = torch.from_numpy(I.batch_vector(B, seed=43)).to(dev)
    for persistent, graph in ((0, 0), (0, 1), (1, 0), (1, 1)):
        say(f"guards: batch persistent={persistent} graph={graph}")
        b = spk.Batch(B, arrays, persistent=bool(persistent), use_graph=bool(graph))
        try:
            yb, y = guarded(nv, 1, dev)
            wb, w = guarded(nv, 1, dev)
            for r in range(2):   # with use_graph: the capture, then a replay
                if r:
                    for t in (yb, wb):
                        t[GUARD:GUARD + nv].fill_(CANARY[1][1])
                b.run(0.5, xd, y, w)
                assert_intact(yb, nv, f"batch y p={persistent} g={graph} run {r}")
                assert_intact(wb, nv, f"batch w p={persistent} g={graph} run {r}")
        finally:
            b.free()


def test_cg_stays_inside_outputs(spk, dev):
    A = I.lap2d(20)
    n = A.nrows
    M = spk.Matrix(A)
    try:
        b = torch.from_numpy(I.uniform(13, 0, n)).to(dev)
        xb, x = guarded(n, 1, dev)
        x.zero_()
        hb, hist = guarded(13, 1, dev)    # r.r for k = 0..12
        say("guards: cg lap2d 20, 12 iterations")
        spk.spk_cg(M, b, x, 12, hist)
        assert_intact(xb, n, "cg x")
        assert_intact(hb, 13, "cg residual history")
    finally:
        M.release()
