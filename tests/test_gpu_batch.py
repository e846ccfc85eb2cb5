"""Batched execution: one (persistent, graph-replayed) launch over many CSR
instances matches the oracle per instance, and gives every instance the same
bits as running it alone."""
import dataclasses
import json

import numpy as np
import pytest
import torch

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I

pytestmark = pytest.mark.gpu


def _dev_batch(B, dev):
    return (torch.from_numpy(B.row_ptr).to(dev), torch.from_numpy(B.col_idx).to(dev),
            torch.from_numpy(B.val).to(dev))


def _check_batch(B, x, y, w, alpha, dt=np.float64):
    yg, wg = y.cpu().numpy(), w.cpu().numpy() if w is not None else None
    for i in range(B.count):
        A = B.instance(i)
        o = int(B.vec_off[i])
        xi = x[o:o + A.nrows]
        ref, absum = O.spmv(A, xi)
        bad, worst, at = O.check_rows(yg[o:o + A.nrows].astype(np.float64), ref, absum, O.tau_for(dt))
        assert bad == 0, f"instance {i}: {bad} rows (worst {worst:g} at {at})"
        if wg is not None:
            d, at = O.max_ulp(wg[o:o + A.nrows], O.waxpy(alpha, yg[o:o + A.nrows], xi))
            assert d <= (0 if dt == np.float64 else 1), (i, d, at)


def mixed_batch(dt=np.float64):
    """Instances of every shape class, including empty rows and one long row."""
    insts = []
    m, b = I.batch_sizes(40, seed=7, mmin=64, ratio=64.0, bmax=32)
    for i in range(40):
        insts.append(I.banded(int(m[i]), int(b[i]), 0.6, seed_struct=7, seed_val=8, stream=i, dtype=dt))
    insts.append(I.zipf(3000, n=3000, kmax=3000, seed_struct=9, seed_val=10, dtype=dt))   # rows up to 3000 > LDS tile
    insts.append(I.banded(500, 3, 0.1, seed_struct=11, seed_val=12, dtype=dt))             # many empty rows
    insts.append(I.lap2d(40, dtype=dt))
    return I.batch_from_instances(insts)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("persistent,graph", [(1, 1), (1, 0), (0, 0), (0, 1)])
def test_batch_matches_oracle(spk, dev, dt, persistent, graph):
    B = mixed_batch(dt)
    x = I.batch_vector(B, seed=13, dtype=dt)
    say(f"batch dtype={dt.__name__} persistent={persistent} graph={graph}: {B.count} instances")
    arrs = _dev_batch(B, dev)
    xd = torch.from_numpy(x).to(dev)
    y = torch.full((x.size,), float("nan"), dtype=xd.dtype, device=dev)
    w = torch.full_like(y, float("nan"))
    b = spk.Batch(B, arrs, persistent=persistent, use_graph=graph)
    try:
        b.run(0.5, xd, y, w)
        torch.cuda.synchronize()
        _check_batch(B, x, y, w, 0.5, dt)
        # replays with eager work in between give the same bits every time
        first = (y.clone(), w.clone())
        for k in range(4):
            y.fill_(float("nan"))
            w.fill_(0.0)
            torch.cuda.synchronize()
            b.run(0.5, xd, y, w)
            torch.cuda.synchronize()
            assert torch.equal(y, first[0]) and torch.equal(w, first[1]), f"replay {k}"
    finally:
        b.free()


def test_instance_alone_equals_in_batch(spk, dev):
    B = mixed_batch()
    x = I.batch_vector(B, seed=14)
    arrs = _dev_batch(B, dev)
    xd = torch.from_numpy(x).to(dev)
    y = torch.empty(x.size, dtype=torch.float64, device=dev)
    w = torch.empty_like(y)
    b = spk.Batch(B, arrs)
    b.run(0.5, xd, y, w)
    torch.cuda.synchronize()
    yb, wb = y.cpu().numpy(), w.cpu().numpy()
    b.free()
    for i in (0, 7, 40, 41, 42):
        single = I.batch_from_instances([B.instance(i)])
        o, m = int(B.vec_off[i]), int(B.m[i])
        xs = x[o:o + m].copy()
        b1 = spk.Batch(single, _dev_batch(single, dev))
        ys = torch.empty(m, dtype=torch.float64, device=dev)
        ws = torch.empty_like(ys)
        b1.run(0.5, torch.from_numpy(xs).to(dev), ys, ws)
        torch.cuda.synchronize()
        assert np.array_equal(ys.cpu().numpy(), yb[o:o + m]), i
        assert np.array_equal(ws.cpu().numpy(), wb[o:o + m]), i
        b1.free()


def test_batch_tune_per_class(spk, dev):
    B = mixed_batch()
    x = I.batch_vector(B, seed=15)
    arrs = _dev_batch(B, dev)
    xd = torch.from_numpy(x).to(dev)
    y = torch.empty(x.size, dtype=torch.float64, device=dev)
    w = torch.empty_like(y)
    h = spk.Handle(0)
    b = spk.Batch(B, arrs, handle=h)
    try:
        rep = b.tune(0.5, xd, y, w, reps=3, warmup=1)
        assert rep.tried > 0 and rep.rejected == 0
        info = b.info()
        assert info["classes"] >= 3 and info["tiles"] > B.count
        y.fill_(float("nan"))
        b.run(0.5, xd, y, w)
        torch.cuda.synchronize()
        _check_batch(B, x, y, w, 0.5)
        # winners are filed per class in the plan DB, and so is the launch shape
        assert any(spk.spk_plan_get(f"batch:f64:c{c}", handle=h) is not None for c in range(8))
        lv = spk.spk_plan_get("batch:f64:launch", handle=h)
        tuned = b.config()
        assert lv is not None and (lv.block, lv.lds, lv.grid) == (tuned["block"], tuned["tile_nnz"],
                                                                   tuned["persistent"])
        # a later plan with block 0 takes the recorded shape; an explicit block does not
        b2 = spk.Batch(B, arrs, handle=h, block=0, persistent=not tuned["persistent"])
        b3 = spk.Batch(B, arrs, handle=h, block=256)
        try:
            c2, c3 = b2.config(), b3.config()
            assert (c2["block"], c2["tile_nnz"], c2["persistent"]) == (tuned["block"], tuned["tile_nnz"],
                                                                       tuned["persistent"])
            assert (c3["block"], c3["tile_nnz"]) == (256, 2048)
            y.fill_(float("nan"))
            w.fill_(float("nan"))
            b2.run(0.5, xd, y, w)
            torch.cuda.synchronize()
            _check_batch(B, x, y, w, 0.5)
        finally:
            b2.free()
            b3.free()
    finally:
        b.free()
        h.close()


def test_batch_tune_reference_is_the_plain_kernel(spk, dev):
    """spk_batch_tune judges candidates by the plain kernels' output: with the
    oracle's y supplied as the reference every candidate passes; with one row
    of that reference planted wrong, every candidate is rejected and nothing
    is recorded."""
    B = mixed_batch()
    x = I.batch_vector(B, seed=17)
    arrs = _dev_batch(B, dev)
    xd = torch.from_numpy(x).to(dev)
    y = torch.empty(x.size, dtype=torch.float64, device=dev)
    w = torch.empty_like(y)
    yr = np.concatenate([O.spmv(B.instance(i), x[int(B.vec_off[i]):int(B.vec_off[i]) + int(B.m[i])])[0]
                         for i in range(B.count)])
    h = spk.Handle(0)
    b = spk.Batch(B, arrs, handle=h)
    try:
        say("batch tune against the oracle's y")
        rep = b.tune(0.5, xd, y, w, reps=2, warmup=1, record=False, ref=yr)
        assert rep.tried > 0 and rep.rejected == 0
        wrong = yr.copy()
        row = int(B.vec_off[7]) + int(B.m[7]) // 2
        wrong[row] += 1e-6 * (1.0 + abs(wrong[row]))
        say("batch tune against a planted wrong reference")
        with pytest.raises(spk.SpkError, match="SPK_ERR_VALIDATION"):
            b.tune(0.5, xd, y, w, reps=2, warmup=1, record=True, ref=wrong)
        assert spk.spk_plan_get("batch:f64:launch", handle=h) is None
        assert all(spk.spk_plan_get(f"batch:f64:c{c}", handle=h) is None for c in range(16))
        # the batch still runs correctly after the failed search
        y.fill_(float("nan"))
        w.fill_(float("nan"))
        b.run(0.5, xd, y, w)
        torch.cuda.synchronize()
        _check_batch(B, x, y, w, 0.5)
    finally:
        b.free()
        h.close()


@pytest.mark.parametrize("persistent,graph", [(1, 1), (1, 0), (0, 1)])
def test_batch_runs_on_two_streams(spk, dev, persistent, graph):
    """One batch run on two streams at once with different x, y and w: each
    stream has its own queue counters and graph, so both results match the
    oracle, every time."""
    B = mixed_batch()
    xa = I.batch_vector(B, seed=18)
    xb = I.batch_vector(B, seed=19)
    arrs = _dev_batch(B, dev)
    xad, xbd = torch.from_numpy(xa).to(dev), torch.from_numpy(xb).to(dev)
    ya, yb = (torch.empty(xa.size, dtype=torch.float64, device=dev) for _ in range(2))
    wa, wb = torch.empty_like(ya), torch.empty_like(yb)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    b = spk.Batch(B, arrs, persistent=persistent, use_graph=graph)
    say(f"batch on two streams persistent={persistent} graph={graph}")
    try:
        for rnd in range(3):
            for t in (ya, yb, wa, wb):
                t.fill_(float("nan"))
            torch.cuda.synchronize()
            for _ in range(4):
                b.run(0.5, xad, ya, wa, stream=sa)
                b.run(0.5, xbd, yb, wb, stream=sb)
            torch.cuda.synchronize()
            _check_batch(B, xa, ya, wa, 0.5)
            _check_batch(B, xb, yb, wb, 0.5)
    finally:
        b.free()


def test_batch_spmv_only_and_empty(spk, dev):
    B = mixed_batch()
    x = I.batch_vector(B, seed=16)
    xd = torch.from_numpy(x).to(dev)
    y = torch.empty(x.size, dtype=torch.float64, device=dev)
    b = spk.Batch(B, _dev_batch(B, dev))
    b.run(0.5, xd, y, None)
    torch.cuda.synchronize()
    _check_batch(B, x, y, None, 0.5)
    b.free()
    E = I.batch_from_instances([])
    e = spk.Batch(E, (torch.zeros(1, dtype=torch.int32, device=dev), torch.zeros(1, dtype=torch.int32, device=dev),
                      torch.zeros(1, dtype=torch.float64, device=dev)))
    assert e.info()["tiles"] == 0
    e.free()


def test_batch_rejects_bad_options(spk, dev):
    B = mixed_batch()
    arrays = _dev_batch(B, dev)
    for kw in ({"persistent": 2}, {"persistent": -1}, {"block": 96}, {"tile_nnz": -5}):
        with pytest.raises(spk.SpkError, match="SPK_ERR_ARG"):
            spk.Batch(B, arrays, **kw)
    # a row_ptr that decreases inside an instance is refused at planning
    i = int(np.argmax(B.m > 2))
    rp = B.row_ptr.copy()
    o = int(B.rp_off[i])
    rp[o + 1] = rp[o + 2] + 1
    with pytest.raises(spk.SpkError, match="SPK_ERR_CSR"):
        spk.Batch(dataclasses.replace(B, row_ptr=rp), arrays)


def test_full_batched_workload(spk, dev):
    """The full 4096-instance batch, every instance against the oracle: with
    the default launch, then tuned and launched exactly as the bench times it
    (persistent and graph requested, spk_batch_tune with the bench's
    repetitions, graph replays)."""
    B = I.batch_banded(4096)
    x = I.batch_vector(B, seed=43)
    say(f"full batch: {int(B.m.sum())} rows, {int(B.nnz.sum())} nnz")
    yr, _, absum = O.batch_spmv_waxpy(B, x, 0.5)
    xd = torch.from_numpy(x).to(dev)
    y = torch.empty(x.size, dtype=torch.float64, device=dev)
    w = torch.empty_like(y)
    h = spk.Handle(0)
    b = spk.Batch(B, _dev_batch(B, dev), persistent=True, use_graph=True, handle=h)

    def check(what):
        yg, wg = y.cpu().numpy(), w.cpu().numpy()
        bad, worst, at = O.check_rows(yg, yr, absum, O.TAU_F64)
        assert bad == 0, f"{what}: {bad} rows (worst {worst:g} at {at})"
        d, at = O.max_ulp(wg, O.waxpy(0.5, yg, x))   # w from the GPU's own y: one fused rounding
        assert d == 0, (what, d, at)

    try:
        b.run(0.5, xd, y, w)
        torch.cuda.synchronize()
        check("default launch")
        b.tune(0.5, xd, y, w, reps=10, warmup=2)
        say(f"tuned launch: {b.config()}")
        y.fill_(float("nan"))
        w.fill_(float("nan"))
        for _ in range(3):
            b.run(0.5, xd, y, w)
        torch.cuda.synchronize()
        check("tuned launch")
    finally:
        b.free()
        h.close()


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_batch_x_window_mode(spk, dev, dt):
    """Every class planned to the row stream with the tile's x window staged
    in LDS (mode 1, a kernel with room for 256 entries of x per wavefront),
    and the same with compact columns (mode 3: one byte per entry, its place
    in the window): each instance matches the oracle, and the bits equal
    the plain row stream's (mode 0; only where x and the columns are read
    from differs), also for tiles whose window is too wide for the room
    (x then read from memory; a mode-3 tile becomes a mode-1 tile)."""
    B = mixed_batch(dt)
    x = I.batch_vector(B, seed=21, dtype=dt)
    arrs = _dev_batch(B, dev)
    xd = torch.from_numpy(x).to(dev)
    outs = {}
    for mode, xw in ((0, 0), (1, 256), (3, 256)):
        h = spk.Handle(0)
        for c in range(20):
            spk.spk_plan_put(f"batch:{'f64' if dt == np.float64 else 'f32'}:c{c}",
                             spk.make_variant(format=spk.SPK_FMT_ADAPTIVE, block=256, group=mode, unroll=1,
                                              streams=1, lds=2048), handle=h)
        b = spk.Batch(B, arrs, handle=h, block=256, x_window=xw)
        y = torch.full((x.size,), float("nan"), dtype=xd.dtype, device=dev)
        w = torch.full_like(y, float("nan"))
        say(f"batch x window: mode {mode} room {xw} dtype={np.dtype(dt).name}")
        try:
            assert b.config()["x_window"] == xw
            modes = b.tile_modes()
            say(f"  tiles per mode: {modes}")
            if mode == 3:
                # windows that fit take one-byte columns; the Zipf instance's
                # wider ones (3,000 columns) two-byte columns (mode 5)
                assert modes.get(3, 0) > 0 and modes.get(5, 0) > 0
            b.run(0.5, xd, y, w)
            torch.cuda.synchronize()
            _check_batch(B, x, y, w, 0.5, dt)
            outs[mode] = (y.clone(), w.clone())
        finally:
            b.free()
            h.close()
    for mode in (1, 3):
        assert torch.equal(outs[0][0], outs[mode][0]) and torch.equal(outs[0][1], outs[mode][1]), mode


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_batch_compact_columns_one_two_four_bytes(spk, dev, dt):
    """A batch planned to compact columns (mode 3) whose tiles take all three
    column widths: banded instances one byte (windows within the kernel's
    room), a 3,000-column Zipf instance two bytes (mode 5: wider windows,
    spans under 65,536), an 80,000-column Zipf instance four (mode 1: its
    tiles span more than 65,536 columns).  Every instance against the
    oracle, and the bits of the plain row stream (mode 0) on the same batch."""
    insts = [I.banded(int(m), int(b), 0.6, seed_struct=13, seed_val=14, stream=i, dtype=dt)
             for i, (m, b) in enumerate(((3000, 5), (700, 32), (12000, 1)))]
    insts.append(I.zipf(3000, n=3000, kmax=300, seed_struct=15, seed_val=16, dtype=dt))
    insts.append(I.zipf(80000, n=80000, kmax=64, seed_struct=17, seed_val=18, dtype=dt))
    B = I.batch_from_instances(insts)
    x = I.batch_vector(B, seed=23, dtype=dt)
    arrs = _dev_batch(B, dev)
    xd = torch.from_numpy(x).to(dev)
    outs = {}
    dname = "f64" if dt == np.float64 else "f32"
    for mode in (0, 3):
        h = spk.Handle(0)
        for c in range(21):
            spk.spk_plan_put(f"batch:{dname}:c{c}",
                             spk.make_variant(format=spk.SPK_FMT_ADAPTIVE, block=256, group=mode, unroll=1,
                                              streams=1, lds=2048), handle=h)
        b = spk.Batch(B, arrs, handle=h, block=256, x_window=256)
        try:
            modes = b.tile_modes()
            say(f"compact columns, mode {mode}, dtype={dname}: tiles per mode {modes}")
            if mode == 3:
                assert modes.get(3, 0) > 0 and modes.get(5, 0) > 0 and modes.get(1, 0) > 0
            y = torch.full((x.size,), float("nan"), dtype=xd.dtype, device=dev)
            w = torch.full_like(y, float("nan"))
            b.run(0.5, xd, y, w)
            torch.cuda.synchronize()
            _check_batch(B, x, y, w, 0.5, dt)
            outs[mode] = (y.clone(), w.clone())
        finally:
            b.free()
            h.close()
    assert torch.equal(outs[0][0], outs[3][0]) and torch.equal(outs[0][1], outs[3][1])


def test_batch_tune_resume(spk, dev, tmp_path):
    """spk_batch_tune journals every timed point: a search cut short after k
    new points leaves them in the DB and the batch on the plan it started
    from (still correct); a new handle resumes the search and times only
    the rest; a third search takes every point from the journal."""
    B = mixed_batch()
    x = I.batch_vector(B, seed=19)
    arrs = _dev_batch(B, dev)
    xd = torch.from_numpy(x).to(dev)
    y = torch.empty(x.size, dtype=torch.float64, device=dev)
    w = torch.empty_like(y)
    db = str(tmp_path / "plans.spkdb")

    def points():
        # every journal line is a distinct (search key, variant): nothing was timed twice
        with open(db) as f:
            pts = [json.loads(ln) for ln in f if ln.startswith('{"point": ')]
        assert len({(p["point"], tuple(p["v"])) for p in pts}) == len(pts)
        return len(pts)

    k = 5
    reps = []
    for run in range(3):
        h = spk.Handle(0, db)
        b = spk.Batch(B, arrs, handle=h)
        try:
            say(f"batch tune resume run {run}")
            if run == 0:
                with pytest.raises(spk.SpkError, match="SPK_ERR_INTERRUPTED"):
                    b.tune(0.5, xd, y, w, reps=2, warmup=1, record=False, resume=True, stop_after=k)
                assert points() == k
                assert spk.spk_plan_get("batch:f64:launch", handle=h) is None
            else:
                # no winners recorded: every search starts from the same plan
                reps.append(b.tune(0.5, xd, y, w, reps=2, warmup=1, record=False, resume=True))
            y.fill_(float("nan"))
            w.fill_(float("nan"))
            b.run(0.5, xd, y, w)
            torch.cuda.synchronize()
            _check_batch(B, x, y, w, 0.5)
        finally:
            b.free()
            h.close()
    first, second = reps
    # the resumed search takes the k points from the journal (and reuses
    # points of its own when a context repeats) and times only the rest
    assert first.resumed >= k and first.tried > 0 and first.rejected == 0
    assert points() == k + first.tried
    assert second.tried == 0 and second.resumed == first.resumed + first.tried
    assert second.best_us == first.best_us


def _diag_plus(m, extra, dt, seed):
    """m x m diagonal plus `extra` (row, col) entries, values seeded uniform."""
    rows = np.concatenate([np.arange(m), np.array([r for r, _ in extra], np.int64)])
    cols = np.concatenate([np.arange(m), np.array([c for _, c in extra], np.int64)])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(m + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    val = I.uniform(seed, 0, rows.size, dt)
    return I.CSR(m, m, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), val)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_batch_compact_columns_width_boundaries(spk, dev, dt):
    """The compact encodings at their limits: a first tile whose window is
    exactly the kernel's room of 256 columns (one-byte offsets up to 255),
    one whose columns span exactly 65,536 (two-byte offsets up to 65,535)
    and one spanning 65,537 (four-byte columns).  Each instance's first
    tile (its first 128 rows) holds the wide entries, the rest are diagonal
    tiles; against the oracle and bit-equal to the plain row stream."""
    insts = [_diag_plus(256, [(0, 255), (99, 0)], dt, 31),          # window 0..255
             _diag_plus(70000, [(0, 65535), (50, 0)], dt, 32),       # span 65,536
             _diag_plus(70000, [(0, 65536), (50, 0)], dt, 33)]       # span 65,537
    B = I.batch_from_instances(insts)
    x = I.batch_vector(B, seed=24, dtype=dt)
    arrs = _dev_batch(B, dev)
    xd = torch.from_numpy(x).to(dev)
    dname = "f64" if dt == np.float64 else "f32"
    outs = {}
    for mode in (0, 3):
        h = spk.Handle(0)
        for c in range(21):
            spk.spk_plan_put(f"batch:{dname}:c{c}",
                             spk.make_variant(format=spk.SPK_FMT_ADAPTIVE, block=256, group=mode, unroll=1,
                                              streams=1, lds=2048), handle=h)
        b = spk.Batch(B, arrs, handle=h, block=256, x_window=256)
        try:
            modes = b.tile_modes()
            say(f"compact width boundaries, mode {mode}, dtype={dname}: tiles per mode {modes}")
            if mode == 3:
                # the 256-column window and the diagonal tiles take one byte,
                # the 65,536-column span two, the 65,537-column span four
                assert modes.get(3, 0) > 0 and modes.get(5, 0) == 1 and modes.get(1, 0) == 1
            y = torch.full((x.size,), float("nan"), dtype=xd.dtype, device=dev)
            w = torch.full_like(y, float("nan"))
            b.run(0.5, xd, y, w)
            torch.cuda.synchronize()
            _check_batch(B, x, y, w, 0.5, dt)
            outs[mode] = (y.clone(), w.clone())
        finally:
            b.free()
            h.close()
    assert torch.equal(outs[0][0], outs[3][0]) and torch.equal(outs[0][1], outs[3][1])
