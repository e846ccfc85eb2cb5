"""Serving: continuous batching of SpMV+WAXPY requests gives each request the
same bits alone and in the mix, stays within its HBM budget (evicting idle
matrices), and matches the oracle."""
import numpy as np
import pytest

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I

pytestmark = pytest.mark.gpu


def pool_mats():
    out = []
    for i in range(10):
        dt = np.float64 if i % 3 else np.float32
        m = [1000, 3000, 20000, 5000, 1500][i % 5]
        if i % 2:
            out.append(I.banded(m, 1 + 3 * i, 0.6, seed_struct=60, seed_val=61, stream=i, dtype=dt))
        else:
            out.append(I.zipf(m, kmax=min(4096, m), seed_struct=62 + i, seed_val=63, dtype=dt))
    return out


def _check(A, x, y, w):
    ref, absum = O.spmv(A, x)
    dt = A.val.dtype
    assert O.check_rows(y.astype(np.float64), ref, absum, O.tau_for(dt))[0] == 0
    assert O.max_ulp(w, O.waxpy(0.5, y, x))[0] <= (0 if dt == np.float64 else 1)


@pytest.mark.parametrize("mode", [0, 1])
def test_serve_matches_oracle_and_alone(spk, dev, mode):
    pool = pool_mats()
    nreq = 200
    mats = (I.u64(70, 0, 0, nreq) % np.uint64(len(pool))).astype(int)
    xs = [I.uniform(71, i, pool[m].ncols, pool[m].val.dtype) for i, m in enumerate(mats)]
    ys = [np.empty(pool[m].nrows, pool[m].val.dtype) for m in mats]
    ws = [np.empty(pool[m].nrows, pool[m].val.dtype) for m in mats]
    say(f"serve mode={mode}: {nreq} requests over {len(pool)} matrices")
    srv = spk.Server(streams=4, max_inflight=64, max_batch=16, mode=mode, alpha=0.5)
    try:
        ids = [srv.add_matrix(A) for A in pool]
        arr = I.poisson_arrivals(nreq, 20000.0, seed=72)
        srv.replay(arr, [ids[m] for m in mats], xs, ys, ws)
        st = srv.stats()
        assert st["completed"] == nreq and st["rejected"] == 0
        lat = srv.latencies()
        assert np.all(lat > 0)
        # arrival -> admission -> completion: the two parts add up to the latency
        wait, run = srv.latency_split()
        assert wait.shape == lat.shape and np.all(wait >= 0) and np.all(run > 0)
        assert np.allclose(wait + run, lat, rtol=0, atol=1e-3)
        if mode == 0:
            assert st["batches"] < nreq   # requests were batched together
    finally:
        srv.close()
    for i in range(nreq):
        _check(pool[mats[i]], xs[i], ys[i], ws[i])
    # each request alone gives the same bits as in the mix
    solo = spk.Server(streams=1, max_inflight=1, max_batch=1, mode=mode, alpha=0.5)
    try:
        ids = [solo.add_matrix(A) for A in pool]
        for i in range(0, nreq, 17):
            y1 = np.empty_like(ys[i])
            w1 = np.empty_like(ws[i])
            solo.submit(ids[mats[i]], xs[i], y1, w1)
            solo.drain()
            assert np.array_equal(y1, ys[i]) and np.array_equal(w1, ws[i]), i
    finally:
        solo.close()


def test_serve_budget_evicts_idle_matrices(spk, dev):
    pool = [I.banded(20000, 16, 0.6, stream=i) for i in range(6)]
    one = 4 * 20001 + 12 * pool[0].nnz
    budget = int(2.5 * one)   # room for two matrices and their vectors
    srv = spk.Server(streams=2, max_inflight=8, max_batch=4, mode=0, hbm_budget=budget, alpha=0.5)
    try:
        ids = [srv.add_matrix(A) for A in pool]
        order = [0, 1, 2, 3, 0, 4, 5, 1, 2, 3] * 3
        xs = [I.uniform(80, k, 20000) for k in range(len(order))]
        ys = [np.empty(20000) for _ in order]
        ws = [np.empty(20000) for _ in order]
        for k, m in enumerate(order):
            srv.submit(ids[m], xs[k], ys[k], ws[k])
        srv.drain()
        st = srv.stats()
        say(f"budget run: {st}")
        assert st["completed"] == len(order)
        assert st["evictions"] > 0 and st["peak_bytes"] <= budget
        for k, m in enumerate(order):
            _check(pool[m], xs[k], ys[k], ws[k])
    finally:
        srv.close()


def test_serve_rejects_oversized_matrix(spk, dev):
    srv = spk.Server(hbm_budget=1 << 20)
    try:
        with pytest.raises(spk.SpkError) as e:
            srv.add_matrix(I.banded(100000, 8, 0.6))
        assert e.value.name == "SPK_ERR_BUDGET"
    finally:
        srv.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_serve_large_vectors_chunked_copies(spk, dev, mode):
    """Requests whose vectors exceed the inline-copy threshold: the host
    copies to and from the pinned staging block are cut into chunks shared by
    the copy threads (a ragged last chunk included); every result still
    matches the oracle and the same request served alone."""
    pool = [I.banded(150001, 5, 0.6, seed_struct=64, seed_val=65),                   # x: 1.2 MB of FP64
            I.zipf(90001, kmax=4096, seed_struct=66, seed_val=67, dtype=np.float32)]  # x: 360 KB of FP32
    nreq = 24
    mats = [i % 2 for i in range(nreq)]
    xs = [I.uniform(73, i, pool[m].ncols, pool[m].val.dtype) for i, m in enumerate(mats)]
    ys = [np.empty(pool[m].nrows, pool[m].val.dtype) for m in mats]
    ws = [np.empty(pool[m].nrows, pool[m].val.dtype) for m in mats]
    say(f"serve large vectors mode={mode}")
    srv = spk.Server(streams=4, max_inflight=16, max_batch=8, mode=mode, alpha=0.5)
    try:
        ids = [srv.add_matrix(A) for A in pool]
        srv.replay(I.poisson_arrivals(nreq, 5000.0, seed=74), [ids[m] for m in mats], xs, ys, ws)
        assert srv.stats()["completed"] == nreq
    finally:
        srv.close()
    for i in range(nreq):
        _check(pool[mats[i]], xs[i], ys[i], ws[i])
    solo = spk.Server(streams=1, max_inflight=1, max_batch=1, mode=mode, alpha=0.5)
    try:
        ids = [solo.add_matrix(A) for A in pool]
        for i in (0, 1, nreq - 1):
            y1, w1 = np.empty_like(ys[i]), np.empty_like(ws[i])
            solo.submit(ids[mats[i]], xs[i], y1, w1)
            solo.drain()
            assert np.array_equal(y1, ys[i]) and np.array_equal(w1, ws[i]), i
    finally:
        solo.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_serve_pinned_buffers_skip_staging(spk, dev, mode):
    """Requests whose vectors are 128 KiB or more and whose x, y, w sit in
    pinned host memory are copied by the copy engines straight between those
    buffers and the device, in launches that also hold staged requests
    (small vectors, or pageable buffers): every result matches the oracle
    and equals, bit for bit, the same request with pageable buffers."""
    import torch
    pool = [I.banded(40000, 6, 0.6, seed_struct=80, seed_val=81),                       # 320 KB vectors
            I.zipf(50000, kmax=2048, seed_struct=82, seed_val=83, dtype=np.float32),      # 200 KB
            I.banded(3000, 4, 0.6, seed_struct=84, seed_val=85),                         # 24 KB: staged
            I.banded(20000, 3, 0.6, seed_struct=86, seed_val=87, dtype=np.float32)]      # 80 KB: staged
    nreq = 48
    mats = [i % len(pool) for i in range(nreq)]

    def pinned(n, dt):
        t = torch.empty(n, dtype=torch.float64 if dt == np.float64 else torch.float32, pin_memory=True)
        return t.numpy()

    xs, ys, ws = [], [], []
    for i, m in enumerate(mats):
        A = pool[m]
        dt = A.val.dtype
        # every fourth request keeps pageable buffers
        if i % 4 == 3:
            x, y, w = np.empty(A.ncols, dt), np.empty(A.nrows, dt), np.empty(A.nrows, dt)
        else:
            x, y, w = pinned(A.ncols, dt), pinned(A.nrows, dt), pinned(A.nrows, dt)
        x[:] = I.uniform(88, i, A.ncols, dt)
        xs.append(x), ys.append(y), ws.append(w)
    expect_direct = sum(1 for i, m in enumerate(mats) if i % 4 != 3 and m in (0, 1))
    say(f"serve pinned buffers mode={mode}: {nreq} requests, {expect_direct} direct")
    srv = spk.Server(streams=4, max_inflight=32, max_batch=12, mode=mode, alpha=0.5)
    try:
        ids = [srv.add_matrix(A) for A in pool]
        srv.replay(I.poisson_arrivals(nreq, 20000.0, seed=89), [ids[m] for m in mats], xs, ys, ws)
        st = srv.stats()
        assert st["completed"] == nreq and st["rejected"] == 0
        assert st["direct"] == expect_direct
    finally:
        srv.close()
    for i in range(nreq):
        _check(pool[mats[i]], xs[i], ys[i], ws[i])
    solo = spk.Server(streams=1, max_inflight=1, max_batch=1, mode=mode, alpha=0.5)
    try:
        ids = [solo.add_matrix(A) for A in pool]
        for i in range(nreq):
            y1, w1 = np.empty_like(ys[i]), np.empty_like(ws[i])
            solo.submit(ids[mats[i]], np.array(xs[i]), y1, w1)
            solo.drain()
            assert np.array_equal(y1, ys[i]) and np.array_equal(w1, ws[i]), i
        assert solo.stats()["direct"] == 0
        # the step without w (SpMV only), pinned x and y: direct, same y
        for i in (0, 1):
            y2 = pinned(pool[mats[i]].nrows, pool[mats[i]].val.dtype)
            solo.submit(ids[mats[i]], xs[i], y2)
            solo.drain()
            assert np.array_equal(y2, ys[i]), i
        assert solo.stats()["direct"] == 2
    finally:
        solo.close()


def test_serve_rejects_bad_launch_cap(spk, dev):
    with pytest.raises(spk.SpkError) as e:
        spk.Server(max_launches=-1)
    assert e.value.name == "SPK_ERR_ARG"


def test_serve_one_launch_in_flight_batches_arrivals(spk, dev):
    """With one launch in flight, requests that arrive while it runs are
    admitted together into the next one; results still match the oracle."""
    pool = pool_mats()
    nreq = 120
    mats = (I.u64(90, 0, 0, nreq) % np.uint64(len(pool))).astype(int)
    xs = [I.uniform(91, i, pool[m].ncols, pool[m].val.dtype) for i, m in enumerate(mats)]
    ys = [np.empty(pool[m].nrows, pool[m].val.dtype) for m in mats]
    ws = [np.empty(pool[m].nrows, pool[m].val.dtype) for m in mats]
    say("serve max_launches=1")
    srv = spk.Server(streams=2, max_inflight=64, max_batch=16, mode=0, alpha=0.5, max_launches=1)
    try:
        ids = [srv.add_matrix(A) for A in pool]
        for i, m in enumerate(mats):
            srv.submit(ids[m], xs[i], ys[i], ws[i])
        srv.drain()
        st = srv.stats()
        assert st["completed"] == nreq and st["batches"] < nreq
    finally:
        srv.close()
    for i in range(nreq):
        _check(pool[mats[i]], xs[i], ys[i], ws[i])


def test_serve_classes_planned_to_compact_columns(spk, dev):
    """Serving keeps four-byte columns: a class whose recorded batch plan is
    compact columns (mode 3) is served with the same tiles run as mode 1
    (x window in LDS) -- every request against the oracle and equal bit
    for bit to the same request under a plan of mode 1."""
    pool = pool_mats()
    nreq = 60
    mats = (I.u64(73, 0, 0, nreq) % np.uint64(len(pool))).astype(int)
    xs = [I.uniform(74, i, pool[m].ncols, pool[m].val.dtype) for i, m in enumerate(mats)]
    outs = {}
    for mode in (3, 1):
        H = spk.Handle(0)
        for dn in ("f64", "f32"):
            for c in range(21):
                spk.spk_plan_put(f"batch:{dn}:c{c}",
                                 spk.make_variant(format=spk.SPK_FMT_ADAPTIVE, block=256, group=mode, unroll=1,
                                                  streams=1, lds=2048), handle=H)
        ys = [np.empty(pool[m].nrows, pool[m].val.dtype) for m in mats]
        ws = [np.empty(pool[m].nrows, pool[m].val.dtype) for m in mats]
        say(f"serve with classes planned to mode {mode}: {nreq} requests")
        srv = spk.Server(streams=2, max_inflight=32, max_batch=8, mode=0, alpha=0.5, handle=H)
        try:
            ids = [srv.add_matrix(A) for A in pool]
            srv.replay(I.poisson_arrivals(nreq, 20000.0, seed=75), [ids[m] for m in mats], xs, ys, ws)
            st = srv.stats()
            assert st["completed"] == nreq and st["rejected"] == 0
        finally:
            srv.close()
            H.close()
        outs[mode] = (ys, ws)
    for i in range(nreq):
        _check(pool[mats[i]], xs[i], outs[3][0][i], outs[3][1][i])
        assert np.array_equal(outs[3][0][i], outs[1][0][i]) and np.array_equal(outs[3][1][i], outs[1][1][i]), i
