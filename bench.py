#!/usr/bin/env python3
"""Benchmark of the autotuned SpMV + WAXPY hot path on one MI355X.

Headline (``value``): achieved HBM GB/s of one Krylov-style step
(y = A_i x_i, w_i = 0.5 y_i + x_i) over 4096 independent random banded FP64
CSR instances (row counts log-uniform in [64, 16384), half-bandwidth 1..32,
60% fill inside the band), all instances in one hipGraph-replayed launch of
the tile kernel, autotuned per shape class (the tuner picks the launch kind:
one workgroup per tile group, or a persistent grid pulling tiles from
per-XCD queues; and per class the tile kernel, compact one-byte columns
among them).  Bytes are the algorithmic ones of the CSR statement: every
array once (values, 4-byte column indices, row pointers, x, y, w), no
re-reads, no padding; the bytes the tuned plan's own form moves (fewer,
with compact columns) are reported beside them (``roofline.form_*``).

Also reported on the same JSON line: the plain (untuned) kernels on the same
batch (two launches over the batch as one block-diagonal matrix, and one
launch pair per instance), the vector sweep (WAXPY/AXPY/dot at n = 2^27, FP64 and FP32,
tuned vs plain), the large single SpMVs (3-D Laplacian 128^3 and a 1M-row
Zipf matrix, tuned vs the better plain kernel, cold cache), the 2-D Laplacian
step, open-loop serving of 20,000 requests over 256 matrices of 1e3..1e6
rows at four offered loads (p50/p99 against a FIFO server), the STREAM copy bandwidth, the
roofline of the dominant kernel and the oracle timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true", help="headline only")
    ap.add_argument("--extras", default="all",
                    help="comma list of extra legs (vector_sweep, spmv_large, krylov_step_lap2d, "
                         "cg_lap3d_128, serving, host_simd; zipf_forms for counter runs) or 'all'")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-instance baseline")
    ap.add_argument("--verbose", action="store_true", help="print every tuning candidate")
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--serve-requests", type=int, default=20000, help="measured requests per offered load")
    ap.add_argument("--serve-warmup", type=int, default=1000, help="warm-up requests before them")
    ap.add_argument("--serve-pool", type=int, default=256, help="matrices in the serving pool")
    return ap.parse_args()


EXTRA_LEGS = ("vector_sweep", "spmv_large", "krylov_step_lap2d", "cg_lap3d_128", "serving", "host_simd")


def main():
    args = parse()
    if args.extras != "all":
        bad = [e for e in args.extras.split(",") if e.strip() and e.strip() not in EXTRA_LEGS + ("zipf_forms",)]
        if bad:
            sys.exit(f"unknown extra leg(s) {bad}; known: {', '.join(EXTRA_LEGS + ('zipf_forms',))}")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    lib = os.path.join(ROOT, "paper_1309_1894_amd", "libspk.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()

    import numpy as np
    import torch

    from paper_1309_1894_amd import inputs as I
    from paper_1309_1894_amd import spk

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    h = spk.default_handle(0)
    ncu, name = h.info()
    log(f"device: {name}, {ncu} CUs")
    stream = torch.cuda.current_stream()
    out = {}

    # ------------------------------------------------ the batched workload
    t0 = time.time()
    B = I.batch_banded(args.instances, fill=0.6, seed_struct=41, seed_val=42)
    x = I.batch_vector(B, seed=43)
    log(f"batch: {B.count} instances, {int(B.m.sum())} rows, {int(B.nnz.sum())} nnz "
        f"(generated in {time.time() - t0:.1f}s)")
    d_rp = torch.from_numpy(B.row_ptr).to(dev)
    d_ci = torch.from_numpy(B.col_idx).to(dev)
    d_val = torch.from_numpy(B.val).to(dev)
    d_x = torch.from_numpy(x).to(dev)
    nv = int(B.m.sum())
    d_y = torch.empty(nv, dtype=torch.float64, device=dev)
    d_w = torch.empty(nv, dtype=torch.float64, device=dev)
    batch = spk.Batch(B, (d_rp, d_ci, d_val), persistent=True, use_graph=True)
    info = batch.info()
    step_bytes = info["bytes"]
    alpha = 0.5

    # tuning (Section 2's search, per shape class), not timed
    t0 = time.time()
    rep = batch.tune(alpha, d_x, d_y, d_w, reps=10, warmup=2, verbose=args.verbose)
    info = batch.info()
    log(f"batch tune: {rep.tried} candidates timed, {rep.rejected} rejected, {info['classes']} classes, "
        f"{info['tiles']} tiles ({time.time() - t0:.1f}s)")

    # the bytes the tuned plan's own form moves: tiles with compact columns
    # (mode 3) read one byte per entry for its column instead of four
    modes = batch.tile_modes(entries=True)
    form_bytes = step_bytes - 3 * modes.get(3, (0, 0))[1]
    log(f"batched tiles per mode (tiles, entries): {modes}; form bytes {form_bytes} of {step_bytes} algorithmic")
    # the same plan with 4-byte columns, timed before the headline so that
    # the headline's steps are the last launches of its kernel
    four_byte = tuned_four_byte_columns(spk, B, (d_rp, d_ci, d_val), d_x, d_y, d_w, alpha, stream, torch, np,
                                        step_bytes, args.steps, args.warmup)
    log(f"batched tuned with 4-byte columns only: {four_byte}")

    # timed region: exactly K steps, synchronised on both sides
    for _ in range(args.warmup):
        batch.run(alpha, d_x, d_y, d_w)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        batch.run(alpha, d_x, d_y, d_w)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    per_launch_ms = [a.elapsed_time(b) for a, b in ev]
    kern_ms = float(np.mean(per_launch_ms))
    ms_per_step = elapsed * 1e3 / args.steps
    value = step_bytes / (ms_per_step * 1e-3) / 1e9
    achieved = step_bytes / (kern_ms * 1e-3) / 1e9
    log(f"batched tuned: {ms_per_step:.3f} ms/step, {value:.1f} GB/s (kernel {kern_ms:.3f} ms, {achieved:.1f} GB/s)")

    # plain baseline on the same batch: per-instance plain kernels, unfused
    cfg = batch.config()
    kname = (f"k_batch_{'persistent' if cfg['persistent'] else 'grid'}<double,{cfg['block']},{cfg['tile_nnz']},"
             f"{cfg['x_window']}>")
    if args.no_plain:
        plain = {"ms": None, "skipped": True}
        plain_bd = {"ms": None, "skipped": True}
    else:
        plain_bd = plain_blockdiag(spk, I, B, d_val, d_x, d_y, d_w, alpha, stream, torch, step_bytes)
        log(f"batched plain, block-diagonal: {plain_bd}")
        plain = plain_batch(spk, B, d_x, d_y, d_w, alpha, stream, torch)
        plain["gbs_of_tuned_bytes"] = round(step_bytes / (plain["ms"] * 1e-3) / 1e9, 1)
    log(f"batched plain, per-instance launches: {plain}")
    out["batched"] = {"tuned_gbs": round(value, 1), "tuned_ms": round(ms_per_step, 4), "launch": cfg,
                      "kernel_ms_p10_p50_p90": [round(float(np.percentile(per_launch_ms, q)), 4)
                                                for q in (10, 50, 90)],
                      "plain_blockdiag": plain_bd,
                      "speedup_vs_plain_blockdiag": (round(plain_bd["ms"] / ms_per_step, 2)
                                                     if plain_bd["ms"] else None),
                      "plain_per_instance_launches": plain,
                      "speedup_vs_plain_per_instance_launches": (round(plain["ms"] / ms_per_step, 2)
                                                                 if plain["ms"] else None),
                      "instances": B.count, "rows": nv, "nnz": int(B.nnz.sum()), "bytes_per_step": step_bytes,
                      "form_bytes_per_step": form_bytes,
                      "tile_modes": {str(m): {"tiles": t, "entries": e} for m, (t, e) in modes.items()},
                      "tuned_4byte_columns": four_byte,
                      "tiles": info["tiles"], "classes": info["classes"]}

    # STREAM copy: measured bandwidth ceiling (and counter calibration)
    out["stream"] = stream_copy(spk, torch, dev, stream)

    if not args.no_extras:
        del d_y, d_w
        legs = {"vector_sweep": lambda: vector_sweep(spk, torch, I, dev),
                "spmv_large": lambda: spmv_large(spk, torch, I, dev),
                "krylov_step_lap2d": lambda: lap2d_step(spk, torch, I, dev),
                "cg_lap3d_128": lambda: cg_lap3d(spk, torch, I, dev),
                "serving": lambda: serving(spk, I, args.serve_requests, args.serve_warmup, args.serve_pool),
                "host_simd": lambda: host_simd(),
                "zipf_forms": lambda: zipf_forms(spk, torch, I, dev)}
        # zipf_forms is a counter-run aid, named explicitly only
        want = [k for k in legs if k in EXTRA_LEGS] if args.extras == "all" else \
            [e.strip() for e in args.extras.split(",") if e.strip()]
        for name in want:
            out[name] = legs[name]()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(B, x, alpha, step_bytes)
        out["cpu_oracle_single_thread"] = cpu_single_thread(B, x, alpha, step_bytes)
        out["cpu_oracle_beside_legs"] = cpu_beside_legs(I, [k for k in out if k in EXTRA_LEGS])

    traffic = load_traffic(kname, step_bytes)
    result = {
        "metric": "achieved HBM GB/s (% of roofline) SpMV+WAXPY, autotuned vs plain; serving p50/p99",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded SplitMix64 generators)",
        "config": {"workload": f"batched SpMV+WAXPY step: {B.count} random banded FP64 CSR instances, "
                               f"rows log-uniform [64,16384), half-band 1..32, fill 0.6, alpha 0.5; "
                               f"one hipGraph-replayed launch of the tile kernel, tiles tuned per size class",
                   "instances": B.count, "rows": nv, "nnz": int(B.nnz.sum()), "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "kernel": kname, "bytes_per_launch": step_bytes,
                     "kernel_ms": round(kern_ms, 4),
                     "form_bytes_per_launch": form_bytes,
                     "form_gbs": round(form_bytes / (kern_ms * 1e-3) / 1e9, 1),
                     "form_frac": round(form_bytes / (kern_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
        "cpu_baseline": cpu,
        "extras": out,
    }
    print(json.dumps(result), flush=True)


def tuned_four_byte_columns(spk, B, arrays, d_x, d_y, d_w, alpha, stream, torch, np, step_bytes, steps, warmup):
    """The tuned plan with every compact-column class (mode 3) run as mode
    1 instead -- the same tiles and x windows, 4-byte columns -- timed like
    the headline: graph replays, HIP events on the launch stream."""
    h = spk.Handle(0)
    changed = 0
    for c in range(21):
        key = f"batch:f64:c{c}"
        v = spk.spk_plan_get(key)
        if v is None:
            continue
        if v.group == 3:
            v.group = 1
            changed += 1
        spk.spk_plan_put(key, v, handle=h)
    lv = spk.spk_plan_get("batch:f64:launch")
    if lv is not None:
        spk.spk_plan_put("batch:f64:launch", lv, handle=h)
    b = spk.Batch(B, arrays, handle=h, block=0)
    try:
        for _ in range(warmup):
            b.run(alpha, d_x, d_y, d_w)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            b.run(alpha, d_x, d_y, d_w)
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        kms = float(np.mean([a.elapsed_time(e) for a, e in ev]))
        return {"classes_moved_to_mode_1": changed, "ms": round(ms, 4), "gbs": round(step_bytes / (ms * 1e-3) / 1e9, 1),
                "kernel_ms": round(kms, 4), "kernel_gbs": round(step_bytes / (kms * 1e-3) / 1e9, 1),
                "tile_modes": {str(m): t for m, t in b.tile_modes().items()}}
    finally:
        b.free()
        h.close()


def plain_blockdiag(spk, I, B, d_val, d_x, d_y, d_w, alpha, stream, torch, step_bytes, reps=10):
    """The plain (untuned) kernels over the whole batch in two launches: the
    batch as one block-diagonal CSR matrix (columns shifted per instance),
    the better of the two plain SpMV kernels (lane per row, wavefront per
    row; 256 threads), then the plain WAXPY over all rows.  GB/s on the
    tuned step's algorithmic bytes and on the unfused pair's own bytes
    (the WAXPY re-reads y and x)."""
    import numpy as np
    D = I.block_diagonal(B)
    M = spk.Matrix(D, validate=False)
    del D
    nv = int(B.m.sum())
    own = int(B.nnz.sum()) * 12 + 4 * (nv + 1) + 16 * nv + 24 * nv
    wv = spk.spk_plain_variant(spk.SPK_OP_WAXPY, 0)
    pw = spk.problem(spk.SPK_OP_WAXPY, x=d_y, y=d_x, w=d_w, alpha=alpha)
    best = None
    try:
        for which in (0, 1):
            v = spk.spk_plain_variant(spk.SPK_OP_SPMV, which)
            ps = spk.problem(spk.SPK_OP_SPMV, A=M, x=d_x, y=d_y)

            def step():
                spk.spk_run(ps, v)
                spk.spk_run(pw, wv)

            step()
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for a, b in ev:
                a.record(stream)
                step()
                b.record(stream)
            torch.cuda.synchronize()
            ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
            rec = {"spmv_kernel": "lane-per-row" if which == 0 else "wavefront-per-row", "ms": round(ms, 4),
                   "launches_per_step": 2, "gbs_of_tuned_bytes": round(step_bytes / (ms * 1e-3) / 1e9, 1),
                   "gbs_own_bytes": round(own / (ms * 1e-3) / 1e9, 1)}
            if best is None or ms < best["ms"]:
                best = rec
    finally:
        M.release()
        torch.cuda.empty_cache()
    return best


def plain_batch(spk, B, d_x, d_y, d_w, alpha, stream, torch):
    """Every instance with the fixed plain kernels, one launch each: SpMV
    (lane per row, or wavefront per row, 256 threads) then WAXPY (one element
    per thread).  Reports the better of the two SpMV kernels."""
    import ctypes as C
    h = spk.default_handle()
    L = spk.lib
    s = stream.cuda_stream
    mats = [spk.Matrix(B.instance(i), validate=False) for i in range(B.count)]
    wv = spk.spk_plain_variant(spk.SPK_OP_WAXPY, 0)
    nbytes = 0
    for i in range(B.count):
        m, nz = int(B.m[i]), int(B.nnz[i])
        nbytes += nz * 12 + 4 * (m + 1) + 16 * m + 24 * m   # SpMV, then WAXPY re-reads y and x
    best = None
    try:
        for which in (0, 1):
            v = spk.spk_plain_variant(spk.SPK_OP_SPMV, which)
            probs = []
            for i, M in enumerate(mats):
                o, m = int(B.vec_off[i]), int(B.m[i])
                ps = spk.spk_problem(spk.SPK_OP_SPMV, 1, 0, 0.0, M.ptr, d_x.data_ptr() + 8 * o,
                                     d_y.data_ptr() + 8 * o, None, None)
                pw = spk.spk_problem(spk.SPK_OP_WAXPY, 1, m, alpha, None, d_y.data_ptr() + 8 * o,
                                     d_x.data_ptr() + 8 * o, d_w.data_ptr() + 8 * o, None)
                probs.append((ps, pw))

            def step():
                for ps, pw in probs:
                    st = L.spk_run(h.ptr, C.byref(ps), C.byref(v), s)
                    if st:
                        raise spk.SpkError(st, "plain spmv")
                    st = L.spk_run(h.ptr, C.byref(pw), C.byref(wv), s)
                    if st:
                        raise spk.SpkError(st, "plain waxpy")

            step()
            torch.cuda.synchronize()
            reps = 3
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                step()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            rec = {"spmv_kernel": "lane-per-row" if which == 0 else "wavefront-per-row", "ms": round(ms, 3),
                   "launches_per_step": 2 * B.count, "gbs_of_tuned_bytes": None,
                   "gbs_own_bytes": round(nbytes / (ms * 1e-3) / 1e9, 1)}
            if best is None or ms < best["ms"]:
                best = rec
    finally:
        for M in mats:
            M.release()
    return best


def stream_copy(spk, torch, dev, stream):
    """STREAM copy (c = a) and triad (c = a + 3b) on 2^28 doubles per array."""
    n = 1 << 28  # 2 GiB per array
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.ones(n, dtype=torch.float64, device=dev)
    c = torch.empty_like(a)
    out = {}
    for kind, name, nbytes in ((0, "copy_gbs", 2 * 8 * n), (1, "triad_gbs", 3 * 8 * n)):
        for _ in range(3):
            spk.spk_stream_probe(kind, a, b, c)
        torch.cuda.synchronize()
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            spk.spk_stream_probe(kind, a, b, c)
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = round(nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9, 1)
    del a, b, c
    return out


def vector_sweep(spk, torch, I, dev):
    """WAXPY/AXPY/dot, FP64 and FP32, n in {1e4, 1e5, 1e6, 1e7, 2^27}:
    tuned vs plain.  Up to 1e7 every timed rep starts with a flushed
    last-level cache (those sizes fit in it); 2^27 is HBM-sized anyway."""
    import numpy as np
    res = {}
    for n in (10 ** 4, 10 ** 5, 10 ** 6, 10 ** 7, 1 << 27):
        key = "2^27" if n == 1 << 27 else f"1e{int(round(np.log10(n)))}"
        for dt, ndt in ((1, "f64"), (0, "f32")):
            npdt = np.float64 if dt == 1 else np.float32
            x = torch.from_numpy(I.uniform(21, 0, n, npdt)).to(dev)
            y = torch.from_numpy(I.uniform(22, 0, n, npdt)).to(dev)
            w = torch.empty_like(x)
            d = torch.empty(1, dtype=torch.float64, device=dev)
            s = x.element_size()
            for op, nm, nbytes in ((spk.SPK_OP_WAXPY, "waxpy", 3 * n * s), (spk.SPK_OP_AXPY, "axpy", 3 * n * s),
                                   (spk.SPK_OP_DOT, "dot", 2 * n * s)):
                p = spk.problem(op, x=x, y=y, w=w if op == spk.SPK_OP_WAXPY else None,
                                d_result=d if op == spk.SPK_OP_DOT else None, alpha=1.5)
                rep = spk.spk_tune(p, reps=5, warmup=1, flush=n <= 10 ** 7, record=True)
                res[f"{nm}_{ndt}_n{key}"] = {
                    "tuned_gbs": round(nbytes / (rep.best_us * 1e-6) / 1e9, 1),
                    "plain_gbs": round(nbytes / (rep.plain_us * 1e-6) / 1e9, 1),
                    "tuned_us": round(rep.best_us, 2), "plain_us": round(rep.plain_us, 2),
                    "best": [rep.best.block, rep.best.vec, rep.best.unroll, rep.best.grid],
                    "variants_timed": rep.tried, "rejected": rep.rejected}
                if n == 1 << 27:
                    log(f"sweep {nm} {ndt} n={key}: {res[f'{nm}_{ndt}_n{key}']}")
            del x, y, w
    res["best_fields"] = "block, vec, unroll, grid (0 = one pass, else workgroups per CU)"
    torch.cuda.empty_cache()
    return res


def spmv_large(spk, torch, I, dev):
    """Single large SpMVs, cold last-level cache: tuned vs the better plain kernel.
    Each candidate is validated against the plain kernel's output (the
    library's own reference run) before it is timed."""
    import numpy as np
    res = {}
    for name, A, seed in (("lap3d_128", I.lap3d(128), 31), ("zipf_1M", I.zipf(1000000), 34)):
        M = spk.Matrix(A)
        x = I.uniform(seed, 0, A.ncols)
        xd = torch.from_numpy(x).to(dev)
        y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
        # CSR formats only: the CSR byte count is the one these GB/s use
        rep = spk.spk_tune(spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y), reps=10, warmup=2, flush=True,
                           record=True, formats=spk.CSR_FORMATS)
        nbytes = A.nnz * 12 + 4 * (A.nrows + 1) + 8 * A.ncols + 8 * A.nrows
        res[name] = {"tuned_gbs": round(nbytes / (rep.best_us * 1e-6) / 1e9, 1),
                     "plain_gbs": round(nbytes / (rep.plain_us * 1e-6) / 1e9, 1),
                     "tuned_us": round(rep.best_us, 2), "plain_us": round(rep.plain_us, 2),
                     "best": rep.best.as_dict(), "variants_timed": rep.tried, "pruned": rep.pruned,
                     "rejected": rep.rejected, "bytes": nbytes}
        res[name]["structured"] = structured_spmv(spk, M, xd, y, rep.best_us)
        res[name]["best_us_per_format"] = per_format(spk, torch, M, xd, y)
        log(f"spmv {name}: {res[name]}")
        M.release()
    return res


def zipf_forms(spk, torch, I, dev, reps=5):
    """The 1M-row Zipf SpMV in three of its forms, for counter runs: one
    fixed variant of each (the tuner's usual pick for this matrix, fixed so
    that every profiling run launches the same kernels), `reps` cold-cache
    runs each, form after form -- row-block tiles in one pass
    (k_spmv_adaptive), column blocks (one k_spmv_adaptive pass per block,
    then k_colblock_sum), x windows in LDS (k_xwin, then k_xwin_sum) --
    timed with HIP events on the stream they run on.  These runs are the
    last dispatches of those kernels in the process."""
    import numpy as np
    A = I.zipf(1000000)
    M = spk.Matrix(A)
    xd = torch.from_numpy(I.uniform(34, 0, A.ncols)).to(dev)
    y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
    p = spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y)
    forms = (("csr_lds_tiles", spk.make_variant(format=spk.SPK_FMT_ADAPTIVE, block=512, group=256, unroll=1,
                                                streams=1, lds=256)),
             ("csr_column_blocks", spk.make_variant(format=spk.SPK_FMT_COLBLOCK, block=128, group=2, unroll=1,
                                                    streams=1, lds=256)),
             ("csr_x_windows_in_lds", spk.make_variant(format=spk.SPK_FMT_XWIN, block=768, group=128, unroll=1,
                                                       grid=1, streams=1, lds=256)))
    nbytes = A.nnz * 12 + 4 * (A.nrows + 1) + 8 * A.ncols + 8 * A.nrows
    res = {"bytes": nbytes, "nnz": A.nnz, "rows": A.nrows, "reps": reps}
    ref, absum = None, None
    s = torch.cuda.current_stream()
    for name, v in forms:
        spk.spk_run(p, v)   # first use: plans the form's layout on the device
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            spk.spk_flush_cache()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            spk.spk_run(p, v)
            e1.record(s)
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1) * 1e3)
        yh = y.cpu().numpy()
        if ref is None:   # every form gives the same y up to rounding
            ref = yh
        res[name] = {"variant": v.as_dict(), "us_median": round(float(np.median(t)), 2),
                     "gbs": round(nbytes / (float(np.median(t)) * 1e-6) / 1e9, 1),
                     "max_rel_diff_vs_first_form": float(np.max(np.abs(yh - ref) / (np.abs(ref) + 1e-300)))}
        log(f"zipf form {name}: {res[name]}")
    M.release()
    return res


def structured_spmv(spk, M, xd, y, csr_tuned_us, op=None, w=None):
    """The tuner restricted to the structured formats (DIA, matrix-free
    stencil) when the matrix admits one; GB/s on that format's own
    algorithmic bytes (fewer than CSR's), speed-up on time vs the tuned CSR
    form.  Not recorded as the class plan."""
    mask = M.formats() & ((1 << spk.SPK_FMT_DIA) | (1 << spk.SPK_FMT_STENCIL))
    if not mask:
        return None
    op = spk.SPK_OP_SPMV if op is None else op
    fused = op == spk.SPK_OP_SPMV_WAXPY
    p = spk.problem(op, A=M, x=xd, y=y, w=w, alpha=0.5 if fused else 0.0)
    rep = spk.spk_tune(p, reps=10, warmup=2, flush=not fused, record=False, formats=mask)
    own = M.format_bytes(rep.best.format, fused)
    names = {spk.SPK_FMT_DIA: "dia", spk.SPK_FMT_STENCIL: "stencil"}
    return {"format": names[rep.best.format], "block": rep.best.block, "rows_per_lane": rep.best.unroll,
            "lds_staged": bool(rep.best.format == spk.SPK_FMT_STENCIL and rep.best.lds), "us": round(rep.best_us, 2),
            "bytes": own, "gbs_own_bytes": round(own / (rep.best_us * 1e-6) / 1e9, 1),
            "speedup_vs_csr_tuned": round(csr_tuned_us / rep.best_us, 2), "variants_timed": rep.tried}


def per_format(spk, torch, M, xd, y, reps=5):
    """Best cold-cache time (us) per storage format: the tuner's search
    (validation, then timing) restricted to one format at a time."""
    names = {spk.SPK_FMT_SCALAR: "csr_scalar", spk.SPK_FMT_VECTOR: "csr_vector", spk.SPK_FMT_SELL: "sliced_ell",
             spk.SPK_FMT_ADAPTIVE: "csr_lds_tiles", spk.SPK_FMT_COLBLOCK: "csr_column_blocks",
             spk.SPK_FMT_XWIN: "csr_x_windows_in_lds", spk.SPK_FMT_DIA: "dia",
             spk.SPK_FMT_STENCIL: "stencil"}
    best = {}
    p = spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y)
    for fmt, name in names.items():
        if fmt in (spk.SPK_FMT_DIA, spk.SPK_FMT_STENCIL, spk.SPK_FMT_COLBLOCK, spk.SPK_FMT_XWIN) and \
                not M.formats() & (1 << fmt):
            continue
        try:
            rep = spk.spk_tune(p, reps=reps, warmup=1, flush=True, record=False, formats=1 << fmt)
        except spk.SpkError:
            continue   # every variant of the format pruned (sliced ELL whose padding would exceed 2x)
        best[name] = round(rep.best_us, 2)
        if fmt == spk.SPK_FMT_STENCIL:
            best["stencil_lds_staged"] = bool(rep.best.lds)
    return best


def lap2d_step(spk, torch, I, dev):
    """2-D Laplacian 256^2 Krylov-style step (cache-resident, launch-bound)."""
    A = I.lap2d(256)
    M = spk.Matrix(A)
    x = I.uniform(11, 0, A.nrows)
    xd = torch.from_numpy(x).to(dev)
    y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
    w = torch.empty_like(y)
    rep = spk.spk_tune(spk.problem(spk.SPK_OP_SPMV_WAXPY, A=M, x=xd, y=y, w=w, alpha=0.5), reps=20, warmup=3,
                       formats=spk.CSR_FORMATS)
    st = structured_spmv(spk, M, xd, y, rep.best_us, spk.SPK_OP_SPMV_WAXPY, w)
    graph = graph_steps(spk, torch, M, xd, y, w)
    M.release()
    return {"tuned_us": round(rep.best_us, 2), "plain_us": round(rep.plain_us, 2), "best": rep.best.as_dict(),
            "variants_timed": rep.tried, "rejected": rep.rejected, "structured": st, "hip_graph": graph}


def graph_steps(spk, torch, M, xd, y, w, steps=1000, reps=5):
    """The tuned fused step (its recorded plan) captured `steps` times in one
    HIP graph and replayed: microseconds per step with the launch cost
    amortised, and whether a replay reproduces the eager result bit for bit."""
    import numpy as np
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        spk.spk_spmv_waxpy(M, 0.5, xd, y, w)    # anything built on first use is built before the capture
    torch.cuda.synchronize()
    y_ref, w_ref = y.clone(), w.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cs):
        for _ in range(steps):
            spk.spk_spmv_waxpy(M, 0.5, xd, y, w)
    y.fill_(float("nan"))
    w.fill_(float("nan"))
    g.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(y, y_ref) and torch.equal(w, w_ref))
    st = torch.cuda.current_stream()
    t = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        g.replay()
        e1.record(st)
        torch.cuda.synchronize()
        t.append(e0.elapsed_time(e1) * 1e3 / steps)
    del g
    return {"steps_per_graph": steps, "us_per_step": round(float(np.median(t)), 3), "replay_equals_eager": same}


def cg_lap3d(spk, torch, I, dev, iters=100):
    """Conjugate gradients on the 7-point Laplacian 128^3 (2,097,152 rows):
    the fused solve (three launches per iteration, scalars on the device,
    SpMV tile shape tuned by spk_cg_tune) vs. the same iteration composed
    from the library's separately tuned SpMV, dot, AXPY and WAXPY calls with
    the step sizes read back to the host.  Per-iteration time = (solve of
    `iters` - solve of 0) / iters; bytes per iteration are the algorithmic
    traffic of the fused schedule: the matrix (12 nnz + 4 (n+1)), p read and
    q written by the SpMV (16 n), r and q read and r written (24 n), x, r, p
    read and x, p written (40 n).  The matrix-free stencil form of the same
    solve is reported separately (80 n bytes per iteration: no matrix)."""
    import numpy as np
    A = I.lap3d(128)
    n, nnz = A.nrows, A.nnz
    M = spk.Matrix(A)
    b = torch.from_numpy(I.uniform(61, 0, n)).to(dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    hist = torch.empty(iters + 1, dtype=torch.float64, device=dev)
    # Section 2's search over the CSR tile shape of the solve (not timed)
    tune = spk.spk_cg_tune(M, b, 10, reps=5, warmup=1, formats=1 << spk.SPK_FMT_ADAPTIVE)

    def solve(k):
        x.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        spk.spk_cg(M, b, x, k, hist=hist[:k + 1])
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3

    solve(10)
    t_full = min(solve(iters) for _ in range(3))
    t_zero = min(solve(0) for _ in range(3))
    fused_us = (t_full - t_zero) / iters
    rr = hist.cpu().numpy()

    # the same iteration from separate library calls, host-synchronised
    r = torch.empty_like(x)
    p = torch.empty_like(x)
    q = torch.empty_like(x)
    d = torch.empty(1, dtype=torch.float64, device=dev)

    def unfused(k):
        x.zero_()
        spk.spk_spmv_mat(M, x, q)
        spk.spk_waxpy(-1.0, q, b, r)
        p.copy_(r)
        rr_ = spk.spk_dot(r, r, d).item()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            spk.spk_spmv_mat(M, p, q)
            pq = spk.spk_dot(p, q, d).item()
            a = rr_ / pq if pq != 0.0 else 0.0
            spk.spk_axpy(a, p, x)
            spk.spk_axpy(-a, q, r)
            rn = spk.spk_dot(r, r, d).item()
            beta = rn / rr_ if rr_ != 0.0 else 0.0
            spk.spk_waxpy(beta, p, r, p)
            rr_ = rn
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e6 / k, rr_

    unfused(5)
    unfused_us, rr_unfused = min(unfused(50) for _ in range(2))
    fused_bytes = 12 * nnz + 4 * (n + 1) + 80 * n

    # the matrix-free SpMV+dot (the matrix is a 7-point stencil): the tuner
    # restricted to it, then the same timing; the matrix bytes drop out
    st = None
    if M.formats() & (1 << spk.SPK_FMT_STENCIL):
        st_tune = spk.spk_cg_tune(M, b, 10, reps=5, warmup=1, formats=1 << spk.SPK_FMT_STENCIL)
        solve(10)
        st_us = (min(solve(iters) for _ in range(3)) - min(solve(0) for _ in range(3))) / iters
        st_bytes = 80 * n   # p read, q written (16 n) + the residual (24 n) and direction (40 n) passes
        st = {"us_per_iter": round(st_us, 2), "bytes_per_iter": st_bytes,
              "gbs_own_bytes": round(st_bytes / (st_us * 1e-6) / 1e9, 1),
              "speedup_vs_csr_tiles": round(fused_us / st_us, 2), "block": st_tune.best.block,
              "rows_per_lane": st_tune.best.unroll, "lds_staged": bool(st_tune.best.lds),
              "rr_ratio_end": float(hist.cpu().numpy()[-1] / hist.cpu().numpy()[0])}
    res = {"rows": n, "nnz": nnz, "iters": iters,
           "fused_us_per_iter": round(fused_us, 2), "unfused_us_per_iter": round(unfused_us, 2),
           "speedup": round(unfused_us / fused_us, 2),
           "bytes_per_iter": fused_bytes,
           "fused_gbs": round(fused_bytes / (fused_us * 1e-6) / 1e9, 1),
           "unfused_gbs_same_bytes": round(fused_bytes / (unfused_us * 1e-6) / 1e9, 1),
           "rr_ratio_end": float(rr[-1] / rr[0]),
           "tuned_shape": {"block": tune.best.block, "entries": tune.best.lds,
                           "two_byte_columns": tune.best.vec == 2},
           "tune_10_iters_us": {"tuned": round(tune.best_us, 1), "default_shape": round(tune.plain_us, 1),
                                "shapes_timed": tune.tried, "rejected": tune.rejected},
           "matrix_free_stencil": st}
    log(f"cg lap3d_128: {res}")
    M.release()
    return res


def host_simd():
    """The paper's own experiment (Figure 1) on this machine's host CPU: the
    annotated vector update expanded into compiler-specific SIMD pragma
    variants (gcc and clang; SSE4.2, AVX2, AVX-512 as the CPU allows;
    unroll, restrict), validated against and timed with the pragma-free
    -O3 baseline, one thread, FP64, a = 1.5."""
    from paper_1309_1894_amd import host_simd as H
    t0 = time.time()
    rep = H.tune(sizes=(10**4, 10**5, 10**6, 10**7), reps=3, target_s=0.005, confirm=5, log=log)
    rep["seconds"] = round(time.time() - t0, 1)
    for v in rep["sizes"].values():
        for k in ("baseline_s", "best_s"):
            v[k] = float(f"{v[k]:.4g}")
        for k in ("speedup", "time_saved_pct", "best_gbs", "baseline_gbs"):
            v[k] = round(v[k], 2)
    return rep


def serving(spk, I, nreq, warm, npool):
    """Open-loop Poisson serving of SpMV+WAXPY requests over a pool of banded
    and Zipf matrices (rows log-uniform in [1e3, 1e6], 70% FP64 / 30% FP32):
    continuous batching vs a FIFO server that runs one request at a time with
    the plain unbatched kernels, both with a 200 GB HBM budget and on the same
    arrival traces at four offered loads (70% of the FIFO server's and
    50/70/90% of the batching server's closed-loop saturation rate).  Each
    load replays warm + nreq requests and reports the last nreq: latency
    p50/p99 (arrival to results in the caller's buffers), its split into the
    wait for admission and the run after it, latency by row-count decade,
    where the scheduler's time goes per launch, and the device and host-link
    rates.  Requests for one pool matrix share its x and its y/w buffers
    (every such request writes the same bytes); the buffers are pinned host
    memory, as a serving front end that owns them would allocate them, and
    one load is replayed from pageable buffers too."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    sizes = I.log_uniform_int(1e3, 1e6, 51, 0, npool)
    kinds = I.u64(51, 1, 0, npool) % np.uint64(2)
    fp64 = I.unit_from_u64(I.u64(51, 2, 0, npool)) < 0.7

    def gen(i):
        m = int(sizes[i])
        dt = np.float64 if fp64[i] else np.float32
        if kinds[i] == 0:
            b = 1 + int(I.u64(51, 3, i, 1)[0] % np.uint64(32))
            return I.banded(m, b, 0.6, seed_struct=53, seed_val=54, stream=i, dtype=dt)
        return I.zipf(m, kmax=min(4096, m), seed_struct=55 + i, seed_val=56, dtype=dt)

    t0 = time.perf_counter()
    threads = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(threads) as ex:
        pool = list(ex.map(gen, range(npool)))
    gen_s = time.perf_counter() - t0
    log(f"serving: pool of {npool} matrices generated in {gen_s:.1f} s on {threads} threads")
    import torch

    def pinned(n, dt):   # a serving front end owns its request buffers: pinned host memory
        return torch.empty(n, dtype=torch.float64 if dt == np.float64 else torch.float32, pin_memory=True).numpy()

    xs_pool, ys_pool, ws_pool = [], [], []
    for i, A in enumerate(pool):
        x = pinned(A.ncols, A.val.dtype)
        x[:] = I.uniform(52, 1 + i, A.ncols, A.val.dtype)
        xs_pool.append(x)
        ys_pool.append(pinned(A.nrows, A.val.dtype))
        ws_pool.append(pinned(A.nrows, A.val.dtype))
    # the same requests from pageable buffers, for one comparison point
    pageable = ([np.array(x) for x in xs_pool], [np.empty(A.nrows, A.val.dtype) for A in pool],
                [np.empty(A.nrows, A.val.dtype) for A in pool])
    total = warm + nreq
    mats = (I.u64(52, 0, 0, total) % np.uint64(npool)).astype(np.int64)
    rows = np.array([A.nrows for A in pool], np.int64)
    link_bytes = np.array([A.val.itemsize * (A.ncols + 2 * A.nrows) for A in pool], np.float64)
    decade = np.minimum(np.floor(np.log10(rows[mats])).astype(np.int64), 5) - 3   # 0: 1e3.., 1: 1e4.., 2: 1e5..1e6
    budget = int(200e9)
    res = {"requests_measured": nreq, "requests_warmup": warm, "pool": npool,
           "pool_rows_min_max": [int(rows.min()), int(rows.max())], "pool_rows_total": int(rows.sum()),
           "pool_nnz_total": int(sum(A.nnz for A in pool)),
           "pool_host_bytes": int(sum(A.row_ptr.nbytes + A.col_idx.nbytes + A.val.nbytes for A in pool)),
           "pool_generation_s": round(gen_s, 1), "hbm_budget_bytes": budget}

    # the host link's own rates: 256 MB copies between pinned host memory and
    # HBM, each direction alone and both at once (two streams)
    hb = torch.empty(1 << 25, dtype=torch.float64, pin_memory=True)
    db = torch.empty(1 << 25, dtype=torch.float64, device="cuda")
    hb2 = torch.empty_like(hb, pin_memory=True)
    db2 = torch.empty_like(db)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def link(h2d, d2h, reps=5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            if h2d:
                with torch.cuda.stream(s1):
                    db.copy_(hb, non_blocking=True)
            if d2h:
                with torch.cuda.stream(s2):
                    hb2.copy_(db2, non_blocking=True)
        torch.cuda.synchronize()
        return round(reps * hb.nbytes * (int(h2d) + int(d2h)) / (time.perf_counter() - t0) / 1e9, 1)

    link(True, True, 1)
    res["host_link_probe_gbs"] = {"h2d": link(True, False), "d2h": link(False, True), "both": link(True, True)}
    del hb, db, hb2, db2
    log(f"serving: host link {res['host_link_probe_gbs']}")

    servers, ids, count = {}, {}, {}
    for mode in (1, 0):
        srv = spk.Server(streams=4, max_inflight=256, max_batch=64, mode=mode, hbm_budget=budget, alpha=0.5)
        ids[mode] = [srv.add_matrix(A) for A in pool]
        for i in range(npool):   # one request per matrix makes it resident
            srv.submit(ids[mode][i], xs_pool[i], ys_pool[i], ws_pool[i])
        srv.drain()
        servers[mode], count[mode] = srv, npool

    def saturation(mode, bufs=None):
        srv = servers[mode]
        bx, by, bw = bufs or (xs_pool, ys_pool, ws_pool)
        k = min(total, 3000)
        t0 = time.perf_counter()
        for i in range(k):
            m = mats[i]
            srv.submit(ids[mode][m], bx[m], by[m], bw[m])
        srv.drain()
        count[mode] += k
        return k / (time.perf_counter() - t0)

    def pct(v, q):
        return round(float(np.percentile(v, q)), 1) if v.size else None

    def replay(mode, arr, bufs=None):
        srv = servers[mode]
        bx, by, bw = bufs or (xs_pool, ys_pool, ws_pool)
        s0 = srv.stats()
        t0 = time.perf_counter()
        srv.replay(arr, [ids[mode][m] for m in mats], [bx[m] for m in mats], [by[m] for m in mats],
                   [bw[m] for m in mats])
        wall = time.perf_counter() - t0
        st = srv.stats()
        lo = count[mode] + warm
        hi = count[mode] + total
        count[mode] += total
        lat = srv.latencies()[lo:hi]
        wait, run = srv.latency_split()
        wait, run = wait[lo:hi], run[lo:hi]
        dec = decade[warm:]
        return {"p50_us": pct(lat, 50), "p99_us": pct(lat, 99), "mean_us": round(float(lat.mean()), 1),
                "p99_over_p50": round(float(np.percentile(lat, 99) / np.percentile(lat, 50)), 1),
                "wait_p50_p99_us": [pct(wait, 50), pct(wait, 99)], "run_p50_p99_us": [pct(run, 50), pct(run, 99)],
                "p50_p99_us_by_rows": {f"1e{d + 3}": [pct(lat[dec == d], 50), pct(lat[dec == d], 99)]
                                       for d in range(3)},
                "launches": st["batches"] - s0["batches"],
                "per_launch_us": {k: round((st[f] - s0[f]) / max(st["batches"] - s0["batches"], 1) * 1e6, 1)
                                  for k, f in (("stage_in", "stage_in_s"), ("device", "device_s"),
                                               ("stage_out", "stage_out_s"))},
                "direct_requests": st["direct"] - s0["direct"],
                "gbs": round((st["bytes_moved"] - s0["bytes_moved"]) / wall / 1e9, 2),
                "host_link_gbs": round(float(link_bytes[mats].sum()) / wall / 1e9, 2),
                "wall_s": round(wall, 2), "evictions": st["evictions"], "peak_hbm_bytes": st["peak_bytes"]}

    try:
        sat = {1: saturation(1), 0: saturation(0)}
        res["closed_loop_saturation_per_s"] = {"fifo_plain": round(sat[1], 1),
                                               "continuous_batching": round(sat[0], 1),
                                               "continuous_batching_pageable_buffers":
                                                   round(saturation(0, pageable), 1)}
        log(f"serving saturation: {res['closed_loop_saturation_per_s']}")
        for load_name, rate in (("load_0.7x_fifo_saturation", 0.7 * sat[1]),
                                ("load_0.5x_batching_saturation", 0.5 * sat[0]),
                                ("load_0.7x_batching_saturation", 0.7 * sat[0]),
                                ("load_0.9x_batching_saturation", 0.9 * sat[0])):
            arr = I.poisson_arrivals(total, rate, seed=51)
            point = {"offered_rate_per_s": round(rate, 1)}
            for mode, label in ((1, "fifo_plain"), (0, "continuous_batching")):
                point[label] = replay(mode, arr)
                log(f"serving {load_name} {label}: {point[label]}")
            if load_name == "load_0.7x_batching_saturation":
                point["continuous_batching_pageable_buffers"] = replay(0, arr, pageable)
                log(f"serving {load_name} pageable: {point['continuous_batching_pageable_buffers']}")
            res[load_name] = point
        # budget pressure: a batching server whose budget holds about 60% of
        # the pool's matrices, so admission evicts idle matrices (least
        # recently used first) and uploads them again from its host copy
        for k in (0, 1):
            servers.pop(k).close()
        budget_small = int(0.6 * res["pool_host_bytes"])
        srv = spk.Server(streams=4, max_inflight=256, max_batch=64, mode=0, hbm_budget=budget_small, alpha=0.5)
        servers["pressure"] = srv
        ids["pressure"] = [srv.add_matrix(A) for A in pool]
        count["pressure"] = 0
        small = min(total, 5000 + warm)
        rate = 0.12 * sat[0]
        arr = I.poisson_arrivals(small, rate, seed=53)
        s0 = srv.stats()
        t0 = time.perf_counter()
        srv.replay(arr, [ids["pressure"][m] for m in mats[:small]], [xs_pool[m] for m in mats[:small]],
                   [ys_pool[m] for m in mats[:small]], [ws_pool[m] for m in mats[:small]])
        wall = time.perf_counter() - t0
        st = srv.stats()
        lat = srv.latencies()[warm:small]
        res["budget_pressure"] = {"hbm_budget_bytes": budget_small, "offered_rate_per_s": round(rate, 1),
                                  "requests_measured": small - warm, "p50_us": pct(lat, 50), "p99_us": pct(lat, 99),
                                  "uploads": st["uploads"] - s0["uploads"], "evictions": st["evictions"] - s0["evictions"],
                                  "peak_hbm_bytes": st["peak_bytes"], "wall_s": round(wall, 2)}
        log(f"serving budget pressure: {res['budget_pressure']}")
    finally:
        for srv in servers.values():
            srv.close()
    return res


def cpu_baseline(B, x, alpha, step_bytes):
    """The oracle as it stands, on the host cores, over the same batch."""
    import numpy as np

    import oracle as O
    threads = O.num_threads()
    t = []
    t_total = 0.0
    # whole steps, repeated until about 10 s of CPU work (at least 3, at
    # most 200 steps)
    while len(t) < 3 or (t_total < 10.0 and len(t) < 200):
        t0 = time.perf_counter()
        O.batch_spmv_waxpy(B, x, alpha)
        dt = time.perf_counter() - t0
        t.append(dt)
        t_total += dt
    sec = float(np.median(t))
    return {"value": round(step_bytes / sec / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole batched step ({B.count} instances), median of {len(t)} runs "
                      f"({t_total:.1f} s), {sec * 1e3:.1f} ms per step"}


def cpu_beside_legs(I, legs):
    """The CPU-baseline leg beside the other results: the oracle as it
    stands, on all host cores, on the same seeded inputs as each GPU leg
    that ran (algorithmic bytes as there; median of a few runs)."""
    import numpy as np

    import oracle as O

    def median_s(fn, reps):
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            t.append(time.perf_counter() - t0)
        return float(np.median(t))

    res = {"threads": O.num_threads()}
    if "spmv_large" in legs:
        for name, A, seed in (("lap3d_128", I.lap3d(128), 31), ("zipf_1M", I.zipf(1000000), 34)):
            xh = I.uniform(seed, 0, A.ncols)
            sec = median_s(lambda: O.spmv(A, xh, with_absum=False), 3)
            nbytes = A.nnz * 12 + 4 * (A.nrows + 1) + 8 * A.ncols + 8 * A.nrows
            res[f"spmv_{name}"] = {"ms": round(sec * 1e3, 2), "gbs": round(nbytes / sec / 1e9, 2)}
    if "vector_sweep" in legs:
        n = 1 << 27
        xh, yh = I.uniform(21, 0, n), I.uniform(22, 0, n)
        for nm, fn, nbytes in (("waxpy", lambda: O.waxpy(1.5, xh, yh), 24 * n), ("dot", lambda: O.dot(xh, yh), 16 * n)):
            sec = median_s(fn, 3)
            res[f"{nm}_f64_n2^27"] = {"ms": round(sec * 1e3, 2), "gbs": round(nbytes / sec / 1e9, 2)}
        del xh, yh
    if "krylov_step_lap2d" in legs:
        A = I.lap2d(256)
        xh = I.uniform(11, 0, A.nrows)
        sec = median_s(lambda: O.spmv_waxpy(A, xh, 0.5), 20)
        res["krylov_step_lap2d"] = {"us": round(sec * 1e6, 1)}
    if "cg_lap3d_128" in legs:
        A = I.lap3d(128)
        bh = I.uniform(61, 0, A.nrows)
        it = 20
        sec = median_s(lambda: O.cg(A, bh, it), 1)
        res["cg_lap3d_128"] = {"us_per_iter": round(sec * 1e6 / it, 1), "iters": it}
    return res


def cpu_single_thread(B, x, alpha, step_bytes, steps=3):
    """The oracle on one host thread (the paper's serial reference), a few
    whole batched steps."""
    import numpy as np

    import oracle as O
    before = O.num_threads()
    O.set_threads(1)
    try:
        t = []
        for _ in range(steps):
            t0 = time.perf_counter()
            O.batch_spmv_waxpy(B, x, alpha)
            t.append(time.perf_counter() - t0)
    finally:
        O.set_threads(before)
    sec = float(np.median(t))
    return {"value": round(step_bytes / sec / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole batched step, median of {steps} runs, {sec * 1e3:.1f} ms per step"}


# The files whose contents define the batched tile kernel's device code:
# the committed counter figures apply only while these are unchanged.
TILE_KERNEL_SOURCES = ["kernels_batch.hip", "device_rows.h", "device_common.h", "batch_types.h", "row_tiles.h"]


def tile_kernel_hash() -> str:
    """Hash of the code (comments and whitespace removed) of the files that
    define the batched tile kernel."""
    import hashlib
    import re
    h = hashlib.sha1()
    for f in TILE_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1309_1894_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(f.encode())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:12]


def load_traffic(kernel, bytes_per_launch):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel calibration),
    or None when the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
        if t.get("kernel_source_hash") != tile_kernel_hash():
            return None
        return t.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")
    except (OSError, ValueError):
        return None


if __name__ == "__main__":
    main()
