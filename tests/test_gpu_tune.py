"""The tuner: validate-then-time over the compiled variant space, rejection of
variants whose output disagrees with the reference, plan DB round trip."""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from conftest import say
from paper_1309_1894_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_tune_waxpy_and_dot(spk, dev, tmp_path):
    db = str(tmp_path / "plans.spkdb")
    h = spk.Handle(0, db)
    try:
        n = 1 << 20
        x = I.uniform(21, 0, n)
        y = I.uniform(22, 0, n)
        xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
        w = torch.empty_like(xd)
        rep = spk.spk_tune(spk.problem(spk.SPK_OP_WAXPY, x=xd, y=yd, w=w, alpha=1.5), reps=3, warmup=1, handle=h)
        say(f"waxpy tune: {rep.best} {rep.best_us:.2f} us vs plain {rep.plain_us:.2f} us")
        assert rep.tried > 100 and rep.rejected == 0 and rep.best_us <= rep.plain_us
        assert O.max_ulp(w.cpu().numpy(), O.waxpy(1.5, x, y))[0] == 0
        key = rep.class_key.decode()
        assert key == "waxpy:f64:n20"
        d = torch.empty(1, dtype=torch.float64, device=dev)
        rep2 = spk.spk_tune(spk.problem(spk.SPK_OP_DOT, x=xd, y=yd, d_result=d), reps=3, handle=h)
        assert rep2.rejected == 0
        assert abs(d.item() - O.dot(x, y)) <= 1e-12 * O.dot_absum(x, y)
        # AXPY (in place) restores y between runs
        y2 = yd.clone()
        rep3 = spk.spk_tune(spk.problem(spk.SPK_OP_AXPY, x=xd, y=y2, alpha=-0.5), reps=3, handle=h)
        assert rep3.rejected == 0
        assert O.max_ulp(y2.cpu().numpy(), O.axpy(-0.5, x, y))[0] == 0
    finally:
        h.close()
    # a new handle loads the recorded winners
    h2 = spk.Handle(0, db)
    try:
        v = spk.spk_plan_get(key, handle=h2)
        assert v is not None and v.as_dict() == rep.best.as_dict()
        w2 = spk.spk_waxpy(1.5, xd, yd, handle=h2)
        assert O.max_ulp(w2.cpu().numpy(), O.waxpy(1.5, x, y))[0] == 0
    finally:
        h2.close()
    assert os.path.getsize(db) > 0


def test_planted_wrong_reference_rejects_everything(spk, dev):
    """A reference that is wrong (perturbed on the host) must make every variant
    fail validation; nothing is timed or recorded."""
    n = 4096
    x = I.uniform(1, 0, n)
    y = I.uniform(2, 0, n)
    ref = O.waxpy(1.5, x, y)
    ref[100] = np.nextafter(np.nextafter(ref[100], 9), 9)   # two ulps off
    h = spk.Handle(0)
    try:
        xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
        w = torch.empty_like(xd)
        with pytest.raises(spk.SpkError) as e:
            spk.spk_tune(spk.problem(spk.SPK_OP_WAXPY, x=xd, y=yd, w=w, alpha=1.5), ref=ref, reps=2, handle=h)
        assert e.value.name == "SPK_ERR_VALIDATION"
        assert spk.spk_plan_get("waxpy:f64:n12", handle=h) is None
        # the correct reference passes
        rep = spk.spk_tune(spk.problem(spk.SPK_OP_WAXPY, x=xd, y=yd, w=w, alpha=1.5), ref=O.waxpy(1.5, x, y),
                           reps=2, handle=h)
        assert rep.rejected == 0
    finally:
        h.close()


@pytest.mark.parametrize("which", ["zipf", "lap2d", "banded"])
def test_tune_spmv(spk, dev, which):
    A = {"zipf": lambda: I.zipf(50000, seed_struct=2, seed_val=3),
         "lap2d": lambda: I.lap2d(200),
         "banded": lambda: I.banded(40000, 12, 0.6, stream=5)}[which]()
    x = I.uniform(4, 0, A.ncols)
    ref, absum = O.spmv(A, x)
    h = spk.Handle(0)
    M = spk.Matrix(A, handle=h)
    try:
        xd = torch.from_numpy(x).to(dev)
        y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
        rep = spk.spk_tune(spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y), ref=ref, ref_scale=absum, reps=3,
                           handle=h)
        say(f"spmv tune {which}: {rep.best} {rep.best_us:.2f} us (plain {rep.plain_us:.2f}), pruned {rep.pruned}")
        assert rep.rejected == 0 and rep.tried > 20
        if which == "zipf":
            assert rep.pruned > 0   # sliced ELL is pruned by the padding model
        assert O.check_rows(y.cpu().numpy(), ref, absum, O.TAU_F64)[0] == 0
        # dispatch now uses the recorded winner
        y.fill_(float("nan"))
        spk.spk_spmv_mat(M, xd, y)
        assert O.check_rows(y.cpu().numpy(), ref, absum, O.TAU_F64)[0] == 0
        # the fused step, validated against the plain run
        w = torch.empty_like(y)
        rep2 = spk.spk_tune(spk.problem(spk.SPK_OP_SPMV_WAXPY, A=M, x=xd, y=y, w=w, alpha=0.5), reps=3, handle=h)
        assert rep2.rejected == 0
        assert O.max_ulp(w.cpu().numpy(), O.waxpy(0.5, y.cpu().numpy(), x))[0] == 0
    finally:
        M.release()
        h.close()


def _journal_points(db):
    """The journal's point lines; each is a distinct (search key, variant)."""
    with open(db) as f:
        pts = [json.loads(ln) for ln in f if ln.startswith('{"point": ')]
    assert len({(p["point"], tuple(p["v"])) for p in pts}) == len(pts)
    return pts


def test_tune_resume_times_only_the_rest(spk, dev, tmp_path):
    """A search cut short after k new points leaves exactly those k points in
    the journal; a new handle on the same DB resumes it, takes the k points
    from the journal and times only the rest; a third search times nothing,
    picks the same winner from the journal and still checks it against the
    reference."""
    db = str(tmp_path / "plans.spkdb")
    A = I.banded(30000, 8, 0.6, seed_struct=120, seed_val=121)
    x = I.uniform(122, 0, A.ncols)
    ref, absum = O.spmv(A, x)
    xd = torch.from_numpy(x).to(dev)
    y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
    k = 5
    reps = []
    for run in range(3):
        h = spk.Handle(0, db)
        M = spk.Matrix(A, handle=h)
        try:
            p = spk.problem(spk.SPK_OP_SPMV, A=M, x=xd, y=y)
            say(f"tune resume run {run}")
            if run == 0:
                with pytest.raises(spk.SpkError) as e:
                    spk.spk_tune(p, reps=3, warmup=1, max_variants=16, resume=True, stop_after=k, handle=h)
                assert e.value.name == "SPK_ERR_INTERRUPTED"
                assert len(_journal_points(db)) == k
                assert spk.spk_plan_get(spk.spk_class_key(p, handle=h), handle=h) is None
                continue
            rep = spk.spk_tune(p, reps=3, warmup=1, max_variants=16, resume=True, handle=h)
            reps.append(rep)
            assert rep.rejected == 0
            assert O.check_rows(y.cpu().numpy(), ref, absum, O.TAU_F64)[0] == 0
        finally:
            M.release()
            h.close()
    first, second = reps
    assert first.resumed >= k and first.tried >= 16 - k
    assert len(_journal_points(db)) == k + first.tried
    assert second.tried == 0 and second.resumed == first.resumed + first.tried
    assert second.best.as_dict() == first.best.as_dict() and second.best_us == first.best_us


def test_tune_resume_needs_a_matching_problem(spk, dev, tmp_path):
    """Journal points are filed under the problem's sizes: a problem of the
    same class but other sizes does not take them; nor does a search take a
    point journaled by another library build."""
    db = str(tmp_path / "plans.spkdb")
    n0 = 1 << 20
    h = spk.Handle(0)
    arch = h.info()[1].rsplit("(", 1)[1].rstrip(")")
    h.close()
    # journal lines of another library build, for every variant under the
    # first problem's key, are ignored
    with open(db, "w") as f:
        for v in spk.variants(spk.SPK_OP_WAXPY, spk.SPK_F64):
            f.write(json.dumps({"point": f"tune|waxpy:f64:n20|op{spk.SPK_OP_WAXPY}|n{n0}", "arch": arch,
                                "build": "another-build", "v": list(v.as_dict().values()), "us": 0.001}) + "\n")
    h = spk.Handle(0, db)
    try:
        for n in (n0, n0 + 4096):
            x = torch.from_numpy(I.uniform(123, 0, n)).to(dev)
            yv = torch.from_numpy(I.uniform(124, 0, n)).to(dev)
            w = torch.empty_like(x)
            rep = spk.spk_tune(spk.problem(spk.SPK_OP_WAXPY, x=x, y=yv, w=w, alpha=0.5), reps=2, max_variants=8,
                               resume=True, handle=h)
            assert rep.resumed == 0 and rep.tried == 8
    finally:
        h.close()
    # the planted lines carried the key this build files the first problem under
    with open(db) as f:
        pts = [json.loads(ln) for ln in f if ln.startswith('{"point": ')]
    mine = {p["point"] for p in pts if p["build"] != "another-build"}
    assert f"tune|waxpy:f64:n20|op{spk.SPK_OP_WAXPY}|n{n0}" in mine and len(mine) == 2


def test_cg_tune_rejects_journal_options(spk, dev):
    A = I.lap2d(32)
    h = spk.Handle(0)
    M = spk.Matrix(A, handle=h)
    try:
        b = torch.ones(A.nrows, dtype=torch.float64, device=dev)
        with pytest.raises(spk.SpkError) as e:
            spk.spk_cg_tune(M, b, 4, resume=True)
        assert e.value.name == "SPK_ERR_ARG"
    finally:
        M.release()
        h.close()
