"""The host-CPU SIMD autotuning of the vector update (the paper's Figure 1
protocol): the annotation expands into compiler-specific pragma variants,
each compiles, and every variant's output agrees with the oracle's WAXPY
within the rounding bound of a fused or unfused multiply-add, including the
ragged tails left by source-level unrolling."""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_1309_1894_amd import host_simd as H
from paper_1309_1894_amd import inputs as I


def test_annotation_space():
    sp = H.parse_annotation()
    assert sp["compiler"] == ["gcc", "clang"]
    assert sp["isa"] == ["default", "sse4.2", "avx2", "avx512"]
    assert sp["pragma"] == ["none", "ivdep", "omp_simd", "omp_simd_len", "vectorize"]
    assert sp["width"] == ["2", "4", "8"] and sp["unroll"] == ["1", "2", "4"] and sp["restrict"] == ["no", "yes"]


def test_expansion_counts_and_compiler_specific_pragmas():
    v = H.expand(isas=["default"], comps=["gcc", "clang"])
    # gcc: none, ivdep, omp_simd, 3 x omp_simd_len; clang: none, omp_simd,
    # 3 x omp_simd_len, 3 x vectorize; times 3 unrolls x 2 restrict
    assert len(v) == (6 + 8) * 3 * 2
    assert not any(x.pragma == "ivdep" and x.compiler == "clang" for x in v)
    assert not any(x.pragma == "vectorize" and x.compiler == "gcc" for x in v)
    assert H.BASELINE in v
    assert len(set(x.name for x in v)) == len(v)


def _sample_variants():
    comps = [c for c in ("gcc", "clang") if c in H.compilers()]
    isas = H.host_isas()
    out = []
    for c, isa in itertools.product(comps, isas):
        for v in H.expand(isas=[isa], comps=[c]):
            # one width per width-taking pragma keeps the CPU suite short
            if v.width in (0, 4) and (v.unroll == 1 or isa == "default"):
                out.append(v)
    return out


@pytest.mark.parametrize("n", [0, 1, 7, 1001])
def test_every_sampled_variant_matches_the_oracle(n):
    a = 1.5
    x = I.uniform(21, 0, n)
    y = I.uniform(22, 0, n)
    ref = O.waxpy(a, x, y)
    for v in _sample_variants():
        f = H.load(H.build_variant(v))
        w = np.full(n, np.nan)
        H.run(f, a, x, y, w)
        assert H.accept(w, ref, a, x, y), v.name


def test_acceptance_rejects_wrong_results():
    a = 1.5
    x = I.uniform(23, 0, 5000)
    y = I.uniform(24, 0, 5000)
    ref = O.waxpy(a, x, y)
    assert H.accept(ref.copy(), ref, a, x, y)
    bad = ref.copy()
    bad[4321] = np.nextafter(bad[4321], np.inf) * (1 + 1e-12)
    assert not H.accept(bad, ref, a, x, y)
    assert not H.accept(a * x - y, ref, a, x, y)
    short = ref.copy()
    short[-1] = 0.0
    assert not H.accept(short, ref, a, x, y)


def test_tune_keeps_a_validated_variant():
    vs = [v for v in H.expand(isas=["default"], comps=["gcc"]) if v.restrict and v.width in (0, 2)]
    rep = H.tune(sizes=(3000,), variants=vs, reps=2, target_s=0.002, confirm=2)
    r = rep["sizes"]["3000"]
    assert r["rejected"] == 0 and r["timed"] == len(vs) - (1 if H.BASELINE in vs else 0)
    assert r["best"] in {v.name for v in vs} | {H.BASELINE.name}
    assert r["speedup"] > 0
