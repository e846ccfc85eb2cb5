"""The C ABI library loads, exports every declared entry point, and rejects
bad arguments before touching the GPU (CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spk.h")
LIB = os.path.join(ROOT, "paper_1309_1894_amd", "libspk.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spk_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["spk_spmv_csr", "spk_waxpy", "spk_axpy", "spk_dot", "spk_tune", "spk_matrix_register",
                 "spk_spmv_waxpy", "spk_cg", "spk_batch_plan", "spk_batch_run", "spk_serve_create", "spk_serve_replay"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol(lib):
    from paper_1309_1894_amd import spk
    missing = [n for n in declared() if n not in spk._SIGS]
    assert not missing, missing


def test_abi_version_and_status_strings(lib):
    from paper_1309_1894_amd import spk
    assert spk.spk_abi_version() == 1
    for code, name in spk.STATUS.items():
        assert spk.spk_status_str(code) == name


def test_null_handle_rejected_before_hip(lib):
    from paper_1309_1894_amd import spk
    L = spk.lib
    assert L.spk_waxpy(None, 1, 10, 1.0, None, None, None, None) == 1
    assert L.spk_axpy(None, 1, 10, 1.0, None, None, None) == 1
    assert L.spk_dot(None, 1, 10, None, None, None, None) == 1
    assert L.spk_spmv_csr(None, None, None, None, None) == 1
    assert L.spk_cg(None, None, None, None, 0, None, None) == 1
    assert L.spk_destroy(None) == 1
    assert L.spk_batch_free(None, None) == 1
    assert L.spk_batch_tile_modes(None, None, None, None) == 1
    assert L.spk_serve_destroy(None) == 1
    assert b"NULL" in L.spk_last_error()


def test_variant_space_is_enumerable_on_the_host(lib):
    from paper_1309_1894_amd import spk
    for op in (spk.SPK_OP_WAXPY, spk.SPK_OP_AXPY, spk.SPK_OP_DOT):
        for dt in (spk.SPK_F32, spk.SPK_F64):
            vs = spk.variants(op, dt)
            assert len(vs) > 50
            # the plain variant comes first: 256 threads, one element per thread
            assert (vs[0].block, vs[0].vec, vs[0].unroll, vs[0].grid) == (256, 1, 1, 0)
            for v in vs:
                assert v.vec * (8 if dt == spk.SPK_F64 else 4) <= 16
    sp = spk.variants(spk.SPK_OP_SPMV, spk.SPK_F64)
    fmts = {v.format for v in sp}
    assert fmts == {spk.SPK_FMT_SCALAR, spk.SPK_FMT_VECTOR, spk.SPK_FMT_SELL, spk.SPK_FMT_ADAPTIVE}
    assert {v.group for v in sp if v.format == spk.SPK_FMT_VECTOR} == {2, 4, 8, 16, 32, 64}
    p0, p1 = spk.spk_plain_variant(spk.SPK_OP_SPMV, 0), spk.spk_plain_variant(spk.SPK_OP_SPMV, 1)
    assert (p0.format, p0.block, p0.group) == (spk.SPK_FMT_SCALAR, 256, 1)
    assert (p1.format, p1.block, p1.group) == (spk.SPK_FMT_VECTOR, 256, 64)
    with pytest.raises(spk.SpkError):
        spk.spk_variant_get(spk.SPK_OP_SPMV, spk.SPK_F64, 10 ** 6)


def test_bad_dtype_and_op(lib):
    from paper_1309_1894_amd import spk
    n = ctypes.c_int32()
    assert spk.lib.spk_variant_count(99, 1, ctypes.byref(n)) == 11
    assert spk.lib.spk_variant_count(1, 7, ctypes.byref(n)) == 3


def test_create_without_a_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1309_1894_amd import spk
    h = ctypes.c_void_p()
    s = spk.lib.spk_create(0, None, ctypes.byref(h))
    assert s != 0 and h.value is None


def test_header_is_plain_c99(tmp_path):
    """The boundary header compiles as C99 on its own (no C++ or HIP types)."""
    import subprocess
    src = tmp_path / "use.c"
    src.write_text('#include "spk.h"\nint main(void) { spk_variant v = {0}; (void)v; return spk_abi_version() < 0; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_binding_rejects_short_tensors():
    """The C entry points take bare pointers; the binding refuses a tensor
    shorter than the call would read or write before passing its pointer."""
    import torch

    from paper_1309_1894_amd import spk
    x, short = torch.zeros(10, dtype=torch.float64), torch.zeros(9, dtype=torch.float64)
    with pytest.raises(ValueError, match="y holds 9"):
        spk.problem(spk.SPK_OP_WAXPY, x=x, y=short, w=x, alpha=1.0)
    with pytest.raises(ValueError, match="w holds 9"):
        spk.problem(spk.SPK_OP_WAXPY, x=x, y=x, w=short, alpha=1.0)
    with pytest.raises(ValueError, match="d_result holds 0"):
        spk.problem(spk.SPK_OP_DOT, x=x, y=x, d_result=torch.zeros(0, dtype=torch.float64))
    ci, val = torch.zeros(0, dtype=torch.int32), torch.zeros(0, dtype=torch.float64)
    with pytest.raises(ValueError, match="y holds 9"):
        spk.spk_spmv_csr(torch.zeros(11, dtype=torch.int32), ci, val, x, y=short, nrows=10)
    with pytest.raises(ValueError, match="row_ptr holds 5"):
        spk.spk_spmv_csr(torch.zeros(5, dtype=torch.int32), ci, val, x, y=x, nrows=10)


def test_binding_constants_match_the_header():
    """Every SPK_* enumerator the binding names has the header's value."""
    from paper_1309_1894_amd import spk
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    values = {}
    for body in re.findall(r"typedef\s+enum\s*\{(.*?)\}", text, flags=re.S):
        nxt = 0
        for item in (x.strip() for x in body.split(",")):
            if not item:
                continue
            name, _, val = item.partition("=")
            nxt = int(val.strip(), 0) if val.strip() else nxt
            values[name.strip()] = nxt
            nxt += 1
    assert values["SPK_FMT_COLBLOCK"] == 7 and values["SPK_ERR_STATE"] == 12
    named = {k: getattr(spk, k) for k in dir(spk) if k.startswith("SPK_") and isinstance(getattr(spk, k), int)}
    assert len(named) >= 15
    for k, v in named.items():
        if k in values:
            assert v == values[k], k
    for k in values:
        if k.startswith(("SPK_FMT_", "SPK_OP_", "SPK_F")):
            assert named.get(k) == values[k], k
    assert spk.STATUS == {v: k for k, v in values.items() if k.startswith(("SPK_OK", "SPK_ERR_"))}


CITES = re.compile(r"Section [1-4]|Figure 1|[Nn]ot in the paper|callers that cannot allocate")


def declaration_comments():
    """(function name, the comment that documents it) for every function the
    header declares: the comment of the blank-line-separated paragraph the
    declaration sits in, else the closest comment above it."""
    text = open(HEADER).read()
    out = []
    last_comment = ""
    for para in re.split(r"\n\s*\n", text):
        comments = re.findall(r"/\*.*?\*/", para, flags=re.S)
        if comments:
            last_comment = comments[0]
        code = re.sub(r"/\*.*?\*/", "", para, flags=re.S)
        for name in re.findall(r"^\s*(?:spk_status|int|const char \*)\s*\**(spk_[a-z0-9_]+)\s*\(", code, flags=re.M):
            out.append((name, " ".join(comments) if comments else last_comment))
    return out


def test_every_declaration_cites_the_paper_or_says_it_is_not_in_it():
    decl = declaration_comments()
    assert {n for n, _ in decl} == set(declared())
    flat = lambda c: re.sub(r"\s+", " ", re.sub(r"^\s*\*(?!/)", " ", c, flags=re.M))
    bad = [n for n, c in decl if not CITES.search(flat(c))]
    assert not bad, bad
