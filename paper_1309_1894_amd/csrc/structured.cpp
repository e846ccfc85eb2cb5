// structured.cpp -- diagonal (DIA) and matrix-free stencil formats of a
// registered matrix: detection at registration, the DIA build on first use,
// dispatch of their SpMV kernels, and the format queries of the ABI.
//
// Section 3 of the paper counts the storage format among the decisions a
// GPU SpMV tuner makes (the prior work it cites chooses among CSR, ELL and
// others); these two formats are extra points of that search for matrices
// whose structure allows them.  Both are exact restatements of the stored
// matrix -- detection checks every entry -- so a tuned run reproduces the
// CSR product within the usual per-row tolerance (bit for bit when the CSR
// rows are sorted, since the products are added in ascending column order).
#include <algorithm>
#include <cstring>

#include "internal.h"

using namespace spk;

namespace spk {

namespace {

template <typename T>
bool same_bits(T a, T b)
{
    return memcmp(&a, &b, sizeof(T)) == 0;
}

// A constant-coefficient stencil with offsets `off` (ascending) on an
// N1 x N2 x N3 grid: every in-grid neighbour present, nothing else, one
// value per offset.
template <typename T>
bool check_stencil(const spk_mat *A, const int32_t *ci, const T *val, StructInfo &st)
{
    const int64_t n = A->nrows;
    const int nd = (int)st.off.size();
    // slot of each diagonal in the 7-slot ascending order -t, -s, -1, 0, 1, s, t
    int slot[kMaxDiag];
    if (nd == 3) {
        slot[0] = 2, slot[1] = 3, slot[2] = 4;
    } else if (nd == 5) {
        slot[0] = 1, slot[1] = 2, slot[2] = 3, slot[3] = 4, slot[4] = 5;
    } else {
        for (int d = 0; d < 7; ++d) slot[d] = d;
    }
    bool seen[7] = {false, false, false, false, false, false, false};
    T coef[7] = {};
    const int64_t N3 = st.N3, N2 = st.N2, N1 = st.N1;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t k = r % N3, j = (r / N3) % N2, i = r / (N3 * N2);
        const bool want[7] = {i > 0, j > 0, k > 0, true, k + 1 < N3, j + 1 < N2, i + 1 < N1};
        bool got[7] = {false, false, false, false, false, false, false};
        const int64_t s0 = A->rp_host[r], s1 = A->rp_host[r + 1];
        for (int64_t e = s0; e < s1; ++e) {
            const int64_t o = (int64_t)ci[e] - r;
            int d = -1;
            for (int q = 0; q < nd; ++q)
                if (st.off[q] == o) d = q;
            if (d < 0) return false;
            const int sl = slot[d];
            if (got[sl]) return false;   // duplicate
            got[sl] = true;
            if (!seen[sl]) {
                coef[sl] = val[e];
                seen[sl] = true;
            } else if (!same_bits(coef[sl], val[e])) {
                return false;
            }
        }
        for (int q = 0; q < 7; ++q) {
            // slots that do not exist in this dimension are never wanted
            const bool exists = (nd == 7) || (nd == 5 && q >= 1 && q <= 5) || (nd == 3 && q >= 2 && q <= 4);
            if (got[q] != (want[q] && exists)) return false;
        }
    }
    for (int q = 0; q < 7; ++q) st.coef[q] = seen[q] ? (double)coef[q] : 0.0;
    return true;
}

}  // namespace

void detect_structure(spk_mat *A, const int32_t *ci, const void *val)
{
    StructInfo st;
    const int64_t m = A->nrows;
    if (m == 0 || A->nnz == 0 || !ci) {
        A->st = st;
        return;
    }
    // diagonals: stop as soon as there are too many
    std::vector<int32_t> off;
    for (int64_t r = 0; r < m; ++r) {
        for (int64_t e = A->rp_host[r]; e < A->rp_host[r + 1]; ++e) {
            const int64_t o = (int64_t)ci[e] - r;
            if (o < INT32_MIN || o > INT32_MAX) {
                A->st = st;
                return;
            }
            if (std::find(off.begin(), off.end(), (int32_t)o) == off.end()) {
                if ((int)off.size() == kMaxDiag) {
                    A->st = st;
                    return;
                }
                off.push_back((int32_t)o);
            }
        }
    }
    std::sort(off.begin(), off.end());
    // no (row, column) twice
    for (int64_t r = 0; r < m; ++r) {
        uint32_t used = 0;
        for (int64_t e = A->rp_host[r]; e < A->rp_host[r + 1]; ++e) {
            const int32_t o = (int32_t)((int64_t)ci[e] - r);
            const int d = (int)(std::lower_bound(off.begin(), off.end(), o) - off.begin());
            if (used & (1u << d)) {
                A->st = st;
                return;
            }
            used |= 1u << d;
        }
    }
    st.dia = true;
    st.off = off;
    // stencil shapes: {-1,0,1}, {-s,-1,0,1,s}, {-t,-s,-1,0,1,s,t}
    const int64_t n = A->ncols;
    const int nd = (int)off.size();
    if (val && m == n && (nd == 3 || nd == 5 || nd == 7)) {
        bool sym = true;
        for (int q = 0; q < nd; ++q) sym = sym && off[q] == -off[nd - 1 - q];
        if (sym && off[nd / 2] == 0 && off[nd / 2 + 1] == 1) {
            bool shape = false;
            if (nd == 3) {
                st.dim = 1, st.N3 = (int)n, st.N2 = 1, st.N1 = 1;
                shape = true;
            } else if (nd == 5) {
                const int64_t s = off[4];
                if (s > 1 && n % s == 0) {
                    st.dim = 2, st.N3 = (int)s, st.N2 = (int)(n / s), st.N1 = 1;
                    shape = true;
                }
            } else {
                const int64_t s = off[5], t = off[6];
                if (s > 1 && t > s && t % s == 0 && n % t == 0) {
                    st.dim = 3, st.N3 = (int)s, st.N2 = (int)(t / s), st.N1 = (int)(n / t);
                    shape = true;
                }
            }
            if (shape)
                st.stencil = A->dtype == SPK_F64 ? check_stencil<double>(A, ci, (const double *)val, st)
                                                 : check_stencil<float>(A, ci, (const float *)val, st);
        }
    }
    if (!st.stencil) st.dim = 0, st.N1 = st.N2 = st.N3 = 1;
    A->st = st;
}

bool format_applies(const spk_mat *A, int format)
{
    if (format == SPK_FMT_DIA) return A && A->st.dia;
    if (format == SPK_FMT_STENCIL) return A && A->st.stencil;
    if (format == SPK_FMT_COLBLOCK) return A && A->dtype == SPK_F64;
    if (format == SPK_FMT_XWIN) return A != nullptr;
    return format >= SPK_FMT_SCALAR && format <= SPK_FMT_ADAPTIVE;
}

const StructEntry *find_struct_entry(int format, int block, int rows, int lds)
{
    int n = 0;
    const StructEntry *t = struct_table(&n);
    for (int i = 0; i < n; ++i)
        if (t[i].format == format && t[i].block == block && t[i].rows == rows && t[i].lds == lds) return &t[i];
    return nullptr;
}

bool struct_entry_fits(const spk_mat *A, const StructEntry &e)
{
    if (!e.lds) return true;
    return stencil_lds_bytes(e.block, e.rows, A->st.dim, A->st.N3, (int)dtype_size(A->dtype)) <= kStencilLdsMaxBytes;
}

int64_t format_bytes(const spk_mat *A, int format, bool fused)
{
    const int64_t s = (int64_t)dtype_size(A->dtype), m = A->nrows, n = A->ncols;
    int64_t b;
    if (format == SPK_FMT_DIA) b = (int64_t)A->st.off.size() * m * s + 2 * m + n * s + m * s;
    else if (format == SPK_FMT_STENCIL) b = n * s + m * s;
    else b = spmv_bytes(m, n, A->nnz, A->dtype, false);
    if (fused) b += m * s;
    return b;
}

static spk_status get_dia(spk_handle h, spk_mat *A, DiaData **out)
{
    std::lock_guard<std::mutex> lk(h->mu);
    if (!A->dia.val) {
        const int64_t m = A->nrows, nd = (int64_t)A->st.off.size();
        const size_t vb = (size_t)(nd * m) * dtype_size(A->dtype);
        DiaData d;
        SPK_HIP(hipMalloc(&d.val, std::max<size_t>(vb, 16)));
        if (hipMalloc(&d.mask, std::max<size_t>((size_t)m * 2, 16)) != hipSuccess) {
            (void)hipFree(d.val);
            return fail(SPK_ERR_OOM, "DIA mask");
        }
        SPK_HIP(hipMemsetAsync(d.val, 0, vb, h->work));
        SPK_HIP(launch_csr_to_dia(A->dtype, (int32_t)m, A->rp, A->ci, A->val, (int32_t)nd, A->st.off.data(), d.val,
                                  d.mask, h->work));
        SPK_HIP(hipStreamSynchronize(h->work));
        d.bytes = (int64_t)vb + 2 * m;
        A->bytes += d.bytes;
        A->dia = d;
    }
    *out = &A->dia;
    return SPK_OK;
}

spk_status run_structured(spk_handle h, const SpmvProblem &p, const spk_variant &v, hipStream_t s)
{
    spk_mat *A = p.mat;
    if (!A) return fail(SPK_ERR_ARG, "format %d needs a registered matrix", v.format);
    if (!format_applies(A, v.format)) return fail(SPK_ERR_ARG, "format %d does not apply to this matrix", v.format);
    const StructEntry *e = find_struct_entry(v.format, v.block, v.unroll, v.lds);
    if (!e)
        return fail(SPK_ERR_NOT_FOUND, "no compiled structured SpMV format=%d block=%d unroll=%d lds=%d", v.format,
                    v.block, v.unroll, v.lds);
    if (!struct_entry_fits(A, *e))
        return fail(SPK_ERR_ARG, "the stencil's grid lines are too long to stage through LDS");
    const StructFn fn = e->fn[A->dtype][p.fused ? 1 : 0];
    if (v.format == SPK_FMT_DIA) {
        DiaData *d = nullptr;
        SPK_TRY(get_dia(h, A, &d));
        DiaArgs a{};
        a.m = (int32_t)A->nrows;
        a.ncols = (int32_t)A->ncols;
        a.ndiag = (int32_t)A->st.off.size();
        for (int q = 0; q < a.ndiag; ++q) a.off[q] = A->st.off[q];
        a.val = d->val;
        a.mask = d->mask;
        a.x = p.x;
        a.y = p.y;
        a.w = p.w;
        a.alpha = p.alpha;
        SPK_HIP(fn(&a, s));
        return SPK_OK;
    }
    StencilArgs a{};
    a.n = (int32_t)A->nrows;
    a.N1 = A->st.N1;
    a.N2 = A->st.N2;
    a.N3 = A->st.N3;
    a.dim = A->st.dim;
    for (int q = 0; q < 7; ++q) a.coef[q] = A->st.coef[q];
    a.x = p.x;
    a.y = p.y;
    a.w = p.w;
    a.alpha = p.alpha;
    SPK_HIP(fn(&a, s));
    return SPK_OK;
}

}  // namespace spk

extern "C" {

spk_status spk_matrix_formats(spk_handle h, spk_matrix A, uint32_t *mask)
{
    if (!h || !A || !mask) return fail(SPK_ERR_NULL, "NULL argument");
    uint32_t m = 0;
    for (int f = SPK_FMT_SCALAR; f <= SPK_FMT_XWIN; ++f)
        if (format_applies(A, f)) m |= 1u << f;
    *mask = m;
    return SPK_OK;
}

spk_status spk_csr_structure(const spk_csr *csr, spk_structure *out)
{
    if (!csr || !out) return fail(SPK_ERR_NULL, "NULL argument");
    if (csr->nrows < 0 || csr->ncols < 0 || csr->nnz < 0) return fail(SPK_ERR_SHAPE, "negative size");
    if (!dtype_ok(csr->dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", csr->dtype);
    if (csr->nrows > 0 && !csr->row_ptr) return fail(SPK_ERR_NULL, "row_ptr is NULL");
    if (csr->nnz > 0 && (!csr->col_idx || !csr->val)) return fail(SPK_ERR_NULL, "col_idx/val are NULL");
    if (csr->nrows >= INT32_MAX || csr->ncols >= INT32_MAX) return fail(SPK_ERR_SHAPE, "too many rows or columns");
    spk_mat M;
    M.nrows = csr->nrows;
    M.ncols = csr->ncols;
    M.nnz = csr->nnz;
    M.dtype = csr->dtype;
    M.rp_host.assign(csr->row_ptr, csr->row_ptr + (csr->nrows > 0 ? csr->nrows + 1 : 0));
    if (M.nrows > 0 && (M.rp_host[0] != 0 || M.rp_host[M.nrows] != M.nnz))
        return fail(SPK_ERR_CSR, "row_ptr does not span [0, nnz]");
    for (int64_t i = 0; i < M.nrows; ++i)
        if (M.rp_host[i + 1] < M.rp_host[i]) return fail(SPK_ERR_CSR, "row_ptr decreases at row %lld", (long long)i);
    detect_structure(&M, csr->col_idx, csr->val);
    memset(out, 0, sizeof *out);
    for (int f = SPK_FMT_SCALAR; f <= SPK_FMT_STENCIL; ++f)
        if (format_applies(&M, f)) out->formats |= 1u << f;
    out->ndiag = M.st.dia ? (int32_t)M.st.off.size() : 0;
    for (int q = 0; q < out->ndiag; ++q) out->offsets[q] = M.st.off[q];
    out->dim = M.st.stencil ? M.st.dim : 0;
    out->n1 = M.st.N1;
    out->n2 = M.st.N2;
    out->n3 = M.st.N3;
    for (int q = 0; q < 7; ++q) out->coef[q] = M.st.coef[q];
    return SPK_OK;
}

spk_status spk_matrix_format_bytes(spk_handle h, spk_matrix A, int32_t format, int32_t fused, int64_t *bytes)
{
    if (!h || !A || !bytes) return fail(SPK_ERR_NULL, "NULL argument");
    if (!format_applies(A, format)) return fail(SPK_ERR_ARG, "format %d does not apply to this matrix", format);
    *bytes = format_bytes(A, format, fused != 0);
    return SPK_OK;
}

}  // extern "C"
