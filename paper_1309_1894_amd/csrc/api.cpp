// api.cpp -- the C ABI of libspk: handles, argument checks, dispatch of
// WAXPY/AXPY/dot and CSR SpMV variants, matrix registration, plan DB.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>

#include "device_common.h"
#include "internal.h"

namespace spk {

namespace {
thread_local char g_err[1024] = "";
}

spk_status fail(spk_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

spk_status hip_fail(hipError_t e, const char *what)
{
    snprintf(g_err, sizeof g_err, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SPK_ERR_OOM;
    return SPK_ERR_HIP;
}

const char *dtype_name(int dtype) { return dtype == SPK_F64 ? "f64" : "f32"; }

double now_seconds()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int64_t spmv_bytes(int64_t m, int64_t n, int64_t nnz, int dtype, bool fused)
{
    const int64_t s = (int64_t)dtype_size(dtype);
    int64_t b = nnz * (s + 4) + 4 * (m + 1) + n * s + m * s;
    if (fused) b += m * s;  // w
    return b;
}

// ------------------------------------------------------------ variants --

const VecEntry *find_vec_entry(int op, int dtype, const spk_variant &v)
{
    int n = 0;
    const VecEntry *t = (op == SPK_OP_DOT) ? dot_table(&n) : waxpy_table(&n);
    for (int i = 0; i < n; ++i)
        if (t[i].block == v.block && t[i].vec == v.vec && t[i].unroll == v.unroll && t[i].fn[dtype]) return &t[i];
    return nullptr;
}

const SpmvEntry *find_spmv_entry(const spk_variant &v)
{
    int n = 0;
    const SpmvEntry *t = spmv_table(&n);
    for (int i = 0; i < n; ++i) {
        const SpmvEntry &e = t[i];
        if (e.format != v.format || e.block != v.block || e.unroll != v.unroll) continue;
        if (std::max(1, e.vec) != std::max(1, v.vec)) continue;
        if (e.format == SPK_FMT_VECTOR && (e.group != v.group || e.lds != v.lds)) continue;
        if (e.format == SPK_FMT_SELL && e.group != v.group) continue;
        if (e.format == SPK_FMT_ADAPTIVE && (e.lds != v.lds || e.group != v.group)) continue;
        return &e;
    }
    return nullptr;
}

// The per-block kernel of a column-blocked variant: the ADAPTIVE row-block
// kernel with the variant's workgroup size and wavefront capacity.
spk_variant colblock_inner(const spk_variant &v)
{
    spk_variant iv{};
    iv.format = SPK_FMT_ADAPTIVE;
    iv.block = v.block;
    iv.group = 1;
    iv.unroll = 1;
    iv.streams = 1;
    iv.lds = v.lds;
    return iv;
}

spk_status check_variant(int op, int dtype, const spk_variant &v)
{
    if (op == SPK_OP_WAXPY || op == SPK_OP_AXPY || op == SPK_OP_DOT) {
        if (!find_vec_entry(op, dtype, v))
            return fail(SPK_ERR_NOT_FOUND, "no compiled %s variant block=%d vec=%d unroll=%d for %s",
                        op == SPK_OP_DOT ? "dot" : "waxpy", v.block, v.vec, v.unroll, dtype_name(dtype));
        if (v.grid < 0 || v.grid > 1024) return fail(SPK_ERR_ARG, "grid %d out of range", v.grid);
        return SPK_OK;
    }
    if (op == SPK_OP_SPMV || op == SPK_OP_SPMV_WAXPY) {
        if (v.format == SPK_FMT_DIA || v.format == SPK_FMT_STENCIL) {
            if (!find_struct_entry(v.format, v.block, v.unroll, v.lds))
                return fail(SPK_ERR_NOT_FOUND,
                            "no compiled structured SpMV variant format=%d block=%d unroll=%d lds=%d", v.format,
                            v.block, v.unroll, v.lds);
            return SPK_OK;
        }
        if (v.format == SPK_FMT_COLBLOCK) {
            if (dtype != SPK_F64) return fail(SPK_ERR_DTYPE, "the column-blocked form is FP64 only");
            if (v.group != 2 && v.group != 4) return fail(SPK_ERR_ARG, "column blocks must be 2 or 4 (got %d)", v.group);
            if (v.streams != 1) return fail(SPK_ERR_ARG, "the column-blocked form runs on one stream");
            if (!find_spmv_entry(colblock_inner(v)))
                return fail(SPK_ERR_NOT_FOUND, "no compiled row-block kernel block=%d lds=%d", v.block, v.lds);
            return SPK_OK;
        }
        if (v.format == SPK_FMT_XWIN) {
            if (!find_xwin_entry(v.block, v.group, v.lds))
                return fail(SPK_ERR_NOT_FOUND, "no compiled x-window kernel block=%d window=%d KiB entries=%d",
                            v.block, v.group, v.lds);
            if (v.grid < 1 || v.grid > 4) return fail(SPK_ERR_ARG, "x-window chunks per CU must be 1..4 (got %d)", v.grid);
            if (v.streams != 1) return fail(SPK_ERR_ARG, "the x-window form runs on one stream");
            return SPK_OK;
        }
        if (!find_spmv_entry(v))
            return fail(SPK_ERR_NOT_FOUND, "no compiled SpMV variant format=%d block=%d group=%d unroll=%d lds=%d",
                        v.format, v.block, v.group, v.unroll, v.lds);
        if (!(v.streams == 1 || v.streams == 2 || v.streams == 4))
            return fail(SPK_ERR_ARG, "streams must be 1, 2 or 4 (got %d)", v.streams);
        return SPK_OK;
    }
    return fail(SPK_ERR_ARG, "unknown op %d", op);
}

spk_variant plain_variant(int op, int which)
{
    spk_variant v{};
    if (op == SPK_OP_SPMV || op == SPK_OP_SPMV_WAXPY) {
        v.format = which == 0 ? SPK_FMT_SCALAR : SPK_FMT_VECTOR;
        v.block = 256;
        v.group = which == 0 ? 1 : 64;
        v.unroll = 1;
        v.streams = 1;
    } else {
        v.block = 256;
        v.vec = 1;
        v.unroll = 1;
        v.grid = 0;
    }
    return v;
}

static int pow2_ceil(double x)
{
    int p = 1;
    while (p < x && p < (1 << 30)) p <<= 1;
    return p;
}

spk_variant default_variant(spk_handle h, const spk_problem &p, const spk_csr *csr)
{
    (void)h;
    spk_variant v{};
    switch (p.op) {
    case SPK_OP_WAXPY:
    case SPK_OP_AXPY:
        v.block = 256;
        v.vec = p.dtype == SPK_F64 ? 2 : 4;
        v.unroll = 2;
        v.grid = 0;
        return v;
    case SPK_OP_DOT:
        v.block = 256;
        v.vec = p.dtype == SPK_F64 ? 2 : 4;
        v.unroll = 4;
        v.grid = 8;
        return v;
    default:
        break;
    }
    v.streams = 1;
    v.unroll = 1;
    if (p.A) {
        v.format = SPK_FMT_ADAPTIVE;
        v.block = 256;
        v.group = 1;
        v.lds = 512;
        return v;
    }
    const double mean = csr && csr->nrows > 0 ? (double)csr->nnz / (double)csr->nrows : 1.0;
    v.format = SPK_FMT_VECTOR;
    v.block = 256;
    v.group = std::min(64, std::max(2, pow2_ceil(mean)));
    return v;
}

static int ilog2_ceil(double x)
{
    int k = 0;
    while ((double)(1ll << k) < x && k < 62) ++k;
    return k;
}

std::string class_key(const spk_problem &p, const spk_csr *csr)
{
    char buf[128];
    switch (p.op) {
    case SPK_OP_WAXPY:
    case SPK_OP_AXPY:
    case SPK_OP_DOT: {
        const char *nm = p.op == SPK_OP_WAXPY ? "waxpy" : p.op == SPK_OP_AXPY ? "axpy" : "dot";
        snprintf(buf, sizeof buf, "%s:%s:n%d", nm, dtype_name(p.dtype), ilog2_ceil((double)std::max<int64_t>(1, p.n)));
        return buf;
    }
    default:
        break;
    }
    const char *nm = p.op == SPK_OP_SPMV ? "spmv" : "spmv_waxpy";
    if (p.A) {
        const spk_mat *A = p.A;
        const double mean = std::max(1.0, A->mean_len);
        const double ratio = (double)std::max<int64_t>(1, A->max_len) / mean;
        const int skew = ratio <= 2.0 ? 0 : ratio <= 16.0 ? 1 : 2;
        // matrices that admit a structured format form classes of their own
        const char *tag = A->st.stencil ? ":st" : A->st.dia ? ":dia" : "";
        snprintf(buf, sizeof buf, "%s:%s:m%d:l%d:s%d%s", nm, dtype_name(A->dtype),
                 ilog2_ceil((double)std::max<int64_t>(1, A->nrows)), (int)std::lround(std::log2(mean)), skew, tag);
        return buf;
    }
    const double mean = csr && csr->nrows > 0 ? std::max(1.0, (double)csr->nnz / (double)csr->nrows) : 1.0;
    snprintf(buf, sizeof buf, "spmv_csr:%s:m%d:l%d", csr ? dtype_name(csr->dtype) : "f64",
             ilog2_ceil((double)std::max<int64_t>(1, csr ? csr->nrows : 1)), (int)std::lround(std::log2(mean)));
    return buf;
}

// ------------------------------------------------------- vector kernels --

spk_status run_waxpy(spk_handle h, int dtype, int64_t n, double alpha, const void *x, const void *y, void *w,
                     const spk_variant &v, hipStream_t s)
{
    if (n == 0) return SPK_OK;
    spk_variant vv = v;
    const size_t bytes = (size_t)vv.vec * dtype_size(dtype);
    // vector accesses need every pointer aligned to the access size
    if (vv.vec > 1 && (((uintptr_t)x | (uintptr_t)y | (uintptr_t)w) % bytes) != 0) vv.vec = 1;
    const VecEntry *e = find_vec_entry(SPK_OP_WAXPY, dtype, vv);
    if (!e) return fail(SPK_ERR_NOT_FOUND, "waxpy variant not compiled");
    VecLaunch L{};
    L.n = n;
    L.alpha = dtype == SPK_F32 ? (double)(float)alpha : alpha;
    L.x = x;
    L.y = y;
    L.w = w;
    L.grid = vec_grid(*e, n, vv.grid, h->num_cu);
    SPK_HIP(e->fn[dtype](L, s));
    return SPK_OK;
}

static spk_status dot_scratch(spk_handle h, hipStream_t s, int64_t need, DotScratch **out)
{
    std::lock_guard<std::mutex> lk(h->mu);
    DotScratch &d = h->dot[s];
    if (d.cap < need) {
        if (d.partial) {
            // the stream may still use the old buffers
            SPK_HIP(hipStreamSynchronize(s));
            SPK_HIP(hipFree(d.partial));
            SPK_HIP(hipFree(d.ticket));
            d.partial = nullptr;
            d.ticket = nullptr;
        }
        const int64_t cap = std::max<int64_t>(need, 4096);
        SPK_HIP(hipMalloc(&d.partial, (size_t)cap * sizeof(double)));
        SPK_HIP(hipMalloc(&d.ticket, 256));
        SPK_HIP(hipMemsetAsync(d.ticket, 0, 256, s));
        d.cap = cap;
    }
    *out = &d;
    return SPK_OK;
}

// Kernel and grid of a dot variant on these operands (vector width 1 when
// x or y is not aligned to the variant's access size).
static spk_status dot_plan(spk_handle h, int dtype, int64_t n, const void *x, const void *y, const spk_variant &v,
                           const VecEntry **e, int64_t *grid)
{
    spk_variant vv = v;
    const size_t bytes = (size_t)vv.vec * dtype_size(dtype);
    if (vv.vec > 1 && (((uintptr_t)x | (uintptr_t)y) % bytes) != 0) vv.vec = 1;
    *e = find_vec_entry(SPK_OP_DOT, dtype, vv);
    if (!*e) return fail(SPK_ERR_NOT_FOUND, "dot variant not compiled");
    *grid = vec_grid(**e, n, vv.grid, h->num_cu);
    return SPK_OK;
}

// One dot on the given scratch: `partial` holds `grid` doubles; `ticket`
// (used when grid <= kDotTicketMaxGrid, else NULL) is zero on entry and left
// at zero by the kernel.
static spk_status dot_launch(const VecEntry *e, int dtype, int64_t n, const void *x, const void *y, double *out,
                             int64_t grid, double *partial, uint32_t *ticket, hipStream_t s)
{
    VecLaunch L{};
    L.n = n;
    L.x = x;
    L.y = y;
    L.partial = partial;
    L.ticket = grid <= kDotTicketMaxGrid ? ticket : nullptr;
    L.out = out;
    L.grid = grid;
    SPK_HIP(e->fn[dtype](L, s));
    if (!L.ticket) SPK_HIP(launch_dot_final(partial, grid, out, s));
    return SPK_OK;
}

spk_status run_dot(spk_handle h, int dtype, int64_t n, const void *x, const void *y, double *out,
                   const spk_variant &v, hipStream_t s)
{
    const VecEntry *e = nullptr;
    int64_t g = 0;
    SPK_TRY(dot_plan(h, dtype, n, x, y, v, &e, &g));
    DotScratch *d = nullptr;
    SPK_TRY(dot_scratch(h, s, g, &d));
    return dot_launch(e, dtype, n, x, y, out, g, d->partial, d->ticket, s);
}

// Scratch of spk_dot_noalloc, one copy per GPU for the life of the process:
// kNoAllocPartials workgroup partials, then one 256-byte line whose first
// word is the dot's ticket.  Host code reaches it only through the address
// spk_create stores in the handle (hipGetSymbolAddress on the handle's
// device); the array's name in host code is not a device address.
constexpr int64_t kNoAllocPartials = 65536;
static __device__ __align__(256) double scratch[kNoAllocPartials + 32];

// ----------------------------------------------------------------- SpMV --

// Row boundaries splitting [0, m) into `parts` pieces of similar nnz.
static std::vector<int64_t> split_rows(const spk_mat *A, int64_t m, int parts, int align)
{
    std::vector<int64_t> cut(parts + 1, 0);
    cut[parts] = m;
    for (int i = 1; i < parts; ++i) {
        int64_t r;
        if (A && !A->rp_host.empty()) {
            const int64_t target = (int64_t)((double)A->nnz * i / parts);
            r = std::lower_bound(A->rp_host.begin(), A->rp_host.end(), (int32_t)target) - A->rp_host.begin();
        } else {
            r = m * i / parts;
        }
        r = (r / align) * align;
        cut[i] = std::max(cut[i - 1], std::min(r, m));
    }
    return cut;
}

template <typename T>
static void fill_args(SpmvArgs<T> &a, const SpmvProblem &p, const int32_t *rp, const int32_t *ci, const void *val)
{
    a.rp = rp;
    a.ci = ci;
    a.val = (const T *)val;
    a.x = (const T *)p.x;
    a.y = (T *)p.y;
    a.w = (T *)p.w;
    a.alpha = (T)p.alpha;
}

spk_status run_spmv(spk_handle h, const SpmvProblem &p, const spk_variant &v, hipStream_t s)
{
    const int64_t m = p.mat ? p.mat->nrows : p.csr->nrows;
    const int dtype = p.mat ? p.mat->dtype : p.csr->dtype;
    if (m == 0) return SPK_OK;
    if (v.format == SPK_FMT_DIA || v.format == SPK_FMT_STENCIL) return run_structured(h, p, v, s);
    if (v.format == SPK_FMT_COLBLOCK) return run_colblock(h, p, v, s);
    if (v.format == SPK_FMT_XWIN) return run_xwin(h, p, v, s);
    const SpmvEntry *e = find_spmv_entry(v);
    if (!e) return fail(SPK_ERR_NOT_FOUND, "SpMV variant not compiled");
    if (!p.mat && (v.format == SPK_FMT_SELL || v.format == SPK_FMT_ADAPTIVE))
        return fail(SPK_ERR_ARG, "format %d needs a registered matrix", v.format);
    const int32_t *rp = p.mat ? p.mat->rp : p.csr->row_ptr;
    const int32_t *ci = p.mat ? p.mat->ci : p.csr->col_idx;
    const void *val = p.mat ? p.mat->val : p.csr->val;
    if (e->vec > 1 && e->format != SPK_FMT_ADAPTIVE &&
        ((uintptr_t)val % ((size_t)e->vec * dtype_size(dtype)) != 0 ||
                       (uintptr_t)ci % ((size_t)e->vec * 4) != 0)) {
        // wider accesses need arrays aligned to their width: one entry at a time
        spk_variant v1 = v;
        v1.vec = 0;
        v1.unroll = 1;
        if (v.format == SPK_FMT_VECTOR) v1.unroll = 2;
        const SpmvEntry *e1 = find_spmv_entry(v1);
        if (e1) e = e1;
    }
    SpmvFn fn = e->fn[dtype][p.fused ? 1 : 0];

    SellData *sd = nullptr;
    BlockData *bd = nullptr;
    if (v.format == SPK_FMT_SELL) SPK_TRY(get_sell(h, p.mat, v.group, &sd));
    if (v.format == SPK_FMT_ADAPTIVE) {
        SPK_TRY(get_blocks(h, p.mat, v.lds, &bd));
        if (v.group > 1) SPK_TRY(get_block_windows(h, p.mat, bd));
        if (e->vec == 2) SPK_TRY(get_block_c16(h, p.mat, bd));
    }

    const int parts = std::max(1, v.streams);
    // launch pieces: rows [cut[i], cut[i+1]) or row blocks for ADAPTIVE
    std::vector<int64_t> cut;
    if (v.format == SPK_FMT_ADAPTIVE) {
        cut.assign(parts + 1, 0);
        for (int i = 0; i <= parts; ++i) cut[i] = (int64_t)bd->nblk * i / parts;
    } else {
        cut = split_rows(p.mat, m, parts, v.format == SPK_FMT_SELL ? v.group : 1);
    }

    // Rows (or ADAPTIVE row blocks) covered by one workgroup.  A range whose
    // launch would exceed kMaxLaunchItems work-items (e.g. a wavefront per
    // row over more than 2^24 rows) is run as consecutive launches.
    const int64_t unit = v.format == SPK_FMT_ADAPTIVE ? v.block / 64
                         : v.format == SPK_FMT_VECTOR ? v.block / v.group : v.block;
    const int64_t span = kMaxLaunchItems / v.block * unit;

    auto launch_range = [&](int64_t lo, int64_t hi, hipStream_t st) -> spk_status {
        union {
            SpmvArgs<float> f;
            SpmvArgs<double> d;
        } args;
        memset(&args, 0, sizeof args);
        dim3 grid;
        auto setup = [&](auto &a) {
            using A = std::remove_reference_t<decltype(a)>;
            using T = std::remove_pointer_t<decltype(A::val)>;
            fill_args<std::remove_const_t<T>>(a, p, rp, ci, val);
            if (v.format == SPK_FMT_ADAPTIVE) {
                a.blocks = bd->blk;
                a.block_k = bd->bk;
                a.block_x = v.group > 1 ? bd->bx : nullptr;
                a.c16 = e->vec == 2 ? bd->c16 : nullptr;
                a.block_c16 = e->vec == 2 ? bd->cbase : nullptr;
                a.blk0 = (int32_t)lo;
                a.nblk = (int32_t)(hi - lo);   // one wavefront tile per wavefront
            } else {
                a.row0 = (int32_t)lo;
                a.m = (int32_t)(hi - lo);
                if (sd) {
                    a.sell_ptr = sd->ptr;
                    a.sell_len = sd->len;
                    a.sell_ci = sd->ci;
                    a.sell_val = (decltype(a.sell_val))sd->val;
                }
            }
        };
        if (dtype == SPK_F64) setup(args.d); else setup(args.f);
        grid = dim3((unsigned)((hi - lo + unit - 1) / unit));
        SPK_HIP(fn(dtype == SPK_F64 ? (const void *)&args.d : (const void *)&args.f, grid, st));
        return SPK_OK;
    };
    auto launch_piece = [&](int i, hipStream_t st) -> spk_status {
        for (int64_t lo = cut[i]; lo < cut[i + 1]; lo += span)
            SPK_TRY(launch_range(lo, std::min(cut[i + 1], lo + span), st));
        return SPK_OK;
    };

    if (parts == 1) return launch_piece(0, s);
    // fork onto the handle's streams and join back on the caller's stream
    SPK_HIP(hipEventRecord(h->ev_fork, s));
    for (int i = 0; i < parts; ++i) {
        SPK_HIP(hipStreamWaitEvent(h->sub[i], h->ev_fork, 0));
        SPK_TRY(launch_piece(i, h->sub[i]));
        SPK_HIP(hipEventRecord(h->ev_join[i], h->sub[i]));
        SPK_HIP(hipStreamWaitEvent(s, h->ev_join[i], 0));
    }
    return SPK_OK;
}

// ------------------------------------------------------ derived formats --

int64_t sell_padded_entries(const spk_mat *A, int C)
{
    int64_t total = 0;
    for (int64_t s0 = 0; s0 < A->nrows; s0 += C) {
        int64_t wmax = 0;
        const int64_t s1 = std::min<int64_t>(A->nrows, s0 + C);
        for (int64_t r = s0; r < s1; ++r) wmax = std::max<int64_t>(wmax, A->rp_host[r + 1] - A->rp_host[r]);
        total += wmax * C;
    }
    return total;
}

spk_status get_sell(spk_handle h, spk_mat *A, int C, SellData **out)
{
    std::lock_guard<std::mutex> lk(h->mu);
    auto it = A->sell.find(C);
    if (it != A->sell.end()) {
        *out = &it->second;
        return SPK_OK;
    }
    SellData d;
    d.C = C;
    d.nslices = (A->nrows + C - 1) / C;
    std::vector<int64_t> ptr(d.nslices + 1, 0);
    for (int64_t s = 0; s < d.nslices; ++s) {
        int64_t wmax = 0;
        const int64_t r1 = std::min<int64_t>(A->nrows, (s + 1) * C);
        for (int64_t r = s * C; r < r1; ++r) wmax = std::max<int64_t>(wmax, A->rp_host[r + 1] - A->rp_host[r]);
        ptr[s + 1] = ptr[s] + wmax * C;
    }
    d.padded = ptr[d.nslices];
    const size_t vs = dtype_size(A->dtype);
    SPK_HIP(hipMalloc(&d.ptr, sizeof(int64_t) * (d.nslices + 1)));
    SPK_HIP(hipMalloc(&d.len, sizeof(int32_t) * std::max<int64_t>(1, A->nrows)));
    SPK_HIP(hipMalloc(&d.ci, sizeof(int32_t) * std::max<int64_t>(1, d.padded)));
    SPK_HIP(hipMalloc(&d.val, vs * std::max<int64_t>(1, d.padded)));
    // everything on the handle's work stream, in order, then wait
    SPK_HIP(hipMemcpyAsync(d.ptr, ptr.data(), sizeof(int64_t) * (d.nslices + 1), hipMemcpyHostToDevice, h->work));
    SPK_HIP(hipMemsetAsync(d.ci, 0, sizeof(int32_t) * std::max<int64_t>(1, d.padded), h->work));
    SPK_HIP(hipMemsetAsync(d.val, 0, vs * std::max<int64_t>(1, d.padded), h->work));
    SPK_HIP(launch_csr_to_sell(A->dtype, (int32_t)A->nrows, C, A->rp, A->ci, A->val, d.ptr, d.len, d.ci, d.val,
                               h->work));
    SPK_HIP(hipStreamSynchronize(h->work));
    d.bytes = (int64_t)(sizeof(int64_t) * (d.nslices + 1) + 4 * A->nrows + (4 + vs) * d.padded);
    A->bytes += d.bytes;
    auto res = A->sell.emplace(C, d);
    *out = &res.first->second;
    return SPK_OK;
}

spk_status get_blocks(spk_handle h, spk_mat *A, int entries, BlockData **out)
{
    std::lock_guard<std::mutex> lk(h->mu);
    const auto key = std::make_pair(0, entries);
    auto it = A->blocks.find(key);
    if (it != A->blocks.end()) {
        *out = &it->second;
        return SPK_OK;
    }
    BlockData d;
    make_blocks(A->rp_host.data(), A->nrows, entries, d.host, d.host_k);
    d.nblk = (int32_t)d.host.size() - 1;
    SPK_HIP(hipMalloc(&d.blk, sizeof(uint32_t) * d.host.size()));
    SPK_HIP(hipMalloc(&d.bk, sizeof(int32_t) * d.host_k.size()));
    SPK_HIP(hipMemcpyAsync(d.blk, d.host.data(), sizeof(uint32_t) * d.host.size(), hipMemcpyHostToDevice, h->work));
    SPK_HIP(hipMemcpyAsync(d.bk, d.host_k.data(), sizeof(int32_t) * d.host_k.size(), hipMemcpyHostToDevice,
                           h->work));
    SPK_HIP(hipStreamSynchronize(h->work));
    d.bytes = (int64_t)(sizeof(uint32_t) * d.host.size() + sizeof(int32_t) * d.host_k.size());
    A->bytes += d.bytes;
    auto res = A->blocks.emplace(key, std::move(d));
    *out = &res.first->second;
    return SPK_OK;
}

// The x windows of a matrix's row-stream blocks (room for 256 entries),
// made on the device when a variant with room for x first needs them.
spk_status get_block_windows(spk_handle h, spk_mat *A, BlockData *bd)
{
    std::lock_guard<std::mutex> lk(h->mu);
    if (bd->bx) return SPK_OK;
    int32_t *bx = nullptr;
    SPK_HIP(hipMalloc(&bx, sizeof(int32_t) * 2 * (size_t)std::max(1, bd->nblk)));
    hipError_t e = launch_block_windows(bd->blk, bd->bk, A->ci, bd->nblk, 256, bx, h->work);
    if (e == hipSuccess) e = hipStreamSynchronize(h->work);
    if (e != hipSuccess) {
        (void)hipFree(bx);
        return hip_fail(e, "block windows");
    }
    bd->bx = bx;
    A->bytes += (int64_t)(sizeof(int32_t) * 2 * (size_t)bd->nblk);
    return SPK_OK;
}

// Two-byte columns of a matrix's row-stream blocks, made on the device when
// a variant that reads them first needs them (nnz + 8 entries: the kernel
// reads whole aligned 16-byte groups).
spk_status get_block_c16(spk_handle h, spk_mat *A, BlockData *bd)
{
    std::lock_guard<std::mutex> lk(h->mu);
    if (bd->cbase) return SPK_OK;
    uint16_t *c16 = nullptr;
    int32_t *base = nullptr;
    const size_t nc = (size_t)std::max<int64_t>(0, A->nnz) + 8;
    SPK_HIP(hipMalloc(&c16, sizeof(uint16_t) * nc));
    hipError_t e = hipMalloc(&base, sizeof(int32_t) * (size_t)std::max(1, bd->nblk));
    if (e == hipSuccess) e = launch_block_c16(bd->blk, bd->bk, A->ci, bd->nblk, c16, base, h->work);
    if (e == hipSuccess) e = hipStreamSynchronize(h->work);
    if (e != hipSuccess) {
        (void)hipFree(c16);
        if (base) (void)hipFree(base);
        return hip_fail(e, "two-byte columns");
    }
    bd->c16 = c16;
    bd->cbase = base;
    A->bytes += (int64_t)(sizeof(uint16_t) * nc + sizeof(int32_t) * (size_t)bd->nblk);
    return SPK_OK;
}

// ------------------------------------------------------- column blocks --

// Frees a matrix and everything derived from it.
static void free_mat(spk_mat *A)
{
    (void)hipFree(A->rp);
    (void)hipFree(A->ci);
    (void)hipFree(A->val);
    for (auto &kv : A->sell) {
        (void)hipFree(kv.second.ptr);
        (void)hipFree(kv.second.len);
        (void)hipFree(kv.second.ci);
        (void)hipFree(kv.second.val);
    }
    for (auto &kv : A->blocks) {
        (void)hipFree(kv.second.blk);
        (void)hipFree(kv.second.bk);
        if (kv.second.bx) (void)hipFree(kv.second.bx);
        if (kv.second.c16) (void)hipFree(kv.second.c16);
        if (kv.second.cbase) (void)hipFree(kv.second.cbase);
    }
    if (A->dia.val) (void)hipFree(A->dia.val);
    if (A->dia.mask) (void)hipFree(A->dia.mask);
    for (auto &kv : A->colblk) {
        for (spk_mat *S : kv.second.sub) free_mat(S);
        for (auto &pp : kv.second.part) (void)hipFree(pp.second);
    }
    for (auto &kv : A->xwin) free_xwin(kv.second);
    delete A;
}

// Sub-matrices of A by column range ([b*n/nblk, (b+1)*n/nblk) for block b),
// each holding every row, built from a host copy of A's entries; they are
// owned by A, not listed with the handle's matrices.
static spk_status get_colblock(spk_handle h, spk_mat *A, int nblk, ColBlockData **out)
{
    {
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = A->colblk.find(nblk);
        if (it != A->colblk.end()) {
            *out = &it->second;
            return SPK_OK;
        }
    }
    const int64_t m = A->nrows, n = A->ncols, nnz = A->nnz;
    std::vector<int32_t> ci((size_t)std::max<int64_t>(1, nnz));
    std::vector<double> val((size_t)std::max<int64_t>(1, nnz));
    if (nnz > 0) {
        SPK_HIP(hipDeviceSynchronize());
        SPK_HIP(hipMemcpy(ci.data(), A->ci, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
        SPK_HIP(hipMemcpy(val.data(), A->val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    }
    ColBlockData d;
    auto bail = [&](spk_status st) {
        for (spk_mat *S : d.sub) free_mat(S);
        return st;
    };
    const std::vector<int32_t> &rp = A->rp_host;
    for (int b = 0; b < nblk; ++b) {
        const int64_t lo = n * b / nblk, hi = n * (b + 1) / nblk;
        std::vector<int32_t> srp((size_t)m + 1, 0), sci;
        std::vector<double> sval;
        for (int64_t i = 0; i < m; ++i) {
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                if (ci[k] >= lo && ci[k] < hi) {
                    sci.push_back(ci[k]);
                    sval.push_back(val[k]);
                }
            srp[i + 1] = (int32_t)sci.size();
        }
        spk_csr view{m, n, (int64_t)sci.size(), SPK_F64, srp.data(), sci.empty() ? nullptr : sci.data(),
                     sval.empty() ? nullptr : sval.data()};
        spk_matrix S = nullptr;
        const spk_status st = spk_matrix_register(h, &view, 0, 0, &S);
        if (st != SPK_OK) return bail(st);
        {
            std::lock_guard<std::mutex> lk(h->mu);
            h->mats.erase(S);
        }
        d.sub.push_back(S);
    }
    std::lock_guard<std::mutex> lk(h->mu);
    auto it = A->colblk.find(nblk);
    if (it != A->colblk.end()) {
        for (spk_mat *S : d.sub) free_mat(S);   // built meanwhile by another call
        *out = &it->second;
        return SPK_OK;
    }
    for (spk_mat *S : d.sub) A->bytes += S->bytes;
    *out = &A->colblk.emplace(nblk, std::move(d)).first->second;
    return SPK_OK;
}

spk_status run_colblock(spk_handle h, const SpmvProblem &p, const spk_variant &v, hipStream_t s)
{
    spk_mat *A = p.mat;
    if (!A) return fail(SPK_ERR_ARG, "the column-blocked form needs a registered matrix");
    if (A->dtype != SPK_F64) return fail(SPK_ERR_DTYPE, "the column-blocked form is FP64 only");
    const int nblk = v.group;
    const int64_t m = A->nrows;
    ColBlockData *cb = nullptr;
    SPK_TRY(get_colblock(h, A, nblk, &cb));
    double *part = nullptr;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = cb->part.find(s);
        if (it != cb->part.end()) part = it->second;
    }
    if (!part) {
        SPK_HIP(hipMalloc(&part, sizeof(double) * (size_t)nblk * (size_t)m));
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = cb->part.find(s);
        if (it != cb->part.end()) {
            (void)hipFree(part);   // made meanwhile by another call on this stream
            part = it->second;
        } else {
            cb->part[s] = part;
            A->bytes += (int64_t)(sizeof(double) * (size_t)nblk * (size_t)m);
        }
    }
    const spk_variant iv = colblock_inner(v);
    for (int b = 0; b < nblk; ++b) {
        SpmvProblem q;
        q.mat = cb->sub[b];
        q.fused = false;
        q.x = p.x;
        q.y = part + (int64_t)b * m;
        SPK_TRY(run_spmv(h, q, iv, s));
    }
    SPK_HIP(launch_colblock_sum(nblk, m, part, (double *)p.y, p.fused ? (double *)p.w : nullptr, (const double *)p.x,
                                p.alpha, s));
    return SPK_OK;
}

// --------------------------------------------------------------- plan DB --

void db_load(spk_handle h)
{
    if (h->db_path.empty()) return;
    std::ifstream f(h->db_path);
    std::string line;
    while (std::getline(f, line)) {
        char key[128] = {0}, arch[64] = {0}, build[64] = {0};
        spk_variant v{};
        double us = 0;
        const int got = sscanf(line.c_str(),
                               "{\"key\": \"%127[^\"]\", \"arch\": \"%63[^\"]\", \"build\": \"%63[^\"]\", "
                               "\"v\": [%d, %d, %d, %d, %d, %d, %d, %d], \"us\": %lf}",
                               key, arch, build, &v.format, &v.block, &v.group, &v.unroll, &v.vec, &v.grid,
                               &v.streams, &v.lds, &us);
        if (got == 12) {
            if (strcmp(arch, h->arch) != 0 || strcmp(build, SPK_BUILD_ID) != 0) continue;
            h->plans[key] = v;
            continue;
        }
        char point[256] = {0};
        const int gp = sscanf(line.c_str(),
                              "{\"point\": \"%255[^\"]\", \"arch\": \"%63[^\"]\", \"build\": \"%63[^\"]\", "
                              "\"v\": [%d, %d, %d, %d, %d, %d, %d, %d], \"us\": %lf}",
                              point, arch, build, &v.format, &v.block, &v.group, &v.unroll, &v.vec, &v.grid,
                              &v.streams, &v.lds, &us);
        if (gp != 12 || strcmp(arch, h->arch) != 0 || strcmp(build, SPK_BUILD_ID) != 0) continue;
        h->points[point].emplace_back(v, us);
    }
}

uint64_t fnv1a(const void *p, size_t n, uint64_t seed)
{
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) seed = (seed ^ b[i]) * 1099511628211ull;
    return seed;
}

static bool same_variant(const spk_variant &a, const spk_variant &b)
{
    return a.format == b.format && a.block == b.block && a.group == b.group && a.unroll == b.unroll &&
           a.vec == b.vec && a.grid == b.grid && a.streams == b.streams && a.lds == b.lds;
}

bool point_get(spk_handle h, const std::string &key, const spk_variant &v, double *us)
{
    std::lock_guard<std::mutex> lk(h->mu);
    auto it = h->points.find(key);
    if (it == h->points.end()) return false;
    for (const auto &pv : it->second)
        if (same_variant(pv.first, v)) {
            *us = pv.second;
            return true;
        }
    return false;
}

void point_put(spk_handle h, const std::string &key, const spk_variant &v, double us)
{
    {
        std::lock_guard<std::mutex> lk(h->mu);
        h->points[key].emplace_back(v, us);
    }
    if (h->db_path.empty()) return;
    FILE *f = fopen(h->db_path.c_str(), "a");
    if (!f) return;
    // one line per point, written whole, so a search cut short keeps every
    // point measured before the cut
    fprintf(f,
            "{\"point\": \"%s\", \"arch\": \"%s\", \"build\": \"%s\", \"v\": [%d, %d, %d, %d, %d, %d, %d, %d], "
            "\"us\": %.17g}\n",
            key.c_str(), h->arch, SPK_BUILD_ID, v.format, v.block, v.group, v.unroll, v.vec, v.grid, v.streams, v.lds,
            us);
    fclose(f);
}

void db_append(spk_handle h, const std::string &key, const spk_variant &v, double us)
{
    if (h->db_path.empty()) return;
    FILE *f = fopen(h->db_path.c_str(), "a");
    if (!f) return;
    fprintf(f,
            "{\"key\": \"%s\", \"arch\": \"%s\", \"build\": \"%s\", \"v\": [%d, %d, %d, %d, %d, %d, %d, %d], "
            "\"us\": %.3f}\n",
            key.c_str(), h->arch, SPK_BUILD_ID, v.format, v.block, v.group, v.unroll, v.vec, v.grid, v.streams, v.lds,
            us);
    fclose(f);
}

spk_status resolve(spk_handle h, const spk_problem &p, const spk_csr *csr, spk_variant *v)
{
    if (h->plain) {
        *v = plain_variant(p.op, 0);
        if ((p.op == SPK_OP_SPMV || p.op == SPK_OP_SPMV_WAXPY) && csr && csr->nrows > 0 &&
            (double)csr->nnz / (double)csr->nrows > 8.0)
            *v = plain_variant(p.op, 1);
        if ((p.op == SPK_OP_SPMV || p.op == SPK_OP_SPMV_WAXPY) && p.A && p.A->mean_len > 8.0)
            *v = plain_variant(p.op, 1);
        return SPK_OK;
    }
    const std::string key = class_key(p, csr);
    {
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = h->plans.find(key);
        if (it != h->plans.end()) {
            *v = it->second;
            return SPK_OK;
        }
    }
    *v = default_variant(h, p, csr);
    return SPK_OK;
}

}  // namespace spk

using namespace spk;

// ================================================================= C ABI ==

extern "C" {

int spk_abi_version(void) { return SPK_ABI_VERSION; }

const char *spk_status_str(spk_status s)
{
    switch (s) {
    case SPK_OK: return "SPK_OK";
    case SPK_ERR_NULL: return "SPK_ERR_NULL";
    case SPK_ERR_SHAPE: return "SPK_ERR_SHAPE";
    case SPK_ERR_DTYPE: return "SPK_ERR_DTYPE";
    case SPK_ERR_ALIAS: return "SPK_ERR_ALIAS";
    case SPK_ERR_CSR: return "SPK_ERR_CSR";
    case SPK_ERR_OOM: return "SPK_ERR_OOM";
    case SPK_ERR_BUDGET: return "SPK_ERR_BUDGET";
    case SPK_ERR_HIP: return "SPK_ERR_HIP";
    case SPK_ERR_VALIDATION: return "SPK_ERR_VALIDATION";
    case SPK_ERR_NOT_FOUND: return "SPK_ERR_NOT_FOUND";
    case SPK_ERR_ARG: return "SPK_ERR_ARG";
    case SPK_ERR_STATE: return "SPK_ERR_STATE";
    case SPK_ERR_INTERRUPTED: return "SPK_ERR_INTERRUPTED";
    }
    return "SPK_ERR_UNKNOWN";
}

const char *spk_last_error(void) { return g_err; }

spk_status spk_create(int device, const char *db_path, spk_handle *out)
{
    if (!out) return fail(SPK_ERR_NULL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    SPK_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(SPK_ERR_ARG, "device %d not present (%d devices)", device, ndev);
    spk_ctx *h = new spk_ctx();
    h->device = device;
    int prev = 0;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(device);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipGetDeviceProperties");
    }
    h->num_cu = prop.multiProcessorCount;
    snprintf(h->name, sizeof h->name, "%s", prop.name);
    snprintf(h->arch, sizeof h->arch, "%s", prop.gcnArchName);
    char *colon = strchr(h->arch, ':');
    if (colon) *colon = 0;
    const char *plain = getenv("SPK_PLAIN");
    h->plain = plain && plain[0] == '1';
    if (db_path && db_path[0]) h->db_path = db_path;
    else if (getenv("SPK_DB_PATH")) h->db_path = getenv("SPK_DB_PATH");
    for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&h->sub[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->work, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
    for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&h->ev_join[i], hipEventDisableTiming);
    // this device's copy of the allocation-free dot's scratch
    if (e == hipSuccess) e = hipGetSymbolAddress((void **)&h->noalloc_scratch, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        spk_status s = hip_fail(e, "stream/event creation");
        delete h;
        return s;
    }
    db_load(h);
    *out = h;
    return SPK_OK;
}

spk_status spk_destroy(spk_handle h)
{
    if (!h) return fail(SPK_ERR_NULL, "handle is NULL");
    DeviceGuard g(h);
    (void)hipDeviceSynchronize();
    for (spk_mat *A : h->mats) free_mat(A);
    for (auto &kv : h->dot) {
        (void)hipFree(kv.second.partial);
        (void)hipFree(kv.second.ticket);
    }
    for (auto &kv : h->cg) {
        (void)hipFree(kv.second.vec);
        (void)hipFree(kv.second.part);
        (void)hipFree(kv.second.sc);
    }
    if (h->flush_buf) (void)hipFree(h->flush_buf);
    for (int i = 0; i < 4; ++i) {
        if (h->sub[i]) (void)hipStreamDestroy(h->sub[i]);
        if (h->ev_join[i]) (void)hipEventDestroy(h->ev_join[i]);
    }
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->work) (void)hipStreamDestroy(h->work);
    delete h;
    return SPK_OK;
}

spk_status spk_check(spk_handle h, spk_stream stream)
{
    if (!h) return fail(SPK_ERR_NULL, "handle is NULL");
    DeviceGuard g(h);
    SPK_HIP(hipStreamSynchronize((hipStream_t)stream));
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

spk_status spk_set_plain(spk_handle h, int plain)
{
    if (!h) return fail(SPK_ERR_NULL, "handle is NULL");
    h->plain = plain != 0;
    return SPK_OK;
}

spk_status spk_device_info(spk_handle h, int32_t *num_cu, char *name, int32_t name_cap)
{
    if (!h) return fail(SPK_ERR_NULL, "handle is NULL");
    if (num_cu) *num_cu = h->num_cu;
    if (name && name_cap > 0) snprintf(name, (size_t)name_cap, "%s (%s)", h->name, h->arch);
    return SPK_OK;
}

// ----------------------------------------------------------- vector ops --


spk_status spk_waxpy(spk_handle h, int32_t dtype, int64_t n, double alpha, const void *x, const void *y, void *w,
                     spk_stream stream)
{
    if (!h) return fail(SPK_ERR_NULL, "handle is NULL");
    if (!dtype_ok(dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", dtype);
    if (n < 0) return fail(SPK_ERR_SHAPE, "n = %lld < 0", (long long)n);
    if (n == 0) return SPK_OK;
    if (!x || !y || !w) return fail(SPK_ERR_NULL, "x, y and w must be non-NULL");
    const size_t nb = (size_t)n * dtype_size(dtype);
    if ((w != x && overlaps(w, nb, x, nb)) || (w != y && overlaps(w, nb, y, nb)))
        return fail(SPK_ERR_ALIAS, "w partially overlaps x or y");
    spk_problem p{};
    p.op = SPK_OP_WAXPY;
    p.dtype = dtype;
    p.n = n;
    spk_variant v;
    SPK_TRY(resolve(h, p, nullptr, &v));
    DeviceGuard g(h);
    return run_waxpy(h, dtype, n, alpha, x, y, w, v, (hipStream_t)stream);
}

spk_status spk_axpy(spk_handle h, int32_t dtype, int64_t n, double alpha, const void *x, void *y, spk_stream stream)
{
    if (!h) return fail(SPK_ERR_NULL, "handle is NULL");
    if (!dtype_ok(dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", dtype);
    if (n < 0) return fail(SPK_ERR_SHAPE, "n = %lld < 0", (long long)n);
    if (n == 0) return SPK_OK;
    if (!x || !y) return fail(SPK_ERR_NULL, "x and y must be non-NULL");
    const size_t nb = (size_t)n * dtype_size(dtype);
    if (x != y && overlaps(x, nb, y, nb)) return fail(SPK_ERR_ALIAS, "y partially overlaps x");
    spk_problem p{};
    p.op = SPK_OP_AXPY;
    p.dtype = dtype;
    p.n = n;
    spk_variant v;
    SPK_TRY(resolve(h, p, nullptr, &v));
    DeviceGuard g(h);
    return run_waxpy(h, dtype, n, alpha, x, y, y, v, (hipStream_t)stream);
}

spk_status spk_dot(spk_handle h, int32_t dtype, int64_t n, const void *x, const void *y, double *d_result,
                   spk_stream stream)
{
    if (!h) return fail(SPK_ERR_NULL, "handle is NULL");
    if (!dtype_ok(dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", dtype);
    if (n < 0) return fail(SPK_ERR_SHAPE, "n = %lld < 0", (long long)n);
    if (!d_result) return fail(SPK_ERR_NULL, "d_result is NULL");
    if (n > 0 && (!x || !y)) return fail(SPK_ERR_NULL, "x and y must be non-NULL");
    const size_t nb = (size_t)n * dtype_size(dtype);
    if (overlaps(d_result, 8, x, nb) || overlaps(d_result, 8, y, nb))
        return fail(SPK_ERR_ALIAS, "d_result overlaps x or y");
    spk_problem p{};
    p.op = SPK_OP_DOT;
    p.dtype = dtype;
    p.n = n;
    spk_variant v;
    SPK_TRY(resolve(h, p, nullptr, &v));
    DeviceGuard g(h);
    return run_dot(h, dtype, n, x, y, d_result, v, (hipStream_t)stream);
}

spk_status spk_dot_noalloc(spk_handle h, int32_t dtype, int64_t n, const void *x, const void *y, double *d_result,
                           spk_stream stream)
{
    if (!h) return fail(SPK_ERR_NULL, "handle is NULL");
    if (!dtype_ok(dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", dtype);
    if (n < 0) return fail(SPK_ERR_SHAPE, "n = %lld < 0", (long long)n);
    if (!d_result) return fail(SPK_ERR_NULL, "d_result is NULL");
    if (n > 0 && (!x || !y)) return fail(SPK_ERR_NULL, "x and y must be non-NULL");
    if (!h->noalloc_scratch) return fail(SPK_ERR_HIP, "the device scratch of this handle is not set up");
    const size_t nb = (size_t)n * dtype_size(dtype);
    if (overlaps(d_result, 8, x, nb) || overlaps(d_result, 8, y, nb))
        return fail(SPK_ERR_ALIAS, "d_result overlaps x or y");
    spk_problem p{};
    p.op = SPK_OP_DOT;
    p.dtype = dtype;
    p.n = n;
    spk_variant v;
    SPK_TRY(resolve(h, p, nullptr, &v));
    const VecEntry *e = nullptr;
    int64_t g = 0;
    SPK_TRY(dot_plan(h, dtype, n, x, y, v, &e, &g));
    if (g > kNoAllocPartials)
        return fail(SPK_ERR_SHAPE,
                    "this dot (n = %lld, block %d, vec %d, unroll %d, grid %d) needs %lld workgroup partials; "
                    "the allocation-free form holds at most %lld",
                    (long long)n, v.block, v.vec, v.unroll, v.grid, (long long)g, (long long)kNoAllocPartials);
    DeviceGuard dg(h);
    hipStream_t s = (hipStream_t)stream;
    uint32_t *ticket = nullptr;
    if (g <= kDotTicketMaxGrid) {
        // the array keeps the last call's contents: the ticket starts at zero
        // (a kernel, not a memset node, so the call can be captured)
        ticket = (uint32_t *)(h->noalloc_scratch + kNoAllocPartials);
        SPK_HIP(launch_zero_u32(ticket, 1, s));
    }
    return dot_launch(e, dtype, n, x, y, d_result, g, h->noalloc_scratch, ticket, s);
}

// ----------------------------------------------------------------- SpMV --

static spk_status check_csr_view(const spk_csr *A)
{
    if (!A) return fail(SPK_ERR_NULL, "A is NULL");
    if (!dtype_ok(A->dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", A->dtype);
    if (A->nrows < 0 || A->ncols < 0 || A->nnz < 0) return fail(SPK_ERR_SHAPE, "negative size");
    if (A->nnz >= (1ll << 31)) return fail(SPK_ERR_SHAPE, "nnz must be < 2^31 (int32 indices)");
    if (A->nrows >= (1ll << 30) || A->ncols >= (1ll << 31)) return fail(SPK_ERR_SHAPE, "matrix too large");
    if (A->nrows > 0 && !A->row_ptr) return fail(SPK_ERR_NULL, "row_ptr is NULL");
    if (A->nnz > 0 && (!A->col_idx || !A->val)) return fail(SPK_ERR_NULL, "col_idx/val are NULL");
    if (A->nnz > 0 && A->ncols == 0) return fail(SPK_ERR_SHAPE, "entries in a matrix with no columns");
    return SPK_OK;
}

spk_status spk_spmv_csr(spk_handle h, const spk_csr *A, const void *x, void *y, spk_stream stream)
{
    if (!h) return fail(SPK_ERR_NULL, "handle is NULL");
    SPK_TRY(check_csr_view(A));
    if (A->nrows == 0) return SPK_OK;
    if (!y || (A->ncols > 0 && !x)) return fail(SPK_ERR_NULL, "x/y are NULL");
    const size_t s = dtype_size(A->dtype);
    if (overlaps(x, (size_t)A->ncols * s, y, (size_t)A->nrows * s)) return fail(SPK_ERR_ALIAS, "y overlaps x");
    spk_problem p{};
    p.op = SPK_OP_SPMV;
    p.dtype = A->dtype;
    spk_variant v;
    SPK_TRY(resolve(h, p, A, &v));
    // formats built from a registered matrix do not apply to a borrowed one
    if (v.format == SPK_FMT_SELL || v.format == SPK_FMT_ADAPTIVE || v.format == SPK_FMT_DIA ||
        v.format == SPK_FMT_STENCIL || v.format == SPK_FMT_COLBLOCK || v.format == SPK_FMT_XWIN)
        v = default_variant(h, p, A);
    SpmvProblem q;
    q.csr = A;
    q.x = x;
    q.y = y;
    DeviceGuard g(h);
    return run_spmv(h, q, v, (hipStream_t)stream);
}

spk_status spk_matrix_register(spk_handle h, const spk_csr *A, int32_t where, int32_t validate, spk_matrix *out)
{
    if (!h || !out) return fail(SPK_ERR_NULL, "handle/out is NULL");
    *out = nullptr;
    SPK_TRY(check_csr_view(A));
    if (where != 0 && where != 1) return fail(SPK_ERR_ARG, "where must be 0 (host) or 1 (device)");
    DeviceGuard g(h);
    const hipMemcpyKind kind = where == 0 ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    std::vector<int32_t> rp((size_t)A->nrows + 1, 0);
    if (A->nrows > 0) {
        if (where == 0) memcpy(rp.data(), A->row_ptr, sizeof(int32_t) * rp.size());
        else {
            SPK_HIP(hipDeviceSynchronize());  // the caller's pending writes to its arrays
            SPK_HIP(hipMemcpy(rp.data(), A->row_ptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost));
        }
    }
    if (validate) {
        if (rp[0] != 0) return fail(SPK_ERR_CSR, "row_ptr[0] = %d, expected 0", rp[0]);
        for (int64_t i = 0; i < A->nrows; ++i)
            if (rp[i + 1] < rp[i]) return fail(SPK_ERR_CSR, "row_ptr decreases at row %lld", (long long)i);
        if (rp[A->nrows] != A->nnz)
            return fail(SPK_ERR_CSR, "row_ptr[nrows] = %d, expected nnz = %lld", rp[A->nrows], (long long)A->nnz);
    }
    spk_mat *M = new spk_mat();
    M->h = h;
    M->nrows = A->nrows;
    M->ncols = A->ncols;
    M->nnz = A->nnz;
    M->dtype = A->dtype;
    M->rp_host = std::move(rp);
    const size_t vs = dtype_size(A->dtype);
    auto cleanup = [&](spk_status s) {
        free_mat(M);
        return s;
    };
    hipError_t e = hipMalloc(&M->rp, sizeof(int32_t) * (M->nrows + 1));
    if (e == hipSuccess) e = hipMalloc(&M->ci, sizeof(int32_t) * std::max<int64_t>(1, M->nnz));
    if (e == hipSuccess) e = hipMalloc(&M->val, vs * std::max<int64_t>(1, M->nnz));
    if (e == hipSuccess)
        e = hipMemcpyAsync(M->rp, M->rp_host.data(), sizeof(int32_t) * (M->nrows + 1), hipMemcpyHostToDevice, h->work);
    if (e == hipSuccess && M->nnz > 0) e = hipMemcpyAsync(M->ci, A->col_idx, sizeof(int32_t) * M->nnz, kind, h->work);
    if (e == hipSuccess && M->nnz > 0) e = hipMemcpyAsync(M->val, A->val, vs * M->nnz, kind, h->work);
    if (e == hipSuccess) e = hipStreamSynchronize(h->work);
    if (e != hipSuccess) return cleanup(hip_fail(e, "matrix upload"));
    if (validate && M->nnz > 0) {
        unsigned long long *bad = nullptr, hbad = 0;
        e = hipMalloc(&bad, sizeof *bad);
        if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof *bad, h->work);
        if (e == hipSuccess) e = launch_csr_colcheck(M->nnz, M->ci, M->ncols, bad, h->work);
        if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, h->work);
        if (e == hipSuccess) e = hipStreamSynchronize(h->work);
        (void)hipFree(bad);
        if (e != hipSuccess) return cleanup(hip_fail(e, "column check"));
        if (hbad) return cleanup(fail(SPK_ERR_CSR, "%llu column indices outside [0, %lld)", hbad, (long long)M->ncols));
    }
    // structured formats (DIA, stencil) need the entries on the host once
    if (M->nnz > 0) {
        if (where == 0) {
            detect_structure(M, A->col_idx, A->val);
        } else {
            std::vector<int32_t> ci_h((size_t)M->nnz);
            std::vector<char> val_h((size_t)M->nnz * vs);
            e = hipMemcpy(ci_h.data(), M->ci, sizeof(int32_t) * M->nnz, hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy(val_h.data(), M->val, vs * M->nnz, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return cleanup(hip_fail(e, "structure detection copy"));
            detect_structure(M, ci_h.data(), val_h.data());
        }
    }
    int64_t mx = 0;
    for (int64_t i = 0; i < M->nrows; ++i) mx = std::max<int64_t>(mx, M->rp_host[i + 1] - M->rp_host[i]);
    M->max_len = mx;
    M->mean_len = M->nrows ? (double)M->nnz / (double)M->nrows : 0.0;
    M->bytes = (int64_t)(4 * (M->nrows + 1) + (4 + vs) * M->nnz);
    {
        std::lock_guard<std::mutex> lk(h->mu);
        h->mats.insert(M);
    }
    *out = M;
    return SPK_OK;
}

spk_status spk_matrix_release(spk_handle h, spk_matrix A)
{
    if (!h || !A) return fail(SPK_ERR_NULL, "handle/matrix is NULL");
    {
        std::lock_guard<std::mutex> lk(h->mu);
        if (!h->mats.erase(A)) return fail(SPK_ERR_NOT_FOUND, "matrix not owned by this handle");
    }
    DeviceGuard g(h);
    (void)hipDeviceSynchronize();
    free_mat(A);
    return SPK_OK;
}

spk_status spk_matrix_bytes(spk_handle h, spk_matrix A, int64_t *bytes)
{
    if (!h || !A || !bytes) return fail(SPK_ERR_NULL, "NULL argument");
    *bytes = A->bytes;
    return SPK_OK;
}

static spk_status spmv_mat_common(spk_handle h, spk_matrix A, bool fused, double alpha, const void *x, void *y,
                                  void *w, spk_stream stream, const spk_variant *forced)
{
    if (!h || !A) return fail(SPK_ERR_NULL, "handle/matrix is NULL");
    if (A->nrows == 0) return SPK_OK;
    if (!y || (A->ncols > 0 && !x)) return fail(SPK_ERR_NULL, "x/y are NULL");
    const size_t s = dtype_size(A->dtype);
    if (overlaps(x, (size_t)A->ncols * s, y, (size_t)A->nrows * s)) return fail(SPK_ERR_ALIAS, "y overlaps x");
    if (fused) {
        if (A->nrows != A->ncols) return fail(SPK_ERR_SHAPE, "the fused step needs a square matrix");
        if (!w) return fail(SPK_ERR_NULL, "w is NULL");
        if (overlaps(w, (size_t)A->nrows * s, x, (size_t)A->ncols * s) ||
            overlaps(w, (size_t)A->nrows * s, y, (size_t)A->nrows * s))
            return fail(SPK_ERR_ALIAS, "w overlaps x or y");
    }
    spk_problem p{};
    p.op = fused ? SPK_OP_SPMV_WAXPY : SPK_OP_SPMV;
    p.dtype = A->dtype;
    p.A = A;
    spk_variant v;
    if (forced) {
        v = *forced;
        SPK_TRY(check_variant(p.op, A->dtype, v));
    } else {
        SPK_TRY(resolve(h, p, nullptr, &v));
        // a plan filed by hand may name a structured format A lacks
        if (!format_applies(A, v.format)) v = default_variant(h, p, nullptr);
    }
    SpmvProblem q;
    q.mat = A;
    q.fused = fused;
    q.alpha = alpha;
    q.x = x;
    q.y = y;
    q.w = w;
    DeviceGuard g(h);
    return run_spmv(h, q, v, (hipStream_t)stream);
}

spk_status spk_spmv_mat(spk_handle h, spk_matrix A, const void *x, void *y, spk_stream stream)
{
    return spmv_mat_common(h, A, false, 0.0, x, y, nullptr, stream, nullptr);
}

spk_status spk_spmv_waxpy(spk_handle h, spk_matrix A, double alpha, const void *x, void *y, void *w,
                          spk_stream stream)
{
    return spmv_mat_common(h, A, true, alpha, x, y, w, stream, nullptr);
}

// -------------------------------------------------- variants and plans --

spk_status spk_run(spk_handle h, const spk_problem *p, const spk_variant *variant, spk_stream stream)
{
    if (!h || !p) return fail(SPK_ERR_NULL, "handle/problem is NULL");
    switch (p->op) {
    case SPK_OP_WAXPY:
    case SPK_OP_AXPY:
    case SPK_OP_DOT: {
        if (!dtype_ok(p->dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", p->dtype);
        if (!variant) {
            if (p->op == SPK_OP_WAXPY) return spk_waxpy(h, p->dtype, p->n, p->alpha, p->x, p->y, p->w, stream);
            if (p->op == SPK_OP_AXPY) return spk_axpy(h, p->dtype, p->n, p->alpha, p->x, p->y, stream);
            return spk_dot(h, p->dtype, p->n, p->x, p->y, p->d_result, stream);
        }
        SPK_TRY(check_variant(p->op, p->dtype, *variant));
        if (p->n < 0) return fail(SPK_ERR_SHAPE, "n < 0");
        const size_t nb = (size_t)p->n * dtype_size(p->dtype);
        DeviceGuard g(h);
        if (p->op == SPK_OP_DOT) {
            if (!p->d_result || (p->n > 0 && (!p->x || !p->y))) return fail(SPK_ERR_NULL, "NULL operand");
            return run_dot(h, p->dtype, p->n, p->x, p->y, p->d_result, *variant, (hipStream_t)stream);
        }
        if (p->n == 0) return SPK_OK;
        void *w = p->op == SPK_OP_AXPY ? p->y : p->w;
        if (!p->x || !p->y || !w) return fail(SPK_ERR_NULL, "NULL operand");
        if ((w != p->x && overlaps(w, nb, p->x, nb)) || (w != p->y && overlaps(w, nb, p->y, nb)))
            return fail(SPK_ERR_ALIAS, "output partially overlaps an input");
        return run_waxpy(h, p->dtype, p->n, p->alpha, p->x, p->y, w, *variant, (hipStream_t)stream);
    }
    case SPK_OP_SPMV:
    case SPK_OP_SPMV_WAXPY:
        if (!p->A) return fail(SPK_ERR_NULL, "problem.A is NULL");
        return spmv_mat_common(h, p->A, p->op == SPK_OP_SPMV_WAXPY, p->alpha, p->x, p->y, p->w, stream, variant);
    default:
        return fail(SPK_ERR_ARG, "unknown op %d", p->op);
    }
}

static void vec_space(int op, int dtype, std::vector<spk_variant> &out)
{
    static const int grids[] = {0, 1, 2, 4, 8, 16, 32};
    int n = 0;
    const VecEntry *t = op == SPK_OP_DOT ? dot_table(&n) : waxpy_table(&n);
    // plain variant first
    out.push_back(plain_variant(op, 0));
    for (int i = 0; i < n; ++i) {
        if (!t[i].fn[dtype]) continue;
        if ((size_t)t[i].vec * dtype_size(dtype) > 16) continue;
        for (int g : grids) {
            spk_variant v{};
            v.block = t[i].block;
            v.vec = t[i].vec;
            v.unroll = t[i].unroll;
            v.grid = g;
            if (v.block == 256 && v.vec == 1 && v.unroll == 1 && v.grid == 0) continue;
            out.push_back(v);
        }
    }
}

static void spmv_space(std::vector<spk_variant> &out)
{
    int n = 0;
    const SpmvEntry *t = spmv_table(&n);
    for (int i = 0; i < n; ++i) {
        spk_variant v{};
        v.format = t[i].format;
        v.block = t[i].block;
        v.group = t[i].group;
        v.unroll = t[i].unroll;
        v.lds = t[i].lds;
        v.vec = t[i].vec > 1 ? t[i].vec : 0;
        v.streams = 1;
        out.push_back(v);
    }
}

spk_status spk_variant_count(int32_t op, int32_t dtype, int32_t *count)
{
    if (!count) return fail(SPK_ERR_NULL, "count is NULL");
    if (!dtype_ok(dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", dtype);
    std::vector<spk_variant> s;
    if (op == SPK_OP_SPMV || op == SPK_OP_SPMV_WAXPY) spmv_space(s);
    else if (op == SPK_OP_WAXPY || op == SPK_OP_AXPY || op == SPK_OP_DOT) vec_space(op, dtype, s);
    else return fail(SPK_ERR_ARG, "unknown op %d", op);
    *count = (int32_t)s.size();
    return SPK_OK;
}

spk_status spk_variant_get(int32_t op, int32_t dtype, int32_t index, spk_variant *out)
{
    if (!out) return fail(SPK_ERR_NULL, "out is NULL");
    if (!dtype_ok(dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", dtype);
    std::vector<spk_variant> s;
    if (op == SPK_OP_SPMV || op == SPK_OP_SPMV_WAXPY) spmv_space(s);
    else if (op == SPK_OP_WAXPY || op == SPK_OP_AXPY || op == SPK_OP_DOT) vec_space(op, dtype, s);
    else return fail(SPK_ERR_ARG, "unknown op %d", op);
    if (index < 0 || index >= (int32_t)s.size()) return fail(SPK_ERR_NOT_FOUND, "variant index %d out of range", index);
    *out = s[index];
    return SPK_OK;
}

spk_status spk_plain_variant(int32_t op, int32_t which, spk_variant *out)
{
    if (!out) return fail(SPK_ERR_NULL, "out is NULL");
    if (op < SPK_OP_SPMV || op > SPK_OP_SPMV_WAXPY) return fail(SPK_ERR_ARG, "unknown op %d", op);
    if (which != 0 && which != 1) return fail(SPK_ERR_ARG, "which must be 0 or 1");
    if (which == 1 && op != SPK_OP_SPMV && op != SPK_OP_SPMV_WAXPY)
        return fail(SPK_ERR_ARG, "vector ops have one plain variant");
    *out = plain_variant(op, which);
    return SPK_OK;
}

spk_status spk_class_key(spk_handle h, const spk_problem *p, char *out, int32_t cap)
{
    if (!h || !p || !out || cap <= 0) return fail(SPK_ERR_NULL, "NULL argument");
    const std::string k = class_key(*p, nullptr);
    snprintf(out, (size_t)cap, "%s", k.c_str());
    return SPK_OK;
}

spk_status spk_plan_get(spk_handle h, const char *class_key_, spk_variant *out)
{
    if (!h || !class_key_ || !out) return fail(SPK_ERR_NULL, "NULL argument");
    std::lock_guard<std::mutex> lk(h->mu);
    auto it = h->plans.find(class_key_);
    if (it == h->plans.end()) return fail(SPK_ERR_NOT_FOUND, "no plan for %s", class_key_);
    *out = it->second;
    return SPK_OK;
}

spk_status spk_plan_put(spk_handle h, const char *class_key_, const spk_variant *v)
{
    if (!h || !class_key_ || !v) return fail(SPK_ERR_NULL, "NULL argument");
    std::lock_guard<std::mutex> lk(h->mu);
    h->plans[class_key_] = *v;
    return SPK_OK;
}

// ------------------------------------------------------------ measurement --

spk_status spk_stream_probe(spk_handle h, int32_t kind, int64_t n, const double *a, const double *b, double *c,
                            spk_stream stream)
{
    if (!h) return fail(SPK_ERR_NULL, "handle is NULL");
    if (n < 0) return fail(SPK_ERR_SHAPE, "n < 0");
    if (n == 0) return SPK_OK;
    DeviceGuard g(h);
    if (kind == 0) {
        if (!a || !c) return fail(SPK_ERR_NULL, "a/c are NULL");
        SPK_HIP(launch_copy(n, a, c, (hipStream_t)stream));
    } else if (kind == 1) {
        if (!a || !b || !c) return fail(SPK_ERR_NULL, "a/b/c are NULL");
        SPK_HIP(launch_triad(n, a, b, 3.0, c, (hipStream_t)stream));
    } else {
        return fail(SPK_ERR_ARG, "kind must be 0 (copy) or 1 (triad)");
    }
    return SPK_OK;
}

spk_status spk_flush_cache(spk_handle h, spk_stream stream)
{
    if (!h) return fail(SPK_ERR_NULL, "handle is NULL");
    DeviceGuard g(h);
    {
        std::lock_guard<std::mutex> lk(h->mu);
        if (!h->flush_buf) {
            // 512 MiB to read (twice the last-level cache) + 16 bytes of sink
            h->flush_bytes = 512ll << 20;
            SPK_HIP(hipMalloc(&h->flush_buf, (size_t)h->flush_bytes + 256));
            SPK_HIP(launch_fill(h->flush_buf, h->flush_bytes + 256, 0x5A5A5A5Au, h->work));
            SPK_HIP(hipStreamSynchronize(h->work));
        }
    }
    SPK_HIP(launch_evict(h->flush_buf, h->flush_bytes, (char *)h->flush_buf + h->flush_bytes, (hipStream_t)stream));
    return SPK_OK;
}

}  // extern "C"
