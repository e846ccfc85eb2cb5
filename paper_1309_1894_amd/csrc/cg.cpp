// cg.cpp -- host side of the conjugate-gradient solve (spk_cg) and of its
// tuner (spk_cg_tune).
//
// The solve is a fixed sequence of launches on the caller's stream: the
// start (q = A x; r = b - q, p = r with the parts of r.r; r.r recorded)
// and, per iteration, the SpMV+dot, residual and direction kernels.  All
// scalars stay on the device, so nothing waits for the host and the whole
// sequence can be captured into a graph by the caller.
//
// The tunable is the SpMV+dot kernel: the wavefront-tile shape of the CSR
// form (threads per workgroup, entries per wavefront), which sets the tile
// count, hence the number of partials every workgroup of the residual
// kernel adds up, so the best shape for the solve need not be the best for
// a lone SpMV; or, for a matrix that is a constant-coefficient grid
// stencil, the matrix-free form.  spk_cg_tune applies Section 2's search to
// it and files the winner under "cg:" + the matrix's SpMV class key.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace spk;

namespace {

constexpr int kCgDefaultBlock = 512;
constexpr int kCgDefaultEntries = 512;

const CgEntry *find_cg_entry(int format, int block, int entries, int lds, int vec = 0)
{
    int n = 0;
    const CgEntry *t = cg_table(&n);
    for (int i = 0; i < n; ++i)
        if (t[i].format == format && t[i].block == block && t[i].entries == entries && t[i].lds == lds &&
            t[i].vec == (vec == 2 ? 2 : 0))
            return &t[i];
    return nullptr;
}

const CgEntry *default_cg_entry()
{
    return find_cg_entry(SPK_FMT_ADAPTIVE, kCgDefaultBlock, kCgDefaultEntries, 0);
}

// Whether entry e can run on A: its format applies, and an LDS-staged
// stencil's halo fits the budget.
bool cg_entry_fits(const spk_mat *A, const CgEntry &e)
{
    if (!format_applies(A, e.format)) return false;
    if (e.format == SPK_FMT_STENCIL && e.lds)
        return stencil_lds_bytes(e.block, e.entries, A->st.dim, A->st.N3, 8) <= kStencilLdsMaxBytes;
    return true;
}

std::string cg_key(spk_mat *A)
{
    spk_problem p{};
    p.op = SPK_OP_SPMV;
    p.dtype = A->dtype;
    p.A = A;
    return "cg:" + class_key(p, nullptr);
}

// The SpMV+dot kernel recorded for A's class, else the default tile shape.
const CgEntry *cg_entry_for(spk_handle h, spk_mat *A)
{
    if (!h->plain) {
        const std::string key = cg_key(A);
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = h->plans.find(key);
        if (it != h->plans.end()) {
            const spk_variant &v = it->second;
            const bool st = v.format == SPK_FMT_STENCIL;
            const CgEntry *e = find_cg_entry(v.format, v.block, st ? v.unroll : v.lds, st ? v.lds : 0, v.vec);
            if (e && cg_entry_fits(A, *e)) return e;
        }
    }
    return default_cg_entry();
}

spk_status cg_scratch(spk_handle h, hipStream_t s, int64_t n, int64_t nparts, CgScratch **out)
{
    std::lock_guard<std::mutex> lk(h->mu);
    CgScratch &c = h->cg[s];
    const int64_t stride = (n + 31) / 32 * 32;   // 256-byte aligned vectors
    if (c.vec_cap < stride || c.part_cap < nparts) {
        const int64_t vcap = std::max(stride, c.vec_cap);
        const int64_t pcap = std::max<int64_t>(std::max(nparts, c.part_cap), 4096);
        if (c.vec) {
            // the stream may still use the old buffers
            SPK_HIP(hipStreamSynchronize(s));
            SPK_HIP(hipFree(c.vec));
            SPK_HIP(hipFree(c.part));
            SPK_HIP(hipFree(c.sc));
            c = CgScratch{};
        }
        if (hipMalloc(&c.vec, (size_t)vcap * 4 * sizeof(double)) != hipSuccess) {
            c = CgScratch{};
            return fail(SPK_ERR_OOM, "CG working vectors (%lld doubles)", (long long)(4 * vcap));
        }
        SPK_HIP(hipMalloc(&c.part, (size_t)pcap * 2 * sizeof(double)));
        SPK_HIP(hipMalloc(&c.sc, 256));
        c.vec_cap = vcap;
        c.part_cap = pcap;
    }
    *out = &c;
    return SPK_OK;
}

// The solve with tile shape e (arguments already checked, n > 0).
spk_status run_cg(spk_handle h, spk_mat *A, const CgEntry *e, const double *b, double *x, int32_t iters,
                  double *hist, hipStream_t s)
{
    const int64_t n = A->nrows;
    // the vector kernels make one pass with at most 8 workgroups per CU
    // (their partials are re-read by every workgroup of the consuming
    // kernel); the tile SpMV runs one workgroup per tile group, the stencil
    // SpMV a grid-stride loop on the same cap
    const int64_t cap = 8ll * h->num_cu;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((n + kCgVecPer - 1) / kCgVecPer, cap));
    CgLaunch c;
    memset(&c, 0, sizeof c);
    int64_t spmv_grid = 1;
    if (e->format == SPK_FMT_STENCIL) {
        if (!cg_entry_fits(A, *e)) return fail(SPK_ERR_ARG, "A is not a grid stencil this kernel can run");
        const int64_t per = (int64_t)e->block * e->entries;
        spmv_grid = std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, cap));
        c.st.n = (int32_t)n;
        c.st.N1 = A->st.N1;
        c.st.N2 = A->st.N2;
        c.st.N3 = A->st.N3;
        c.st.dim = A->st.dim;
        for (int q = 0; q < 7; ++q) c.st.coef[q] = A->st.coef[q];
    } else {
        BlockData *bd = nullptr;
        SPK_TRY(get_blocks(h, A, e->entries, &bd));
        const int nw = e->block / 64;
        spmv_grid = std::max<int64_t>(1, ((int64_t)bd->nblk + nw - 1) / nw);
        c.blocks = bd->blk;
        c.block_k = bd->bk;
        c.nblk = bd->nblk;
        if (e->vec == 2) {
            SPK_TRY(get_block_c16(h, A, bd));
            c.c16 = bd->c16;
            c.block_c16 = bd->cbase;
        }
    }
    CgScratch *cs = nullptr;
    SPK_TRY(cg_scratch(h, s, n, std::max(spmv_grid, grid), &cs));

    c.n = n;
    c.rp = A->rp;
    c.ci = A->ci;
    c.val = (const double *)A->val;
    c.spmv_grid = (int32_t)spmv_grid;
    c.b = b;
    c.r = cs->vec;
    c.p = cs->vec + cs->vec_cap;
    c.q = cs->vec + 2 * cs->vec_cap;
    // the vector kernels use 16-byte accesses: an x that is not 16-byte
    // aligned is iterated in an aligned copy
    const size_t nb = (size_t)n * sizeof(double);
    const bool copy_x = ((uintptr_t)x % 16) != 0;
    c.x = copy_x ? cs->vec + 3 * cs->vec_cap : x;
    c.part2 = cs->part + cs->part_cap;
    c.sc = cs->sc;
    c.grid = grid;
    if (copy_x) SPK_HIP(hipMemcpyAsync(c.x, x, nb, hipMemcpyDeviceToDevice, s));

    // start: q = A x (no dot), r = b - q, p = r, rr_0 into slot 0 and hist[0]
    c.spmv_x = c.x;
    c.part1 = nullptr;
    SPK_HIP(e->spmv_dot(c, s));
    SPK_HIP(launch_cg_start(c, s));
    c.slot = 0;
    c.hist = hist;
    SPK_HIP(launch_cg_record(c, s));
    c.spmv_x = c.p;
    c.part1 = cs->part;
    for (int32_t k = 0; k < iters; ++k) {
        c.slot = k & 1;
        c.hist = hist + k + 1;
        SPK_HIP(e->spmv_dot(c, s));
        SPK_HIP(launch_cg_residual(c, s));
        SPK_HIP(launch_cg_direction(c, s));
    }
    if (copy_x) SPK_HIP(hipMemcpyAsync(x, c.x, nb, hipMemcpyDeviceToDevice, s));
    return SPK_OK;
}

spk_status check_cg_args(spk_handle h, spk_matrix A, const void *b, const void *x, int32_t iters,
                         const double *hist)
{
    if (!h || !A) return fail(SPK_ERR_NULL, "handle/matrix is NULL");
    if (A->dtype != SPK_F64) return fail(SPK_ERR_DTYPE, "CG needs an FP64 matrix");
    if (A->nrows != A->ncols) return fail(SPK_ERR_SHAPE, "CG needs a square matrix");
    if (iters < 0) return fail(SPK_ERR_SHAPE, "iters < 0");
    if (!hist) return fail(SPK_ERR_NULL, "d_rr_hist is NULL");
    const int64_t n = A->nrows;
    if (n > 0 && (!b || !x)) return fail(SPK_ERR_NULL, "b/x are NULL");
    const size_t nb = (size_t)n * sizeof(double), hb = ((size_t)iters + 1) * sizeof(double);
    if (overlaps(x, nb, b, nb)) return fail(SPK_ERR_ALIAS, "x overlaps b");
    if (overlaps(x, nb, hist, hb) || overlaps(b, nb, hist, hb))
        return fail(SPK_ERR_ALIAS, "the history overlaps x or b");
    if (((uintptr_t)x | (uintptr_t)b | (uintptr_t)hist) % sizeof(double))
        return fail(SPK_ERR_ARG, "x, b and d_rr_hist must be 8-byte aligned");
    return SPK_OK;
}

struct DevMem {
    void *p = nullptr;
    ~DevMem()
    {
        if (p) (void)hipFree(p);
    }
};

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

spk_status spk_cg(spk_handle h, spk_matrix A, const void *b, void *x, int32_t iters, double *d_rr_hist,
                  spk_stream stream)
{
    SPK_TRY(check_cg_args(h, A, b, x, iters, d_rr_hist));
    DeviceGuard g(h);
    hipStream_t s = (hipStream_t)stream;
    if (A->nrows == 0) {
        SPK_HIP(launch_cg_zero(d_rr_hist, (int64_t)iters + 1, s));
        return SPK_OK;
    }
    const CgEntry *e = cg_entry_for(h, A);
    if (!e) return fail(SPK_ERR_NOT_FOUND, "no CG SpMV kernel compiled");
    return run_cg(h, A, e, (const double *)b, (double *)x, iters, d_rr_hist, s);
}

spk_status spk_cg_tune(spk_handle h, spk_matrix A, const void *b, int32_t iters, const spk_tune_opts *opts,
                       spk_tune_report *report)
{
    if (!report) return fail(SPK_ERR_NULL, "report is NULL");
    memset(report, 0, sizeof *report);
    if (!h || !A) return fail(SPK_ERR_NULL, "handle/matrix is NULL");
    if (A->dtype != SPK_F64) return fail(SPK_ERR_DTYPE, "CG needs an FP64 matrix");
    if (A->nrows != A->ncols) return fail(SPK_ERR_SHAPE, "CG needs a square matrix");
    if (iters < 1) return fail(SPK_ERR_SHAPE, "tuning needs iters >= 1");
    if (A->nrows == 0) return fail(SPK_ERR_SHAPE, "empty matrix");
    if (!b) return fail(SPK_ERR_NULL, "b is NULL");
    if ((uintptr_t)b % sizeof(double)) return fail(SPK_ERR_ARG, "b must be 8-byte aligned");
    if (opts && (opts->resume != 0 || opts->stop_after != 0))
        return fail(SPK_ERR_ARG, "spk_cg_tune keeps no journal: resume and stop_after must be 0");
    const int64_t n = A->nrows;
    const int reps = opts && opts->reps > 0 ? opts->reps : 10;
    const int warmup = opts && opts->warmup > 0 ? opts->warmup : 2;
    const double tau = opts && opts->tau > 0 ? opts->tau : 1e-10;
    const bool record = opts ? opts->record != 0 : true;
    const bool verbose = opts && opts->verbose;
    const int limit_opt = opts ? opts->max_variants : 0;
    DeviceGuard g(h);
    hipStream_t s = h->work;
    const size_t nb = (size_t)n * sizeof(double), hb = ((size_t)iters + 1) * sizeof(double);
    DevMem xr, xt, hr, ht;
    SPK_HIP(hipMalloc(&xr.p, nb));
    SPK_HIP(hipMalloc(&xt.p, nb));
    SPK_HIP(hipMalloc(&hr.p, hb));
    SPK_HIP(hipMalloc(&ht.p, hb));
    EventPair ev;
    SPK_HIP(timing_event(&ev.a));
    SPK_HIP(timing_event(&ev.b));

    auto solve = [&](const CgEntry *e, void *xd, void *hd) -> spk_status {
        SPK_HIP(hipMemsetAsync(xd, 0, nb, s));
        return run_cg(h, A, e, (const double *)b, (double *)xd, iters, (double *)hd, s);
    };
    auto fetch = [&](void *xd, void *hd, std::vector<double> &xh, std::vector<double> &hh) -> spk_status {
        SPK_HIP(hipMemcpyAsync(xh.data(), xd, nb, hipMemcpyDeviceToHost, s));
        SPK_HIP(hipMemcpyAsync(hh.data(), hd, hb, hipMemcpyDeviceToHost, s));
        SPK_HIP(hipStreamSynchronize(s));
        return SPK_OK;
    };
    auto time_entry = [&](const CgEntry *e, double *us) -> spk_status {
        std::vector<double> t;
        for (int r = 0; r < warmup + reps; ++r) {
            SPK_HIP(hipMemsetAsync(xt.p, 0, nb, s));
            SPK_HIP(hipEventRecord(ev.a, s));
            SPK_TRY(run_cg(h, A, e, (const double *)b, (double *)xt.p, iters, (double *)ht.p, s));
            SPK_HIP(hipEventRecord(ev.b, s));
            SPK_HIP(hipStreamSynchronize(s));
            float ms = 0.f;
            SPK_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
            if (r >= warmup) t.push_back(ms * 1e3);
        }
        std::sort(t.begin(), t.end());
        *us = t[t.size() / 2];
        return SPK_OK;
    };

    // reference: the default shape, from x = 0 (Section 2: the unannotated
    // variant's outputs are what every candidate must reproduce)
    const CgEntry *ref = default_cg_entry();
    if (!ref) return fail(SPK_ERR_NOT_FOUND, "no CG SpMV kernel compiled");
    std::vector<double> x_ref(n), h_ref(iters + 1), x_try(n), h_try(iters + 1);
    SPK_TRY(solve(ref, xr.p, hr.p));
    SPK_TRY(fetch(xr.p, hr.p, x_ref, h_ref));
    double xmax = 0.0;
    for (double v : x_ref) xmax = std::max(xmax, std::fabs(v));

    int count = 0;
    const CgEntry *table = cg_table(&count);
    const int limit = limit_opt > 0 ? std::min(limit_opt, count) : count;
    double best_us = 1e300;
    const CgEntry *best = nullptr;
    const uint32_t formats = opts ? opts->formats : 0u;
    for (int i = 0; i < limit; ++i) {
        const CgEntry *e = &table[i];
        if (!cg_entry_fits(A, *e) || (formats && !(formats & (1u << e->format)))) continue;
        SPK_TRY(solve(e, xt.p, ht.p));
        SPK_TRY(fetch(xt.p, ht.p, x_try, h_try));
        bool ok = true;
        for (int k = 0; k <= iters && ok; ++k)
            ok = std::isfinite(h_try[k]) && std::fabs(h_try[k] - h_ref[k]) <= tau * h_ref[k];
        for (int64_t j = 0; j < n && ok; ++j) ok = std::fabs(x_try[j] - x_ref[j]) <= tau * xmax;
        if (!ok) {
            ++report->rejected;
            if (verbose)
                fprintf(stderr, "spk_cg_tune: format %d block %d entries %d rejected\n", e->format, e->block,
                        e->entries);
            continue;
        }
        double us = 0.0;
        SPK_TRY(time_entry(e, &us));
        ++report->tried;
        if (verbose)
            fprintf(stderr, "spk_cg_tune: format %d block %d entries %d lds %d vec %d: %.2f us\n", e->format,
                    e->block, e->entries, e->lds, e->vec, us);
        if (e == ref) report->plain_us = us;
        if (us < best_us) {
            best_us = us;
            best = e;
        }
    }
    if (!best) return fail(SPK_ERR_VALIDATION, "no tile shape reproduced the reference solve");
    spk_variant v{};
    v.format = best->format;
    v.block = best->block;
    v.group = 1;
    v.streams = 1;
    // tile shapes report their entries per wavefront as `lds`, the
    // matrix-free kernel its rows per lane as `unroll`
    v.unroll = best->format == SPK_FMT_STENCIL ? best->entries : 1;
    v.lds = best->format == SPK_FMT_STENCIL ? best->lds : best->entries;
    v.vec = best->vec;   // 2: two-byte columns
    report->best = v;
    report->best_us = best_us;
    const std::string key = cg_key(A);
    snprintf(report->class_key, sizeof report->class_key, "%s", key.c_str());
    if (record) {
        {
            std::lock_guard<std::mutex> lk(h->mu);
            h->plans[key] = v;
        }
        db_append(h, key, v, best_us);
    }
    return SPK_OK;
}
