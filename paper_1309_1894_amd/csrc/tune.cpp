// tune.cpp -- the variant search of Section 2 of the paper, on the GPU.
//
// The paper's loop: the unannotated code is the reference; every variant
// generated from the annotations is compiled and run, its outputs compared
// with the reference outputs, and the fastest variant is kept.  Here the
// variants are the precompiled kernel instantiations; the reference output
// is either supplied by the caller or produced by a run of the plain
// variant (the library's unannotated code); a variant whose output fails the
// acceptance test is discarded before it is timed.  Section 3's knobs --
// threads per block, blocks per grid, streams, cache-sized staging, unroll
// -- span the space.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.h"

namespace spk {

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t n)
    {
        return hipMalloc(&p, std::max<size_t>(n, 16));
    }
};

struct Ctx {
    spk_handle h;
    spk_problem p;
    hipStream_t s;
    int dtype;
    int64_t nout;          // outputs validated: rows (SpMV), n (vector), 1 (dot)
    const void *out;       // device output of a run (y, w or d_result)
    void *out2 = nullptr;  // fused step: w
    DevBuf ref, scale, ref2, scale2, bad, saved;
    double tau;
    int check_mode;        // 0 per-element tolerance, 1 ulp
    unsigned long long *hbad = nullptr;
};

spk_status run_variant(Ctx &c, const spk_variant &v)
{
    if (c.p.op == SPK_OP_AXPY) {
        // AXPY updates its input: restore y before every run
        SPK_HIP(hipMemcpyAsync(c.p.y, c.saved.p, (size_t)c.p.n * dtype_size(c.dtype), hipMemcpyDeviceToDevice, c.s));
    }
    return spk_run(c.h, &c.p, &v, (spk_stream)c.s);
}

spk_status validate(Ctx &c, const spk_variant &v, bool *ok)
{
    SPK_HIP(hipMemsetAsync(c.bad.p, 0, sizeof(unsigned long long), c.s));
    SPK_TRY(run_variant(c, v));
    const int out_dtype = c.p.op == SPK_OP_DOT ? SPK_F64 : c.dtype;
    SPK_HIP(launch_check(out_dtype, c.check_mode, c.nout, c.out, (const double *)c.ref.p,
                         (const double *)c.scale.p, c.tau, (unsigned long long *)c.bad.p, c.s));
    if (c.p.op == SPK_OP_SPMV_WAXPY) {
        // w = alpha*y + x from the variant's own y: the y tolerance scaled by
        // |alpha|, plus a rounding of w
        SPK_HIP(launch_check(c.dtype, 0, c.nout, c.out2, (const double *)c.ref2.p, (const double *)c.scale2.p,
                             c.tau, (unsigned long long *)c.bad.p, c.s));
    }
    SPK_HIP(hipMemcpyAsync(c.hbad, c.bad.p, sizeof(unsigned long long), hipMemcpyDeviceToHost, c.s));
    SPK_HIP(hipStreamSynchronize(c.s));
    *ok = (*c.hbad == 0);
    return SPK_OK;
}

spk_status time_variant(Ctx &c, const spk_variant &v, int warmup, int reps, bool flush, double *median_us)
{
    for (int i = 0; i < warmup; ++i) SPK_TRY(run_variant(c, v));
    std::vector<hipEvent_t> ev(2 * (size_t)reps);
    for (auto &e : ev) SPK_HIP(timing_event(&e));
    spk_status st = SPK_OK;
    for (int r = 0; r < reps && st == SPK_OK; ++r) {
        if (c.p.op == SPK_OP_AXPY) {
            const hipError_t re = hipMemcpyAsync(c.p.y, c.saved.p, (size_t)c.p.n * dtype_size(c.dtype),
                                                 hipMemcpyDeviceToDevice, c.s);
            if (re != hipSuccess) {
                st = hip_fail(re, "restore y");
                break;
            }
        }
        if (flush && (st = spk_flush_cache(c.h, (spk_stream)c.s)) != SPK_OK) break;
        (void)hipEventRecord(ev[2 * r], c.s);
        st = spk_run(c.h, &c.p, &v, (spk_stream)c.s);
        (void)hipEventRecord(ev[2 * r + 1], c.s);
    }
    hipError_t e = hipStreamSynchronize(c.s);
    std::vector<double> t;
    if (st == SPK_OK && e == hipSuccess) {
        for (int r = 0; r < reps; ++r) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]);
            t.push_back(ms * 1e3);
        }
    }
    for (auto &x : ev) hipEventDestroy(x);
    if (st != SPK_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "timing sync");
    std::sort(t.begin(), t.end());
    *median_us = t[t.size() / 2];
    return SPK_OK;
}

void candidate_space(const Ctx &c, uint32_t formats, std::vector<spk_variant> &out, int *pruned)
{
    int32_t n = 0;
    spk_variant_count(c.p.op, c.dtype, &n);
    const bool spmv = c.p.op == SPK_OP_SPMV || c.p.op == SPK_OP_SPMV_WAXPY;
    for (int32_t i = 0; i < n; ++i) {
        spk_variant v{};
        spk_variant_get(c.p.op, c.dtype, i, &v);
        if (spmv) {
            const spk_mat *A = c.p.A;
            if (formats && !(formats & (1u << v.format))) continue;
            // byte model: sliced ELL is skipped when padding would more than
            // double the stored entries
            if (v.format == SPK_FMT_SELL && A->nnz > 0 && sell_padded_entries(A, v.group) > 2 * A->nnz) {
                ++*pruned;
                continue;
            }
            // lane groups far wider than the longest row only idle
            if (v.format == SPK_FMT_VECTOR && v.group > 2 && (int64_t)v.group > 8 * std::max<int64_t>(1, A->max_len)) {
                ++*pruned;
                continue;
            }
        } else if (c.p.op == SPK_OP_DOT && v.grid == 0 && !(v.block == 256 && v.vec == 1 && v.unroll == 1)) {
            // one-pass dot grids only for the plain variant (partials grow with n)
            ++*pruned;
            continue;
        }
        out.push_back(v);
    }
    if (!spmv) return;
    const spk_mat *A = c.p.A;
    // column blocks (FP64): only when x is larger than one XCD's L2, the
    // case they are for; the per-block kernel from the row-block shapes
    if ((!formats || (formats & (1u << SPK_FMT_COLBLOCK))) && format_applies(A, SPK_FMT_COLBLOCK)) {
        if (A->ncols * (int64_t)sizeof(double) > ((int64_t)4 << 20)) {
            for (int nb : {2, 4})
                for (const auto &bl : {std::pair<int, int>{512, 256}, {128, 256}, {256, 1024}}) {
                    spk_variant v{};
                    v.format = SPK_FMT_COLBLOCK;
                    v.block = bl.first;
                    v.group = nb;
                    v.unroll = 1;
                    v.streams = 1;
                    v.lds = bl.second;
                    if (find_spmv_entry(colblock_inner(v))) out.push_back(v);
                }
        } else {
            ++*pruned;
        }
    }
    // x staged in LDS by column window: when x is larger than one XCD's L2
    if ((!formats || (formats & (1u << SPK_FMT_XWIN))) && format_applies(A, SPK_FMT_XWIN)) {
        if (A->ncols * (int64_t)dtype_size(A->dtype) > ((int64_t)4 << 20)) {
            int nx = 0;
            const XwinEntry *xt = xwin_table(&nx);
            for (int i = 0; i < nx; ++i)
                for (int g : {1, 2}) {
                    spk_variant v{};
                    v.format = SPK_FMT_XWIN;
                    v.block = xt[i].block;
                    v.group = xt[i].window_kib;
                    v.lds = xt[i].entries;
                    v.grid = g;
                    v.unroll = 1;
                    v.streams = 1;
                    out.push_back(v);
                }
        } else {
            ++*pruned;
        }
    }
    // structured formats, when the matrix admits them
    int ns = 0;
    const StructEntry *st = struct_table(&ns);
    for (int i = 0; i < ns; ++i) {
        if (formats && !(formats & (1u << st[i].format))) continue;
        if (!format_applies(A, st[i].format) || !struct_entry_fits(A, st[i])) continue;
        // byte model: DIA is skipped when its stored slots exceed twice the entries
        if (st[i].format == SPK_FMT_DIA && (int64_t)A->st.off.size() * A->nrows > 2 * A->nnz) {
            ++*pruned;
            continue;
        }
        spk_variant v{};
        v.format = st[i].format;
        v.block = st[i].block;
        v.group = 1;
        v.unroll = st[i].rows;
        v.lds = st[i].lds;
        v.streams = 1;
        out.push_back(v);
    }
}

}  // namespace

}  // namespace spk

using namespace spk;

extern "C" spk_status spk_tune(spk_handle h, const spk_problem *problem, const spk_tune_opts *opts,
                               spk_tune_report *report)
{
    if (!h || !problem || !report) return fail(SPK_ERR_NULL, "handle/problem/report is NULL");
    spk_tune_opts o{};
    if (opts) o = *opts;
    const int reps = o.reps > 0 ? o.reps : 10;
    const int warmup = o.warmup > 0 ? o.warmup : 2;
    memset(report, 0, sizeof *report);

    Ctx c;
    c.h = h;
    c.p = *problem;
    c.s = h->work;
    const int op = c.p.op;
    const bool spmv = (op == SPK_OP_SPMV || op == SPK_OP_SPMV_WAXPY);
    if (spmv) {
        if (!c.p.A) return fail(SPK_ERR_NULL, "problem.A is NULL");
        c.dtype = c.p.A->dtype;
        c.nout = c.p.A->nrows;
        c.out = c.p.y;
        if (!c.p.y || (c.p.A->ncols > 0 && !c.p.x)) return fail(SPK_ERR_NULL, "x/y are NULL");
        if (op == SPK_OP_SPMV_WAXPY) {
            if (!c.p.w) return fail(SPK_ERR_NULL, "w is NULL");
            c.out2 = c.p.w;
        }
    } else if (op == SPK_OP_WAXPY || op == SPK_OP_AXPY || op == SPK_OP_DOT) {
        c.dtype = c.p.dtype;
        if (!dtype_ok(c.dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", c.dtype);
        if (c.p.n < 0) return fail(SPK_ERR_SHAPE, "n < 0");
        if (!c.p.x || !c.p.y) return fail(SPK_ERR_NULL, "x/y are NULL");
        if (op == SPK_OP_WAXPY && !c.p.w) return fail(SPK_ERR_NULL, "w is NULL");
        if (op == SPK_OP_DOT && !c.p.d_result) return fail(SPK_ERR_NULL, "d_result is NULL");
        c.nout = op == SPK_OP_DOT ? 1 : c.p.n;
        c.out = op == SPK_OP_WAXPY ? c.p.w : op == SPK_OP_AXPY ? c.p.y : (const void *)c.p.d_result;
        if (op == SPK_OP_WAXPY && (c.p.w == c.p.x || c.p.w == c.p.y))
            return fail(SPK_ERR_ALIAS, "tuning WAXPY needs w distinct from x and y");
    } else {
        return fail(SPK_ERR_ARG, "unknown op %d", op);
    }
    c.tau = o.tau > 0 ? o.tau : (c.dtype == SPK_F64 ? 1e-12 : 1e-5);
    c.check_mode = (op == SPK_OP_WAXPY || op == SPK_OP_AXPY) ? 1 : 0;

    DeviceGuard g(h);
    SPK_HIP(hipDeviceSynchronize());  // the caller's pending work on the buffers
    const size_t nbytes_d = (size_t)std::max<int64_t>(1, c.nout) * sizeof(double);
    SPK_HIP(c.bad.alloc(sizeof(unsigned long long)));
    SPK_HIP(hipHostMalloc((void **)&c.hbad, sizeof(unsigned long long), hipHostMallocDefault));
    struct HostFree {
        void *p;
        ~HostFree() { if (p) hipHostFree(p); }
    } hf{c.hbad};
    SPK_HIP(c.ref.alloc(nbytes_d));
    if (op == SPK_OP_AXPY) {
        SPK_HIP(c.saved.alloc((size_t)c.p.n * dtype_size(c.dtype)));
        SPK_HIP(hipMemcpyAsync(c.saved.p, c.p.y, (size_t)c.p.n * dtype_size(c.dtype), hipMemcpyDeviceToDevice, c.s));
    }

    // ----- reference outputs (Section 2: the unannotated program's results)
    const spk_variant plain0 = plain_variant(op, 0);
    if (o.ref_host) {
        SPK_HIP(hipMemcpyAsync(c.ref.p, o.ref_host, nbytes_d, hipMemcpyHostToDevice, c.s));
        if (op == SPK_OP_SPMV_WAXPY) return fail(SPK_ERR_ARG, "ref_host is not supported for the fused step");
    } else {
        SPK_TRY(run_variant(c, plain0));
        if (op == SPK_OP_DOT) SPK_HIP(hipMemcpyAsync(c.ref.p, c.p.d_result, 8, hipMemcpyDeviceToDevice, c.s));
        else SPK_HIP(launch_widen(c.dtype, c.nout, c.out, (double *)c.ref.p, c.s));
    }
    if (c.check_mode == 0) {
        SPK_HIP(c.scale.alloc(nbytes_d));
        if (o.ref_host && o.ref_scale) {
            SPK_HIP(hipMemcpyAsync(c.scale.p, o.ref_scale, nbytes_d, hipMemcpyHostToDevice, c.s));
        } else if (spmv) {
            const spk_mat *A = c.p.A;
            SPK_HIP(launch_row_absum(c.dtype, (int32_t)A->nrows, A->rp, A->ci, A->val, c.p.x, (double *)c.scale.p, c.s));
        } else {
            SPK_HIP(hipMemsetAsync(c.scale.p, 0, 8, c.s));
            SPK_HIP(launch_dot_absum(c.dtype, c.p.n, c.p.x, c.p.y, (double *)c.scale.p, c.s));
        }
    }
    if (op == SPK_OP_SPMV_WAXPY) {
        // reference w from the plain run, tolerance |alpha|*tau*scale + 2 rounding units of w
        SPK_HIP(c.ref2.alloc(nbytes_d));
        SPK_HIP(c.scale2.alloc(nbytes_d));
        SPK_HIP(launch_widen(c.dtype, c.nout, c.out2, (double *)c.ref2.p, c.s));
        std::vector<double> sc((size_t)c.nout), wr((size_t)c.nout);
        SPK_HIP(hipMemcpyAsync(sc.data(), c.scale.p, nbytes_d, hipMemcpyDeviceToHost, c.s));
        SPK_HIP(hipMemcpyAsync(wr.data(), c.ref2.p, nbytes_d, hipMemcpyDeviceToHost, c.s));
        SPK_HIP(hipStreamSynchronize(c.s));
        const double eps = c.dtype == SPK_F64 ? 0x1p-52 : 0x1p-23;
        for (size_t i = 0; i < sc.size(); ++i) sc[i] = std::fabs(c.p.alpha) * sc[i] + 2.0 * eps * std::fabs(wr[i]) / c.tau;
        SPK_HIP(hipMemcpyAsync(c.scale2.p, sc.data(), nbytes_d, hipMemcpyHostToDevice, c.s));
    }
    SPK_HIP(hipStreamSynchronize(c.s));

    // ----- search
    std::vector<spk_variant> space;
    int pruned = 0;
    candidate_space(c, o.formats, space, &pruned);
    if (o.max_variants > 0 && (int)space.size() > o.max_variants) space.resize((size_t)o.max_variants);
    const bool flush = o.flush != 0;
    double best = 1e300, plain_best = 1e300;
    spk_variant bestv{};
    int tried = 0, rejected = 0, resumed = 0, fresh = 0;
    bool best_journaled = false;
    // the journal's key for this search: the class plus the problem's sizes
    std::string pkey;
    if (o.resume) {
        char fp[160];
        if (spmv)
            snprintf(fp, sizeof fp, "|op%d|m%lld|n%lld|nnz%lld", op, (long long)c.p.A->nrows, (long long)c.p.A->ncols,
                     (long long)c.p.A->nnz);
        else
            snprintf(fp, sizeof fp, "|op%d|n%lld", op, (long long)c.p.n);
        pkey = "tune|" + class_key(c.p, nullptr) + fp;
    }
    // validates, then times one point (*us = -1 when rejected)
    auto measure = [&](const spk_variant &v, double *us_out) -> spk_status {
        *us_out = -1.0;
        bool ok = false;
        SPK_TRY(validate(c, v, &ok));
        if (!ok) {
            ++rejected;
            if (o.verbose)
                fprintf(stderr, "spk_tune: reject fmt=%d bs=%d g=%d u=%d vec=%d grid=%d s=%d lds=%d (%llu bad)\n",
                        v.format, v.block, v.group, v.unroll, v.vec, v.grid, v.streams, v.lds, *c.hbad);
            return SPK_OK;
        }
        double us = 0;
        SPK_TRY(time_variant(c, v, warmup, reps, flush, &us));
        ++tried;
        if (o.verbose)
            fprintf(stderr, "spk_tune: %9.2f us fmt=%d bs=%d g=%d u=%d vec=%d grid=%d s=%d lds=%d\n", us, v.format,
                    v.block, v.group, v.unroll, v.vec, v.grid, v.streams, v.lds);
        *us_out = us;
        return SPK_OK;
    };
    auto consider = [&](const spk_variant &v) -> spk_status {
        double us = 0;
        bool journaled = false;
        if (o.resume && point_get(h, pkey, v, &us)) {
            // measured (and validated) before: take its median
            ++resumed;
            journaled = true;
        } else {
            if (o.stop_after > 0 && fresh >= o.stop_after) {
                report->tried = tried;
                report->rejected = rejected;
                report->resumed = resumed;
                return fail(SPK_ERR_INTERRUPTED, "search stopped after %d new points", fresh);
            }
            ++fresh;
            SPK_TRY(measure(v, &us));
            if (us < 0) return SPK_OK;   // rejected
            if (o.resume) point_put(h, pkey, v, us);
        }
        const bool is_plain = spmv ? ((v.format == SPK_FMT_SCALAR && v.block == 256 && v.unroll == 1 && v.streams == 1) ||
                                      (v.format == SPK_FMT_VECTOR && v.block == 256 && v.group == 64 && v.unroll == 1 &&
                                       v.lds == 0 && v.streams == 1))
                                   : (v.block == 256 && v.vec == 1 && v.unroll == 1 && v.grid == 0);
        if (is_plain) plain_best = std::min(plain_best, us);
        if (us < best) {
            best = us;
            bestv = v;
            best_journaled = journaled;
        }
        return SPK_OK;
    };
    for (const spk_variant &v : space) SPK_TRY(consider(v));
    if (spmv && tried + resumed > 0 && bestv.format != SPK_FMT_DIA && bestv.format != SPK_FMT_STENCIL &&
        bestv.format != SPK_FMT_COLBLOCK && bestv.format != SPK_FMT_XWIN) {
        // refinement: the winner split over 2 and 4 streams
        for (int s2 : {2, 4}) {
            spk_variant v = bestv;
            v.streams = s2;
            SPK_TRY(consider(v));
        }
    }
    report->tried = tried;
    report->rejected = rejected;
    report->pruned = pruned;
    report->resumed = resumed;
    if (tried + resumed == 0)
        return fail(SPK_ERR_VALIDATION, "no variant reproduced the reference output (%d rejected)", rejected);
    if (best_journaled) {
        // a winner taken from the journal is checked against this problem's reference
        bool ok = false;
        SPK_TRY(validate(c, bestv, &ok));
        if (!ok)
            return fail(SPK_ERR_VALIDATION, "the journaled winner does not reproduce this problem's reference output");
    }
    report->best = bestv;
    report->best_us = best;
    report->plain_us = plain_best < 1e300 ? plain_best : -1.0;
    const std::string key = class_key(c.p, nullptr);
    snprintf(report->class_key, sizeof report->class_key, "%s", key.c_str());
    if (o.record) {
        {
            std::lock_guard<std::mutex> lk(h->mu);
            h->plans[key] = bestv;
        }
        db_append(h, key, bestv, best);
    }
    // leave the winner's output in the caller's buffers
    SPK_TRY(run_variant(c, bestv));
    SPK_HIP(hipStreamSynchronize(c.s));
    return SPK_OK;
}
