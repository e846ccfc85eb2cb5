// cg.cpp -- host side of the conjugate-gradient solve (spk_cg).
//
// The solve is a fixed sequence of launches on the caller's stream: the
// start (q = A x; r = b - q, p = r with the parts of r.r; r.r recorded)
// and, per iteration, the SpMV+dot, update+dot and direction kernels (the
// last iteration records r.r instead of updating the direction).  All
// scalars stay on the device, so nothing waits for the host and the whole
// sequence can be captured into a graph by the caller.
#include <algorithm>
#include <cstring>

#include "internal.h"

using namespace spk;

namespace {

constexpr int kCgDefaultBlock = 256;
constexpr int kCgDefaultEntries = 512;

const CgEntry *find_cg_entry(int block, int entries)
{
    int n = 0;
    const CgEntry *t = cg_table(&n);
    for (int i = 0; i < n; ++i)
        if (t[i].block == block && t[i].entries == entries) return &t[i];
    return nullptr;
}

// The wavefront-tile shape of the SpMV plan recorded for A's class when it
// is a row-block (ADAPTIVE) plan, else the default shape.
const CgEntry *cg_entry_for(spk_handle h, spk_mat *A)
{
    spk_problem p{};
    p.op = SPK_OP_SPMV;
    p.dtype = A->dtype;
    p.A = A;
    spk_variant v{};
    if (!h->plain && resolve(h, p, nullptr, &v) == SPK_OK && v.format == SPK_FMT_ADAPTIVE) {
        const CgEntry *e = find_cg_entry(v.block, v.lds);
        if (e) return e;
    }
    return find_cg_entry(kCgDefaultBlock, kCgDefaultEntries);
}

spk_status cg_scratch(spk_handle h, hipStream_t s, int64_t n, int64_t nparts, CgScratch **out)
{
    std::lock_guard<std::mutex> lk(h->mu);
    CgScratch &c = h->cg[s];
    const int64_t stride = (n + 31) / 32 * 32;   // 256-byte aligned vectors
    if (c.vec_cap < stride || c.part_cap < nparts) {
        if (c.vec) {
            // the stream may still use the old buffers
            SPK_HIP(hipStreamSynchronize(s));
            SPK_HIP(hipFree(c.vec));
            SPK_HIP(hipFree(c.part));
            SPK_HIP(hipFree(c.sc));
            c = CgScratch{};
        }
        const int64_t vcap = std::max(stride, c.vec_cap);
        const int64_t pcap = std::max<int64_t>(nparts, 4096);
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

}  // namespace

spk_status spk_cg(spk_handle h, spk_matrix A, const void *b, void *x, int32_t iters, double *d_rr_hist,
                  spk_stream stream)
{
    if (!h || !A) return fail(SPK_ERR_NULL, "handle/matrix is NULL");
    if (A->dtype != SPK_F64) return fail(SPK_ERR_DTYPE, "CG needs an FP64 matrix");
    if (A->nrows != A->ncols) return fail(SPK_ERR_SHAPE, "CG needs a square matrix");
    if (iters < 0) return fail(SPK_ERR_SHAPE, "iters < 0");
    if (!d_rr_hist) return fail(SPK_ERR_NULL, "d_rr_hist is NULL");
    const int64_t n = A->nrows;
    if (n > 0 && (!b || !x)) return fail(SPK_ERR_NULL, "b/x are NULL");
    const size_t nb = (size_t)n * sizeof(double), hb = ((size_t)iters + 1) * sizeof(double);
    if (overlaps(x, nb, b, nb)) return fail(SPK_ERR_ALIAS, "x overlaps b");
    if (overlaps(x, nb, d_rr_hist, hb) || overlaps(b, nb, d_rr_hist, hb))
        return fail(SPK_ERR_ALIAS, "the history overlaps x or b");
    if (((uintptr_t)x | (uintptr_t)b | (uintptr_t)d_rr_hist) % sizeof(double))
        return fail(SPK_ERR_ARG, "x, b and d_rr_hist must be 8-byte aligned");
    DeviceGuard g(h);
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        SPK_HIP(launch_cg_zero(d_rr_hist, (int64_t)iters + 1, s));
        return SPK_OK;
    }

    const CgEntry *e = cg_entry_for(h, A);
    if (!e) return fail(SPK_ERR_NOT_FOUND, "no CG SpMV kernel compiled");
    BlockData *bd = nullptr;
    SPK_TRY(get_blocks(h, A, e->entries, &bd));
    const int nw = e->block / 64;
    const int64_t ngroups = ((int64_t)bd->nblk + nw - 1) / nw;
    // one pass over the vectors, at most 8 workgroups per CU (their
    // partials are re-read by every workgroup of the consuming kernel)
    const int64_t cap = 8ll * h->num_cu;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((n + kCgVecPer - 1) / kCgVecPer, cap));
    const int64_t spmv_grid = std::max<int64_t>(1, std::min<int64_t>(ngroups, cap));
    CgScratch *cs = nullptr;
    SPK_TRY(cg_scratch(h, s, n, std::max(spmv_grid, grid), &cs));

    CgLaunch c;
    memset(&c, 0, sizeof c);
    c.n = n;
    c.rp = A->rp;
    c.ci = A->ci;
    c.val = (const double *)A->val;
    c.blocks = bd->blk;
    c.block_k = bd->bk;
    c.nblk = bd->nblk;
    c.spmv_grid = (int32_t)spmv_grid;
    c.b = (const double *)b;
    c.r = cs->vec;
    c.p = cs->vec + cs->vec_cap;
    c.q = cs->vec + 2 * cs->vec_cap;
    // the vector kernels use 16-byte accesses: an x that is not 16-byte
    // aligned is iterated in an aligned copy
    const bool copy_x = ((uintptr_t)x % 16) != 0;
    c.x = copy_x ? cs->vec + 3 * cs->vec_cap : (double *)x;
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
    c.hist = d_rr_hist;
    SPK_HIP(launch_cg_record(c, s));
    c.spmv_x = c.p;
    c.part1 = cs->part;
    for (int32_t k = 0; k < iters; ++k) {
        c.slot = k & 1;
        c.hist = d_rr_hist + k + 1;
        SPK_HIP(e->spmv_dot(c, s));
        SPK_HIP(launch_cg_update(c, s));
        // the last direction is never used: only record r.r
        if (k + 1 < iters) SPK_HIP(launch_cg_direction(c, s));
        else SPK_HIP(launch_cg_record(c, s));
    }
    if (copy_x) SPK_HIP(hipMemcpyAsync(x, c.x, nb, hipMemcpyDeviceToDevice, s));
    return SPK_OK;
}
