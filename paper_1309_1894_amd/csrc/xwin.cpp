// xwin.cpp -- host side of SPK_FMT_XWIN (x staged in LDS by column
// window): the regrouping of a registered matrix's entries into (row,
// window) pairs, the wavefront tiles and workgroup chunks over them, and
// the two launches of one product.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "internal.h"
#include "xwin_layout.h"

namespace spk {

const XwinEntry *find_xwin_entry(int block, int window_kib, int entries)
{
    int n = 0;
    const XwinEntry *t = xwin_table(&n);
    for (int i = 0; i < n; ++i)
        if (t[i].block == block && t[i].window_kib == window_kib && t[i].entries == entries) return &t[i];
    return nullptr;
}

void free_xwin(XwinData &d)
{
    (void)hipFree(d.ci);
    (void)hipFree(d.val);
    (void)hipFree(d.ent);
    (void)hipFree(d.pos_ptr);
    (void)hipFree(d.rowpos);
    (void)hipFree(d.first);
    (void)hipFree(d.pre);
    for (auto &kv : d.plans) {
        (void)hipFree(kv.second.tiles);
        (void)hipFree(kv.second.tile_k);
        (void)hipFree(kv.second.chunk_t);
        (void)hipFree(kv.second.chunk_w);
    }
    for (auto &kv : d.part) (void)hipFree(kv.second);
    d = XwinData();
}

namespace {

// Regroups A's entries by window of `wc` columns from a host copy of them,
// then uploads the layout.
spk_status build_xwin(spk_handle h, spk_mat *A, int64_t wc, XwinData &d)
{
    const int64_t m = A->nrows, nnz = A->nnz;
    const size_t vs = dtype_size(A->dtype);
    std::vector<int32_t> ci((size_t)std::max<int64_t>(1, nnz));
    std::vector<char> val((size_t)std::max<int64_t>(1, nnz) * vs);
    if (nnz > 0) {
        SPK_HIP(hipDeviceSynchronize());
        SPK_HIP(hipMemcpy(ci.data(), A->ci, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
        SPK_HIP(hipMemcpy(val.data(), A->val, vs * nnz, hipMemcpyDeviceToHost));
    }
    XwinHost hx;
    switch (xwin_layout(m, A->ncols, nnz, A->rp_host.data(), ci.data(), val.data(), vs, wc, hx)) {
    case kXwinOk: break;
    case kXwinTooManyPairs: return fail(SPK_ERR_SHAPE, "too many (row, window) pairs for the x-window form");
    case kXwinTooManyWindows:
        return fail(SPK_ERR_SHAPE, "%lld columns make more than %lld windows", (long long)A->ncols,
                    (long long)kXwinMaxWin);
    default: return fail(SPK_ERR_SHAPE, "the x-window form's block tables would be too large");
    }
    d.wc = hx.wc;
    d.nwin = hx.nwin;
    d.npairs = hx.npairs;
    d.rb = hx.rb;
    d.nblk = hx.nblk;
    auto up = [&](void **dst, const void *src, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 16));
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, h->work);
        return e;
    };
    hipError_t e = up((void **)&d.ci, hx.ci.data(), sizeof(uint16_t) * nnz);
    if (e == hipSuccess) e = up(&d.val, hx.val.data(), vs * nnz);
    if (e == hipSuccess) e = up((void **)&d.ent, hx.ent.data(), sizeof(int32_t) * (d.npairs + 1));
    if (e == hipSuccess) e = up((void **)&d.pos_ptr, hx.pos_ptr.data(), sizeof(int32_t) * (m + 1));
    if (e == hipSuccess) e = up((void **)&d.rowpos, hx.rowpos.data(), sizeof(uint16_t) * d.npairs);
    if (e == hipSuccess) e = up((void **)&d.first, hx.first.data(), sizeof(int32_t) * hx.first.size());
    if (e == hipSuccess) e = up((void **)&d.pre, hx.pre.data(), sizeof(int32_t) * hx.pre.size());
    if (e == hipSuccess) e = hipStreamSynchronize(h->work);
    if (e != hipSuccess) {
        free_xwin(d);
        return hip_fail(e, "x-window upload");
    }
    d.ent_host = std::move(hx.ent);
    d.pair_off = std::move(hx.pair_off);
    d.bytes = (int64_t)((2 + vs) * nnz + 4 * (d.npairs + 1) + 4 * (m + 1) + 2 * d.npairs +
                        4 * (hx.first.size() + hx.pre.size()));
    return SPK_OK;
}

// Tiles and chunks of one (entries per wavefront, chunk target), uploaded.
spk_status build_plan(spk_handle h, const XwinData &d, int E, int64_t target, XwinPlan &pl)
{
    XwinHost view;   // the planner reads the pair layout only
    view.nwin = d.nwin;
    view.npairs = d.npairs;
    view.ent = d.ent_host;
    view.pair_off = d.pair_off;
    std::vector<uint32_t> tiles;
    std::vector<int32_t> tile_k, chunk_t, chunk_w;
    xwin_plan(view, E, target, tiles, tile_k, chunk_t, chunk_w);
    pl.ntiles = (int32_t)tiles.size() - 1;
    pl.nchunk = (int32_t)chunk_w.size();
    auto up = [&](void **dst, const void *src, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 16));
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, h->work);
        return e;
    };
    hipError_t e = up((void **)&pl.tiles, tiles.data(), sizeof(uint32_t) * tiles.size());
    if (e == hipSuccess) e = up((void **)&pl.tile_k, tile_k.data(), sizeof(int32_t) * tile_k.size());
    if (e == hipSuccess) e = up((void **)&pl.chunk_t, chunk_t.data(), sizeof(int32_t) * chunk_t.size());
    if (e == hipSuccess) e = up((void **)&pl.chunk_w, chunk_w.data(), sizeof(int32_t) * chunk_w.size());
    if (e == hipSuccess) e = hipStreamSynchronize(h->work);
    if (e != hipSuccess) return hip_fail(e, "x-window plan upload");
    pl.bytes = (int64_t)(8 * tiles.size() + 4 * chunk_t.size() + 4 * chunk_w.size());
    return SPK_OK;
}

spk_status get_xwin(spk_handle h, spk_mat *A, int kib, int E, int grid, XwinData **dout, XwinPlan **pout)
{
    XwinData *d = nullptr;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = A->xwin.find(kib);
        if (it != A->xwin.end()) d = &it->second;
    }
    if (!d) {
        XwinData nd;
        SPK_TRY(build_xwin(h, A, (int64_t)kib * 1024 / (int64_t)dtype_size(A->dtype), nd));
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = A->xwin.find(kib);
        if (it != A->xwin.end()) {
            free_xwin(nd);   // built meanwhile by another call
            d = &it->second;
        } else {
            A->bytes += nd.bytes;
            d = &A->xwin.emplace(kib, std::move(nd)).first->second;
        }
    }
    const auto key = std::make_pair(E, grid);
    XwinPlan *pl = nullptr;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = d->plans.find(key);
        if (it != d->plans.end()) pl = &it->second;
    }
    if (!pl) {
        XwinPlan np;
        const spk_status st = build_plan(h, *d, E, (int64_t)grid * h->num_cu, np);
        if (st != SPK_OK) {
            (void)hipFree(np.tiles);
            (void)hipFree(np.tile_k);
            (void)hipFree(np.chunk_t);
            (void)hipFree(np.chunk_w);
            return st;
        }
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = d->plans.find(key);
        if (it != d->plans.end()) {
            (void)hipFree(np.tiles);
            (void)hipFree(np.tile_k);
            (void)hipFree(np.chunk_t);
            (void)hipFree(np.chunk_w);
            pl = &it->second;
        } else {
            A->bytes += np.bytes;
            pl = &d->plans.emplace(key, np).first->second;
        }
    }
    *dout = d;
    *pout = pl;
    return SPK_OK;
}

}  // namespace

spk_status run_xwin(spk_handle h, const SpmvProblem &p, const spk_variant &v, hipStream_t s)
{
    spk_mat *A = p.mat;
    if (!A) return fail(SPK_ERR_ARG, "the x-window form needs a registered matrix");
    const XwinEntry *e = find_xwin_entry(v.block, v.group, v.lds);
    if (!e) return fail(SPK_ERR_NOT_FOUND, "x-window kernel not compiled");
    XwinData *d = nullptr;
    XwinPlan *pl = nullptr;
    SPK_TRY(get_xwin(h, A, v.group, v.lds, std::max(1, v.grid), &d, &pl));
    double *part = nullptr;
    if (d->npairs > 0) {
        {
            std::lock_guard<std::mutex> lk(h->mu);
            auto it = d->part.find(s);
            if (it != d->part.end()) part = it->second;
        }
        if (!part) {
            SPK_HIP(hipMalloc(&part, sizeof(double) * (size_t)d->npairs));
            std::lock_guard<std::mutex> lk(h->mu);
            auto it = d->part.find(s);
            if (it != d->part.end()) {
                (void)hipFree(part);   // made meanwhile by another call on this stream
                part = it->second;
            } else {
                d->part[s] = part;
                A->bytes += (int64_t)(sizeof(double) * (size_t)d->npairs);
            }
        }
        XwinArgs a{};
        a.tiles = pl->tiles;
        a.tile_k = pl->tile_k;
        a.chunk_t = pl->chunk_t;
        a.chunk_w = pl->chunk_w;
        a.ent = d->ent;
        a.ci = d->ci;
        a.val = d->val;
        a.x = p.x;
        a.n = A->ncols;
        a.part = part;
        a.nchunk = pl->nchunk;
        if (pl->nchunk > 0) SPK_HIP(e->fn[A->dtype](a, s));
    }
    XsumArgs sa{};
    sa.m = A->nrows;
    sa.rb = (int32_t)d->rb;
    sa.nwin = (int32_t)d->nwin;
    sa.first = d->first;
    sa.pre = d->pre;
    sa.pos_ptr = d->pos_ptr;
    sa.rowpos = d->rowpos;
    sa.part = part;
    sa.y = p.y;
    sa.w = p.w;
    sa.x = p.x;
    sa.alpha = p.alpha;
    SPK_HIP(launch_xwin_sum(A->dtype, p.fused, sa, s));
    return SPK_OK;
}

}  // namespace spk
