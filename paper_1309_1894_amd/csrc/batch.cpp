// batch.cpp -- many independent CSR instances in one launch.
//
// Planning: each instance gets a shape class (ceil(log2) of its mean row
// length); each class is served by one tile kernel (LDS row stream, or G
// lanes per row), taken from the plan DB or from spk_batch_tune.  Instances
// are cut into tiles of about `tile_nnz` entries; tiles are listed instance
// by instance and executed by one persistent launch that pulls them from a
// queue (or one workgroup per tile).  The launch is captured in a hipGraph
// once per (x, y, w, alpha) and replayed.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "device_common.h"
#include "internal.h"

// State a batch keeps per stream it runs on: the persistent kind's queue
// heads and completion count (a run on another stream must not share them:
// two runs in flight would claim each other's tiles), and the executable
// graph of the launch, which bakes those counters in.
struct BatchStream {
    uint32_t *ctr = nullptr;              // 8 per-XCD queue heads (256 B apart), then the done count
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *gx = nullptr;
    void *gy = nullptr, *gw = nullptr;
    double galpha = 0.0;
};

struct spk_batch_s {
    spk_handle h = nullptr;
    int32_t dtype = SPK_F64;
    int64_t count = 0;
    std::vector<int64_t> m, nnz, rp_off, nz_off, vec_off;
    std::vector<int32_t> rp_host;         // concatenated row_ptr (host copy)
    const int32_t *rp = nullptr, *ci = nullptr;
    const void *val = nullptr;
    spk_batch_opts opts{};
    const spk::BatchEntry *entry = nullptr;
    std::vector<int> cls;                 // class per instance
    std::map<int, int> mode;              // class -> tile mode
    std::vector<spk::BatchTile> tiles;
    spk::BatchTile *d_tiles = nullptr;
    int64_t d_tiles_cap = 0;
    uint8_t *c8 = nullptr;                // one-byte compact columns (laid out like the caller's col_idx)
    uint16_t *c16 = nullptr;              // two-byte compact columns (the same layout), made when needed
    int *d_need16 = nullptr;              // tiles that would take two-byte columns, while c16 is absent
    int64_t grid_persistent = 0;
    std::mutex mu;                        // guards `streams`
    std::map<hipStream_t, BatchStream> streams;
};

namespace spk {

constexpr size_t kCounterBytes = 9 * 256;

int batch_class(int64_t m, int64_t nnz)
{
    const double mean = m > 0 ? (double)nnz / (double)m : 0.0;
    int c = 0;
    while ((double)(1 << c) < mean && c < 20) ++c;
    return c;
}

int batch_default_mode(int cls, int entries)
{
    // mean row length <= 2^cls: short rows go through the LDS stream
    const int mean = 1 << cls;
    if (mean <= 64 && mean * 4 <= entries) return 0;
    return std::min(64, std::max(8, mean / 4));
}

std::string batch_key(int dtype, int cls)
{
    char b[64];
    snprintf(b, sizeof b, "batch:%s:c%d", dtype_name(dtype), cls);
    return b;
}

// Plan-DB key of the launch shape spk_batch_tune found for a dtype: block =
// threads per workgroup, lds = LDS tile entries per workgroup, grid = 1 for
// the persistent launch kind.
static std::string batch_launch_key(int dtype)
{
    return std::string("batch:") + dtype_name(dtype) + ":launch";
}

const BatchEntry *batch_entry(int block, int tile, int xw)
{
    int n = 0;
    const BatchEntry *t = batch_table(&n);
    for (int i = 0; i < n; ++i)
        if (t[i].block == block && t[i].tile == tile && t[i].xw == xw) return &t[i];
    return nullptr;
}

bool is_stream_mode(int mode) { return mode == 0 || mode == 1 || mode == 3; }

void cut_rows(const int32_t *rp, int64_t m, int mode, int entries, int64_t target, std::vector<BatchTile> &out)
{
    int64_t r = 0;
    while (r < m) {
        BatchTile t{};
        t.r0 = (int32_t)r;
        t.mode = mode;
        if (is_stream_mode(mode)) {
            if (rp[r + 1] - rp[r] > entries) {
                // a row that does not fit the wavefront's LDS slice gets one wavefront
                t.mode = 64;
                t.r1 = (int32_t)(r + 1);
                t.k0 = rp[t.r0];
                t.k1 = rp[t.r1];
                out.push_back(t);
                ++r;
                continue;
            }
            int64_t nz = 0, c = 0;
            while (r < m && c < 2 * 64) {
                const int64_t l = rp[r + 1] - rp[r];
                if (nz + l > entries) break;
                nz += l;
                ++r;
                ++c;
            }
            t.r1 = (int32_t)r;
        } else {
            // G lanes per row: passes of 64/G rows until about `target` entries
            const int64_t rows_per_pass = 64 / mode;
            int64_t r1 = r, nz = 0;
            while (r1 < m && nz < target) {
                const int64_t r2 = std::min<int64_t>(m, r1 + rows_per_pass);
                nz += rp[r2] - rp[r1];
                r1 = r2;
            }
            t.r1 = (int32_t)r1;
            r = r1;
        }
        t.k0 = rp[t.r0];
        t.k1 = rp[t.r1];
        out.push_back(t);
    }
}

spk_status launch_tiles(const BatchEntry *e, int dtype, const BatchTile *d_tiles, int64_t ntiles, double alpha,
                        const void *x, void *y, void *w, int kind, uint32_t *ctr, int64_t persistent_grid,
                        hipStream_t s, const BatchReq *reqs, const uint16_t *req_of_tile)
{
    if (ntiles == 0) return SPK_OK;
    if (ntiles > kMaxLaunchTiles)
        return fail(SPK_ERR_SHAPE, "%lld tiles are more than one launch takes (%lld)", (long long)ntiles,
                    (long long)kMaxLaunchTiles);
    if (reqs && kind != kBatchGrid) return fail(SPK_ERR_ARG, "request tables need the grid launch");
    union {
        BatchArgs<float> f;
        BatchArgs<double> d;
    } a;
    memset(&a, 0, sizeof a);
    auto fill = [&](auto &q) {
        using Q = std::remove_reference_t<decltype(q)>;
        using T = std::remove_const_t<std::remove_pointer_t<decltype(Q::x)>>;
        q.tiles = d_tiles;
        q.ntiles = (int32_t)ntiles;
        q.x = (const T *)x;
        q.y = (T *)y;
        q.w = (T *)w;
        q.alpha = (T)alpha;
        q.next = ctr;                              // 8 queue heads, 256 bytes apart
        q.done = ctr ? ctr + 8 * 64 : nullptr;     // then the completion count
        q.reqs = reqs;
        q.req_of_tile = reqs ? req_of_tile : nullptr;
    };
    if (dtype == SPK_F64) fill(a.d); else fill(a.f);
    const int64_t nw = e->block / 64;
    int64_t g = (ntiles + nw - 1) / nw;   // tile groups, one per workgroup
    // persistent: every XCD queue that holds tiles needs a workgroup of its
    // own (workgroup b serves queue b % 8), so at least min(8, ntiles)
    if (kind == kBatchPersistent)
        g = std::min<int64_t>(persistent_grid, std::max<int64_t>(g, std::min<int64_t>(8, ntiles)));
    SPK_HIP(e->fn[dtype][kind](dtype == SPK_F64 ? (const void *)&a.d : (const void *)&a.f, dim3((unsigned)g), s));
    return SPK_OK;
}

namespace {

void invalidate_graph(spk_batch b)
{
    // a replay may still be queued on any of the caller's streams: let it
    // finish before its executable graph goes (rare: a change of x, y, w,
    // alpha or of the plan)
    std::lock_guard<std::mutex> lk(b->mu);
    bool any = false;
    for (auto &kv : b->streams) any = any || kv.second.exec;
    if (any) (void)hipDeviceSynchronize();
    for (auto &kv : b->streams) {
        BatchStream &st = kv.second;
        if (st.exec) (void)hipGraphExecDestroy(st.exec);
        if (st.graph) (void)hipGraphDestroy(st.graph);
        st.exec = nullptr;
        st.graph = nullptr;
    }
}

// The state of stream s; on the first use of s, its queue counters are
// allocated and zeroed (an allocation and a synchronisation: not inside a
// graph capture, so a captured run needs an eager run on its stream first).
spk_status stream_state(spk_batch b, hipStream_t s, BatchStream **out)
{
    std::lock_guard<std::mutex> lk(b->mu);
    BatchStream &st = b->streams[s];
    if (!st.ctr) {
        uint32_t *c = nullptr;
        SPK_HIP(hipMalloc(&c, kCounterBytes));
        hipError_t e = hipMemsetAsync(c, 0, kCounterBytes, b->h->work);
        if (e == hipSuccess) e = hipStreamSynchronize(b->h->work);
        if (e != hipSuccess) {
            (void)hipFree(c);
            return hip_fail(e, "batch queue counters");
        }
        st.ctr = c;
    }
    *out = &st;
    return SPK_OK;
}

// Whether the batch's kernel can run mode-3 tiles (compact columns index a
// window of at most 256 entries of x in LDS).
bool compact_ok(const spk_batch b) { return b->entry->xw > 0 && b->entry->xw <= 256; }

// Tiles of instance i under `mode` (mode 3 on a kernel that cannot run it
// is cut as mode 1).
void cut_instance(const spk_batch b, int64_t i, int mode, std::vector<BatchTile> &out)
{
    if (mode == 3 && !compact_ok(b)) mode = 1;
    const size_t first = out.size();
    cut_rows(b->rp_host.data() + b->rp_off[i], b->m[i], mode, batch_wave_entries(*b->entry), b->opts.tile_nnz,
             out);
    const size_t vs = dtype_size(b->dtype);
    for (size_t k = first; k < out.size(); ++k) {
        out[k].rp = b->rp + b->rp_off[i];
        out[k].ci = b->ci + b->nz_off[i];
        out[k].val = (const char *)b->val + vs * b->nz_off[i];
        out[k].vec_off = b->vec_off[i];
    }
}

spk_status upload_tiles(spk_batch b, const std::vector<BatchTile> &tiles)
{
    if ((int64_t)tiles.size() > b->d_tiles_cap) {
        if (b->d_tiles) SPK_HIP(hipFree(b->d_tiles));
        b->d_tiles = nullptr;
        const int64_t cap = std::max<int64_t>(1, (int64_t)tiles.size());
        SPK_HIP(hipMalloc(&b->d_tiles, sizeof(BatchTile) * cap));
        b->d_tiles_cap = cap;
    }
    // the compact-column arrays of mode-3 tiles, sized like the caller's
    // col_idx span plus one 16-byte group (the kernel reads whole aligned
    // groups): one byte per entry at the first plan that has such tiles,
    // two bytes per entry once a tile needs them (a tile whose window is
    // wider than the kernel's room)
    bool any3 = false;
    for (const BatchTile &t : tiles) any3 = any3 || t.mode == 3;
    int64_t len = 0;
    for (int64_t i = 0; i < b->count; ++i) len = std::max<int64_t>(len, b->nz_off[i] + b->nnz[i]);
    len = (len + 15) / 16 * 16 + 16;
    if (any3 && !b->c8) {
        SPK_HIP(hipMalloc(&b->c8, (size_t)len));
        SPK_HIP(hipMalloc(&b->d_need16, sizeof(int)));
    }
    if (tiles.empty()) return SPK_OK;
    // the x windows of mode-1 and mode-3 tiles, for a kernel with room for
    // them; mode-3 tiles get their compact columns.  Ordered after any
    // launch already queued on the work stream that reads the old tiles.
    auto place = [&]() -> spk_status {
        SPK_HIP(hipMemcpyAsync(b->d_tiles, tiles.data(), sizeof(BatchTile) * tiles.size(), hipMemcpyHostToDevice,
                               b->h->work));
        if (b->d_need16) SPK_HIP(hipMemsetAsync(b->d_need16, 0, sizeof(int), b->h->work));
        if (b->entry->xw > 0)
            SPK_HIP(launch_tile_windows(b->d_tiles, (int64_t)tiles.size(), b->entry->xw, b->h->work, b->ci, b->c8,
                                        b->c16, b->d_need16));
        SPK_HIP(hipStreamSynchronize(b->h->work));
        return SPK_OK;
    };
    SPK_TRY(place());
    if (any3 && !b->c16 && b->entry->xw > 0) {
        int need = 0;
        SPK_HIP(hipMemcpy(&need, b->d_need16, sizeof(int), hipMemcpyDeviceToHost));
        if (need > 0) {
            SPK_HIP(hipMalloc(&b->c16, sizeof(uint16_t) * (size_t)len));
            SPK_TRY(place());
        }
    }
    return SPK_OK;
}

spk_status replan(spk_batch b)
{
    b->tiles.clear();
    for (int64_t i = 0; i < b->count; ++i) cut_instance(b, i, b->mode[b->cls[i]], b->tiles);
    invalidate_graph(b);
    if ((int64_t)b->tiles.size() > kMaxLaunchTiles)
        return fail(SPK_ERR_SHAPE, "the batch needs %lld tiles, more than one launch takes (%lld): split it",
                    (long long)b->tiles.size(), (long long)kMaxLaunchTiles);
    return upload_tiles(b, b->tiles);
}

// Launches the tile kernel over `ntiles` tiles already on the device, on
// stream s with s's queue counters.
spk_status launch(spk_batch b, int64_t ntiles, double alpha, const void *x, void *y, void *w, hipStream_t s)
{
    uint32_t *ctr = nullptr;
    if (b->opts.persistent == kBatchPersistent) {
        BatchStream *st = nullptr;
        SPK_TRY(stream_state(b, s, &st));
        ctr = st->ctr;
    }
    return launch_tiles(b->entry, b->dtype, b->d_tiles, ntiles, alpha, x, y, w, b->opts.persistent, ctr,
                        b->grid_persistent, s);
}

spk_status occupancy(spk_batch b)
{
    // resident workgroups per CU: the runtime's occupancy figure, raised to
    // what the kernel's static LDS (products + row offsets per wavefront)
    // and the 32 wavefront slots of a CU allow.  The persistent kernel never
    // waits on another workgroup, so a workgroup that does not fit at once
    // simply starts later.
    const int nw = b->entry->block / 64;
    const int64_t lds = (int64_t)b->entry->tile * 8 + (int64_t)nw * (2 * 64 + 1) * 4 +
                        (int64_t)nw * b->entry->xw * (int64_t)dtype_size(b->dtype);
    const int64_t by_lds = (160 * 1024) / std::max<int64_t>(1, lds);
    const int64_t by_waves = 32 / nw;
    int64_t per_cu = std::max<int64_t>(b->entry->occupancy[b->dtype](), std::min(by_lds, by_waves));
    if (b->opts.waves_per_cu > 0) per_cu = std::max<int64_t>(1, b->opts.waves_per_cu / nw);
    b->grid_persistent = std::max<int64_t>(1, per_cu) * b->h->num_cu;
    return SPK_OK;
}

}  // namespace

}  // namespace spk

using namespace spk;

extern "C" {

spk_status spk_batch_plan(spk_handle h, const spk_batch_desc *d, const spk_batch_opts *opts, spk_batch *out)
{
    if (!h || !d || !out) return fail(SPK_ERR_NULL, "NULL argument");
    *out = nullptr;
    if (!dtype_ok(d->dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", d->dtype);
    if (d->count < 0) return fail(SPK_ERR_SHAPE, "count < 0");
    if (d->count > 0 && (!d->m || !d->nnz || !d->rp_off || !d->nz_off || !d->vec_off))
        return fail(SPK_ERR_NULL, "size/offset arrays are NULL");
    if (d->count > 0 && (!d->row_ptr || !d->col_idx || !d->val)) return fail(SPK_ERR_NULL, "device arrays are NULL");
    spk_batch_opts o{};
    o.persistent = 1;
    o.use_graph = 1;
    if (opts) {
        o = *opts;
    }
    // block 0: the launch shape recorded by spk_batch_tune for this dtype,
    // if any (workgroup size, LDS tile, room for x and launch kind), else
    // 256 threads with 2048-entry tiles and no room for x
    const BatchEntry *e = nullptr;
    if (o.block == 0) {
        spk_variant lv{};
        if (spk_plan_get(h, batch_launch_key(d->dtype).c_str(), &lv) == SPK_OK &&
            (e = batch_entry(lv.block, lv.lds, lv.unroll)) != nullptr)
            o.persistent = lv.grid ? kBatchPersistent : kBatchGrid;
        o.block = e ? e->block : 256;
        if (!e) o.x_window = 0;
    }
    if (o.tile_nnz == 0) o.tile_nnz = 1024;
    if (o.persistent != kBatchGrid && o.persistent != kBatchPersistent)
        return fail(SPK_ERR_ARG, "persistent must be 0 or 1 (got %d)", o.persistent);
    if (o.tile_nnz < 0 || o.waves_per_cu < 0) return fail(SPK_ERR_ARG, "negative tile_nnz or waves_per_cu");
    if (!e) e = batch_entry(o.block, 2048, o.x_window);
    if (!e) return fail(SPK_ERR_ARG, "no batched kernel with block %d and x window %d", o.block, o.x_window);

    int64_t rp_total = 0;
    for (int64_t i = 0; i < d->count; ++i) {
        if (d->m[i] < 0 || d->nnz[i] < 0 || d->m[i] >= (1ll << 30)) return fail(SPK_ERR_SHAPE, "instance %lld size", (long long)i);
        rp_total = std::max<int64_t>(rp_total, d->rp_off[i] + d->m[i] + 1);
    }
    DeviceGuard g(h);
    spk_batch b = new spk_batch_s();
    b->h = h;
    b->dtype = d->dtype;
    b->count = d->count;
    b->opts = o;
    b->entry = e;
    b->rp = d->row_ptr;
    b->ci = d->col_idx;
    b->val = d->val;
    b->m.assign(d->m, d->m + d->count);
    b->nnz.assign(d->nnz, d->nnz + d->count);
    b->rp_off.assign(d->rp_off, d->rp_off + d->count);
    b->nz_off.assign(d->nz_off, d->nz_off + d->count);
    b->vec_off.assign(d->vec_off, d->vec_off + d->count);
    b->rp_host.resize((size_t)rp_total);
    auto bail = [&](spk_status s) {
        spk_batch_free(h, b);
        return s;
    };
    if (rp_total > 0) {
        if (d->row_ptr_host) {
            memcpy(b->rp_host.data(), d->row_ptr_host, sizeof(int32_t) * rp_total);
        } else {
            hipError_t he = hipDeviceSynchronize();
            if (he == hipSuccess)
                he = hipMemcpy(b->rp_host.data(), d->row_ptr, sizeof(int32_t) * rp_total, hipMemcpyDeviceToHost);
            if (he != hipSuccess) return bail(hip_fail(he, "row_ptr download"));
        }
    }
    for (int64_t i = 0; i < b->count; ++i) {
        const int32_t *rp = b->rp_host.data() + b->rp_off[i];
        if (rp[0] != 0 || rp[b->m[i]] != b->nnz[i])
            return bail(fail(SPK_ERR_CSR, "instance %lld: row_ptr does not span [0, nnz]", (long long)i));
        for (int64_t r = 0; r < b->m[i]; ++r)
            if (rp[r + 1] < rp[r])
                return bail(fail(SPK_ERR_CSR, "instance %lld: row_ptr decreases at row %lld", (long long)i,
                                 (long long)r));
    }
    b->cls.resize((size_t)b->count);
    for (int64_t i = 0; i < b->count; ++i) {
        const int c = batch_class(b->m[i], b->nnz[i]);
        b->cls[i] = c;
        if (!b->mode.count(c)) {
            spk_variant v{};
            if (spk_plan_get(h, batch_key(b->dtype, c).c_str(), &v) == SPK_OK && (v.group >= 0 && v.group <= 64))
                b->mode[c] = v.group;
            else
                b->mode[c] = batch_default_mode(c, batch_wave_entries(*e));
        }
    }
    spk_status st = occupancy(b);
    if (st == SPK_OK) st = replan(b);
    if (st != SPK_OK) return bail(st);
    *out = b;
    return SPK_OK;
}

spk_status spk_batch_run(spk_handle h, spk_batch b, double alpha, const void *x, void *y, void *w, spk_stream stream)
{
    if (!h || !b) return fail(SPK_ERR_NULL, "handle/batch is NULL");
    if (b->h != h) return fail(SPK_ERR_ARG, "batch belongs to another handle");
    if (b->count == 0 || b->tiles.empty()) return SPK_OK;
    if (!x || !y) return fail(SPK_ERR_NULL, "x/y are NULL");
    DeviceGuard g(h);
    hipStream_t s = (hipStream_t)stream;
    if (!b->opts.use_graph) return launch(b, (int64_t)b->tiles.size(), alpha, x, y, w, s);
    BatchStream *st = nullptr;
    SPK_TRY(stream_state(b, s, &st));
    if (!st->exec || st->gx != x || st->gy != y || st->gw != w || st->galpha != alpha) {
        if (st->exec) {
            // a replay of the old graph may still be queued on s
            SPK_HIP(hipStreamSynchronize(s));
            (void)hipGraphExecDestroy(st->exec);
            (void)hipGraphDestroy(st->graph);
            st->exec = nullptr;
            st->graph = nullptr;
        }
        // captured on the library's own stream (s may itself be capturing),
        // with s's counters, for replay on s
        SPK_HIP(hipStreamSynchronize(h->work));
        SPK_HIP(hipStreamBeginCapture(h->work, hipStreamCaptureModeThreadLocal));
        spk_status ls = launch_tiles(b->entry, b->dtype, b->d_tiles, (int64_t)b->tiles.size(), alpha, x, y, w,
                                     b->opts.persistent, st->ctr, b->grid_persistent, h->work);
        hipGraph_t graph = nullptr;
        const hipError_t ce = hipStreamEndCapture(h->work, &graph);
        if (ls != SPK_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return ls;
        }
        if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
        const hipError_t ie = hipGraphInstantiate(&st->exec, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(graph);
            st->exec = nullptr;
            return hip_fail(ie, "hipGraphInstantiate");
        }
        st->graph = graph;
        st->gx = x;
        st->gy = y;
        st->gw = w;
        st->galpha = alpha;
    }
    SPK_HIP(hipGraphLaunch(st->exec, s));
    return SPK_OK;
}

spk_status spk_batch_info(spk_handle h, spk_batch b, int64_t *tiles, int32_t *classes, int64_t *bytes)
{
    if (!h || !b) return fail(SPK_ERR_NULL, "handle/batch is NULL");
    if (tiles) *tiles = (int64_t)b->tiles.size();
    if (classes) *classes = (int32_t)b->mode.size();
    if (bytes) {
        int64_t t = 0;
        for (int64_t i = 0; i < b->count; ++i) t += spmv_bytes(b->m[i], b->m[i], b->nnz[i], b->dtype, true);
        *bytes = t;
    }
    return SPK_OK;
}

spk_status spk_batch_tune(spk_handle h, spk_batch b, double alpha, const void *x, void *y, void *w,
                          const spk_tune_opts *opts, spk_tune_report *report)
{
    if (!h || !b || !report) return fail(SPK_ERR_NULL, "NULL argument");
    if (!x || !y) return fail(SPK_ERR_NULL, "x/y are NULL");
    spk_tune_opts o{};
    if (opts) o = *opts;
    const int reps = o.reps > 0 ? o.reps : 10;
    const int warmup = o.warmup > 0 ? o.warmup : 2;
    const double tau = o.tau > 0 ? o.tau : (b->dtype == SPK_F64 ? 1e-12 : 1e-5);
    memset(report, 0, sizeof *report);
    DeviceGuard g(h);
    SPK_HIP(hipDeviceSynchronize());
    hipStream_t s = h->work;
    const size_t vs = dtype_size(b->dtype);
    int64_t nvec = 0;
    for (int64_t i = 0; i < b->count; ++i) nvec = std::max<int64_t>(nvec, b->vec_off[i] + b->m[i]);
    if (nvec == 0) return SPK_OK;

    // Reference (Section 2: the unannotated program's results): the
    // library's plain kernel -- one lane per row, the fused step when w is
    // given -- run instance by instance on borrowed views of the batch's
    // arrays.  It shares no code with the tile kernels it judges.  Its
    // output stays in the caller's y / w and is kept in native precision
    // too, and every trial starts from it, so rows a trial does not
    // rewrite (other classes, gaps between instances) hold reference values.
    double *ref_y = nullptr, *ref_w = nullptr, *scale = nullptr, *scale_w = nullptr;
    void *nat_y = nullptr, *nat_w = nullptr;
    unsigned long long *bad = nullptr, *hbad = nullptr;
    struct Free {
        std::vector<void *> d;
        void *hp = nullptr;
        ~Free()
        {
            for (void *p : d) (void)hipFree(p);
            if (hp) (void)hipHostFree(hp);
        }
    } fr;
    SPK_HIP(hipMalloc(&ref_y, 8 * nvec)); fr.d.push_back(ref_y);
    SPK_HIP(hipMalloc(&nat_y, vs * nvec)); fr.d.push_back(nat_y);
    SPK_HIP(hipMalloc(&scale, 8 * nvec)); fr.d.push_back(scale);
    SPK_HIP(hipMalloc(&bad, 8)); fr.d.push_back(bad);
    SPK_HIP(hipHostMalloc((void **)&hbad, 8, hipHostMallocDefault)); fr.hp = hbad;
    if (w) {
        SPK_HIP(hipMalloc(&ref_w, 8 * nvec)); fr.d.push_back(ref_w);
        SPK_HIP(hipMalloc(&nat_w, vs * nvec)); fr.d.push_back(nat_w);
        SPK_HIP(hipMalloc(&scale_w, 8 * nvec)); fr.d.push_back(scale_w);
    }
    {
        const spk_variant plain = plain_variant(w ? SPK_OP_SPMV_WAXPY : SPK_OP_SPMV, 0);
        for (int64_t i = 0; i < b->count; ++i) {
            if (b->m[i] == 0) continue;
            spk_csr view{};
            view.nrows = b->m[i];
            view.ncols = b->m[i];
            view.nnz = b->nnz[i];
            view.dtype = b->dtype;
            view.row_ptr = b->rp + b->rp_off[i];
            view.col_idx = b->ci + b->nz_off[i];
            view.val = (const char *)b->val + vs * b->nz_off[i];
            SpmvProblem q;
            q.csr = &view;
            q.fused = w != nullptr;
            q.alpha = alpha;
            q.x = (const char *)x + vs * b->vec_off[i];
            q.y = (char *)y + vs * b->vec_off[i];
            q.w = w ? (char *)w + vs * b->vec_off[i] : nullptr;
            SPK_TRY(run_spmv(h, q, plain, s));
        }
    }
    SPK_HIP(hipMemcpyAsync(nat_y, y, vs * nvec, hipMemcpyDeviceToDevice, s));
    SPK_HIP(launch_widen(b->dtype, nvec, y, ref_y, s));
    if (w) {
        SPK_HIP(hipMemcpyAsync(nat_w, w, vs * nvec, hipMemcpyDeviceToDevice, s));
        SPK_HIP(launch_widen(b->dtype, nvec, w, ref_w, s));
    }
    SPK_HIP(hipMemsetAsync(scale, 0, 8 * nvec, s));   // gaps between instances: exact match required
    SPK_HIP(launch_tiles_absum(b->dtype, b->d_tiles, (int64_t)b->tiles.size(), x, scale, s));
    if (w) {
        std::vector<double> sc((size_t)nvec), wr((size_t)nvec);
        SPK_HIP(hipMemcpyAsync(sc.data(), scale, 8 * nvec, hipMemcpyDeviceToHost, s));
        SPK_HIP(hipMemcpyAsync(wr.data(), ref_w, 8 * nvec, hipMemcpyDeviceToHost, s));
        SPK_HIP(hipStreamSynchronize(s));
        const double eps = b->dtype == SPK_F64 ? 0x1p-52 : 0x1p-23;
        for (int64_t i = 0; i < nvec; ++i) sc[i] = std::fabs(alpha) * sc[i] + 2.0 * eps * std::fabs(wr[i]) / tau;
        SPK_HIP(hipMemcpyAsync(scale_w, sc.data(), 8 * nvec, hipMemcpyHostToDevice, s));
    }
    if (o.ref_host) {
        // a caller-supplied reference y (FP64, nvec entries) replaces the
        // plain kernels' y; its tolerance scale stays the batch's own
        SPK_HIP(hipMemcpyAsync(ref_y, o.ref_host, 8 * nvec, hipMemcpyHostToDevice, s));
    }
    SPK_HIP(hipStreamSynchronize(s));

    std::vector<hipEvent_t> ev(2 * (size_t)reps);
    for (auto &e : ev) SPK_HIP(timing_event(&e));
    struct EvFree {
        std::vector<hipEvent_t> &e;
        ~EvFree() { for (auto x : e) (void)hipEventDestroy(x); }
    } ef{ev};

    int tried = 0, rejected = 0, resumed = 0, fresh = 0;
    double total_best = 0.0, total_plain = 0.0;

    // The journal (opts->resume): every timed point is filed under a key
    // naming the batch (its sizes, dtype and whether w is written) and the
    // context the point was timed in -- the per-class modes for a launch
    // shape, the launch shape for a class's mode.
    std::string bkey;
    if (o.resume) {
        uint64_t f = fnv1a(&b->count, sizeof b->count);
        f = fnv1a(b->m.data(), sizeof(int64_t) * b->m.size(), f);
        f = fnv1a(b->nnz.data(), sizeof(int64_t) * b->nnz.size(), f);
        f = fnv1a(b->vec_off.data(), sizeof(int64_t) * b->vec_off.size(), f);
        char k[96];
        snprintf(k, sizeof k, "batch|%s|%016llx|w%d", dtype_name(b->dtype), (unsigned long long)f, w ? 1 : 0);
        bkey = k;
    }
    auto modes_key = [&]() {
        std::string k;
        for (const auto &kv : b->mode) k += std::to_string(kv.first) + ":" + std::to_string(kv.second) + ",";
        return k;
    };
    // the state a search cut short leaves behind: the plan it started from
    const BatchEntry *entry0 = b->entry;
    const int pers0 = b->opts.persistent;
    const std::map<int, int> mode0 = b->mode;
    auto interrupted = [&]() -> spk_status {
        b->entry = entry0;
        b->opts.persistent = pers0;
        b->mode = mode0;
        SPK_TRY(occupancy(b));
        SPK_TRY(replan(b));
        report->tried = tried;
        report->rejected = rejected;
        report->resumed = resumed;
        return fail(SPK_ERR_INTERRUPTED, "search stopped after %d new points", fresh);
    };
    // a point from the journal, or -- unless the search is to stop -- a fresh one
    auto journaled = [&](const std::string &key, const spk_variant &v, double *med) {
        if (o.resume && point_get(h, key, v, med)) {
            ++resumed;
            return true;
        }
        return false;
    };
    auto must_stop = [&]() { return o.stop_after > 0 && fresh >= o.stop_after; };

    // times `ntiles` tiles already uploaded; rejects (returns -1) when the
    // output disagrees with the reference
    auto validate_and_time = [&](int64_t ntiles, double *med) -> spk_status {
        *med = -1.0;
        SPK_HIP(hipMemsetAsync(bad, 0, 8, s));
        SPK_HIP(hipMemcpyAsync(y, nat_y, vs * nvec, hipMemcpyDeviceToDevice, s));
        if (w) SPK_HIP(hipMemcpyAsync(w, nat_w, vs * nvec, hipMemcpyDeviceToDevice, s));
        SPK_TRY(launch(b, ntiles, alpha, x, y, w, s));
        SPK_HIP(launch_check(b->dtype, 0, nvec, y, ref_y, scale, tau, bad, s));
        if (w) SPK_HIP(launch_check(b->dtype, 0, nvec, w, ref_w, scale_w, tau, bad, s));
        SPK_HIP(hipMemcpyAsync(hbad, bad, 8, hipMemcpyDeviceToHost, s));
        SPK_HIP(hipStreamSynchronize(s));
        if (*hbad) {
            ++rejected;
            return SPK_OK;
        }
        for (int r = 0; r < warmup; ++r) SPK_TRY(launch(b, ntiles, alpha, x, y, w, s));
        for (int r = 0; r < reps; ++r) {
            if (o.flush) SPK_TRY(spk_flush_cache(h, (spk_stream)s));
            SPK_HIP(hipEventRecord(ev[2 * r], s));
            SPK_TRY(launch(b, ntiles, alpha, x, y, w, s));
            SPK_HIP(hipEventRecord(ev[2 * r + 1], s));
        }
        SPK_HIP(hipStreamSynchronize(s));
        std::vector<double> t;
        for (int r = 0; r < reps; ++r) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]);
            t.push_back(ms * 1e3);
        }
        std::sort(t.begin(), t.end());
        *med = t[t.size() / 2];
        ++tried;
        return SPK_OK;
    };

    // launch configuration: workgroup size / LDS tile and persistence,
    // timed on the whole batch with the current per-class kernels; run
    // before the per-class search and once more after it (the shape that
    // wins with the default kernels need not win with the tuned ones)
    auto pick_launch = [&]() -> spk_status {
        int n = 0;
        const BatchEntry *tab = batch_table(&n);
        const BatchEntry *best_e = b->entry;
        int best_p = b->opts.persistent;
        double best_t = 1e300;
        const std::string key = bkey + "|launch|" + modes_key();
        for (int i = 0; i < n; ++i) {
            for (int pers : {kBatchGrid, kBatchPersistent}) {
                spk_variant pv{};
                pv.block = tab[i].block;
                pv.lds = tab[i].tile;
                pv.unroll = tab[i].xw;
                pv.grid = pers;
                double med = 0;
                if (!journaled(key, pv, &med)) {
                    if (must_stop()) return interrupted();
                    ++fresh;
                    b->entry = &tab[i];
                    b->opts.persistent = pers;
                    SPK_TRY(occupancy(b));
                    SPK_TRY(replan(b));
                    SPK_TRY(validate_and_time((int64_t)b->tiles.size(), &med));
                    if (o.resume && med > 0) point_put(h, key, pv, med);
                }
                if (o.verbose)
                    fprintf(stderr, "spk_batch_tune: block %d tile %d x window %d persistent %d: %.2f us\n",
                            tab[i].block, tab[i].tile, tab[i].xw, pers, med);
                if (med > 0 && med < best_t) {
                    best_t = med;
                    best_e = &tab[i];
                    best_p = pers;
                }
            }
        }
        b->entry = best_e;
        b->opts.persistent = best_p;
        SPK_TRY(occupancy(b));
        SPK_TRY(replan(b));
        return SPK_OK;
    };
    SPK_TRY(pick_launch());

    std::map<int, std::vector<int64_t>> by_class;
    std::map<int, double> class_best;
    for (int64_t i = 0; i < b->count; ++i) by_class[b->cls[i]].push_back(i);
    for (auto &kv : by_class) {
        const int c = kv.first;
        double best = 1e300;
        int best_mode = b->mode[c];
        double plain_time = -1.0;
        char ctx[64];
        snprintf(ctx, sizeof ctx, "|c%d|%d,%d,%d,%d", c, b->entry->block, b->entry->tile, b->entry->xw,
                 b->opts.persistent);
        const std::string key = bkey + ctx;
        for (int mode : {0, 1, 3, 2, 4, 8, 16, 32, 64}) {
            spk_variant pv{};
            pv.group = mode;
            double med = 0;
            if (journaled(key, pv, &med)) {
                if (o.verbose) fprintf(stderr, "spk_batch_tune: class %d mode %d: %.2f us (journal)\n", c, mode, med);
                if (mode == batch_default_mode(c, batch_wave_entries(*b->entry))) plain_time = med;
                if (med < best) {
                    best = med;
                    best_mode = mode;
                }
                continue;
            }
            if (must_stop()) return interrupted();
            ++fresh;
            // modes 1 and 3 are timed with the kernel of the same shape
            // that has room for x (without that room mode 1 would run as
            // mode 0, and mode 3 as mode 1)
            const BatchEntry *keep = b->entry;
            if (mode == 1 || mode == 3) {
                const BatchEntry *xe = keep->xw > 0 ? keep : batch_entry(keep->block, keep->tile, 256);
                if (!xe) continue;
                b->entry = xe;
                SPK_TRY(occupancy(b));
            }
            std::vector<BatchTile> tl;
            for (int64_t i : kv.second) cut_instance(b, i, mode, tl);
            spk_status ts = upload_tiles(b, tl);
            // only this class's rows are rewritten by the trial launches
            if (ts == SPK_OK) ts = validate_and_time((int64_t)tl.size(), &med);
            if (b->entry != keep) {
                b->entry = keep;
                SPK_TRY(occupancy(b));
            }
            SPK_TRY(ts);
            if (med < 0) continue;
            if (o.resume) point_put(h, key, pv, med);
            if (o.verbose) fprintf(stderr, "spk_batch_tune: class %d mode %d: %.2f us\n", c, mode, med);
            if (mode == batch_default_mode(c, batch_wave_entries(*b->entry))) plain_time = med;
            if (med < best) {
                best = med;
                best_mode = mode;
            }
        }
        b->mode[c] = best_mode;
        class_best[c] = best;
        total_best += best;
        total_plain += plain_time > 0 ? plain_time : best;
    }
    SPK_TRY(replan(b));
    SPK_TRY(pick_launch());
    if (tried + resumed == 0) {
        report->rejected = rejected;
        return fail(SPK_ERR_VALIDATION, "no tile kernel reproduced the reference (%d rejected)", rejected);
    }
    if (resumed > 0) {
        // a plan built from journaled points is checked against this batch's reference
        const int tried0 = tried, rejected0 = rejected;
        double med = 0;
        SPK_TRY(validate_and_time((int64_t)b->tiles.size(), &med));
        tried = tried0;
        rejected = rejected0;
        if (med < 0) {
            b->entry = entry0;
            b->opts.persistent = pers0;
            b->mode = mode0;
            SPK_TRY(occupancy(b));
            SPK_TRY(replan(b));
            return fail(SPK_ERR_VALIDATION, "the plan from journaled points does not reproduce this batch's reference");
        }
    }
    if (o.record) {
        for (const auto &kv : class_best) {
            spk_variant v{};
            v.format = is_stream_mode(b->mode[kv.first]) ? SPK_FMT_ADAPTIVE : SPK_FMT_VECTOR;
            v.block = b->entry->block;
            v.group = b->mode[kv.first];
            v.lds = b->entry->tile;
            v.streams = 1;
            const std::string key = batch_key(b->dtype, kv.first);
            spk_plan_put(h, key.c_str(), &v);
            db_append(h, key, v, kv.second);
        }
        spk_variant lv{};
        lv.block = b->entry->block;
        lv.lds = b->entry->tile;
        lv.unroll = b->entry->xw;
        lv.grid = b->opts.persistent == kBatchPersistent ? 1 : 0;
        lv.streams = 1;
        const std::string key = batch_launch_key(b->dtype);
        spk_plan_put(h, key.c_str(), &lv);
        db_append(h, key, lv, total_best);
    }
    // leave a full-batch result in the caller's buffers
    SPK_TRY(launch(b, (int64_t)b->tiles.size(), alpha, x, y, w, s));
    SPK_HIP(hipStreamSynchronize(s));
    report->tried = tried;
    report->rejected = rejected;
    report->resumed = resumed;
    report->best_us = total_best;
    report->plain_us = total_plain;
    report->best.block = b->entry->block;
    report->best.lds = b->entry->tile;
    snprintf(report->class_key, sizeof report->class_key, "batch:%s:%d-classes", dtype_name(b->dtype),
             (int)by_class.size());
    return SPK_OK;
}

spk_status spk_batch_tile_modes(spk_handle h, spk_batch b, int64_t *tiles, int64_t *entries)
{
    if (!h || !b || !tiles) return fail(SPK_ERR_NULL, "NULL argument");
    if (b->h != h) return fail(SPK_ERR_ARG, "batch belongs to another handle");
    for (int i = 0; i <= 64; ++i) {
        tiles[i] = 0;
        if (entries) entries[i] = 0;
    }
    if (b->tiles.empty()) return SPK_OK;
    DeviceGuard g(h);
    std::vector<BatchTile> t(b->tiles.size());
    SPK_HIP(hipStreamSynchronize(h->work));
    SPK_HIP(hipMemcpy(t.data(), b->d_tiles, sizeof(BatchTile) * t.size(), hipMemcpyDeviceToHost));
    for (const BatchTile &x : t) {
        if (x.mode < 0 || x.mode > 64) continue;
        ++tiles[x.mode];
        if (entries) entries[x.mode] += (int64_t)x.k1 - x.k0;
    }
    return SPK_OK;
}

spk_status spk_batch_config(spk_handle h, spk_batch b, spk_batch_opts *out)
{
    if (!h || !b || !out) return fail(SPK_ERR_NULL, "NULL argument");
    *out = b->opts;
    out->block = b->entry->block;
    out->tile_nnz = b->entry->tile;
    out->x_window = b->entry->xw;
    out->waves_per_cu = (int32_t)(b->grid_persistent / std::max(1, b->h->num_cu)) * (b->entry->block / 64);
    return SPK_OK;
}

spk_status spk_batch_free(spk_handle h, spk_batch b)
{
    if (!h || !b) return fail(SPK_ERR_NULL, "handle/batch is NULL");
    DeviceGuard g(h);
    (void)hipDeviceSynchronize();
    invalidate_graph(b);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->c8) (void)hipFree(b->c8);
    if (b->c16) (void)hipFree(b->c16);
    if (b->d_need16) (void)hipFree(b->d_need16);
    for (auto &kv : b->streams)
        if (kv.second.ctr) (void)hipFree(kv.second.ctr);
    delete b;
    return SPK_OK;
}

}  // extern "C"
