// serve.cpp -- a continuous-batching request loop for the Krylov-style step
// (y = A*x, w = alpha*y + x) over a pool of matrices.
//
// A scheduler thread owns the GPU side.  Each turn it
//   1. retires finished launches (event query): copies results from the
//      pinned staging block to the callers' buffers, stamps completion
//      times, frees slots and bytes;
//   2. while fewer launches than max_launches are in flight, admits queued
//      requests (all that arrived meanwhile, up to max_batch) in arrival
//      order while a request slot is free
//      and the HBM budget covers the request's vectors plus, if its matrix
//      is not resident, the matrix (idle matrices are evicted least recently
//      used first to make room; a matrix in use is never evicted);
//   3. launches the admitted group as one batched tile kernel on the next of
//      its streams, so groups admitted while others run overlap on the GPU:
//      the requests' x are copied into one pinned staging block, moved to
//      the device by one copy, and the results come back the same way
//      (large vectors in pinned caller buffers skip the staging block).
// The tile kernel is the batched one, with each matrix cut into tiles by the
// kernel of its shape class (the tiles live on the device with the matrix;
// a launch names them through a small request table), so a request's
// result does not depend on what it was batched with.  Mode 1 is the
// baseline: one request at a time with the plain unbatched kernels (SpMV,
// then WAXPY).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "copy_pool.h"
#include "device_common.h"
#include "internal.h"

namespace spk {

namespace {

size_t round_pow2(size_t n)
{
    size_t p = 256;
    while (p < n) p <<= 1;
    return p;
}

// Recycles device or pinned host blocks by power-of-two size (a free
// goes back to the pool: hipFree would wait for the whole device).
struct Pool {
    bool device;
    std::multimap<size_t, void *> free_;
    std::map<void *, size_t> size_of;
    int64_t held = 0, idle = 0;   // bytes allocated / of them in free_
    hipError_t get(size_t n, void **out)
    {
        const size_t sz = round_pow2(n);
        auto it = free_.find(sz);
        if (it != free_.end()) {
            *out = it->second;
            free_.erase(it);
            idle -= (int64_t)sz;
            return hipSuccess;
        }
        hipError_t e = device ? hipMalloc(out, sz) : hipHostMalloc(out, sz, hipHostMallocDefault);
        if (e == hipSuccess) {
            size_of[*out] = sz;
            held += (int64_t)sz;
        }
        return e;
    }
    void put(void *p)
    {
        if (!p) return;
        const size_t sz = size_of[p];
        free_.emplace(sz, p);
        idle += (int64_t)sz;
    }
    // releases idle blocks, largest first, until at most max_idle bytes stay
    void trim(int64_t max_idle)
    {
        while (idle > max_idle && !free_.empty()) {
            auto it = std::prev(free_.end());
            void *p = it->second;
            const size_t sz = it->first;
            free_.erase(it);
            size_of.erase(p);
            idle -= (int64_t)sz;
            held -= (int64_t)sz;
            if (device) (void)hipFree(p);
            else (void)hipHostFree(p);
        }
    }
    void release_all()
    {
        for (auto &kv : size_of) {
            if (device) (void)hipFree(kv.first);
            else (void)hipHostFree(kv.first);
        }
        free_.clear();
        size_of.clear();
        held = 0;
        idle = 0;
    }
};

struct PoolMat {
    int32_t dtype = SPK_F64;
    int64_t m = 0, n = 0, nnz = 0;
    int32_t *h_rp = nullptr, *h_ci = nullptr;
    void *h_val = nullptr;
    bool h_pinned = false;
    int32_t *d_rp = nullptr, *d_ci = nullptr;
    void *d_val = nullptr;
    BatchTile *d_tiles = nullptr;   // its tiles, on the device while resident (vector offsets 0)
    int64_t dev_bytes = 0;
    bool resident = false;
    bool upload_done = false;   // its upload event has been seen complete
    int refs = 0;
    double last_use = 0.0;
    hipEvent_t uploaded = nullptr;
    std::vector<BatchTile> tiles;   // row ranges of this matrix (pointers set when made resident)
};

struct Request {
    int32_t mat = 0;
    const void *x = nullptr;
    void *y = nullptr;
    void *w = nullptr;
    double t_arrival = 0.0, t_admit = -1.0, t_done = -1.0;
};

struct Flight {
    std::vector<std::pair<int64_t, Request>> reqs;
    std::vector<int64_t> off;   // vector offset of each request
    std::vector<char> direct;   // its vectors move between the caller's pinned buffers and the device
    void *dev = nullptr, *pin = nullptr;
    size_t y_off = 0, w_off = 0;
    int64_t vec_bytes = 0;
    int stream = 0;            // index of the stream it runs on
    double t_enqueued = 0.0;   // when its input copy was enqueued
    hipEvent_t done = nullptr;
    int dtype = SPK_F64;
};

}  // namespace

}  // namespace spk

struct spk_server_s {
    spk_handle h = nullptr;
    spk_serve_opts opts{};
    const spk::BatchEntry *entry = nullptr;
    std::vector<hipStream_t> streams;
    hipStream_t upload = nullptr;
    std::vector<int> stream_load;           // launches in flight per stream
    std::deque<spk::PoolMat> mats;          // guarded by mats_mu
    std::mutex mats_mu;                     // held by the scheduler for a whole turn
    std::atomic<int32_t> nmats{0};
    std::vector<spk::Request> reqs;        // by id, guarded by mu (stats)
    std::deque<std::pair<int64_t, spk::Request>> incoming;   // guarded by mu
    std::deque<std::pair<int64_t, spk::Request>> pending;    // scheduler only
    std::vector<spk::Flight> flights;
    std::vector<hipEvent_t> spare_events;
    spk::Pool dpool{true}, hpool{false};
    spk::Pool mpool{true};                  // device arrays of resident matrices
    spk::CopyPool copies;                   // used by the scheduler thread only
    int64_t used_mat = 0, used_vec = 0, peak = 0;
    int64_t inflight = 0;
    int64_t completed = 0, rejected = 0, batches = 0, uploads = 0, evictions = 0;
    double first_arrival = -1.0, last_done = 0.0, bytes_moved = 0.0;
    double stage_in_s = 0.0, stage_out_s = 0.0, device_s = 0.0;
    int64_t direct = 0;
    std::vector<int64_t> done_ids;
    std::mutex mu;
    std::condition_variable cv_in, cv_done;
    bool stop = false;
    spk_status error = SPK_OK;
    char error_msg[512] = {0};
    std::thread thr;
};

namespace spk {

namespace {

using Server = spk_server_s;

hipEvent_t take_event(Server *S)
{
    if (!S->spare_events.empty()) {
        hipEvent_t e = S->spare_events.back();
        S->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    return e;
}

int64_t vec_bytes_of(const PoolMat &M) { return (M.n + 2 * M.m) * (int64_t)dtype_size(M.dtype); }

// The matrix's device arrays go back to the server's matrix pool, where a
// later upload (on the same upload stream, so in order after this
// matrix's own copies) reuses them; idle blocks beyond a quarter of the
// budget are released.
void free_device_copy(Server *S, PoolMat &M)
{
    S->mpool.put(M.d_rp);
    S->mpool.put(M.d_ci);
    S->mpool.put(M.d_val);
    S->mpool.put(M.d_tiles);
    M.d_rp = M.d_ci = nullptr;
    M.d_val = nullptr;
    M.d_tiles = nullptr;
    S->mpool.trim(S->opts.hbm_budget / 4);
}

spk_status upload(Server *S, PoolMat &M);

spk_status make_resident(Server *S, PoolMat &M)
{
    const spk_status st = upload(S, M);
    if (st != SPK_OK) {
        // nothing of a failed upload stays allocated (copies already queued finish first)
        (void)hipStreamSynchronize(S->upload);
        free_device_copy(S, M);
        return st;
    }
    M.resident = true;
    M.upload_done = false;
    S->used_mat += M.dev_bytes;
    ++S->uploads;
    return SPK_OK;
}

spk_status upload(Server *S, PoolMat &M)
{
    const size_t vs = dtype_size(M.dtype);
    SPK_HIP(S->mpool.get(sizeof(int32_t) * (M.m + 1), (void **)&M.d_rp));
    SPK_HIP(S->mpool.get(sizeof(int32_t) * std::max<int64_t>(1, M.nnz), (void **)&M.d_ci));
    SPK_HIP(S->mpool.get(vs * std::max<int64_t>(1, M.nnz), &M.d_val));
    SPK_HIP(hipMemcpyAsync(M.d_rp, M.h_rp, sizeof(int32_t) * (M.m + 1), hipMemcpyHostToDevice, S->upload));
    if (M.nnz) {
        SPK_HIP(hipMemcpyAsync(M.d_ci, M.h_ci, sizeof(int32_t) * M.nnz, hipMemcpyHostToDevice, S->upload));
        SPK_HIP(hipMemcpyAsync(M.d_val, M.h_val, vs * M.nnz, hipMemcpyHostToDevice, S->upload));
    }
    if (!M.tiles.empty()) {
        for (BatchTile &t : M.tiles) {
            t.rp = M.d_rp;
            t.ci = M.d_ci;
            t.val = M.d_val;
            t.vec_off = 0;
        }
        SPK_HIP(S->mpool.get(sizeof(BatchTile) * M.tiles.size(), (void **)&M.d_tiles));
        // pageable source: the call returns once the tiles are staged
        SPK_HIP(hipMemcpyAsync(M.d_tiles, M.tiles.data(), sizeof(BatchTile) * M.tiles.size(), hipMemcpyHostToDevice,
                               S->upload));
        // the x windows of mode-1 tiles, after the columns and tiles arrive
        if (S->entry->xw > 0)
            SPK_HIP(launch_tile_windows(M.d_tiles, (int64_t)M.tiles.size(), S->entry->xw, S->upload));
    }
    if (!M.uploaded) SPK_HIP(hipEventCreateWithFlags(&M.uploaded, hipEventDisableTiming));
    SPK_HIP(hipEventRecord(M.uploaded, S->upload));
    return SPK_OK;
}

void evict(Server *S, PoolMat &M)
{
    // idle: no launch references it (refs == 0 and its last launch retired)
    free_device_copy(S, M);
    M.resident = false;
    S->used_mat -= M.dev_bytes;
    ++S->evictions;
}

// Frees room for `need` bytes by evicting idle matrices (LRU), never those
// listed in `keep`.  Returns whether the budget now covers `need`.
bool make_room(Server *S, int64_t need, const std::vector<int32_t> &keep)
{
    const int64_t budget = S->opts.hbm_budget;
    while (S->used_mat + S->used_vec + need > budget) {
        int32_t victim = -1;
        double oldest = 1e300;
        for (size_t i = 0; i < S->mats.size(); ++i) {
            const PoolMat &M = S->mats[i];
            if (!M.resident || M.refs > 0) continue;
            if (std::find(keep.begin(), keep.end(), (int32_t)i) != keep.end()) continue;
            if (M.last_use < oldest) {
                oldest = M.last_use;
                victim = (int32_t)i;
            }
        }
        if (victim < 0) return false;
        evict(S, S->mats[victim]);
    }
    return true;
}

void set_error(Server *S, spk_status st)
{
    if (S->error == SPK_OK) {
        S->error = st;
        snprintf(S->error_msg, sizeof S->error_msg, "%s", spk_last_error());
    }
}

// Vectors of at least this many bytes skip the staging copies when the
// caller's buffers are pinned host memory: the copy engines move them
// between those buffers and the device directly.  Below it one memcpy into
// the staging block costs less than a copy command of its own.
constexpr size_t kDirectMin = 128 << 10;

// Whether [p, p + n) lies inside one pinned host allocation of the HIP
// runtime (hipHostMalloc).  Pageable memory, or a pointer the runtime does
// not know, is not.
bool pinned_range(const void *p, size_t n)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (a.type != hipMemoryTypeHost) return false;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)const_cast<void *>(p)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const uintptr_t b = (uintptr_t)base, q = (uintptr_t)p;
    return q >= b && q + n <= b + size;
}

// Launches a group of admitted requests (all of one dtype).  Requests whose
// vectors are staged come first in the launch's vectors, then those copied
// directly from and to the callers' pinned buffers.
spk_status launch_group(Server *S, std::vector<std::pair<int64_t, Request>> &group)
{
    const int dtype = S->mats[group[0].second.mat].dtype;
    const size_t vs = dtype_size(dtype);
    Flight F;
    F.dtype = dtype;
    F.reqs = group;
    const bool batched = S->opts.mode != 1;
    // batched launches name each request's resident tiles through a table
    // [request records | request of each launch tile] staged before x
    std::vector<BatchReq> rq;
    int64_t ntiles = 0, total = 0, staged = 0;
    F.direct.assign(group.size(), 0);
    for (size_t k = 0; k < group.size(); ++k) {
        const Request &R = group[k].second;
        const PoolMat &M = S->mats[R.mat];
        const size_t nb = vs * (size_t)M.m;
        F.direct[k] = nb >= kDirectMin && pinned_range(R.x, nb) && pinned_range(R.y, nb) &&
                      (!R.w || pinned_range(R.w, nb));
        if (!F.direct[k]) staged += M.m;
    }
    F.off.assign(group.size(), 0);
    for (int pass = 0; pass < 2; ++pass)
        for (size_t k = 0; k < group.size(); ++k)
            if ((bool)F.direct[k] == (pass == 1)) {
                F.off[k] = total;
                total += S->mats[group[k].second.mat].m;
            }
    for (size_t k = 0; k < group.size(); ++k) {
        const PoolMat &M = S->mats[group[k].second.mat];
        if (batched) rq.push_back({M.d_tiles, F.off[k], (int32_t)ntiles, 0});
        ntiles += (int64_t)M.tiles.size();
    }
    // one staging block: [requests | tile map | x | y | w], 256-byte aligned parts
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t req_b = batched ? al(sizeof(BatchReq) * std::max<size_t>(1, rq.size())) : 0;
    const size_t map_b = batched ? al(sizeof(uint16_t) * (size_t)std::max<int64_t>(1, ntiles)) : 0;
    const size_t head_b = req_b + map_b;
    const size_t vec_b = al(vs * (size_t)std::max<int64_t>(1, total));
    const size_t in_b = head_b + vec_b;
    F.y_off = in_b;
    F.w_off = in_b + vec_b;
    const size_t all_b = in_b + 2 * vec_b;
    SPK_HIP(S->dpool.get(all_b, &F.dev));
    SPK_HIP(S->hpool.get(all_b, &F.pin));
    char *pin = (char *)F.pin;
    if (batched) {
        memcpy(pin, rq.data(), sizeof(BatchReq) * rq.size());
        uint16_t *map = (uint16_t *)(pin + req_b);
        for (size_t k = 0; k < rq.size(); ++k)
            std::fill(map + rq[k].first, map + rq[k].first + (int64_t)S->mats[group[k].second.mat].tiles.size(),
                      (uint16_t)k);
    }
    std::vector<CopyPool::Chunk> cp;
    for (size_t k = 0; k < group.size(); ++k) {
        const Request &R = group[k].second;
        const PoolMat &M = S->mats[R.mat];
        if (!F.direct[k]) cp.push_back({pin + head_b + vs * F.off[k], R.x, vs * (size_t)M.n});
    }
    const double t_stage = now_seconds();
    S->copies.copy(cp);
    // the stream with the fewest launches in flight (the lowest index among
    // equals): a launch does not queue behind another while a stream is idle
    F.stream = (int)(std::min_element(S->stream_load.begin(), S->stream_load.end()) - S->stream_load.begin());
    ++S->stream_load[(size_t)F.stream];
    // a launch that fails before it becomes a flight gives its stream back
    struct Unload {
        Server *S;
        int stream;
        bool keep = false;
        ~Unload()
        {
            if (!keep) --S->stream_load[(size_t)stream];
        }
    } unload{S, F.stream};
    hipStream_t s = S->streams[(size_t)F.stream];
    // order the launch after uploads still in flight (each matrix once)
    for (const auto &g : group) {
        PoolMat &M = S->mats[g.second.mat];
        if (M.upload_done) continue;
        if (hipEventQuery(M.uploaded) == hipSuccess) {
            M.upload_done = true;
            continue;
        }
        SPK_HIP(hipStreamWaitEvent(s, M.uploaded, 0));
    }
    char *dev = (char *)F.dev;
    if (head_b + vs * (size_t)staged > 0)
        SPK_HIP(hipMemcpyAsync(dev, pin, head_b + vs * (size_t)staged, hipMemcpyHostToDevice, s));
    for (size_t k = 0; k < group.size(); ++k)
        if (F.direct[k])
            SPK_HIP(hipMemcpyAsync(dev + head_b + vs * F.off[k], group[k].second.x,
                                   vs * (size_t)S->mats[group[k].second.mat].n, hipMemcpyHostToDevice, s));
    F.t_enqueued = now_seconds();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stage_in_s += F.t_enqueued - t_stage;
        S->direct += (int64_t)std::count(F.direct.begin(), F.direct.end(), (char)1);
    }
    const void *x = dev + head_b;
    void *y = dev + F.y_off;
    void *w = dev + F.w_off;
    if (S->opts.mode == 1) {
        // baseline: the plain unbatched kernels, SpMV then WAXPY
        const PoolMat &M = S->mats[group[0].second.mat];
        spk_csr view{M.m, M.n, M.nnz, M.dtype, M.d_rp, M.d_ci, M.d_val};
        SpmvProblem q;
        q.csr = &view;
        q.x = x;
        q.y = y;
        const spk_variant pv = plain_variant(SPK_OP_SPMV, M.nnz > 8 * M.m ? 1 : 0);
        SPK_TRY(run_spmv(S->h, q, pv, s));
        SPK_TRY(run_waxpy(S->h, M.dtype, M.m, S->opts.alpha, y, x, w, plain_variant(SPK_OP_WAXPY, 0), s));
    } else {
        SPK_TRY(launch_tiles(S->entry, dtype, nullptr, ntiles, S->opts.alpha, x, y, w, kBatchGrid, nullptr, 0, s,
                             (const BatchReq *)dev, (const uint16_t *)(dev + req_b)));
    }
    if (staged == total) {
        SPK_HIP(hipMemcpyAsync(pin + F.y_off, y, 2 * vec_b, hipMemcpyDeviceToHost, s));
    } else {
        if (staged > 0) {
            SPK_HIP(hipMemcpyAsync(pin + F.y_off, y, vs * (size_t)staged, hipMemcpyDeviceToHost, s));
            SPK_HIP(hipMemcpyAsync(pin + F.w_off, w, vs * (size_t)staged, hipMemcpyDeviceToHost, s));
        }
        for (size_t k = 0; k < group.size(); ++k) {
            if (!F.direct[k]) continue;
            const Request &R = group[k].second;
            const size_t nb = vs * (size_t)S->mats[R.mat].m;
            SPK_HIP(hipMemcpyAsync(R.y, dev + F.y_off + vs * F.off[k], nb, hipMemcpyDeviceToHost, s));
            if (R.w) SPK_HIP(hipMemcpyAsync(R.w, dev + F.w_off + vs * F.off[k], nb, hipMemcpyDeviceToHost, s));
        }
    }
    F.done = take_event(S);
    SPK_HIP(hipEventRecord(F.done, s));
    F.vec_bytes = 0;
    for (const auto &g : group) F.vec_bytes += vec_bytes_of(S->mats[g.second.mat]);
    ++S->batches;
    S->flights.push_back(std::move(F));
    unload.keep = true;
    return SPK_OK;
}

bool retire(Server *S)
{
    bool any = false;
    for (size_t i = 0; i < S->flights.size();) {
        Flight &F = S->flights[i];
        if (hipEventQuery(F.done) != hipSuccess) {
            ++i;
            continue;
        }
        const size_t vs = dtype_size(F.dtype);
        const double t = now_seconds();
        const char *pin = (const char *)F.pin;
        std::vector<CopyPool::Chunk> cp;
        for (size_t k = 0; k < F.reqs.size(); ++k) {
            if (F.direct[k]) continue;   // already in the caller's buffers
            const Request &R = F.reqs[k].second;
            const PoolMat &M = S->mats[R.mat];
            cp.push_back({R.y, pin + F.y_off + vs * F.off[k], vs * (size_t)M.m});
            if (R.w) cp.push_back({R.w, pin + F.w_off + vs * F.off[k], vs * (size_t)M.m});
        }
        S->copies.copy(cp);
        const double t_out = now_seconds();   // the results are in the callers' buffers
        double bytes = 0.0;
        for (size_t k = 0; k < F.reqs.size(); ++k) {
            const Request &R = F.reqs[k].second;
            PoolMat &M = S->mats[R.mat];
            M.refs--;
            M.last_use = t;
            bytes += (double)spmv_bytes(M.m, M.n, M.nnz, M.dtype, true);
        }
        S->dpool.put(F.dev);
        S->hpool.put(F.pin);
        S->spare_events.push_back(F.done);
        --S->stream_load[(size_t)F.stream];
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->used_vec -= F.vec_bytes;
            S->inflight -= (int64_t)F.reqs.size();
            S->completed += (int64_t)F.reqs.size();
            S->last_done = t_out;
            S->bytes_moved += bytes;
            S->device_s += t - F.t_enqueued;
            S->stage_out_s += t_out - t;
            for (const auto &r : F.reqs) {
                S->reqs[r.first].t_done = t_out;
                S->done_ids.push_back(r.first);
            }
        }
        S->cv_done.notify_all();
        S->flights.erase(S->flights.begin() + (long)i);
        any = true;
    }
    return any;
}

bool admit(Server *S)
{
    if (S->opts.mode == 1 && !S->flights.empty()) return false;
    if ((int64_t)S->flights.size() >= S->opts.max_launches) return false;
    std::vector<std::pair<int64_t, Request>> group;
    std::vector<int32_t> keep;
    int group_dtype = -1;
    int64_t group_vec = 0, group_tiles = 0;
    const int64_t max_group = S->opts.mode == 1 ? 1 : S->opts.max_batch;
    while (!S->pending.empty() && (int64_t)group.size() < max_group &&
           S->inflight + (int64_t)group.size() < S->opts.max_inflight) {
        const Request &R = S->pending.front().second;
        PoolMat &M = S->mats[R.mat];
        if (group_dtype >= 0 && M.dtype != group_dtype) break;
        if (!group.empty() && group_tiles + (int64_t)M.tiles.size() > kMaxLaunchTiles) break;
        const int64_t need = group_vec + vec_bytes_of(M) + (M.resident ? 0 : M.dev_bytes);
        keep.push_back(R.mat);
        if (!make_room(S, need, keep)) {
            keep.pop_back();
            break;  // head of the queue waits for memory (no overtaking)
        }
        if (!M.resident) {
            spk_status st = make_resident(S, M);
            if (st != SPK_OK) {
                set_error(S, st);
                break;
            }
        }
        M.refs++;
        M.last_use = now_seconds();
        group_dtype = M.dtype;
        group_vec += vec_bytes_of(M);
        group_tiles += (int64_t)M.tiles.size();
        group.push_back(S->pending.front());
        S->pending.pop_front();
    }
    if (group.empty()) return false;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->inflight += (int64_t)group.size();
        S->used_vec += group_vec;
        S->peak = std::max(S->peak, S->used_mat + S->used_vec);
        const double t = now_seconds();
        for (const auto &g : group) S->reqs[g.first].t_admit = t;
    }
    spk_status st = launch_group(S, group);
    if (st != SPK_OK) {
        // the group never reaches a flight: release it and count its
        // requests as rejected, so that waiters are not left behind
        set_error(S, st);
        for (const auto &g : group) S->mats[g.second.mat].refs--;
        std::lock_guard<std::mutex> lk(S->mu);
        S->inflight -= (int64_t)group.size();
        S->used_vec -= group_vec;
        S->rejected += (int64_t)group.size();
        S->completed += (int64_t)group.size();
        S->cv_done.notify_all();
    }
    return true;
}

void scheduler(Server *S)
{
    (void)hipSetDevice(S->h->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->incoming.empty() && S->pending.empty() && S->flights.empty()) {
                if (S->stop) break;
                S->cv_in.wait_for(lk, std::chrono::milliseconds(2));
            }
            while (!S->incoming.empty()) {
                S->pending.push_back(S->incoming.front());
                S->incoming.pop_front();
            }
            if (S->stop && S->error != SPK_OK) {
                // drop what cannot run
                S->pending.clear();
            }
        }
        bool progress;
        {
            std::lock_guard<std::mutex> mk(S->mats_mu);
            progress = retire(S);
            if (S->error == SPK_OK) progress = admit(S) || progress;
        }
        if (!progress && !S->flights.empty()) std::this_thread::yield();
        if (S->error != SPK_OK) {
            // unblock waiters: count dropped requests as rejected
            std::lock_guard<std::mutex> lk(S->mu);
            S->rejected += (int64_t)S->pending.size();
            S->completed += (int64_t)S->pending.size();
            S->pending.clear();
            S->cv_done.notify_all();
        }
    }
}

double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

}  // namespace spk

using namespace spk;

extern "C" {

spk_status spk_serve_create(spk_handle h, const spk_serve_opts *opts, spk_server *out)
{
    if (!h || !out) return fail(SPK_ERR_NULL, "handle/out is NULL");
    *out = nullptr;
    spk_serve_opts o{};
    if (opts) o = *opts;
    if (o.streams <= 0) o.streams = 4;
    if (o.max_inflight <= 0) o.max_inflight = 256;
    if (o.max_batch <= 0) o.max_batch = 64;
    if (o.max_batch > 4096) return fail(SPK_ERR_ARG, "max_batch above 4096");
    if (o.hbm_budget <= 0) o.hbm_budget = 200ll * 1000 * 1000 * 1000;
    if (o.mode != 0 && o.mode != 1) return fail(SPK_ERR_ARG, "mode must be 0 or 1");
    if (o.streams > 16) return fail(SPK_ERR_ARG, "at most 16 streams");
    if (o.max_launches < 0 || o.max_launches > 256) return fail(SPK_ERR_ARG, "max_launches must be in [0, 256]");
    if (o.max_launches == 0) o.max_launches = o.streams;
    DeviceGuard g(h);
    Server *S = new Server();
    S->h = h;
    S->opts = o;
    // with room for x in LDS: classes tuned to the windowed row stream run it
    S->entry = batch_entry(256, 2048, 256);
    for (int i = 0; i < (o.mode == 1 ? 1 : o.streams); ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            spk_serve_destroy(S);
            return fail(SPK_ERR_HIP, "stream creation failed");
        }
        S->streams.push_back(s);
    }
    S->stream_load.assign(S->streams.size(), 0);
    if (hipStreamCreateWithFlags(&S->upload, hipStreamNonBlocking) != hipSuccess) {
        spk_serve_destroy(S);
        return fail(SPK_ERR_HIP, "stream creation failed");
    }
    S->copies.start(3);   // three copy threads beside the scheduler
    S->thr = std::thread(scheduler, S);
    *out = S;
    return SPK_OK;
}

spk_status spk_serve_add_matrix(spk_server S, const spk_csr *A, int32_t *id)
{
    if (!S || !A || !id) return fail(SPK_ERR_NULL, "NULL argument");
    if (!dtype_ok(A->dtype)) return fail(SPK_ERR_DTYPE, "bad dtype %d", A->dtype);
    if (A->nrows < 0 || A->nnz < 0 || A->nrows != A->ncols) return fail(SPK_ERR_SHAPE, "the step needs a square matrix");
    if (A->nnz >= (1ll << 31) || A->nrows >= (1ll << 30)) return fail(SPK_ERR_SHAPE, "matrix too large");
    if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val))) return fail(SPK_ERR_NULL, "CSR arrays are NULL");
    const int32_t *rp = A->row_ptr;
    if (rp[0] != 0 || rp[A->nrows] != A->nnz) return fail(SPK_ERR_CSR, "row_ptr does not span [0, nnz]");
    for (int64_t i = 0; i < A->nrows; ++i)
        if (rp[i + 1] < rp[i]) return fail(SPK_ERR_CSR, "row_ptr decreases at row %lld", (long long)i);
    for (int64_t k = 0; k < A->nnz; ++k)
        if (A->col_idx[k] < 0 || A->col_idx[k] >= A->ncols) return fail(SPK_ERR_CSR, "column index out of range");
    PoolMat M;
    // tiles by the plan of the matrix's shape class
    const int cls = batch_class(A->nrows, A->nnz);
    int mode = batch_default_mode(cls, batch_wave_entries(*S->entry));
    spk_variant v{};
    if (spk_plan_get(S->h, batch_key(A->dtype, cls).c_str(), &v) == SPK_OK) mode = v.group;
    if (mode == 3) mode = 1;   // resident matrices keep 4-byte columns only
    cut_rows(rp, A->nrows, mode, batch_wave_entries(*S->entry), 1024, M.tiles);
    if ((int64_t)M.tiles.size() > kMaxLaunchTiles)
        return fail(SPK_ERR_SHAPE, "the matrix needs %lld tiles, more than one launch takes",
                    (long long)M.tiles.size());
    M.dtype = A->dtype;
    M.m = A->nrows;
    M.n = A->ncols;
    M.nnz = A->nnz;
    const size_t vs = dtype_size(A->dtype);
    DeviceGuard g(S->h);
    const size_t brp = sizeof(int32_t) * (M.m + 1), bci = sizeof(int32_t) * std::max<int64_t>(1, M.nnz),
                 bv = vs * std::max<int64_t>(1, M.nnz);
    M.h_pinned = hipHostMalloc((void **)&M.h_rp, brp, hipHostMallocDefault) == hipSuccess &&
                 hipHostMalloc((void **)&M.h_ci, bci, hipHostMallocDefault) == hipSuccess &&
                 hipHostMalloc(&M.h_val, bv, hipHostMallocDefault) == hipSuccess;
    if (!M.h_pinned) {
        if (M.h_rp) (void)hipHostFree(M.h_rp);
        if (M.h_ci) (void)hipHostFree(M.h_ci);
        if (M.h_val) (void)hipHostFree(M.h_val);
        M.h_rp = (int32_t *)malloc(brp);
        M.h_ci = (int32_t *)malloc(bci);
        M.h_val = malloc(bv);
        if (!M.h_rp || !M.h_ci || !M.h_val) {
            free(M.h_rp);
            free(M.h_ci);
            free(M.h_val);
            return fail(SPK_ERR_OOM, "host copy of the matrix");
        }
    }
    memcpy(M.h_rp, A->row_ptr, brp);
    if (M.nnz) {
        memcpy(M.h_ci, A->col_idx, sizeof(int32_t) * M.nnz);
        memcpy(M.h_val, A->val, vs * M.nnz);
    }
    M.dev_bytes = (int64_t)(brp + bci + bv);
    M.dev_bytes += (int64_t)(sizeof(BatchTile) * M.tiles.size());
    std::lock_guard<std::mutex> lk(S->mats_mu);
    if (M.dev_bytes + vec_bytes_of(M) > S->opts.hbm_budget) {
        if (M.h_pinned) {
            (void)hipHostFree(M.h_rp);
            (void)hipHostFree(M.h_ci);
            (void)hipHostFree(M.h_val);
        } else {
            free(M.h_rp);
            free(M.h_ci);
            free(M.h_val);
        }
        return fail(SPK_ERR_BUDGET, "matrix needs %lld bytes, budget is %lld", (long long)(M.dev_bytes + vec_bytes_of(M)),
                    (long long)S->opts.hbm_budget);
    }
    *id = (int32_t)S->mats.size();
    S->mats.push_back(std::move(M));
    S->nmats.store((int32_t)S->mats.size());
    return SPK_OK;
}

static spk_status submit_at(spk_server S, int32_t mat_id, const void *x, void *y, void *w, double t_arrival,
                            int64_t *req)
{
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->error != SPK_OK) return fail(S->error, "server failed: %s", S->error_msg);
    if (mat_id < 0 || mat_id >= S->nmats.load()) return fail(SPK_ERR_NOT_FOUND, "unknown matrix %d", mat_id);
    if (!x || !y) return fail(SPK_ERR_NULL, "x/y are NULL");
    Request R;
    R.mat = mat_id;
    R.x = x;
    R.y = y;
    R.w = w;
    R.t_arrival = t_arrival;
    const int64_t id = (int64_t)S->reqs.size();
    S->reqs.push_back(R);
    if (S->first_arrival < 0 || t_arrival < S->first_arrival) S->first_arrival = t_arrival;
    S->incoming.emplace_back(id, R);
    if (req) *req = id;
    S->cv_in.notify_one();
    return SPK_OK;
}

spk_status spk_serve_submit(spk_server S, int32_t mat_id, const void *x, void *y, void *w, int64_t *req)
{
    if (!S) return fail(SPK_ERR_NULL, "server is NULL");
    return submit_at(S, mat_id, x, y, w, now_seconds(), req);
}

spk_status spk_serve_poll(spk_server S, int64_t *ids, int32_t cap, int32_t *n)
{
    if (!S || !n || (cap > 0 && !ids)) return fail(SPK_ERR_NULL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    const int32_t k = (int32_t)std::min<size_t>((size_t)std::max(cap, 0), S->done_ids.size());
    for (int32_t i = 0; i < k; ++i) ids[i] = S->done_ids[i];
    S->done_ids.erase(S->done_ids.begin(), S->done_ids.begin() + k);
    *n = k;
    return SPK_OK;
}

spk_status spk_serve_drain(spk_server S)
{
    if (!S) return fail(SPK_ERR_NULL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->completed >= (int64_t)S->reqs.size(); });
    if (S->error != SPK_OK) return fail(S->error, "server failed: %s", S->error_msg);
    return SPK_OK;
}

spk_status spk_serve_replay(spk_server S, int64_t n, const double *arrival_s, const int32_t *mat_ids,
                            const void *const *x, void *const *y, void *const *w)
{
    if (!S || (n > 0 && (!arrival_s || !mat_ids || !x || !y))) return fail(SPK_ERR_NULL, "NULL argument");
    for (int64_t i = 0; i < n; ++i) {
        if (mat_ids[i] < 0 || mat_ids[i] >= S->nmats.load())
            return fail(SPK_ERR_NOT_FOUND, "request %lld: unknown matrix %d", (long long)i, mat_ids[i]);
        if (i > 0 && arrival_s[i] < arrival_s[i - 1]) return fail(SPK_ERR_ARG, "arrival times must not decrease");
    }
    const double t0 = now_seconds();
    for (int64_t i = 0; i < n; ++i) {
        const double target = t0 + arrival_s[i];
        for (;;) {
            const double dt = target - now_seconds();
            if (dt <= 0) break;
            if (dt > 200e-6) std::this_thread::sleep_for(std::chrono::microseconds((int64_t)((dt - 100e-6) * 1e6)));
            else std::this_thread::yield();
        }
        // latency counts from the scheduled arrival, so a late submission is
        // charged to the server
        SPK_TRY(submit_at(S, mat_ids[i], x[i], y[i], w ? w[i] : nullptr, target, nullptr));
    }
    return spk_serve_drain(S);
}

spk_status spk_serve_stats_get(spk_server S, spk_serve_stats *out)
{
    if (!S || !out) return fail(SPK_ERR_NULL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    memset(out, 0, sizeof *out);
    std::vector<double> lat;
    double mx = 0.0, sum = 0.0;
    for (const Request &R : S->reqs) {
        if (R.t_done < 0) continue;
        const double us = (R.t_done - R.t_arrival) * 1e6;
        lat.push_back(us);
        mx = std::max(mx, us);
        sum += us;
    }
    out->submitted = (int64_t)S->reqs.size();
    out->completed = S->completed;
    out->rejected = S->rejected;
    out->batches = S->batches;
    out->uploads = S->uploads;
    out->evictions = S->evictions;
    out->resident_bytes = S->used_mat;
    out->peak_bytes = S->peak;
    out->p50_us = percentile(lat, 0.50);
    out->p99_us = percentile(lat, 0.99);
    out->mean_us = lat.empty() ? 0.0 : sum / (double)lat.size();
    out->max_us = mx;
    out->wall_s = S->first_arrival >= 0 ? S->last_done - S->first_arrival : 0.0;
    out->bytes_moved = S->bytes_moved;
    out->stage_in_s = S->stage_in_s;
    out->stage_out_s = S->stage_out_s;
    out->device_s = S->device_s;
    out->direct = S->direct;
    return SPK_OK;
}

spk_status spk_serve_latencies(spk_server S, double *out_us, int64_t cap, int64_t *n)
{
    if (!S || !n || (cap > 0 && !out_us)) return fail(SPK_ERR_NULL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    const int64_t k = std::min<int64_t>(cap, (int64_t)S->reqs.size());
    for (int64_t i = 0; i < k; ++i) {
        const Request &R = S->reqs[i];
        out_us[i] = R.t_done < 0 ? -1.0 : (R.t_done - R.t_arrival) * 1e6;
    }
    *n = k;
    return SPK_OK;
}

spk_status spk_serve_latency_split(spk_server S, double *wait_us, double *run_us, int64_t cap, int64_t *n)
{
    if (!S || !n || (cap > 0 && (!wait_us || !run_us))) return fail(SPK_ERR_NULL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    const int64_t k = std::min<int64_t>(cap, (int64_t)S->reqs.size());
    for (int64_t i = 0; i < k; ++i) {
        const Request &R = S->reqs[i];
        const bool done = R.t_done >= 0 && R.t_admit >= 0;
        wait_us[i] = done ? (R.t_admit - R.t_arrival) * 1e6 : -1.0;
        run_us[i] = done ? (R.t_done - R.t_admit) * 1e6 : -1.0;
    }
    *n = k;
    return SPK_OK;
}

spk_status spk_serve_destroy(spk_server S)
{
    if (!S) return fail(SPK_ERR_NULL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_in.notify_all();
    if (S->thr.joinable()) S->thr.join();
    S->copies.finish();
    DeviceGuard g(S->h);
    for (hipStream_t s : S->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    if (S->upload) {
        (void)hipStreamSynchronize(S->upload);
        (void)hipStreamDestroy(S->upload);
    }
    for (PoolMat &M : S->mats) {
        free_device_copy(S, M);
        if (M.uploaded) (void)hipEventDestroy(M.uploaded);
        if (M.h_pinned) {
            (void)hipHostFree(M.h_rp);
            (void)hipHostFree(M.h_ci);
            (void)hipHostFree(M.h_val);
        } else {
            free(M.h_rp);
            free(M.h_ci);
            free(M.h_val);
        }
    }
    for (Flight &F : S->flights) hipEventDestroy(F.done);
    for (hipEvent_t e : S->spare_events) hipEventDestroy(e);
    S->dpool.release_all();
    S->hpool.release_all();
    S->mpool.release_all();
    delete S;
    return SPK_OK;
}

}  // extern "C"
