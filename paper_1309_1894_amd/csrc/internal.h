// internal.h -- host-side state of libspk shared by the API, tuner, batch
// planner and serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdint>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/spk.h"
#include "batch_types.h"
#include "kernels.h"

#ifndef SPK_BUILD_ID
#define SPK_BUILD_ID "dev"
#endif

namespace spk {

// ---------------------------------------------------------------- errors

spk_status fail(spk_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
spk_status hip_fail(hipError_t e, const char *what);

#define SPK_HIP(call)                                       \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return ::spk::hip_fail(e_, #call); \
    } while (0)

#define SPK_TRY(call)                          \
    do {                                       \
        spk_status s_ = (call);                \
        if (s_ != SPK_OK) return s_;           \
    } while (0)

inline size_t dtype_size(int dtype) { return dtype == SPK_F64 ? 8 : 4; }
inline bool dtype_ok(int dtype) { return dtype == SPK_F32 || dtype == SPK_F64; }
const char *dtype_name(int dtype);

// True when [a, a+na) and [b, b+nb) share a byte.
inline bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return na && nb && x < y + nb && y < x + na;
}

// ------------------------------------------------------------- matrices

struct SellData {
    int32_t C = 0;
    int64_t nslices = 0, padded = 0;
    int64_t *ptr = nullptr;     // nslices + 1
    int32_t *len = nullptr;     // nrows
    int32_t *ci = nullptr;      // padded
    void *val = nullptr;        // padded
    int64_t bytes = 0;
};

// Column-blocked form of a matrix (SPK_FMT_COLBLOCK): sub-matrices of all
// rows holding the entries of one column range each (built on first use),
// and the FP64 partial results, nblk * nrows doubles per stream.
struct ColBlockData {
    std::vector<spk_mat *> sub;
    std::map<hipStream_t, double *> part;
};

// SPK_FMT_XWIN (see kernels.h, XwinArgs): the entries regrouped by column
// window, built on first use for one window size; the wavefront tiles and
// chunks of each (entries per wavefront, chunks per compute unit); the FP64
// partials, one per (row, window) pair, per stream.
struct XwinPlan {
    uint32_t *tiles = nullptr;      // ntiles + 1
    int32_t *tile_k = nullptr;      // ntiles + 1
    int32_t *chunk_t = nullptr;     // nchunk + 1
    int32_t *chunk_w = nullptr;     // nchunk
    int32_t ntiles = 0, nchunk = 0;
    int64_t bytes = 0;
};

struct XwinData {
    int64_t wc = 0;                 // window columns
    int64_t nwin = 0, npairs = 0;
    uint16_t *ci = nullptr;         // nnz, column inside the window
    void *val = nullptr;            // nnz, window-major
    int32_t *ent = nullptr;         // npairs + 1
    int32_t *pos_ptr = nullptr;     // nrows + 1: row i's pairs are [pos_ptr[i], pos_ptr[i+1]) in window order
    uint16_t *rowpos = nullptr;     // npairs: each staged partial's place in its row block's row order
    int32_t *first = nullptr;       // nblk * nwin: first pair of each window's run in each row block
    int32_t *pre = nullptr;         // nblk * (nwin + 1): staging slot of each run
    int64_t rb = 0, nblk = 0;       // rows per block of the second pass, blocks
    std::vector<int32_t> ent_host;
    std::vector<int64_t> pair_off;  // nwin + 1: first pair of each window
    std::map<std::pair<int, int>, XwinPlan> plans;
    std::map<hipStream_t, double *> part;
    int64_t bytes = 0;
};

struct BlockData {
    uint32_t *blk = nullptr;    // nblk + 1 entries (start row | mode << 30)
    int32_t *bk = nullptr;      // nblk + 1 entries (first entry of each block)
    int32_t *bx = nullptr;      // 2 * nblk: x window of each row-stream block (made when first needed)
    uint16_t *c16 = nullptr;    // two-byte columns (nnz entries, made when first needed)
    int32_t *cbase = nullptr;   // nblk: base column of each block's two-byte columns, -1 = none
    int32_t nblk = 0;
    std::vector<uint32_t> host;
    std::vector<int32_t> host_k;
    int64_t bytes = 0;
};

// Structure found at registration (see spk_matrix_formats).
struct StructInfo {
    bool dia = false;               // at most kMaxDiag diagonals, no duplicates
    std::vector<int32_t> off;       // ascending diagonal offsets
    bool stencil = false;           // constant-coefficient grid stencil
    int dim = 0, N1 = 1, N2 = 1, N3 = 1;
    double coef[7] = {0, 0, 0, 0, 0, 0, 0};
};

struct DiaData {
    void *val = nullptr;            // T[ndiag*m], diagonal-major
    uint16_t *mask = nullptr;       // m
    int64_t bytes = 0;
};

}  // namespace spk

struct spk_mat {
    spk_handle h = nullptr;
    int64_t nrows = 0, ncols = 0, nnz = 0;
    int32_t dtype = SPK_F64;
    int32_t *rp = nullptr;
    int32_t *ci = nullptr;
    void *val = nullptr;
    std::vector<int32_t> rp_host;
    double mean_len = 0.0;
    int64_t max_len = 0;
    int64_t bytes = 0;
    std::map<int, spk::SellData> sell;                       // by slice height
    std::map<std::pair<int, int>, spk::BlockData> blocks;    // by (0, wavefront entries)
    spk::StructInfo st;
    spk::DiaData dia;                                        // built on first use
    std::map<int, spk::ColBlockData> colblk;                 // by block count, built on first use
    std::map<int, spk::XwinData> xwin;                       // by window KiB, built on first use
};

namespace spk {

struct DotScratch {
    double *partial = nullptr;
    uint32_t *ticket = nullptr;
    int64_t cap = 0;
};

// Working set of a CG solve on one stream: r, p, q and an aligned copy of
// x (vec_cap doubles each), two partial arrays (part_cap doubles each) and
// the scalars.
struct CgScratch {
    double *vec = nullptr;
    int64_t vec_cap = 0;
    double *part = nullptr;
    int64_t part_cap = 0;
    double *sc = nullptr;         // kCgScalars doubles
};

}  // namespace spk

namespace spk {

// Events used only to time work between them (the elapsed time is read
// after a stream synchronisation): created without the system-scope
// release/acquire an event record otherwise performs, so that a short
// kernel's time does not include an L2 write-back and invalidate.
inline hipError_t timing_event(hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

}  // namespace spk

struct spk_ctx {
    int device = 0;
    int num_cu = 0;
    char name[256] = {0};
    char arch[64] = {0};
    bool plain = false;
    std::string db_path;
    std::mutex mu;
    std::map<std::string, spk_variant> plans;
    // measured search points (the tuners' journal): point key -> (variant, median us)
    std::map<std::string, std::vector<std::pair<spk_variant, double>>> points;
    std::map<hipStream_t, spk::DotScratch> dot;
    double *noalloc_scratch = nullptr;   // this device's copy of spk_dot_noalloc's static scratch
    std::map<hipStream_t, spk::CgScratch> cg;
    void *flush_buf = nullptr;
    int64_t flush_bytes = 0;
    hipStream_t sub[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[4] = {nullptr, nullptr, nullptr, nullptr};
    hipStream_t work = nullptr;   // tuner / planner stream
    std::set<spk_mat *> mats;
};

namespace spk {

// Makes the handle's device current for the scope.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(spk_handle h)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != h->device) (void)hipSetDevice(h->device);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// ------------------------------------------------------------- dispatch

// Selection of the kernel entry for a variant (nullptr if not compiled).
const VecEntry *find_vec_entry(int op, int dtype, const spk_variant &v);
const SpmvEntry *find_spmv_entry(const spk_variant &v);

spk_status check_variant(int op, int dtype, const spk_variant &v);

spk_status run_waxpy(spk_handle h, int dtype, int64_t n, double alpha, const void *x, const void *y, void *w,
                     const spk_variant &v, hipStream_t s);
spk_status run_dot(spk_handle h, int dtype, int64_t n, const void *x, const void *y, double *out,
                   const spk_variant &v, hipStream_t s);

// SpMV (optionally fused) on a registered matrix or a borrowed CSR view
// (mat == nullptr; then only SCALAR/VECTOR apply).
struct SpmvProblem {
    spk_mat *mat = nullptr;
    const spk_csr *csr = nullptr;
    bool fused = false;
    double alpha = 0.0;
    const void *x = nullptr;
    void *y = nullptr;
    void *w = nullptr;
};

spk_status run_spmv(spk_handle h, const SpmvProblem &p, const spk_variant &v, hipStream_t s);
spk_status run_colblock(spk_handle h, const SpmvProblem &p, const spk_variant &v, hipStream_t s);
spk_variant colblock_inner(const spk_variant &v);

// Variant the dispatcher uses for a problem (the plan recorded for its
// class, else the default).
spk_status resolve(spk_handle h, const spk_problem &p, const spk_csr *csr, spk_variant *v);

// Variant used when the caller does not name one.
spk_variant default_variant(spk_handle h, const spk_problem &p, const spk_csr *csr);
spk_variant plain_variant(int op, int which);

// Shape-class key of a problem (plan DB key).
std::string class_key(const spk_problem &p, const spk_csr *csr);

// Structured formats (structured.cpp).  detect_structure fills A->st from
// host copies of the CSR arrays; format_applies tells whether a variant's
// format can run on A; run_structured runs a DIA or STENCIL variant.
void detect_structure(spk_mat *A, const int32_t *ci_host, const void *val_host);
bool format_applies(const spk_mat *A, int format);
const StructEntry *find_struct_entry(int format, int block, int rows, int lds);
bool struct_entry_fits(const spk_mat *A, const StructEntry &e);
spk_status run_structured(spk_handle h, const SpmvProblem &p, const spk_variant &v, hipStream_t s);
int64_t format_bytes(const spk_mat *A, int format, bool fused);

// Derived formats of a registered matrix (built on first use; synchronous).
spk_status get_sell(spk_handle h, spk_mat *A, int C, SellData **out);
spk_status get_blocks(spk_handle h, spk_mat *A, int entries, BlockData **out);
spk_status get_block_windows(spk_handle h, spk_mat *A, BlockData *bd);
spk_status get_block_c16(spk_handle h, spk_mat *A, BlockData *bd);

// SPK_FMT_XWIN: kernel entry, validity, run and release.
const XwinEntry *find_xwin_entry(int block, int window_kib, int entries);
spk_status run_xwin(spk_handle h, const SpmvProblem &p, const spk_variant &v, hipStream_t s);
void free_xwin(XwinData &d);
int64_t sell_padded_entries(const spk_mat *A, int C);

// Plan DB persistence.
void db_load(spk_handle h);
void db_append(spk_handle h, const std::string &key, const spk_variant &v, double us);
// The search journal: point_get finds a point measured before (this
// process, or a journal line of the same arch and build in the plan DB);
// point_put records one and appends its line to the DB.
bool point_get(spk_handle h, const std::string &key, const spk_variant &v, double *us);
void point_put(spk_handle h, const std::string &key, const spk_variant &v, double us);
// 64-bit FNV-1a over a byte range, chained through `seed`.
uint64_t fnv1a(const void *p, size_t n, uint64_t seed = 1469598103934665603ull);

// Algorithmic bytes of one SpMV (+ step) on a matrix.
int64_t spmv_bytes(int64_t m, int64_t n, int64_t nnz, int dtype, bool fused);

double now_seconds();

// ------------------------------------------------------- batched tiles

int batch_class(int64_t m, int64_t nnz);
bool is_stream_mode(int mode);
int batch_default_mode(int cls, int entries);
std::string batch_key(int dtype, int cls);
const BatchEntry *batch_entry(int block, int tile, int xw);

// Cuts rows [0, m) of one CSR (host row_ptr) into wavefront tiles for
// `mode` (0 = LDS row stream of at most `entries` entries and 128 rows;
// G = G lanes per row, about `target` entries per tile).  Fills r0, r1, k0,
// k1 and mode; the caller sets the matrix pointers and vector offset.
void cut_rows(const int32_t *rp, int64_t m, int mode, int entries, int64_t target, std::vector<BatchTile> &out);

// One launch of the tile kernel of launch kind `kind` (kBatchGrid, or
// kBatchPersistent with queue counters `ctr`).  With `reqs` (grid launches
// only) the ntiles launch tiles are named through the request table and
// `req_of_tile` instead of `d_tiles`.
spk_status launch_tiles(const BatchEntry *e, int dtype, const BatchTile *d_tiles, int64_t ntiles, double alpha,
                        const void *x, void *y, void *w, int kind, uint32_t *ctr, int64_t persistent_grid,
                        hipStream_t s, const BatchReq *reqs = nullptr, const uint16_t *req_of_tile = nullptr);

}  // namespace spk
