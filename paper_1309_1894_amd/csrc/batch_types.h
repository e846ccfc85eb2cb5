// batch_types.h -- plain-data descriptors of the batched tile kernel,
// shared by host planners and device code.
#pragma once

#include <stdint.h>

namespace spk {

// A tile is rows [r0, r1) (entries [k0, k1)) of one CSR matrix, processed
// with kernel `mode`: 0 = LDS-staged row stream summed one lane per row,
// 1 = the same with the tile's window of x staged in LDS too (columns
// [xlo, xlo + xn), found on the device after planning; xn = 0 when the
// window is wider than the kernel's room for it, and then x is gathered
// from memory as in mode 0), 3 = mode 1 with compact columns (once the
// window is found and fits, ci points to one byte per entry, the entry's
// column minus xlo, written by the planner; a tile whose window does not
// fit becomes a mode-5 tile when its columns span at most 65,536 -- ci
// then points to two-byte offsets from xlo and x is gathered from memory
// -- else a mode-1 tile), G in {2, 4, ..., 64} = G lanes per
// row straight from memory.  The tile carries its matrix's arrays and the
// offset of the matrix's vectors inside the launch's x / y / w, so a
// wavefront needs one 64-byte descriptor load before it can start
// streaming.
struct BatchTile {
    const int32_t *rp;
    const int32_t *ci;
    const void *val;
    int64_t vec_off;
    int32_t r0, r1, k0, k1;
    int32_t mode, xlo, xn, pad;
};

static_assert(sizeof(BatchTile) == 64, "tile descriptor is one 64-byte line");

// Serving launches: each request's matrix keeps its tiles on the device
// (vector offsets 0), and a launch over several requests names them through
// this table instead of copying tiles: launch tile t is tile
// t - first of request req_of_tile[t], its vectors at vec_off in x / y / w.
struct BatchReq {
    const BatchTile *tiles;
    int64_t vec_off;
    int32_t first, pad;
};

static_assert(sizeof(BatchReq) == 24, "request record");

}  // namespace spk
