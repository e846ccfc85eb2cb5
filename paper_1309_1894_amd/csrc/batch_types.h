// batch_types.h -- plain-data descriptors of the batched tile kernel,
// shared by host planners and device code.
#pragma once

#include <stdint.h>

namespace spk {

// One instance: its own CSR arrays, and the offset of its vectors inside
// the launch's x / y / w.
struct BatchInst {
    const int32_t *rp;
    const int32_t *ci;
    const void *val;
    int64_t vec_off;
    int32_t m, pad;
};

// A tile is rows [r0, r1) of one instance processed with kernel `mode`:
// 0 = LDS-staged row stream, G in {2..64} = G lanes per row.
struct BatchTile {
    int32_t inst, r0, r1, mode;
};

}  // namespace spk
