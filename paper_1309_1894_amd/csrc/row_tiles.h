// row_tiles.h -- wavefront tiles over the rows of a CSR matrix (host
// planning, shared by the LDS-staged row-block kernel and the x-window
// form; plain C++, no GPU headers).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace spk {

// A tile is recorded as its start row | mode << 30 and its first entry.
constexpr uint32_t kBlkRowMask = 0x3FFFFFFFu;
constexpr uint32_t kBlkStream = 0u;     // short rows streamed through the wavefront's LDS slice
constexpr int kStreamRowsPerThread = 2; // a workgroup row stream holds at most 2*BS rows
constexpr uint32_t kBlkWave = 1u;       // medium rows, one after another, 64 lanes per row
constexpr uint32_t kBlkLong = 2u;       // one long row, 64 lanes

// Wavefront tiles for the LDS-staged kernels, E = row-stream capacity:
// runs of short rows (at most 96 entries each) whose entries fit E and that
// number at most 128; runs of medium rows, up to 4E entries in all, one
// wavefront with 64 lanes per row; single long rows (over 8E entries).
inline void make_blocks(const int32_t *rp, int64_t m, int E, std::vector<uint32_t> &out, std::vector<int32_t> &out_k)
{
    const int64_t kShort = std::min<int64_t>(96, E);
    const int64_t kLong = 8 * (int64_t)E;
    const int64_t kRows = 2 * 64;
    out.clear();
    out_k.clear();
    int64_t r = 0;
    while (r < m) {
        const int64_t len = rp[r + 1] - rp[r];
        out_k.push_back(rp[r]);
        if (len > kLong) {
            out.push_back((uint32_t)r | (kBlkLong << 30));
            ++r;
        } else if (len > kShort) {
            out.push_back((uint32_t)r | (kBlkWave << 30));
            int64_t nz = 0;
            while (r < m) {
                const int64_t l = rp[r + 1] - rp[r];
                if (l <= kShort || l > kLong || (nz > 0 && nz + l > 4 * (int64_t)E)) break;
                nz += l;
                ++r;
            }
        } else {
            out.push_back((uint32_t)r | (kBlkStream << 30));
            int64_t nz = 0, c = 0;
            while (r < m && c < kRows) {
                const int64_t l = rp[r + 1] - rp[r];
                if (l > kShort || nz + l > E) break;
                nz += l;
                ++r;
                ++c;
            }
        }
    }
    out.push_back((uint32_t)m);
    out_k.push_back(rp[m]);
}

}  // namespace spk
