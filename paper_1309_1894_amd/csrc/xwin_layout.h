// xwin_layout.h -- host construction of the x-window form (SPK_FMT_XWIN):
// the regrouping of CSR entries into (row, column window) pairs and the
// wavefront tiles and workgroup chunks over them.  Plain C++ (no GPU
// headers), so the layout can be checked on the CPU.
#pragma once

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "row_tiles.h"

namespace spk {

// Second pass of the x-window form: rows are taken in blocks of rb rows
// (one workgroup each).  A block's pairs lie, window by window, in runs of
// consecutive pairs (a window's pairs are in row order), so the workgroup
// copies those runs -- window order, each run in pair order -- into an LDS
// staging area of at most kXwinStage partials, then each row adds its own
// staged partials in window order.  rb is the largest power of two up to
// kXwinMaxRb whose blocks all fit the staging area: the larger the block,
// the longer its runs, and the fewer 128-byte lines two blocks share.
constexpr int64_t kXwinStage = 7168;      // FP64 partials staged per block (56 KiB of LDS)
constexpr int64_t kXwinMaxRb = 1024;      // rows per block at most (one per thread of the adding pass)
constexpr int64_t kXwinMaxWin = 1023;     // windows one matrix may have
constexpr int64_t kXwinMaxTable = (int64_t)1 << 26;   // block table entries

enum XwinLayoutStatus { kXwinOk = 0, kXwinTooManyPairs, kXwinTooManyWindows, kXwinTableTooLarge };

struct XwinHost {
    int64_t wc = 0;                   // columns per window
    int64_t nwin = 0, npairs = 0;
    std::vector<uint16_t> ci;         // nnz: column inside the window
    std::vector<char> val;            // nnz values (vs bytes each), window-major
    std::vector<int32_t> ent;         // npairs + 1: first entry of each pair
    std::vector<int32_t> pos_ptr;     // m + 1
    std::vector<int32_t> pos;         // npairs: each row's pairs in window order
    std::vector<int64_t> pair_off;    // nwin + 1: first pair of each window
    // second pass
    int64_t rb = 0, nblk = 0;         // rows per block, blocks
    std::vector<int32_t> first;       // nblk * nwin: first pair of window w in block b (at [b*nwin + w])
    std::vector<int32_t> pre;         // nblk * (nwin + 1): staging offset of window w's run in block b
    std::vector<uint16_t> lpos;       // npairs, aligned with pos: the pair's staging slot in its row's block
    std::vector<uint16_t> rowpos;     // npairs, block by block in staging order: the slot's place in its
                                      // block's row-ordered pair list (the inverse of lpos)
};

// Regroups the entries of an m x n CSR matrix (values of vs bytes) by
// windows of wc columns (wc <= 65536): pairs window-major, within a window
// in row order; a pair's entries keep their order in the row.  Then the
// row blocks of the second pass and their staging tables.
inline XwinLayoutStatus xwin_layout(int64_t m, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                                    const void *val, size_t vs, int64_t wc, XwinHost &d)
{
    d = XwinHost();
    d.wc = wc;
    d.nwin = n > 0 ? (n + wc - 1) / wc : 0;
    const char *vb = (const char *)val;
    std::vector<int64_t> npair((size_t)d.nwin, 0), nent((size_t)d.nwin, 0), mark((size_t)d.nwin, -1);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t w = ci[k] / wc;
            ++nent[w];
            if (mark[w] != i) {
                mark[w] = i;
                ++npair[w];
            }
        }
    d.pair_off.assign((size_t)d.nwin + 1, 0);
    std::vector<int64_t> ent_off((size_t)d.nwin + 1, 0);
    for (int64_t w = 0; w < d.nwin; ++w) {
        d.pair_off[w + 1] = d.pair_off[w] + npair[w];
        ent_off[w + 1] = ent_off[w] + nent[w];
    }
    d.npairs = d.pair_off[d.nwin];
    if (d.npairs >= (int64_t)kBlkRowMask) return kXwinTooManyPairs;
    if (d.nwin > kXwinMaxWin) return kXwinTooManyWindows;
    d.ci.assign((size_t)nnz, 0);
    d.val.assign((size_t)nnz * vs, 0);
    d.ent.assign((size_t)d.npairs + 1, 0);
    d.pos_ptr.assign((size_t)m + 1, 0);
    d.pos.clear();
    d.pos.reserve((size_t)d.npairs);
    std::vector<int64_t> cur_pair(d.pair_off.begin(), d.pair_off.begin() + d.nwin);
    std::vector<int64_t> cur_ent(ent_off.begin(), ent_off.begin() + d.nwin);
    std::vector<int64_t> pair_of((size_t)d.nwin, -1), touched;
    std::fill(mark.begin(), mark.end(), -1);
    for (int64_t i = 0; i < m; ++i) {
        touched.clear();
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t w = ci[k] / wc;
            if (mark[w] != i) {
                mark[w] = i;
                const int64_t p = cur_pair[w]++;
                pair_of[w] = p;
                d.ent[p] = (int32_t)cur_ent[w];
                touched.push_back(w);
            }
            const int64_t e = cur_ent[w]++;
            d.ci[e] = (uint16_t)(ci[k] - w * wc);
            memcpy(&d.val[(size_t)e * vs], vb + (size_t)k * vs, vs);
        }
        std::sort(touched.begin(), touched.end());
        for (int64_t w : touched) d.pos.push_back((int32_t)pair_of[w]);
        d.pos_ptr[i + 1] = (int32_t)d.pos.size();
    }
    d.ent[d.npairs] = (int32_t)nnz;
    // row blocks of the second pass
    d.rb = kXwinMaxRb;
    for (;;) {
        int64_t worst = 0;
        for (int64_t r0 = 0; r0 < m; r0 += d.rb)
            worst = std::max<int64_t>(worst, d.pos_ptr[std::min(m, r0 + d.rb)] - d.pos_ptr[r0]);
        if (worst <= kXwinStage || d.rb == 1) break;
        d.rb /= 2;
    }
    d.nblk = (m + d.rb - 1) / d.rb;
    if (d.nblk * (2 * d.nwin + 1) > kXwinMaxTable) return kXwinTableTooLarge;
    d.first.assign((size_t)(d.nblk * d.nwin), 0);
    d.pre.assign((size_t)(d.nblk * (d.nwin + 1)), 0);
    d.lpos.assign((size_t)d.npairs, 0);
    d.rowpos.assign((size_t)d.npairs, 0);
    std::vector<int64_t> win_of((size_t)d.npairs);
    for (int64_t w = 0; w < d.nwin; ++w)
        for (int64_t p = d.pair_off[w]; p < d.pair_off[w + 1]; ++p) win_of[p] = w;
    std::vector<int64_t> seen(d.pair_off.begin(), d.pair_off.begin() + d.nwin);   // pairs of earlier blocks
    std::vector<int64_t> cnt((size_t)d.nwin);
    for (int64_t b = 0; b < d.nblk; ++b) {
        const int64_t r0 = b * d.rb, r1 = std::min(m, r0 + d.rb);
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int64_t k = d.pos_ptr[r0]; k < d.pos_ptr[r1]; ++k) ++cnt[win_of[d.pos[k]]];
        int32_t *pre = d.pre.data() + b * (d.nwin + 1);
        int32_t *first = d.first.data() + b * d.nwin;
        for (int64_t w = 0; w < d.nwin; ++w) {
            first[w] = (int32_t)seen[w];
            pre[w + 1] = pre[w] + (int32_t)cnt[w];
            seen[w] += cnt[w];
        }
        for (int64_t k = d.pos_ptr[r0]; k < d.pos_ptr[r1]; ++k) {
            const int64_t p = d.pos[k], w = win_of[p];
            d.lpos[k] = (uint16_t)(pre[w] + (p - first[w]));
            d.rowpos[(size_t)(d.pos_ptr[r0] + d.lpos[k])] = (uint16_t)(k - d.pos_ptr[r0]);
        }
    }
    return kXwinOk;
}

// Wavefront tiles of each window (E = row-stream capacity; a tile never
// crosses a window), recorded as start pair | mode << 30 and first entry,
// closed by (npairs, nnz); and the workgroup chunks: `target` chunks shared
// out over the windows that hold pairs by work (entries plus two per pair;
// largest remainders, at least one each, at most one per tile), each
// window's tiles cut into its chunks by work.  chunk_t has nchunk + 1
// entries (tile boundaries), chunk_w the window of each chunk.
inline void xwin_plan(const XwinHost &d, int E, int64_t target, std::vector<uint32_t> &tiles,
                      std::vector<int32_t> &tile_k, std::vector<int32_t> &chunk_t, std::vector<int32_t> &chunk_w)
{
    tiles.clear();
    tile_k.clear();
    chunk_t.clear();
    chunk_w.clear();
    std::vector<uint32_t> wt;
    std::vector<int32_t> wk;
    std::vector<int64_t> win_t0((size_t)d.nwin + 1, 0);
    for (int64_t w = 0; w < d.nwin; ++w) {
        win_t0[w] = (int64_t)tiles.size();
        const int64_t p0 = d.pair_off[w], np = d.pair_off[w + 1] - p0;
        if (np == 0) continue;
        make_blocks(d.ent.data() + p0, np, E, wt, wk);
        for (size_t t = 0; t + 1 < wt.size(); ++t) {
            tiles.push_back((uint32_t)(((int64_t)(wt[t] & kBlkRowMask) + p0) | (wt[t] & ~kBlkRowMask)));
            tile_k.push_back(wk[t]);
        }
    }
    win_t0[d.nwin] = (int64_t)tiles.size();
    tiles.push_back((uint32_t)d.npairs);
    tile_k.push_back(d.ent[d.npairs]);
    const int64_t ntiles = (int64_t)tiles.size() - 1;
    auto work = [&](int64_t t) -> double {
        const int64_t np = (int64_t)(tiles[t + 1] & kBlkRowMask) - (int64_t)(tiles[t] & kBlkRowMask);
        return (double)(tile_k[t + 1] - tile_k[t]) + 2.0 * (double)np;
    };
    std::vector<double> wwork((size_t)d.nwin, 0.0);
    double total = 0.0;
    int64_t busy = 0;
    for (int64_t w = 0; w < d.nwin; ++w) {
        for (int64_t t = win_t0[w]; t < win_t0[w + 1]; ++t) wwork[w] += work(t);
        total += wwork[w];
        busy += win_t0[w + 1] > win_t0[w];
    }
    std::vector<int64_t> nch((size_t)d.nwin, 0);
    if (busy > 0) {
        const int64_t G = std::max<int64_t>(target, busy);
        std::vector<std::pair<double, int64_t>> rem;
        int64_t given = 0;
        for (int64_t w = 0; w < d.nwin; ++w) {
            if (win_t0[w + 1] == win_t0[w]) continue;
            const double q = total > 0 ? (double)G * wwork[w] / total : 1.0;
            nch[w] = std::max<int64_t>(1, (int64_t)std::floor(q));
            given += nch[w];
            rem.push_back({q - std::floor(q), w});
        }
        std::sort(rem.begin(), rem.end(), [](const std::pair<double, int64_t> &a, const std::pair<double, int64_t> &b) {
            return a.first != b.first ? a.first > b.first : a.second < b.second;
        });
        for (size_t r = 0; given < G && r < rem.size(); ++r, ++given) ++nch[rem[r].second];
        for (int64_t w = 0; w < d.nwin; ++w) nch[w] = std::min<int64_t>(nch[w], win_t0[w + 1] - win_t0[w]);
    }
    for (int64_t w = 0; w < d.nwin; ++w) {
        if (nch[w] == 0) continue;
        const int64_t t0 = win_t0[w], t1 = win_t0[w + 1];
        double acc = 0.0;
        int64_t c = 0;
        chunk_t.push_back((int32_t)t0);
        chunk_w.push_back((int32_t)w);
        for (int64_t t = t0; t < t1; ++t) {
            acc += work(t);
            // close chunk c at its share of the work, keeping a tile for every later chunk
            if (c + 1 < nch[w] && acc >= wwork[w] * (double)(c + 1) / (double)nch[w] && t1 - (t + 1) >= nch[w] - (c + 1)) {
                chunk_t.push_back((int32_t)(t + 1));
                chunk_w.push_back((int32_t)w);
                ++c;
            }
        }
    }
    chunk_t.push_back((int32_t)ntiles);
}

}  // namespace spk
