// CPU check of the x-window layout and plan (no GPU): random CSR matrices
// with the structural edge cases are regrouped and planned, every invariant
// the kernels rely on is checked (index ranges, tile limits, each pair in
// exactly one tile of exactly one chunk of its own window), and the two
// passes are replayed on the host from the layout alone and compared with a
// direct CSR product.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <cstdint>
#include <random>
#include <vector>

#include "xwin_layout.h"

using namespace spk;

static int failures = 0;
#define CHECK(c, ...)                                            \
    do {                                                         \
        if (!(c)) {                                              \
            ++failures;                                          \
            printf("FAIL %s:%d: %s: ", __FILE__, __LINE__, #c);  \
            printf(__VA_ARGS__);                                 \
            printf("\n");                                        \
            return;                                              \
        }                                                        \
    } while (0)

struct Csr {
    int64_t m = 0, n = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> val;
};

static void check_one(const Csr &A, int64_t wc, int E, int64_t target, const char *name)
{
    const int64_t m = A.m, n = A.n, nnz = (int64_t)A.ci.size();
    XwinHost d;
    CHECK(xwin_layout(m, n, nnz, A.rp.data(), A.ci.data(), A.val.data(), 8, wc, d) == kXwinOk, "%s", name);
    CHECK(d.nwin == (n > 0 ? (n + wc - 1) / wc : 0), "%s nwin", name);
    CHECK((int64_t)d.pair_off.size() == d.nwin + 1 && d.pair_off[0] == 0 && d.pair_off[d.nwin] == d.npairs, "%s", name);
    CHECK((int64_t)d.ent.size() == d.npairs + 1 && d.ent[d.npairs] == nnz, "%s ent end", name);
    for (int64_t p = 0; p < d.npairs; ++p) CHECK(d.ent[p] < d.ent[p + 1], "%s pair %lld empty", name, (long long)p);
    std::vector<int64_t> win_of((size_t)d.npairs, -1);
    for (int64_t w = 0; w < d.nwin; ++w) {
        CHECK(d.pair_off[w] <= d.pair_off[w + 1], "%s", name);
        for (int64_t p = d.pair_off[w]; p < d.pair_off[w + 1]; ++p) {
            win_of[p] = w;
            for (int32_t k = d.ent[p]; k < d.ent[p + 1]; ++k)
                CHECK(d.ci[k] < wc && w * wc + d.ci[k] < n, "%s column %d in window %lld", name, d.ci[k], (long long)w);
        }
    }
    // each row's pairs: windows ascending, together exactly the row's entries (as a multiset, in row order per pair)
    CHECK((int64_t)d.pos_ptr.size() == m + 1 && d.pos_ptr[0] == 0 && d.pos_ptr[m] == d.npairs, "%s pos_ptr", name);
    std::vector<int> used((size_t)d.npairs, 0);
    std::vector<int64_t> pair_in_win((size_t)std::max<int64_t>(1, d.nwin), -1), cursor((size_t)d.npairs, 0);
    for (int64_t i = 0; i < m; ++i) {
        int64_t prev_w = -1, cnt = 0;
        for (int32_t q = d.pos_ptr[i]; q < d.pos_ptr[i + 1]; ++q) {
            const int32_t p = d.pos[q];
            CHECK(p >= 0 && p < d.npairs && !used[p], "%s pos", name);
            used[p] = 1;
            CHECK(win_of[p] > prev_w, "%s row %lld windows not ascending", name, (long long)i);
            prev_w = win_of[p];
            pair_in_win[win_of[p]] = p;
            cursor[p] = d.ent[p];
            cnt += d.ent[p + 1] - d.ent[p];
        }
        CHECK(cnt == A.rp[i + 1] - A.rp[i], "%s row %lld entry count", name, (long long)i);
        // the pair of each window holds the row's entries of that window, in row order
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int64_t w = A.ci[k] / wc;
            const int64_t p = pair_in_win[w];
            CHECK(p >= 0 && win_of[p] == w && cursor[p] < d.ent[p + 1], "%s row %lld: no pair for window", name,
                  (long long)i);
            const int64_t k2 = cursor[p]++;
            CHECK(w * wc + d.ci[k2] == A.ci[k], "%s row %lld entry order", name, (long long)i);
            double v;
            memcpy(&v, &d.val[(size_t)k2 * 8], 8);
            CHECK(v == A.val[k], "%s value", name);
        }
        for (int32_t q = d.pos_ptr[i]; q < d.pos_ptr[i + 1]; ++q) {
            CHECK(cursor[d.pos[q]] == d.ent[d.pos[q] + 1], "%s row %lld pair length", name, (long long)i);
            pair_in_win[win_of[d.pos[q]]] = -1;
        }
    }
    // plan
    std::vector<uint32_t> tiles;
    std::vector<int32_t> tile_k, chunk_t, chunk_w;
    xwin_plan(d, E, target, tiles, tile_k, chunk_t, chunk_w);
    const int64_t ntiles = (int64_t)tiles.size() - 1, nchunk = (int64_t)chunk_w.size();
    CHECK(ntiles >= 0 && (int64_t)tile_k.size() == ntiles + 1 && (int64_t)chunk_t.size() == nchunk + 1, "%s", name);
    CHECK((tiles[ntiles] & kBlkRowMask) == (uint32_t)d.npairs && tile_k[ntiles] == nnz, "%s closing tile", name);
    CHECK(chunk_t[0] == 0 && chunk_t[nchunk] == ntiles, "%s chunk cover", name);
    if (d.npairs > 0) CHECK(nchunk >= 1 && nchunk <= std::max<int64_t>(target, d.nwin), "%s chunk count %lld", name, (long long)nchunk);
    std::vector<double> part((size_t)d.npairs, NAN);
    std::vector<int> done((size_t)d.npairs, 0);
    for (int64_t c = 0; c < nchunk; ++c) {
        CHECK(chunk_t[c] < chunk_t[c + 1], "%s chunk %lld empty", name, (long long)c);
        const int64_t w = chunk_w[c];
        CHECK(w >= 0 && w < d.nwin, "%s chunk window", name);
        for (int64_t t = chunk_t[c]; t < chunk_t[c + 1]; ++t) {
            const int64_t p0 = tiles[t] & kBlkRowMask, p1 = tiles[t + 1] & kBlkRowMask;
            const uint32_t mode = tiles[t] >> 30;
            CHECK(p0 < p1 && p1 <= d.npairs, "%s tile %lld pairs", name, (long long)t);
            CHECK(tile_k[t] == d.ent[p0] && tile_k[t + 1] == d.ent[p1], "%s tile %lld entries", name, (long long)t);
            for (int64_t p = p0; p < p1; ++p) CHECK(win_of[p] == w, "%s tile %lld crosses windows", name, (long long)t);
            if (mode == kBlkStream) {
                CHECK(p1 - p0 <= 128 && tile_k[t + 1] - tile_k[t] <= E, "%s stream tile %lld too big", name, (long long)t);
            } else {
                CHECK(mode == kBlkWave || mode == kBlkLong, "%s mode", name);
            }
            for (int64_t p = p0; p < p1; ++p) {
                CHECK(!done[p], "%s pair twice", name);
                done[p] = 1;
                double s = 0.0;
                for (int32_t k = d.ent[p]; k < d.ent[p + 1]; ++k) {
                    double v;
                    memcpy(&v, &d.val[(size_t)k * 8], 8);
                    s += v * (double)(w * wc + d.ci[k]) * 1e-6;   // x_j = j * 1e-6
                }
                part[p] = s;
            }
        }
    }
    for (int64_t p = 0; p < d.npairs; ++p) CHECK(done[p], "%s pair %lld in no tile", name, (long long)p);
    // second pass as the kernel runs it: stage each block's runs, then each row sums its slots
    CHECK(d.rb >= 1 && d.rb <= kXwinMaxRb && (d.rb & (d.rb - 1)) == 0 && d.nblk == (m + d.rb - 1) / d.rb, "%s rb", name);
    CHECK((int64_t)d.first.size() == d.nblk * d.nwin && (int64_t)d.pre.size() == d.nblk * (d.nwin + 1) &&
          (int64_t)d.lpos.size() == d.npairs, "%s table sizes", name);
    std::vector<double> y((size_t)m, 0.0);
    for (int64_t b = 0; b < d.nblk; ++b) {
        const int32_t *pre = d.pre.data() + b * (d.nwin + 1);
        const int32_t *first = d.first.data() + b * d.nwin;
        const int64_t total = pre[d.nwin];
        CHECK(pre[0] == 0 && total <= kXwinStage, "%s block %lld staging %lld", name, (long long)b, (long long)total);
        std::vector<double> stage((size_t)total, NAN);
        std::vector<int64_t> wof((size_t)total, -1);
        for (int64_t w = 0; w < d.nwin; ++w)
            for (int64_t j = pre[w]; j < pre[w + 1]; ++j) wof[j] = w;
        for (int64_t j = 0; j < total; ++j) {
            const int64_t w = wof[j];
            CHECK(w >= 0, "%s block %lld slot %lld has no window", name, (long long)b, (long long)j);
            const int64_t p = first[w] + (j - pre[w]);
            CHECK(p >= 0 && p < d.npairs && win_of[p] == w, "%s block %lld slot %lld", name, (long long)b, (long long)j);
            stage[j] = part[p];
        }
        const int64_t r0 = b * d.rb, r1 = std::min(m, r0 + d.rb);
        CHECK(total == d.pos_ptr[r1] - d.pos_ptr[r0], "%s block %lld pair count", name, (long long)b);
        // slots placed in row order, as the kernel places them
        std::vector<double> rowv((size_t)total, NAN);
        std::vector<int> placed((size_t)total, 0);
        for (int64_t j = 0; j < total; ++j) {
            const int64_t q = d.rowpos[(size_t)(d.pos_ptr[r0] + j)];
            CHECK(q < total && !placed[q], "%s block %lld rowpos", name, (long long)b);
            placed[q] = 1;
            rowv[q] = stage[j];
        }
        for (int64_t i = r0; i < r1; ++i)
            for (int32_t q = d.pos_ptr[i]; q < d.pos_ptr[i + 1]; ++q) {
                CHECK(d.lpos[q] < total && stage[d.lpos[q]] == part[d.pos[q]], "%s row %lld slot", name, (long long)i);
                CHECK(rowv[q - d.pos_ptr[r0]] == part[d.pos[q]], "%s row %lld row order", name, (long long)i);
                y[i] += rowv[q - d.pos_ptr[r0]];
            }
    }
    for (int64_t i = 0; i < m; ++i) {
        double ref = 0.0, absum = 0.0;
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            ref += A.val[k] * (double)A.ci[k] * 1e-6;
            absum += std::fabs(A.val[k] * (double)A.ci[k] * 1e-6);
        }
        CHECK(std::fabs(y[i] - ref) <= 1e-12 * absum, "%s row %lld: %g vs %g", name, (long long)i, y[i], ref);
    }
}

static Csr random_csr(std::mt19937_64 &g, int64_t m, int64_t n, int64_t maxlen, bool dups, double p_long)
{
    Csr A;
    A.m = m;
    A.n = n;
    A.rp.push_back(0);
    std::uniform_real_distribution<double> u(-1, 1);
    for (int64_t i = 0; i < m; ++i) {
        int64_t len = n > 0 ? (int64_t)(g() % (uint64_t)(maxlen + 1)) : 0;
        if (n > 0 && u(g) < 2 * p_long - 1) len = std::min<int64_t>(n, 20000 + (int64_t)(g() % 30000));
        for (int64_t k = 0; k < len; ++k) {
            int32_t c = (int32_t)(g() % (uint64_t)n);
            if (dups && k > 0 && (g() % 5) == 0) c = A.ci.back();
            A.ci.push_back(c);
            A.val.push_back(u(g));
        }
        A.rp.push_back((int32_t)A.ci.size());
    }
    return A;
}

int main()
{
    std::mt19937_64 g(12345);
    // structural edge cases
    check_one(Csr{0, 5, {0}, {}, {}}, 16384, 256, 256, "m0");
    check_one(Csr{6, 0, {0, 0, 0, 0, 0, 0, 0}, {}, {}}, 16384, 256, 256, "n0");
    check_one(Csr{4, 4, {0, 0, 0, 0, 0}, {}, {}}, 8192, 256, 64, "all_empty");
    check_one(Csr{1, 1, {0, 1}, {0}, {2.5}}, 16384, 256, 256, "1x1");
    // long pairs, many windows, duplicates and unsorted columns, narrow windows
    for (int rep = 0; rep < 4; ++rep) {
        const int64_t m = 1 + (int64_t)(g() % 2000), n = 1 + (int64_t)(g() % 150000);
        Csr A = random_csr(g, m, n, 1 + (int64_t)(g() % 200), rep % 2 == 1, rep == 3 ? 0.501 : 0.0);
        for (int64_t wc : {8192, 16384, 32768})
            for (int E : {128, 256})
                for (int64_t target : {1, 7, 512}) {
                    char name[96];
                    snprintf(name, sizeof name, "rand rep %d m %lld n %lld wc %lld E %d target %lld", rep, (long long)m,
                             (long long)n, (long long)wc, E, (long long)target);
                    check_one(A, wc, E, target, name);
                    if (failures) return 1;
                }
    }
    // a dense row across every window, and columns only at both ends
    {
        Csr A;
        A.m = 3;
        A.n = 100000;
        A.rp = {0};
        for (int32_t c = 0; c < 100000; ++c) A.ci.push_back(c), A.val.push_back(1e-3 * (c % 97));
        A.rp.push_back((int32_t)A.ci.size());
        A.rp.push_back((int32_t)A.ci.size());
        A.ci.push_back(5), A.val.push_back(1.0);
        A.ci.push_back(99999), A.val.push_back(-1.0);
        A.rp.push_back((int32_t)A.ci.size());
        for (int E : {128, 256}) check_one(A, 16384, E, 256, "dense_row");
    }
    if (failures) return 1;
    printf("ok\n");
    return 0;
}
