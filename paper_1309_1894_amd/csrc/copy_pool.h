// copy_pool.h -- host copies shared by a few persistent threads (used by the
// serving loop; plain C++, no HIP).
#pragma once

#include <algorithm>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

namespace spk {

// Host copies between the callers' buffers and the pinned staging blocks
// are the scheduler's largest cost per request (about two thirds of its
// busy time at saturation, memcpy on one core).  A few persistent threads
// share them: a batch of copies is cut into chunks of at least kCopyChunk
// bytes, the scheduler thread takes chunks too, and returns when all are
// done.  Batches below kCopyInline bytes are copied inline.
struct CopyPool {
    static constexpr size_t kCopyChunk = 256 << 10;
    static constexpr size_t kCopyInline = 512 << 10;
    struct Chunk {
        void *dst;
        const void *src;
        size_t n;
    };
    std::vector<std::thread> thr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<Chunk> chunks;
    size_t next = 0, done = 0;
    uint64_t gen = 0;
    bool stop = false;

    void start(int workers)
    {
        for (int i = 0; i < workers; ++i) thr.emplace_back([this] { loop(); });
    }
    void finish()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_work.notify_all();
        for (auto &t : thr) t.join();
        thr.clear();
    }
    // takes chunks until none is left; returns how many it copied
    size_t take(std::unique_lock<std::mutex> &lk)
    {
        size_t mine = 0;
        while (next < chunks.size()) {
            const Chunk c = chunks[next++];
            lk.unlock();
            memcpy(c.dst, c.src, c.n);
            lk.lock();
            ++mine;
            if (++done == chunks.size()) cv_done.notify_all();
        }
        return mine;
    }
    void loop()
    {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_work.wait(lk, [&] { return stop || gen != seen; });
            if (stop) return;
            seen = gen;
            take(lk);
        }
    }
    // copies every (dst, src, n); returns when all are done
    void copy(const std::vector<Chunk> &items)
    {
        size_t total = 0;
        for (const Chunk &c : items) total += c.n;
        if (thr.empty() || total < kCopyInline) {
            for (const Chunk &c : items)
                if (c.n) memcpy(c.dst, c.src, c.n);
            return;
        }
        std::unique_lock<std::mutex> lk(mu);
        chunks.clear();
        for (const Chunk &c : items)
            for (size_t o = 0; o < c.n; o += kCopyChunk)
                chunks.push_back({(char *)c.dst + o, (const char *)c.src + o, std::min(kCopyChunk, c.n - o)});
        next = done = 0;
        ++gen;
        cv_work.notify_all();
        take(lk);
        cv_done.wait(lk, [&] { return done == chunks.size(); });
    }
};

}  // namespace spk
