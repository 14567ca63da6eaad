/*
 * host_malloc_baseline.cpp -- a context figure, not a baseline the device
 * allocator is measured against: the host C library's malloc/free over the
 * same request streams as the device sweep (one size per round, n requests
 * allocated, then all freed), split across host threads.  The paper's
 * driver allocates, writes, checks and frees each round (Methods); only the
 * allocation and the free are timed here, as on the device.
 *
 * Host code only (C++17, std::thread); built into libhbheap.so.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <vector>

#include "hbheap.h"

namespace {

/* A reusable barrier for a fixed number of threads (generation counted). */
class Barrier {
public:
    explicit Barrier(uint32_t n) : n_(n) {}
    void arrive_and_wait()
    {
        std::unique_lock<std::mutex> lk(m_);
        const uint64_t gen = gen_;
        if (++count_ == n_) {
            count_ = 0;
            ++gen_;
            cv_.notify_all();
            return;
        }
        cv_.wait(lk, [&] { return gen_ != gen; });
    }

private:
    std::mutex m_;
    std::condition_variable cv_;
    uint32_t n_, count_ = 0;
    uint64_t gen_ = 0;
};

}  // namespace

extern "C" int hb_host_malloc_sweep(const uint64_t* sizes, uint32_t n_sizes, uint64_t requests, uint32_t iterations,
                                    uint32_t threads, double* seconds, uint64_t* failed)
{
    if (!sizes || !seconds || !failed || !n_sizes || !iterations || !threads || threads > 1024) return HBHEAP_E_INVAL;
    if (requests == 0) {
        memset(seconds, 0, sizeof(double) * n_sizes * iterations);
        *failed = 0;
        return HBHEAP_OK;
    }
    std::vector<void*> ptrs;
    try {
        ptrs.assign(requests, nullptr);
    } catch (...) {
        return HBHEAP_E_NOMEM;
    }
    std::atomic<uint64_t> nfail{0};
    Barrier bar(threads + 1);
    std::atomic<uint64_t> cur_size{0};
    std::atomic<bool> stop{false};
    std::vector<std::thread> pool;
    for (uint32_t t = 0; t < threads; ++t) {
        pool.emplace_back([&, t] {
            const uint64_t lo = requests * t / threads, hi = requests * (t + 1) / threads;
            for (;;) {
                bar.arrive_and_wait(); /* round start (or stop) */
                if (stop.load()) return;
                const size_t s = (size_t)cur_size.load();
                uint64_t bad = 0;
                for (uint64_t i = lo; i < hi; ++i) {
                    ptrs[i] = malloc(s);
                    bad += ptrs[i] == nullptr;
                }
                bar.arrive_and_wait(); /* every allocation made */
                for (uint64_t i = lo; i < hi; ++i) free(ptrs[i]);
                if (bad) nfail += bad;
                bar.arrive_and_wait(); /* every free made */
            }
        });
    }
    for (uint32_t si = 0; si < n_sizes; ++si) {
        for (uint32_t it = 0; it < iterations; ++it) {
            cur_size.store(sizes[si]);
            const auto t0 = std::chrono::steady_clock::now();
            bar.arrive_and_wait();
            bar.arrive_and_wait();
            bar.arrive_and_wait();
            const auto t1 = std::chrono::steady_clock::now();
            seconds[(uint64_t)si * iterations + it] = std::chrono::duration<double>(t1 - t0).count();
        }
    }
    stop.store(true);
    bar.arrive_and_wait();
    for (auto& th : pool) th.join();
    *failed = nfail.load();
    return HBHEAP_OK;
}
