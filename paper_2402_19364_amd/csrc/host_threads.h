// Host thread helpers of the decomposition and plan builders.
#pragma once

#include <algorithm>
#include <cstdint>
#include <thread>
#include <vector>

namespace arrow {

// Threads to use for `threads` (0 = every hardware thread, at most 256).
inline int host_threads(int threads) {
    return threads > 0 ? threads
                       : (int)std::max(1u, std::min(256u, std::thread::hardware_concurrency()));
}

// Runs fn(lo, hi, t) for t = 0 .. nt-1 over [0, count) split into contiguous
// ranges of equal size (thread t takes the t-th range), on nt threads; small
// counts run the same ranges one after the other on the calling thread.
// Every t is called (possibly with an empty range), so per-thread results
// are always written.
template <class F>
void par_for(int nt, int64_t count, F &&fn) {
    if (nt <= 1 || count < 4096) {
        for (int t = 0; t < std::max(nt, 1); ++t)
            fn(count * t / std::max(nt, 1), count * (t + 1) / std::max(nt, 1), t);
        return;
    }
    std::vector<std::thread> ts;
    ts.reserve(nt);
    for (int t = 0; t < nt; ++t) {
        const int64_t lo = count * t / nt, hi = count * (t + 1) / nt;
        ts.emplace_back([&fn, lo, hi, t] { fn(lo, hi, t); });
    }
    for (auto &th : ts) th.join();
}

// Runs fn(t) for t = 0 .. nt-1, one thread each (tasks of uneven size).
template <class F>
void par_each(int nt, F &&fn) {
    if (nt <= 1) {
        fn(0);
        return;
    }
    std::vector<std::thread> ts;
    ts.reserve(nt);
    for (int t = 0; t < nt; ++t) ts.emplace_back([&fn, t] { fn(t); });
    for (auto &th : ts) th.join();
}

// Exclusive prefix sum of per-thread counts; returns the total.
template <class V>
int64_t exclusive_scan(V &c) {
    int64_t s = 0;
    for (auto &v : c) {
        const int64_t x = v;
        v = s;
        s += x;
    }
    return s;
}

}  // namespace arrow
