// Host worker threads for the set-up loops of libvms (internal header).
//
// Loops split [0, n) into contiguous ranges, one per thread, in index order,
// so that per-thread results concatenated in thread order equal those of the
// serial loop. The thread count comes from VMS_HOST_THREADS, else
// OMP_NUM_THREADS, else the hardware concurrency, and is at most 64.
#pragma once
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <thread>
#include <vector>

namespace vms {

inline int host_threads() {
    static const int n = [] {
        for (const char *v : {"VMS_HOST_THREADS", "OMP_NUM_THREADS"}) {
            const char *s = std::getenv(v);
            if (s && std::atoi(s) > 0) return std::min(64, std::atoi(s));
        }
        return std::max(1, std::min(64, (int)std::thread::hardware_concurrency()));
    }();
    return n;
}

// fn(t) for t in [0, T), each on its own thread (the caller runs t = 0)
template <typename F>
void run_tasks(int T, F &&fn) {
    if (T <= 1) {
        if (T == 1) fn(0);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(T - 1);
    for (int t = 1; t < T; ++t) th.emplace_back([&fn, t] { fn(t); });
    fn(0);
    for (auto &x : th) x.join();
}

// number of ranges used for n items with at least `grain` items per range
inline int n_ranges(int64_t n, int64_t grain) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / std::max<int64_t>(grain, 1)));
}

// fn(begin, end, t) over [0, n) in T = n_ranges(n, grain) contiguous ranges
template <typename F>
int parallel_for(int64_t n, F &&fn, int64_t grain = 1 << 15) {
    const int T = n_ranges(n, grain);
    run_tasks(T, [&](int t) { fn(n * t / T, n * (t + 1) / T, t); });
    return T;
}

// sort by chunks on worker threads, then pairwise merges (same result as
// std::sort for a strict total order)
template <typename T>
void parallel_sort(std::vector<T> &v) {
    const int64_t n = (int64_t)v.size();
    const int P = n_ranges(n, 1 << 16);
    if (P <= 1) {
        std::sort(v.begin(), v.end());
        return;
    }
    std::vector<int64_t> b(P + 1);
    for (int t = 0; t <= P; ++t) b[t] = n * t / P;
    run_tasks(P, [&](int t) { std::sort(v.begin() + b[t], v.begin() + b[t + 1]); });
    std::vector<T> tmp(n);
    for (int w = 1; w < P; w *= 2) {
        const int groups = (P + 2 * w - 1) / (2 * w);
        run_tasks(groups, [&](int g) {
            const int i = g * 2 * w, j = std::min(i + w, P), k = std::min(i + 2 * w, P);
            std::merge(v.begin() + b[i], v.begin() + b[j], v.begin() + b[j], v.begin() + b[k],
                       tmp.begin() + b[i]);
        });
        v.swap(tmp);
    }
}

}  // namespace vms
