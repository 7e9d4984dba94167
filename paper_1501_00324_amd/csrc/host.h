// Host-side helpers shared by the library's C++ translation units: wall
// clock, device selection guard, device allocation with accounting, and a
// small chunked thread pool.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "internal.h"

namespace fs {

inline double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(
               steady_clock::now().time_since_epoch()).count();
}

// Makes device d current for the guard's lifetime.
struct DeviceGuard {
    int prev = -1, want;
    explicit DeviceGuard(int d) : want(d)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != want)
            (void)hipSetDevice(want);
    }
    ~DeviceGuard()
    {
        if (prev >= 0 && prev != want) (void)hipSetDevice(prev);
    }
};

// hipMalloc of count elements; adds the bytes to acct.  count <= 0 leaves
// *p NULL.
template <class T>
fs_status dalloc(T **p, int64_t count, int64_t &acct)
{
    *p = nullptr;
    if (count <= 0) return FS_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p),
                             size_t(count) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(e == hipErrorOutOfMemory ? FS_E_OOM : FS_E_HIP,
                         "hipMalloc(%lld bytes): %s",
                         (long long)(count * int64_t(sizeof(T))),
                         hipGetErrorString(e));
    }
    acct += count * int64_t(sizeof(T));
    return FS_OK;
}

template <class T> void dfree(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Pinned host array (hipHostMalloc), freed on destruction or release().
template <class T> struct PinnedBuf {
    T *p = nullptr;
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf &) = delete;
    PinnedBuf &operator=(const PinnedBuf &) = delete;
    ~PinnedBuf() { release(); }
    fs_status alloc(int64_t n)
    {
        release();
        if (n <= 0) return FS_OK;
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&p),
                                     size_t(n) * sizeof(T),
                                     hipHostMallocDefault);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return set_error(FS_E_OOM, "hipHostMalloc(%lld bytes): %s",
                             (long long)(n * int64_t(sizeof(T))),
                             hipGetErrorString(e));
        }
        return FS_OK;
    }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
    }
    T *data() const { return p; }
};

// f(c) for every chunk c in [0, nchunks), spread over up to 16 host
// threads.  Chunks are independent; results must not depend on which
// thread ran which chunk.
template <class F> void parallel_chunks(int64_t nchunks, F f)
{
    const int64_t hw = std::max<int64_t>(1, std::thread::hardware_concurrency());
    const int64_t nt = std::min<int64_t>({hw, int64_t(16), nchunks});
    if (nt <= 1) {
        for (int64_t c = 0; c < nchunks; ++c) f(c);
        return;
    }
    std::atomic<int64_t> next(0);
    std::vector<std::thread> th;
    th.reserve(size_t(nt));
    for (int64_t t = 0; t < nt; ++t)
        th.emplace_back([&]() {
            for (int64_t c = next++; c < nchunks; c = next++) f(c);
        });
    for (auto &t : th) t.join();
}

}  // namespace fs
