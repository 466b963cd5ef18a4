// fsr_sched.h -- the serving path's scheduling policy, free of any device
// call: the allocator of the server's HBM budget and the choice of what each
// batched launch takes.  fsr_serve.cpp drives it with HIP streams and
// events; the tests drive it with a simulated device on a virtual clock.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace fsr {
namespace sched {

inline size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing of neighbouring holes.
class Arena {
public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
        used_ = 0;
    }
    bool alloc(size_t n, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, start = it->first + n;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used_ += n;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        used_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
    size_t used() const { return used_; }
    size_t holes() const { return free_.size(); }
    size_t largest_hole() const {
        size_t m = 0;
        for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }

private:
    std::map<size_t, size_t> free_;   // offset -> length
    size_t used_ = 0;
};

// Arena bytes of one request: image (float32), mask (uint8) and output
// (float32), each 256-byte aligned.
inline size_t request_bytes(int32_t height, int32_t width) {
    const size_t px = (size_t)height * (size_t)width;
    return align256(4 * px) + align256(px) + align256(4 * px);
}

// Work of a request in block-iterations; the 8 stand for the transforms
// and the gather around the iterations.
inline double request_work(int32_t height, int32_t width, int32_t iterations, int32_t block) {
    const double blocks = (double)((height + block - 1) / block) * (double)((width + block - 1) / block);
    return blocks * (double)(iterations + 8);
}

// A batch is started beside a running one only if it is at most this share
// of the running batch's block-iterations: a small frame then finishes long
// before the large one, while two large batches sharing the device would
// both finish late.
constexpr double kBesideShare = 0.25;

// How many admitted requests, taken from the front, the next launch takes.
// `works` lists the admitted requests' works in admission order;
// `running_work` is the largest work of the launches in flight (0 if none).
// With nothing running: up to max_batch.  Beside a running launch: the
// longest leading run (at most max_batch) whose total stays within
// kBesideShare of it, which may be none (then wait).
template <typename WorkAt>
size_t batch_size(size_t n_admitted, WorkAt work_at, size_t max_batch, double running_work) {
    const size_t n = n_admitted < max_batch ? n_admitted : max_batch;
    if (running_work <= 0.0) return n;
    double w = 0.0;
    size_t k = 0;
    for (; k < n; ++k) {
        const double wk = work_at(k);
        if (w + wk > kBesideShare * running_work) break;
        w += wk;
    }
    return k;
}

}  // namespace sched
}  // namespace fsr
