// Drives the serving path's scheduling policy (fsr_sched.h, the code the
// server runs) with a simulated device on a virtual clock: requests arrive,
// are admitted in FIFO order while the in-flight limit and the HBM arena
// allow, are batched onto free streams by the same rule as the server, and
// finish after a time proportional to the work of their launch.  Checks the
// invariants the server relies on and prints "ok" (test infrastructure;
// built and run by tests/test_sched.py on the CPU).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <vector>

#include "fsr_sched.h"

using namespace fsr::sched;

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::printf("FAILED: %s (line %d)\n", #cond, __LINE__);              \
            std::exit(1);                                                        \
        }                                                                        \
    } while (0)

namespace {

struct Req {
    int h, w, iters;
    double arrive, admit = -1, launch = -1, done = -1;
    size_t off = 0, bytes = 0;
};

struct Launch {
    int stream;
    double end, work;
    std::vector<int> ids;
};

struct Config {
    size_t budget;
    int max_inflight, max_batch, streams;
    bool one_per_launch;      // the FIFO reference mode: one request per launch, one stream
    double sec_per_work;      // simulated device speed
    double beside_slowdown;   // a launch beside another runs this much slower
};

struct Result {
    std::vector<Req> reqs;
    size_t peak_bytes = 0;
    int launches = 0, beside_launches = 0;
};

uint32_t rng_state = 1;
uint32_t rnd() {
    rng_state = rng_state * 1664525u + 1013904223u;
    return rng_state >> 8;
}

std::vector<Req> trace(int n, double rate_hz, uint32_t seed) {
    static const int sizes[][2] = {{480, 640}, {600, 800}, {1080, 1920}, {64, 64}, {150, 200}};
    rng_state = seed;
    std::vector<Req> r;
    double t = 0.0;
    for (int i = 0; i < n; ++i) {
        t += -std::log(1.0 - (rnd() % 1000000) / 1000000.0) / rate_hz;   // Poisson arrivals
        const int k = (int)(rnd() % 5);
        r.push_back(Req{sizes[k][0], sizes[k][1], 100, t});
    }
    return r;
}

Result simulate(std::vector<Req> reqs, const Config& c) {
    Result res;
    Arena arena;
    arena.init(c.budget);
    std::deque<int> queue, admitted;
    std::vector<Launch> inflight;
    std::vector<bool> busy(c.streams, false);
    size_t next_arrival = 0, completed = 0, n_admitted = 0;
    std::vector<int> admit_order;
    double now = 0.0;
    const int B = 4;
    while (completed < reqs.size()) {
        // next event: an arrival or a completion
        double t_next = 1e300;
        if (next_arrival < reqs.size()) t_next = reqs[next_arrival].arrive;
        for (const Launch& l : inflight) t_next = std::min(t_next, l.end);
        CHECK(t_next < 1e300);
        now = t_next;
        while (next_arrival < reqs.size() && reqs[next_arrival].arrive <= now) {
            Req& q = reqs[next_arrival];
            q.bytes = request_bytes(q.h, q.w);
            CHECK(q.bytes <= c.budget);   // the server refuses larger frames at submission
            queue.push_back((int)next_arrival++);
        }
        for (size_t i = 0; i < inflight.size();) {
            if (inflight[i].end > now) {
                ++i;
                continue;
            }
            for (int id : inflight[i].ids) {
                reqs[id].done = now;
                arena.release(reqs[id].off, reqs[id].bytes);   // output fetched at once
                ++completed;
            }
            busy[inflight[i].stream] = false;
            inflight.erase(inflight.begin() + (long)i);
        }
        // admission: FIFO, head of line waits for the in-flight limit or space
        while (!queue.empty()) {
            if ((int)(n_admitted - completed) >= c.max_inflight) break;
            Req& q = reqs[queue.front()];
            size_t off = 0;
            if (!arena.alloc(q.bytes, &off)) break;
            CHECK(off + q.bytes <= c.budget);
            q.off = off;
            q.admit = now;
            admit_order.push_back(queue.front());
            admitted.push_back(queue.front());
            queue.pop_front();
            ++n_admitted;
            res.peak_bytes = std::max(res.peak_bytes, arena.used());
            CHECK(arena.used() <= c.budget);
        }
        // launches
        for (;;) {
            if (admitted.empty()) break;
            int si = -1;
            for (int i = 0; i < c.streams; ++i)
                if (!busy[i]) {
                    si = i;
                    break;
                }
            if (si < 0) break;
            double running = 0.0;
            for (const Launch& l : inflight) running = std::max(running, l.work);
            size_t n;
            if (c.one_per_launch) {
                if (!inflight.empty()) break;
                n = 1;
            } else {
                n = batch_size(
                    admitted.size(),
                    [&](size_t k) {
                        const Req& q = reqs[admitted[k]];
                        return request_work(q.h, q.w, q.iters, B);
                    },
                    (size_t)c.max_batch, running);
            }
            if (n == 0) break;
            CHECK(n <= (size_t)c.max_batch);
            Launch l{si, 0.0, 0.0, {}};
            for (size_t k = 0; k < n; ++k) {
                const int id = admitted.front();
                admitted.pop_front();
                reqs[id].launch = now;
                l.work += request_work(reqs[id].h, reqs[id].w, reqs[id].iters, B);
                l.ids.push_back(id);
            }
            if (running > 0.0) {
                CHECK(l.work <= kBesideShare * running);
                ++res.beside_launches;
            }
            l.end = now + l.work * c.sec_per_work * (running > 0.0 ? c.beside_slowdown : 1.0);
            busy[si] = true;
            inflight.push_back(l);
            ++res.launches;
        }
    }
    // FIFO admission and a clean arena afterwards
    for (size_t i = 0; i < admit_order.size(); ++i) CHECK(admit_order[i] == (int)i);
    CHECK(arena.used() == 0 && arena.holes() == 1 && arena.largest_hole() == c.budget);
    res.reqs = reqs;
    return res;
}

double percentile(std::vector<double> v, double p) {
    std::sort(v.begin(), v.end());
    const double x = p * (double)(v.size() - 1);
    const size_t i = (size_t)x;
    return i + 1 < v.size() ? v[i] + (x - (double)i) * (v[i + 1] - v[i]) : v[i];
}

std::vector<double> latencies(const Result& r) {
    std::vector<double> v;
    for (const Req& q : r.reqs) {
        CHECK(q.admit >= q.arrive && q.launch >= q.admit && q.done > q.launch);
        v.push_back(q.done - q.arrive);
    }
    return v;
}

void arena_unit_checks() {
    Arena a;
    a.init(1000);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(300, &o1) && o1 == 0);
    CHECK(a.alloc(300, &o2) && o2 == 300);
    CHECK(a.alloc(300, &o3) && o3 == 600);
    CHECK(!a.alloc(200, &o4));                  // only 100 left
    a.release(o2, 300);                         // hole in the middle
    CHECK(a.holes() == 2 && a.used() == 600);
    CHECK(a.alloc(200, &o4) && o4 == 300);      // first fit reuses the freed slot
    a.release(o4, 200);
    a.release(o1, 300);                         // coalesces with the hole on its right
    CHECK(a.holes() == 2 && a.largest_hole() == 600);
    a.release(o3, 300);                         // and everything merges
    CHECK(a.holes() == 1 && a.largest_hole() == 1000 && a.used() == 0);
    // batch_size: full batch alone, a small leading run beside a running one
    const double works[] = {10.0, 10.0, 50.0, 1.0};
    auto at = [&](size_t k) { return works[k]; };
    CHECK(batch_size(4, at, 3, 0.0) == 3);
    CHECK(batch_size(4, at, 8, 0.0) == 4);
    CHECK(batch_size(4, at, 8, 80.0) == 2);     // 10 + 10 <= 20 < 10 + 10 + 50
    CHECK(batch_size(4, at, 8, 30.0) == 0);     // 10 > 7.5: wait
    CHECK(batch_size(0, at, 8, 0.0) == 0);
    CHECK(request_bytes(1080, 1920) == 2 * 4 * 1080 * 1920 + 1080 * 1920);
    CHECK(request_work(1080, 1920, 100, 4) == 129600.0 * 108.0);
}

}  // namespace

int main() {
    arena_unit_checks();
    const auto tr = trace(2000, 240.0, 1400);
    const double spw = 3.75e-3 / (129600.0 * 108.0);   // a 1080p frame in 3.75 ms
    const Config cont{size_t(4) << 30, 64, 16, 2, false, spw, 1.1};
    const Config fifo{size_t(4) << 30, 64, 16, 1, true, spw, 1.0};
    const Config tight{size_t(48) << 20, 64, 16, 2, false, spw, 1.1};
    const Config narrow{size_t(4) << 30, 4, 16, 2, false, spw, 1.1};
    const Result rc = simulate(tr, cont), rf = simulate(tr, fifo), rt = simulate(tr, tight),
                 rn = simulate(tr, narrow);
    const auto lc = latencies(rc), lf = latencies(rf), lt = latencies(rt), ln = latencies(rn);
    const double c50 = percentile(lc, 0.5), c99 = percentile(lc, 0.99);
    const double f50 = percentile(lf, 0.5), f99 = percentile(lf, 0.99);
    std::printf("continuous p50 %.2f ms p99 %.2f ms, %d launches (%d beside)\n", c50 * 1e3, c99 * 1e3,
                rc.launches, rc.beside_launches);
    std::printf("one per launch p50 %.2f ms p99 %.2f ms, %d launches\n", f50 * 1e3, f99 * 1e3, rf.launches);
    std::printf("48 MiB budget: peak %.1f MiB, p99 %.2f ms; 4 in flight: p99 %.2f ms\n",
                rt.peak_bytes / 1048576.0, percentile(lt, 0.99) * 1e3, percentile(ln, 0.99) * 1e3);
    CHECK(rf.launches == 2000 && rc.launches < 2000);   // batching took several requests per launch
    CHECK(rc.beside_launches > 0);                      // small frames ran beside large ones
    CHECK(c50 < f50);                                   // and that shortens the typical wait
    CHECK(rt.peak_bytes <= tight.budget && rt.peak_bytes > tight.budget / 2);
    CHECK(percentile(lt, 0.99) >= c99);                 // a tight budget can only delay
    CHECK(percentile(ln, 0.99) >= c99);                 // so can a low in-flight limit
    std::printf("ok\n");
    return 0;
}
