// fsr_serve.cpp -- continuous-batching frame server on one GPU.
//
// One scheduler thread per server owns every HIP call after creation:
//   admit    requests leave the FIFO queue while the in-flight limit and the
//            device arena allow; their image and mask are copied into the
//            arena (copy stream in continuous mode);
//   launch   continuous mode: whenever fewer than `streams` launches are in
//            flight, all admitted requests (up to max_batch) form one
//            batched launch on a free compute stream, after their uploads;
//            FIFO mode: each admitted request is uploaded and reconstructed
//            by the one-image kernel on a single stream, in arrival order;
//   complete launches are polled through events; their requests become done
//            and keep their output in the arena until fetched or released.
// Client calls (submit, poll, wait, result, release, timing) only touch the
// shared state under the server mutex.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fsr_runtime.h"
#include "fsr_sched.h"

namespace fsr {
namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

using sched::align256;
using sched::Arena;

enum class State { Queued, Admitted, Launched, Done };

struct Request {
    fsr_request r{};
    State state = State::Queued;
    size_t off = 0, bytes = 0;
    float* d_img = nullptr;
    uint8_t* d_mask = nullptr;
    float* d_out = nullptr;
    hipEvent_t uploaded = nullptr;
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
};

struct Launch {
    int stream = 0;
    hipEvent_t done = nullptr;
    std::vector<uint64_t> ids;
    double work = 0.0;   // block-iterations of the batch
};

double request_work(const fsr_request& r, const fsr_params& p) {
    return sched::request_work(r.height, r.width, r.iterations, p.block);
}

size_t request_bytes(const fsr_request& r) { return sched::request_bytes(r.height, r.width); }

}  // namespace
}  // namespace fsr

using namespace fsr;

struct fsr_server {
    fsr_context* ctx = nullptr;
    fsr_params params{};
    fsr_server_config cfg{};
    int device = 0;
    char* arena_base = nullptr;
    Arena arena;
    hipStream_t copy_stream = nullptr;
    hipStream_t streams[2] = {nullptr, nullptr};
    bool stream_busy[2] = {false, false};
    void* workspace[2] = {nullptr, nullptr};
    size_t ws_bytes = 0;
    StagingSlot staging[2];
    std::vector<hipEvent_t> events;           // idle events for reuse

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;               // submitted, waiting for admission
    std::deque<uint64_t> admitted;            // admitted, not launched (continuous mode)
    std::unordered_map<uint64_t, Request> reqs;
    std::vector<Launch> inflight;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    fsr_server_stats stats{};
    double busy_since = -1.0;
    fsr_status error = FSR_OK;
    std::string error_msg;
};

namespace fsr {
namespace {

hipEvent_t take_event(fsr_server* s) {
    if (!s->events.empty()) {
        hipEvent_t e = s->events.back();
        s->events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void give_event(fsr_server* s, hipEvent_t e) {
    if (e) s->events.push_back(e);
}

void fail_server(fsr_server* s, fsr_status st, const std::string& msg) {
    if (s->error == FSR_OK) {
        s->error = st;
        s->error_msg = msg;
    }
    s->cv_done.notify_all();
}

// The address under which the device reads `p`: device memory as is,
// pinned host memory through its device mapping; nullptr for memory the
// device cannot address (pageable host memory).
const void* device_view(const void* p, int32_t memory) {
    if (memory == FSR_MEM_DEVICE) return p;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (a.type != hipMemoryTypeHost || a.devicePointer == nullptr) return nullptr;
    return static_cast<const char*>(a.devicePointer) +
           (static_cast<const char*>(p) - static_cast<const char*>(a.hostPointer));
}

// Host frames up to this size go through the copy kernel; larger ones
// through the runtime's copy.
constexpr size_t kKernelUploadMaxBytes = size_t(4) << 20;

// Copies a request's image and mask into its arena slot on `stream`.  A copy
// command waits for the kernels that other streams are running, so frames
// that should start beside a running one are moved by a copy kernel: device
// memory always, pinned host frames up to kKernelUploadMaxBytes.  Larger host
// frames use the runtime's copy, which moves them faster over PCIe than a
// kernel's reads and occupies no compute units (measured on the 240 frames/s
// stream of 720p to 2160p frames: p50 34 against 47 ms).
bool upload(fsr_server* s, Request& q, hipStream_t stream) {
    const fsr_request& r = q.r;
    const size_t bytes = (size_t)r.height * (size_t)r.width * 5;
    const bool by_kernel = r.memory == FSR_MEM_DEVICE || bytes <= kKernelUploadMaxBytes;
    const void* img = by_kernel ? device_view(r.image, r.memory) : nullptr;
    const void* msk = img ? device_view(r.mask, r.memory) : nullptr;
    hipError_t e;
    if (img && msk) {
        e = launch_copy2d(q.d_img, (size_t)r.width * 4, img, (size_t)r.stride * 4, (size_t)r.width * 4,
                          (size_t)r.height, stream);
        if (e == hipSuccess)
            e = launch_copy2d(q.d_mask, (size_t)r.width, msk, (size_t)r.stride, (size_t)r.width,
                              (size_t)r.height, stream);
    } else {
        const hipMemcpyKind kind = r.memory == FSR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        e = hipMemcpy2DAsync(q.d_img, (size_t)r.width * 4, r.image, (size_t)r.stride * 4,
                             (size_t)r.width * 4, r.height, kind, stream);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(q.d_mask, (size_t)r.width, r.mask, (size_t)r.stride, (size_t)r.width,
                                 r.height, kind, stream);
    }
    if (e != hipSuccess) {
        fail_server(s, FSR_ERR_HIP, std::string("request upload: ") + hipGetErrorString(e));
        return false;
    }
    return true;
}

void mark_busy(fsr_server* s) {
    if (s->busy_since < 0.0) s->busy_since = now_s();
}

void admit(fsr_server* s) {
    while (!s->queue.empty() && s->error == FSR_OK) {
        const size_t active = s->stats.admitted - s->stats.completed;
        if (active >= (size_t)s->cfg.max_inflight) return;
        Request& q = s->reqs[s->queue.front()];
        size_t off = 0;
        if (!s->arena.alloc(q.bytes, &off)) return;          // wait for space, keep FIFO order
        q.off = off;
        const size_t px = (size_t)q.r.height * (size_t)q.r.width;
        q.d_img = reinterpret_cast<float*>(s->arena_base + off);
        q.d_mask = reinterpret_cast<uint8_t*>(s->arena_base + off + align256(4 * px));
        q.d_out = reinterpret_cast<float*>(s->arena_base + off + align256(4 * px) + align256(px));
        q.state = State::Admitted;
        q.t_admit = now_s();
        const uint64_t id = s->queue.front();
        s->queue.pop_front();
        ++s->stats.admitted;
        s->stats.bytes_in_use = s->arena.used();
        s->stats.peak_bytes_in_use = std::max(s->stats.peak_bytes_in_use, s->stats.bytes_in_use);
        if (s->cfg.mode == FSR_SERVE_FIFO) {
            // reference loop: upload and one-image reconstruction in stream order
            if (!upload(s, q, s->streams[0])) return;
            fsr_params p = s->params;
            p.iterations = q.r.iterations;
            fsr_status st = fsr_reconstruct(s->ctx, q.d_img, q.d_mask, q.d_out, q.r.height, q.r.width,
                                            q.r.width, &p, nullptr, s->streams[0]);
            Launch l;
            l.stream = 0;
            l.done = take_event(s);
            if (st != FSR_OK || !l.done || hipEventRecord(l.done, s->streams[0]) != hipSuccess) {
                fail_server(s, st != FSR_OK ? st : FSR_ERR_HIP, fsr_last_error_message());
                give_event(s, l.done);
                return;
            }
            l.ids.push_back(id);
            q.state = State::Launched;
            q.t_launch = now_s();
            ++s->stats.launches;
            mark_busy(s);
            s->inflight.push_back(std::move(l));
        } else {
            q.uploaded = take_event(s);
            if (!q.uploaded) {
                fail_server(s, FSR_ERR_HIP, "event creation failed");
                return;
            }
            if (!upload(s, q, s->copy_stream)) return;
            if (hipEventRecord(q.uploaded, s->copy_stream) != hipSuccess) {
                fail_server(s, FSR_ERR_HIP, "hipEventRecord after upload");
                return;
            }
            s->admitted.push_back(id);
        }
    }
}

void launch_batches(fsr_server* s) {
    while (!s->admitted.empty() && s->error == FSR_OK) {
        int si = -1;
        for (int i = 0; i < s->cfg.streams; ++i)
            if (!s->stream_busy[i]) {
                si = i;
                break;
            }
        if (si < 0) return;
        hipStream_t st = s->streams[si];
        // beside a running batch only a small one (sched::batch_size)
        double running = 0.0;
        for (const Launch& r : s->inflight) running = std::max(running, r.work);
        const size_t n = sched::batch_size(
            s->admitted.size(), [&](size_t k) { return request_work(s->reqs[s->admitted[k]].r, s->params); },
            (size_t)s->cfg.max_batch, running);
        if (n == 0) return;   // wait for the running batch
        std::vector<fsr_image_desc> descs(n);
        Launch l;
        l.stream = si;
        for (size_t k = 0; k < n; ++k) {
            const uint64_t id = s->admitted.front();
            s->admitted.pop_front();
            Request& q = s->reqs[id];
            if (hipStreamWaitEvent(st, q.uploaded, 0) != hipSuccess) {
                fail_server(s, FSR_ERR_HIP, "hipStreamWaitEvent");
                return;
            }
            descs[k] = fsr_image_desc{q.d_img, q.d_mask, q.d_out, nullptr, q.r.height, q.r.width,
                                      (int64_t)q.r.width, q.r.iterations, 0};
            l.ids.push_back(id);
            l.work += request_work(q.r, s->params);
        }
        const fsr_batch_schedule flat{1, 0, 10, 0};
        fsr_status rs = batched_enqueue(s->ctx, descs.data(), (int32_t)n, &s->params, &flat,
                                        s->workspace[si], s->ws_bytes, st, &s->staging[si], nullptr);
        l.done = take_event(s);
        if (rs != FSR_OK || !l.done || hipEventRecord(l.done, st) != hipSuccess) {
            fail_server(s, rs != FSR_OK ? rs : FSR_ERR_HIP, fsr_last_error_message());
            give_event(s, l.done);
            return;
        }
        const double t = now_s();
        for (uint64_t id : l.ids) {
            Request& q = s->reqs[id];
            q.state = State::Launched;
            q.t_launch = t;
            give_event(s, q.uploaded);
            q.uploaded = nullptr;
        }
        s->stream_busy[si] = true;
        ++s->stats.launches;
        mark_busy(s);
        s->inflight.push_back(std::move(l));
    }
}

// Returns true when at least one launch finished.
bool poll_completions(fsr_server* s) {
    bool any = false;
    for (size_t i = 0; i < s->inflight.size();) {
        Launch& l = s->inflight[i];
        const hipError_t e = hipEventQuery(l.done);
        if (e == hipErrorNotReady) {
            ++i;
            continue;
        }
        if (e != hipSuccess) {
            fail_server(s, FSR_ERR_HIP, std::string("reconstruction failed: ") + hipGetErrorString(e));
            return any;
        }
        const double t = now_s();
        for (uint64_t id : l.ids) {
            Request& q = s->reqs[id];
            q.state = State::Done;
            q.t_done = t;
            ++s->stats.completed;
        }
        s->stream_busy[l.stream] = false;
        give_event(s, l.done);
        s->inflight.erase(s->inflight.begin() + (long)i);
        any = true;
    }
    if (s->inflight.empty() && s->busy_since >= 0.0) {
        s->stats.busy_s += now_s() - s->busy_since;
        s->busy_since = -1.0;
    }
    if (any) s->cv_done.notify_all();
    return any;
}

void worker_main(fsr_server* s) {
    DeviceGuard g(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        poll_completions(s);
        if (s->stop) {
            // drop what was never admitted; finish what was
            for (uint64_t id : s->queue) s->reqs.erase(id);
            s->queue.clear();
        } else if (s->error == FSR_OK) {
            admit(s);
            if (s->cfg.mode == FSR_SERVE_CONTINUOUS) launch_batches(s);
        }
        const bool pending_admitted = !s->admitted.empty() && s->error == FSR_OK && !s->stop;
        if (s->stop && s->inflight.empty() && !pending_admitted) break;
        if (s->error != FSR_OK && s->inflight.empty()) {
            if (s->stop) break;
            s->cv_work.wait(lk);
            continue;
        }
        if (!s->inflight.empty())
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));   // poll the device
        else if (!pending_admitted && !s->stop)
            s->cv_work.wait(lk);                                      // idle until a submit
    }
    // launches admitted but never started are discarded at shutdown
    for (uint64_t id : s->admitted) {
        give_event(s, s->reqs[id].uploaded);
        s->reqs[id].uploaded = nullptr;
    }
    s->admitted.clear();
    s->cv_done.notify_all();
}

fsr_status check_config(const fsr_server_config* c) {
    if (!c) return errorf(FSR_ERR_INVALID_ARG, "config is NULL");
    if (c->hbm_budget < 4096) return errorf(FSR_ERR_INVALID_ARG, "hbm_budget must be >= 4096 bytes");
    if (c->max_inflight < 1 || c->max_inflight > 4096)
        return errorf(FSR_ERR_INVALID_ARG, "max_inflight must lie in [1, 4096] (got %d)", c->max_inflight);
    if (c->max_batch < 1 || c->max_batch > c->max_inflight)
        return errorf(FSR_ERR_INVALID_ARG, "max_batch must lie in [1, max_inflight] (got %d)", c->max_batch);
    if (c->streams != 1 && c->streams != 2)
        return errorf(FSR_ERR_INVALID_ARG, "streams must be 1 or 2 (got %d)", c->streams);
    if (c->mode != FSR_SERVE_CONTINUOUS && c->mode != FSR_SERVE_FIFO)
        return errorf(FSR_ERR_INVALID_ARG, "unknown serving mode %d", c->mode);
    for (int32_t v : c->reserved)
        if (v != 0) return errorf(FSR_ERR_INVALID_ARG, "config.reserved must be 0");
    return FSR_OK;
}

void free_resources(fsr_server* s) {
    DeviceGuard g(s->device);
    for (int i = 0; i < 2; ++i) {
        if (s->streams[i]) (void)hipStreamSynchronize(s->streams[i]);
        release_staging(s->staging[i]);
        if (s->workspace[i]) (void)hipFree(s->workspace[i]);
        if (s->streams[i]) (void)hipStreamDestroy(s->streams[i]);
    }
    if (s->copy_stream) {
        (void)hipStreamSynchronize(s->copy_stream);
        (void)hipStreamDestroy(s->copy_stream);
    }
    for (auto& kv : s->reqs)
        if (kv.second.uploaded) s->events.push_back(kv.second.uploaded);
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    if (s->arena_base) (void)hipFree(s->arena_base);
}

// A compute stream with a hardware queue of its own.  The runtime maps
// ordinary streams onto a few hardware queues by itself, and two streams in
// one queue run their launches one after the other: a small frame then waits
// for a large one launched on the other stream.  A stream created with a CU
// mask gets its own queue; the mask enables every compute unit.  Such
// streams synchronise with the legacy null stream.  If the call fails, an
// ordinary non-blocking stream is used.
hipError_t create_compute_stream(hipStream_t* out) {
    int device = 0, cus = 0;
    hipError_t e = hipGetDevice(&device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess && cus > 0) {
        std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0xFFFFFFFFu);
        if (cus % 32) mask.back() = (1u << (cus % 32)) - 1u;
        if (hipExtStreamCreateWithCUMask(out, (uint32_t)mask.size(), mask.data()) == hipSuccess) return hipSuccess;
        (void)hipGetLastError();
    }
    return hipStreamCreateWithFlags(out, hipStreamNonBlocking);
}

}  // namespace
}  // namespace fsr

extern "C" {

fsr_status fsr_server_create(fsr_context* ctx, const fsr_params* params, const fsr_server_config* cfg,
                             fsr_server** out) {
    if (!out) return errorf(FSR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx) return errorf(FSR_ERR_INVALID_ARG, "context is NULL");
    fsr_status st = validate_params(params);
    if (st != FSR_OK) return st;
    if ((st = check_supported(params)) != FSR_OK) return st;
    if (params->flags & FSR_FLAG_LDS_ARGMAX)
        return errorf(FSR_ERR_UNSUPPORTED, "the LDS argmax runs in fsr_reconstruct only");
    const int S = params->block + 2 * params->border;
    if (S != kS && params->dft != FSR_DFT_FP32)
        return errorf(FSR_ERR_UNSUPPORTED, "support %d runs with FSR_DFT_FP32 only", S);
    if ((st = check_config(cfg)) != FSR_OK) return st;
    fsr_server* s = new (std::nothrow) fsr_server();
    if (!s) return errorf(FSR_ERR_OUT_OF_MEMORY, "server allocation failed");
    s->ctx = ctx;
    s->params = *params;
    s->cfg = *cfg;
    s->device = context_device(ctx);
    DeviceGuard g(s->device);
    hipError_t e = g.error();
    if (e == hipSuccess) e = hipMalloc(&s->arena_base, cfg->hbm_budget);
    if (e != hipSuccess) {
        delete s;
        return errorf(FSR_ERR_OUT_OF_MEMORY, "arena of %zu bytes: %s", cfg->hbm_budget, hipGetErrorString(e));
    }
    s->arena.init(cfg->hbm_budget & ~(size_t)255);
    (void)fsr_batched_workspace_size(cfg->max_batch, &s->ws_bytes);
    e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = create_compute_stream(&s->streams[i]);
        if (e == hipSuccess) e = hipMalloc(&s->workspace[i], s->ws_bytes);
    }
    if (e != hipSuccess) {
        free_resources(s);
        delete s;
        return errorf(FSR_ERR_HIP, "server streams or workspace: %s", hipGetErrorString(e));
    }
    BlockTables tab;
    if ((st = context_tables(ctx, S, params->rho, &tab)) != FSR_OK) {   // build tables before serving
        free_resources(s);
        delete s;
        return st;
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return FSR_OK;
}

fsr_status fsr_server_submit(fsr_server* s, const fsr_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket) return errorf(FSR_ERR_INVALID_ARG, "server, request and ticket must be non-NULL");
    *ticket = 0;
    if (!req->image || !req->mask) return errorf(FSR_ERR_INVALID_ARG, "image and mask must be non-NULL");
    if (req->height < 1 || req->width < 1 || req->stride < req->width)
        return errorf(FSR_ERR_INVALID_ARG, "bad request size %d x %d, stride %lld", req->height, req->width,
                      (long long)req->stride);
    if (req->iterations < 0) return errorf(FSR_ERR_INVALID_ARG, "iterations must be >= 0");
    if (req->memory != FSR_MEM_HOST && req->memory != FSR_MEM_DEVICE)
        return errorf(FSR_ERR_INVALID_ARG, "unknown memory kind %d", req->memory);
    if ((int64_t)req->height * req->width > (int64_t(1) << 32))
        return errorf(FSR_ERR_INVALID_ARG, "request too large");
    const size_t bytes = request_bytes(*req);
    if (bytes > (s->cfg.hbm_budget & ~(size_t)255))
        return errorf(FSR_ERR_BUDGET, "a %d x %d frame needs %zu bytes, over the %zu-byte budget",
                      req->height, req->width, bytes, s->cfg.hbm_budget);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error != FSR_OK) return errorf(s->error, "server failed: %s", s->error_msg.c_str());
    if (s->stop) return errorf(FSR_ERR_INVALID_ARG, "server is shutting down");
    const uint64_t id = s->next_id++;
    Request& q = s->reqs[id];
    q.r = *req;
    q.bytes = bytes;
    q.t_submit = now_s();
    s->queue.push_back(id);
    ++s->stats.submitted;
    *ticket = id;
    s->cv_work.notify_one();
    return FSR_OK;
}

fsr_status fsr_server_poll(fsr_server* s, uint64_t ticket, int32_t* done) {
    if (!s || !done) return errorf(FSR_ERR_INVALID_ARG, "server and done must be non-NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return errorf(FSR_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    *done = it->second.state == State::Done;
    if (!*done && s->error != FSR_OK) return errorf(s->error, "server failed: %s", s->error_msg.c_str());
    return FSR_OK;
}

fsr_status fsr_server_wait(fsr_server* s, uint64_t ticket, int32_t timeout_ms) {
    if (!s) return errorf(FSR_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] {
        auto it = s->reqs.find(ticket);
        return it == s->reqs.end() || it->second.state == State::Done || s->error != FSR_OK || s->stop;
    };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
        return errorf(FSR_ERR_TIMEOUT, "ticket %llu not done after %d ms", (unsigned long long)ticket, timeout_ms);
    }
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return errorf(FSR_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second.state != State::Done) {
        if (s->error != FSR_OK) return errorf(s->error, "server failed: %s", s->error_msg.c_str());
        return errorf(FSR_ERR_INVALID_ARG, "server is shutting down");
    }
    return FSR_OK;
}

static fsr_status finish_request(fsr_server* s, uint64_t ticket, float* out, int64_t out_stride,
                                 int32_t memory, bool copy) {
    if (!s) return errorf(FSR_ERR_INVALID_ARG, "server is NULL");
    float* src = nullptr;
    int32_t H = 0, W = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return errorf(FSR_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
        if (it->second.state != State::Done)
            return errorf(FSR_ERR_NOT_READY, "ticket %llu has not finished", (unsigned long long)ticket);
        src = it->second.d_out;
        H = it->second.r.height;
        W = it->second.r.width;
    }
    if (copy) {
        if (!out) return errorf(FSR_ERR_INVALID_ARG, "out is NULL");
        if (out_stride < W) return errorf(FSR_ERR_INVALID_ARG, "out_stride %lld < width %d", (long long)out_stride, W);
        if (memory != FSR_MEM_HOST && memory != FSR_MEM_DEVICE)
            return errorf(FSR_ERR_INVALID_ARG, "unknown memory kind %d", memory);
        DeviceGuard g(s->device);
        const hipMemcpyKind kind = memory == FSR_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        hipError_t e = hipMemcpy2D(out, (size_t)out_stride * 4, src, (size_t)W * 4, (size_t)W * 4, H, kind);
        if (e != hipSuccess) return hip_fail(e, "result copy");
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return errorf(FSR_ERR_INVALID_ARG, "ticket %llu released twice", (unsigned long long)ticket);
    s->arena.release(it->second.off, it->second.bytes);
    s->stats.bytes_in_use = s->arena.used();
    ++s->stats.released;
    s->reqs.erase(it);
    s->cv_work.notify_one();            // space for the next admission
    return FSR_OK;
}

fsr_status fsr_server_result(fsr_server* s, uint64_t ticket, float* out, int64_t out_stride,
                             int32_t memory) {
    return finish_request(s, ticket, out, out_stride, memory, true);
}

fsr_status fsr_server_release(fsr_server* s, uint64_t ticket) {
    return finish_request(s, ticket, nullptr, 0, FSR_MEM_HOST, false);
}

fsr_status fsr_server_timing(fsr_server* s, uint64_t ticket, double* submit_s, double* admit_s,
                             double* launch_s, double* done_s) {
    if (!s) return errorf(FSR_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return errorf(FSR_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    if (submit_s) *submit_s = it->second.t_submit;
    if (admit_s) *admit_s = it->second.t_admit;
    if (launch_s) *launch_s = it->second.t_launch;
    if (done_s) *done_s = it->second.t_done;
    return FSR_OK;
}

fsr_status fsr_server_get_stats(fsr_server* s, fsr_server_stats* out) {
    if (!s || !out) return errorf(FSR_ERR_INVALID_ARG, "server and out must be non-NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    if (s->busy_since >= 0.0) out->busy_s += now_s() - s->busy_since;
    return FSR_OK;
}

fsr_status fsr_server_destroy(fsr_server* s) {
    if (!s) return FSR_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    free_resources(s);
    delete s;
    return FSR_OK;
}

}  // extern "C"
