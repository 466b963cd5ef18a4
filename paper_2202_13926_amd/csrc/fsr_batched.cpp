// fsr_batched.cpp -- host side of the batched path: planning (validation,
// queue order, prefix sums), descriptor upload, schedules, the autotuner and
// HIP-graph capture.
#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <numeric>
#include <vector>

#include "fsr_runtime.h"

namespace fsr {

namespace {

constexpr size_t kCtrlBytes = kQueueCtrlBytes;
constexpr int64_t kMaxBlocks = int64_t(1) << 30;   // keeps the 32-bit queue head from wrapping
constexpr int kMaxGroupsPerCu = 32;                // a compute unit holds at most 32 wavefronts

size_t workspace_bytes_for(int32_t n) {
    return kCtrlBytes + ((size_t)n * sizeof(DevDesc) + 255) / 256 * 256;
}

// What the schedule choice needs to know about a planned batch.
struct PlanTotals {
    int64_t total_blocks = 0;
    double work = 0.0;            // sum over images of blocks x iterations
    int32_t max_iterations = 0;
};

struct BatchPlan {
    std::vector<DevDesc> table;   // queue order
    PlanTotals totals;
};

fsr_status check_schedule(const fsr_batch_schedule* s) {
    if (!s) return FSR_OK;
    if (s->waves_per_group != 1 && s->waves_per_group != 2 && s->waves_per_group != 4)
        return errorf(FSR_ERR_INVALID_ARG, "waves_per_group must be 1, 2 or 4 (got %d)", s->waves_per_group);
    if (s->chunk < 0 || s->chunk > 64)
        return errorf(FSR_ERR_INVALID_ARG, "chunk must lie in [0, 64] (got %d)", s->chunk);
    if (s->chunk > 0 && (s->groups_per_cu < 1 || s->groups_per_cu > kMaxGroupsPerCu))
        return errorf(FSR_ERR_INVALID_ARG, "groups_per_cu must lie in [1, %d] (got %d)", kMaxGroupsPerCu,
                      s->groups_per_cu);
    if (s->reserved != 0) return errorf(FSR_ERR_INVALID_ARG, "schedule.reserved must be 0");
    return FSR_OK;
}

// Validates every descriptor and stores its block count in blocks[i].
fsr_status check_images(const fsr_image_desc* descs, int32_t n, const fsr_params* params, int64_t* blocks) {
    if (n < 0) return errorf(FSR_ERR_INVALID_ARG, "n_images must be >= 0 (got %d)", n);
    if (n > 0 && !descs) return errorf(FSR_ERR_INVALID_ARG, "descs is NULL");
    const int B = params->block;
    for (int32_t i = 0; i < n; ++i) {
        const fsr_image_desc& d = descs[i];
        fsr_status st = validate_image(d.image, d.mask, d.out, d.height, d.width, d.stride, B);
        if (st != FSR_OK) return errorf(st, "image %d: %s", i, fsr_last_error_message());
        if (d.iterations < 0) return errorf(FSR_ERR_INVALID_ARG, "image %d: iterations must be >= 0", i);
        if (d.reserved != 0) return errorf(FSR_ERR_INVALID_ARG, "image %d: reserved must be 0", i);
        blocks[i] = fsr_num_blocks(d.height, d.width, B);
    }
    return FSR_OK;
}

// Queue order: decreasing iterations, then decreasing size, then input order.
struct QueueOrder {
    const fsr_image_desc* descs;
    const int64_t* blocks;
    bool operator()(int32_t a, int32_t b) const {
        if (descs[a].iterations != descs[b].iterations) return descs[a].iterations > descs[b].iterations;
        return blocks[a] > blocks[b];
    }
};

// Fills table[0..n) in the queue order `order` and the totals.
fsr_status fill_table(const fsr_image_desc* descs, int32_t n, const fsr_params* params, const int32_t* order,
                      const int64_t* blocks, DevDesc* table, PlanTotals* tot) {
    const int B = params->block;
    // blocks per wavefront: each image's range in the index space is padded
    // to a multiple of it, so that no wavefront spans two images
    const int64_t unit = batch_unit(params->block + 2 * params->border, B);
    *tot = PlanTotals{};
    int64_t begin = 0;
    for (int32_t j = 0; j < n; ++j) {
        const fsr_image_desc& d = descs[order[j]];
        DevDesc& e = table[j];
        e.image = d.image;
        e.mask = d.mask;
        e.out = d.out;
        e.argmax_log = d.argmax_log;
        e.stride = d.stride;
        e.block_begin = begin;
        e.height = d.height;
        e.width = d.width;
        e.iterations = d.iterations;
        e.nbx = (d.width + B - 1) / B;
        begin += (blocks[order[j]] + unit - 1) / unit * unit;
        tot->work += (double)blocks[order[j]] * (double)(d.iterations + 8);
        tot->max_iterations = std::max(tot->max_iterations, d.iterations);
    }
    if (begin > kMaxBlocks) return errorf(FSR_ERR_UNSUPPORTED, "a batch may hold at most 2^30 blocks");
    tot->total_blocks = begin;
    return FSR_OK;
}

fsr_status plan_batch(const fsr_image_desc* descs, int32_t n, const fsr_params* params,
                      BatchPlan* plan) {
    std::vector<int64_t> blocks(n > 0 ? n : 0);
    fsr_status st = check_images(descs, n, params, blocks.data());
    if (st != FSR_OK) return st;
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), QueueOrder{descs, blocks.data()});
    plan->table.resize(n);
    return fill_table(descs, n, params, order.data(), blocks.data(), plan->table.data(), &plan->totals);
}

// Key of the tuned-schedule table: log2 of the batch's work, the support
// size and the DFT mode (the kernels differ in register and LDS use) and the
// largest iteration count.
uint64_t size_class(const PlanTotals& plan, const fsr_params& params) {
    uint64_t w = 0;
    for (double x = plan.work; x >= 2.0; x /= 2.0) ++w;
    const uint64_t S = (uint64_t)(params.block + 2 * params.border);
    return (w << 48) | (S << 40) | ((uint64_t)(uint32_t)params.dft << 32) |
           (uint64_t)(uint32_t)plan.max_iterations;
}

fsr_batch_schedule default_schedule() { return fsr_batch_schedule{1, 0, 10, 0}; }

fsr_status cu_count(fsr_context* ctx, int* out) {
    BatchState& bs = context_batch(ctx);
    if (bs.cu_count == 0) {
        hipDeviceProp_t prop;
        hipError_t e = hipGetDeviceProperties(&prop, context_device(ctx));
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        bs.cu_count = prop.multiProcessorCount;
    }
    *out = bs.cu_count;
    return FSR_OK;
}

struct Prepared {
    BatchLaunch launch{};
    fsr_batch_schedule schedule{};
    int64_t groups = 0;
};

// Checks of the parameters and the schedule, before any image is looked at.
fsr_status check_batch_params(fsr_context* ctx, const fsr_params* params, const fsr_batch_schedule* schedule) {
    if (!ctx) return errorf(FSR_ERR_INVALID_ARG, "context is NULL");
    fsr_status st = validate_params(params);
    if (st != FSR_OK) return st;
    if ((st = check_supported(params)) != FSR_OK) return st;
    if (params->flags & FSR_FLAG_LDS_ARGMAX)
        return errorf(FSR_ERR_UNSUPPORTED, "the LDS argmax runs in fsr_reconstruct only");
    const int S = params->block + 2 * params->border;
    if (S != kS && params->dft != FSR_DFT_FP32)
        return errorf(FSR_ERR_UNSUPPORTED, "support %d runs with FSR_DFT_FP32 only", S);
    return check_schedule(schedule);
}

// The launch description of a planned batch whose workspace is `workspace`,
// and its schedule (given, tuned for its size class, or the default).
fsr_status finish_prepare(fsr_context* ctx, int32_t n, const fsr_params* params,
                          const fsr_batch_schedule* schedule, const PlanTotals& plan, void* workspace,
                          Prepared* prep) {
    const int S = params->block + 2 * params->border;
    prep->launch.descs = reinterpret_cast<const DevDesc*>(static_cast<char*>(workspace) + kCtrlBytes);
    prep->launch.counter = static_cast<unsigned*>(workspace);
    prep->launch.total_blocks = plan.total_blocks;
    prep->launch.n_images = n;
    prep->launch.block = params->block;
    prep->launch.border = params->border;
    prep->launch.support = S;
    prep->launch.unit = batch_unit(S, params->block);
    prep->launch.gamma = params->gamma;
    prep->launch.dft = params->dft == FSR_DFT_SPLIT_BF16 ? 1 : 0;
    if (schedule) {
        prep->schedule = *schedule;
    } else {
        BatchState& bs = context_batch(ctx);
        std::lock_guard<std::mutex> lock(context_mutex(ctx));
        auto it = bs.tuned.find(size_class(plan, *params));
        prep->schedule = it != bs.tuned.end() ? it->second : default_schedule();
    }
    prep->launch.chunk = prep->schedule.chunk;
    if (prep->schedule.chunk > 0) {
        int cus = 0;
        fsr_status st = cu_count(ctx, &cus);
        if (st != FSR_OK) return st;
        prep->groups = (int64_t)cus * prep->schedule.groups_per_cu;
    }
    return FSR_OK;
}

// Everything common to eager launches, autotuning and graph capture.
fsr_status prepare(fsr_context* ctx, const fsr_image_desc* descs, int32_t n, const fsr_params* params,
                   const fsr_batch_schedule* schedule, void* workspace, size_t ws_bytes,
                   BatchPlan* plan, Prepared* prep) {
    fsr_status st = check_batch_params(ctx, params, schedule);
    if (st != FSR_OK) return st;
    if ((st = plan_batch(descs, n, params, plan)) != FSR_OK) return st;
    if (!workspace && n > 0) return errorf(FSR_ERR_INVALID_ARG, "workspace is NULL");
    if (ws_bytes < workspace_bytes_for(n))
        return errorf(FSR_ERR_INVALID_ARG, "workspace of %zu bytes is smaller than the %zu needed",
                      ws_bytes, workspace_bytes_for(n));
    return finish_prepare(ctx, n, params, schedule, plan->totals, workspace, prep);
}

// Puts the descriptor table into the workspace, ordered on `stream`: up to
// kDescKernelMax descriptors with kernels, more through a pinned staging slot
// (the previous copy out of it must be done before it is overwritten).
fsr_status upload_async(const BatchPlan& plan, void* workspace, hipStream_t stream,
                        StagingSlot* slot) {
    const size_t bytes = plan.table.size() * sizeof(DevDesc);
    if (bytes == 0) return FSR_OK;
    hipError_t e;
    if (plan.table.size() <= (size_t)kDescKernelMax) {
        // small tables travel as kernel arguments: no copy command, so the
        // launch can run beside kernels of other streams
        e = launch_write_descs(plan.table.data(), (int)plan.table.size(),
                               reinterpret_cast<DevDesc*>(static_cast<char*>(workspace) + kCtrlBytes), stream);
        if (e != hipSuccess) return hip_fail(e, "descriptor upload");
        return FSR_OK;
    }
    if (slot->done) {
        if ((e = hipEventSynchronize(slot->done)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    } else if ((e = hipEventCreateWithFlags(&slot->done, hipEventDisableTiming)) != hipSuccess) {
        return hip_fail(e, "hipEventCreate");
    }
    if (slot->bytes < bytes) {
        if (slot->host) (void)hipHostFree(slot->host);
        slot->host = nullptr;
        slot->bytes = 0;
        if ((e = hipHostMalloc(&slot->host, bytes, hipHostMallocDefault)) != hipSuccess)
            return errorf(FSR_ERR_OUT_OF_MEMORY, "hipHostMalloc(%zu): %s", bytes, hipGetErrorString(e));
        slot->bytes = bytes;
    }
    std::memcpy(slot->host, plan.table.data(), bytes);
    e = hipMemcpyAsync(static_cast<char*>(workspace) + kCtrlBytes, slot->host, bytes,
                       hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    if ((e = hipEventRecord(slot->done, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    return FSR_OK;
}

fsr_status launch_prepared(const Prepared& prep, hipStream_t stream) {
    hipError_t e = launch_batched(prep.launch, prep.schedule.waves_per_group, prep.groups, stream);
    if (e != hipSuccess) return hip_fail(e, "launch of the batched kernel");
    return FSR_OK;
}

}  // namespace

void release_staging(StagingSlot& slot) {
    if (slot.done) {
        (void)hipEventSynchronize(slot.done);
        (void)hipEventDestroy(slot.done);
    }
    if (slot.host) (void)hipHostFree(slot.host);
    slot = StagingSlot{};
}

void release_batch_state(BatchState& st) {
    release_staging(st.staging);
    st.tuned.clear();
}

fsr_status batched_enqueue(fsr_context* ctx, const fsr_image_desc* descs, int32_t n,
                           const fsr_params* params, const fsr_batch_schedule* schedule,
                           void* workspace, size_t ws_bytes, hipStream_t stream,
                           StagingSlot* slot, std::mutex* slot_mutex) {
    BatchPlan plan;
    Prepared prep;
    fsr_status st = prepare(ctx, descs, n, params, schedule, workspace, ws_bytes, &plan, &prep);
    if (st != FSR_OK) return st;
    if (plan.totals.total_blocks == 0) return FSR_OK;
    DeviceGuard g(context_device(ctx));
    if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cap);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (cap != hipStreamCaptureStatusNone)
        return errorf(FSR_ERR_UNSUPPORTED, "stream is being captured: use fsr_batch_graph_create");
    if ((st = context_tables(ctx, prep.launch.support, params->rho, &prep.launch.tab)) != FSR_OK) return st;
    if (slot_mutex) {
        std::lock_guard<std::mutex> lock(*slot_mutex);
        if ((st = upload_async(plan, workspace, stream, slot)) != FSR_OK) return st;
    } else if ((st = upload_async(plan, workspace, stream, slot)) != FSR_OK) {
        return st;
    }
    return launch_prepared(prep, stream);
}

}  // namespace fsr

using namespace fsr;

struct fsr_batch_graph {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

fsr_status fsr_batched_workspace_size(int32_t n_images, size_t* bytes) {
    if (!bytes) return errorf(FSR_ERR_INVALID_ARG, "bytes is NULL");
    if (n_images < 0) return errorf(FSR_ERR_INVALID_ARG, "n_images must be >= 0 (got %d)", n_images);
    *bytes = workspace_bytes_for(n_images);
    return FSR_OK;
}

fsr_status fsr_reconstruct_batched(fsr_context* ctx, const fsr_image_desc* descs, int32_t n_images,
                                   const fsr_params* params, const fsr_batch_schedule* schedule,
                                   void* workspace, size_t workspace_bytes, void* stream) {
    if (!ctx) return errorf(FSR_ERR_INVALID_ARG, "context is NULL");
    return batched_enqueue(ctx, descs, n_images, params, schedule, workspace, workspace_bytes,
                           (hipStream_t)stream, &context_batch(ctx).staging,
                           &context_batch_mutex(ctx));
}

fsr_status fsr_reconstruct_batched_noalloc(fsr_context* ctx, const fsr_image_desc* descs, int32_t n_images,
                                           const fsr_params* params, const fsr_batch_schedule* schedule,
                                           void* stream) {
    // planned in fixed arrays: nothing is allocated on the host either
    fsr_status st = check_batch_params(ctx, params, schedule);
    if (st != FSR_OK) return st;
    if (n_images > kStaticImages)
        return errorf(FSR_ERR_INVALID_ARG, "at most %d images per call without allocation (got %d)",
                      kStaticImages, n_images);
    int64_t blocks[kStaticImages];
    int32_t order[kStaticImages];
    DevDesc table[kStaticImages];
    if ((st = check_images(descs, n_images, params, blocks)) != FSR_OK) return st;
    // queue order by a stable insertion sort (std::stable_sort may allocate)
    const QueueOrder before{descs, blocks};
    for (int32_t i = 0; i < n_images; ++i) {
        int32_t j = i;
        for (; j > 0 && before(i, order[j - 1]); --j) order[j] = order[j - 1];
        order[j] = i;
    }
    PlanTotals tot;
    if ((st = fill_table(descs, n_images, params, order, blocks, table, &tot)) != FSR_OK) return st;
    void* ws = static_workspace(context_device(ctx));
    if (!ws) return errorf(FSR_ERR_HIP, "the fixed workspace of device %d was not found", context_device(ctx));
    Prepared prep;
    if ((st = finish_prepare(ctx, n_images, params, schedule, tot, ws, &prep)) != FSR_OK) return st;
    if (tot.total_blocks == 0) return FSR_OK;
    // tables must exist already: building them would allocate
    if ((st = context_tables(ctx, prep.launch.support, params->rho, &prep.launch.tab, false)) != FSR_OK)
        return st;
    DeviceGuard g(context_device(ctx));
    if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
    const hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_write_descs(table, n_images,
                                      reinterpret_cast<DevDesc*>(static_cast<char*>(ws) + kCtrlBytes), s);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    return launch_prepared(prep, s);
}

fsr_status fsr_batch_autotune(fsr_context* ctx, const fsr_image_desc* descs, int32_t n_images,
                              const fsr_params* params, void* workspace, size_t workspace_bytes,
                              void* stream, fsr_batch_schedule* best) {
    if (!best) return errorf(FSR_ERR_INVALID_ARG, "best is NULL");
    // fixed candidates, then persistent ones that fill every compute unit
    // with as many workgroups as the kernel's registers and LDS allow
    static const fsr_batch_schedule kFixed[] = {
        {1, 0, 10, 0}, {2, 0, 5, 0}, {4, 0, 2, 0},
        {1, 1, 10, 0}, {1, 2, 10, 0}, {1, 4, 10, 0}, {1, 8, 10, 0}, {1, 16, 10, 0},
        {2, 2, 5, 0}, {2, 4, 5, 0}, {2, 8, 5, 0}, {1, 4, 8, 0}, {4, 4, 2, 0},
    };
    std::vector<fsr_batch_schedule> cands(std::begin(kFixed), std::end(kFixed));
    BatchPlan plan;
    Prepared prep;
    fsr_status st = prepare(ctx, descs, n_images, params, &cands[0], workspace, workspace_bytes,
                            &plan, &prep);
    if (st != FSR_OK) return st;
    *best = default_schedule();
    if (plan.totals.total_blocks == 0) return FSR_OK;
    DeviceGuard g(context_device(ctx));
    if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if ((st = context_tables(ctx, prep.launch.support, params->rho, &prep.launch.tab)) != FSR_OK) return st;
    {
        std::lock_guard<std::mutex> lock(context_batch_mutex(ctx));
        if ((st = upload_async(plan, workspace, s, &context_batch(ctx).staging)) != FSR_OK) return st;
    }
    int cus = 0;
    if ((st = cu_count(ctx, &cus)) != FSR_OK) return st;
    for (const int wpg : {1, 2, 4}) {
        int resident = 0;
        hipError_t re = batched_resident_groups(prep.launch, wpg, &resident);
        if (re != hipSuccess) return hip_fail(re, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
        resident = std::min(std::max(resident, 1), kMaxGroupsPerCu);
        for (const int chunk : {4, 16}) {
            const fsr_batch_schedule c{wpg, chunk, resident, 0};
            const bool seen = std::any_of(cands.begin(), cands.end(), [&](const fsr_batch_schedule& o) {
                return o.waves_per_group == c.waves_per_group && o.chunk == c.chunk &&
                       o.groups_per_cu == c.groups_per_cu;
            });
            if (!seen) cands.push_back(c);
        }
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    float best_ms = -1.0f;
    for (const fsr_batch_schedule& cand : cands) {
        Prepared p = prep;
        p.schedule = cand;
        p.launch.chunk = cand.chunk;
        p.groups = cand.chunk > 0 ? (int64_t)cus * cand.groups_per_cu : 0;
        if ((st = launch_prepared(p, s)) != FSR_OK) break;          // warm-up run
        if ((e = hipEventRecord(t0, s)) != hipSuccess) { st = hip_fail(e, "hipEventRecord"); break; }
        for (int r = 0; r < 2 && st == FSR_OK; ++r) st = launch_prepared(p, s);
        if (st != FSR_OK) break;
        if ((e = hipEventRecord(t1, s)) != hipSuccess) { st = hip_fail(e, "hipEventRecord"); break; }
        if ((e = hipEventSynchronize(t1)) != hipSuccess) { st = hip_fail(e, "hipEventSynchronize"); break; }
        float ms = 0.0f;
        if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) { st = hip_fail(e, "hipEventElapsedTime"); break; }
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            *best = cand;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (st != FSR_OK) return st;
    std::lock_guard<std::mutex> lock(context_mutex(ctx));
    context_batch(ctx).tuned[size_class(plan.totals, *params)] = *best;
    return FSR_OK;
}

fsr_status fsr_batch_graph_create(fsr_context* ctx, const fsr_image_desc* descs, int32_t n_images,
                                  const fsr_params* params, const fsr_batch_schedule* schedule,
                                  void* workspace, size_t workspace_bytes, fsr_batch_graph** out) {
    if (!out) return errorf(FSR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    BatchPlan plan;
    Prepared prep;
    fsr_status st = prepare(ctx, descs, n_images, params, schedule, workspace, workspace_bytes, &plan, &prep);
    if (st != FSR_OK) return st;
    DeviceGuard g(context_device(ctx));
    if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
    if ((st = context_tables(ctx, prep.launch.support, params->rho, &prep.launch.tab)) != FSR_OK) return st;
    hipError_t e;
    if (!plan.table.empty()) {
        e = hipMemcpy(static_cast<char*>(workspace) + kCtrlBytes, plan.table.data(),
                      plan.table.size() * sizeof(DevDesc), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    }
    hipStream_t cs = nullptr;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
    fsr_batch_graph* gr = new (std::nothrow) fsr_batch_graph();
    if (!gr) {
        (void)hipStreamDestroy(cs);
        return errorf(FSR_ERR_OUT_OF_MEMORY, "graph allocation failed");
    }
    gr->device = context_device(ctx);
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        if (plan.totals.total_blocks > 0) st = launch_prepared(prep, cs);
        hipError_t e2 = hipStreamEndCapture(cs, &gr->graph);
        if (st == FSR_OK && e2 != hipSuccess) st = hip_fail(e2, "hipStreamEndCapture");
    } else {
        st = hip_fail(e, "hipStreamBeginCapture");
    }
    if (st == FSR_OK && (e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0)) != hipSuccess)
        st = hip_fail(e, "hipGraphInstantiate");
    (void)hipStreamDestroy(cs);
    if (st != FSR_OK) {
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
        delete gr;
        return st;
    }
    *out = gr;
    return FSR_OK;
}

fsr_status fsr_batch_graph_launch(fsr_batch_graph* graph, void* stream) {
    if (!graph || !graph->exec) return errorf(FSR_ERR_INVALID_ARG, "graph is NULL");
    DeviceGuard g(graph->device);
    if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
    hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return FSR_OK;
}

fsr_status fsr_batch_graph_destroy(fsr_batch_graph* graph) {
    if (!graph) return FSR_OK;
    {
        DeviceGuard g(graph->device);
        if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
        if (graph->graph) (void)hipGraphDestroy(graph->graph);
    }
    delete graph;
    return FSR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- tuning cache
namespace fsr {
namespace {

constexpr const char* kTuningFormat = "fsr-batch-tuning-1";

fsr_status device_identity(fsr_context* ctx, std::string* arch, int* cus) {
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, context_device(ctx));
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    *arch = prop.gcnArchName;
    *cus = prop.multiProcessorCount;
    return FSR_OK;
}

// A strict reader of the one JSON shape fsr_batch_tuning_export writes.
struct Reader {
    const char* p;
    void ws() {
        while (*p && std::isspace((unsigned char)*p)) ++p;
    }
    bool lit(char c) {
        ws();
        if (*p != c) return false;
        ++p;
        return true;
    }
    bool str(std::string* out) {
        if (!lit('"')) return false;
        out->clear();
        while (*p && *p != '"') {
            if (*p == '\\' || (unsigned char)*p < 0x20) return false;   // no escapes in this format
            out->push_back(*p++);
        }
        if (*p != '"') return false;
        ++p;
        return true;
    }
    bool num(long long lo, long long hi, long long* out) {
        ws();
        if (!(*p == '-' || std::isdigit((unsigned char)*p))) return false;
        char* end = nullptr;
        const long long v = std::strtoll(p, &end, 10);
        if (end == p || v < lo || v > hi) return false;
        p = end;
        *out = v;
        return true;
    }
    bool unum(unsigned long long* out) {
        ws();
        if (!std::isdigit((unsigned char)*p)) return false;
        char* end = nullptr;
        *out = std::strtoull(p, &end, 10);
        if (end == p) return false;
        p = end;
        return true;
    }
};

}  // namespace
}  // namespace fsr

extern "C" {

fsr_status fsr_batch_tuning_export(fsr_context* ctx, char* buf, size_t cap, size_t* len) {
    if (!ctx || !len) return errorf(FSR_ERR_INVALID_ARG, "context and len must be non-NULL");
    DeviceGuard g(context_device(ctx));
    if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
    std::string arch;
    int cus = 0;
    fsr_status st = device_identity(ctx, &arch, &cus);
    if (st != FSR_OK) return st;
    std::string out = std::string("{\"format\": \"") + kTuningFormat + "\", \"arch\": \"" + arch +
                      "\", \"cus\": " + std::to_string(cus) + ", \"entries\": [";
    {
        std::lock_guard<std::mutex> lock(context_mutex(ctx));
        bool first = true;
        for (const auto& kv : context_batch(ctx).tuned) {
            char item[160];
            std::snprintf(item, sizeof item, "%s[%llu, %d, %d, %d]", first ? "" : ", ",
                          (unsigned long long)kv.first, kv.second.waves_per_group, kv.second.chunk,
                          kv.second.groups_per_cu);
            out += item;
            first = false;
        }
    }
    out += "]}";
    *len = out.size() + 1;
    if (!buf) return FSR_OK;
    if (cap < *len) return errorf(FSR_ERR_INVALID_ARG, "buffer of %zu bytes is smaller than %zu", cap, *len);
    std::memcpy(buf, out.c_str(), *len);
    return FSR_OK;
}

fsr_status fsr_batch_tuning_import(fsr_context* ctx, const char* json) {
    if (!ctx || !json) return errorf(FSR_ERR_INVALID_ARG, "context and json must be non-NULL");
    // parse and check everything before the context is touched
    Reader r{json};
    std::string key, format, arch;
    long long cus = -1;
    std::map<uint64_t, fsr_batch_schedule> entries;
    bool have_entries = false;
    if (!r.lit('{')) return errorf(FSR_ERR_INVALID_ARG, "tuning text: expected '{'");
    for (bool first = true;; first = false) {
        if (!first && !r.lit(',')) break;
        if (!r.str(&key) || !r.lit(':')) return errorf(FSR_ERR_INVALID_ARG, "tuning text: expected a key");
        if (key == "format") {
            if (!r.str(&format)) return errorf(FSR_ERR_INVALID_ARG, "tuning text: bad format");
        } else if (key == "arch") {
            if (!r.str(&arch)) return errorf(FSR_ERR_INVALID_ARG, "tuning text: bad arch");
        } else if (key == "cus") {
            if (!r.num(1, 1 << 20, &cus)) return errorf(FSR_ERR_INVALID_ARG, "tuning text: bad cus");
        } else if (key == "entries") {
            if (!r.lit('[')) return errorf(FSR_ERR_INVALID_ARG, "tuning text: entries must be a list");
            have_entries = true;
            if (!r.lit(']')) {
                do {
                    unsigned long long k = 0;
                    long long w = 0, c = 0, gpc = 0;
                    if (!r.lit('[') || !r.unum(&k) || !r.lit(',') || !r.num(0, 64, &w) || !r.lit(',') ||
                        !r.num(0, 64, &c) || !r.lit(',') || !r.num(0, 1 << 20, &gpc) || !r.lit(']'))
                        return errorf(FSR_ERR_INVALID_ARG, "tuning text: bad entry");
                    const fsr_batch_schedule sch{(int32_t)w, (int32_t)c, (int32_t)gpc, 0};
                    fsr_status st = check_schedule(&sch);
                    if (st != FSR_OK) return st;
                    entries[(uint64_t)k] = sch;
                } while (r.lit(','));
                if (!r.lit(']')) return errorf(FSR_ERR_INVALID_ARG, "tuning text: unterminated entries");
            }
        } else {
            return errorf(FSR_ERR_INVALID_ARG, "tuning text: unknown key '%s'", key.c_str());
        }
    }
    if (!r.lit('}')) return errorf(FSR_ERR_INVALID_ARG, "tuning text: expected '}'");
    r.ws();
    if (*r.p) return errorf(FSR_ERR_INVALID_ARG, "tuning text: trailing characters");
    if (format != kTuningFormat || arch.empty() || cus < 0 || !have_entries)
        return errorf(FSR_ERR_INVALID_ARG, "tuning text: format, arch, cus and entries are required");

    DeviceGuard g(context_device(ctx));
    if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
    std::string my_arch;
    int my_cus = 0;
    fsr_status st = device_identity(ctx, &my_arch, &my_cus);
    if (st != FSR_OK) return st;
    if (arch != my_arch || cus != my_cus)
        return errorf(FSR_ERR_UNSUPPORTED, "tuning made on %s with %lld CUs; this device is %s with %d",
                      arch.c_str(), cus, my_arch.c_str(), my_cus);
    std::lock_guard<std::mutex> lock(context_mutex(ctx));
    for (const auto& kv : entries) context_batch(ctx).tuned[kv.first] = kv.second;
    return FSR_OK;
}

}  // extern "C"
