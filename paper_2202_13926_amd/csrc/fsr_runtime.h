// fsr_runtime.h -- host runtime pieces shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>

#include "fsr.h"
#include "fsr_batch_internal.h"
#include "fsr_internal.h"

namespace fsr {

// Makes `device` current for the lifetime of the guard and restores the
// caller's device afterwards.
class DeviceGuard {
public:
    explicit DeviceGuard(int device);
    ~DeviceGuard();
    hipError_t error() const { return err_; }
    DeviceGuard(const DeviceGuard&) = delete;
    DeviceGuard& operator=(const DeviceGuard&) = delete;

private:
    int prev_ = -1;
    bool changed_ = false;
    hipError_t err_ = hipSuccess;
};

// Pinned host buffer through which a batch's descriptors reach the device,
// and the event that marks the last copy out of it as done.
struct StagingSlot {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
};

void release_staging(StagingSlot& slot);

// Per-context state of the batched path: the staging slot of
// fsr_reconstruct_batched, the device's compute-unit count and the
// schedules chosen by the autotuner.
struct BatchState {
    StagingSlot staging;
    int cu_count = 0;
    std::map<uint64_t, fsr_batch_schedule> tuned;
};

void release_batch_state(BatchState& st);

// Validates a batch and enqueues descriptor upload (through `slot`, under
// `slot_mutex` when given) plus the batched kernel on `stream`.  Nothing is
// touched before validation passes.  Shared by fsr_reconstruct_batched and
// the server.
fsr_status batched_enqueue(fsr_context* ctx, const fsr_image_desc* descs, int32_t n,
                           const fsr_params* params, const fsr_batch_schedule* schedule,
                           void* workspace, size_t ws_bytes, hipStream_t stream,
                           StagingSlot* slot, std::mutex* slot_mutex);

fsr_status set_error(fsr_status st, const char* msg);
fsr_status errorf(fsr_status st, const char* fmt, ...);
fsr_status hip_fail(hipError_t e, const char* what);
fsr_status validate_params(const fsr_params* p);
fsr_status check_supported(const fsr_params* p);
fsr_status validate_image(const float* image, const uint8_t* mask, const float* out, int32_t height,
                          int32_t width, int64_t stride, int32_t block);
fsr_status context_tables(fsr_context* ctx, int S, float rho, BlockTables* out, bool may_build = true);
int context_device(const fsr_context* ctx);
BatchState& context_batch(fsr_context* ctx);
std::mutex& context_mutex(fsr_context* ctx);
std::mutex& context_batch_mutex(fsr_context* ctx);   // guards the batch staging slot

}  // namespace fsr
