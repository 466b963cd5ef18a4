// fsr_runtime.h -- host runtime pieces shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>

#include "fsr.h"
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

// Per-context state of the batched path: pinned staging for descriptor
// uploads, the event that marks the last upload as consumed, the device's
// compute-unit count and the schedules chosen by the autotuner.
struct BatchState {
    void* staging = nullptr;
    size_t staging_bytes = 0;
    hipEvent_t staging_done = nullptr;
    int cu_count = 0;
    std::map<uint64_t, fsr_batch_schedule> tuned;
};

void release_batch_state(BatchState& st);

fsr_status set_error(fsr_status st, const char* msg);
fsr_status errorf(fsr_status st, const char* fmt, ...);
fsr_status hip_fail(hipError_t e, const char* what);
fsr_status validate_params(const fsr_params* p);
fsr_status check_supported(const fsr_params* p);
fsr_status validate_image(const float* image, const uint8_t* mask, const float* out, int32_t height,
                          int32_t width, int64_t stride, int32_t block);
fsr_status context_tables(fsr_context* ctx, float rho, BlockTables* out);
int context_device(const fsr_context* ctx);
BatchState& context_batch(fsr_context* ctx);
std::mutex& context_mutex(fsr_context* ctx);

}  // namespace fsr
