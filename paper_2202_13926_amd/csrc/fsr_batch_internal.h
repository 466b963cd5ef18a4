// fsr_batch_internal.h -- declarations of the batched path shared by its
// host runtime and its kernels.
#pragma once

#include "fsr.h"
#include "fsr_internal.h"

namespace fsr {

// Device-side descriptor of one image of a batch (64 bytes).  Images are
// stored in queue order; block_begin is the prefix sum of block counts.
struct DevDesc {
    const float* image;
    const uint8_t* mask;
    float* out;
    uint16_t* argmax_log;
    int64_t stride;
    int64_t block_begin;
    int32_t height, width;
    int32_t iterations;
    int32_t nbx;
};
static_assert(sizeof(DevDesc) == 64, "descriptor layout");

struct BatchLaunch {
    const DevDesc* descs;   // device, n_images entries
    unsigned* counter;      // device queue head (reset before every launch)
    int64_t total_blocks;
    int32_t n_images;
    int32_t chunk;          // blocks per queue pop; 0 = one wavefront per block, no queue
    int32_t block, border;
    int32_t support;        // S = B + 2L: 32, or 8, 16, 24 (FP32 DFTs only)
    float gamma;
    BlockTables tab;
    int32_t dft;            // 0: FP32 FFTs, 1: split-bf16 matrix products
    int32_t unit;           // blocks per wavefront: 1, or 8 (S = 8, B <= 4);
                            // every image's block range is a multiple of it,
                            // and chunk counts units
};

// Blocks per wavefront of the batched kernels for these parameters.
inline int32_t batch_unit(int32_t support, int32_t block) {
    return support == 8 && block * block <= 16 ? 8 : 1;
}

// Launches the queue reset (when chunk > 0) and the batched kernel with
// `waves_per_group` wavefronts per workgroup and `groups` workgroups
// (persistent mode) on `stream`.
hipError_t launch_batched(const BatchLaunch& p, int waves_per_group, int64_t groups,
                          hipStream_t stream);

// Device copies written by kernels rather than by the runtime's copy
// commands: on this runtime a copy enqueued on one stream does not start
// while a kernel of another stream runs, whereas kernels of different
// streams share the device.  Keeping the launch path of a batch free of
// copies lets a small batch run beside a large one.
constexpr int kDescsPerKernel = 16;    // descriptors carried by one kernel's arguments
constexpr int kDescKernelMax = 64;     // larger tables go through a pinned copy

// Bytes of a batch workspace ahead of its descriptor table: the queue head,
// padded.
constexpr size_t kQueueCtrlBytes = 256;

// The fixed workspace of fsr_reconstruct_batched_noalloc: a device array of
// the library (one copy per device) holding the queue head and the
// descriptors of at most kStaticImages images.
constexpr int kStaticImages = FSR_NOALLOC_MAX_IMAGES;
constexpr size_t kStaticWorkspaceBytes = kQueueCtrlBytes + kStaticImages * sizeof(DevDesc);
static_assert(kStaticImages <= kDescKernelMax, "the descriptors of a fixed-workspace batch travel by kernel");

// Looks up the device address of that array on `device`, which the caller
// has made current, once per device (later calls return at once).
hipError_t static_workspace_init(int device);

// That address on `device`, or nullptr if static_workspace_init has not
// succeeded there.
void* static_workspace(int device);

// Writes the n <= kDescKernelMax descriptors of `table` to `dst` (device)
// with kernels on `stream`.
hipError_t launch_write_descs(const DevDesc* table, int n, DevDesc* dst, hipStream_t stream);

// Copies a height x width_bytes region between pitched buffers that the
// device can address (device memory, or pinned host memory) with a kernel.
hipError_t launch_copy2d(void* dst, size_t dst_pitch, const void* src, size_t src_pitch, size_t width_bytes,
                         size_t height, hipStream_t stream);

// Workgroups of `waves_per_group` wavefronts that one compute unit holds at
// once in the persistent batched kernel for p.support and p.dft (register
// and LDS limits, from the HIP occupancy calculator).
hipError_t batched_resident_groups(const BatchLaunch& p, int waves_per_group, int* groups);

}  // namespace fsr
