// fsr_batched.hip -- many images of different sizes and iteration counts in
// one launch.  Blocks of all images form one index space in queue order
// (heaviest images first); wavefronts either take one block each (chunk 0,
// a plain grid) or run persistently, popping `chunk` consecutive blocks at a
// time from a global counter until the index space is exhausted.  Each block
// runs exactly the same routine as the one-image kernel, so its result does
// not depend on the batch it is part of.
#include "fsr_block.h"

namespace fsr {

__global__ void fsr_queue_reset(unsigned* counter) {
    if (threadIdx.x == 0) *counter = 0u;
}

__device__ __forceinline__ void batch_block(const BatchLaunch& p, int64_t g, float* lds) {
    // last image whose first block is <= g (descriptors sorted by block_begin)
    int lo = 0, hi = p.n_images - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.descs[mid].block_begin <= g) lo = mid;
        else hi = mid - 1;
    }
    const DevDesc& d = p.descs[lo];
    const int64_t local = g - d.block_begin;
    BlockJob jb;
    jb.image = d.image;
    jb.mask = d.mask;
    jb.out = d.out;
    jb.log = d.argmax_log ? d.argmax_log + local * (int64_t)d.iterations : nullptr;
    jb.height = d.height;
    jb.width = d.width;
    jb.stride = d.stride;
    jb.by = (int32_t)(local / d.nbx);
    jb.bx = (int32_t)(local % d.nbx);
    jb.iterations = d.iterations;
    reconstruct_block(jb, p.block, p.border, p.gamma, p.tab, lds);
}

template <int kWaves>
__global__ __launch_bounds__(64 * kWaves) void fsr_batched_s32(BatchLaunch p) {
    __shared__ float lds[kWaves * kLdsFloats];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    float* mine = lds + wave * kLdsFloats;
    // [next, end): blocks this wavefront still owns.  Without a queue a
    // wavefront owns exactly one block; with one it refills from the queue.
    int64_t next = 0, end = 0;
    if (p.chunk <= 0) {
        const int64_t groups = (p.total_blocks + kWaves - 1) / kWaves;
        next = xcd_contiguous(blockIdx.x, groups) * kWaves + wave;
        end = next < p.total_blocks ? next + 1 : next;
    }
    for (;;) {
        if (next >= end) {
            if (p.chunk <= 0) break;
            unsigned start = 0;
            if (lane == 0) start = atomicAdd(p.counter, (unsigned)p.chunk);
            start = __builtin_amdgcn_readfirstlane(start);
            if ((int64_t)start >= p.total_blocks) break;   // every wavefront ends here
            next = start;
            end = next + p.chunk;
            if (end > p.total_blocks) end = p.total_blocks;
        }
        batch_block(p, next, mine);
        ++next;
    }
}

hipError_t launch_batched(const BatchLaunch& p, int waves_per_group, int64_t groups,
                          hipStream_t stream) {
    if (p.total_blocks <= 0) return hipSuccess;
    if (p.chunk > 0) {
        hipLaunchKernelGGL(fsr_queue_reset, dim3(1), dim3(64), 0, stream, p.counter);
    } else {
        groups = (p.total_blocks + waves_per_group - 1) / waves_per_group;
    }
    const dim3 grid((unsigned)groups), block(64 * waves_per_group);
    switch (waves_per_group) {
    case 1: hipLaunchKernelGGL(fsr_batched_s32<1>, grid, block, 0, stream, p); break;
    case 2: hipLaunchKernelGGL(fsr_batched_s32<2>, grid, block, 0, stream, p); break;
    case 4: hipLaunchKernelGGL(fsr_batched_s32<4>, grid, block, 0, stream, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fsr
