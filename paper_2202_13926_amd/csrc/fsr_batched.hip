// fsr_batched.hip -- many images of different sizes and iteration counts in
// one launch.  Blocks of all images form one index space in queue order
// (heaviest images first); wavefronts either take one block each (chunk 0,
// a plain grid: fsr_batched_grid_s32) or run persistently, popping `chunk`
// consecutive blocks at a time from a global counter until the index space
// is exhausted (fsr_batched_s32).  Supports 8, 16 and 24 have the same two
// forms (fsr_batched_grid_sg, fsr_batched_sg); at S = 8 with B <= 4 a
// wavefront takes units of eight blocks of one image (fsr_batched_grid_multi,
// fsr_batched_multi), every image's block range then being padded to a
// multiple of eight.  Each block runs the same arithmetic as in the one-image
// kernel, so its result does not depend on the batch it is part of.
#include "fsr_batch_internal.h"
#include "fsr_block.h"
#include "fsr_block_multi.h"
#include "fsr_block_s24.h"
#include "fsr_block_sg.h"

#include <mutex>

namespace fsr {

// The fixed workspace of fsr_reconstruct_batched_noalloc (queue head, then
// descriptors).  Host code never passes this name to a kernel: it stands for
// a host-side shadow; the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace {
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxStaticDevices] = {};
}  // namespace

hipError_t static_workspace_init(int device) {
    if (device < 0 || device >= kMaxStaticDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_static_ptr[device] = ptr;
    return hipSuccess;
}

void* static_workspace(int device) {
    if (device < 0 || device >= kMaxStaticDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_static_mu);
    return g_static_ptr[device];
}

__global__ void fsr_queue_reset(unsigned* counter) {
    if (threadIdx.x == 0) *counter = 0u;
}

struct DescChunk {
    DevDesc d[kDescsPerKernel];
};

// Thread t < n writes descriptor t (64 bytes as four 16-byte stores).
__global__ __launch_bounds__(64) void fsr_write_descs(DescChunk c, DevDesc* dst, int n) {
    const int t = threadIdx.x;
    if (t >= n) return;
    const uint4* s = reinterpret_cast<const uint4*>(&c.d[t]);
    uint4* o = reinterpret_cast<uint4*>(dst + t);
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = s[i];
}

hipError_t launch_write_descs(const DevDesc* table, int n, DevDesc* dst, hipStream_t stream) {
    if (n < 0 || n > kDescKernelMax) return hipErrorInvalidValue;
    for (int first = 0; first < n; first += kDescsPerKernel) {
        const int m = n - first < kDescsPerKernel ? n - first : kDescsPerKernel;
        DescChunk c{};
        for (int i = 0; i < m; ++i) c.d[i] = table[first + i];
        hipLaunchKernelGGL(fsr_write_descs, dim3(1), dim3(64), 0, stream, c, dst + first, m);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Row y of the region in blockIdx.y-strided passes; 16-byte words where the
// region's width, pitches and addresses allow, else bytes.  Workgroups of
// one wavefront: while another kernel keeps every compute unit busy, a
// workgroup of several wavefronts waits for that many free slots on one
// compute unit, in practice for the other kernel to drain.
template <typename W>
__global__ __launch_bounds__(64) void fsr_copy2d(char* dst, size_t dst_pitch, const char* src, size_t src_pitch,
                                                  size_t words, size_t height) {
    for (size_t y = blockIdx.y; y < height; y += gridDim.y) {
        W* d = reinterpret_cast<W*>(dst + y * dst_pitch);
        const W* s = reinterpret_cast<const W*>(src + y * src_pitch);
        for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
            d[i] = s[i];
    }
}

hipError_t launch_copy2d(void* dst, size_t dst_pitch, const void* src, size_t src_pitch, size_t width_bytes,
                         size_t height, hipStream_t stream) {
    if (width_bytes == 0 || height == 0) return hipSuccess;
    const bool wide = (width_bytes % 16 == 0) && (dst_pitch % 16 == 0) && (src_pitch % 16 == 0) &&
                      ((uintptr_t)dst % 16 == 0) && ((uintptr_t)src % 16 == 0);
    const size_t words = wide ? width_bytes / 16 : width_bytes;
    const unsigned gx = (unsigned)((words + 63) / 64 < 64 ? (words + 63) / 64 : 64);
    const unsigned gy = (unsigned)(height < 4096 ? height : 4096);
    if (wide)
        hipLaunchKernelGGL(fsr_copy2d<uint4>, dim3(gx, gy), dim3(64), 0, stream, static_cast<char*>(dst),
                           dst_pitch, static_cast<const char*>(src), src_pitch, words, height);
    else
        hipLaunchKernelGGL(fsr_copy2d<uint8_t>, dim3(gx, gy), dim3(64), 0, stream, static_cast<char*>(dst),
                           dst_pitch, static_cast<const char*>(src), src_pitch, words, height);
    return hipGetLastError();
}

// Image of global block g: the cached one when g still lies in [begin, end),
// else a binary search over the descriptors (sorted by block_begin).
__device__ __forceinline__ void locate(const BatchLaunch& p, int64_t g, int& img, int64_t& begin,
                                       int64_t& end) {
    if (g >= begin && g < end) return;
    int lo = 0, hi = p.n_images - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.descs[mid].block_begin <= g) lo = mid;
        else hi = mid - 1;
    }
    img = lo;
    begin = p.descs[lo].block_begin;
    end = lo + 1 < p.n_images ? p.descs[lo + 1].block_begin : p.total_blocks;
}

__device__ __forceinline__ BlockJob batch_job(const BatchLaunch& p, int64_t g, int img) {
    const DevDesc& d = p.descs[img];
    const int64_t local = g - d.block_begin;
    BlockJob jb;
    jb.image = global_ptr(d.image);
    jb.mask = global_ptr(d.mask);
    jb.out = global_ptr(d.out);
    jb.log = d.argmax_log ? global_ptr(d.argmax_log) + local * (int64_t)d.iterations : nullptr;
    jb.height = d.height;
    jb.width = d.width;
    jb.stride = d.stride;
    jb.by = (int32_t)(local / d.nbx);
    jb.bx = (int32_t)(local % d.nbx);
    jb.iterations = d.iterations;
    return jb;
}

// Block routine of support S: the S = 32 routine in its DFT mode, or the
// smaller-support one (FP32 DFTs).
template <int S, int kDft, bool kPersistent>
__device__ __forceinline__ void batch_block(const BatchLaunch& p, int64_t g, int img, float* lds) {
    if constexpr (S == kS)
        reconstruct_block<kDft, kArgmaxWave, kPersistent>(batch_job(p, g, img), p.block, p.border,
                                                          p.gamma, p.tab, lds);
    else if constexpr (S == S24::S)
        reconstruct_block_s24<kPersistent>(batch_job(p, g, img), p.block, p.border, p.gamma, p.tab, lds);
    else
        reconstruct_block_sg<S, kPersistent>(batch_job(p, g, img), p.block, p.border, p.gamma, p.tab, lds);
}

template <int S>
constexpr int lds_floats_of() {
    if constexpr (S == kS) return kLdsFloats;
    else if constexpr (S == S24::S) return S24::kLdsFloats;
    else return SgShape<S>::kLdsFloats;
}

// Plain grid (chunk 0): one block per wavefront, no loop, so the block
// routine runs in its one-block form (padded planes, both spectra in
// registers), as in the one-image kernel.
template <int kWaves, int S, int kDft>
__device__ __forceinline__ void grid_body(const BatchLaunch& p, float* lds) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t groups = (p.total_blocks + kWaves - 1) / kWaves;
    const int64_t g = xcd_contiguous(blockIdx.x, groups) * kWaves + wave;
    if (g >= p.total_blocks) return;
    int img = 0;
    int64_t img_begin = 0, img_end = 0;
    locate(p, g, img, img_begin, img_end);
    batch_block<S, kDft, false>(p, g, img, lds + wave * lds_floats_of<S>());
}

// Persistent (chunk > 0): wavefronts pop `chunk` blocks at a time.
template <int kWaves, int S, int kDft>
__device__ __forceinline__ void queue_body(const BatchLaunch& p, float* lds) {
    // wave-uniform by construction; readfirstlane lets the compiler see it,
    // so block indices and descriptors stay in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    float* mine = lds + wave * lds_floats_of<S>();
    // [next, end): blocks this wavefront still owns; refilled from the queue
    int64_t next = 0, end = 0;
    int img = 0;
    int64_t img_begin = 0, img_end = 0;   // empty: the first block searches
    for (;;) {
        if (next >= end) {
            unsigned start = 0;
            if (lane == 0) start = atomicAdd(p.counter, (unsigned)p.chunk);
            start = __builtin_amdgcn_readfirstlane(start);
            if ((int64_t)start >= p.total_blocks) break;   // every wavefront ends here
            next = start;
            end = next + p.chunk;
            if (end > p.total_blocks) end = p.total_blocks;
        }
        locate(p, next, img, img_begin, img_end);
        batch_block<S, kDft, true>(p, next, img, mine);
        ++next;
    }
}

template <int kWaves, int kDft>
__global__ __launch_bounds__(64 * kWaves) void fsr_batched_grid_s32(BatchLaunch p) {
    __shared__ __align__(16) float lds[kWaves * kLdsFloats];
    grid_body<kWaves, kS, kDft>(p, lds);
}

template <int kWaves, int kDft>
__global__ __launch_bounds__(64 * kWaves) void fsr_batched_s32(BatchLaunch p) {
    __shared__ __align__(16) float lds[kWaves * kLdsFloats];
    queue_body<kWaves, kS, kDft>(p, lds);
}

template <int kWaves, int S>
__global__ __launch_bounds__(64 * kWaves) void fsr_batched_grid_sg(BatchLaunch p) {
    __shared__ __align__(16) float lds[kWaves * lds_floats_of<S>()];
    grid_body<kWaves, S, kDftFft32>(p, lds);
}

template <int kWaves, int S>
__global__ __launch_bounds__(64 * kWaves) void fsr_batched_sg(BatchLaunch p) {
    __shared__ __align__(16) float lds[kWaves * lds_floats_of<S>()];
    queue_body<kWaves, S, kDftFft32>(p, lds);
}

// ---- S = 8, B <= 4: units of eight blocks of one image
__device__ __forceinline__ MultiJob batch_multi_job(const BatchLaunch& p, int64_t g, int img) {
    const DevDesc& d = p.descs[img];
    MultiJob jb;
    jb.image = d.image;
    jb.mask = d.mask;
    jb.out = d.out;
    jb.argmax_log = d.argmax_log;
    jb.height = d.height;
    jb.width = d.width;
    jb.stride = d.stride;
    jb.iterations = d.iterations;
    jb.nbx = d.nbx;
    jb.first_block = g - d.block_begin;
    jb.n_blocks = (int64_t)((d.height + p.block - 1) / p.block) * d.nbx;
    return jb;
}

template <int kWaves, int T>
__global__ __launch_bounds__(64 * kWaves) void fsr_batched_grid_multi(BatchLaunch p) {
    constexpr int kUnit = MultiShape<8, T>::NB;
    __shared__ __align__(16) float lds[kWaves * MultiShape<8, T>::kLdsFloats];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t units = p.total_blocks / kUnit;
    const int64_t groups = (units + kWaves - 1) / kWaves;
    const int64_t unit = xcd_contiguous(blockIdx.x, groups) * kWaves + wave;
    if (unit >= units) return;
    const int64_t g = unit * kUnit;
    int img = 0;
    int64_t img_begin = 0, img_end = 0;
    locate(p, g, img, img_begin, img_end);
    reconstruct_multi<8, T>(batch_multi_job(p, g, img), p.block, p.border, p.gamma, p.tab,
                            lds + wave * MultiShape<8, T>::kLdsFloats);
}

template <int kWaves, int T>
__global__ __launch_bounds__(64 * kWaves) void fsr_batched_multi(BatchLaunch p) {
    constexpr int kUnit = MultiShape<8, T>::NB;
    __shared__ __align__(16) float lds[kWaves * MultiShape<8, T>::kLdsFloats];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    float* mine = lds + wave * MultiShape<8, T>::kLdsFloats;
    const int64_t units = p.total_blocks / kUnit;
    int64_t next = 0, end = 0;   // units this wavefront still owns
    int img = 0;
    int64_t img_begin = 0, img_end = 0;
    for (;;) {
        if (next >= end) {
            unsigned start = 0;
            if (lane == 0) start = atomicAdd(p.counter, (unsigned)p.chunk);
            start = __builtin_amdgcn_readfirstlane(start);
            if ((int64_t)start >= units) break;   // every wavefront ends here
            next = start;
            end = next + p.chunk;
            if (end > units) end = units;
        }
        const int64_t g = next * kUnit;
        locate(p, g, img, img_begin, img_end);
        reconstruct_multi<8, T, true>(batch_multi_job(p, g, img), p.block, p.border, p.gamma, p.tab, mine);
        ++next;
    }
}

template <int T>
static hipError_t launch_waves_multi(const BatchLaunch& p, int waves_per_group, dim3 grid, dim3 block,
                                     hipStream_t stream) {
    const bool queue = p.chunk > 0;
    switch (waves_per_group) {
    case 1:
        if (queue) hipLaunchKernelGGL((fsr_batched_multi<1, T>), grid, block, 0, stream, p);
        else hipLaunchKernelGGL((fsr_batched_grid_multi<1, T>), grid, block, 0, stream, p);
        break;
    case 2:
        if (queue) hipLaunchKernelGGL((fsr_batched_multi<2, T>), grid, block, 0, stream, p);
        else hipLaunchKernelGGL((fsr_batched_grid_multi<2, T>), grid, block, 0, stream, p);
        break;
    case 4:
        if (queue) hipLaunchKernelGGL((fsr_batched_multi<4, T>), grid, block, 0, stream, p);
        else hipLaunchKernelGGL((fsr_batched_grid_multi<4, T>), grid, block, 0, stream, p);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int kDft>
static hipError_t launch_waves(const BatchLaunch& p, int waves_per_group, dim3 grid, dim3 block,
                               hipStream_t stream) {
    const bool queue = p.chunk > 0;
    switch (waves_per_group) {
    case 1:
        if (queue) hipLaunchKernelGGL((fsr_batched_s32<1, kDft>), grid, block, 0, stream, p);
        else hipLaunchKernelGGL((fsr_batched_grid_s32<1, kDft>), grid, block, 0, stream, p);
        break;
    case 2:
        if (queue) hipLaunchKernelGGL((fsr_batched_s32<2, kDft>), grid, block, 0, stream, p);
        else hipLaunchKernelGGL((fsr_batched_grid_s32<2, kDft>), grid, block, 0, stream, p);
        break;
    case 4:
        if (queue) hipLaunchKernelGGL((fsr_batched_s32<4, kDft>), grid, block, 0, stream, p);
        else hipLaunchKernelGGL((fsr_batched_grid_s32<4, kDft>), grid, block, 0, stream, p);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int S>
static hipError_t launch_waves_sg(const BatchLaunch& p, int waves_per_group, dim3 grid, dim3 block,
                                  hipStream_t stream) {
    const bool queue = p.chunk > 0;
    switch (waves_per_group) {
    case 1:
        if (queue) hipLaunchKernelGGL((fsr_batched_sg<1, S>), grid, block, 0, stream, p);
        else hipLaunchKernelGGL((fsr_batched_grid_sg<1, S>), grid, block, 0, stream, p);
        break;
    case 2:
        if (queue) hipLaunchKernelGGL((fsr_batched_sg<2, S>), grid, block, 0, stream, p);
        else hipLaunchKernelGGL((fsr_batched_grid_sg<2, S>), grid, block, 0, stream, p);
        break;
    case 4:
        if (queue) hipLaunchKernelGGL((fsr_batched_sg<4, S>), grid, block, 0, stream, p);
        else hipLaunchKernelGGL((fsr_batched_grid_sg<4, S>), grid, block, 0, stream, p);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename K>
static hipError_t resident(K kernel, int waves_per_group, int* groups) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(groups, kernel, 64 * waves_per_group, 0);
}

template <int kWaves>
static hipError_t resident_of(const BatchLaunch& p, int* groups) {
    if (p.unit == 8) {
        if (p.block * p.block <= 8) return resident(fsr_batched_multi<kWaves, 1>, kWaves, groups);
        return resident(fsr_batched_multi<kWaves, 2>, kWaves, groups);
    }
    switch (p.support) {
    case 8: return resident(fsr_batched_sg<kWaves, 8>, kWaves, groups);
    case 16: return resident(fsr_batched_sg<kWaves, 16>, kWaves, groups);
    case 24: return resident(fsr_batched_sg<kWaves, 24>, kWaves, groups);
    case kS:
        if (p.dft == kDftSplitBf16) return resident(fsr_batched_s32<kWaves, kDftSplitBf16>, kWaves, groups);
        return resident(fsr_batched_s32<kWaves, kDftFft32>, kWaves, groups);
    default: return hipErrorInvalidValue;
    }
}

hipError_t batched_resident_groups(const BatchLaunch& p, int waves_per_group, int* groups) {
    switch (waves_per_group) {
    case 1: return resident_of<1>(p, groups);
    case 2: return resident_of<2>(p, groups);
    case 4: return resident_of<4>(p, groups);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batched(const BatchLaunch& p, int waves_per_group, int64_t groups,
                          hipStream_t stream) {
    if (p.total_blocks <= 0) return hipSuccess;
    if (p.unit != 1 && p.unit != 8) return hipErrorInvalidValue;
    if (p.chunk > 0) {
        hipLaunchKernelGGL(fsr_queue_reset, dim3(1), dim3(64), 0, stream, p.counter);
    } else {
        const int64_t units = p.total_blocks / p.unit;
        groups = (units + waves_per_group - 1) / waves_per_group;
    }
    const dim3 grid((unsigned)groups), block(64 * waves_per_group);
    if (p.unit == 8) {
        if (p.block * p.block <= 8) return launch_waves_multi<1>(p, waves_per_group, grid, block, stream);
        return launch_waves_multi<2>(p, waves_per_group, grid, block, stream);
    }
    switch (p.support) {
    case kS: break;
    case 8: return launch_waves_sg<8>(p, waves_per_group, grid, block, stream);
    case 16: return launch_waves_sg<16>(p, waves_per_group, grid, block, stream);
    case 24: return launch_waves_sg<24>(p, waves_per_group, grid, block, stream);
    default: return hipErrorInvalidValue;
    }
    if (p.dft == kDftSplitBf16) return launch_waves<kDftSplitBf16>(p, waves_per_group, grid, block, stream);
    return launch_waves<kDftFft32>(p, waves_per_group, grid, block, stream);
}

}  // namespace fsr
