// fsr_reuse.hip -- the sequential variant that reuses reconstructed pixels
// (the original FSR that Sec. II departs from), at S = 32.
//
// The variant is defined by raster order: block (by, bx) sees the
// reconstructions of every earlier block whose target meets its support.
// With r = ceil(L / B) those are the blocks of rows by - r .. by - 1 and
// columns bx - r .. bx + r, and those of row by and columns bx - r .. bx - 1.
// Giving block (by, bx) the step t = bx + (r + 1) by puts every such block
// at a smaller step, and two blocks of one step lie at least r + 1 block
// columns apart, so that neither's target meets the other's support.  One
// launch per step (a wavefront schedule) therefore gives exactly the raster
// result, with the stream's order between launches as the only
// synchronisation.  Frames of one size are independent: one launch per step
// takes that step's blocks of every frame.
#include <algorithm>

#include "fsr_block.h"
#include "fsr_block_split4.h"

namespace fsr {

// Blocks (by, step - slope * by) for by = by_lo + blockIdx.x of frame
// blockIdx.y; the host sizes the grid so that every bx lies in [0, nbx).
// Frame f's image, mask and output start f * frame_stride elements after
// frame 0's, its argmax log (if any) f * log_stride entries after.
__global__ __launch_bounds__(64) void fsr_reuse_s32(PlainLaunch p, float delta, int32_t step,
                                                    int32_t by_lo, int32_t slope, int64_t frame_stride,
                                                    int64_t log_stride) {
    __shared__ __align__(16) float lds[kLdsFloats];
    const int by = by_lo + (int)blockIdx.x;
    const int bx = step - slope * by;
    const int64_t f = blockIdx.y;
    BlockJob jb = plain_job(p, (int64_t)by * p.img.nbx + bx);
    jb.image += f * frame_stride;
    jb.mask += f * frame_stride;
    jb.out += f * frame_stride;
    if (jb.log != nullptr) jb.log += f * log_stride;
    jb.delta = delta;
    reconstruct_block<kDftFft32, kArgmaxWave, false, true>(jb, p.block, p.border, p.gamma, p.tab, lds);
}

// The same blocks with four wavefronts each (fsr_block_split4.h), for steps
// too small to fill the device; bitwise the same result.
__global__ __launch_bounds__(256) void fsr_reuse_split4_s32(PlainLaunch p, float delta, int32_t step,
                                                            int32_t by_lo, int32_t slope, int64_t frame_stride,
                                                            int64_t log_stride) {
    __shared__ __align__(16) float lds[kLdsFloats];
    __shared__ Split4Lds sh;
    const int by = by_lo + (int)blockIdx.x;
    const int bx = step - slope * by;
    const int64_t f = blockIdx.y;
    BlockJob jb = plain_job(p, (int64_t)by * p.img.nbx + bx);
    jb.image += f * frame_stride;
    jb.mask += f * frame_stride;
    jb.out += f * frame_stride;
    if (jb.log != nullptr) jb.log += f * log_stride;
    jb.delta = delta;
    reconstruct_block_reuse_split4(jb, p.block, p.border, p.gamma, p.tab, lds, sh);
}

// Steps with at most this many blocks (over all frames) run four wavefronts
// per block.  Measured on 1080p frames (at most 96 blocks per step and
// frame), ms per call of 1 / 2 / 3 / 4 / 8 frames: one wavefront per block
// 105.4 / 105.8 / 107.5 / 108.1 / 108.8; four for every step 92.0 / 92.0 /
// 97.8 / 99.1 / 110.7.
constexpr int64_t kSplit4MaxBlocks = 512;

int64_t reuse_steps(int32_t height, int32_t width, int32_t block, int32_t border) {
    const int64_t nby = (height + block - 1) / block, nbx = (width + block - 1) / block;
    const int64_t slope = (border + block - 1) / block + 1;
    return (nbx - 1) + slope * (nby - 1) + 1;
}

hipError_t launch_reuse(const PlainLaunch& p, float delta, int32_t n_frames, int64_t frame_stride,
                        hipStream_t stream) {
    const int32_t B = p.block;
    const int64_t nbx = p.img.nbx, nby = (p.img.height + B - 1) / B;
    const int64_t slope = (p.border + B - 1) / B + 1;
    const int64_t steps = reuse_steps(p.img.height, p.img.width, B, p.border);
    const int64_t log_stride = p.n_blocks * (int64_t)p.img.iterations;
    for (int64_t t = 0; t < steps; ++t) {
        // by in [ceil((t - (nbx - 1)) / slope), floor(t / slope)] within [0, nby)
        const int64_t over = t - (nbx - 1);
        const int64_t lo = over > 0 ? (over + slope - 1) / slope : 0;
        const int64_t hi = std::min<int64_t>(nby - 1, t / slope);
        if (hi < lo) continue;   // no block at this step (possible when slope > nbx)
        const dim3 grid((unsigned)(hi - lo + 1), (unsigned)n_frames);
        if ((hi - lo + 1) * (int64_t)n_frames <= kSplit4MaxBlocks)
            hipLaunchKernelGGL(fsr_reuse_split4_s32, grid, dim3(256), 0, stream, p, delta, (int32_t)t,
                               (int32_t)lo, (int32_t)slope, frame_stride, log_stride);
        else
            hipLaunchKernelGGL(fsr_reuse_s32, grid, dim3(64), 0, stream, p, delta, (int32_t)t, (int32_t)lo,
                               (int32_t)slope, frame_stride, log_stride);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace fsr
