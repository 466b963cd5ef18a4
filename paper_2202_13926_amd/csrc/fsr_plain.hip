// fsr_plain.hip -- one-image FSR: one workgroup of one wavefront per block.
#include "fsr_block.h"

namespace fsr {

template <int kDft>
__global__ __launch_bounds__(64) void fsr_plain_s32(PlainLaunch p) {
    __shared__ float lds[kLdsFloats];
    const int64_t blk = xcd_contiguous(blockIdx.x, p.n_blocks);
    const ImageDesc& im = p.img;
    BlockJob jb;
    jb.image = im.image;
    jb.mask = im.mask;
    jb.out = im.out;
    jb.log = im.argmax_log ? im.argmax_log + blk * (int64_t)im.iterations : nullptr;
    jb.height = im.height;
    jb.width = im.width;
    jb.stride = im.stride;
    jb.by = (int32_t)(blk / im.nbx);
    jb.bx = (int32_t)(blk % im.nbx);
    jb.iterations = im.iterations;
    reconstruct_block<kDft>(jb, p.block, p.border, p.gamma, p.tab, lds);
}

hipError_t launch_plain(const PlainLaunch& p, hipStream_t stream) {
    if (p.n_blocks <= 0) return hipSuccess;
    if (p.dft == kDftSplitBf16)
        hipLaunchKernelGGL(fsr_plain_s32<kDftSplitBf16>, dim3((unsigned)p.n_blocks), dim3(64), 0, stream, p);
    else
        hipLaunchKernelGGL(fsr_plain_s32<kDftFft32>, dim3((unsigned)p.n_blocks), dim3(64), 0, stream, p);
    return hipGetLastError();
}

}  // namespace fsr
