// fsr_plain.hip -- one-image FSR: one workgroup of one wavefront per block.
#include "fsr_block.h"
#include "fsr_block_sg.h"

namespace fsr {

__device__ __forceinline__ BlockJob plain_job(const PlainLaunch& p, int64_t blk) {
    const ImageDesc& im = p.img;
    BlockJob jb;
    jb.image = global_ptr(im.image);
    jb.mask = global_ptr(im.mask);
    jb.out = global_ptr(im.out);
    jb.log = im.argmax_log ? global_ptr(im.argmax_log) + blk * (int64_t)im.iterations : nullptr;
    jb.height = im.height;
    jb.width = im.width;
    jb.stride = im.stride;
    jb.by = (int32_t)(blk / im.nbx);
    jb.bx = (int32_t)(blk % im.nbx);
    jb.iterations = im.iterations;
    return jb;
}

// Supports S = 8, 16, 24 (fsr_block_sg.h).
template <int S>
__global__ __launch_bounds__(64) void fsr_plain_sg(PlainLaunch p) {
    __shared__ __align__(16) float lds[SgShape<S>::kLdsFloats];
    const int64_t blk = xcd_contiguous(blockIdx.x, p.n_blocks);
    reconstruct_block_sg<S>(plain_job(p, blk), p.block, p.border, p.gamma, p.tab, lds);
}

template <int kDft, int kArgmax>
__global__ __launch_bounds__(64) void fsr_plain_s32(PlainLaunch p) {
    __shared__ __align__(16) float lds[kLdsFloats + (kArgmax == kArgmaxLds ? kArgmaxLdsFloats : 0)];
    const int64_t blk = xcd_contiguous(blockIdx.x, p.n_blocks);
    reconstruct_block<kDft, kArgmax, false>(plain_job(p, blk), p.block, p.border, p.gamma, p.tab, lds,
                                     reinterpret_cast<uint2*>(lds + kLdsFloats));
}

hipError_t launch_plain(const PlainLaunch& p, hipStream_t stream) {
    if (p.n_blocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)p.n_blocks), block(64);
    if (p.support != kS) {   // the host API admits FP32 FFTs and no flags here
        switch (p.support) {
        case 8: hipLaunchKernelGGL(fsr_plain_sg<8>, grid, block, 0, stream, p); break;
        case 16: hipLaunchKernelGGL(fsr_plain_sg<16>, grid, block, 0, stream, p); break;
        case 24: hipLaunchKernelGGL(fsr_plain_sg<24>, grid, block, 0, stream, p); break;
        default: return hipErrorInvalidValue;
        }
    } else if (p.lds_argmax) {
        if (p.dft != kDftFft32) return hipErrorInvalidValue;   // rejected by the host API first
        hipLaunchKernelGGL((fsr_plain_s32<kDftFft32, kArgmaxLds>), grid, block, 0, stream, p);
    } else if (p.dft == kDftSplitBf16) {
        hipLaunchKernelGGL((fsr_plain_s32<kDftSplitBf16, kArgmaxWave>), grid, block, 0, stream, p);
    } else {
        hipLaunchKernelGGL((fsr_plain_s32<kDftFft32, kArgmaxWave>), grid, block, 0, stream, p);
    }
    return hipGetLastError();
}

}  // namespace fsr
