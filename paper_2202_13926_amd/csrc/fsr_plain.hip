// fsr_plain.hip -- one-image FSR at S = 32: one workgroup of one wavefront
// per block.  Supports 8, 16 and 24 are in fsr_plain_sg.hip.
#include "fsr_block.h"

namespace fsr {

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
    if (p.support != kS) return launch_plain_sg(p, stream);
    if (p.lds_argmax) {
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
