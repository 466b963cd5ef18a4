// fsr_plain_sg.hip -- one-image FSR at supports 8, 16 and 24
// (fsr_block_sg.h): one workgroup of one wavefront per block.
#include "fsr_block.h"
#include "fsr_block_sg.h"

namespace fsr {

template <int S>
__global__ __launch_bounds__(64) void fsr_plain_sg(PlainLaunch p) {
    __shared__ __align__(16) float lds[SgShape<S>::kLdsFloats];
    const int64_t blk = xcd_contiguous(blockIdx.x, p.n_blocks);
    reconstruct_block_sg<S>(plain_job(p, blk), p.block, p.border, p.gamma, p.tab, lds);
}

// The host API admits FP32 DFTs and no flags at these supports.
hipError_t launch_plain_sg(const PlainLaunch& p, hipStream_t stream) {
    if (p.n_blocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)p.n_blocks), block(64);
    switch (p.support) {
    case 8: hipLaunchKernelGGL(fsr_plain_sg<8>, grid, block, 0, stream, p); break;
    case 16: hipLaunchKernelGGL(fsr_plain_sg<16>, grid, block, 0, stream, p); break;
    case 24: hipLaunchKernelGGL(fsr_plain_sg<24>, grid, block, 0, stream, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fsr
