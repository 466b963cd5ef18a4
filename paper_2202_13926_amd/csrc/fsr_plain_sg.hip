// fsr_plain_sg.hip -- one-image FSR at supports 8, 16 and 24: one workgroup
// of one wavefront per block (fsr_block_sg.h; at S = 24 fsr_block_s24.h), or
// at S = 8 with B <= 4 eight blocks per wavefront (fsr_block_multi.h; bitwise
// the result of the one-block routine).
#include "fsr_block.h"
#include "fsr_block_multi.h"
#include "fsr_block_s24.h"
#include "fsr_block_sg.h"

namespace fsr {

template <int S, int kArgmax = kArgmaxWave>
__global__ __launch_bounds__(64) void fsr_plain_sg(PlainLaunch p) {
    constexpr int kExtra = kArgmax == kArgmaxLds ? 2 * sg_argmax_pairs<S>() : 0;
    __shared__ __align__(16) float lds[SgShape<S>::kLdsFloats + kExtra];
    const int64_t blk = xcd_contiguous(blockIdx.x, p.n_blocks);
    reconstruct_block_sg<S, false, kArgmax>(plain_job(p, blk), p.block, p.border, p.gamma, p.tab, lds,
                                            reinterpret_cast<uint2*>(lds + SgShape<S>::kLdsFloats));
}

template <int kArgmax = kArgmaxWave>
__global__ __launch_bounds__(64) void fsr_plain_s24(PlainLaunch p) {
    constexpr int kExtra = kArgmax == kArgmaxLds ? 2 * S24::kArgmaxPairs : 0;
    __shared__ __align__(16) float lds[S24::kLdsFloats + kExtra];
    const int64_t blk = xcd_contiguous(blockIdx.x, p.n_blocks);
    reconstruct_block_s24<false, kArgmax>(plain_job(p, blk), p.block, p.border, p.gamma, p.tab, lds,
                                          reinterpret_cast<uint2*>(lds + S24::kLdsFloats));
}

template <int S, int T>
__global__ __launch_bounds__(64) void fsr_plain_multi(PlainLaunch p) {
    __shared__ __align__(16) float lds[MultiShape<S, T>::kLdsFloats];
    constexpr int NB = MultiShape<S, T>::NB;
    const int64_t waves = (p.n_blocks + NB - 1) / NB;
    const ImageDesc& im = p.img;
    MultiJob jb;
    jb.image = im.image;
    jb.mask = im.mask;
    jb.out = im.out;
    jb.argmax_log = im.argmax_log;
    jb.height = im.height;
    jb.width = im.width;
    jb.stride = im.stride;
    jb.iterations = im.iterations;
    jb.nbx = im.nbx;
    jb.first_block = xcd_contiguous(blockIdx.x, waves) * NB;
    jb.n_blocks = p.n_blocks;
    reconstruct_multi<S, T>(jb, p.block, p.border, p.gamma, p.tab, lds);
}

template <int S, int T>
static hipError_t launch_multi(const PlainLaunch& p, hipStream_t stream) {
    const int64_t waves = (p.n_blocks + MultiShape<S, T>::NB - 1) / MultiShape<S, T>::NB;
    hipLaunchKernelGGL((fsr_plain_multi<S, T>), dim3((unsigned)waves), dim3(64), 0, stream, p);
    return hipGetLastError();
}

// The host API admits FP32 DFTs at these supports, and of the flags the
// LDS argmax, which always runs one block per wavefront.
hipError_t launch_plain_sg(const PlainLaunch& p, hipStream_t stream) {
    if (p.n_blocks <= 0) return hipSuccess;
    if (p.lds_argmax) {
        const dim3 grid((unsigned)p.n_blocks), block(64);
        switch (p.support) {
        case 8: hipLaunchKernelGGL((fsr_plain_sg<8, kArgmaxLds>), grid, block, 0, stream, p); break;
        case 16: hipLaunchKernelGGL((fsr_plain_sg<16, kArgmaxLds>), grid, block, 0, stream, p); break;
        case 24: hipLaunchKernelGGL((fsr_plain_s24<kArgmaxLds>), grid, block, 0, stream, p); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int bb = p.block * p.block;   // target pixels per block
    if (p.support == 8 && bb <= 8) return launch_multi<8, 1>(p, stream);
    if (p.support == 8 && bb <= 16) return launch_multi<8, 2>(p, stream);
    const dim3 grid((unsigned)p.n_blocks), block(64);
    switch (p.support) {
    case 8: hipLaunchKernelGGL(fsr_plain_sg<8>, grid, block, 0, stream, p); break;
    case 16: hipLaunchKernelGGL(fsr_plain_sg<16>, grid, block, 0, stream, p); break;
    case 24: hipLaunchKernelGGL(fsr_plain_s24<>, grid, block, 0, stream, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fsr
