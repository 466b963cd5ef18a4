// fsr_internal.h -- declarations shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsr {

constexpr int kS = 32;            // support edge handled by these kernels
constexpr int kBins = kS * kS;    // 1024 frequency bins per block

// Device tables for one (S, rho) pair: the spatial weight rho^dist (Eq. 5
// before masking) and the frequency weight w_f (Eq. 9), both S x S,
// row-major, float32, and the DFT operands of the support size.
struct BlockTables {
    const float* rho_pow;   // [m * S + n]
    const float* freq_w;    // [k * S + l]
    // S < 32: F[m][k] = exp(-j 2 pi m k / S), S x S float2, exactly
    // conjugate-symmetric in k
    const float2* dft_sg;
    // DFT-matrix operands of the split-bf16 matrix-core transform in MFMA
    // lane order, bf16 bit patterns [part 2][q 2][term kMfmaMaxTerms][lane 64][8]
    const uint16_t* mfma_dft;
};

constexpr int kMfmaMaxTerms = 3;
constexpr int kMfmaDftElems = 2 * 2 * kMfmaMaxTerms * 64 * 8;

// One image of a reconstruction call.
struct ImageDesc {
    const float* image;
    const uint8_t* mask;
    float* out;
    uint16_t* argmax_log;   // nullable: n_blocks x iterations
    int32_t height, width;
    int64_t stride;
    int32_t iterations;
    int32_t nbx;            // blocks per row, ceil(width / B)
    int64_t block_begin;    // first global block id of this image (batched path)
};

struct PlainLaunch {
    ImageDesc img;
    int32_t block, border;  // B, L
    int32_t support;        // S = B + 2L: 32, or 8, 16, 24 (fsr_block_sg.h)
    float gamma;
    BlockTables tab;
    int64_t n_blocks;
    int32_t dft;            // 0: FP32 FFTs, 1: split-bf16 matrix products
    int32_t lds_argmax;     // 1: argmax reduced through an LDS tree (FP32 FFTs only)
};

hipError_t launch_plain(const PlainLaunch& p, hipStream_t stream);
// The reuse variant at S = 32 (fsr_reuse.hip): one launch per wavefront step
// over n_frames frames of p.img's size, frame_stride elements apart.
hipError_t launch_reuse(const PlainLaunch& p, float delta, int32_t n_frames, int64_t frame_stride,
                        hipStream_t stream);
int64_t reuse_steps(int32_t height, int32_t width, int32_t block, int32_t border);
hipError_t launch_plain_sg(const PlainLaunch& p, hipStream_t stream);   // S = 8, 16, 24

}  // namespace fsr
