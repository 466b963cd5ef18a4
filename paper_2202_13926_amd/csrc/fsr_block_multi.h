// fsr_block_multi.h -- eight support blocks of FSR per wavefront at the
// support S = 8 (Sec. II; the paper sweeps S from 8 to 32).
//
// With one block per wavefront (fsr_block_sg.h) the per-iteration work that
// does not grow with the number of bins -- the cross-lane argmax, reading the
// winner back, the model update and the addressing -- is shared by the
// S^2 / 64 = 1 bin of a lane at S = 8.  Here a wavefront holds NB = 64 / S
// blocks: block b owns lanes [b S, b S + S), lane c of it holds column c of
// the support in S slots (slot s: pixel row m = s, bin (k = s, l = c)), and
// every cross-lane step runs within the S lanes of one block, for all NB
// blocks in the same instructions.  (At S = 16 the same layout, four blocks
// per wavefront, needs 16 KiB of W tables per wavefront and ran slower than
// one block per wavefront: 2.5 against 7 resident wavefronts per SIMD.)
//
// Every block runs the arithmetic of the one-block routine operation for
// operation, so the two give bitwise the same output and argmax log (the
// batched path keeps the one-block routine):
//  - the weighted mean is summed in the one-block routine's order: there it
//    is a pairwise tree over the lanes c + S h of per-lane partials over the
//    slots; here per-row-group partials, the same DPP tree over the S lanes
//    of the block, then the tree over h in registers (float addition is
//    commutative, so the direction of each DPP step does not matter);
//  - the direct DFT sums run over the same operands in the same order;
//  - the key of bin (k, l) carries the slot code 15 - k instead of
//    15 - (k div G) with ties left to the lane order: both select the
//    largest objective and, among equal keys, the smallest index k S + l.
//
// Target pixels: pixel p < B^2 of a block (row p / B, column p % B) belongs
// to lane p % S of the block, accumulator p / S (T = ceil(B^2 / S)).
//
// LDS per wavefront: the DFT table (S^2 float2) and per block the tile, then
// the first DFT pass (S^2 float2); during the iterations per block W with
// duplicated rows (2S x S float2), over the same space, the blocks' rows
// interleaved.  One read takes a row of S entries for each block, at the
// block's own u; with the tables one after another a row of 16 words starts
// at a bank that depends on u alone, so blocks whose u agree mod 4 collide,
// while interleaved the block decides the bank (0.317 against 0.335 ms for
// the 1080p frame at I = 100, the same output).
#pragma once

#include "fsr_block.h"
#include "fsr_block_sg.h"

namespace fsr {

template <int S, int T>
struct MultiShape {
    static_assert(S == 8, "several blocks per wavefront at S = 8");
    static_assert(T >= 1 && T * S <= 64, "target pixels per lane");
    static constexpr int NB = 64 / S;             // blocks per wavefront
    static constexpr int G1 = SgShape<S>::G;      // lane groups of the one-block layout
    static constexpr int NS1 = SgShape<S>::NS;    // its slots per lane
    static constexpr int kTabFloats = 2 * S * S;             // DFT table F[m][k]
    static constexpr int kBlockScratch = 2 * S * S;          // tile, then first pass [k][n]
    // blocks' scratch areas 8 words apart beyond their size, so that the
    // eight blocks' rows of one access start at banks 8 b (a multiple of 64
    // words apart, every block's row fell on the same 8 or 16 banks): the
    // same output, 0.33 against 0.34 ms for the 1080p frame at I = 100
    static constexpr int kScratchPitch = kBlockScratch + 8;
    static constexpr int kWFloats = NB * 4 * S * S;          // W per block, 2S x S float2
    static constexpr int kLdsFloats = kTabFloats + NB * kScratchPitch > kWFloats
                                          ? kTabFloats + NB * kScratchPitch : kWFloats;
};

// Maximum and sum over the 8 lanes of this lane's block; every lane of the
// block gets the result.  The sum pairs lanes as the first three steps of
// wave_sum_f32 do.
template <int S>
__device__ __forceinline__ uint32_t block_max_u32(uint32_t v) {
    static_assert(S == 8, "half-row steps");
    v = umax(v, dpp_u32<0xB1>(v));          // quad_perm [1,0,3,2]
    v = umax(v, dpp_u32<0x4E>(v));          // quad_perm [2,3,0,1]
    v = umax(v, dpp_u32<0x141>(v));         // row_half_mirror
    return v;
}

template <int S>
__device__ __forceinline__ float block_sum_f32(float v) {
    static_assert(S == 8, "half-row steps");
    v += dpp_f32_or_zero<0xB1>(v);
    v += dpp_f32_or_zero<0x4E>(v);
    v += dpp_f32_or_zero<0x141>(v);
    return v;
}

// a * b + c on the full-rate 24-bit multiplier, all per-lane values below 2^24
__device__ __forceinline__ int mad_u24_lanes(int a, int b, int c) {
    int r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// The S bits of a wave-wide ballot that belong to the block starting at lane
// `first`.
template <int S>
__device__ __forceinline__ uint32_t block_bits(uint64_t m, int first) {
    const uint32_t half = first < 32 ? (uint32_t)m : (uint32_t)(m >> 32);
    return (half >> (first & 31)) & ((1u << S) - 1u);
}

// 2D DFT of this lane's column v (slot m = pixel row m) into (re, im) (slot
// k = bin row k), as the one-block routine computes it: the first pass along
// m per column against the table, the second along n across the block's
// lanes through LDS.  `tile` is this block's scratch (2 S^2 floats).
template <int S>
__device__ __forceinline__ void dft2_multi(const float (&v)[S], float (&re)[S], float (&im)[S],
                                           const float2* ftab, float* tile, int c) {
    float2* pass1 = reinterpret_cast<float2*>(tile);   // [k][n], after the tile is read
#pragma unroll
    for (int m = 0; m < S; ++m) tile[m * S + c] = v[m];
    wave_sync();
    float ar[S], ai[S];
#pragma unroll
    for (int k = 0; k < S; ++k) ar[k] = ai[k] = 0.0f;
#pragma unroll 2
    for (int m = 0; m < S; ++m) {
        const float x = tile[m * S + c];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const float2 f = ftab[m * S + k];
            ar[k] = fmaf(x, f.x, ar[k]);
            ai[k] = fmaf(x, f.y, ai[k]);
        }
    }
    wave_sync();   // every lane has read the tile
#pragma unroll
    for (int k = 0; k < S; ++k) pass1[k * S + c] = make_float2(ar[k], ai[k]);
    wave_sync();
    float br[S], bi[S];
#pragma unroll
    for (int k = 0; k < S; ++k) br[k] = bi[k] = 0.0f;
#pragma unroll 2
    for (int n = 0; n < S; ++n) {
        const float2 f = ftab[n * S + c];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const float2 a = pass1[k * S + n];
            br[k] = fmaf(a.x, f.x, br[k]);
            br[k] = fmaf(-a.y, f.y, br[k]);
            bi[k] = fmaf(a.x, f.y, bi[k]);
            bi[k] = fmaf(a.y, f.x, bi[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
        re[k] = br[k];
        im[k] = bi[k];
    }
    wave_sync();   // the scratch is reused by the caller
}

// This lane's residual at slot u (u is uniform within each block): a select
// tree on the bits of u, as bit blends under opaque masks (written as
// selects, the compiler turns it into an indexed read of the registers
// spilled to scratch).
template <int S>
__device__ __forceinline__ void residual_at(const float (&xr)[S], const float (&xi)[S], int u, float& tr,
                                            float& ti) {
    static_assert(S == 8, "three levels");
    const uint32_t m0 = (uint32_t)opaque(-(u & 1)), m1 = (uint32_t)opaque(-((u >> 1) & 1)),
                   m2 = (uint32_t)opaque(-((u >> 2) & 1));
    float r4[4], i4[4], r2[2], i2[2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        r4[j] = blend(m0, xr[2 * j + 1], xr[2 * j]);
        i4[j] = blend(m0, xi[2 * j + 1], xi[2 * j]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        r2[j] = blend(m1, r4[2 * j + 1], r4[2 * j]);
        i2[j] = blend(m1, i4[2 * j + 1], i4[2 * j]);
    }
    tr = blend(m2, r2[1], r2[0]);
    ti = blend(m2, i2[1], i2[0]);
}

// Up to eight consecutive blocks of one image: blocks first_block ..
// first_block + 7 that lie below n_blocks (the others idle and write
// nothing).
struct MultiJob {
    const float* image;
    const uint8_t* mask;
    float* out;
    uint16_t* argmax_log;   // nullable: n_blocks x iterations for the image
    int32_t height, width;
    int64_t stride;
    int32_t iterations;
    int32_t nbx;            // blocks per row
    int64_t first_block;
    int64_t n_blocks;
};

// kPersistent: the caller loops over units of eight blocks; as in the other
// block routines the lane index and table pointers are then made opaque.
template <int S, int T, bool kPersistent = false>
__device__ __forceinline__ void reconstruct_multi(const MultiJob& im, int B, int L, float gamma,
                                                  const BlockTables& tab_in, float* lds) {
    using Sh = MultiShape<S, T>;
    constexpr int NB = Sh::NB, G1 = Sh::G1, NS1 = Sh::NS1;
    const int lane = kPersistent ? opaque((int)(threadIdx.x & 63)) : (int)(threadIdx.x & 63);
    BlockTables tab = tab_in;
    if constexpr (kPersistent) {
        tab.rho_pow = opaque_ptr(tab_in.rho_pow);
        tab.freq_w = opaque_ptr(tab_in.freq_w);
        tab.dft_sg = opaque_ptr(tab_in.dft_sg);
    }
    const int b = lane / S, c = lane % S, first = b * S;
    const int64_t blk = im.first_block + b;
    const bool valid = blk < im.n_blocks;
    const int32_t blk32 = valid ? (int32_t)blk : 0;   // block counts are below 2^31
    const int by = blk32 / im.nbx, bx = blk32 - by * im.nbx;
    const int y0 = by * B - L, x0 = bx * B - L;
    const global_t<const float>* image = global_ptr(im.image);
    const global_t<const uint8_t>* mask = global_ptr(im.mask);
    global_t<float>* out = global_ptr(im.out);
    global_t<uint16_t>* logp =
        im.argmax_log && valid ? global_ptr(im.argmax_log) + blk * (int64_t)im.iterations : nullptr;
    float2* ftab = reinterpret_cast<float2*>(lds);
    float* scratch = lds + Sh::kTabFloats + b * Sh::kScratchPitch;

    // ---- DFT table into LDS (the same for every block)
    {
        const global_t<const uint64_t>* src = global_ptr(reinterpret_cast<const uint64_t*>(tab.dft_sg));
        uint64_t* dst = reinterpret_cast<uint64_t*>(ftab);
        for (int i = lane; i < S * S; i += 64) dst[i] = src[i];
    }

    // ---- gather and weighting: slot s holds pixel (s, c)
    float xr[S], wr[S];
    uint32_t known_here = 0;
    const int x = x0 + c;
    const bool xin = valid && (unsigned)x < (unsigned)im.width;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int y = y0 + s;
        const bool in = xin && (unsigned)y < (unsigned)im.height;
        const int64_t off = in ? (int64_t)y * im.stride + x : 0;
        const uint8_t kraw = mask[off];
        const float fraw = image[off];
        const float rp = global_ptr(tab.rho_pow)[s * S + c];
        const uint8_t k = in ? kraw : (uint8_t)0;
        known_here |= k;
        xr[s] = k ? fraw : 0.0f;
        wr[s] = k ? rp : 0.0f;
    }
    const bool has_known = block_bits<S>(ballot(known_here != 0), first) != 0;

    // ---- target pixels of this lane
    float acc[T];
    int tm4[T], tn4[T];
    bool own[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int px = c + S * t;
        own[t] = px < B * B;
        const int ti = own[t] ? px / B : 0, tj = own[t] ? px - (px / B) * B : 0;
        tm4[t] = opaque(4 * (L + ti));
        tn4[t] = opaque(4 * (L + tj));
        acc[t] = 0.0f;
    }
    const int iters = im.iterations;
    wave_sync();   // DFT table written

    // ---- R_w = mu W + DFT2((f~ - mu) w), mu summed in the one-block order
    float sxh[G1], swh[G1];
#pragma unroll
    for (int h = 0; h < G1; ++h) {
        float sx = 0.0f, sw = 0.0f;
#pragma unroll
        for (int s1 = 0; s1 < NS1; ++s1) {
            const int m = G1 * s1 + h;
            sx = fmaf(xr[m], wr[m], sx);
            sw += wr[m];
        }
        sxh[h] = block_sum_f32<S>(sx);
        swh[h] = block_sum_f32<S>(sw);
    }
    // pairwise over h: level j adds entry h + 2^j into entry h
#pragma unroll
    for (int j = 0; (1 << j) < G1; ++j) {
#pragma unroll
        for (int h = 0; h < G1; h += 2 << j) {
            sxh[h] = sxh[h] + sxh[h + (1 << j)];
            swh[h] = swh[h] + swh[h + (1 << j)];
        }
    }
    const float mu = swh[0] > 0.0f ? sxh[0] / swh[0] : 0.0f;
#pragma unroll
    for (int s = 0; s < S; ++s) xr[s] = (xr[s] - mu) * wr[s];
    float xi[S], wi[S];
    dft2_multi<S>(xr, xr, xi, ftab, scratch, c);
    dft2_multi<S>(wr, wr, wi, ftab, scratch, c);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        xr[s] = fmaf(mu, wr[s], xr[s]);
        xi[s] = fmaf(mu, wi[s], xi[s]);
    }
    // W[0][0] of this block lives on its first lane, slot 0
    const float w00 = __int_as_float(__builtin_amdgcn_ds_bpermute(4 * first, __float_as_int(wr[0])));
    const float gi = w00 > 0.0f ? gamma / w00 : 0.0f;
    float wf[S];
#pragma unroll
    for (int s = 0; s < S; ++s) wf[s] = global_ptr(tab.freq_w)[s * S + c];
    // lane c of each block holds F[1][c] = exp(-j 2 pi c / S), read before W
    // overwrites the table
    const float2 tw = ftab[S + c];
    const int tw_re = __float_as_int(tw.x), tw_im = __float_as_int(tw.y);
    // the loads of the loop's constants complete here, not at their first
    // use inside the loop (which would put their waits in the loop body)
#pragma unroll
    for (int s = 0; s < S; ++s) wf[s] = __int_as_float(opaque(__float_as_int(wf[s])));
    wave_sync();
    // W with duplicated rows: entry (R, C) of block b holds W[R mod S][C],
    // at (R NB + b) S + C: the rows of the blocks interleaved, so that one
    // read (a row per block, each at its own u) spreads over the banks by b
    float2* wtab = reinterpret_cast<float2*>(lds) + b * S;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const float2 wv = make_float2(wr[s], wi[s]);
        wtab[s * NB * S + c] = wv;
        wtab[(s + S) * NB * S + c] = wv;
    }
    const char* wbytes = reinterpret_cast<const char*>(lds);
    const int wb = opaque(8 * b * S);   // byte offset of this block's rows
    const int first4 = opaque(4 * first);
    wave_sync();

    // the loop comes in two copies, with and without the argmax log, so that
    // the one without carries no per-iteration branch for it
    auto iterate = [&](auto with_log) {
        for (int it = 0; it < iters; ++it) {
            // objective key (Eq. 16): float32 bits, the 4 low mantissa bits
            // replaced by 15 - k
            uint32_t lmax = 0;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const float e = fmaf(xr[s], xr[s], xi[s] * xi[s]);
                const uint32_t key = (__float_as_uint(e * wf[s]) & 0xFFFFFFF0u) | (uint32_t)(15 - s);
                lmax = umax(lmax, key);
            }
            const uint32_t mx = block_max_u32<S>(lmax);
            const int v = __builtin_ctz(block_bits<S>(ballot(lmax == mx), first));   // winner's lane
            const int u = 15 - (int)(mx & 15u);                                       // and row
            float tr, ti;
            residual_at<S>(xr, xi, u, tr, ti);
            const int src = first4 + 4 * v;
            const float pr = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(tr)));
            const float pim = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(ti)));
            const float cr = gi * pr, ci = gi * pim;    // gamma * p (Eqs. 10-11)
            if constexpr (decltype(with_log)::value) {
                if (logp != nullptr && c == 0) logp[it] = has_known ? (uint16_t)(u * S + v) : (uint16_t)0xFFFF;
            }

            // model: g += gamma p exp(+j 2 pi (u m + v n) / S) on the target
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const int q4 = mad_u24_lanes(u, tm4[t], mad_u24_lanes(v, tn4[t], 0)) & (4 * S - 1);
                const float er = __int_as_float(__builtin_amdgcn_ds_bpermute(first4 + q4, tw_re));
                const float ei = __int_as_float(__builtin_amdgcn_ds_bpermute(first4 + q4, tw_im));
                acc[t] = fmaf(cr, er, acc[t]);
                acc[t] = fmaf(ci, ei, acc[t]);
            }

            // residual (Eqs. 12, 14-15): bin (s, c) reads entry (s - u + S,
            // (c - v) mod S) of its block's table
            const float2* wrow = reinterpret_cast<const float2*>(
                wbytes + wb + 8 * ((S - u) * NB * S + ((c - v) & (S - 1))));
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const float2 w = wrow[NB * S * s];
                xr[s] = fmaf(-cr, w.x, xr[s]);
                xr[s] = fmaf(ci, w.y, xr[s]);
                xi[s] = fmaf(-cr, w.y, xi[s]);
                xi[s] = fmaf(-ci, w.x, xi[s]);
            }
        }
    };
    if (im.argmax_log != nullptr) iterate(std::true_type{});
    else iterate(std::false_type{});

    // ---- compose (Sec. II): known pixels copied, unknown pixels Re g
#pragma unroll
    for (int t = 0; t < T; ++t) {
        if (!(own[t] && valid)) continue;
        const int px = c + S * t;
        const int y = by * B + px / B, xx = bx * B + (px - (px / B) * B);
        if (y < im.height && xx < im.width) {
            const int64_t off = (int64_t)y * im.stride + xx;
            const uint8_t k = mask[off];
            out[off] = k ? image[off] : acc[t];
        }
    }
}

}  // namespace fsr
