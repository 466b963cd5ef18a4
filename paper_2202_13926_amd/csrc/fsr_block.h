// fsr_block.h -- one support block of FSR on one wavefront (S = 32).
//
// Steps (Regensky et al., Sec. II and III-A):
//   gather     support tile at (by*B - L, bx*B - L); pixels outside the image
//              or masked out are unknown: f~ = 0, w = 0            (Eqs. 2, 5)
//   DFT        R_w = DFT2(f~ w), W = DFT2(w) (Eq. 7): one complex FFT of
//              both real tiles (in-register FFTs along the slot axis, an LDS
//              transpose between the passes) split into two exactly
//              Hermitian spectra; or two split-bf16 matrix-product transforms
//              on the matrix cores, each made Hermitian,
//              X <- (X + conj X[-k]) / 2
//   loop       I times: objective w_f |R_w|^2 (Eq. 16), wave argmax with
//              ties to the smaller bin, p = R_w[u,v] / W[0,0] (Eq. 10), model
//              update accumulated directly into the target pixels (Eq. 11
//              followed by the inverse DFT restricted to the target; a
//              compensated sum in the split-bf16 variant), residual
//              update R_w -= gamma p W[k-u, l-v] with cyclic indices
//              (Eqs. 12, 14-15)
//   compose    known target pixels copied, unknown ones take Re g
//
// LDS: 16 KiB per wavefront.  The weight spectrum W is stored with its 32
// rows duplicated (64 rows x 32 bins x float2) so that the rows a lane needs
// for its 16 bins, (k - u) mod 32 for k = 2s + h, form one contiguous run and
// every slot's address is the lane's base plus an immediate offset.  The
// same buffer first serves as the transpose scratch of the FFTs, or, in the
// matrix-core variant, holds the first spectrum (upper half) while the
// second is transformed.
#pragma once

#include <type_traits>

#include "fsr_device.h"
#include "fsr_internal.h"
#include "fsr_mfma.h"

namespace fsr {

// 2D DFT of the complex tile z = (zr, zi) (spatial layout) into the
// transpose planes: Z[k][l] at Planes::idx(k, l).  In-register FFTs along
// the slot axis, an LDS transpose between the passes.
__device__ __forceinline__ void dft2_complex_to_planes(float (&zr)[16], float (&zi)[16], float* lds,
                                                       int lane) {
    using P = Planes;
    const int c = lane & 31, h = lane >> 5;
    float* pr = P::re(lds);
    float* pi = P::im(lds);
    // pass 1: along m (rows of the tile) for every column n = c
    dft32_lane_pair(zr, zi, h);                 // slot k' -> bin row k = k' + 16h, column n = c
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        pr[P::idx(k + 16 * h, c)] = zr[k];
        pi[P::idx(k + 16 * h, c)] = zi[k];
    }
    wave_sync();
    // pass 2: along n for every k = c; slot s takes n = 2s + h
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        zr[s] = pr[P::idx(c, 2 * s + h)];
        zi[s] = pi[P::idx(c, 2 * s + h)];
    }
    wave_sync();
    dft32_lane_pair(zr, zi, h);                 // slot l' -> (k = c, l = l' + 16h)
#pragma unroll
    for (int l = 0; l < 16; ++l) {
        pr[P::idx(c, l + 16 * h)] = zr[l];
        pi[P::idx(c, l + 16 * h)] = zi[l];
    }
    wave_sync();
}

// Splits Z = F2{x + j s w} of two real tiles, left in the planes, into the
// bin layouts of X = F2{x} = (Z + conj Z[-k]) / 2 and
// W = F2{w} = (Z - conj Z[-k]) / (2 j s), with half_inv_s = 1 / (2 s) exact
// (s a power of two).  Bins k and -k read the same pair of values in swapped
// roles, so both spectra come out exactly Hermitian.
__device__ __forceinline__ void planes_split_two_real(float (&xr)[16], float (&xi)[16], float (&wr)[16],
                                                      float (&wi)[16], float half_inv_s, float* lds,
                                                      int lane) {
    using P = Planes;
    const int c = lane & 31, h = lane >> 5;
    const float* pr = P::re(lds);
    const float* pi = P::im(lds);
    const int lm = (kS - c) & 31;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int k = 2 * s + h, km = (kS - k) & 31;
        const float ar = pr[P::idx(k, c)], ai = pi[P::idx(k, c)];
        const float br = pr[P::idx(km, lm)], bi = pi[P::idx(km, lm)];
        xr[s] = 0.5f * (ar + br);
        xi[s] = 0.5f * (ai - bi);
        wr[s] = (ai + bi) * half_inv_s;
        wi[s] = (br - ar) * half_inv_s;
    }
    wave_sync();
}

// The FFT path takes the two real tiles x = (f~ - mu) w and w through one
// complex transform of z = x + j s w, with s the power of two at or below
// max |x| over the block: the scaling is exact and neither part is small
// beside the other (a transform's rounding is shared between the parts in
// proportion to their sizes).  Returns max |x| (wave-uniform) and s (1 when
// x = 0).
__device__ __forceinline__ float max_abs_and_scale(const float (&x)[16], float& scale) {
    uint32_t amax = 0;
#pragma unroll
    for (int s = 0; s < 16; s += 2) {
        const float m2 = fmaxf(fabsf(x[s]), fabsf(x[s + 1]));
        amax = umax(amax, __float_as_uint(m2));
    }
    amax = wave_max_u32(amax);
    const uint32_t sbits = amax & 0x7F800000u;
    scale = sbits ? __uint_as_float(sbits) : 1.0f;
    return __uint_as_float(amax);
}

// Everything a block needs to know about its image and the method.
struct BlockJob {
    const global_t<float>* image;
    const global_t<uint8_t>* mask;
    global_t<float>* out;
    global_t<uint16_t>* log;   // this block's I log entries, or nullptr
    int32_t height, width;
    int64_t stride;
    int32_t by, bx;
    int32_t iterations;
    // reuse variant only: weight factor of reused pixels (0 reuses nothing)
    float delta = 0.0f;
};

// Block `blk` of a one-image launch.
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

// kDft selects the forward transforms: kDftFft32 (FP32 FFTs on the vector
// ALUs) or kDftSplitBf16 (split-bf16 products on the matrix cores).
constexpr int kDftFft32 = 0;
constexpr int kDftSplitBf16 = 1;

// kArgmax selects the cross-bin reduction of the argmax: kArgmaxWave (each
// lane's 16 keys combined in registers, then DPP steps across the wavefront)
// or kArgmaxLds, the shared-memory scheme the paper compares against: all
// 1024 (key, bin) pairs are written to LDS and halved in a tree of ten
// LDS rounds.  Both pick the same bin (largest key, then smallest bin).
constexpr int kArgmaxWave = 0;
constexpr int kArgmaxLds = 1;
constexpr int kArgmaxLdsFloats = 2 * kBins;   // (key, bin) pairs, 8 KiB

// Pair order of the LDS tree: larger key, then smaller bin.
__device__ __forceinline__ uint2 better_pair(uint2 a, uint2 b) {
    return (b.x > a.x || (b.x == a.x && b.y < a.y)) ? b : a;
}

// kPersistent: the caller loops over blocks (the persistent batched
// kernel).  Its per-block values are then made opaque, so that the compiler
// does not hoist the table loads and lane constants out of the caller's loop
// and keep them live across every block.
// kReuse: the sequential variant (the original FSR that Sec. II departs
// from).  A support pixel that is missing but lies in the target of a block
// earlier in raster order takes part with its reconstruction, read from
// jb.out, and the weight jb.delta rho^dist; the caller guarantees that those
// blocks have finished.
template <int kDft, int kArgmax, bool kPersistent, bool kReuse = false>
__device__ __forceinline__ void reconstruct_block(const BlockJob& jb, int B, int L, float gamma,
                                                  const BlockTables& tab_in, float* lds,
                                                  uint2* argmax_lds = nullptr) {
    const int lane = kPersistent ? opaque((int)(threadIdx.x & 63)) : (int)(threadIdx.x & 63);
    BlockTables tab = tab_in;
    if constexpr (kPersistent) {
        tab.rho_pow = opaque_ptr(tab_in.rho_pow);
        tab.freq_w = opaque_ptr(tab_in.freq_w);
        if constexpr (kDft == kDftSplitBf16) tab.mfma_dft = opaque_ptr(tab_in.mfma_dft);
    }
    const int c = lane & 31, h = lane >> 5;
    const int y0 = jb.by * B - L, x0 = jb.bx * B - L;

    // ---- gather and weighting: pixel (m, n) = (2s + h, c), or
    // (mfma_tile_row(s, h), c) for the matrix-core transform
    float xr[16], wr[16];   // f~ first, then (f~ - mu) w
    uint64_t any_known = 0;
    const int x = x0 + c;
    const bool xin = (unsigned)x < (unsigned)jb.width;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int m = kDft == kDftSplitBf16 ? mfma_tile_row(s, h) : 2 * s + h, y = y0 + m;
        const bool in = xin && (unsigned)y < (unsigned)jb.height;
        // out-of-image lanes load pixel 0 (always valid) and discard it
        const int64_t off = in ? (int64_t)y * jb.stride + x : 0;
        const uint8_t kraw = jb.mask[off];
        const float fraw = jb.image[off];
        const float rp = global_ptr(tab.rho_pow)[m * kS + c];
        const uint8_t k = in ? kraw : (uint8_t)0;
        const float f = fraw;
        const float w = k ? rp : 0.0f;
        if constexpr (kReuse) {
            // earlier targets: the rows above this target, and this target's
            // rows left of it
            const bool earlier = m < L || (m < L + B && c < L);
            const bool reused = in && !k && earlier && jb.delta > 0.0f;
            any_known |= ballot(k != 0 || reused);
            xr[s] = k ? f : reused ? (float)jb.out[off] : 0.0f;
            wr[s] = reused ? jb.delta * rp : w;
        } else {
            any_known |= ballot(k != 0);
            xr[s] = k ? f : 0.0f;
            wr[s] = w;
        }
    }

    // ---- target pixel owned by this lane (lanes 0 .. B*B-1)
    const int ti = lane / B, tj = lane - (lane / B) * B;
    const int tm = L + ti, tn = L + tj;
    float acc = 0.0f;
    // running compensation of acc (Kahan), kept by the precision variant
    float acc_comp = 0.0f;
    const int iters = jb.iterations;

    if (any_known != 0) {
        // ---- forward DFTs (R in registers, W to LDS).  R_w = DFT2(f~ w) is
        // evaluated as mu W + DFT2((f~ - mu) w) with mu the weighted mean of
        // the known support pixels: the same value in exact arithmetic, but
        // the rounding error of the large mean component becomes a multiple
        // of the very W that the iterations subtract, and the transformed
        // remainder is small.
        float sx = 0.0f, sw = 0.0f;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            sx = fmaf(xr[s], wr[s], sx);
            sw += wr[s];
        }
        sx = wave_sum_f32(sx);
        sw = wave_sum_f32(sw);
        const float mu = sw > 0.0f ? sx / sw : 0.0f;
#pragma unroll
        for (int s = 0; s < 16; ++s) xr[s] = (xr[s] - mu) * wr[s];
        float xi[16], wi[16];
        if constexpr (kDft == kDftSplitBf16) {
            // two real transforms; the first spectrum waits in LDS while the
            // second is computed.  (The one-transform split used below for
            // the FFTs does not suit the matrix cores: there Z[k] and
            // conj Z[-k] of a purely imaginary input do not cancel exactly,
            // measured up to 2^-21 of max w, which leaks W's rounding into X.)
            const bf16x8* fop = reinterpret_cast<const bf16x8*>(tab.mfma_dft);
            dft2_real_mfma(xr, xi, fop, lane);
            float2* pk = park(lds);
#pragma unroll
            for (int s = 0; s < 16; ++s) pk[64 * s + lane] = make_float2(xr[s], xi[s]);
            wave_sync();
            dft2_real_mfma(wr, wi, fop, lane);
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const float2 v = pk[64 * s + lane];
                xr[s] = v.x;
                xi[s] = v.y;
            }
            wave_sync();
        } else {
            // both real tiles in one complex FFT: z = x + j s w
            float scale;
            const float xmax = max_abs_and_scale(xr, scale);
#pragma unroll
            for (int s = 0; s < 16; ++s) xi[s] = wr[s] * scale;
            dft2_complex_to_planes(xr, xi, lds, lane);
            planes_split_two_real(xr, xi, wr, wi, 0.5f / scale, lds, lane);
            if (xmax == 0.0f) {
                // a support whose known pixels all equal mu (a flat or
                // clipped region): X is exactly 0, and no rounding of the w
                // part may leak into it (with mu = 0 it would be all of R_w)
#pragma unroll
                for (int s = 0; s < 16; ++s) xr[s] = xi[s] = 0.0f;
            }
        }
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            xr[s] = fmaf(mu, wr[s], xr[s]);
            xi[s] = fmaf(mu, wi[s], xi[s]);
        }
        // W itself, not gamma W / W[0,0]: a per-bin rounding of the table
        // would not cancel against R_w where R_w is proportional to W (a
        // support with one known pixel), and as R_w shrinks the error of the
        // early iterations would take over the argmax
        float2* wtab = reinterpret_cast<float2*>(lds);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int k = 2 * s + h;
            wtab[k * kS + c] = make_float2(wr[s], wi[s]);
            wtab[(k + kS) * kS + c] = make_float2(wr[s], wi[s]);
        }
        const float w00 = readlane_f(wr[0], 0);
        const float gi = w00 > 0.0f ? gamma / w00 : 0.0f;
        float wf[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) wf[s] = global_ptr(tab.freq_w)[(2 * s + h) * kS + c];
        // lane i of tw_re/tw_im holds t32[i & 31] for the target model's
        // phases; ds_bpermute reads lane (address / 4) mod 64, so the byte
        // address 4 q needs no reduction mod 32
        const int tw_re = opaque(__float_as_int(kTw.re[c])), tw_im = opaque(__float_as_int(kTw.im[c]));
        // the loads of the loop's constants complete here, not at their first
        // use inside the loop (which would put their waits in the loop body)
#pragma unroll
        for (int s = 0; s < 16; ++s) wf[s] = __int_as_float(opaque(__float_as_int(wf[s])));
        // loop-invariant lane constants: the target pixel's (4 m, 4 n) packed
        // for the phase's bpermute byte address 4 (u m + v n), and the LDS
        // byte offset 256 h + 8 c of the lane's entry (h, c) in W
        const int tmn4 = opaque((4 * tm) | ((4 * tn) << 16));
        const int hc8 = opaque(256 * h + 8 * c);
        wave_sync();

        // the residual spectrum lives in two 16-wide vectors during the
        // loop: one contiguous register tuple each, which the indexed read
        // of the winning bin needs (as separate floats the allocator may
        // scatter them and then copy them into a tuple every iteration)
        f32x16 vr, vi;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            vr[s] = xr[s];
            vi[s] = xi[s];
        }

        // the loop comes in two copies, with and without the argmax log, so
        // that the one without carries no per-iteration branch for it
        auto iterate = [&](auto with_log) {
            for (int it = 0; it < iters; ++it) {
                // objective (Eq. 16) as an argmax key: the IEEE bits of the
                // non-negative float32 objective (so unsigned order is float
                // order) with the 4 lowest mantissa bits replaced by 15 - slot.
                // Objectives that agree to 2^-19 relative tie, and ties go to the
                // smaller slot, then (below) to the lower lane: the smaller bin.
                int idx;
                if constexpr (kArgmax == kArgmaxWave) {
                    uint32_t lmax = 0;
#pragma unroll
                    for (int s = 0; s < 16; ++s) {
                        const float e = fmaf(vr[s], vr[s], vi[s] * vi[s]);
                        const uint32_t key = (__float_as_uint(e * wf[s]) & 0xFFFFFFF0u) | (uint32_t)(15 - s);
                        lmax = umax(lmax, key);
                    }
                    const uint32_t mx = wave_max_u32(lmax);
                    const int ln = (int)__builtin_ctzll(ballot(lmax == mx));
                    idx = 64 * (15 - (int)(mx & 15u)) + ln;
                } else {
#pragma unroll
                    for (int s = 0; s < 16; ++s) {
                        const float e = fmaf(vr[s], vr[s], vi[s] * vi[s]);
                        const uint32_t key = (__float_as_uint(e * wf[s]) & 0xFFFFFFF0u) | (uint32_t)(15 - s);
                        argmax_lds[64 * s + lane] = make_uint2(key, (uint32_t)(64 * s + lane));
                    }
                    wave_sync();
                    // halve 1024 -> 64 entries, each lane owning entries lane + 64 j
#pragma unroll
                    for (int half = kBins / 2; half >= 64; half >>= 1) {
#pragma unroll
                        for (int j = 0; j < half / 64; ++j) {
                            const int e = lane + 64 * j;
                            argmax_lds[e] = better_pair(argmax_lds[e], argmax_lds[e + half]);
                        }
                        wave_sync();
                    }
                    // 64 -> 1 with a shrinking set of lanes
#pragma unroll
                    for (int half = 32; half >= 1; half >>= 1) {
                        if (lane < half) argmax_lds[lane] = better_pair(argmax_lds[lane], argmax_lds[lane + half]);
                        wave_sync();
                    }
                    idx = __builtin_amdgcn_readfirstlane((int)argmax_lds[0].y);
                    wave_sync();   // the next iteration overwrites the pairs
                }
                const int slot = idx >> 6, ln = idx & 63;
                const float pr = readlane_f(vr[slot], ln);
                const float pim = readlane_f(vi[slot], ln);
                const int u = idx >> 5, v = idx & 31;
                const float cr = gi * pr, ci = gi * pim;    // gamma * p (Eqs. 10-11)
                if constexpr (decltype(with_log)::value) {
                    if (lane == 0) jb.log[it] = (uint16_t)idx;
                }

                // residual: R_w[k,l] -= gamma p W[(k-u) mod S, (l-v) mod S]; slot s
                // reads duplicated row h + 32 - u + 2s (rows 1 .. 63 of the
                // table), column (c - v) mod 32: byte offset 256 (h + 32 - u) +
                // 8 ((c - v) mod 32) + 512 s.  All sixteen reads go out before
                // the model's lane exchange and are waited for together: issued
                // a pair at a time behind the exchange (the compiler's order
                // otherwise), their latency showed through the 2.5 wavefronts
                // per SIMD that the table's LDS leaves, 3.75 against 3.48 ms
                // per 1080p frame
                const int woff = sub_low_byte(hc8 + (8192 - 256 * u), 8 * v);
                const float2* wrow = reinterpret_cast<const float2*>(
                    reinterpret_cast<const char*>(wtab) + woff);
                float2 wv[16];
#pragma unroll
                for (int s = 0; s < 16; ++s) wv[s] = wrow[64 * s];
                // model: g += gamma p exp(+j 2 pi (u m + v n) / S) on the target
                const int q4 = dot2_u16(u | (v << 16), tmn4);
                const float er = __int_as_float(__builtin_amdgcn_ds_bpermute(q4, tw_re));
                const float ei = __int_as_float(__builtin_amdgcn_ds_bpermute(q4, tw_im));
                if constexpr (kDft == kDftSplitBf16) {
                    // compensated sum of the I model terms
                    const float y = fmaf(cr, er, ci * ei) - acc_comp;
                    const float t = acc + y;
                    acc_comp = (t - acc) - y;
                    acc = t;
                } else {
                    acc = fmaf(cr, er, acc);
                    acc = fmaf(ci, ei, acc);
                }

#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    const float2 w = wv[s];
                    vr[s] = fmaf(-cr, w.x, vr[s]);
                    vr[s] = fmaf(ci, w.y, vr[s]);
                    vi[s] = fmaf(-cr, w.y, vi[s]);
                    vi[s] = fmaf(-ci, w.x, vi[s]);
                }
            }
        };
        if (jb.log != nullptr) iterate(std::true_type{});
        else iterate(std::false_type{});
        wave_sync();   // the LDS is reused by the next block of a persistent wave
    } else if (jb.log != nullptr) {
        for (int it = lane; it < iters; it += 64) jb.log[it] = (uint16_t)0xFFFF;
    }

    // ---- compose (Sec. II): known pixels copied, unknown pixels Re g
    if (lane < B * B) {
        const int y = jb.by * B + ti, xx = jb.bx * B + tj;
        if (y < jb.height && xx < jb.width) {
            const int64_t off = (int64_t)y * jb.stride + xx;
            const uint8_t k = jb.mask[off];
            jb.out[off] = k ? jb.image[off] : acc - acc_comp;
        }
    }
}

}  // namespace fsr
