// fsr_block_split4.h -- one S = 32 support block of the sequential variant
// (the original FSR that Sec. II departs from) on four wavefronts.
//
// The variant runs one launch per wavefront step of its schedule, and a step
// holds at most a few hundred blocks: with one wavefront per block most
// SIMDs idle and each block's time is the latency of one wavefront alone.
// Here a workgroup of four wavefronts takes one block.  Wavefront 0 runs
// the gather, the mean split and the forward transforms exactly as
// fsr_block.h does (kDftFft32, kReuse), then parks bins of slots 4..15 and
// the W table in LDS; wavefront q keeps slots 4q .. 4q + 3 (bins
// (2s + h, c)) for the iterations.  Per iteration each wavefront reduces its
// own 256 keys (same keys, same tie codes 15 - s) to a candidate (key,
// lane, R_w at the winner), the four candidates meet in LDS behind one
// workgroup barrier (double-buffered, so one barrier per iteration
// suffices), and every wavefront takes the largest: the same bin as the
// one-wavefront routine, whose keys are unique across slots.  Each bin's
// residual update is the same arithmetic in the same order, and every
// wavefront accumulates the target model as before (wavefront 0 writes
// it), so the result is bitwise that of the one-wavefront routine.
#pragma once

#include "fsr_block.h"

namespace fsr {

// Four residual bins as one register tuple, for the indexed read of the
// winner's slot.
typedef float f32x4 __attribute__((ext_vector_type(4)));

// LDS of the routine beyond the block's kLdsFloats: bins of slots 4..15
// (12 x 64 float2), two buffers of four candidates, the "any pixel known"
// flag.
struct Split4Lds {
    float2 bins[12 * 64];
    uint4 cand[2][4];
    int any_known;
};

__device__ __forceinline__ void reconstruct_block_reuse_split4(const BlockJob& jb, int B, int L, float gamma,
                                                               const BlockTables& tab, float* lds,
                                                               Split4Lds& sh) {
    const int lane = (int)(threadIdx.x & 63);
    const int q = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wavefront of the block
    const int c = lane & 31, h = lane >> 5;
    const int ti = lane / B, tj = lane - (lane / B) * B;
    const int tm = L + ti, tn = L + tj;
    float2* wtab = reinterpret_cast<float2*>(lds);
    f32x4 vr = {}, vi = {};

    if (q == 0) {
        // ---- gather and weighting, pixel (m, n) = (2s + h, c); earlier
        // targets (the rows above this target, and this target's rows left
        // of it) take part with their reconstruction
        const int y0 = jb.by * B - L, x0 = jb.bx * B - L;
        float xr[16], wr[16];
        uint64_t any_known = 0;
        const int x = x0 + c;
        const bool xin = (unsigned)x < (unsigned)jb.width;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int m = 2 * s + h, y = y0 + m;
            const bool in = xin && (unsigned)y < (unsigned)jb.height;
            const int64_t off = in ? (int64_t)y * jb.stride + x : 0;
            const uint8_t kraw = jb.mask[off];
            const float fraw = jb.image[off];
            const float rp = global_ptr(tab.rho_pow)[m * kS + c];
            const uint8_t k = in ? kraw : (uint8_t)0;
            const float w = k ? rp : 0.0f;
            const bool earlier = m < L || (m < L + B && c < L);
            const bool reused = in && !k && earlier && jb.delta > 0.0f;
            any_known |= ballot(k != 0 || reused);
            xr[s] = k ? fraw : reused ? (float)jb.out[off] : 0.0f;
            wr[s] = reused ? jb.delta * rp : w;
        }
        if (any_known != 0) {
            // ---- R_w = mu W + DFT2((f~ - mu) w) and W, both real tiles in
            // one complex FFT, as in fsr_block.h
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
            float scale;
            const float xmax = max_abs_and_scale(xr, scale);
#pragma unroll
            for (int s = 0; s < 16; ++s) xi[s] = wr[s] * scale;
            dft2_complex_to_planes(xr, xi, lds, lane);
            planes_split_two_real(xr, xi, wr, wi, 0.5f / scale, lds, lane);
            if (xmax == 0.0f) {
#pragma unroll
                for (int s = 0; s < 16; ++s) xr[s] = xi[s] = 0.0f;
            }
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                xr[s] = fmaf(mu, wr[s], xr[s]);
                xi[s] = fmaf(mu, wi[s], xi[s]);
            }
            // W with duplicated rows, as in fsr_block.h; slots 4..15 parked
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int k = 2 * s + h;
                wtab[k * kS + c] = make_float2(wr[s], wi[s]);
                wtab[(k + kS) * kS + c] = make_float2(wr[s], wi[s]);
            }
#pragma unroll
            for (int s = 4; s < 16; ++s) sh.bins[64 * (s - 4) + lane] = make_float2(xr[s], xi[s]);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                vr[s] = xr[s];
                vi[s] = xi[s];
            }
        }
        if (lane == 0) sh.any_known = any_known != 0;
    }
    __syncthreads();

    float acc = 0.0f;
    const int iters = jb.iterations;
    if (sh.any_known) {
        if (q != 0) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const float2 v = sh.bins[64 * (4 * q - 4 + s) + lane];
                vr[s] = v.x;
                vi[s] = v.y;
            }
        }
        const float w00 = wtab[0].x;   // W[0][0]: row 0, column 0
        const float gi = w00 > 0.0f ? gamma / w00 : 0.0f;
        float wf[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) wf[s] = global_ptr(tab.freq_w)[(2 * (4 * q + s) + h) * kS + c];
        const int tw_re = __float_as_int(kTw.re[c]), tw_im = __float_as_int(kTw.im[c]);
        const int tmn4 = opaque((4 * tm) | ((4 * tn) << 16));
        // byte offset of the lane's entry (h, c) in W, plus this wavefront's
        // first slot (512 bytes per slot): the low byte stays 8 c
        const int hc8 = opaque(256 * h + 8 * c + 2048 * q);
        const uint32_t code0 = 15u - 4u * (uint32_t)q;

        for (int it = 0; it < iters; ++it) {
            // this wavefront's candidate: its largest key (Eq. 16, the same
            // keys as the one-wavefront routine), lane and R_w
            uint32_t lmax = 0;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const float e = fmaf(vr[s], vr[s], vi[s] * vi[s]);
                const uint32_t key = (__float_as_uint(e * wf[s]) & 0xFFFFFFF0u) | (code0 - (uint32_t)s);
                lmax = umax(lmax, key);
            }
            const uint32_t mx = wave_max_u32(lmax);
            const int ln = (int)__builtin_ctzll(ballot(lmax == mx));
            const int sl = (int)(code0 - (mx & 15u));   // slot within this wavefront
            const float pr_q = readlane_f(vr[sl], ln);
            const float pi_q = readlane_f(vi[sl], ln);
            uint4* cb = sh.cand[it & 1];
            if (lane == 0) cb[q] = make_uint4(mx, (uint32_t)ln, __float_as_uint(pr_q), __float_as_uint(pi_q));
            __syncthreads();
            // the largest of the four (keys differ: each slot has its own code)
            const uint4 cq = cb[lane & 3];
            uint32_t best = umax(cq.x, dpp_u32<0xB1>(cq.x));
            best = umax(best, dpp_u32<0x4E>(best));
            const int qw = (int)__builtin_ctzll(ballot(cq.x == best));   // lanes 0..3 hold wavefronts 0..3
            const uint32_t mxw = (uint32_t)__builtin_amdgcn_readlane((int)cq.x, qw);
            const int lnw = __builtin_amdgcn_readlane((int)cq.y, qw);
            const float pr = __int_as_float(__builtin_amdgcn_readlane((int)cq.z, qw));
            const float pim = __int_as_float(__builtin_amdgcn_readlane((int)cq.w, qw));
            const int idx = 64 * (15 - (int)(mxw & 15u)) + lnw;
            const int u = idx >> 5, v = idx & 31;
            const float cr = gi * pr, ci = gi * pim;    // gamma * p (Eqs. 10-11)
            // residual (Eqs. 12, 14-15) on this wavefront's slots, as in
            // fsr_block.h: slot 4q + s reads duplicated row h + 32 - u +
            // 2 (4q + s), column (c - v) mod 32.  The reads go out first so
            // that the model's lane exchange waits alongside them.
            const int woff = sub_low_byte(hc8 + (8192 - 256 * u), 8 * v);
            const float2* wrow = reinterpret_cast<const float2*>(reinterpret_cast<const char*>(wtab) + woff);
            float2 w[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) w[s] = wrow[64 * s];
            // model: g += gamma p exp(+j 2 pi (u m + v n) / S) on the target;
            // every wavefront computes it (no branch in the loop's chain),
            // wavefront 0's is the one written
            const int q4 = dot2_u16(u | (v << 16), tmn4);
            const float er = __int_as_float(__builtin_amdgcn_ds_bpermute(q4, tw_re));
            const float ei = __int_as_float(__builtin_amdgcn_ds_bpermute(q4, tw_im));
            acc = fmaf(cr, er, acc);
            acc = fmaf(ci, ei, acc);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                vr[s] = fmaf(-cr, w[s].x, vr[s]);
                vr[s] = fmaf(ci, w[s].y, vr[s]);
                vi[s] = fmaf(-cr, w[s].y, vi[s]);
                vi[s] = fmaf(-ci, w[s].x, vi[s]);
            }
            if (q == 0 && jb.log != nullptr && lane == 0) jb.log[it] = (uint16_t)idx;
        }
    } else if (q == 0 && jb.log != nullptr) {
        for (int it = lane; it < iters; it += 64) jb.log[it] = (uint16_t)0xFFFF;
    }

    // ---- compose (Sec. II): known pixels copied, unknown pixels Re g
    if (q == 0 && lane < B * B) {
        const int y = jb.by * B + ti, xx = jb.bx * B + tj;
        if (y < jb.height && xx < jb.width) {
            const int64_t off = (int64_t)y * jb.stride + xx;
            const uint8_t k = jb.mask[off];
            jb.out[off] = k ? jb.image[off] : acc;
        }
    }
}

}  // namespace fsr
