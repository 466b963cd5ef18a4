// fsr_block_s24.h -- one support block of FSR on one wavefront at S = 24
// with every lane busy (Sec. II; the paper sweeps S up to 32 in Sec. IV).
//
// Layout: lane = 8 a + b (a, b < 8), slot s = 3 i + j (i, j < 3); slot s of
// lane (a, b) holds pixel, or bin, (a + 8 i, b + 8 j): the 576 bins fill
// 64 lanes x 9 slots, where the generic layout of fsr_block_sg.h (one column
// per lane) leaves 16 lanes idle at this size.
//
// Argmax ties (Eq. 8: equal objectives go to the smaller bin k S + l).  The
// bin index 192 i + 24 a + 8 j + b does not order as (slot, lane), so the
// key's tie code cannot be the slot alone.  The ties that occur exactly are
// those between a bin and its conjugate (-k, -l), which R_w has while it is
// Hermitian.  Each bin therefore carries a per-lane code: 15 - s when it is
// the smaller bin of its conjugate pair (or its own conjugate), 6 - r when
// it is the r-th larger-of-pair bin of its lane (a lane holds at most six
// of either kind).  The smaller bin of a pair thus always has the larger
// code; equal keys, which share a code, go to the lower lane, and within one
// slot that is the smaller bin.  A key's code and lane give back its slot.
//
// DFT: both real tiles in one complex transform z = (f~ - mu) w + j s w
// (s a power of two, as in the S = 32 kernel), two radix-3 x 8 passes
// (s24_pass) with twiddles from the table F[m][k] = exp(-j 2 pi m k / S) in
// LDS, then split into the two exactly Hermitian spectra.
//
// LDS per wavefront: the DFT table (S^2 float2) and a scratch area (the
// passes' 24 x 25 float2, then the spectrum) during the transforms; during the iterations W with its columns repeated once (24
// rows of 48 entries, entry (R, C) = W[R][C mod S]) at a row pitch of 52
// entries, 9.75 KiB.  Slot (i, j) of lane (a, b) reads row (a - u + 8 i)
// mod S, wrapped per row slot i, and column b + 8 j + S - v, which needs no
// wrap: three row bases per iteration, each with immediate offsets for j.
// One read covers eight consecutive rows (mod S) of eight consecutive
// entries; at a pitch of 52 entries (104 words, 40 mod 64) the eight rows
// start 0, 40, 16, 56, 32, 8, 48, 24 words into the 64 banks, so every bank
// serves two words, the fewest for 64 lanes of 8 bytes, and every half
// wavefront (four rows) covers the 32 banks of a half twice.  A pitch of 48
// (96 words) starts the rows alternately at 0 and 32: 3,072 bank-conflict
// cycles per block.  Measured on the 1080p frame at I = 100 (before the W
// reads were issued ahead of the model's lane exchange, which took 2.40 to
// 2.33-2.37 ms), pitches timed side by side: pitch 52 2.40 ms, 48
// 2.45-2.47 ms, 50 2.48 ms on one box;
// 56 (10.5 KiB, fewer resident wavefronts) 2.51 ms against 2.41 ms at 48 on
// another.  Earlier layouts against 2.40 ms at pitch 48: rows and columns
// both repeated up to 40 (12.5 KiB, two wraps) 2.57 ms; both repeated in
// full (48 x 48, 19.5 KiB, a uniform shift) 3.50 ms; the 48-lane layout of
// fsr_block_sg.h 3.27 ms.
#pragma once

#include "fsr_block.h"
#include "fsr_block_sg.h"

namespace fsr {

struct S24 {
    static constexpr int S = 24;
    static constexpr int NS = 9;                  // slots per lane
    static constexpr int kPitch = 52;             // W table: S rows of 2S entries (float2), this pitch
    static constexpr int kTabFloats = 2 * S * S;  // DFT table, then scratch
    static constexpr int kLdsFloats = 2 * S * kPitch;
    static_assert(kTabFloats + 2 * 24 * 25 <= kLdsFloats, "transforms fit in the W table's space");
    static constexpr int kArgmaxPairs = 1024;     // 576 (key, lane) pairs, padded to 2^10
};

// Tie codes of this lane's bins (see above) and the slot of each code:
// nibble c of the 64-bit map (*map_hi, *map_lo) holds the slot whose code is
// c (codes no slot of the lane carries hold 0).
__device__ __forceinline__ void s24_codes(int a, int b, uint32_t (&code)[S24::NS], uint32_t* map_lo,
                                          uint32_t* map_hi) {
    constexpr int S = S24::S;
    int r = 0;
    uint64_t m = 0;
#pragma unroll
    for (int s = 0; s < S24::NS; ++s) {
        const int k = a + 8 * (s / 3), l = b + 8 * (s % 3);
        const int kc = k ? S - k : 0, lc = l ? S - l : 0;
        const bool larger = k * S + l > kc * S + lc;
        code[s] = larger ? (uint32_t)(6 - r) : (uint32_t)(15 - s);
        m |= (uint64_t)s << (4 * code[s]);
        r += larger ? 1 : 0;
    }
    *map_lo = (uint32_t)m;
    *map_hi = (uint32_t)(m >> 32);
}

// One 24-point DFT pass over the 24 sequences of one axis, radix 3 x 8:
// with element x = p + 8 q (p < 8 across lanes, q < 3 in the lane's slots)
// and output k = k1 + 3 k2 (k1 < 3, k2 < 8),
//   X[k1 + 3 k2] = sum_p W8^(p k2) W24^(p k1) sum_q x[p + 8 q] W3^(q k1).
// A 3-point DFT over the lane's slots and the twiddle W24^(p k1) go to buf
// (entry (8 k1 + p) 25 + sequence: the three k1 groups of a read start 0,
// 16 and 32 words apart); each output then sums its eight terms over p by
// Horner's rule in W8^k2, which keeps the natural layout (output k = p + 8 q
// in the slot of element p + 8 q).  kAlongM: along m (p = a, q = i, the
// sequence n = b + 8 j), else along n (p = b, q = j, the sequence
// k = a + 8 i).  ftab is the DFT table, row F[1] = W24^q.
template <bool kAlongM>
__device__ __forceinline__ void s24_pass(float (&re)[S24::NS], float (&im)[S24::NS], const float2* ftab,
                                         float2* buf, int a, int b) {
    constexpr int S = S24::S, P = 25;
    constexpr float kH3 = 0.866025403784438647f;   // sin(pi / 3)
    const int p = kAlongM ? a : b, o = kAlongM ? b : a;
    const float2 t1 = ftab[S + p], t2 = ftab[S + 2 * p];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int s0 = kAlongM ? r : 3 * r, ds = kAlongM ? 3 : 1;   // slot of q = 0, step per q
        const float x0r = re[s0], x0i = im[s0];
        const float tr = re[s0 + ds] + re[s0 + 2 * ds], ti = im[s0 + ds] + im[s0 + 2 * ds];
        const float dr = re[s0 + ds] - re[s0 + 2 * ds], di = im[s0 + ds] - im[s0 + 2 * ds];
        const float hr = fmaf(-0.5f, tr, x0r), hi = fmaf(-0.5f, ti, x0i);
        float y1r = fmaf(kH3, di, hr), y1i = fmaf(-kH3, dr, hi);    // x0 + W3 x1 + W3^2 x2
        float y2r = fmaf(-kH3, di, hr), y2i = fmaf(kH3, dr, hi);    // x0 + W3^2 x1 + W3 x2
        cmul(y1r, y1i, t1.x, t1.y);
        cmul(y2r, y2i, t2.x, t2.y);
        const int col = o + 8 * r;
        buf[p * P + col] = make_float2(x0r + tr, x0i + ti);
        buf[(8 + p) * P + col] = make_float2(y1r, y1i);
        buf[(16 + p) * P + col] = make_float2(y2r, y2i);
    }
    wave_sync();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int k = p + 8 * q, k1 = k % 3, k2 = k / 3;
        const float2 w = ftab[S + 3 * k2];   // W8^k2
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float2* col = buf + 8 * k1 * P + o + 8 * r;
            float xr = col[7 * P].x, xi = col[7 * P].y;
#pragma unroll
            for (int pp = 6; pp >= 0; --pp) {
                const float2 v = col[pp * P];
                cmul(xr, xi, w.x, w.y);
                xr += v.x;
                xi += v.y;
            }
            const int s = kAlongM ? 3 * q + r : 3 * r + q;
            re[s] = xr;
            im[s] = xi;
            // no reads of the next sum ahead of this one: 8 reads in flight
            // instead of 72, which would take the persistent kernels past
            // 128 VGPRs (three wavefronts per SIMD instead of four)
            asm volatile("" ::: "memory");
        }
    }
    wave_sync();   // every lane has read buf
}

// kPersistent as in the other block routines (the caller loops over blocks).
// kArgmax: kArgmaxWave, or kArgmaxLds (every (key, lane) pair through a
// shared-memory tree, argmax_lds holding S24::kArgmaxPairs pairs); both pick
// the same bin.
template <bool kPersistent = false, int kArgmax = kArgmaxWave>
__device__ __forceinline__ void reconstruct_block_s24(const BlockJob& jb, int B, int L, float gamma,
                                                      const BlockTables& tab_in, float* lds,
                                                      uint2* argmax_lds = nullptr) {
    constexpr int S = S24::S, NS = S24::NS, P = S24::kPitch;
    const int lane = kPersistent ? opaque((int)(threadIdx.x & 63)) : (int)(threadIdx.x & 63);
    BlockTables tab = tab_in;
    if constexpr (kPersistent) {
        tab.rho_pow = opaque_ptr(tab_in.rho_pow);
        tab.freq_w = opaque_ptr(tab_in.freq_w);
        tab.dft_sg = opaque_ptr(tab_in.dft_sg);
    }
    const int a = lane >> 3, b = lane & 7;
    const int y0 = jb.by * B - L, x0 = jb.bx * B - L;
    float2* ftab = reinterpret_cast<float2*>(lds);
    float2* scr = reinterpret_cast<float2*>(lds + S24::kTabFloats);

    // ---- DFT table into LDS (the same for every block)
    {
        const global_t<const uint64_t>* src = global_ptr(reinterpret_cast<const uint64_t*>(tab.dft_sg));
        uint64_t* dst = reinterpret_cast<uint64_t*>(ftab);
        for (int i = lane; i < S * S; i += 64) dst[i] = src[i];
    }

    // ---- gather and weighting: slot s holds pixel (a + 8 i, b + 8 j)
    float xr[NS], wr[NS];
    uint64_t any_known = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int m = a + 8 * (s / 3), n = b + 8 * (s % 3);
        const int y = y0 + m, x = x0 + n;
        const bool in = (unsigned)y < (unsigned)jb.height && (unsigned)x < (unsigned)jb.width;
        const int64_t off = in ? (int64_t)y * jb.stride + x : 0;
        const uint8_t kraw = jb.mask[off];
        const float fraw = jb.image[off];
        const float rp = global_ptr(tab.rho_pow)[m * S + n];
        const uint8_t k = in ? kraw : (uint8_t)0;
        any_known |= ballot(k != 0);
        xr[s] = k ? fraw : 0.0f;
        wr[s] = k ? rp : 0.0f;
    }

    // ---- target pixel owned by this lane (lanes 0 .. B*B-1; the other
    // lanes model pixel (L, L) and discard it)
    const bool owner = lane < B * B;
    const int ti = owner ? lane / B : 0, tj = owner ? lane - (lane / B) * B : 0;
    const int tm = L + ti, tn = L + tj;
    float acc = 0.0f;
    const int iters = jb.iterations;
    wave_sync();   // DFT table written

    if (any_known != 0) {
        // ---- R_w = mu W + DFT2((f~ - mu) w), mu the weighted mean of the
        // known support pixels, as in the other block routines
        float sx = 0.0f, sw = 0.0f;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            sx = fmaf(xr[s], wr[s], sx);
            sw += wr[s];
        }
        sx = wave_sum_f32(sx);
        sw = wave_sum_f32(sw);
        const float mu = sw > 0.0f ? sx / sw : 0.0f;
        uint32_t amax = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            xr[s] = (xr[s] - mu) * wr[s];
            amax = umax(amax, __float_as_uint(fabsf(xr[s])));
        }
        amax = wave_max_u32(amax);
        // z = x + j sc w with sc the power of two at or below max |x| (exact)
        const uint32_t sbits = amax & 0x7F800000u;
        const float sc = sbits ? __uint_as_float(sbits) : 1.0f;
        // the two passes, radix 3 x 8 (s24_pass), on z = x + j sc w in registers
        float zr[NS], zi[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            zr[s] = xr[s];
            zi[s] = wr[s] * sc;
        }
        s24_pass<true>(zr, zi, ftab, scr, a, b);    // along m: C[k][n]
        s24_pass<false>(zr, zi, ftab, scr, a, b);   // along n: Z[k][l]
#pragma unroll
        for (int s = 0; s < NS; ++s) scr[(a + 8 * (s / 3)) * S + b + 8 * (s % 3)] = make_float2(zr[s], zi[s]);
        wave_sync();
        // split Z = F2{x + j sc w} into X = (Z + conj Z[-k]) / 2 and
        // W = (Z - conj Z[-k]) / (2 j sc): bins k and -k read the same pair
        // of values in swapped roles, so both come out exactly Hermitian
        const float h = 0.5f / sc;
        float xi[NS], wi[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k = a + 8 * (s / 3), l = b + 8 * (s % 3);
            const int km = k ? S - k : 0, lm = l ? S - l : 0;
            const float2 zm = scr[km * S + lm];
            const float ar = zr[s], ai = zi[s];
            xr[s] = 0.5f * (ar + zm.x);
            xi[s] = 0.5f * (ai - zm.y);
            wr[s] = (ai + zm.y) * h;
            wi[s] = (zm.x - ar) * h;
        }
        if (amax == 0) {
            // every known pixel equals mu: X is exactly 0 (no rounding of the
            // w part may leak into it)
#pragma unroll
            for (int s = 0; s < NS; ++s) xr[s] = xi[s] = 0.0f;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            xr[s] = fmaf(mu, wr[s], xr[s]);
            xi[s] = fmaf(mu, wi[s], xi[s]);
        }
        const float w00 = readlane_f(wr[0], 0);
        const float gi = w00 > 0.0f ? gamma / w00 : 0.0f;
        float wf[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) wf[s] = global_ptr(tab.freq_w)[(a + 8 * (s / 3)) * S + b + 8 * (s % 3)];
        // lane i of tw_re / tw_im holds F[1][i mod S], read before the W
        // table overwrites the DFT table
        const float2 tw = ftab[S + (lane % S)];
        const int tw_re = __float_as_int(tw.x), tw_im = __float_as_int(tw.y);
        uint32_t code[NS], map_lo, map_hi;
        s24_codes(a, b, code, &map_lo, &map_hi);
        // the loads of the loop's constants complete here, not at their first
        // use inside the loop (which would put their waits in the loop body)
#pragma unroll
        for (int s = 0; s < NS; ++s) wf[s] = __int_as_float(opaque(__float_as_int(wf[s])));
        wave_sync();   // every lane has read the spectrum and the table
        // W, rows and columns duplicated
        float2* wtab = reinterpret_cast<float2*>(lds);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k = a + 8 * (s / 3), l = b + 8 * (s % 3);
            const float2 wv = make_float2(wr[s], wi[s]);
            wtab[k * P + l] = wv;
            wtab[k * P + l + S] = wv;
        }
        // lane constants kept as computed here
        // the lane's byte offset 8 P a + 8 b of entry (a, b)
        const int ab8 = opaque(8 * P * a + 8 * b);
        const int tmn = opaque(tm | (tn << 16));
        const char* wbytes = reinterpret_cast<const char*>(wtab);
        wave_sync();

        // the loop comes in two copies, with and without the argmax log, so
        // that the one without carries no per-iteration branch for it
        auto iterate = [&](auto with_log) {
            for (int it = 0; it < iters; ++it) {
                // objective (Eq. 16) as an argmax key: the float32 bits with the
                // 4 low mantissa bits replaced by the bin's tie code
                uint32_t key[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const float e = fmaf(xr[s], xr[s], xi[s] * xi[s]);
                    key[s] = (__float_as_uint(e * wf[s]) & 0xFFFFFFF0u) | code[s];
                }
                uint32_t mx;
                int ln;
                if constexpr (kArgmax == kArgmaxWave) {
                    uint32_t lmax = 0;
#pragma unroll
                    for (int s = 0; s < NS; ++s) lmax = umax(lmax, key[s]);
                    mx = wave_max_u32(lmax);
                    ln = (int)__builtin_ctzll(ballot(lmax == mx));
                } else {
#pragma unroll
                    for (int s = 0; s < NS; ++s) argmax_lds[64 * s + lane] = make_uint2(key[s], (uint32_t)lane);
#pragma unroll
                    for (int e = 64 * NS; e < S24::kArgmaxPairs; e += 64)
                        argmax_lds[e + lane] = make_uint2(0u, 0xFFFFFFFFu);
                    wave_sync();
#pragma unroll
                    for (int half = S24::kArgmaxPairs / 2; half >= 64; half >>= 1) {
#pragma unroll
                        for (int j = 0; j < half / 64; ++j) {
                            const int e = lane + 64 * j;
                            argmax_lds[e] = better_pair(argmax_lds[e], argmax_lds[e + half]);
                        }
                        wave_sync();
                    }
#pragma unroll
                    for (int half = 32; half >= 1; half >>= 1) {
                        if (lane < half) argmax_lds[lane] = better_pair(argmax_lds[lane], argmax_lds[lane + half]);
                        wave_sync();
                    }
                    mx = (uint32_t)__builtin_amdgcn_readfirstlane((int)argmax_lds[0].x);
                    ln = __builtin_amdgcn_readfirstlane((int)argmax_lds[0].y);
                    wave_sync();   // the next iteration overwrites the pairs
                }
                // the winner's slot from its code, through the winning lane's map
                const int cw = (int)(mx & 15u);
                const uint64_t wmap = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)map_lo, ln) |
                                      (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)map_hi, ln) << 32;
                const int slot = (int)((wmap >> (4 * cw)) & 15u);
                const int u = (ln >> 3) + 8 * (slot / 3), v = (ln & 7) + 8 * (slot % 3);
                const float pr = readlane_f(xr[slot], ln);
                const float pim = readlane_f(xi[slot], ln);
                const float cr = gi * pr, ci = gi * pim;    // gamma * p (Eqs. 10-11)
                if constexpr (decltype(with_log)::value) {
                    if (lane == 0) jb.log[it] = (uint16_t)(u * S + v);
                }

                // residual (Eqs. 12, 14-15): bin (k, l) = (a + 8 i, b + 8 j) reads
                // W[(k - u) mod S][(l - v) mod S], table entry
                // ((a - u + 8 i) mod S, b + 8 j + S - v).  Byte offset 8 P x + y
                // of row x, with the column part y = 8 (b + S - v) in [8, 8 P):
                // a row below 0 or at S and above is wrapped by a minimum of
                // unsigned values (x itself when in range, else x +/- S rows;
                // out of range the other one is negative, i.e. huge unsigned)
                const int uv8 = __builtin_amdgcn_readfirstlane(8 * (S - v) - 8 * P * u);   // scalar
                const uint32_t y0 = (uint32_t)(ab8 + uv8);
                const uint32_t ad0 = umin(y0, y0 + 8 * P * S);
                const uint32_t r1a = ad0 + 64 * P, r2a = ad0 + 128 * P;
                const uint32_t ad1 = umin(r1a, r1a - 8 * P * S);
                const uint32_t ad2 = umin(r2a, r2a - 8 * P * S);
                const float2* wrow0 = reinterpret_cast<const float2*>(wbytes + ad0);
                const float2* wrow1 = reinterpret_cast<const float2*>(wbytes + ad1);
                const float2* wrow2 = reinterpret_cast<const float2*>(wbytes + ad2);
                const float2* wrows[3] = {wrow0, wrow1, wrow2};
                // the reads go out before the model's lane exchange, so that the
                // two wait together
                float2 w[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) w[s] = wrows[s / 3][8 * (s % 3)];
                // model: g += gamma p exp(+j 2 pi (u m + v n) / S) on the target
                const int q4 = 4 * mod_small<S>(dot2_u16(u | (v << 16), tmn));
                const float er = __int_as_float(__builtin_amdgcn_ds_bpermute(q4, tw_re));
                const float ei = __int_as_float(__builtin_amdgcn_ds_bpermute(q4, tw_im));
                acc = fmaf(cr, er, acc);
                acc = fmaf(ci, ei, acc);

#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    xr[s] = fmaf(-cr, w[s].x, xr[s]);
                    xr[s] = fmaf(ci, w[s].y, xr[s]);
                    xi[s] = fmaf(-cr, w[s].y, xi[s]);
                    xi[s] = fmaf(-ci, w[s].x, xi[s]);
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
    if (owner) {
        const int y = jb.by * B + ti, xx = jb.bx * B + tj;
        if (y < jb.height && xx < jb.width) {
            const int64_t off = (int64_t)y * jb.stride + xx;
            const uint8_t k = jb.mask[off];
            jb.out[off] = k ? jb.image[off] : acc;
        }
    }
}

}  // namespace fsr
