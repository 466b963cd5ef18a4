// fsr_block_sg.h -- one support block of FSR on one wavefront for the smaller
// even supports S = 8, 16, 24 (Sec. II; the paper sweeps S over 8..32 in
// Sec. IV and runs its real-time table at S = 16).
//
// Layout: G = 64 / S lane groups; lane = c + S h (c < S, h < G) is active
// when lane < G S (all 64 lanes for S = 8 and 16, 48 for S = 24).  Slot s of
// an active lane holds pixel (m = G s + h, n = c) of the tile, and bin
// (k = G s + h, l = c) of a spectrum, so the bin index k S + l = s G S + lane
// orders as (slot, lane), as in the S = 32 kernel.
//
// DFT: direct separable sums against a DFT table F[m][k] = exp(-j 2 pi m k / S)
// held in LDS, built on the host with exact symmetries (F[m][S-k] is the
// exact conjugate of F[m][k]).  Bins k and -k are then summed by the same
// instruction sequence on exactly conjugated operands, so the FP32 spectrum
// of a real tile is bitwise Hermitian without a symmetrisation step (the
// rounding of a negated operand is the negated rounding).  At S = 16 the two
// real tiles instead go through one complex transform z = x + j s w, split
// into the two exactly Hermitian spectra as in the S = 24 and 32 routines,
// as two radix-4 x 4 passes (fft16_pass) with one transpose through LDS
// between them.
//
// LDS per wavefront: during the transforms the DFT table (S^2 float2) and
// a scratch area for the tile and then, over it, the first pass of the DFT
// (4 S^2 floats), at S = 16 the passes' exchange and transpose areas;
// during the iterations W with duplicated rows, and for S <= kFullDupMax
// duplicated columns too (2S x 2S float2, entry (R, C) = W[R mod S][C mod S],
// 8 S^2 floats), so that the cyclic shift of Eqs. 14-15 is one uniform
// offset added to a per-lane address; above that the column wraps per lane.
#pragma once

#include "fsr_block.h"

namespace fsr {

// Largest support whose W table also duplicates its columns.  Measured: at
// S = 16 the 2S x 2S table (8 KiB) costs more in resident wavefronts than
// the column wrap it saves (1080p, I = 100: 1.28 against 1.25 ms); at S = 8
// it costs nothing (2 KiB).
constexpr int kFullDupMax = 8;

template <int S>
struct SgShape {
    static constexpr int G = 64 / S;          // lane groups
    static constexpr int NS = S / G;          // slots per lane
    static constexpr int NL = G * S;          // active lanes
    static constexpr bool kFullDup = S <= kFullDupMax;   // columns duplicated too
    static constexpr int P = kFullDup ? 2 * S : S;        // W table pitch, float2
    static constexpr int kLdsFloats = kFullDup ? 8 * S * S : 4 * S * S;
    static constexpr uint32_t kModMagic = (65536u + S - 1) / S;
    static_assert(S % 2 == 0 && S >= 8 && S < 32 && S % G == 0, "even S in [8, 32)");
    static_assert(NS <= 16, "slot code fits in 4 bits");
};

// q mod S for 0 <= q < 2 S^2 (the target-model phase index): a mask for
// powers of two, else a multiply-shift division checked at compile time.
template <int S>
constexpr bool mod_magic_exact() {
    for (uint32_t q = 0; q < 2u * S * S; ++q)
        if (q - S * ((q * SgShape<S>::kModMagic) >> 16) != q % S) return false;
    return true;
}

template <int S>
__device__ __forceinline__ int mod_small(int q) {
    if constexpr ((S & (S - 1)) == 0) {
        return q & (S - 1);
    } else {
        static_assert(mod_magic_exact<S>(), "division by multiply-shift must be exact");
        // q < 2 S^2 and the magic number are below 2^12 and 2^16: the
        // product fits the full-rate 24-bit multiplier
        return q - S * (int)((uint32_t)mul_u24((int)SgShape<S>::kModMagic, q) >> 16);
    }
}

// 2D DFT of the real values v (slot s = pixel (G s + h, c)) into (re, im)
// (slot s = bin (G s + h, c)).  Active lanes only carry data; inactive lanes
// compute duplicates that the caller discards.  `ftab` is the DFT table in
// LDS, `scr` the scratch area (the tile, S^2 floats, then over it the
// first pass, S^2 float2).
template <int S>
__device__ __forceinline__ void dft2_sg(const float (&v)[SgShape<S>::NS], float (&re)[SgShape<S>::NS],
                                        float (&im)[SgShape<S>::NS], const float2* ftab, float* scr,
                                        int c, int h, bool active) {
    constexpr int G = SgShape<S>::G, NS = SgShape<S>::NS;
    float* tile = scr;                                // [m][n]
    float2* pass1 = reinterpret_cast<float2*>(scr);   // [k][n], over the tile once it is read
    if (active) {
#pragma unroll
        for (int s = 0; s < NS; ++s) tile[(G * s + h) * S + c] = v[s];
    }
    wave_sync();
    // pass 1 along m: C[k][n] = sum_m x[m][n] F[m][k], k = G s + h, n = c
    float ar[NS], ai[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) ar[s] = ai[s] = 0.0f;
    // the row loops are only partly unrolled: fully unrolled, the compiler
    // hoists all S x NS table reads ahead of the arithmetic
#pragma unroll 2
    for (int m = 0; m < S; ++m) {
        const float x = tile[m * S + c];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const float2 f = ftab[m * S + G * s + h];
            ar[s] = fmaf(x, f.x, ar[s]);
            ai[s] = fmaf(x, f.y, ai[s]);
        }
    }
    wave_sync();   // every lane has read the tile
    if (active) {
#pragma unroll
        for (int s = 0; s < NS; ++s) pass1[(G * s + h) * S + c] = make_float2(ar[s], ai[s]);
    }
    wave_sync();
    // pass 2 along n: X[k][l] = sum_n C[k][n] F[n][l], k = G s + h, l = c
    float br[NS], bi[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) br[s] = bi[s] = 0.0f;
#pragma unroll 2
    for (int n = 0; n < S; ++n) {
        const float2 f = ftab[n * S + c];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const float2 a = pass1[(G * s + h) * S + n];
            br[s] = fmaf(a.x, f.x, br[s]);
            br[s] = fmaf(-a.y, f.y, br[s]);
            bi[s] = fmaf(a.x, f.y, bi[s]);
            bi[s] = fmaf(a.y, f.x, bi[s]);
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        re[s] = br[s];
        im[s] = bi[s];
    }
    wave_sync();   // the scratch area is reused by the caller
}

// ---- S = 16: the 2D DFT in radix-4 x 4 passes (G = 4 lane groups, NS = 4
// slots)

// In-place 4-point DFT (W4 = -j) of a lane's four slots, natural order in
// and out.
__device__ __forceinline__ void dft4_slots(float (&re)[4], float (&im)[4]) {
    const float t0r = re[0] + re[2], t0i = im[0] + im[2];
    const float t1r = re[0] - re[2], t1i = im[0] - im[2];
    const float t2r = re[1] + re[3], t2i = im[1] + im[3];
    const float t3r = re[1] - re[3], t3i = im[1] - im[3];
    re[0] = t0r + t2r; im[0] = t0i + t2i;   // y0
    re[2] = t0r - t2r; im[2] = t0i - t2i;   // y2
    re[1] = t1r + t3i; im[1] = t1i - t3r;   // y1 = t1 - j t3
    re[3] = t1r - t3i; im[3] = t1i + t3r;   // y3 = t1 + j t3
}

// One 16-point DFT of 16 sequences: slot s of lane (c, h) holds element
// 4 s + h of sequence c, and on return its output 4 s + h.  With element
// m = 4 s + h and output k = k1 + 4 k2,
//   X[k1 + 4 k2] = sum_h W4^(h k2) W16^(h k1) sum_s x[4 s + h] W4^(s k1):
// the inner sum is a 4-point DFT over the lane's slots; after the twiddle
// W16^(h k1) (tw_r / tw_i[k1], for this lane's h) lane (c, h) gathers the
// values of k1 = h from the lanes (c, h'), h' = 0..3, through ex (entry
// 80 k1 + 16 h + c: the writes of one k1 and the reads of one h' each
// cover the 64 banks), and a 4-point DFT over h' gives outputs h + 4 k2 in
// slots k2.
__device__ __forceinline__ void fft16_pass(float (&re)[4], float (&im)[4], const float (&tw_r)[4],
                                           const float (&tw_i)[4], float2* ex, int c, int h) {
    dft4_slots(re, im);
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) cmul(re[k1], im[k1], tw_r[k1], tw_i[k1]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) ex[80 * k1 + 16 * h + c] = make_float2(re[k1], im[k1]);
    wave_sync();
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const float2 v = ex[80 * h + 16 * g + c];
        re[g] = v.x;
        im[g] = v.y;
    }
    wave_sync();   // every lane has read ex
    dft4_slots(re, im);
}

// Entry i (re, im) of a float2 table in global memory.
__device__ __forceinline__ void table_entry(const float2* tab, int i, float& re, float& im) {
    const uint64_t v = global_ptr(reinterpret_cast<const uint64_t*>(tab))[i];
    re = __uint_as_float((uint32_t)v);
    im = __uint_as_float((uint32_t)(v >> 32));
}

// Row pitch (float2) of the S = 16 tiles in LDS: the 16 lanes of a row
// group reading a column start 36 words apart, 32 lanes cover the 64 banks.
constexpr int kS16Pitch = 18;

// 2D DFT of the complex S = 16 tile z (slot s of lane (c, h) = pixel
// (4 s + h, c)), along m, then, after a transpose through buf, along n: on
// return slot s of lane (c, h) holds bin (c, 4 s + h), i.e. the spectrum
// transposed.  buf holds 304 float2 (the exchange areas' extent).
__device__ __forceinline__ void fft2_s16(float (&zr)[4], float (&zi)[4], const float (&tw_r)[4],
                                         const float (&tw_i)[4], float2* buf, int c, int h) {
    constexpr int P = kS16Pitch;
    fft16_pass(zr, zi, tw_r, tw_i, buf, c, h);   // slot s: C[4 s + h][c]
#pragma unroll
    for (int s = 0; s < 4; ++s) buf[(4 * s + h) * P + c] = make_float2(zr[s], zi[s]);
    wave_sync();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const float2 v = buf[c * P + 4 * s + h];   // C[c][4 s + h]: row c as sequence c
        zr[s] = v.x;
        zi[s] = v.y;
    }
    wave_sync();   // every lane has read the transpose
    fft16_pass(zr, zi, tw_r, tw_i, buf, c, h);   // slot s: Z[c][4 s + h]
}

// kPersistent: the caller loops over blocks; as in the S = 32 routine, the
// lane index and table pointers are made opaque so that the compiler keeps
// no per-block constant live across the caller's loop.
// (key, position) pairs of the shared-memory argmax: NS slots of 64 lanes,
// padded to a power of two for the halving tree
template <int S>
constexpr int sg_argmax_pairs() {
    int n = 64;
    while (n < SgShape<S>::NS * 64) n *= 2;
    return n;
}

// kArgmax: kArgmaxWave (keys reduced in registers and across the wavefront)
// or kArgmaxLds, the shared-memory scheme Sec. IV compares against: every
// (key, 64 slot + lane) pair goes to argmax_lds (sg_argmax_pairs<S>()
// entries) and is halved in a tree; both choose the same bin.
template <int S, bool kPersistent = false, int kArgmax = kArgmaxWave>
__device__ __forceinline__ void reconstruct_block_sg(const BlockJob& jb, int B, int L, float gamma,
                                                     const BlockTables& tab_in, float* lds,
                                                     uint2* argmax_lds = nullptr) {
    constexpr int G = SgShape<S>::G, NS = SgShape<S>::NS, NL = SgShape<S>::NL;
    const int lane = kPersistent ? opaque((int)(threadIdx.x & 63)) : (int)(threadIdx.x & 63);
    BlockTables tab = tab_in;
    if constexpr (kPersistent) {
        tab.rho_pow = opaque_ptr(tab_in.rho_pow);
        tab.freq_w = opaque_ptr(tab_in.freq_w);
        tab.dft_sg = opaque_ptr(tab_in.dft_sg);
    }
    const bool active = lane < NL;
    // inactive lanes (S = 24) get an in-range (c, h) so that every LDS
    // address they form stays inside the tables
    const int c = active ? lane % S : lane - NL;
    const int h = active ? lane / S : 0;
    const int y0 = jb.by * B - L, x0 = jb.bx * B - L;
    float2* ftab = reinterpret_cast<float2*>(lds);
    float* scr = lds + 2 * S * S;

    // ---- DFT table into LDS (S^2 float2, the same for every block); the
    // S = 16 transform takes its few twiddles from global memory instead
    if constexpr (S != 16) {
        const global_t<const uint64_t>* src = global_ptr(reinterpret_cast<const uint64_t*>(tab.dft_sg));
        uint64_t* dst = reinterpret_cast<uint64_t*>(ftab);
        for (int i = lane; i < S * S; i += 64) dst[i] = src[i];
    }

    // ---- gather and weighting: slot s holds pixel (G s + h, c)
    float xr[NS], wr[NS];
    uint64_t any_known = 0;
    const int x = x0 + c;
    const bool xin = active && (unsigned)x < (unsigned)jb.width;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int m = G * s + h, y = y0 + m;
        const bool in = xin && (unsigned)y < (unsigned)jb.height;
        const int64_t off = in ? (int64_t)y * jb.stride + x : 0;
        const uint8_t kraw = jb.mask[off];
        const float fraw = jb.image[off];
        const float rp = global_ptr(tab.rho_pow)[m * S + c];
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
        // R_w = mu W + DFT2((f~ - mu) w), as in the S = 32 kernel
        float sx = 0.0f, sw = 0.0f;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            sx = fmaf(xr[s], wr[s], sx);
            sw += wr[s];
        }
        sx = wave_sum_f32(sx);
        sw = wave_sum_f32(sw);
        const float mu = sw > 0.0f ? sx / sw : 0.0f;
#pragma unroll
        for (int s = 0; s < NS; ++s) xr[s] = (xr[s] - mu) * wr[s];
        float xi[NS], wi[NS];
        if constexpr (S == 16) {
            // both real tiles in one complex transform z = x + j s w (s the
            // power of two at or below max |x|, as in the S = 24 and 32
            // routines), then split into the two exactly Hermitian spectra:
            // half the sums of two real transforms
            uint32_t amax = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) amax = umax(amax, __float_as_uint(fabsf(xr[s])));
            amax = wave_max_u32(amax);
            const uint32_t sbits = amax & 0x7F800000u;
            const float sc = sbits ? __uint_as_float(sbits) : 1.0f;
#pragma unroll
            for (int s = 0; s < NS; ++s) xi[s] = wr[s] * sc;
            // W16^(h k1), k1 = 1..3, from the table's row F[1]
            float tw_r[4] = {1.0f, 0.0f, 0.0f, 0.0f}, tw_i[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1) table_entry(tab.dft_sg, S + ((h * k1) & (S - 1)), tw_r[k1], tw_i[k1]);
            float2* zs = reinterpret_cast<float2*>(lds);   // the whole area: no table at S = 16
            fft2_s16(xr, xi, tw_r, tw_i, zs, c, h);       // slot s: Z[c][4 s + h]
            // X = (Z + conj Z[-k]) / 2, W = (Z - conj Z[-k]) / (2 j s): bins
            // k and -k read the same pair of values in swapped roles (Z in
            // natural order at zs[k P + l], P = kS16Pitch)
            constexpr int P16 = kS16Pitch;
#pragma unroll
            for (int s = 0; s < NS; ++s) zs[c * P16 + G * s + h] = make_float2(xr[s], xi[s]);
            wave_sync();
            const float hs = 0.5f / sc;
            const int lm = (S - c) & (S - 1);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int km = (S - (G * s + h)) & (S - 1);
                const float2 zo = zs[(G * s + h) * P16 + c];   // this lane's bin
                const float2 zm = zs[km * P16 + lm];
                const float ar = zo.x, ai = zo.y;
                xr[s] = 0.5f * (ar + zm.x);
                xi[s] = 0.5f * (ai - zm.y);
                wr[s] = (ai + zm.y) * hs;
                wi[s] = (zm.x - ar) * hs;
            }
            if (amax == 0) {
                // every known pixel equals mu: X is exactly 0
#pragma unroll
                for (int s = 0; s < NS; ++s) xr[s] = xi[s] = 0.0f;
            }
            wave_sync();   // every lane has read the spectrum
        } else {
            dft2_sg<S>(xr, xr, xi, ftab, scr, c, h, active);
            dft2_sg<S>(wr, wr, wi, ftab, scr, c, h, active);
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
        for (int s = 0; s < NS; ++s) wf[s] = global_ptr(tab.freq_w)[(G * s + h) * S + c];
        // lane i (< S) of tw_re / tw_im holds F[1][i] = exp(-j 2 pi i / S)
        float twx, twy;
        table_entry(tab.dft_sg, S + (lane % S), twx, twy);
        const int tw_re = opaque(__float_as_int(twx)), tw_im = opaque(__float_as_int(twy));
        // the loads of the loop's constants complete here, not at their first
        // use inside the loop (which would put their waits in the loop body)
#pragma unroll
        for (int s = 0; s < NS; ++s) wf[s] = __int_as_float(opaque(__float_as_int(wf[s])));
        wave_sync();
        // W with duplicated rows (and columns when kFullDup): entry (R, C)
        // holds W[R mod S][C mod S]
        constexpr int P = SgShape<S>::P;   // table pitch in float2
        constexpr bool kFullDup = SgShape<S>::kFullDup;
        float2* wtab = reinterpret_cast<float2*>(lds);
        if (active) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int k = G * s + h;
                const float2 wv = make_float2(wr[s], wi[s]);
                wtab[k * P + c] = wv;
                wtab[(k + S) * P + c] = wv;
                if constexpr (kFullDup) {
                    wtab[k * P + c + S] = wv;
                    wtab[(k + S) * P + c + S] = wv;
                }
            }
        }
        // lane constants kept as computed here (the compiler would otherwise
        // re-derive them inside the loop)
        const int lbase = opaque(8 * (h * P + (kFullDup ? c : 0)));   // entry (h, c), or row h
        // the target pixel's (m, n) packed for the phase index u m + v n,
        // scaled by 4 (a bpermute byte address) where no reduction follows
        constexpr int kQs = 64 % S == 0 ? 4 : 1;
        const int tmn = opaque((kQs * tm) | ((kQs * tn) << 16));
        const int c8 = opaque(8 * c);
        const char* wbytes = reinterpret_cast<const char*>(wtab);
        wave_sync();

        // the loop comes in two copies, with and without the argmax log, so
        // that the one without carries no per-iteration branch for it
        auto iterate = [&](auto with_log) {
            for (int it = 0; it < iters; ++it) {
                // objective key (Eq. 16), as in the S = 32 kernel: float32 bits
                // with the 4 low mantissa bits replaced by 15 - slot
                int slot, ln;
                if constexpr (kArgmax == kArgmaxWave) {
                    uint32_t lmax = 0;
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        const float e = fmaf(xr[s], xr[s], xi[s] * xi[s]);
                        const uint32_t key = (__float_as_uint(e * wf[s]) & 0xFFFFFFF0u) | (uint32_t)(15 - s);
                        lmax = umax(lmax, key);
                    }
                    if (!active) lmax = 0;   // real keys carry a slot code >= 4
                    const uint32_t mx = wave_max_u32(lmax);
                    ln = (int)__builtin_ctzll(ballot(lmax == mx));
                    slot = 15 - (int)(mx & 15u);
                } else {
                    constexpr int kPairs = sg_argmax_pairs<S>();
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        const float e = fmaf(xr[s], xr[s], xi[s] * xi[s]);
                        const uint32_t key = (__float_as_uint(e * wf[s]) & 0xFFFFFFF0u) | (uint32_t)(15 - s);
                        argmax_lds[64 * s + lane] = make_uint2(active ? key : 0u, (uint32_t)(64 * s + lane));
                    }
#pragma unroll
                    for (int e = 64 * NS; e < kPairs; e += 64) argmax_lds[e + lane] = make_uint2(0u, 0xFFFFFFFFu);
                    wave_sync();
#pragma unroll
                    for (int half = kPairs / 2; half >= 64; half >>= 1) {
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
                    const int pos = __builtin_amdgcn_readfirstlane((int)argmax_lds[0].y);
                    wave_sync();   // the next iteration overwrites the pairs
                    slot = pos >> 6;
                    ln = pos & 63;
                }
                const int u = G * slot + ln / S, v = ln % S;
                const int idx = u * S + v;
                // the winner's slot is uniform: with few slots, branch on it
                // (scalar) and read two fixed registers instead of selecting
                // among the slots on the vector ALUs; with many, the compiler's
                // relative move is cheaper than the branches
                float pr = 0.0f, pim = 0.0f;
                if constexpr (NS <= 4) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        if (slot == s) {
                            pr = readlane_f(xr[s], ln);
                            pim = readlane_f(xi[s], ln);
                        }
                    }
                } else {
                    pr = readlane_f(xr[slot], ln);
                    pim = readlane_f(xi[slot], ln);
                }
                const float cr = gi * pr, ci = gi * pim;    // gamma * p (Eqs. 10-11)
                if constexpr (decltype(with_log)::value) {
                    if (lane == 0) jb.log[it] = (uint16_t)idx;
                }

                // model: g += gamma p exp(+j 2 pi (u m + v n) / S) on the target.
                // Lane i holds F[1][i mod S]; ds_bpermute reads
                // lane (address / 4) mod 64, so for S dividing 64 the byte
                // address 4 q needs no reduction mod S
                int q4;
                if constexpr (64 % S == 0) q4 = dot2_u16(u | (v << 16), tmn);
                else q4 = 4 * mod_small<S>(dot2_u16(u | (v << 16), tmn));
                const float er = __int_as_float(__builtin_amdgcn_ds_bpermute(q4, tw_re));
                const float ei = __int_as_float(__builtin_amdgcn_ds_bpermute(q4, tw_im));
                acc = fmaf(cr, er, acc);
                acc = fmaf(ci, ei, acc);

                // residual (Eqs. 12, 14-15): bin (G s + h, c) reads entry
                // (G s + h - u + S, c - v + S), i.e. this lane's entry (h, c)
                // moved by a uniform offset, plus G rows per slot; without
                // duplicated columns the column (c - v) mod S wraps per lane
                const float2* wrow;
                if constexpr (kFullDup) {
                    wrow = reinterpret_cast<const float2*>(wbytes + lbase + 8 * ((S - u) * P + (S - v)));
                } else if constexpr ((S & (S - 1)) == 0) {
                    // the row offset is a multiple of 8 S, the wrapped column
                    // offset 8 ((c - v) mod S) lies below it
                    const int col8 = (c8 - 8 * v) & (8 * S - 8);
                    wrow = reinterpret_cast<const float2*>(wbytes + ((lbase + 8 * (S - u) * P) | col8));
                } else {
                    int col = c - v;
                    col += col < 0 ? S : 0;
                    wrow = reinterpret_cast<const float2*>(wbytes + lbase + 8 * ((S - u) * P + col));
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const float2 w = wrow[G * P * s];
                    xr[s] = fmaf(-cr, w.x, xr[s]);
                    xr[s] = fmaf(ci, w.y, xr[s]);
                    xi[s] = fmaf(-cr, w.y, xi[s]);
                    xi[s] = fmaf(-ci, w.x, xi[s]);
                }
            }
        };
        if (jb.log != nullptr) iterate(std::true_type{});
        else iterate(std::false_type{});
        wave_sync();
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
