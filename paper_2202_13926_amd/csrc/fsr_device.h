// fsr_device.h -- device building blocks of the FSR kernels (gfx950, wave64).
//
// Layout conventions used by every kernel in this library (S = 32):
//   * one wavefront reconstructs one support block; lane = c + 32*h with
//     c = lane & 31 and h = lane >> 5;
//   * spatial tile: lane (c, h), slot s (0..15) holds pixel (m = 2s + h, n = c);
//   * spectrum ("bin layout"): lane, slot s holds bin b = 64*s + lane, i.e.
//     (k = 2s + h, l = c), so the bin index b = k*S + l orders lexicographically
//     as (slot, lane) -- the argmax tie rule "smallest b" becomes "first slot,
//     lowest lane".
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fsr_internal.h"

namespace fsr {

constexpr int kSlots = 16;        // bins (or pixels) per lane

// ---------------------------------------------------------------- LDS of a block
constexpr int kLdsFloats = 2 * 64 * kS;   // 4096 floats = 16 KiB

// Transpose scratch of the FFTs: two planes (re, im) of 32 x 32 floats,
// element (r, j) at 33 r + j: rows and columns of a half-wavefront hit 32
// distinct banks and every address is a lane base plus an immediate.
struct Planes {
    static constexpr int kPitch = kS + 1;
    static __device__ __forceinline__ float* re(float* lds) { return lds; }
    static __device__ __forceinline__ float* im(float* lds) { return lds + kS * kPitch; }
    static __device__ __forceinline__ int idx(int r, int j) { return r * kPitch + j; }
};
static_assert(2 * kS * Planes::kPitch <= kLdsFloats, "planes fit the block's LDS");

// Upper 8 KiB of the block's LDS: one spectrum in bin layout, parked while
// the matrix-core path transforms the second.
__device__ __forceinline__ float2* park(float* lds) {
    return reinterpret_cast<float2*>(lds + 2 * kS * kS);
}

// ---------------------------------------------------------------- twiddles
// t[q] = exp(-j 2 pi q / 32).  Built at compile time from the first octant
// only (cos/sin series on [0, pi/4]) and the exact symmetries of the circle,
// so t[32 - q] == conj(t[q]) and the quarter points are exact.
struct Twiddles32 {
    float re[kS];
    float im[kS];
};

constexpr double series_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 16; ++n) {
        term *= -x * x / double((2 * n - 1) * (2 * n));
        sum += term;
    }
    return sum;
}

constexpr double series_sin(double x) {
    double term = x, sum = x;
    for (int n = 1; n < 16; ++n) {
        term *= -x * x / double((2 * n) * (2 * n + 1));
        sum += term;
    }
    return sum;
}

constexpr Twiddles32 make_twiddles32() {
    constexpr double pi = 3.14159265358979323846264338327950288;
    double c[9] = {}, s[9] = {};
    for (int r = 0; r <= 4; ++r) {          // angles 2 pi r / 32 in [0, pi/4]
        c[r] = series_cos(2.0 * pi * r / 32.0);
        s[r] = series_sin(2.0 * pi * r / 32.0);
    }
    c[0] = 1.0;
    s[0] = 0.0;
    s[4] = c[4];                            // cos(pi/4) == sin(pi/4)
    for (int r = 5; r <= 8; ++r) {          // cos(pi/2 - x) = sin(x)
        c[r] = s[8 - r];
        s[r] = c[8 - r];
    }
    Twiddles32 t{};
    for (int q = 0; q < kS; ++q) {
        const int a = q / 8, r = q % 8;     // exp(-j2pi q/32) = (-j)^a exp(-j2pi r/32)
        const float cr = float(c[r]), sr = float(s[r]);
        switch (a) {
        case 0: t.re[q] = cr;  t.im[q] = -sr; break;
        case 1: t.re[q] = -sr; t.im[q] = -cr; break;
        case 2: t.re[q] = -cr; t.im[q] = sr;  break;
        default: t.re[q] = sr; t.im[q] = cr;  break;
        }
    }
    return t;
}

constexpr Twiddles32 kTw = make_twiddles32();

// ---------------------------------------------------------------- complex helpers
__device__ __forceinline__ void cmul(float& re, float& im, float tr, float ti) {
    const float r = fmaf(re, tr, -(im * ti));
    const float i = fmaf(re, ti, im * tr);
    re = r;
    im = i;
}

// In-place 4-point DFT (W4 = -j) of elements (i0, i1, i2, i3).
__device__ __forceinline__ void dft4(float (&re)[16], float (&im)[16], int i0, int i1, int i2,
                                     int i3) {
    const float t0r = re[i0] + re[i2], t0i = im[i0] + im[i2];
    const float t1r = re[i0] - re[i2], t1i = im[i0] - im[i2];
    const float t2r = re[i1] + re[i3], t2i = im[i1] + im[i3];
    const float t3r = re[i1] - re[i3], t3i = im[i1] - im[i3];
    re[i0] = t0r + t2r; im[i0] = t0i + t2i;   // y0
    re[i2] = t0r - t2r; im[i2] = t0i - t2i;   // y2
    re[i1] = t1r + t3i; im[i1] = t1i - t3r;   // y1 = t1 - j t3
    re[i3] = t1r - t3i; im[i3] = t1i + t3r;   // y3 = t1 + j t3
}

// 16-point DFT over the 16 slots of one lane, natural order in and out:
// X[k] = sum_s x[s] exp(-j 2 pi k s / 16).  Radix 4 x 4:
// s = 4 s1 + s2, k = k1 + 4 k2.
__device__ __forceinline__ void fft16(float (&re)[16], float (&im)[16]) {
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) dft4(re, im, s2, s2 + 4, s2 + 8, s2 + 12);   // over s1
    // element 4*k1 + s2 now holds A[s2][k1]; twiddle by w16^(k1 s2) = t32[2 k1 s2]
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
        for (int s2 = 1; s2 < 4; ++s2) {
            const int q = (2 * k1 * s2) & 31;
            cmul(re[4 * k1 + s2], im[4 * k1 + s2], kTw.re[q], kTw.im[q]);
        }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(re, im, 4 * k1, 4 * k1 + 1, 4 * k1 + 2, 4 * k1 + 3);
    // element 4*k1 + k2 holds X[k1 + 4 k2]: transpose the 4x4 index grid
    float tr[16], ti[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            tr[k1 + 4 * k2] = re[4 * k1 + k2];
            ti[k1 + 4 * k2] = im[4 * k1 + k2];
        }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        re[i] = tr[i];
        im[i] = ti[i];
    }
}

// Exchange across the two 32-lane halves: returns, in every lane L, the value
// v held by lane (L & 31) (`lo`) and by lane (L & 31) + 32 (`hi`).
// v_permlane32_swap(a, b) swaps a's upper half with b's lower half, so with
// a = b = v the two results are [v_lo, v_lo] and [v_hi, v_hi].
__device__ __forceinline__ void split_halves(float v, float& lo, float& hi) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    lo = __uint_as_float(r[0]);
    hi = __uint_as_float(r[1]);
}

// 32-point DFT along the slot axis when the even samples of the sequence live
// in lane h = 0 and the odd samples in lane h = 1 (partner lane = lane ^ 32):
// on return lane h holds X[k' + 16 h] in slot k'.  Radix-2 split:
// X[k'] = E[k'] + t^k' O[k'], X[k' + 16] = E[k'] - t^k' O[k'].
__device__ __forceinline__ void dft32_lane_pair(float (&re)[16], float (&im)[16], int h) {
    fft16(re, im);                                      // lane h=0: E, lane h=1: O
    const float sgn = h ? -1.0f : 1.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        float er, ei, orr, oi;
        split_halves(re[k], er, orr);
        split_halves(im[k], ei, oi);
        cmul(orr, oi, kTw.re[k], kTw.im[k]);            // t^k O[k]
        re[k] = fmaf(sgn, orr, er);                     // h=0: E + tO, h=1: E - tO
        im[k] = fmaf(sgn, oi, ei);
    }
}

// ---------------------------------------------------------------- wave reductions
// DPP move whose masked-out lanes read 0, the identity of the unsigned max
// (objective bit patterns are never negative), so the move can fuse into the
// max instruction.
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xf, false);
}

__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Maximum of v over the 64 lanes, returned as a wave-uniform value.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = umax(v, dpp_u32<0xB1>(v));          // quad_perm [1,0,3,2]
    v = umax(v, dpp_u32<0x4E>(v));          // quad_perm [2,3,0,1]
    v = umax(v, dpp_u32<0x141>(v));         // row_half_mirror
    v = umax(v, dpp_u32<0x140>(v));         // row_mirror: every lane holds its row max
    v = umax(v, dpp_u32<0x142, 0xa>(v));    // row_bcast:15 into rows 1, 3
    v = umax(v, dpp_u32<0x143, 0xc>(v));    // row_bcast:31 into rows 2, 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Sum of v over the 64 lanes in a fixed order, returned wave-uniform.  Rows
// masked out of a broadcast step add 0.
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ float dpp_f32_or_zero(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, kRowMask, 0xf, false));
}

__device__ __forceinline__ float wave_sum_f32(float v) {
    v += dpp_f32_or_zero<0xB1>(v);
    v += dpp_f32_or_zero<0x4E>(v);
    v += dpp_f32_or_zero<0x141>(v);
    v += dpp_f32_or_zero<0x140>(v);
    v += dpp_f32_or_zero<0x142, 0xa>(v);
    v += dpp_f32_or_zero<0x143, 0xc>(v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Returns x unchanged but hides how it was computed from the optimiser, so a
// precomputed lane constant (e.g. 8 * lane) is used as is instead of being
// re-derived inside a loop.
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// a * b + c on the 24-bit multiplier (full rate), a wave-uniform.  The
// compiler otherwise widens small products to the quarter-rate 32/64-bit
// multiply-add.
__device__ __forceinline__ int mad_u24(int a, int b, int c) {
    int r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "s"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ int mul_u24(int a, int b) {
    int r;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "s"(a), "v"(b));
    return r;
}

// u a + v b in one instruction (packed 16-bit dot product): uv = u | v << 16
// is wave-uniform, ab = a | b << 16 a lane constant, all four below 2^16 and
// the result below 2^32.
__device__ __forceinline__ int dot2_u16(int uv, int ab) {
    int r;
    asm("v_dot2_u32_u16 %0, %1, %2, 0" : "=v"(r) : "s"(uv), "v"(ab));
    return r;
}

// y with its lowest byte replaced by (y - b) mod 256 and the other bytes
// kept (a sub-dword write): with y's low byte 8 c and b = 8 v, the cyclic
// column (c - v) mod 32 of a 32-entry row of 8-byte elements in one
// instruction.  b is wave-uniform.
__device__ __forceinline__ int sub_low_byte(int y, int b) {
    asm("v_sub_u32_sdwa %0, %0, %1 dst_sel:BYTE_0 dst_unused:UNUSED_PRESERVE src0_sel:DWORD "
        "src1_sel:DWORD"
        : "+v"(y)
        : "s"(b));
    return y;
}

// Orders this wavefront's LDS accesses (its own LDS region only): a fence at
// wavefront scope plus a code-motion barrier.  Workgroup barriers are never
// used by the block routine, so workgroups may hold several wavefronts that
// work on different blocks with different control flow.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ __forceinline__ T* opaque_ptr(T* p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Objects in global memory (never LDS or scratch), addressed with global
// instructions.  A pointer read from memory (a batch descriptor) is otherwise
// generic, and the compiler then uses FLAT instructions, which also count on
// the LDS wait counter: one FLAT store in a loop turns every LDS wait there
// into a full drain.
template <typename T>
using global_t = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ global_t<T>* global_ptr(T* p) {
    return (global_t<T>*)p;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Workgroup index -> block index so that each of the 8 XCDs (which take
// workgroups round-robin) walks one contiguous range of blocks and its L2
// sees the overlapping supports of neighbouring blocks.
__device__ __forceinline__ int64_t xcd_contiguous(int64_t wg, int64_t n) {
    const int64_t per = n / 8, rem = n % 8;
    const int64_t x = wg % 8, j = wg / 8;
    return x * per + (x < rem ? x : rem) + j;
}

}  // namespace fsr
