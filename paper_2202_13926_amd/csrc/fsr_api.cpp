// fsr_api.cpp -- host side of the C ABI declared in include/fsr.h.
//
// Argument validation happens before any HIP call so that invalid calls are
// rejected on machines without a GPU and leave every output untouched.
#include "fsr.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fsr_internal.h"
#include "fsr_runtime.h"

namespace {

thread_local std::string g_last_error;

fsr_status fail(fsr_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

}  // namespace

namespace fsr {

fsr_status errorf(fsr_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

fsr_status set_error(fsr_status st, const char* msg) {
    g_last_error = msg;
    return st;
}

fsr_status hip_fail(hipError_t e, const char* what) {
    return fail(FSR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

DeviceGuard::DeviceGuard(int device) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != device) {
        err_ = hipSetDevice(device);
        changed_ = err_ == hipSuccess;
    }
}

DeviceGuard::~DeviceGuard() {
    if (changed_ && prev_ >= 0) (void)hipSetDevice(prev_);
}

fsr_status validate_params(const fsr_params* p) {
    if (!p) return fail(FSR_ERR_INVALID_ARG, "params is NULL");
    if (p->block < 1) return fail(FSR_ERR_INVALID_ARG, "block must be >= 1 (got %d)", p->block);
    if (p->border < 0) return fail(FSR_ERR_INVALID_ARG, "border must be >= 0 (got %d)", p->border);
    const int64_t S = (int64_t)p->block + 2 * (int64_t)p->border;
    if (S > 32 || S % 2 != 0)
        return fail(FSR_ERR_INVALID_ARG, "support B + 2L = %lld must be even and <= 32", (long long)S);
    if (p->iterations < 0)
        return fail(FSR_ERR_INVALID_ARG, "iterations must be >= 0 (got %d)", p->iterations);
    if (!(p->rho > 0.0f && p->rho <= 1.0f))
        return fail(FSR_ERR_INVALID_ARG, "rho must lie in (0, 1] (got %g)", (double)p->rho);
    if (!(p->gamma > 0.0f && p->gamma <= 1.0f))
        return fail(FSR_ERR_INVALID_ARG, "gamma must lie in (0, 1] (got %g)", (double)p->gamma);
    if (p->dft != FSR_DFT_FP32 && p->dft != FSR_DFT_SPLIT_BF16)
        return fail(FSR_ERR_INVALID_ARG, "unknown dft mode %d", p->dft);
    if ((p->flags & ~(uint32_t)FSR_FLAG_LDS_ARGMAX) != 0)
        return fail(FSR_ERR_INVALID_ARG, "unknown flags 0x%x", p->flags);
    return FSR_OK;
}

fsr_status check_supported(const fsr_params* p) {
    const int S = p->block + 2 * p->border;
    if (S != 8 && S != 16 && S != 24 && S != kS)
        return fail(FSR_ERR_UNSUPPORTED, "the library runs support sizes 8, 16, 24 and 32 (got %d)", S);
    if (p->block > 8) return fail(FSR_ERR_UNSUPPORTED, "the library runs block <= 8 (got %d)", p->block);
    return FSR_OK;
}

static bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + nb && pb < pa + na;
}

fsr_status validate_image(const float* image, const uint8_t* mask, const float* out, int32_t height,
                          int32_t width, int64_t stride, int32_t block) {
    if (!image || !mask || !out) return fail(FSR_ERR_INVALID_ARG, "image, mask and out must be non-NULL");
    if (height < 1 || width < 1)
        return fail(FSR_ERR_INVALID_ARG, "image size must be positive (got %d x %d)", height, width);
    if (stride < width)
        return fail(FSR_ERR_INVALID_ARG, "stride %lld is smaller than width %d", (long long)stride, width);
    if (stride > (int64_t(1) << 40) / height) return fail(FSR_ERR_INVALID_ARG, "image too large");
    const int64_t n_blocks = fsr_num_blocks(height, width, block);
    if (n_blocks > 0x7fffffff) return fail(FSR_ERR_UNSUPPORTED, "more than 2^31-1 blocks");
    const size_t extent = (size_t)((int64_t)(height - 1) * stride + width);
    if (ranges_overlap(out, extent * sizeof(float), image, extent * sizeof(float)) ||
        ranges_overlap(out, extent * sizeof(float), mask, extent))
        return fail(FSR_ERR_INVALID_ARG, "out must not overlap image or mask");
    return FSR_OK;
}

// ---------------------------------------------------------------- tables
// Spatial weight rho^dist from the support centre (S-1)/2 (Eq. 5, before
// masking) and frequency weight w_f (Eq. 9), evaluated in double and rounded
// once to float.
static std::vector<float> host_rho_pow(int S, float rho) {
    std::vector<float> t((size_t)S * S);
    const double c = 0.5 * (S - 1);
    for (int m = 0; m < S; ++m)
        for (int n = 0; n < S; ++n) {
            const double d = std::sqrt((m - c) * (m - c) + (n - c) * (n - c));
            t[(size_t)m * S + n] = (float)std::pow((double)rho, d);
        }
    return t;
}

static std::vector<float> host_freq_w(int S) {
    std::vector<float> t((size_t)S * S);
    const double half = 0.5 * S;
    for (int k = 0; k < S; ++k)
        for (int l = 0; l < S; ++l) {
            const double kt = half - std::fabs(k - half), lt = half - std::fabs(l - half);
            const double a = 1.0 - std::sqrt(2.0) * std::sqrt((kt * kt + lt * lt) / (double)(S * S));
            t[(size_t)k * S + l] = (float)(a * a);
        }
    return t;
}

// DFT table of the smaller supports: F[m][k] = exp(-j 2 pi m k / S) as float2,
// from twiddles t[q] = exp(-j 2 pi q / S) computed on [0, pi] and mirrored,
// so that t[S - q] is exactly conj(t[q]) and t[0], t[S/4], t[S/2] are exact.
static std::vector<float> host_dft_sg(int S) {
    const double pi = 3.14159265358979323846;
    std::vector<double> tr(S), ti(S);
    for (int q = 0; 2 * q <= S; ++q) {
        double c = std::cos(2.0 * pi * q / S), s = std::sin(2.0 * pi * q / S);
        if (q == 0) { c = 1.0; s = 0.0; }
        if (4 * q == S) { c = 0.0; s = 1.0; }
        if (2 * q == S) { c = -1.0; s = 0.0; }
        tr[q] = c;
        ti[q] = -s;
        if (q > 0 && 2 * q < S) {
            tr[S - q] = c;
            ti[S - q] = s;
        }
    }
    std::vector<float> t((size_t)2 * S * S);
    for (int m = 0; m < S; ++m)
        for (int k = 0; k < S; ++k) {
            const int q = (m * k) % S;
            t[2 * ((size_t)m * S + k)] = (float)tr[q];
            t[2 * ((size_t)m * S + k) + 1] = (float)ti[q];
        }
    return t;
}

// bf16 bit pattern nearest to a float (round to nearest, ties to even).
static uint16_t bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, sizeof u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

static float bf16_value(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, sizeof f);
    return f;
}

// Operands of the DFT-matrix products of the split-bf16 transform.  The
// 32-point DFT matrix F[m][k] = exp(-j 2 pi m k / 32) (exactly symmetric in
// sign and index) is split per entry into bf16 terms: term 0 = bf16(F),
// term i = bf16 of what terms 0 .. i-1 leave.  Entry [part][q][term][lane][v]
// is part (Re F, Im F) of
// F[16 q + 8 (v / 4) + 4 (lane / 32) + v % 4][lane % 32]: the B operand of
// K-step q of both matrix products in the device transform.
static void dft_table(std::vector<uint16_t>& t) {
    const double pi = 3.14159265358979323846;
    double fr[kS], fi[kS];                   // exp(-j 2 pi q / 32), exact symmetries
    for (int q = 0; q < kS; ++q) {
        const int a = q / 8, r = q % 8;
        const int rr = r <= 4 ? r : 8 - r;
        double c = std::cos(2.0 * pi * rr / kS), sn = std::sin(2.0 * pi * rr / kS);
        if (rr == 4) sn = c;
        if (r > 4) std::swap(c, sn);
        switch (a) {
        case 0: fr[q] = c; fi[q] = -sn; break;
        case 1: fr[q] = -sn; fi[q] = -c; break;
        case 2: fr[q] = -c; fi[q] = sn; break;
        default: fr[q] = sn; fi[q] = c; break;
        }
    }
    t.assign(kMfmaDftElems, 0);
    for (int part = 0; part < 2; ++part)
        for (int q = 0; q < 2; ++q)
            for (int lane = 0; lane < 64; ++lane)
                for (int v = 0; v < 8; ++v) {
                    const int n = 16 * q + 8 * (v / 4) + 4 * (lane / 32) + v % 4, l = lane % 32;
                    const int e = (n * l) % kS;
                    const double f = part == 0 ? fr[e] : fi[e];
                    double rest = f;
                    for (int term = 0; term < kMfmaMaxTerms; ++term) {
                        const uint16_t b = bf16_bits((float)rest);
                        t[((size_t)((part * 2 + q) * kMfmaMaxTerms + term) * 64 + lane) * 8 + v] = b;
                        rest -= (double)bf16_value(b);
                    }
                }
}

}  // namespace fsr

using namespace fsr;

struct fsr_context {
    int device = 0;
    std::mutex mu;
    std::mutex batch_mu;
    std::map<int, float*> freq_w;          // keyed by S
    std::map<int, float*> dft_sg;          // DFT tables of the smaller supports, by S
    uint16_t* mfma_tab = nullptr;          // split-bf16 DFT operands (S = 32)
    std::map<uint64_t, float*> rho_pow;    // keyed by S << 32 | bits of rho
    fsr::BatchState batch;
};

namespace fsr {

// Uploads a host table once; `slot` caches the device copy and `make` builds
// the host values only when the table is missing.  With may_build false a
// missing table is an error and no HIP call is made (stream capture).
template <typename T, typename Make>
static fsr_status device_table(T** slot, bool may_build, const char* what, int S, float rho, Make make) {
    if (*slot) return FSR_OK;
    if (!may_build)
        return fail(FSR_ERR_UNSUPPORTED,
                    "%s for support %d and rho %g is not on the context yet: make one call with these "
                    "parameters outside stream capture first", what, S, (double)rho);
    const std::vector<T> h = make();
    T* d = nullptr;
    hipError_t e = hipMalloc(&d, h.size() * sizeof(T));
    if (e != hipSuccess) return fail(FSR_ERR_OUT_OF_MEMORY, "hipMalloc(%s): %s", what, hipGetErrorString(e));
    e = hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, what);
    }
    *slot = d;
    return FSR_OK;
}

fsr_status context_tables(fsr_context* ctx, int S, float rho, BlockTables* out, bool may_build) {
    std::lock_guard<std::mutex> lock(ctx->mu);
    fsr_status st;
    *out = BlockTables{};
    uint32_t bits;
    std::memcpy(&bits, &rho, sizeof bits);
    const uint64_t key = ((uint64_t)(uint32_t)S << 32) | bits;
    if (!may_build) {
        // look the tables up without inserting (a map insertion allocates)
        const bool have = ctx->freq_w.count(S) && ctx->rho_pow.count(key) &&
                          (S == kS ? ctx->mfma_tab != nullptr : ctx->dft_sg.count(S) != 0);
        if (!have)
            return fail(FSR_ERR_UNSUPPORTED,
                        "the tables of support %d and rho %g are not on the context yet: make one "
                        "call with these parameters that may build them first", S, (double)rho);
    }
    if ((st = device_table(&ctx->freq_w[S], may_build, "frequency table", S, rho,
                           [&] { return host_freq_w(S); })) != FSR_OK)
        return st;
    if (S == kS) {
        st = device_table(&ctx->mfma_tab, may_build, "dft table", S, rho, [] {
            std::vector<uint16_t> t;
            dft_table(t);
            return t;
        });
    } else {
        st = device_table(&ctx->dft_sg[S], may_build, "dft table", S, rho, [&] { return host_dft_sg(S); });
    }
    if (st != FSR_OK) return st;
    if ((st = device_table(&ctx->rho_pow[key], may_build, "weight table", S, rho,
                           [&] { return host_rho_pow(S, rho); })) != FSR_OK)
        return st;
    out->rho_pow = ctx->rho_pow[key];
    out->freq_w = ctx->freq_w[S];
    out->mfma_dft = S == kS ? ctx->mfma_tab : nullptr;
    out->dft_sg = S == kS ? nullptr : reinterpret_cast<const float2*>(ctx->dft_sg[S]);
    return FSR_OK;
}

int context_device(const fsr_context* ctx) { return ctx->device; }
BatchState& context_batch(fsr_context* ctx) { return ctx->batch; }
std::mutex& context_mutex(fsr_context* ctx) { return ctx->mu; }
std::mutex& context_batch_mutex(fsr_context* ctx) { return ctx->batch_mu; }

}  // namespace fsr

extern "C" {

int32_t fsr_version(void) { return 100; }

const char* fsr_status_string(int32_t s) {
    switch (s) {
    case FSR_OK: return "FSR_OK";
    case FSR_ERR_INVALID_ARG: return "FSR_ERR_INVALID_ARG";
    case FSR_ERR_UNSUPPORTED: return "FSR_ERR_UNSUPPORTED";
    case FSR_ERR_OUT_OF_MEMORY: return "FSR_ERR_OUT_OF_MEMORY";
    case FSR_ERR_BUDGET: return "FSR_ERR_BUDGET";
    case FSR_ERR_HIP: return "FSR_ERR_HIP";
    case FSR_ERR_TIMEOUT: return "FSR_ERR_TIMEOUT";
    case FSR_ERR_NOT_READY: return "FSR_ERR_NOT_READY";
    }
    return "FSR_ERR_UNKNOWN";
}

const char* fsr_last_error_message(void) { return g_last_error.c_str(); }

fsr_status fsr_params_default(fsr_params* p) {
    if (!p) return fail(FSR_ERR_INVALID_ARG, "params is NULL");
    p->block = 4;
    p->border = 14;
    p->iterations = 100;
    p->rho = 0.7f;
    p->gamma = 0.5f;
    p->dft = FSR_DFT_FP32;
    p->flags = 0;
    return FSR_OK;
}

fsr_status fsr_params_validate(const fsr_params* p) { return validate_params(p); }

int64_t fsr_num_blocks(int32_t height, int32_t width, int32_t block) {
    if (height < 1 || width < 1 || block < 1) return -1;
    return (int64_t)((height + block - 1) / block) * (int64_t)((width + block - 1) / block);
}

fsr_status fsr_context_create(fsr_context** out, int32_t device) {
    if (!out) return fail(FSR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n)
        return fail(FSR_ERR_INVALID_ARG, "device %d out of range (%d devices)", device, n);
    {
        // the device address of the fixed workspace of
        // fsr_reconstruct_batched_noalloc, looked up once per device
        DeviceGuard g(device);
        if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
        if ((e = static_workspace_init(device)) != hipSuccess) return hip_fail(e, "hipGetSymbolAddress");
    }
    fsr_context* ctx = new (std::nothrow) fsr_context();
    if (!ctx) return fail(FSR_ERR_OUT_OF_MEMORY, "context allocation failed");
    ctx->device = device;
    *out = ctx;
    return FSR_OK;
}

fsr_status fsr_context_destroy(fsr_context* ctx) {
    if (!ctx) return FSR_OK;
    {
        DeviceGuard g(ctx->device);
        release_batch_state(ctx->batch);
        for (auto& kv : ctx->freq_w)
            if (kv.second) (void)hipFree(kv.second);
        for (auto& kv : ctx->dft_sg)
            if (kv.second) (void)hipFree(kv.second);
        if (ctx->mfma_tab) (void)hipFree(ctx->mfma_tab);
        for (auto& kv : ctx->rho_pow)
            if (kv.second) (void)hipFree(kv.second);
    }
    delete ctx;
    return FSR_OK;
}

}  // extern "C"

namespace fsr {

// The launch description of one image; the caller has validated every argument.
static PlainLaunch plain_launch(const float* image, const uint8_t* mask, float* out, int32_t height,
                                int32_t width, int64_t stride, const fsr_params* params,
                                uint16_t* argmax_log) {
    PlainLaunch p{};
    p.img.image = image;
    p.img.mask = mask;
    p.img.out = out;
    p.img.argmax_log = argmax_log;
    p.img.height = height;
    p.img.width = width;
    p.img.stride = stride;
    p.img.iterations = params->iterations;
    p.img.nbx = (width + params->block - 1) / params->block;
    p.img.block_begin = 0;
    p.block = params->block;
    p.border = params->border;
    p.support = params->block + 2 * params->border;
    p.gamma = params->gamma;
    p.n_blocks = fsr_num_blocks(height, width, params->block);
    p.dft = params->dft == FSR_DFT_SPLIT_BF16 ? 1 : 0;
    p.lds_argmax = (params->flags & FSR_FLAG_LDS_ARGMAX) ? 1 : 0;
    return p;
}

}  // namespace fsr

extern "C" {

fsr_status fsr_reconstruct(fsr_context* ctx, const float* image, const uint8_t* mask, float* out,
                           int32_t height, int32_t width, int64_t stride, const fsr_params* params,
                           uint16_t* argmax_log, void* stream) {
    if (!ctx) return fail(FSR_ERR_INVALID_ARG, "context is NULL");
    fsr_status st = validate_params(params);
    if (st != FSR_OK) return st;
    if ((st = check_supported(params)) != FSR_OK) return st;
    if ((st = validate_image(image, mask, out, height, width, stride, params->block)) != FSR_OK)
        return st;

    if ((params->flags & FSR_FLAG_LDS_ARGMAX) && params->dft != FSR_DFT_FP32)
        return fail(FSR_ERR_UNSUPPORTED, "the LDS argmax runs with FSR_DFT_FP32 only");
    const int S = params->block + 2 * params->border;
    if (S != kS && (params->dft != FSR_DFT_FP32 || (params->flags & ~FSR_FLAG_LDS_ARGMAX) != 0))
        return fail(FSR_ERR_UNSUPPORTED, "support %d runs with FSR_DFT_FP32 only", S);

    DeviceGuard g(ctx->device);
    if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
    // under stream capture only a kernel launch may be recorded: the tables
    // must already be on the context
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t ce = hipStreamIsCapturing((hipStream_t)stream, &cap);
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamIsCapturing");
    PlainLaunch p = plain_launch(image, mask, out, height, width, stride, params, argmax_log);
    if ((st = context_tables(ctx, S, params->rho, &p.tab, cap == hipStreamCaptureStatusNone)) != FSR_OK)
        return st;
    hipError_t e = launch_plain(p, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch of the reconstruction kernel");
    return FSR_OK;
}

}  // extern "C"

namespace fsr {

// The reuse variant over n_frames frames of one size, frame_stride elements
// apart (1 and 0 for a single frame); validates everything first.
static fsr_status reuse_call(fsr_context* ctx, const float* image, const uint8_t* mask, float* out,
                             int32_t n_frames, int32_t height, int32_t width, int64_t stride,
                             int64_t frame_stride, const fsr_params* params, float reuse_weight,
                             uint16_t* argmax_log, void* stream) {
    if (!ctx) return fail(FSR_ERR_INVALID_ARG, "context is NULL");
    fsr_status st = validate_params(params);
    if (st != FSR_OK) return st;
    if (!(reuse_weight >= 0.0f && reuse_weight <= 1.0f))
        return fail(FSR_ERR_INVALID_ARG, "reuse_weight must lie in [0, 1] (got %g)", (double)reuse_weight);
    if ((st = check_supported(params)) != FSR_OK) return st;
    if ((st = validate_image(image, mask, out, height, width, stride, params->block)) != FSR_OK)
        return st;
    if (n_frames < 1 || n_frames > 65535)
        return fail(FSR_ERR_INVALID_ARG, "n_frames must lie in [1, 65535] (got %d)", n_frames);
    if (n_frames > 1) {
        const int64_t frame_extent = (int64_t)(height - 1) * stride + width;
        if (frame_stride < frame_extent)
            return fail(FSR_ERR_INVALID_ARG, "frame_stride %lld is smaller than one frame (%lld elements)",
                        (long long)frame_stride, (long long)frame_extent);
        if (frame_stride > ((int64_t)1 << 40) / n_frames) return fail(FSR_ERR_INVALID_ARG, "frames too large");
        const size_t extent = (size_t)((int64_t)(n_frames - 1) * frame_stride + frame_extent);
        if (ranges_overlap(out, extent * sizeof(float), image, extent * sizeof(float)) ||
            ranges_overlap(out, extent * sizeof(float), mask, extent))
            return fail(FSR_ERR_INVALID_ARG, "out must not overlap image or mask");
    }
    const int S = params->block + 2 * params->border;
    if (S != kS || params->dft != FSR_DFT_FP32 || params->flags != 0)
        return fail(FSR_ERR_UNSUPPORTED, "the reuse variant runs at S = 32 with FSR_DFT_FP32 and no flags "
                                         "only (got S = %d)", S);
    if (reuse_steps(height, width, params->block, params->border) > 0x7fffffff)
        return fail(FSR_ERR_UNSUPPORTED, "more than 2^31-1 wavefront steps");

    DeviceGuard g(ctx->device);
    if (g.error() != hipSuccess) return hip_fail(g.error(), "hipSetDevice");
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t ce = hipStreamIsCapturing((hipStream_t)stream, &cap);
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamIsCapturing");
    PlainLaunch p = plain_launch(image, mask, out, height, width, stride, params, argmax_log);
    if ((st = context_tables(ctx, S, params->rho, &p.tab, cap == hipStreamCaptureStatusNone)) != FSR_OK)
        return st;
    hipError_t e = launch_reuse(p, reuse_weight, n_frames, n_frames > 1 ? frame_stride : 0,
                                (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch of the reuse-variant kernels");
    return FSR_OK;
}

}  // namespace fsr

extern "C" {

fsr_status fsr_reconstruct_reuse(fsr_context* ctx, const float* image, const uint8_t* mask, float* out,
                                 int32_t height, int32_t width, int64_t stride, const fsr_params* params,
                                 float reuse_weight, uint16_t* argmax_log, void* stream) {
    return reuse_call(ctx, image, mask, out, 1, height, width, stride, 0, params, reuse_weight, argmax_log,
                      stream);
}

fsr_status fsr_reconstruct_reuse_frames(fsr_context* ctx, const float* image, const uint8_t* mask,
                                        float* out, int32_t n_frames, int32_t height, int32_t width,
                                        int64_t stride, int64_t frame_stride, const fsr_params* params,
                                        float reuse_weight, uint16_t* argmax_log, void* stream) {
    return reuse_call(ctx, image, mask, out, n_frames, height, width, stride, frame_stride, params,
                      reuse_weight, argmax_log, stream);
}

}  // extern "C"
