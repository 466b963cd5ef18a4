/*
 * fsr.h -- C ABI of libfsr, block-parallel Frequency Selective Reconstruction
 * (FSR) on AMD Instinct MI355X (gfx950).
 *
 * FSR (Regensky et al., MMSP 2020, Sec. II) fills the missing pixels of an
 * image sampled under a sparse, non-regular mask.  The image is cut into
 * B x B target blocks; each block plus an L-pixel border (an S x S support,
 * S = B + 2L) is modelled independently as a sparse sum of 2D-DFT basis
 * images, grown greedily in the frequency domain: per iteration an argmax of
 * the frequency-weighted residual energy (Eq. 8), a relaxed projection
 * coefficient (Eqs. 10-11) and a subtraction of the shifted weight spectrum
 * from the residual (Eq. 12).  Unknown target pixels take the real part of
 * the model's inverse DFT; known pixels are copied.
 *
 * Conventions shared by every entry point:
 *   - Images are float32 gray values (any scale; the paper's is [0, 255]),
 *     row-major with a row stride in elements.  Masks are uint8, same shape
 *     and stride, nonzero = known.  Pixels outside the image are unknown.
 *   - All image, mask, output and log pointers are DEVICE pointers owned by
 *     the caller.  The library never frees them.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *     that take a stream are asynchronous with respect to the host; faults of
 *     the work they enqueue surface at a later call or synchronisation.
 *   - Every function returns an fsr_status.  Invalid arguments are detected
 *     on the host before anything is enqueued and leave all outputs
 *     untouched.  fsr_last_error_message() describes the last failure of the
 *     calling thread.  No exception and no abort crosses this interface.
 *   - The DFT convention is forward unnormalised with exp(-j 2 pi (km+ln)/S)
 *     (k pairs with rows); argmax ties go to the smaller bin index k*S + l.
 */
#ifndef FSR_H
#define FSR_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define FSR_API __attribute__((visibility("default")))
#else
#define FSR_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fsr_status {
    FSR_OK = 0,
    FSR_ERR_INVALID_ARG = 1,   /* a pointer, size or parameter is invalid  */
    FSR_ERR_UNSUPPORTED = 2,   /* valid, but outside what the library runs */
    FSR_ERR_OUT_OF_MEMORY = 3, /* a device or host allocation failed       */
    FSR_ERR_BUDGET = 4,        /* request exceeds the configured budget    */
    FSR_ERR_HIP = 5,           /* the HIP runtime reported an error        */
    FSR_ERR_TIMEOUT = 6,       /* a wait ran out of time                   */
    FSR_ERR_NOT_READY = 7      /* polled work has not finished yet         */
} fsr_status;

/* How the two forward block DFTs of Eq. 7 are computed; the iterations are
 * FP32 either way.  FSR_DFT_SPLIT_BF16 (the precision variant) runs them as
 * 32 x 32 DFT-matrix products on the matrix cores (bf16 inputs, FP32
 * accumulation) with every operand split into three bf16 terms (hi + mid +
 * lo, 6 products per real product), which keeps the spectra as accurate as
 * the FP32 FFT's, and sums the model terms of the target pixels with
 * compensation (Kahan). */
enum {
    FSR_DFT_FP32 = 0,        /* FP32 in-register FFT on the vector ALUs    */
    FSR_DFT_SPLIT_BF16 = 1   /* split-bf16 DFT-matrix products on MFMA     */
};

/* Flags of fsr_params.flags. */
enum {
    /* Reduce the argmax of Eq. 8 through a shared-memory (LDS) tree over
     * all S^2 (objective, bin) pairs instead of in registers across the
     * wavefront: the scheme Sec. IV compares the register-based argmax
     * against.  Same choices, hence bitwise the same output; slower.  For
     * fsr_reconstruct with FSR_DFT_FP32 only, at every support (S = 8 then
     * runs one block per wavefront); FSR_ERR_UNSUPPORTED elsewhere. */
    FSR_FLAG_LDS_ARGMAX = 1u
};

/*
 * Method parameters (Sec. II; the paper's defaults B = 4, rho = 0.7,
 * gamma = 0.5 are Sec. IV's).  Validated before any launch:
 *   block >= 1, border >= 0, S = block + 2*border even and <= 32,
 *   iterations >= 0, 0 < rho <= 1, 0 < gamma <= 1 (Sec. II), flags a
 *   combination of FSR_FLAG_*.
 * The library runs S in {8, 16, 24, 32} with block <= 8 (FSR_ERR_UNSUPPORTED
 * otherwise), on the one-image, batched and served paths alike;
 * FSR_DFT_SPLIT_BF16 runs S = 32 only; FSR_FLAG_LDS_ARGMAX runs every
 * support on the one-image path.
 */
typedef struct fsr_params {
    int32_t block;       /* B: target block edge in pixels                  */
    int32_t border;      /* L: border on each side of the target            */
    int32_t iterations;  /* I: fixed number of greedy iterations            */
    float rho;           /* spatial decay factor of the weight, Eq. 5       */
    float gamma;         /* orthogonality deficiency compensation, Eq. 11   */
    int32_t dft;         /* FSR_DFT_*                                       */
    uint32_t flags;      /* FSR_FLAG_* bits                                 */
} fsr_params;

typedef struct fsr_context fsr_context;

/* Library version as major*10000 + minor*100 + patch. */
FSR_API int32_t fsr_version(void);

/* Human-readable name of a status code (static storage); any other value
 * gives "FSR_ERR_UNKNOWN". */
FSR_API const char *fsr_status_string(int32_t status);

/* Message of the calling thread's last failure ("" if none; thread-local,
 * valid until the thread's next failing call). */
FSR_API const char *fsr_last_error_message(void);

/* Fills *params with B = 4, L = 14, I = 100, rho = 0.7, gamma = 0.5, FP32 DFT. */
FSR_API fsr_status fsr_params_default(fsr_params *params);

/* Checks a parameter set without touching any device (see fsr_params). */
FSR_API fsr_status fsr_params_validate(const fsr_params *params);

/* Number of target blocks of a height x width image, ceil(Y/B) * ceil(X/B)
 * (Eq. 13); -1 if an argument is not positive. */
FSR_API int64_t fsr_num_blocks(int32_t height, int32_t width, int32_t block);

/*
 * Creates a context on HIP device `device`: device-resident weight and
 * frequency tables (per support size and rho, built on first use) and the
 * tuning state of the batched path.  A context may be used from one thread
 * at a time (or with external synchronisation).  The caller's current device
 * is restored before returning.
 */
FSR_API fsr_status fsr_context_create(fsr_context **out, int32_t device);
FSR_API fsr_status fsr_context_destroy(fsr_context *ctx);

/*
 * Reconstructs one image (Sec. II; one wavefront per block, Sec. III-A).
 *   image, mask  height x width, row stride `stride` elements (>= width)
 *   out          height x width, row stride `stride`; every pixel is
 *                written: known pixels bit-exactly copied from `image`,
 *                unknown ones set to the real part of the block model
 *                (unclipped; 0 for a block whose support has no known
 *                pixel).  Must not overlap `image` or `mask`.
 *   argmax_log   NULL, or N x I uint16 (N = fsr_num_blocks): the bin
 *                u*S + v chosen by each block at each iteration, block-major;
 *                0xFFFF for every iteration of a block without known pixels.
 * Asynchronous on `stream`.  The call may be captured into a HIP graph once
 * the context holds the tables of this support and rho (built by the first
 * call with them); under capture a missing table is FSR_ERR_UNSUPPORTED and
 * nothing is recorded.
 */
FSR_API fsr_status fsr_reconstruct(fsr_context *ctx, const float *image, const uint8_t *mask,
                           float *out, int32_t height, int32_t width, int64_t stride,
                           const fsr_params *params, uint16_t *argmax_log, void *stream);

/*
 * The sequential variant that reuses reconstructed pixels: the original FSR
 * that Sec. II departs from to make blocks independent.  The result is that
 * of reconstructing the blocks one after another in raster order (block
 * row, then block column) where, in the support of a block, a pixel that is
 * missing but lies in the target of an earlier block takes part with its
 * reconstructed value and the weight reuse_weight * rho^dist (Eq. 5
 * scaled); known pixels keep Eq. 5's weight, and the other missing pixels
 * and those outside the image take no part.
 *   reuse_weight  in [0, 1] (the binding's default is 0.5);
 *                 0 reuses nothing and gives fsr_reconstruct's result
 *   other arguments as for fsr_reconstruct; `out` is also read: the
 *                 blocks read earlier blocks' reconstructions from it
 * Schedule: with r = ceil(L / B), block (by, bx) runs at wavefront step
 * bx + (r + 1) by, one kernel launch per step; the blocks of a step are
 * independent and every block a block reuses ran at an earlier step.  That
 * is (nbx - 1) + (r + 1)(nby - 1) + 1 launches (1,825 for 1920 x 1080 at
 * B = 4, L = 14), each with at most min(nby, ceil(nbx / (r + 1))) blocks, so
 * the call is bound by the latency of one block per step rather than by
 * throughput; a step of at most 512 blocks (over all frames) runs each
 * block on four wavefronts, a larger one on one, with bitwise the same
 * result.  S = 32, FSR_DFT_FP32, no flags (FSR_ERR_UNSUPPORTED
 * otherwise); a reuse_weight outside [0, 1] or NaN is FSR_ERR_INVALID_ARG.
 * Asynchronous on `stream`; capturable into a HIP graph under the same
 * condition as fsr_reconstruct.
 */
FSR_API fsr_status fsr_reconstruct_reuse(fsr_context *ctx, const float *image, const uint8_t *mask,
                                 float *out, int32_t height, int32_t width, int64_t stride,
                                 const fsr_params *params, float reuse_weight,
                                 uint16_t *argmax_log, void *stream);

/*
 * fsr_reconstruct_reuse over n_frames frames of one size (a video's frames),
 * each reconstructed on its own as above; one launch per wavefront step
 * takes that step's blocks of every frame, which fills the device where one
 * frame's at most min(nby, ceil(nbx / (r + 1))) blocks per step cannot.
 *   image, mask, out  frame f starts f * frame_stride elements after frame 0;
 *                     rows `stride` elements apart within a frame;
 *                     frame_stride >= (height - 1) * stride + width (frames
 *                     do not overlap)
 *   argmax_log        NULL, or n_frames x N x I uint16, frame-major
 *   n_frames          1 .. 65535
 * Every frame's output and log are bitwise those of fsr_reconstruct_reuse on
 * it alone.  Errors and stream behaviour as for fsr_reconstruct_reuse.
 */
FSR_API fsr_status fsr_reconstruct_reuse_frames(fsr_context *ctx, const float *image,
                                        const uint8_t *mask, float *out, int32_t n_frames,
                                        int32_t height, int32_t width, int64_t stride,
                                        int64_t frame_stride, const fsr_params *params,
                                        float reuse_weight, uint16_t *argmax_log, void *stream);

/* ------------------------------------------------------------------ batches */

/* One image of a batch.  Pointers are device memory owned by the caller; the
 * meaning of each field is that of the same argument of fsr_reconstruct. */
typedef struct fsr_image_desc {
    const float *image;
    const uint8_t *mask;
    float *out;
    uint16_t *argmax_log;   /* NULL, or fsr_num_blocks(...) x iterations   */
    int32_t height, width;
    int64_t stride;
    int32_t iterations;     /* this image's I (params->iterations ignored)  */
    int32_t reserved;       /* must be 0                                    */
} fsr_image_desc;

/* How the batched kernel distributes blocks over the GPU. */
typedef struct fsr_batch_schedule {
    int32_t waves_per_group;  /* wavefronts per workgroup: 1, 2 or 4          */
    int32_t chunk;            /* 0: one wavefront per block on a plain grid;
                                 1..64: persistent wavefronts take `chunk`
                                 consecutive blocks per pop of a global queue */
    int32_t groups_per_cu;    /* persistent grid = compute units x this (1..32);
                                 ignored when chunk == 0                       */
    int32_t reserved;         /* must be 0                                     */
} fsr_batch_schedule;

/* Device workspace needed for a batch of n_images images (queue head and
 * the device copy of the descriptors).  The caller allocates it. */
FSR_API fsr_status fsr_batched_workspace_size(int32_t n_images, size_t *bytes);

/*
 * Reconstructs n_images images of any sizes and iteration counts in one
 * kernel launch (plus a one-thread queue reset when the schedule uses the
 * queue).  The blocks of all images form one index space ordered by
 * decreasing iteration count, so the heaviest blocks start first.  Every
 * block runs the same arithmetic as in fsr_reconstruct: each image's output
 * and log are bitwise identical to a fsr_reconstruct call on it alone.
 *   descs      HOST array of n_images descriptors (copied; may be reused
 *              once the call returns)
 *   params     block, border, rho, gamma, dft shared by all images
 *   schedule   NULL: the schedule fsr_batch_autotune chose for a batch of
 *              this size class, support and dft mode on this context, else
 *              a plain grid
 *   workspace  device memory of >= fsr_batched_workspace_size bytes; it must
 *              not be in use by another call that has not completed
 * Asynchronous on `stream`; must not be called while `stream` is being
 * captured (use fsr_batch_graph_create for graphs).
 */
FSR_API fsr_status fsr_reconstruct_batched(fsr_context *ctx, const fsr_image_desc *descs,
                                           int32_t n_images, const fsr_params *params,
                                           const fsr_batch_schedule *schedule, void *workspace,
                                           size_t workspace_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * reconstruction as fsr_reconstruct_batched with the same schedule argument,
 * bitwise the same outputs and logs, without a caller workspace and without
 * allocating anything.  The queue head and the descriptor table live in a
 * fixed device array of the library, FSR_NOALLOC_WORKSPACE_BYTES bytes on
 * each device (looked up when a context is created there, held until the
 * process ends), so a call takes at most FSR_NOALLOC_MAX_IMAGES images
 * (FSR_ERR_INVALID_ARG beyond).  The context must already hold the tables
 * of this support and rho (built by an earlier fsr_reconstruct or
 * fsr_reconstruct_batched call with them); else FSR_ERR_UNSUPPORTED and
 * nothing is enqueued.  Every call on a device shares that device's array
 * and overwrites what the previous call left there (the queue head is reset
 * by each launch): calls whose work can overlap on one device (other
 * streams, other contexts or threads) race, and the caller must order them,
 * e.g. on one stream.  Asynchronous on `stream`.
 */
#define FSR_NOALLOC_MAX_IMAGES 64
#define FSR_NOALLOC_WORKSPACE_BYTES (256 + 64 * FSR_NOALLOC_MAX_IMAGES)
FSR_API fsr_status fsr_reconstruct_batched_noalloc(fsr_context *ctx, const fsr_image_desc *descs,
                                                   int32_t n_images, const fsr_params *params,
                                                   const fsr_batch_schedule *schedule, void *stream);

/* Times the batch under candidate schedules: a fixed list plus persistent
 * schedules sized to the number of workgroups a compute unit holds for this
 * support and dft mode.  Each run reconstructs the batch, so outputs are
 * written.  Stores the fastest on the context for this batch's size class,
 * support and dft mode and returns it in *best.  Blocks the host until the
 * timing runs finish. */
FSR_API fsr_status fsr_batch_autotune(fsr_context *ctx, const fsr_image_desc *descs,
                                      int32_t n_images, const fsr_params *params,
                                      void *workspace, size_t workspace_bytes, void *stream,
                                      fsr_batch_schedule *best);

/*
 * The context's autotune results as text, to be kept across processes:
 * JSON of the form
 *   {"format": "fsr-batch-tuning-1", "arch": "<gcnArchName>", "cus": <CUs>,
 *    "entries": [[<size-class key>, waves_per_group, chunk, groups_per_cu], ...]}
 * where the key packs log2 of the batch's work, the support, the dft mode
 * and the largest iteration count.  Export writes a NUL-terminated string
 * of *len bytes (NUL included) into buf when cap suffices (buf NULL: only
 * *len is set; cap too small: FSR_ERR_INVALID_ARG with *len set).  Import
 * reads exactly that form, checks every schedule as fsr_reconstruct_batched
 * does and merges the entries into the context; text from another kind of
 * device (arch or CU count) is FSR_ERR_UNSUPPORTED, malformed text
 * FSR_ERR_INVALID_ARG, and nothing is merged then.
 */
FSR_API fsr_status fsr_batch_tuning_export(fsr_context *ctx, char *buf, size_t cap, size_t *len);
FSR_API fsr_status fsr_batch_tuning_import(fsr_context *ctx, const char *json);

/* A batch captured once into a HIP graph (queue reset + batched kernel) and
 * replayed many times: the images' device buffers are fixed at creation and
 * their contents are read at each replay.  Creation uploads the descriptors
 * synchronously.  The context, the workspace and every buffer must outlive
 * the graph; replays of one graph must not overlap. */
typedef struct fsr_batch_graph fsr_batch_graph;
FSR_API fsr_status fsr_batch_graph_create(fsr_context *ctx, const fsr_image_desc *descs,
                                          int32_t n_images, const fsr_params *params,
                                          const fsr_batch_schedule *schedule, void *workspace,
                                          size_t workspace_bytes, fsr_batch_graph **out);
FSR_API fsr_status fsr_batch_graph_launch(fsr_batch_graph *graph, void *stream);
FSR_API fsr_status fsr_batch_graph_destroy(fsr_batch_graph *graph);

/* ------------------------------------------------------------------ serving */

/* Where the pixels of a request live. */
enum {
    FSR_MEM_HOST = 0,     /* host memory (pinned memory gives asynchronous copies) */
    FSR_MEM_DEVICE = 1    /* device memory of the server's device               */
};

/* How a server schedules admitted requests. */
enum {
    FSR_SERVE_CONTINUOUS = 0,  /* every launch takes all admitted, uploaded
                                  requests (up to max_batch) as one batch; up to
                                  `streams` launches overlap on the device while
                                  new requests are admitted and uploaded       */
    FSR_SERVE_FIFO = 1         /* reference loop: one request per launch, in
                                  arrival order, upload and reconstruction in
                                  one stream                                   */
};

typedef struct fsr_server_config {
    size_t hbm_budget;      /* device bytes for request buffers; each admitted
                               request holds image, mask and output
                               (9 bytes per pixel, 256-byte aligned parts)     */
    int32_t max_inflight;   /* requests admitted at once (1..4096)           */
    int32_t max_batch;      /* requests per launch (1..max_inflight)          */
    int32_t streams;        /* compute streams, 1 or 2                         */
    int32_t mode;           /* FSR_SERVE_*                                     */
    int32_t reserved[4];    /* must be 0                                       */
} fsr_server_config;

/* One frame to reconstruct.  The buffers must stay valid and unchanged until
 * the request is done (fsr_server_poll reports it). */
typedef struct fsr_request {
    const float *image;
    const uint8_t *mask;
    int32_t height, width;
    int64_t stride;         /* row stride of image and mask, elements          */
    int32_t iterations;     /* I for this frame                                */
    int32_t memory;         /* FSR_MEM_HOST or FSR_MEM_DEVICE                  */
} fsr_request;

typedef struct fsr_server_stats {
    uint64_t submitted, admitted, completed, released, launches, rejected;
    uint64_t bytes_in_use, peak_bytes_in_use;
    double busy_s;          /* time with at least one launch in flight         */
} fsr_server_stats;

typedef struct fsr_server fsr_server;

/*
 * Creates a server with its own scheduler thread, copy stream, compute
 * streams and a device arena of cfg->hbm_budget bytes on the context's
 * device (method parameters are fixed per server; per-request I comes with
 * each request).  Requests are admitted in arrival order while the arena and
 * the in-flight limit allow; an admitted request is copied into the arena
 * and reconstructed there, and its output stays in device memory until
 * fetched or released.  Each result is bitwise identical to fsr_reconstruct
 * on the same frame, whatever else shares its launch.  While a batch runs, a
 * second one starts beside it on the other compute stream only if it is at
 * most a quarter of the running batch's work.  The compute streams are
 * created with a CU mask enabling every compute unit (each then has a
 * hardware queue of its own) and therefore synchronise with the legacy null
 * stream.
 */
FSR_API fsr_status fsr_server_create(fsr_context *ctx, const fsr_params *params,
                                     const fsr_server_config *cfg, fsr_server **out);

/* Queues a request; returns immediately with a ticket.  FSR_ERR_BUDGET if the
 * frame alone exceeds the arena, FSR_ERR_INVALID_ARG for bad fields. */
FSR_API fsr_status fsr_server_submit(fsr_server *srv, const fsr_request *req, uint64_t *ticket);

/* *done = 1 once the reconstruction of `ticket` has finished on the device. */
FSR_API fsr_status fsr_server_poll(fsr_server *srv, uint64_t ticket, int32_t *done);

/* Blocks until `ticket` is done or timeout_ms passes (FSR_ERR_TIMEOUT);
 * timeout_ms < 0 waits without limit. */
FSR_API fsr_status fsr_server_wait(fsr_server *srv, uint64_t ticket, int32_t timeout_ms);

/* Copies a finished result into `out` (row stride out_stride elements, host
 * or device memory as given) and releases the request's arena space.
 * FSR_ERR_NOT_READY if it has not finished. */
FSR_API fsr_status fsr_server_result(fsr_server *srv, uint64_t ticket, float *out,
                                     int64_t out_stride, int32_t memory);

/* Releases a finished request without copying its result. */
FSR_API fsr_status fsr_server_release(fsr_server *srv, uint64_t ticket);

/* Timestamps (seconds on the host's steady clock) of a request: submission,
 * admission, launch and observed completion (completion is observed by the
 * scheduler thread, which polls the device every ~20 us while busy). */
FSR_API fsr_status fsr_server_timing(fsr_server *srv, uint64_t ticket, double *submit_s,
                                     double *admit_s, double *launch_s, double *done_s);

FSR_API fsr_status fsr_server_get_stats(fsr_server *srv, fsr_server_stats *out);

/* Waits for every admitted request to finish, stops the scheduler thread and
 * frees the arena.  Requests still queued are dropped. */
FSR_API fsr_status fsr_server_destroy(fsr_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* FSR_H */
