"""ctypes binding of libfsr (include/fsr.h): argument marshalling only.

Every step of the reconstruction runs in the HIP kernels of libfsr.so; this
module checks tensor shapes, dtypes and devices, passes raw device pointers
and the current HIP stream, and turns status codes into exceptions.  If the
library is missing it raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfsr.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "fsr.h")

FSR_OK = 0
FSR_ERR_INVALID_ARG = 1
FSR_ERR_UNSUPPORTED = 2
FSR_ERR_OUT_OF_MEMORY = 3
FSR_ERR_BUDGET = 4
FSR_ERR_HIP = 5
FSR_ERR_TIMEOUT = 6
FSR_ERR_NOT_READY = 7

FSR_DFT_FP32 = 0
FSR_DFT_SPLIT_BF16 = 1

FSR_FLAG_LDS_ARGMAX = 1

FSR_NOALLOC_MAX_IMAGES = 64


class FsrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


class fsr_params(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("border", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("rho", ctypes.c_float),
                ("gamma", ctypes.c_float), ("dft", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class fsr_image_desc(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("argmax_log", ctypes.c_void_p), ("height", ctypes.c_int32),
                ("width", ctypes.c_int32), ("stride", ctypes.c_int64),
                ("iterations", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class fsr_batch_schedule(ctypes.Structure):
    _fields_ = [("waves_per_group", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_tuple(self):
        return (self.waves_per_group, self.chunk, self.groups_per_cu)


def make_schedule(waves_per_group=1, chunk=0, groups_per_cu=10) -> fsr_batch_schedule:
    return fsr_batch_schedule(waves_per_group, chunk, groups_per_cu, 0)


FSR_MEM_HOST = 0
FSR_MEM_DEVICE = 1
FSR_SERVE_CONTINUOUS = 0
FSR_SERVE_FIFO = 1


class fsr_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("streams", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class fsr_request(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("height", ctypes.c_int32),
                ("width", ctypes.c_int32), ("stride", ctypes.c_int64),
                ("iterations", ctypes.c_int32), ("memory", ctypes.c_int32)]


class fsr_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("released", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("bytes_in_use", ctypes.c_uint64), ("peak_bytes_in_use", ctypes.c_uint64),
                ("busy_s", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def make_server_config(hbm_budget=4 << 30, max_inflight=64, max_batch=16, streams=2,
                       mode=FSR_SERVE_CONTINUOUS) -> fsr_server_config:
    return fsr_server_config(int(hbm_budget), max_inflight, max_batch, streams, mode)


def make_params(block=4, border=14, iterations=100, rho=0.7, gamma=0.5, dft=FSR_DFT_FP32,
                flags=0) -> fsr_params:
    return fsr_params(block, border, iterations, rho, gamma, dft, flags)


_lib = None


def declared_functions() -> list[str]:
    """Names of the functions include/fsr.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^FSR_API\s+[^;(]*?\b(fsr_\w+)\s*\(", text, flags=re.M)))


def load_library(path: str | None = None):
    """Load libfsr.so (built in-tree by ``python -m paper_2202_13926_amd.build``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise FsrError(FSR_ERR_UNSUPPORTED,
                       f"{p} is missing: build it with `python -m paper_2202_13926_amd.build`")
    lib = ctypes.CDLL(p)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER(fsr_params)
    sig = {
        "fsr_version": (i32, []),
        "fsr_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "fsr_last_error_message": (ctypes.c_char_p, []),
        "fsr_params_default": (ctypes.c_int, [P]),
        "fsr_params_validate": (ctypes.c_int, [P]),
        "fsr_num_blocks": (i64, [i32, i32, i32]),
        "fsr_context_create": (ctypes.c_int, [ctypes.POINTER(vp), i32]),
        "fsr_context_destroy": (ctypes.c_int, [vp]),
        "fsr_reconstruct": (ctypes.c_int, [vp, vp, vp, vp, i32, i32, i64, P, vp, vp]),
        "fsr_reconstruct_reuse": (ctypes.c_int, [vp, vp, vp, vp, i32, i32, i64, P, ctypes.c_float,
                                                 vp, vp]),
        "fsr_reconstruct_reuse_frames": (ctypes.c_int, [vp, vp, vp, vp, i32, i32, i32, i64, i64, P,
                                                        ctypes.c_float, vp, vp]),
        "fsr_batched_workspace_size": (ctypes.c_int, [i32, ctypes.POINTER(ctypes.c_size_t)]),
        "fsr_reconstruct_batched": (ctypes.c_int, [vp, ctypes.POINTER(fsr_image_desc), i32, P,
                                                   ctypes.POINTER(fsr_batch_schedule), vp,
                                                   ctypes.c_size_t, vp]),
        "fsr_reconstruct_batched_noalloc": (ctypes.c_int, [vp, ctypes.POINTER(fsr_image_desc), i32, P,
                                                           ctypes.POINTER(fsr_batch_schedule), vp]),
        "fsr_batch_autotune": (ctypes.c_int, [vp, ctypes.POINTER(fsr_image_desc), i32, P, vp,
                                              ctypes.c_size_t, vp,
                                              ctypes.POINTER(fsr_batch_schedule)]),
        "fsr_batch_graph_create": (ctypes.c_int, [vp, ctypes.POINTER(fsr_image_desc), i32, P,
                                                  ctypes.POINTER(fsr_batch_schedule), vp,
                                                  ctypes.c_size_t, ctypes.POINTER(vp)]),
        "fsr_batch_graph_launch": (ctypes.c_int, [vp, vp]),
        "fsr_batch_tuning_export": (ctypes.c_int, [vp, ctypes.c_char_p, ctypes.c_size_t,
                                                   ctypes.POINTER(ctypes.c_size_t)]),
        "fsr_batch_tuning_import": (ctypes.c_int, [vp, ctypes.c_char_p]),
        "fsr_batch_graph_destroy": (ctypes.c_int, [vp]),
        "fsr_server_create": (ctypes.c_int, [vp, P, ctypes.POINTER(fsr_server_config),
                                             ctypes.POINTER(vp)]),
        "fsr_server_submit": (ctypes.c_int, [vp, ctypes.POINTER(fsr_request),
                                             ctypes.POINTER(ctypes.c_uint64)]),
        "fsr_server_poll": (ctypes.c_int, [vp, ctypes.c_uint64, ctypes.POINTER(i32)]),
        "fsr_server_wait": (ctypes.c_int, [vp, ctypes.c_uint64, i32]),
        "fsr_server_result": (ctypes.c_int, [vp, ctypes.c_uint64, vp, i64, i32]),
        "fsr_server_release": (ctypes.c_int, [vp, ctypes.c_uint64]),
        "fsr_server_timing": (ctypes.c_int, [vp, ctypes.c_uint64] + [ctypes.POINTER(ctypes.c_double)] * 4),
        "fsr_server_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(fsr_server_stats)]),
        "fsr_server_destroy": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def status_name(status: int) -> str:
    try:
        return load_library().fsr_status_string(status).decode()
    except Exception:  # the library may be what is missing
        return f"status {status}"


def _check(status: int):
    if status != FSR_OK:
        msg = load_library().fsr_last_error_message().decode()
        raise FsrError(status, msg)


# ---------------------------------------------------------------- plain calls
def fsr_version() -> int:
    return int(load_library().fsr_version())


def fsr_params_default() -> fsr_params:
    p = fsr_params()
    _check(load_library().fsr_params_default(ctypes.byref(p)))
    return p


def fsr_params_validate(params: fsr_params) -> None:
    _check(load_library().fsr_params_validate(ctypes.byref(params)))


def fsr_num_blocks(height: int, width: int, block: int) -> int:
    return int(load_library().fsr_num_blocks(height, width, block))


class Context:
    """Owns an fsr_context on one HIP device."""

    def __init__(self, device: int = 0):
        self._ptr = ctypes.c_void_p()
        _check(load_library().fsr_context_create(ctypes.byref(self._ptr), int(device)))
        self.device = int(device)

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._ptr:
            raise FsrError(FSR_ERR_INVALID_ARG, "context is closed")
        return self._ptr

    def close(self):
        if self._ptr:
            load_library().fsr_context_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fsr_context_create(device: int = 0) -> Context:
    return Context(device)


def fsr_context_destroy(ctx: Context) -> None:
    ctx.close()


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _image_args(image, mask, out):
    import torch
    if image.dtype != torch.float32 or out.dtype != torch.float32:
        raise FsrError(FSR_ERR_INVALID_ARG, "image and out must be float32")
    if mask.dtype != torch.uint8:
        raise FsrError(FSR_ERR_INVALID_ARG, "mask must be uint8")
    if image.dim() != 2 or mask.shape != image.shape or out.shape != image.shape:
        raise FsrError(FSR_ERR_INVALID_ARG, "image, mask and out must be 2-D of equal shape")
    if not (image.is_cuda and mask.is_cuda and out.is_cuda):
        raise FsrError(FSR_ERR_INVALID_ARG, "image, mask and out must be device tensors")
    if not (image.device == mask.device == out.device):
        raise FsrError(FSR_ERR_INVALID_ARG, "image, mask and out must be on one device")
    H, W = image.shape
    # strides of size-1 dimensions carry no meaning in torch; normalise them
    rows = {t.stride(0) if H > 1 else W for t in (image, mask, out)}
    if len(rows) != 1 or any(W > 1 and t.stride(1) != 1 for t in (image, mask, out)):
        raise FsrError(FSR_ERR_INVALID_ARG, "image, mask and out need unit column stride and one row stride")
    return H, W, rows.pop()


def fsr_reconstruct(ctx: Context, image, mask, out, params: fsr_params, argmax_log=None,
                    stream=None) -> None:
    """Enqueue one reconstruction on ``stream`` (default: torch's current stream)."""
    import torch
    H, W, stride = _image_args(image, mask, out)
    log_ptr = None
    if argmax_log is not None:
        n = fsr_num_blocks(H, W, params.block)
        if (argmax_log.dtype not in (torch.int16, torch.uint16) or not argmax_log.is_cuda
                or argmax_log.numel() < n * params.iterations or not argmax_log.is_contiguous()):
            raise FsrError(FSR_ERR_INVALID_ARG, "argmax_log must be a contiguous 16-bit device tensor of N*I entries")
        log_ptr = ctypes.c_void_p(argmax_log.data_ptr())
    _check(load_library().fsr_reconstruct(
        ctx.handle, ctypes.c_void_p(image.data_ptr()), ctypes.c_void_p(mask.data_ptr()),
        ctypes.c_void_p(out.data_ptr()), H, W, stride, ctypes.byref(params), log_ptr,
        _stream_handle(stream, image.device)))


def _log_arg(argmax_log, H, W, params):
    import torch
    if argmax_log is None:
        return None
    n = fsr_num_blocks(H, W, params.block)
    if (argmax_log.dtype not in (torch.int16, torch.uint16) or not argmax_log.is_cuda
            or argmax_log.numel() < n * params.iterations or not argmax_log.is_contiguous()):
        raise FsrError(FSR_ERR_INVALID_ARG, "argmax_log must be a contiguous 16-bit device tensor of N*I entries")
    return ctypes.c_void_p(argmax_log.data_ptr())


def fsr_reconstruct_reuse(ctx: Context, image, mask, out, params: fsr_params, reuse_weight: float,
                          argmax_log=None, stream=None) -> None:
    """Enqueue the sequential variant that reuses reconstructed pixels (one
    launch per wavefront step) on ``stream``."""
    H, W, stride = _image_args(image, mask, out)
    log_ptr = _log_arg(argmax_log, H, W, params)
    _check(load_library().fsr_reconstruct_reuse(
        ctx.handle, ctypes.c_void_p(image.data_ptr()), ctypes.c_void_p(mask.data_ptr()),
        ctypes.c_void_p(out.data_ptr()), H, W, stride, ctypes.byref(params), float(reuse_weight),
        log_ptr, _stream_handle(stream, image.device)))


def fsr_reconstruct_reuse_frames(ctx: Context, images, masks, outs, params: fsr_params,
                                 reuse_weight: float, argmax_log=None, stream=None) -> None:
    """The reuse variant over the frames of 3-D (n, H, W) device tensors that
    share one frame stride and one row stride (e.g. contiguous, or views of
    wider buffers); ``argmax_log`` is None or n x N x I 16-bit."""
    import torch
    if images.dim() != 3 or masks.shape != images.shape or outs.shape != images.shape:
        raise FsrError(FSR_ERR_INVALID_ARG, "images, masks and outs must be 3-D of equal shape")
    n, H, W = images.shape
    H2, W2, stride = _image_args(images[0], masks[0], outs[0])
    fstrides = {t.stride(0) if n > 1 else 0 for t in (images, masks, outs)}
    if len(fstrides) != 1:
        raise FsrError(FSR_ERR_INVALID_ARG, "images, masks and outs need one frame stride")
    log_ptr = None
    if argmax_log is not None:
        nb = fsr_num_blocks(H, W, params.block)
        if (argmax_log.dtype not in (torch.int16, torch.uint16) or not argmax_log.is_cuda
                or argmax_log.numel() < n * nb * params.iterations or not argmax_log.is_contiguous()):
            raise FsrError(FSR_ERR_INVALID_ARG, "argmax_log must be a contiguous 16-bit device tensor of n*N*I entries")
        log_ptr = ctypes.c_void_p(argmax_log.data_ptr())
    _check(load_library().fsr_reconstruct_reuse_frames(
        ctx.handle, ctypes.c_void_p(images.data_ptr()), ctypes.c_void_p(masks.data_ptr()),
        ctypes.c_void_p(outs.data_ptr()), n, H, W, stride, fstrides.pop(), ctypes.byref(params),
        float(reuse_weight), log_ptr, _stream_handle(stream, images.device)))


def reconstruct_reuse(image, mask, params: fsr_params | None = None, reuse_weight: float = 0.5,
                      ctx: Context | None = None, log: bool = False, stream=None):
    """Allocate the output (and the argmax log) and run
    :func:`fsr_reconstruct_reuse`.  Returns ``out`` or ``(out, log)``."""
    import torch
    params = params or make_params()
    ctx = ctx or Context(image.device.index or 0)
    out = torch.empty_like(image)
    lg = None
    if log:
        n = fsr_num_blocks(image.shape[0], image.shape[1], params.block)
        lg = torch.empty((n, max(params.iterations, 1)), dtype=torch.int16, device=image.device)
    fsr_reconstruct_reuse(ctx, image, mask, out, params, reuse_weight, lg, stream)
    if log:
        return out, lg[:, :params.iterations]
    return out


def reconstruct(image, mask, params: fsr_params | None = None, ctx: Context | None = None,
                log: bool = False, stream=None):
    """Allocate the output (and the argmax log) and run :func:`fsr_reconstruct`.
    Returns ``out`` or ``(out, log)`` with ``log`` of shape (N, I) int16."""
    import torch
    params = params or make_params()
    ctx = ctx or Context(image.device.index or 0)
    out = torch.empty_like(image)
    lg = None
    if log:
        n = fsr_num_blocks(image.shape[0], image.shape[1], params.block)
        lg = torch.empty((n, max(params.iterations, 1)), dtype=torch.int16, device=image.device)
    fsr_reconstruct(ctx, image, mask, out, params, lg, stream)
    if log:
        return out, lg[:, :params.iterations]
    return out


# ---------------------------------------------------------------- batches
def fsr_batch_tuning_export(ctx: Context) -> str:
    """The context's autotune results as JSON text (see include/fsr.h)."""
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.fsr_batch_tuning_export(ctx.handle, None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(lib.fsr_batch_tuning_export(ctx.handle, buf, n.value, ctypes.byref(n)))
    return buf.value.decode()


def fsr_batch_tuning_import(ctx: Context, text: str) -> None:
    """Merge autotune results exported on a device of the same kind."""
    _check(load_library().fsr_batch_tuning_import(ctx.handle, text.encode()))


class BatchItem:
    """One image of a batch: device tensors plus its iteration count."""

    def __init__(self, image, mask, out, iterations: int, argmax_log=None):
        self.image, self.mask, self.out = image, mask, out
        self.iterations = int(iterations)
        self.argmax_log = argmax_log


def _descs(items, block):
    arr = (fsr_image_desc * max(len(items), 1))()
    for i, it in enumerate(items):
        H, W, stride = _image_args(it.image, it.mask, it.out)
        log_ptr = None
        if it.argmax_log is not None:
            n = fsr_num_blocks(H, W, block)
            if (not it.argmax_log.is_cuda or not it.argmax_log.is_contiguous()
                    or it.argmax_log.element_size() != 2 or it.argmax_log.numel() < n * it.iterations):
                raise FsrError(FSR_ERR_INVALID_ARG, f"image {i}: argmax_log must be a contiguous "
                                                    "16-bit device tensor of N*I entries")
            log_ptr = it.argmax_log.data_ptr()
        arr[i] = fsr_image_desc(it.image.data_ptr(), it.mask.data_ptr(), it.out.data_ptr(), log_ptr,
                                H, W, stride, it.iterations, 0)
    return arr


def fsr_batched_workspace_size(n_images: int) -> int:
    b = ctypes.c_size_t()
    _check(load_library().fsr_batched_workspace_size(int(n_images), ctypes.byref(b)))
    return int(b.value)


class Workspace:
    """Device workspace of a batch, owned by a torch tensor."""

    def __init__(self, n_images: int, device):
        import torch
        self.nbytes = fsr_batched_workspace_size(n_images)
        self.tensor = torch.empty(self.nbytes, dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return ctypes.c_void_p(self.tensor.data_ptr())


def fsr_reconstruct_batched(ctx: Context, items, params: fsr_params, workspace: Workspace,
                            schedule: fsr_batch_schedule | None = None, stream=None) -> None:
    descs = _descs(items, params.block)
    dev = items[0].image.device if items else None
    sched = ctypes.byref(schedule) if schedule is not None else None
    _check(load_library().fsr_reconstruct_batched(
        ctx.handle, descs, len(items), ctypes.byref(params), sched, workspace.ptr,
        workspace.nbytes, _stream_handle(stream, dev) if dev is not None else None))


def fsr_reconstruct_batched_noalloc(ctx: Context, items, params: fsr_params,
                                    schedule: fsr_batch_schedule | None = None, stream=None) -> None:
    """fsr_reconstruct_batched without a workspace and without any allocation
    (at most FSR_NOALLOC_MAX_IMAGES images; the context must hold the tables
    of this support and rho already)."""
    descs = _descs(items, params.block)
    dev = items[0].image.device if items else None
    sched = ctypes.byref(schedule) if schedule is not None else None
    _check(load_library().fsr_reconstruct_batched_noalloc(
        ctx.handle, descs, len(items), ctypes.byref(params), sched,
        _stream_handle(stream, dev) if dev is not None else None))


def fsr_batch_autotune(ctx: Context, items, params: fsr_params, workspace: Workspace,
                       stream=None) -> fsr_batch_schedule:
    descs = _descs(items, params.block)
    best = fsr_batch_schedule()
    _check(load_library().fsr_batch_autotune(
        ctx.handle, descs, len(items), ctypes.byref(params), workspace.ptr, workspace.nbytes,
        _stream_handle(stream, items[0].image.device), ctypes.byref(best)))
    return best


class BatchGraph:
    """A batch captured into a HIP graph (see fsr_batch_graph_create)."""

    def __init__(self, ctx: Context, items, params: fsr_params, workspace: Workspace,
                 schedule: fsr_batch_schedule | None = None):
        descs = _descs(items, params.block)
        self._ptr = ctypes.c_void_p()
        sched = ctypes.byref(schedule) if schedule is not None else None
        _check(load_library().fsr_batch_graph_create(
            ctx.handle, descs, len(items), ctypes.byref(params), sched, workspace.ptr,
            workspace.nbytes, ctypes.byref(self._ptr)))
        self._keep = (ctx, items, workspace)     # buffers must outlive the graph
        self.device = items[0].image.device if items else None

    def launch(self, stream=None):
        _check(load_library().fsr_batch_graph_launch(self._ptr, _stream_handle(stream, self.device)))

    def close(self):
        if self._ptr:
            load_library().fsr_batch_graph_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- serving
class Server:
    """A continuous-batching frame server (see fsr_server_create)."""

    def __init__(self, ctx: Context, params: fsr_params, config: fsr_server_config):
        self._ptr = ctypes.c_void_p()
        _check(load_library().fsr_server_create(ctx.handle, ctypes.byref(params),
                                                 ctypes.byref(config), ctypes.byref(self._ptr)))
        self._ctx = ctx
        self._keep = {}          # ticket -> buffers that must outlive the request

    def submit(self, image, mask, iterations: int) -> int:
        """Queue a frame held in torch tensors (host or device); returns a ticket."""
        import torch
        if image.dtype != torch.float32 or mask.dtype != torch.uint8 or image.dim() != 2 \
                or mask.shape != image.shape:
            raise FsrError(FSR_ERR_INVALID_ARG, "image float32 and mask uint8 of one 2-D shape")
        H, W = image.shape
        rows = {t.stride(0) if H > 1 else W for t in (image, mask)}
        if len(rows) != 1 or any(W > 1 and t.stride(1) != 1 for t in (image, mask)):
            raise FsrError(FSR_ERR_INVALID_ARG, "image and mask need unit column stride and one row stride")
        if image.is_cuda != mask.is_cuda:
            raise FsrError(FSR_ERR_INVALID_ARG, "image and mask must both be host or both device")
        req = fsr_request(image.data_ptr(), mask.data_ptr(), H, W, rows.pop(), int(iterations),
                          FSR_MEM_DEVICE if image.is_cuda else FSR_MEM_HOST)
        t = ctypes.c_uint64()
        _check(load_library().fsr_server_submit(self._ptr, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (image, mask)
        return int(t.value)

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        _check(load_library().fsr_server_poll(self._ptr, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int, timeout_ms: int = -1) -> None:
        _check(load_library().fsr_server_wait(self._ptr, ticket, int(timeout_ms)))

    def result(self, ticket: int, out) -> None:
        """Copy the finished frame into the 2-D float32 tensor ``out`` and release it."""
        W = out.shape[1]
        stride = out.stride(0) if out.shape[0] > 1 else W
        _check(load_library().fsr_server_result(self._ptr, ticket, ctypes.c_void_p(out.data_ptr()),
                                                stride, FSR_MEM_DEVICE if out.is_cuda else FSR_MEM_HOST))
        self._keep.pop(ticket, None)

    def release(self, ticket: int) -> None:
        _check(load_library().fsr_server_release(self._ptr, ticket))
        self._keep.pop(ticket, None)

    def timing(self, ticket: int) -> tuple:
        v = [ctypes.c_double() for _ in range(4)]
        _check(load_library().fsr_server_timing(self._ptr, ticket, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def stats(self) -> dict:
        st = fsr_server_stats()
        _check(load_library().fsr_server_get_stats(self._ptr, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self._ptr:
            load_library().fsr_server_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
