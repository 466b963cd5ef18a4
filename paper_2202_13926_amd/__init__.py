"""Block-parallel Frequency Selective Reconstruction (FSR) on MI355X.

The reconstruction runs in hand-written HIP kernels for gfx950 behind the C
ABI of include/fsr.h (libfsr.so, built in-tree); this package is its thin
Python binding.  See :mod:`paper_2202_13926_amd.binding`.
"""
from .binding import (  # noqa: F401
    FSR_DFT_FP32, FSR_DFT_SPLIT_BF16, FSR_FLAG_LDS_ARGMAX, FSR_NOALLOC_MAX_IMAGES, BatchGraph, BatchItem, Context, FsrError, Workspace,
    declared_functions, fsr_batch_autotune, fsr_batch_schedule, fsr_batch_tuning_export,
    fsr_batch_tuning_import, fsr_batched_workspace_size,
    fsr_context_create, fsr_context_destroy, fsr_image_desc, fsr_num_blocks, fsr_params,
    fsr_params_default, fsr_params_validate, fsr_reconstruct, fsr_reconstruct_batched, fsr_reconstruct_batched_noalloc,
    fsr_reconstruct_reuse, fsr_reconstruct_reuse_frames, fsr_version,
    load_library, make_params, make_schedule, reconstruct, reconstruct_reuse,
)
from .binding import (  # noqa: F401
    FSR_MEM_DEVICE, FSR_MEM_HOST, FSR_SERVE_CONTINUOUS, FSR_SERVE_FIFO, Server, fsr_request,
    fsr_server_config, fsr_server_stats, make_server_config,
)
