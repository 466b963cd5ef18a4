"""Evaluation helpers shared by the tests and the benchmark (no method arithmetic).

PSNR follows the usual 8-bit definition, 10 log10(255^2 / MSE), computed after
clipping the reconstruction to [0, 255]; "missing-only" restricts the mean to
the pixels the mask marks unknown.
"""
from __future__ import annotations

import numpy as np


def psnr(ref: np.ndarray, x: np.ndarray, where: np.ndarray | None = None) -> float:
    d = np.clip(np.asarray(x, np.float64), 0.0, 255.0) - np.asarray(ref, np.float64)
    if where is not None:
        d = d[where]
    mse = float(np.mean(d * d))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(255.0 ** 2 / mse)


def mirror_bin(idx, S: int = 32):
    idx = np.asarray(idx, np.int64)
    k, l = idx // S, idx % S
    return ((S - k) % S) * S + (S - l) % S


def parity_report(ref_img, mask, gpu_out, oracle_out, gpu_log=None, oracle_log=None) -> dict:
    """Compare a GPU reconstruction with the FP64 oracle on the same inputs.

    ``gpu_out``/``oracle_out`` may be full frames or gathered target pixels of
    the same blocks; ``mask`` and ``ref_img`` must have the same shape."""
    unknown = np.asarray(mask) == 0
    g = np.asarray(gpu_out, np.float64)
    o = np.asarray(oracle_out, np.float64)
    d = np.abs(g - o)[unknown]
    rep = {
        "n_unknown": int(unknown.sum()),
        "max_abs": float(d.max()) if d.size else 0.0,
        "frac_le_1": float(np.mean(d <= 1.0)) if d.size else 1.0,
        "frac_le_1_over_255": float(np.mean(d <= 1.0 / 255.0)) if d.size else 1.0,
        "psnr_gpu": psnr(ref_img, g),
        "psnr_oracle": psnr(ref_img, o),
        "known_bitwise": bool(np.array_equal(g[~unknown], np.asarray(ref_img)[~unknown].astype(g.dtype))),
    }
    a, b = rep["psnr_gpu"], rep["psnr_oracle"]
    rep["psnr_gap"] = 0.0 if a == b else abs(a - b)     # equal also covers inf == inf
    if gpu_log is not None and oracle_log is not None:
        gl = np.asarray(gpu_log).astype(np.int64) & 0xFFFF
        ol = np.asarray(oracle_log).astype(np.int64)
        same = gl == ol
        rep["argmax_agree"] = float(same.mean()) if same.size else 1.0
        mir = gl == mirror_bin(ol)
        per_block = np.maximum(same.mean(axis=1), mir.mean(axis=1)) if same.size else np.ones(1)
        rep["argmax_agree_mirror_aware"] = float(per_block.mean())
        rep["blocks_diverging"] = int((~same.all(axis=1)).sum()) if same.size else 0
    return rep
