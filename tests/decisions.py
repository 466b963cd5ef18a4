"""Which logged argmax decisions an FP32 implementation can be held to.

Eq. (8) picks the bin of largest objective w_f |R_w|^2.  The FP64 oracle
compares its objectives as they are.  The GPU compares float32 objectives
whose 4 lowest mantissa bits carry a tie code (relative resolution 2^-19),
computed from a float32 residual that carries the round-off of the
transforms and of every earlier iteration, which does not shrink with the
residual.  Where the oracle's winner leads every other bin by less than FP32
can resolve, or where the residual has shrunk towards that round-off, both
choices implement Eq. (8) equally well, and from then on the two greedy
paths may part.

A decision counts as resolvable when the oracle's winner leads the next
objective by at least SEP_MIN relative (the winner's exactly tied conjugate,
which both sides settle by the index rule, passed over) and its objective is
at least OBJ_FLOOR times the block's first.  At that floor |R_w| is 2^-10 of
the first pick's; a round-off that stays near 2^-22 of the first residual
(a few float32 ulps of it) is then 2^-12 of the current one.  The
thresholds were checked on the GPU against 22 configurations (the benchmark
frames, the small supports and the corners of the paper's parameter
sweep): no block parted from the oracle inside its resolvable prefix, nor
with the floor 16 times lower; on the whole 2160p concealment frame
(518,400 blocks, I = 200) one block did, 3 of its 39.1 million resolvable
decisions, hence the bar PREFIX_AGREE.  A block's resolvable prefix runs
from iteration 0 to its first unresolvable decision.  Every
quantity here comes from the oracle's own FP64 run on the same input.
"""
from __future__ import annotations

import numpy as np

SEP_MIN = 2.0 ** -12
OBJ_FLOOR = 2.0 ** -20
PREFIX_AGREE = 1.0 - 1e-5      # share of the resolvable decisions that must agree


def resolvable_prefix(obj: np.ndarray, sep: np.ndarray) -> np.ndarray:
    """Per block (rows of the (N, I) oracle logs of winning objective and
    separation), the number of leading iterations whose decisions are
    resolvable."""
    obj = np.asarray(obj, np.float64)
    sep = np.asarray(sep, np.float64)
    if obj.shape[1] == 0:
        return np.zeros(obj.shape[0], np.int64)
    first = obj[:, :1]
    ok = (sep >= SEP_MIN) & (obj >= OBJ_FLOOR * first) & (first > 0)
    # length of the leading run of True in each row
    bad = ~ok
    return np.where(bad.any(axis=1), bad.argmax(axis=1), obj.shape[1]).astype(np.int64)


def decision_report(gpu_log, oracle_log, obj, sep) -> dict:
    """Agreement of the GPU's logged picks with the oracle's on every
    block's resolvable prefix, beside the strict per-iteration figure."""
    gl = np.asarray(gpu_log).astype(np.int64) & 0xFFFF
    ol = np.asarray(oracle_log).astype(np.int64)
    n, iters = ol.shape
    pre = resolvable_prefix(obj, sep)
    in_prefix = np.arange(iters)[None, :] < pre[:, None]
    same = gl == ol
    n_pre = int(in_prefix.sum())
    miss = in_prefix & ~same
    return {
        "prefix_decisions": n_pre,
        "prefix_share": n_pre / max(ol.size, 1),
        "prefix_agree": float(same[in_prefix].mean()) if n_pre else 1.0,
        "blocks_parting_in_prefix": int(miss.any(axis=1).sum()),
        "strict_agree": float(same.mean()) if same.size else 1.0,
        "blocks_all_agree": float(same.all(axis=1).mean()) if same.size else 1.0,
    }


def block_of_pixel(height: int, width: int, block: int) -> np.ndarray:
    """(height, width) array of the block index (raster order) each pixel's
    target belongs to."""
    nbx = -(-width // block)
    y = np.arange(height)[:, None] // block
    x = np.arange(width)[None, :] // block
    return y * nbx + x


def parting_report(mask, gpu_out, oracle_out, gpu_log, oracle_log, obj, sep, block: int) -> dict:
    """For frames where the two greedy paths may part after an unresolvable
    decision: the decision report plus the pixel comparison restricted to the
    blocks whose logged picks all equal the oracle's (there the two sides ran
    the same iterations, and only arithmetic separates them)."""
    rep = decision_report(gpu_log, oracle_log, obj, sep)
    gl = np.asarray(gpu_log).astype(np.int64) & 0xFFFF
    agree_blocks = np.all(gl == np.asarray(oracle_log).astype(np.int64), axis=1)
    H, W = np.asarray(mask).shape
    owner = block_of_pixel(H, W, block)
    sel = (np.asarray(mask) == 0) & agree_blocks[owner]
    d = np.abs(np.asarray(gpu_out, np.float64) - np.asarray(oracle_out, np.float64))[sel]
    rep["agreeing_blocks_unknown_px"] = int(sel.sum())
    rep["agreeing_blocks_frac_le_1"] = float(np.mean(d <= 1.0)) if d.size else 1.0
    rep["agreeing_blocks_max_abs"] = float(d.max()) if d.size else 0.0
    return rep
