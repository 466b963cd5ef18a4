"""The oracle's reconstruction of whole benchmark frames, computed once per
test process and shared by the parity tests of both DFT modes.

The 2160p concealment frame at I = 200 is 518,400 blocks: about half a
minute of the oracle on sixteen host threads, so it is computed once.
"""
from __future__ import annotations

import functools

import numpy as np

import oracle
import synth


@functools.lru_cache(maxsize=None)
def oracle_frame(name: str):
    """``(img32, mask, out, log, obj, sep)`` for the named workload: the
    float32 input both sides receive, its mask, and the oracle's FP64 output
    frame, (N, I) argmax log, winning objectives and their separations over
    every block."""
    w = synth.workload(name)
    img, mask = w.inputs()
    img32 = img.astype(np.float32)
    out, log, _, (obj, sep) = oracle.reconstruct(img32.astype(np.float64), mask, w.iterations,
                                                 block_size=w.block, border=w.border, rho=w.rho,
                                                 gamma=w.gamma, log=True, separations=True)
    for a in (img32, mask, out, log, obj, sep):
        a.setflags(write=False)
    return img32, mask, out, log, obj, sep
