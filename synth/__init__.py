"""Seeded synthetic inputs for Frequency Selective Reconstruction (FSR).

This module is shared by the tests, the benchmark and both sides of every
parity check (the HIP library and the CPU oracle).  It holds no arithmetic of
the reconstruction method itself: only image/mask generators, workload
descriptions and request traces.

The paper evaluates on 8-bit grayscale photographs sampled by a quarter
sampling sensor (Sec. IV): one random pixel of every 2x2 cell is known.  No
dataset is available here, so images are synthetic with the same value range
and a mix of smooth content, edges and noise:

    f = 128 + sum_{i<8} A_i cos(2 pi (fy_i y / Y + fx_i x / X) + phi_i)
            + sum_{j<3} h_j [ (y - py_j) sin t_j + (x - px_j) cos t_j > 0 ]
            + N(0, 2^2),                          clipped to [0, 255]

with A ~ U(0,60), fy, fx ~ U(0,8) cycles per frame (so the content statistics
do not depend on the frame size), phi ~ U(0, 2 pi), t ~ U(0, pi), (py, px) a
uniform random pixel and h ~ U(-60, 60).  All draws come from
``numpy.random.default_rng(seed)`` in the order listed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "make_image", "quarter_mask", "uniform_loss_mask", "macroblock_mask",
    "Workload", "workload", "batch_items", "serving_trace", "image_seed",
    "BatchItem", "Request",
]


def image_seed(config: int, index: int = 0) -> int:
    """Seed of image ``index`` of workload ``config``; its mask uses seed + 1."""
    return 1000 + 100 * config + index


def make_image(height: int, width: int, seed: int) -> np.ndarray:
    """Synthetic grayscale frame, float64 in [0, 255], shape (height, width)."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.0, 60.0, 8)
    fy = rng.uniform(0.0, 8.0, 8)
    fx = rng.uniform(0.0, 8.0, 8)
    phi = rng.uniform(0.0, 2.0 * math.pi, 8)
    y = np.arange(height, dtype=np.float64)[:, None]
    x = np.arange(width, dtype=np.float64)[None, :]
    img = np.full((height, width), 128.0)
    for i in range(8):
        img += amp[i] * np.cos(2.0 * math.pi * (fy[i] * y / height + fx[i] * x / width) + phi[i])
    for _ in range(3):
        theta = rng.uniform(0.0, math.pi)
        py = rng.integers(0, height)
        px = rng.integers(0, width)
        h = rng.uniform(-60.0, 60.0)
        side = (y - py) * math.sin(theta) + (x - px) * math.cos(theta) > 0.0
        img += h * side
    img += rng.normal(0.0, 2.0, (height, width))
    return np.clip(img, 0.0, 255.0)


def quarter_mask(height: int, width: int, seed: int) -> np.ndarray:
    """Quarter sampling: one uniformly chosen known pixel per 2x2 cell (uint8, 1 = known).

    Odd sizes: the grid is generated for the next even size and cropped, so a
    border cell may end up with no known pixel."""
    rng = np.random.default_rng(seed)
    ch, cw = (height + 1) // 2, (width + 1) // 2
    pick = rng.integers(0, 4, (ch, cw))
    full = np.zeros((2 * ch, 2 * cw), dtype=np.uint8)
    for q in range(4):
        dy, dx = divmod(q, 2)
        full[dy::2, dx::2] = (pick == q)
    return np.ascontiguousarray(full[:height, :width])


def uniform_loss_mask(height: int, width: int, loss: float, seed: int) -> np.ndarray:
    """Each pixel is lost independently with probability ``loss`` (uint8, 1 = known)."""
    rng = np.random.default_rng(seed)
    return (rng.random((height, width)) >= loss).astype(np.uint8)


def macroblock_mask(height: int, width: int, seed: int, drop: float = 0.25,
                    mb: int = 16, extra_loss: float = 0.10) -> np.ndarray:
    """Error-concealment mask: exactly round(drop * #MB) of the mb x mb
    macroblocks (partial ones at the border included) are lost, chosen by a
    seeded permutation; every pixel outside them is then lost with
    probability ``extra_loss``."""
    rng = np.random.default_rng(seed)
    mby, mbx = -(-height // mb), -(-width // mb)
    n_mb = mby * mbx
    lost = rng.permutation(n_mb)[: int(round(drop * n_mb))]
    mb_known = np.ones(n_mb, dtype=np.uint8)
    mb_known[lost] = 0
    grid = np.repeat(np.repeat(mb_known.reshape(mby, mbx), mb, 0), mb, 1)[:height, :width]
    px_known = (rng.random((height, width)) >= extra_loss).astype(np.uint8)
    return np.ascontiguousarray(grid & px_known)


@dataclass
class Workload:
    """One named workload: frame size, mask recipe and method parameters."""
    name: str
    height: int
    width: int
    mask: str                      # "quarter" | "macroblock" | "uniform:<p>"
    iterations: int
    block: int = 4
    border: int = 14
    rho: float = 0.7
    gamma: float = 0.5
    config: int = 0

    @property
    def support(self) -> int:
        return self.block + 2 * self.border

    @property
    def n_blocks(self) -> int:
        return -(-self.height // self.block) * -(-self.width // self.block)

    def inputs(self, index: int = 0):
        s = image_seed(self.config, index)
        img = make_image(self.height, self.width, s)
        return img, make_mask(self.mask, self.height, self.width, s + 1)


def make_mask(kind: str, height: int, width: int, seed: int) -> np.ndarray:
    if kind == "quarter":
        return quarter_mask(height, width, seed)
    if kind == "macroblock":
        return macroblock_mask(height, width, seed)
    if kind.startswith("uniform:"):
        return uniform_loss_mask(height, width, float(kind.split(":", 1)[1]), seed)
    raise ValueError(f"unknown mask kind {kind!r}")


_WORKLOADS = {
    # 64x64 frame, quarter sampling, 256 blocks: small enough for the oracle.
    "small64": Workload("small64", 64, 64, "quarter", 100, config=0),
    # one 1920x1080 frame, quarter sampling, 129,600 blocks, I = 100.
    "fhd_quarter": Workload("fhd_quarter", 1080, 1920, "quarter", 100, config=1),
    # one 3840x2160 frame, 25 % macroblock loss + 10 % pixel loss, I = 200.
    "uhd_concealment": Workload("uhd_concealment", 2160, 3840, "macroblock", 200, config=2),
}


def workload(name: str) -> Workload:
    return _WORKLOADS[name]


# --------------------------------------------------------------------------
# Uneven batches and request streams
# --------------------------------------------------------------------------

_BATCH_SIZES = ((256, 256), (480, 640), (720, 1280), (1080, 1920))
_BATCH_ITERS = (50, 100, 200)


@dataclass
class BatchItem:
    height: int
    width: int
    mask: str
    iterations: int
    seed: int

    def inputs(self):
        return make_image(self.height, self.width, self.seed), \
            make_mask(self.mask, self.height, self.width, self.seed + 1)


def batch_items(n: int = 64, seed: int = 1300, sizes=_BATCH_SIZES,
                iters=_BATCH_ITERS) -> list[BatchItem]:
    """``n`` images of uneven sizes drawn uniformly from ``sizes`` with mixed
    masks (quarter sampling, or uniform loss with p ~ U(0.1, 0.5)) and
    iteration counts drawn uniformly from ``iters``."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        h, w = sizes[rng.integers(0, len(sizes))]
        if rng.random() < 0.5:
            mask = "quarter"
        else:
            mask = f"uniform:{rng.uniform(0.1, 0.5):.4f}"
        it = int(iters[rng.integers(0, len(iters))])
        out.append(BatchItem(int(h), int(w), mask, it, seed + 1 + 2 * i))
    return out


@dataclass
class Request:
    arrival_s: float
    item: BatchItem = field(repr=False)


_SERVE_SIZES = ((720, 1280),) * 5 + ((1080, 1920),) * 3 + ((2160, 3840),)


def serving_trace(n: int = 10000, rate_hz: float = 240.0, seed: int = 1400,
                  iterations: int = 100) -> list[Request]:
    """Poisson arrivals at ``rate_hz`` with frame sizes 720p:1080p:2160p in the
    ratio 5:3:1 and masks as in :func:`batch_items`."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n):
        h, w = _SERVE_SIZES[rng.integers(0, len(_SERVE_SIZES))]
        if rng.random() < 0.5:
            mask = "quarter"
        else:
            mask = f"uniform:{rng.uniform(0.1, 0.5):.4f}"
        reqs.append(Request(float(t[i]), BatchItem(int(h), int(w), mask, iterations, seed + 1 + 2 * i)))
    return reqs


_REALTIME_SIZES = ((480, 640), (600, 800), (1080, 1920), (2160, 3840))


def realtime_trace(seconds: float = 5.0, fps: float = 30.0, sizes=_REALTIME_SIZES,
                   seed: int = 1500, iterations: int = 100) -> list[Request]:
    """One periodic video stream per frame size, each at ``fps`` frames per
    second for ``seconds``, with quarter-sampling masks; stream k starts at
    the phase k / (len(sizes) * fps), so arrivals interleave.  Requests are
    returned in arrival order."""
    reqs = []
    n = int(round(seconds * fps))
    for k, (h, w) in enumerate(sizes):
        phase = k / (len(sizes) * fps)
        for i in range(n):
            reqs.append(Request(phase + i / fps,
                                BatchItem(int(h), int(w), "quarter", iterations, seed + 100 * k + 2 * (i % 3))))
    reqs.sort(key=lambda r: r.arrival_s)
    return reqs
