"""Benchmark of block-parallel FSR on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: one 1920x1080 synthetic frame, quarter-sampling mask, B = 4, L = 14
(32 x 32 support and DFT), I = 100 iterations, rho = 0.7, gamma = 0.5:
129,600 independent blocks.  One step reconstructs the whole frame (gather,
weighting, forward DFTs, I greedy iterations, target inverse DFT, compose)
with inputs already resident in device memory.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "reconstructed Mpixel/s + p99 frame latency, served/batched vs plain, PSNR gap≤0.05dB"
WORKLOAD = "fhd_quarter"
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector peak (256 CU x 2.4 GHz x 256 flop/clk)
NONPACKED_FP32_TFLOPS = 78.6   # the same with one FP32 FMA per lane and cycle (no packed FP32)
HBM_PEAK_GB_S = 8000.0         # MI355X HBM3E


def algorithmic_flops_per_block(S: int, B: int, iters: int) -> float:
    """Flops the method itself requires per block (stated in the design notes):
    12 S^2 per iteration (objective 4, residual complex update 8), the two real
    forward DFTs at the radix-2 count 2 * 2.5 S^2 log2(S^2), and 4 B^2 per
    iteration for the target model."""
    return 12.0 * S * S * iters + 5.0 * S * S * math.log2(S * S) + 4.0 * B * B * iters


# what the code of fsr_plain_s32 is built from: its sources and the compiler
# flags (not the rest of the build script)
KERNEL_SOURCES = ("paper_2202_13926_amd/csrc/fsr_block.h", "paper_2202_13926_amd/csrc/fsr_device.h",
                  "paper_2202_13926_amd/csrc/fsr_mfma.h", "paper_2202_13926_amd/csrc/fsr_plain.hip",
                  "paper_2202_13926_amd/csrc/fsr_internal.h")
PMC_SUMMARY = "profiles/fsr_plain_s32_fhd_quarter_pmc.md"


def kernel_hash() -> str:
    import hashlib

    from paper_2202_13926_amd import build
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    flags = [f for f in build.FLAGS if not f.startswith(ROOT)]   # include paths vary by checkout
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary,
    or None when the kernel sources changed after the counters were taken."""
    try:
        text = open(os.path.join(ROOT, PMC_SUMMARY)).read()
    except OSError:
        return None
    for line in text.splitlines():
        if line.startswith("traffic-record:"):
            kv = dict(item.split("=") for item in line.split()[1:])
            if kv.get("kernel_hash") != kernel_hash():
                return None
            return int(kv["fetch_bytes"]) + int(kv["write_bytes"])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-blocks", type=int, default=129600,
                    help="blocks in the oracle's timed sample (default: the whole 1080p frame)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-image batched comparison")
    ap.add_argument("--no-reuse", action="store_true",
                    help="skip the leg of the sequential variant that reuses reconstructed pixels")
    ap.add_argument("--reuse-frames", default="4,16,64",
                    help="frame counts (multiples of 4) timed by the reuse leg's several-frames part; "
                         "'' for none")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the split-bf16 vs FP32-FFT comparison on the 3840x2160 frame")
    ap.add_argument("--serve-max-batch", type=int, default=2,
                    help="frames per launch of the continuous-batching server")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests of the served comparison, the serving workload's 10,000 by "
                         "default (about 42 s per mode; 0 skips it)")
    ap.add_argument("--tuning-cache", default=None, metavar="PATH",
                    help="load the batched path's autotune results from PATH if it exists, and "
                         "write them back after the run")
    ap.add_argument("--serve-log", default=None, metavar="PATH",
                    help="append one JSON line per served request (both modes) to PATH")
    ap.add_argument("--realtime-seconds", type=float, default=5.0,
                    help="length of the four-stream real-time leg at S = 16 (0 skips it)")
    ap.add_argument("--sweep", action="store_true",
                    help="only run the paper's 640-point parameter grid (S, I, rho, gamma) on a "
                         "1200x1200 frame and print it as one JSON object")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline launches and nothing else (for profiler runs of "
                         "that one configuration)")
    ap.add_argument("--support", type=int, default=32, choices=(8, 16, 24, 32),
                    help="support S of the timed launches (B = 4, L = (S - 4) / 2); the "
                         "headline configuration is S = 32, others serve per-support profiles")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (a kernel of known "
                         "traffic, used to scale the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def copy_calibration(mib: int):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4,
                      "copies": 5}), flush=True)


def cpu_baseline(img32, mask, w, n_blocks_sample):
    import oracle
    threads = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(12345)
    ids = np.sort(rng.choice(w.n_blocks, size=min(n_blocks_sample, w.n_blocks), replace=False))
    img64 = img32.astype(np.float64)
    oracle.reconstruct_blocks(img64, mask, ids[:64], w.iterations, threads=threads)  # warm
    t0 = time.perf_counter()
    oracle.reconstruct_blocks(img64, mask, ids, w.iterations, threads=threads)
    dt = time.perf_counter() - t0
    px = len(ids) * w.block * w.block
    what = (f"all {len(ids)} blocks of the frame" if len(ids) == w.n_blocks
            else f"{len(ids)} seeded random blocks of the same frame")
    # one thread on a smaller seeded sample of the same blocks
    ids1 = ids[rng.choice(len(ids), size=min(4000, len(ids)), replace=False)]
    ids1.sort()
    t0 = time.perf_counter()
    oracle.reconstruct_blocks(img64, mask, ids1, w.iterations, threads=1)
    dt1 = time.perf_counter() - t0
    px1 = len(ids1) * w.block * w.block
    # one thread over the supports of Fig. 3 (B = 4, L = 2, 6, 10, 14): the
    # frame time extrapolated from a seeded sample of 2,000 blocks
    by_support = {}
    ids_s = ids[rng.choice(len(ids), size=min(2000, len(ids)), replace=False)]
    ids_s.sort()
    for L in (2, 6, 10, 14):
        t0 = time.perf_counter()
        oracle.reconstruct_blocks(img64, mask, ids_s, w.iterations, block_size=4, border=L, threads=1)
        dts = time.perf_counter() - t0
        by_support[f"S{4 + 2 * L}"] = {"frame_ms": round(dts / len(ids_s) * w.n_blocks * 1e3, 1),
                                       "sample_s": round(dts, 3)}
    return {"value": px / dt / 1e6, "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
            "sample": f"{what} ({px} pixels), FP64 C oracle, OpenMP over blocks on {threads} "
                      f"threads, {dt:.2f} s wall",
            "single_thread": {"value": px1 / dt1 / 1e6, "unit": "Mpixel/s", "cores": 1,
                              "sample": f"{len(ids1)} of those blocks ({px1} pixels), {dt1:.2f} s wall",
                              "by_support": by_support}}


def bench_precision(ctx, steps: int = 3):
    """3840x2160 concealment frame (25 % of 16x16 macroblocks dropped, 10 %
    uniform loss elsewhere), I = 200: the FP32-FFT path against the split-bf16
    matrix-core DFTs, timed on the same buffers, each scored against the
    ground-truth frame, and the two outputs against each other."""
    import torch

    import paper_2202_13926_amd as fsr
    import synth
    from synth.metrics import psnr

    w = synth.workload("uhd_concealment")
    img, mask = w.inputs()
    img32 = img.astype(np.float32)
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(img32).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    stream = torch.cuda.current_stream(dev)
    res = {"workload": "uhd_concealment: 3840x2160, 25% of 16x16 macroblocks dropped + 10% uniform "
                       "loss, B=4 L=14 (S=32), I=200, rho=0.7, gamma=0.5",
           "blocks": w.n_blocks}
    outs = {}
    for tag, dft in (("fp32_fft", fsr.FSR_DFT_FP32), ("split_bf16", fsr.FSR_DFT_SPLIT_BF16)):
        p = fsr.make_params(block=w.block, border=w.border, iterations=w.iterations, rho=w.rho,
                            gamma=w.gamma, dft=dft)
        o = torch.empty_like(ti)
        fsr.fsr_reconstruct(ctx, ti, tm, o, p, None, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fsr.fsr_reconstruct(ctx, ti, tm, o, p, None, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        g = o.cpu().numpy()
        outs[tag] = g
        res[tag] = {"ms": round(ms, 3), "mpx_s": round(img.size / ms / 1e3, 2),
                    "psnr_missing_db": round(psnr(img32, g, mask == 0), 4)}
    d = np.abs(outs["fp32_fft"] - outs["split_bf16"])[mask == 0]
    res["split_bf16_vs_fp32_fft"] = {"max_abs": round(float(d.max()), 5),
                                     "frac_le_1_code": round(float(np.mean(d <= 1.0)), 6)}
    return res


def bench_argmax_ablation(ctx, img32, mask, params, steps: int = 20, warmup: int = 3):
    """The paper's comparison (Sec. IV): the same frame and parameters with
    the argmax reduced through an LDS tree instead of in registers."""
    import torch

    import paper_2202_13926_amd as fsr

    dev = torch.device("cuda:0")
    ti = torch.from_numpy(img32).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    o = torch.empty_like(ti)
    stream = torch.cuda.current_stream(dev)
    # every (border, argmax) variant: the headline parameters and the supports
    # of Fig. 3 (B = 4, L = 2, 6, 10); at S = 8 the register path takes eight
    # blocks per wavefront
    borders = (2, 6, 10, params.border) if params.block == 4 else (2, 6, 10)
    variants = {}
    for L in borders:
        for tag, flags in (("register_ms", 0), ("lds_ms", fsr.FSR_FLAG_LDS_ARGMAX)):
            b = params.block if L == params.border else 4
            variants[(L, tag)] = fsr.make_params(block=b, border=L, iterations=params.iterations,
                                                 rho=params.rho, gamma=params.gamma, flags=flags)
    if params.block != 4:
        for tag, flags in (("register_ms", 0), ("lds_ms", fsr.FSR_FLAG_LDS_ARGMAX)):
            variants[(None, tag)] = fsr.make_params(block=params.block, border=params.border,
                                                    iterations=params.iterations, rho=params.rho,
                                                    gamma=params.gamma, flags=flags)
    # two rounds, each the register variants first, then the (much longer)
    # shared-memory ones, so that no register timing of the first round
    # follows a long run at a lowered clock; each variant keeps its best round
    # of as many warm-up and timed launches as the headline leg
    order = sorted(variants, key=lambda k: (k[1] != "register_ms", -1 if k[0] is None else k[0]))
    best = {}
    for _ in range(2):
        for key in order:
            p = variants[key]
            for _ in range(warmup):
                fsr.fsr_reconstruct(ctx, ti, tm, o, p, None, stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                fsr.fsr_reconstruct(ctx, ti, tm, o, p, None, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            best[key] = min(best.get(key, 1e30), e0.elapsed_time(e1) / steps)
    head = params.border if params.block == 4 else None
    res = {name: {"ms": round(best[(head, tag)], 4), "mpx_s": round(img32.size / best[(head, tag)] / 1e3, 2)}
           for name, tag in (("register_argmax", "register_ms"), ("lds_argmax", "lds_ms"))}
    res["speedup_register_over_lds"] = round(res["lds_argmax"]["ms"] / res["register_argmax"]["ms"], 3)
    by_support = {}
    for L in (2, 6, 10):
        times = {tag: round(best[(L, tag)], 4) for tag in ("register_ms", "lds_ms")}
        times["speedup_register_over_lds"] = round(times["lds_ms"] / times["register_ms"], 3)
        by_support[f"S{4 + 2 * L}"] = times
    by_support[f"S{params.block + 2 * params.border}"] = {
        "register_ms": res["register_argmax"]["ms"], "lds_ms": res["lds_argmax"]["ms"],
        "speedup_register_over_lds": res["speedup_register_over_lds"]}
    # the register path of each support against the FP32 vector peak, with the
    # same algorithmic flop count as the headline line (B = 4)
    blocks = -(-img32.shape[0] // 4) * -(-img32.shape[1] // 4)
    for key, t in by_support.items():
        flops = algorithmic_flops_per_block(int(key[1:]), 4, params.iterations) * blocks
        tf = flops / (t["register_ms"] * 1e-3) / 1e12
        t["register_tflop_s"] = round(tf, 3)
        t["register_frac_of_peak"] = round(tf / PEAK_FP32_TFLOPS, 4)
    res["by_support"] = by_support
    return res


def bench_reuse(ctx, img32, mask, params, delta: float = 0.5, steps: int = 3, frame_counts=(4, 16, 64)):
    """The sequential variant that reuses reconstructed pixels (the original
    FSR the paper departs from) on the same frame: one launch per wavefront
    step, eagerly and as a replayed HIP graph, with its quality beside the
    block-independent result's."""
    import torch

    import paper_2202_13926_amd as fsr
    from synth.metrics import psnr

    dev = torch.device("cuda:0")
    ti = torch.from_numpy(img32).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    o = torch.empty_like(ti)
    ind = torch.empty_like(ti)
    stream = torch.cuda.current_stream(dev)
    fsr.fsr_reconstruct(ctx, ti, tm, ind, params, None, stream)
    fsr.fsr_reconstruct_reuse(ctx, ti, tm, o, params, delta, None, stream)
    torch.cuda.synchronize()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    eager_ms = timed(lambda: fsr.fsr_reconstruct_reuse(ctx, ti, tm, o, params, delta, None, stream))
    side = torch.cuda.Stream(dev)
    side.wait_stream(stream)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        fsr.fsr_reconstruct_reuse(ctx, ti, tm, o, params, delta, None, side)
    torch.cuda.synchronize()
    graph_ms = timed(g.replay)
    # frames of one size in one call: one launch per step takes every frame's blocks
    frames = {}
    for n in frame_counts:
        imgs = torch.stack([ti, ti.flip(0), ti.flip(1), ti.flip(0, 1)] * (n // 4)).contiguous()
        masks = torch.stack([tm, tm.flip(1), tm.flip(0), tm.flip(0, 1)] * (n // 4)).contiguous()
        outs = torch.empty_like(imgs)
        fsr.fsr_reconstruct_reuse_frames(ctx, imgs, masks, outs, params, delta, None, stream)
        torch.cuda.synchronize()
        ms = timed(lambda: fsr.fsr_reconstruct_reuse_frames(ctx, imgs, masks, outs, params, delta, None, stream))
        frames[f"frames_{n}"] = {"ms": round(ms, 3), "ms_per_frame": round(ms / n, 3),
                                 "mpx_s": round(n * img32.size / ms / 1e3, 2)}
        del imgs, masks, outs
    H, W = img32.shape
    B, L = params.block, params.border
    nby, nbx, slope = -(-H // B), -(-W // B), (L + B - 1) // B + 1
    n_steps = (nbx - 1) + slope * (nby - 1) + 1
    r, miss = o.cpu().numpy(), mask == 0
    a = ind.cpu().numpy()
    return {"delta": delta, "wavefront_steps": n_steps,
            "max_blocks_per_step": min(nby, -(-nbx // slope)),
            "eager_ms": round(eager_ms, 3), "graph_ms": round(graph_ms, 3),
            "us_per_step_graph": round(graph_ms * 1e3 / n_steps, 2),
            "mpx_s_graph": round(img32.size / graph_ms / 1e3, 2), **frames,
            "psnr_missing_db": {"independent": round(psnr(img32, a, miss), 4),
                                "reuse": round(psnr(img32, r, miss), 4)}}


def bench_multiresolution(ctx, steps: int = 20, warmup: int = 3):
    """Frame rates at S = 16 (B = 4, L = 6), I = 100, quarter-sampling masks,
    for the paper's real-time table resolutions (Sec. IV: VGA, SVGA, FHD,
    UHD), the four frames as one batch (tuned batched launch in a graph
    against one launch per frame), and the 1080p frame at every support size
    the library runs."""
    import torch

    import paper_2202_13926_amd as fsr
    import synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        # as many warm-up and timed launches as the headline leg
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def frame(h, w, seed):
        img = synth.make_image(h, w, seed).astype(np.float32)
        mask = synth.quarter_mask(h, w, seed + 1)
        ti = torch.from_numpy(img).to(dev)
        return ti, torch.from_numpy(mask).to(dev), torch.empty_like(ti)

    def frame_ms(h, w, B, L, seed):
        ti, tm, o = frame(h, w, seed)
        p = fsr.make_params(block=B, border=L, iterations=100)
        return timed(lambda: fsr.fsr_reconstruct(ctx, ti, tm, o, p, None, stream))

    res = {"workload": "synthetic frames, quarter-sampling masks, I=100, rho=0.7, gamma=0.5",
           "s16_fps": {}, "fhd_ms_by_support": {}}
    sizes = (("VGA 640x480", (480, 640)), ("SVGA 800x600", (600, 800)),
             ("FHD 1920x1080", (1080, 1920)), ("UHD 3840x2160", (2160, 3840)))
    for name, (h, w) in sizes:
        res["s16_fps"][name] = round(1e3 / frame_ms(h, w, 4, 6, 1700), 2)

    p16 = fsr.make_params(block=4, border=6, iterations=100)
    items = [fsr.BatchItem(*frame(h, w, 1700), 100) for _, (h, w) in sizes]
    best = fsr.fsr_batch_autotune(ctx, items, p16, fsr.Workspace(len(items), dev), stream)
    graph = fsr.BatchGraph(ctx, items, p16, fsr.Workspace(len(items), dev), best)
    # the two forms alternate over two rounds and each keeps its best: a few
    # milliseconds each, they would otherwise read the clock state the
    # previous leg left
    graph_ms = plain_ms = 1e30
    for _ in range(2):
        graph_ms = min(graph_ms, timed(lambda: graph.launch(stream)))
        plain_ms = min(plain_ms, timed(lambda: [fsr.fsr_reconstruct(ctx, it.image, it.mask, it.out, p16,
                                                                     None, stream) for it in items]))
    graph.close()
    res["s16_batch_of_four"] = {
        "frames": "VGA + SVGA + FHD + UHD, one each",
        "schedule": {"waves_per_group": best.waves_per_group, "chunk": best.chunk,
                     "groups_per_cu": best.groups_per_cu},
        "graph_ms": round(graph_ms, 4), "plain_loop_ms": round(plain_ms, 4),
        "sets_per_s": round(1e3 / graph_ms, 2)}
    for S in (8, 16, 24, 32):
        res["fhd_ms_by_support"][f"S={S}"] = round(frame_ms(1080, 1920, 4, (S - 4) // 2, 1800), 4)
    return res


def parameter_sweep(ctx, size: int = 1200, steps: int = 3):
    """The paper's parameter grid (Sec. IV): I in {100, ..., 400}, S in
    {8, 16, 24, 32} (B = 4), rho in {0.68, ..., 0.82}, gamma in {0.2, ..., 0.6}:
    640 parameterisations on one size x size synthetic frame with a
    quarter-sampling mask.  Returns time per frame and PSNR (missing pixels
    and full frame, against the ground-truth frame) for each."""
    import torch

    import paper_2202_13926_amd as fsr
    import synth
    from synth.metrics import psnr

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    img = synth.make_image(size, size, 2100).astype(np.float32)
    mask = synth.quarter_mask(size, size, 2101)
    ti = torch.from_numpy(img).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    o = torch.empty_like(ti)
    rows = []
    for S in (8, 16, 24, 32):
        for iters in (100, 200, 300, 400):
            for rho in np.round(np.arange(0.68, 0.8201, 0.02), 2):
                for gamma in np.round(np.arange(0.2, 0.6001, 0.1), 1):
                    p = fsr.make_params(block=4, border=(S - 4) // 2, iterations=iters,
                                        rho=float(rho), gamma=float(gamma))
                    fsr.fsr_reconstruct(ctx, ti, tm, o, p, None, stream)
                    torch.cuda.synchronize()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(steps):
                        fsr.fsr_reconstruct(ctx, ti, tm, o, p, None, stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    g = o.cpu().numpy()
                    rows.append({"S": S, "I": iters, "rho": float(rho), "gamma": float(gamma),
                                 "ms": round(e0.elapsed_time(e1) / steps, 4),
                                 "psnr_missing_db": round(psnr(img, g, mask == 0), 3),
                                 "psnr_db": round(psnr(img, g), 3)})
    return {"workload": f"{size}x{size} synthetic frame, quarter-sampling mask, B=4",
            "parameterisations": len(rows), "rows": rows}


def bench_batched(ctx, steps: int = 5):
    """64 uneven images (256x256 .. 1920x1080, quarter or 10-50 % uniform loss,
    I in {50, 100, 200}) with split-bf16 DFTs and FP32 iterations: the tuned
    batched launch, its graph replay and the plain loop of one fsr_reconstruct
    launch per image, on the same buffers; the graph replay with FP32 FFTs for
    reference."""
    import torch

    import paper_2202_13926_amd as fsr
    import synth

    dev = torch.device("cuda:0")
    specs = synth.batch_items(64)
    items, pixels, work = [], 0, 0
    for sp in specs:
        img, mask = sp.inputs()
        ti = torch.from_numpy(img.astype(np.float32)).to(dev)
        tm = torch.from_numpy(mask).to(dev)
        items.append(fsr.BatchItem(ti, tm, torch.empty_like(ti), sp.iterations))
        pixels += img.size
        work += fsr.fsr_num_blocks(sp.height, sp.width, 4) * sp.iterations
    params = fsr.make_params(dft=fsr.FSR_DFT_SPLIT_BF16)
    ws = fsr.Workspace(len(items), dev)
    stream = torch.cuda.current_stream(dev)
    t0 = time.perf_counter()
    best = fsr.fsr_batch_autotune(ctx, items, params, ws, stream)
    tune_s = time.perf_counter() - t0

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    batched_ms = timed(lambda: fsr.fsr_reconstruct_batched(ctx, items, params, ws, best, stream), steps)
    graph = fsr.BatchGraph(ctx, items, params, fsr.Workspace(len(items), dev), best)
    graph_ms = timed(lambda: graph.launch(stream), steps)
    graph.close()
    graph32 = fsr.BatchGraph(ctx, items, fsr.make_params(), fsr.Workspace(len(items), dev), best)
    graph32_ms = timed(lambda: graph32.launch(stream), steps)
    graph32.close()

    def plain_loop():
        for it in items:
            p = fsr.make_params(iterations=it.iterations, dft=fsr.FSR_DFT_SPLIT_BF16)
            fsr.fsr_reconstruct(ctx, it.image, it.mask, it.out, p, None, stream)

    plain_ms = timed(plain_loop, max(2, steps // 2))
    mpx = pixels / 1e6
    return {"workload": "64 uneven images 256x256..1920x1080, quarter or 10-50% uniform loss, "
                        "I in {50,100,200}, S=32, rho=0.7, gamma=0.5",
            "dft": "split-bf16 (3 terms) on the matrix cores, FP32 iterations",
            "pixels": pixels, "block_iterations": int(work),
            "schedule": {"waves_per_group": best.waves_per_group, "chunk": best.chunk,
                         "groups_per_cu": best.groups_per_cu}, "autotune_s": round(tune_s, 3),
            "batched_ms": round(batched_ms, 3), "batched_mpx_s": round(mpx / batched_ms * 1e3, 2),
            "graph_ms": round(graph_ms, 3), "graph_mpx_s": round(mpx / graph_ms * 1e3, 2),
            "plain_loop_ms": round(plain_ms, 3), "plain_loop_mpx_s": round(mpx / plain_ms * 1e3, 2),
            "graph_fp32_fft_ms": round(graph32_ms, 3),
            "speedup_vs_plain_loop": round(plain_ms / min(batched_ms, graph_ms), 3)}


def replay_trace(srv, trace, frame_of):
    """Submits the requests of ``trace`` to ``srv`` at their arrival times
    (``frame_of(k, request)`` gives the k-th request's pinned image and mask)
    while a second thread waits for and releases them in submission order.
    Returns one row per request: submit, admit, launch and done times in
    seconds, pixels, frame height."""
    import queue
    import threading

    q = queue.Queue()
    rec = []

    def reaper():
        while True:
            item = q.get()
            if item is None:
                return
            t, px, h = item
            srv.wait(t)
            sub, adm, lau, done = srv.timing(t)
            srv.release(t)
            rec.append((sub, adm, lau, done, px, h))

    th = threading.Thread(target=reaper)
    th.start()
    t0 = time.perf_counter()
    for k, req in enumerate(trace):
        delay = t0 + req.arrival_s - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        img, mask = frame_of(k, req)
        q.put((srv.submit(img, mask, req.item.iterations), req.item.height * req.item.width,
               req.item.height))
    q.put(None)
    th.join()
    return np.array(rec)


def pinned_pool(trace, per_size: int = 3):
    """Up to ``per_size`` distinct pinned host frames per frame size of a trace."""
    import torch

    pool = {}
    for req in trace:
        key = (req.item.height, req.item.width)
        if key in pool and len(pool[key]) >= per_size:
            continue
        img, mask = req.item.inputs()
        pool.setdefault(key, []).append((torch.from_numpy(img.astype(np.float32)).pin_memory(),
                                         torch.from_numpy(mask).pin_memory()))
    return pool


def pick(pool, k, req):
    frames = pool[(req.item.height, req.item.width)]
    return frames[k % len(frames)]


def bench_realtime_s16(ctx, seconds: float = 5.0, fps: float = 60.0, budget: int = 2 << 30):
    """The paper's real-time setting through the server: four periodic video
    streams at ``fps`` (VGA, SVGA, FHD, UHD; quarter-sampling masks, I = 100,
    S = 16 with B = 4, L = 6), frames uploaded from pinned host memory.  Per
    resolution: latency (arrival to result on the device) p50 / p99 / max and
    the frames that missed the 1 / fps deadline; continuous batching against
    the FIFO one-frame-per-launch loop."""
    import paper_2202_13926_amd as fsr
    import synth

    trace = synth.realtime_trace(seconds, fps)
    pool = pinned_pool(trace)
    params = fsr.make_params(block=4, border=6, iterations=100)
    deadline_ms = 1e3 / fps
    names = {480: "VGA 640x480", 600: "SVGA 800x600", 1080: "FHD 1920x1080", 2160: "UHD 3840x2160"}
    out = {"workload": f"4 periodic streams (VGA, SVGA, FHD, UHD) at {fps:g} fps for {seconds:g} s, "
                       "quarter-sampling masks, S=16 (B=4, L=6), I=100, host-resident frames",
           "requests": len(trace), "deadline_ms": round(deadline_ms, 3)}
    for name, mode, streams, max_batch in (("continuous", fsr.FSR_SERVE_CONTINUOUS, 2, 4),
                                           ("fifo_one_frame_per_launch", fsr.FSR_SERVE_FIFO, 1, 1)):
        cfg = fsr.make_server_config(hbm_budget=budget, max_inflight=64, max_batch=max_batch,
                                     streams=streams, mode=mode)
        srv = fsr.Server(ctx, params, cfg)
        for frames in pool.values():                          # warm-up
            t = srv.submit(frames[0][0], frames[0][1], 100)
            srv.wait(t)
            srv.release(t)
        a = replay_trace(srv, trace, lambda k, req: pick(pool, k, req))
        st = srv.stats()
        srv.close()
        lat = (a[:, 3] - a[:, 0]) * 1e3
        span = a[:, 3].max() - a[:, 0].min()
        per = {}
        for h, label in names.items():
            sel = a[:, 5] == h
            m = lat[sel]
            per[label] = {"p50_ms": round(float(np.percentile(m, 50)), 3),
                          "p99_ms": round(float(np.percentile(m, 99)), 3),
                          "max_ms": round(float(m.max()), 3),
                          "missed_deadline": int((m > deadline_ms).sum()), "frames": int(m.size),
                          # where the time goes: submit -> launch, launch -> done (medians)
                          "to_launch_ms": round(float(np.median(a[sel, 2] - a[sel, 0]) * 1e3), 3),
                          "launch_to_done_ms": round(float(np.median(a[sel, 3] - a[sel, 2]) * 1e3), 3)}
        out[name] = {"by_resolution": per,
                     "throughput_mpx_s": round(float(a[:, 4].sum() / span / 1e6), 2),
                     "frames_per_launch": round(st["completed"] / max(st["launches"], 1), 3),
                     "gpu_busy_frac": round(st["busy_s"] / span, 3)}
    return out


def bench_served(ctx, n_requests: int, rate_hz: float = 240.0, budget: int = 4 << 30,
                 max_batch: int = 2, log_path: str | None = None):
    """Poisson stream of frames (720p:1080p:2160p = 5:3:1, I = 100, quarter or
    10-50 % uniform-loss masks) replayed in real time against the
    continuous-batching server and against the FIFO one-frame-per-launch loop.
    Frame contents come from a pinned host pool of 3 frames per size; the
    arrival times, sizes and order follow the seeded trace.  With
    ``log_path``, one JSON line per request and mode is appended there
    (server clock times of submission, admission, launch and completion)."""
    import paper_2202_13926_amd as fsr
    import synth

    trace = synth.serving_trace(n_requests, rate_hz)
    pool = pinned_pool(trace)
    params = fsr.make_params()
    out = {"workload": f"Poisson {rate_hz:g} frames/s, {n_requests} requests, 720p:1080p:2160p = 5:3:1, "
                       "I=100, quarter or 10-50% uniform-loss masks, host-resident input frames",
           "requests": n_requests, "hbm_budget_bytes": budget, "max_batch": max_batch}
    offered = sum(r.item.height * r.item.width for r in trace) / max(trace[-1].arrival_s, 1e-9) / 1e6
    out["offered_mpx_s"] = round(offered, 2)
    for name, mode, streams in (("continuous", fsr.FSR_SERVE_CONTINUOUS, 2),
                                ("fifo_one_frame_per_launch", fsr.FSR_SERVE_FIFO, 1)):
        cfg = fsr.make_server_config(hbm_budget=budget, max_inflight=64,
                                     max_batch=max_batch if mode == fsr.FSR_SERVE_CONTINUOUS else 1,
                                     streams=streams, mode=mode)
        srv = fsr.Server(ctx, params, cfg)
        for key, frames in pool.items():                     # warm-up
            t = srv.submit(frames[0][0], frames[0][1], 100)
            srv.wait(t)
            srv.release(t)
        a = replay_trace(srv, trace, lambda k, req: pick(pool, k, req))
        st = srv.stats()
        srv.close()
        lat = (a[:, 3] - a[:, 0]) * 1e3
        span = a[:, 3].max() - a[:, 0].min()
        if log_path:
            with open(log_path, "a") as fh:
                for k, (row, req) in enumerate(zip(a, trace)):
                    fh.write(json.dumps({"mode": name, "request": k, "height": req.item.height,
                                         "width": req.item.width, "iterations": req.item.iterations,
                                         "arrival_s": round(req.arrival_s, 6), "submit_s": row[0],
                                         "admit_s": row[1], "launch_s": row[2], "done_s": row[3],
                                         "latency_ms": round(float(lat[k]), 4)}) + "\n")
        print(f"[bench] served, {name}: {len(trace)} requests done", file=sys.stderr, flush=True)
        out[name] = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                     "p99_ms": round(float(np.percentile(lat, 99)), 3),
                     "max_ms": round(float(lat.max()), 3),
                     "mean_queue_ms": round(float(np.mean(a[:, 1] - a[:, 0]) * 1e3), 3),
                     "throughput_mpx_s": round(float(a[:, 4].sum() / span / 1e6), 2),
                     "frames_per_launch": round(st["completed"] / max(st["launches"], 1), 3),
                     "gpu_busy_frac": round(st["busy_s"] / span, 3),
                     "peak_hbm_bytes": int(st["peak_bytes_in_use"])}
    return out


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described in the design notes only)"}))
        sys.exit(2)
    import torch

    import paper_2202_13926_amd as fsr
    import synth

    if args.sweep:
        ctx = fsr.Context(0)
        print(json.dumps(parameter_sweep(ctx)), flush=True)
        ctx.close()
        return

    w = synth.workload(WORKLOAD)
    img, mask = w.inputs()
    img32 = img.astype(np.float32)
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(img32).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    out = torch.empty_like(ti)
    ctx = fsr.Context(0)
    border = w.border if args.support == w.support else (args.support - w.block) // 2
    params = fsr.make_params(block=w.block, border=border, iterations=w.iterations, rho=w.rho,
                             gamma=w.gamma)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        fsr.fsr_reconstruct(ctx, ti, tm, out, params, None, stream)
    torch.cuda.synchronize()

    K = args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(K):
        fsr.fsr_reconstruct(ctx, ti, tm, out, params, None, stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(K)])   # ms, device clock
    total_ms = ev[0].elapsed_time(ev[K])
    ms_per_step = total_ms / K
    pixels = w.height * w.width
    value = pixels / (ms_per_step * 1e-3) / 1e6

    flops = algorithmic_flops_per_block(args.support, w.block, w.iterations) * w.n_blocks
    achieved = flops / (ms_per_step * 1e-3) / 1e12

    # quality of this run (vs. the ground-truth frame)
    g = out.cpu().numpy()
    from synth.metrics import psnr
    quality = {"psnr_db": round(psnr(img32, g), 4),
               "psnr_missing_db": round(psnr(img32, g, mask == 0), 4)}

    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator standing in for the paper's photographs)",
        "config": {"workload": "fhd_quarter: 1920x1080 frame, quarter-sampling mask, B=4 L=14 "
                               "(S=32), I=100, rho=0.7, gamma=0.5, plain one-launch path",
                   "blocks": w.n_blocks, "pixels": pixels, "path": "fsr_reconstruct"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 5),
                       "p99": round(float(np.percentile(lat, 99)), 5),
                       "max": round(float(lat.max()), 5)},
        "wall_s": round(wall, 4),
        "quality": quality,
        "roofline": {"bound": "alu", "kernel": "fsr_plain_s32",
                     "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "algorithmic_flop_per_launch": flops,
                     "avg_launch_ms": round(ms_per_step, 5),
                     "traffic": measured_traffic(),
                     # the same rate against the non-packed FP32 issue rate (this
                     # build never emits packed FP32), and the HBM side
                     "frac_of_nonpacked_fp32": round(achieved / NONPACKED_FP32_TFLOPS, 4)},
    }
    if res["roofline"]["traffic"] is not None:
        gb_s = res["roofline"]["traffic"] / (ms_per_step * 1e-3) / 1e9
        res["roofline"]["hbm_gb_s"] = round(gb_s, 2)
        res["roofline"]["hbm_frac"] = round(gb_s / HBM_PEAK_GB_S, 6)
    if args.support != w.support:
        res["config"]["workload"] += f"; timed at S={args.support} (B=4, L={border}) instead"
        res["roofline"]["kernel"] = "fsr_plain_multi" if args.support == 8 else (
            "fsr_plain_s24" if args.support == 24 else "fsr_plain_sg")
        res["roofline"]["traffic"] = None
        res["roofline"].pop("hbm_gb_s", None)
        res["roofline"].pop("hbm_frac", None)
    if args.only_headline:
        ctx.close()
        print(json.dumps(res), flush=True)
        return
    t_leg = time.perf_counter()

    def leg_done(name):
        # one progress line per finished leg (stderr: stdout carries the JSON line only)
        nonlocal t_leg
        now = time.perf_counter()
        print(f"[bench] {name} done in {now - t_leg:.1f} s", file=sys.stderr, flush=True)
        t_leg = now

    leg_done("headline")
    res["argmax_ablation"] = bench_argmax_ablation(ctx, img32, mask, params)
    leg_done("argmax ablation")
    res["multiresolution"] = bench_multiresolution(ctx)
    leg_done("multiresolution")
    if not args.no_reuse:
        counts = tuple(int(x) for x in args.reuse_frames.split(",") if x.strip())
        if any(n < 4 or n % 4 for n in counts):
            sys.exit("--reuse-frames takes multiples of 4")
        res["reuse_variant"] = bench_reuse(ctx, img32, mask, params, frame_counts=counts)
        leg_done("reuse variant")
    if args.tuning_cache and os.path.exists(args.tuning_cache):
        with open(args.tuning_cache) as fh:
            fsr.fsr_batch_tuning_import(ctx, fh.read())
    if not args.no_batched:
        res["batched"] = bench_batched(ctx)
        leg_done("batched")
    if args.tuning_cache:
        with open(args.tuning_cache, "w") as fh:
            fh.write(fsr.fsr_batch_tuning_export(ctx) + "\n")
    if not args.no_precision:
        res["precision"] = bench_precision(ctx)
        leg_done("precision")
    if args.serve_requests > 0:
        res["served"] = bench_served(ctx, args.serve_requests, max_batch=args.serve_max_batch,
                                     log_path=args.serve_log)
        leg_done("served")
    if args.realtime_seconds > 0:
        res["realtime_s16"] = bench_realtime_s16(ctx, args.realtime_seconds)
        leg_done("real-time S = 16")
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(img32, mask, w, args.cpu_blocks)
        leg_done("cpu baseline")
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
