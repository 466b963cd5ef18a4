"""Output with and without the argmax log, on every kernel.

Each block routine runs its iteration loop in one of two copies, with and
without the log store, chosen by whether the caller passed a log.  The
other tests mostly pass one; the bench's timed launches do not.  A call
without a log must give bitwise the output of the same call with one: the
one-image kernels at S = 8, 16, 24 and 32 (FP32 FFTs; at S = 32 also the
split-bf16 DFTs; the shared-memory argmax at every support), the batched
kernels under a queue and a grid schedule, and the sequential reuse variant.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_2202_13926_amd as fsr  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SUPPORTS = [(4, 14), (4, 10), (4, 6), (4, 2)]   # (B, L): S = 32, 24, 16, 8


@pytest.fixture(scope="module")
def ctx():
    return fsr.Context(0)


@pytest.fixture(scope="module")
def frame():
    # several blocks across, a ragged edge at B = 4 in both directions
    img = synth.make_image(150, 203, 901).astype(np.float32)
    mask = synth.quarter_mask(150, 203, 902)
    return torch.from_numpy(img).to(DEV), torch.from_numpy(mask).to(DEV)


def one(ctx, ti, tm, p, with_log):
    out = torch.full_like(ti, float("nan"))   # every pixel is written
    lg = None
    if with_log:
        n = fsr.fsr_num_blocks(ti.shape[0], ti.shape[1], p.block)
        lg = torch.full((n, max(p.iterations, 1)), -1, dtype=torch.int16, device=DEV)
    fsr.fsr_reconstruct(ctx, ti, tm, out, p, lg, None)
    torch.cuda.synchronize()
    return out.cpu().numpy()


# the split-bf16 DFTs run at S = 32 only
ONE_IMAGE = [(B, L, v) for B, L in SUPPORTS for v in ("fp32", "lds_argmax")] + [(4, 14, "split_bf16")]


@pytest.mark.parametrize("B,L,variant", ONE_IMAGE)
def test_one_image_kernels(ctx, frame, B, L, variant):
    S = B + 2 * L
    print(f"\n[gpu case] one-image S={S} {variant} with and without log", flush=True)
    kw = {}
    if variant == "lds_argmax":
        kw["flags"] = fsr.FSR_FLAG_LDS_ARGMAX
    if variant == "split_bf16":
        kw["dft"] = fsr.FSR_DFT_SPLIT_BF16
    p = fsr.make_params(block=B, border=L, iterations=100, **kw)
    ti, tm = frame
    a = one(ctx, ti, tm, p, True)
    b = one(ctx, ti, tm, p, False)
    assert np.isfinite(a).all()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("B,L", SUPPORTS[:3])
def test_batched_kernels(ctx, B, L):
    S = B + 2 * L
    print(f"\n[gpu case] batched S={S} with and without log", flush=True)
    shapes = [(64, 64, 100), (37, 50, 25), (96, 128, 60), (8, 8, 40)]
    batch = []
    for i, (h, w, it) in enumerate(shapes):
        img = synth.make_image(h, w, 910 + i).astype(np.float32)
        batch.append((torch.from_numpy(img).to(DEV),
                      torch.from_numpy(synth.quarter_mask(h, w, 920 + i)).to(DEV), it))
    ws = fsr.Workspace(len(batch), DEV)
    params = fsr.make_params(block=B, border=L)
    for sched in (fsr.make_schedule(1, 0, 10), fsr.make_schedule(2, 8, 5)):
        outs = []
        for with_log in (True, False):
            items = []
            for ti, tm, it in batch:
                lg = None
                if with_log:
                    n = fsr.fsr_num_blocks(ti.shape[0], ti.shape[1], B)
                    lg = torch.full((n, max(it, 1)), -1, dtype=torch.int16, device=DEV)
                items.append(fsr.BatchItem(ti, tm, torch.full_like(ti, float("nan")), it, lg))
            fsr.fsr_reconstruct_batched(ctx, items, params, ws, sched)
            torch.cuda.synchronize()
            outs.append([item.out.cpu().numpy() for item in items])
        for k, (a, b) in enumerate(zip(*outs)):
            assert np.isfinite(a).all(), f"image {k} not fully written"
            assert np.array_equal(a, b), f"image {k} differs without the log"


def test_reuse_variant(ctx, frame):
    print("\n[gpu case] reuse variant with and without log", flush=True)
    ti, tm = frame
    p = fsr.make_params(iterations=100)
    a, _ = fsr.reconstruct_reuse(ti, tm, p, 0.5, ctx=ctx, log=True)
    b = fsr.reconstruct_reuse(ti, tm, p, 0.5, ctx=ctx, log=False)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
