"""The batched entry point that allocates nothing (fsr_reconstruct_batched_noalloc).

It shares the batched kernels and differs only in where the queue head and
the descriptor table live (a fixed device array of the library instead of a
caller workspace), so its outputs and argmax logs must be bitwise those of
fsr_reconstruct_batched on the same images, under the plain grid and under
a persistent queue schedule (whose head must be reset in the fixed array by
every call).  Two calls in a row, the second with fewer and smaller images,
check that nothing of the first call's descriptors leaks into the second.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_2202_13926_amd as fsr  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def announce(name):
    print(f"\n[gpu case] {name}", flush=True)


def make_batch(shapes, seed):
    batch = []
    for i, (h, w, mk, it) in enumerate(shapes):
        img = synth.make_image(h, w, seed * 100 + i).astype(np.float32)
        mask = synth.make_mask(mk, h, w, seed * 100 + i + 50)
        batch.append((img, mask, it))
    return batch


def to_items(batch, block):
    items = []
    for img, mask, it in batch:
        ti = torch.from_numpy(img).to(DEV)
        tm = torch.from_numpy(mask).to(DEV)
        out = torch.full_like(ti, -3.0)
        n = fsr.fsr_num_blocks(img.shape[0], img.shape[1], block)
        lg = torch.full((n, max(it, 1)), -1, dtype=torch.int16, device=DEV)
        items.append(fsr.BatchItem(ti, tm, out, it, lg))
    return items


def fetch(items):
    torch.cuda.synchronize()
    return [(it.out.cpu().numpy(), it.argmax_log.cpu().numpy()[:, :it.iterations]) for it in items]


BIG = [(96, 128, "quarter", 100), (150, 200, "macroblock", 60), (64, 64, "uniform:0.3", 200),
       (37, 50, "quarter", 25), (1, 1, "quarter", 10), (33, 1, "uniform:0.2", 0)]
SMALL = [(40, 24, "quarter", 50), (8, 8, "uniform:0.5", 30)]


@pytest.mark.parametrize("support", [(4, 14), (4, 6)])
@pytest.mark.parametrize("schedule", [None, (1, 0, 10), (2, 4, 5)])
def test_noalloc_matches_the_workspace_call_twice(support, schedule):
    B, L = support
    announce(f"noalloc batched S={B + 2 * L} schedule={schedule}: two calls, the second smaller")
    ctx = fsr.Context(0)
    params = fsr.make_params(block=B, border=L)
    sched = fsr.make_schedule(*schedule) if schedule else None
    ws = fsr.Workspace(len(BIG), DEV)
    for k, shapes in enumerate((BIG, SMALL)):
        batch = make_batch(shapes, 70 + k)
        ref = to_items(batch, B)
        fsr.fsr_reconstruct_batched(ctx, ref, params, ws, sched)   # builds the tables first
        got = to_items(batch, B)
        fsr.fsr_reconstruct_batched_noalloc(ctx, got, params, sched)
        for i, ((g, gl), (r, rl)) in enumerate(zip(fetch(got), fetch(ref))):
            assert np.array_equal(g, r), f"call {k} image {i}: output differs"
            assert np.array_equal(gl, rl), f"call {k} image {i}: argmax log differs"
    ctx.close()


def test_noalloc_refusals():
    announce("noalloc batched: refused cases leave the outputs untouched")
    ctx = fsr.Context(0)
    batch = make_batch(SMALL, 90)
    # the tables of this rho were never built on this context: refused
    params = fsr.make_params(rho=0.61)
    items = to_items(batch, 4)
    with pytest.raises(fsr.FsrError) as e:
        fsr.fsr_reconstruct_batched_noalloc(ctx, items, params)
    assert e.value.status == 2   # FSR_ERR_UNSUPPORTED
    # more images than the fixed workspace holds
    params = fsr.make_params()
    fsr.reconstruct(torch.from_numpy(batch[0][0]).to(DEV), torch.from_numpy(batch[0][1]).to(DEV),
                    params, ctx=ctx)
    many = to_items(batch * (fsr.FSR_NOALLOC_MAX_IMAGES // 2 + 1), 4)
    with pytest.raises(fsr.FsrError) as e:
        fsr.fsr_reconstruct_batched_noalloc(ctx, many, params)
    assert e.value.status == 1   # FSR_ERR_INVALID_ARG
    for it in items + many:
        assert torch.all(it.out == -3.0)
    ctx.close()
