"""Supports 8, 16 and 24 on the batched and served paths (GPU).

The batched and served kernels run the same per-block arithmetic as the
one-image kernel of the same support (at S = 8 with B <= 4 both take eight
blocks per wavefront, the batch padding each image's block range to a
multiple of eight), so every image's output and argmax log must be bitwise
identical to a fsr_reconstruct call on it alone, under every schedule, in a
graph replay and in a server's mixed launches.  The one-image
kernels of these supports are checked against the oracle in
test_gpu_small_supports.py.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_2202_13926_amd as fsr  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
# (B, L): S = 8 (B = 2 and 4: eight blocks per wavefront), 16 (B = 4 and 8)
# and 24
SPLITS = [(4, 2), (2, 3), (4, 6), (8, 4), (4, 10)]
SCHEDULES = [fsr.make_schedule(1, 0, 10), fsr.make_schedule(4, 0, 2), fsr.make_schedule(1, 4, 10),
             fsr.make_schedule(2, 8, 5), fsr.make_schedule(4, 1, 2)]


def announce(name):
    print(f"\n[gpu case] {name}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    return fsr.Context(0)


def mixed_batch(seed):
    shapes = [(64, 64, "quarter", 100), (37, 50, "uniform:0.3", 25), (96, 128, "quarter", 200),
              (1, 1, "quarter", 10), (33, 1, "uniform:0.2", 0), (150, 200, "macroblock", 100),
              (8, 8, "quarter", 60)]
    items = []
    for i, (h, w, mk, it) in enumerate(shapes):
        img = synth.make_image(h, w, seed * 100 + i).astype(np.float32)
        mask = synth.make_mask(mk, h, w, seed * 100 + i + 50)
        items.append((img, mask, it))
    return items


def params_of(block, border, iterations=100):
    return fsr.make_params(block=block, border=border, iterations=iterations)


def to_items(batch, block):
    items = []
    for img, mask, it in batch:
        ti = torch.from_numpy(img).to(DEV)
        tm = torch.from_numpy(mask).to(DEV)
        out = torch.full_like(ti, -1.0)
        n = fsr.fsr_num_blocks(img.shape[0], img.shape[1], block)
        lg = torch.full((n, max(it, 1)), -1, dtype=torch.int16, device=DEV)
        items.append(fsr.BatchItem(ti, tm, out, it, lg))
    return items


def plain_reference(ctx, batch, block, border):
    refs = []
    for img, mask, it in batch:
        ti, tm = torch.from_numpy(img).to(DEV), torch.from_numpy(mask).to(DEV)
        out, lg = fsr.reconstruct(ti, tm, params_of(block, border, it), ctx=ctx, log=True)
        torch.cuda.synchronize()
        refs.append((out.cpu().numpy(), lg.cpu().numpy()))
    return refs


def results(items):
    torch.cuda.synchronize()
    return [(it.out.cpu().numpy(), it.argmax_log.cpu().numpy()[:, :it.iterations]) for it in items]


def assert_same(got, refs):
    for k, ((g, gl), (r, rl)) in enumerate(zip(got, refs)):
        assert np.array_equal(g, r), f"image {k} output differs"
        assert np.array_equal(gl, rl), f"image {k} argmax log differs"


@pytest.mark.parametrize("block,border", SPLITS)
def test_batched_matches_single_image_calls(ctx, block, border):
    announce(f"B={block} L={border}: batch under every schedule vs one-image calls")
    batch = mixed_batch(21)
    refs = plain_reference(ctx, batch, block, border)
    ws = fsr.Workspace(len(batch), DEV)
    for sched in SCHEDULES:
        items = to_items(batch, block)
        fsr.fsr_reconstruct_batched(ctx, items, params_of(block, border), ws, sched)
        assert_same(results(items), refs)


@pytest.mark.parametrize("block,border", [(4, 2), (4, 6), (4, 10)])
def test_graph_and_autotune(ctx, block, border):
    announce(f"B={block} L={border}: graph replays and the autotuned schedule")
    batch = mixed_batch(23)
    refs = plain_reference(ctx, batch, block, border)
    p = params_of(block, border)
    ws = fsr.Workspace(len(batch), DEV)
    items = to_items(batch, block)
    g = fsr.BatchGraph(ctx, items, p, ws, fsr.make_schedule(2, 4, 5))
    for _ in range(3):
        for it in items:
            it.out.fill_(-5.0)
            it.argmax_log.fill_(-3)
        torch.cuda.synchronize()
        g.launch()
        assert_same(results(items), refs)
    g.close()
    items = to_items(batch, block)
    best = fsr.fsr_batch_autotune(ctx, items, p, ws)
    print("[autotune] best", best.as_tuple(), flush=True)
    assert_same(results(items), refs)
    items = to_items(batch, block)
    fsr.fsr_reconstruct_batched(ctx, items, p, ws)   # the tuned schedule of this support
    assert_same(results(items), refs)


@pytest.mark.parametrize("mode", [fsr.FSR_SERVE_CONTINUOUS, fsr.FSR_SERVE_FIFO])
def test_served_support_16_equals_alone(ctx, mode):
    announce(f"server at S = 16, mode {mode}: mixed frames vs one-image calls")
    block, border = 4, 6
    fr = mixed_batch(25)
    refs = [r for r, _ in plain_reference(ctx, fr, block, border)]
    cfg = fsr.make_server_config(hbm_budget=64 << 20, max_inflight=16, max_batch=8, streams=2,
                                 mode=mode)
    with fsr.Server(ctx, params_of(block, border), cfg) as srv:
        tickets = []
        for k, (img, mask, it) in enumerate(fr):
            if k % 2 == 0:
                ti, tm = torch.from_numpy(img).to(DEV), torch.from_numpy(mask).to(DEV)
                torch.cuda.synchronize()
            else:
                ti, tm = torch.from_numpy(img).pin_memory(), torch.from_numpy(mask).pin_memory()
            tickets.append(srv.submit(ti, tm, it))
        for t, (img, _, _), ref in zip(tickets, fr, refs):
            srv.wait(t, 20000)
            host = torch.empty(img.shape, dtype=torch.float32)
            srv.result(t, host)
            assert np.array_equal(host.numpy(), ref)
        st = srv.stats()
        print("[serve] stats", st, flush=True)
        assert st["completed"] == len(fr) and st["released"] == len(fr)
