"""Continuous-batching server on the GPU.

Results are bitwise identical to fsr_reconstruct on the same frame whether
the frame was served alone or batched with others; admission respects the
HBM budget; failure paths (oversized frame, wait timeout, shutdown with
pending work) are forced from the host, never by a faulting kernel.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_2202_13926_amd as fsr  # noqa: E402
from paper_2202_13926_amd import binding  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def announce(name):
    print(f"\n[gpu case] {name}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    return fsr.Context(0)


def frames(seed=3):
    shapes = [(64, 64, "quarter", 100), (37, 50, "uniform:0.3", 40), (96, 128, "quarter", 150),
              (128, 96, "uniform:0.5", 60), (1, 1, "quarter", 5), (200, 160, "macroblock", 100),
              (8, 9, "quarter", 20), (130, 70, "uniform:0.1", 0)]
    out = []
    for i, (h, w, mk, it) in enumerate(shapes):
        img = synth.make_image(h, w, seed * 100 + i).astype(np.float32)
        mask = synth.make_mask(mk, h, w, seed * 100 + i + 50)
        out.append((img, mask, it))
    return out


def alone(ctx, img, mask, it):
    o = fsr.reconstruct(torch.from_numpy(img).to(DEV), torch.from_numpy(mask).to(DEV),
                        fsr.make_params(iterations=it), ctx=ctx)
    torch.cuda.synchronize()
    return o.cpu().numpy()


def submit_all(srv, fr, device_every=2):
    tickets = []
    for k, (img, mask, it) in enumerate(fr):
        if k % device_every == 0:
            ti, tm = torch.from_numpy(img).to(DEV), torch.from_numpy(mask).to(DEV)
            torch.cuda.synchronize()
        else:
            ti, tm = torch.from_numpy(img).pin_memory(), torch.from_numpy(mask).pin_memory()
        tickets.append(srv.submit(ti, tm, it))
    return tickets


@pytest.mark.parametrize("mode", [fsr.FSR_SERVE_CONTINUOUS, fsr.FSR_SERVE_FIFO])
def test_results_equal_alone_and_in_the_mix(ctx, mode):
    announce(f"server mode {mode}: mixed frames vs one-image calls")
    fr = frames()
    refs = [alone(ctx, *f) for f in fr]
    # one compute stream, kept busy by a 1080p frame first, so that the small
    # frames submitted behind it are admitted together and share launches
    heavy_img, heavy_mask = synth.workload("fhd_quarter").inputs()
    th = torch.from_numpy(heavy_img.astype(np.float32)).to(DEV)
    tmh = torch.from_numpy(heavy_mask).to(DEV)
    torch.cuda.synchronize()
    cfg = fsr.make_server_config(hbm_budget=256 << 20, max_inflight=16, max_batch=8, streams=1,
                                 mode=mode)
    with fsr.Server(ctx, fsr.make_params(), cfg) as srv:
        for rnd in range(2):
            heavy = srv.submit(th, tmh, 200)
            tickets = submit_all(srv, fr, device_every=2 + rnd)
            srv.wait(heavy, 20000)
            srv.release(heavy)
            for t, (img, _, _), ref in zip(tickets, fr, refs):
                srv.wait(t, 20000)
                host = torch.empty(img.shape, dtype=torch.float32)
                srv.result(t, host)
                assert np.array_equal(host.numpy(), ref)
        st = srv.stats()
        print("[serve] stats", st, flush=True)
        n = 2 * (len(fr) + 1)
        assert st["completed"] == n and st["released"] == n
        if mode == fsr.FSR_SERVE_CONTINUOUS:
            assert st["launches"] < st["completed"]      # frames shared launches
        else:
            assert st["launches"] == st["completed"]


def test_device_result_copy_and_strided_output(ctx):
    announce("result copied to a strided device tensor")
    img, mask, it = frames(5)[2]
    ref = alone(ctx, img, mask, it)
    with fsr.Server(ctx, fsr.make_params(), fsr.make_server_config(hbm_budget=64 << 20)) as srv:
        t = srv.submit(torch.from_numpy(img).to(DEV), torch.from_numpy(mask).to(DEV), it)
        srv.wait(t, 20000)
        big = torch.full((img.shape[0], img.shape[1] + 13), -1.0, device=DEV)
        srv.result(t, big[:, :img.shape[1]])
        torch.cuda.synchronize()
        assert np.array_equal(big[:, :img.shape[1]].cpu().numpy(), ref)
        assert torch.all(big[:, img.shape[1]:] == -1.0)


def test_admission_respects_the_budget(ctx):
    announce("budget for about two frames, eight submitted")
    fr = [(synth.make_image(128, 128, 40 + i).astype(np.float32), synth.quarter_mask(128, 128, 60 + i), 40)
          for i in range(8)]
    per = 2 * (128 * 128 * 4) + 128 * 128      # 9 bytes per pixel (all parts 256-aligned)
    cfg = fsr.make_server_config(hbm_budget=2 * per + 4096, max_inflight=8, max_batch=4)
    with fsr.Server(ctx, fsr.make_params(), cfg) as srv:
        tickets = submit_all(srv, fr)
        # without releases only two frames fit: the third cannot be admitted
        srv.wait(tickets[0], 20000)
        srv.wait(tickets[1], 20000)
        with pytest.raises(fsr.FsrError) as e:
            srv.wait(tickets[2], 100)
        assert e.value.status == binding.FSR_ERR_TIMEOUT
        assert srv.stats()["admitted"] == 2
        for t, f in zip(tickets, fr):
            srv.wait(t, 20000)
            out = torch.empty(f[0].shape, dtype=torch.float32)
            srv.result(t, out)
            assert np.array_equal(out.numpy(), alone(ctx, *f))
        st = srv.stats()
        assert st["peak_bytes_in_use"] <= cfg.hbm_budget and st["bytes_in_use"] == 0


def test_oversized_frame_is_refused(ctx):
    announce("frame larger than the budget")
    with fsr.Server(ctx, fsr.make_params(), fsr.make_server_config(hbm_budget=1 << 20)) as srv:
        img = torch.zeros((512, 512), dtype=torch.float32)
        mask = torch.ones((512, 512), dtype=torch.uint8)
        with pytest.raises(fsr.FsrError) as e:
            srv.submit(img, mask, 10)
        assert e.value.status == binding.FSR_ERR_BUDGET
        with pytest.raises(fsr.FsrError) as e:
            srv.result(12345, torch.empty((1, 1)))
        assert e.value.status == binding.FSR_ERR_INVALID_ARG


def test_not_ready_and_shutdown_with_pending_work(ctx):
    announce("result before completion, destroy with queued and running frames")
    w = synth.workload("fhd_quarter")
    img, mask = w.inputs()
    ti = torch.from_numpy(img.astype(np.float32)).to(DEV)
    tm = torch.from_numpy(mask).to(DEV)
    torch.cuda.synchronize()
    srv = fsr.Server(ctx, fsr.make_params(), fsr.make_server_config(hbm_budget=64 << 20, max_inflight=2,
                                                                     max_batch=1, streams=1))
    tickets = [srv.submit(ti, tm, 400) for _ in range(6)]
    with pytest.raises(fsr.FsrError) as e:
        srv.result(tickets[-1], torch.empty(img.shape))
    assert e.value.status == binding.FSR_ERR_NOT_READY
    srv.close()                                   # must not hang
    # a fresh server still works afterwards
    with fsr.Server(ctx, fsr.make_params(), fsr.make_server_config(hbm_budget=64 << 20)) as srv2:
        t = srv2.submit(ti, tm, 10)
        srv2.wait(t, 20000)
        srv2.release(t)


def test_every_upload_route_gives_the_same_result(ctx):
    """Inputs reach the server's arena by a copy kernel (device memory, strided
    or not, and pinned host frames up to 4 MiB) or by the runtime's copy
    (larger pinned host frames, pageable host memory); every route must give
    the one-image result."""
    announce("uploads: device strided, pinned small and large, pageable")
    small = frames(6)[3]                                   # 128 x 96, pinned: copy kernel
    h, w = 1000, 1100                                      # 5.5 MB: the runtime's copy when pinned
    large = (synth.make_image(h, w, 611).astype(np.float32), synth.make_mask("uniform:0.3", h, w, 612), 40)
    refs = [alone(ctx, *small), alone(ctx, *large)]
    cfg = fsr.make_server_config(hbm_budget=256 << 20, max_inflight=16, max_batch=4, streams=2)
    with fsr.Server(ctx, fsr.make_params(), cfg) as srv:
        tickets = []
        for (img, mask, it), ref in zip((small, large), refs):
            H, W = img.shape
            pad = 7
            bi = torch.zeros((H, W + pad), dtype=torch.float32, device=DEV)
            bm = torch.zeros((H, W + pad), dtype=torch.uint8, device=DEV)
            bi[:, :W] = torch.from_numpy(img)
            bm[:, :W] = torch.from_numpy(mask)
            torch.cuda.synchronize()
            routes = [("device strided", bi[:, :W], bm[:, :W]),
                      ("pinned", torch.from_numpy(img).pin_memory(), torch.from_numpy(mask).pin_memory()),
                      ("pageable", torch.from_numpy(img.copy()), torch.from_numpy(mask.copy()))]
            for name, ti, tm in routes:
                tickets.append((name, H, W, ref, srv.submit(ti, tm, it)))
        for name, H, W, ref, t in tickets:
            srv.wait(t, 30000)
            host = torch.empty((H, W), dtype=torch.float32)
            srv.result(t, host)
            assert np.array_equal(host.numpy(), ref), f"{name} {H}x{W}"
