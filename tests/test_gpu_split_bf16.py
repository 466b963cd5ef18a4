"""Split-bf16 forward DFTs on the matrix cores (dft = FSR_DFT_SPLIT_BF16).

Both forward transforms of a block (R_w and W, Eq. 7) run as bf16 matrix
products with FP32 accumulation, every operand split into three bf16 terms
(hi + mid + lo); the rest of the block routine is the FP32 one.  The same
acceptance bar as the FP32 path applies, against the same FP64 oracle: known
pixels bitwise, |gpu - oracle| <= 1 code value on >= 99.9 % of the unknown
pixels, PSNR gap <= 0.05 dB, argmax agreement >= 99 %, and all but 1e-5 of
the decisions of the blocks' resolvable prefixes (tests/decisions.py).  Each case prints its
error figures next to those of the FP32 FFT path on the same input, so the
error of each transform is stated per result.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.decisions import PREFIX_AGREE, decision_report
from tests.frames import oracle_frame
from synth.metrics import parity_report

torch = pytest.importorskip("torch")
import paper_2202_13926_amd as fsr  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL_FRAC = 0.999
PSNR_GAP = 0.05
ARGMAX = 0.99
BF16 = fsr.FSR_DFT_SPLIT_BF16


@pytest.fixture(scope="module")
def ctx():
    return fsr.Context(0)


def announce(name):
    print(f"\n[gpu case] {name}", flush=True)


def params_of(w, dft):
    return fsr.make_params(block=w.block, border=w.border, iterations=w.iterations, rho=w.rho,
                           gamma=w.gamma, dft=dft)


def run(ctx, img, mask, params):
    ti = torch.from_numpy(np.ascontiguousarray(img, np.float32)).to(DEV)
    tm = torch.from_numpy(np.ascontiguousarray(mask, np.uint8)).to(DEV)
    out, lg = fsr.reconstruct(ti, tm, params, ctx=ctx, log=True)
    torch.cuda.synchronize()
    return out.cpu().numpy(), lg.cpu().numpy().view(np.uint16)[:, :params.iterations]


def check(rep, name):
    print(f"[parity] {name}: {rep}", flush=True)
    assert rep["known_bitwise"]
    assert rep["frac_le_1"] >= TOL_FRAC
    assert rep["psnr_gap"] <= PSNR_GAP
    if "argmax_agree" in rep:
        assert rep["argmax_agree"] >= ARGMAX


def check_decisions(gl, ol, obj, sep, name):
    dec = decision_report(gl, ol, obj, sep)
    print(f"[decisions] {name}: {dec}", flush=True)
    assert dec["prefix_agree"] >= PREFIX_AGREE, dec


def test_small64_against_oracle(ctx):
    announce("split-bf16 DFT: small64 64x64 quarter I=100, every pixel")
    w = synth.workload("small64")
    img, mask = w.inputs()
    img32 = img.astype(np.float32)
    o, ol, _, (obj, sep) = oracle.reconstruct(img32.astype(np.float64), mask, w.iterations, log=True,
                                              separations=True)
    for dft, tag in ((fsr.FSR_DFT_FP32, "fp32"), (BF16, "split-bf16")):
        g, gl = run(ctx, img32, mask, params_of(w, dft))
        rep = parity_report(img32, mask, g, o, gl, ol)
        check(rep, f"small64 {tag}")
        check_decisions(gl, ol, obj, sep, f"small64 {tag}")


@pytest.mark.parametrize("name", ["fhd_quarter", "uhd_concealment"])
def test_full_frames_every_block(ctx, name):
    """The 1080p quarter frame (I = 100) and the 2160p concealment frame
    (I = 200) through both DFT modes, each against the oracle on every block
    and every logged (block, iteration)."""
    announce(f"split-bf16 DFT: {name}, full frame, every block, beside the FP32 FFTs")
    w = synth.workload(name)
    img32, mask, o, ol, obj, sep = oracle_frame(name)
    for dft, tag in ((fsr.FSR_DFT_FP32, "fp32"), (BF16, "split-bf16")):
        g, gl = run(ctx, img32, mask, params_of(w, dft))
        assert np.array_equal(g[mask != 0], img32[mask != 0])
        assert np.all(np.isfinite(g))
        check(parity_report(img32, mask, g, o, gl, ol), f"{name} {tag} every block")
        check_decisions(gl, ol, obj, sep, f"{name} {tag} every block")


def test_edge_cases_against_oracle(ctx):
    announce("split-bf16 DFT: ragged frame, empty supports, I = 0, fully known")
    img, mask = synth.make_image(96, 100, 9), synth.quarter_mask(96, 100, 10)
    mask[8:88, 8:88] = 0                      # a hole: supports without known pixels
    img32 = img.astype(np.float32)
    p = fsr.make_params(iterations=40, dft=BF16)
    g, gl = run(ctx, img32, mask, p)
    o, ol, n_empty = oracle.reconstruct(img32.astype(np.float64), mask, 40, log=True)
    assert n_empty > 0
    check(parity_report(img32, mask, g, o, gl, ol), "hole 96x100")
    assert np.all(gl[np.all(ol == 0xFFFF, axis=1)] == 0xFFFF)

    g0, _ = run(ctx, img32, mask, fsr.make_params(iterations=0, dft=BF16))
    assert np.all(g0[mask == 0] == 0.0)
    g1, _ = run(ctx, img32, np.ones_like(mask), fsr.make_params(iterations=10, dft=BF16))
    assert np.array_equal(g1, img32)


def test_batched_and_served_equal_plain(ctx):
    announce("split-bf16 DFT: batched kernel and server equal one-image calls bitwise")
    shapes = [(64, 64, "quarter", 100), (37, 50, "uniform:0.3", 25), (150, 200, "macroblock", 100),
              (8, 8, "quarter", 60)]
    batch = []
    for i, (h, wd, mk, it) in enumerate(shapes):
        batch.append((synth.make_image(h, wd, 700 + i).astype(np.float32),
                      synth.make_mask(mk, h, wd, 750 + i), it))
    refs = [run(ctx, img, mask, fsr.make_params(iterations=it, dft=BF16)) for img, mask, it in batch]

    items = []
    for img, mask, it in batch:
        ti, tm = torch.from_numpy(img).to(DEV), torch.from_numpy(mask).to(DEV)
        n = fsr.fsr_num_blocks(img.shape[0], img.shape[1], 4)
        items.append(fsr.BatchItem(ti, tm, torch.full_like(ti, -1.0), it,
                                   torch.full((n, max(it, 1)), -1, dtype=torch.int16, device=DEV)))
    ws = fsr.Workspace(len(items), DEV)
    for sched in (fsr.make_schedule(1, 0, 10), fsr.make_schedule(2, 4, 5)):
        fsr.fsr_reconstruct_batched(ctx, items, fsr.make_params(dft=BF16), ws, schedule=sched)
        torch.cuda.synchronize()
        for k, (item, (r, rl)) in enumerate(zip(items, refs)):
            assert np.array_equal(item.out.cpu().numpy(), r), f"batched image {k}"
            gl = item.argmax_log.cpu().numpy().view(np.uint16)[:, :item.iterations]
            assert np.array_equal(gl, rl), f"batched log {k}"

    with fsr.Server(ctx, fsr.make_params(dft=BF16), fsr.make_server_config(streams=1)) as srv:
        tickets = [srv.submit(torch.from_numpy(img).to(DEV), torch.from_numpy(mask).to(DEV), it)
                   for img, mask, it in batch]
        for k, (t, (r, _)) in enumerate(zip(tickets, refs)):
            srv.wait(t, 60000)
            out = torch.empty(batch[k][0].shape, dtype=torch.float32, device=DEV)
            srv.result(t, out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), r), f"served image {k}"
