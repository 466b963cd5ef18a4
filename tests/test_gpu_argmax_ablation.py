"""The shared-memory (LDS) argmax against the register argmax (Sec. IV).

Both reductions order the (objective key, bin) pairs the same way, largest
key first and the smaller bin on equal keys, so a frame reconstructed with
FSR_FLAG_LDS_ARGMAX must be bitwise identical, output and argmax log, to one
reconstructed with the default wavefront reduction; the oracle pins the
LDS variant independently on the small frame.
"""
import numpy as np
import pytest

import oracle
import synth
from synth.metrics import parity_report
from tests.decisions import PREFIX_AGREE, parting_report

torch = pytest.importorskip("torch")
import paper_2202_13926_amd as fsr  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    return fsr.Context(0)


def run(ctx, img, mask, params):
    ti = torch.from_numpy(np.ascontiguousarray(img, np.float32)).to(DEV)
    tm = torch.from_numpy(np.ascontiguousarray(mask, np.uint8)).to(DEV)
    out, lg = fsr.reconstruct(ti, tm, params, ctx=ctx, log=True)
    torch.cuda.synchronize()
    return out.cpu().numpy(), lg.cpu().numpy().view(np.uint16)[:, :params.iterations]


def test_lds_argmax_small64_against_oracle(ctx):
    print("\n[gpu case] LDS argmax: small64 vs the FP64 oracle", flush=True)
    w = synth.workload("small64")
    img, mask = w.inputs()
    img32 = img.astype(np.float32)
    g, gl = run(ctx, img32, mask, fsr.make_params(flags=fsr.FSR_FLAG_LDS_ARGMAX))
    o, ol, _ = oracle.reconstruct(img32.astype(np.float64), mask, w.iterations, log=True)
    rep = parity_report(img32, mask, g, o, gl, ol)
    print(f"[parity] small64 lds-argmax: {rep}", flush=True)
    assert rep["known_bitwise"] and rep["frac_le_1"] >= 0.999 and rep["psnr_gap"] <= 0.05
    assert rep["argmax_agree"] == 1.0


@pytest.mark.parametrize("name,iters", [("small64", 100), ("fhd_quarter", 100), ("uhd_concealment", 20)])
def test_lds_argmax_equals_register_argmax(ctx, name, iters):
    print(f"\n[gpu case] LDS argmax vs register argmax, {name} I={iters}, bitwise", flush=True)
    img, mask = synth.workload(name).inputs()
    a, la = run(ctx, img, mask, fsr.make_params(iterations=iters))
    b, lb = run(ctx, img, mask, fsr.make_params(iterations=iters, flags=fsr.FSR_FLAG_LDS_ARGMAX))
    assert np.array_equal(la, lb)
    assert np.array_equal(a, b)


def test_lds_argmax_edge_cases(ctx):
    print("\n[gpu case] LDS argmax: empty supports, I = 0, ragged 37x50", flush=True)
    img, mask = synth.make_image(96, 96, 9), synth.quarter_mask(96, 96, 10)
    mask[8:88, 8:88] = 0
    for it in (0, 25):
        a, la = run(ctx, img, mask, fsr.make_params(iterations=it))
        b, lb = run(ctx, img, mask, fsr.make_params(iterations=it, flags=fsr.FSR_FLAG_LDS_ARGMAX))
        assert np.array_equal(a, b) and np.array_equal(la, lb)
    img, mask = synth.make_image(37, 50, 41), synth.quarter_mask(37, 50, 42)
    a, la = run(ctx, img, mask, fsr.make_params(iterations=60))
    b, lb = run(ctx, img, mask, fsr.make_params(iterations=60, flags=fsr.FSR_FLAG_LDS_ARGMAX))
    assert np.array_equal(a, b) and np.array_equal(la, lb)


@pytest.mark.parametrize("B,L", [(4, 2), (6, 1), (4, 6), (8, 4), (4, 10)])
def test_lds_argmax_at_smaller_supports(ctx, B, L):
    """Supports 8, 16, 24 (Fig. 3 spans S = 8 to 32): the LDS tree gives the
    register path's result bitwise (at S = 8 with B <= 4 the register path
    takes eight blocks per wavefront, the LDS variant one), and the oracle
    pins it on a ragged frame: the decisions FP32 can resolve agree, and
    the blocks whose decisions all agree match to a code value (a block
    that parts at a near-tie beyond FP32's resolution carries up to B^2
    pixels of this small frame with it)."""
    S = B + 2 * L
    print(f"\n[gpu case] LDS argmax at S = {S} (B={B} L={L})", flush=True)
    img = synth.make_image(90, 75, 3100 + S).astype(np.float32)
    mask = synth.make_mask("quarter", 90, 75, 3200 + S)
    reg = fsr.make_params(block=B, border=L, iterations=80)
    lds = fsr.make_params(block=B, border=L, iterations=80, flags=fsr.FSR_FLAG_LDS_ARGMAX)
    a, la = run(ctx, img, mask, reg)
    b, lb = run(ctx, img, mask, lds)
    assert np.array_equal(a, b) and np.array_equal(la, lb)
    o, ol, _, (obj, sep) = oracle.reconstruct(img.astype(np.float64), mask, 80, block_size=B, border=L,
                                              log=True, separations=True)
    rep = parity_report(img, mask, b, o, lb, ol)
    part = parting_report(mask, b, o, lb, ol, obj, sep, B)
    print(f"[parity] S={S}: {rep} {part}", flush=True)
    assert rep["known_bitwise"] and rep["psnr_gap"] <= 0.05
    assert rep["argmax_agree"] >= 0.99
    assert part["prefix_agree"] >= PREFIX_AGREE
    assert part["agreeing_blocks_frac_le_1"] >= 0.999
