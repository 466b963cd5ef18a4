"""Pins of the oracle's sequential variant that reuses reconstructed pixels.

The paper's method treats every block independently (Sec. II) and says that
it departs from the original FSR there, which lets pixels reconstructed by
earlier blocks take part in later supports with a reduced weight.  The
oracle's `reconstruct_reuse` is that original scheme under the readings in
its header: blocks in raster order, reused pixels weighted delta rho^dist.

The pins check it against facts that do not depend on its own code:
delta = 0 is the block-independent method, the first block has nothing to
reuse, a uniform scaling of the weights changes nothing (Eqs. 7, 10 and 8 are
homogeneous in w), a brute-force restatement of the raster definition built
from block ownership, and causality (a change reaches earlier blocks only
through their own supports; with reuse, also the blocks after the first one
that sees it).  The per-block form (`reconstruct_reuse_given`, each block
handed the frame its reused pixels come from) is pinned to the scan itself
and to exactly which blocks a reused pixel reaches.  Planted slips in a copy
of the C source must fail at least one of them.
"""
import os
import subprocess

import numpy as np
import pytest

import synth


def tiny_case(seed=5, H=22, W=18):
    img = synth.make_image(H, W, seed)
    mask = synth.quarter_mask(H, W, seed + 1)
    return img, mask


def bruteforce_reuse(o, img, mask, iters, delta, B, L, rho, gamma):
    """The raster definition written out pixel by pixel: a support pixel is
    reused when it is missing and the block that owns it has a smaller raster
    index than the current one."""
    H, W = img.shape
    S = B + 2 * L
    nby, nbx = -(-H // B), -(-W // B)
    owner = (np.arange(H)[:, None] // B) * nbx + (np.arange(W)[None, :] // B)
    rp = o.spatial_weight(np.ones((S, S), np.uint8), rho)
    out = np.full((H, W), np.nan)
    logs = []
    for b in range(nby * nbx):
        by, bx = divmod(b, nbx)
        ft, w = np.zeros((S, S)), np.zeros((S, S))
        for m in range(S):
            for n in range(S):
                y, x = by * B - L + m, bx * B - L + n
                if not (0 <= y < H and 0 <= x < W):
                    continue
                if mask[y, x]:
                    ft[m, n], w[m, n] = img[y, x], rp[m, n]
                elif owner[y, x] < b and delta > 0:
                    ft[m, n], w[m, n] = out[y, x], delta * rp[m, n]
        r = o.block_weighted(ft, w, iters, gamma)
        logs.append(r["idx"])
        for i in range(B):
            for j in range(B):
                y, x = by * B + i, bx * B + j
                if y < H and x < W:
                    out[y, x] = img[y, x] if mask[y, x] else o.model_pixel(r["G"], L + i, L + j)
    return out, np.array(logs)


# ---------------------------------------------------------------- delta = 0
def test_delta_zero_is_the_block_independent_method(oracle_lib):
    img, mask = synth.workload("small64").inputs()
    a, la, ea = oracle_lib.reconstruct(img, mask, 40, log=True)
    b, lb, eb = oracle_lib.reconstruct_reuse(img, mask, 40, delta=0.0, log=True)
    assert np.array_equal(a, b) and np.array_equal(la, lb) and ea == eb


# ---------------------------------------------------------------- first block
@pytest.mark.parametrize("delta", [0.25, 0.5, 1.0])
def test_first_block_has_nothing_to_reuse(oracle_lib, delta):
    img, mask = synth.workload("small64").inputs()
    a, la, _ = oracle_lib.reconstruct(img, mask, 40, log=True)
    b, lb, _ = oracle_lib.reconstruct_reuse(img, mask, 40, delta=delta, log=True)
    assert np.array_equal(a[:4, :4], b[:4, :4]) and np.array_equal(la[0], lb[0])
    # and reuse does change later blocks
    assert not np.array_equal(a, b)


# ---------------------------------------------------------------- homogeneity in w
def test_uniform_weight_scaling_is_invisible(oracle_lib):
    """Eqs. 7 and 10 are homogeneous in w: R_w and W scale alike, p and the
    argmax of w_f |R_w|^2 do not change.  Scaling by a power of two is exact
    in binary floating point, so the result is bitwise the same."""
    S = 32
    rng = np.random.default_rng(9)
    known = (rng.random((S, S)) < 0.3).astype(np.uint8)
    ft = np.where(known != 0, rng.uniform(0, 255, (S, S)), 0.0)
    w = oracle_lib.spatial_weight(known, 0.7)
    base = oracle_lib.block_weighted(ft, w, 50, 0.5)
    ref = oracle_lib.block(ft, known, 50, 0.7, 0.5)
    assert np.array_equal(base["G"], ref["G"]) and np.array_equal(base["idx"], ref["idx"])
    half = oracle_lib.block_weighted(ft, 0.5 * w, 50, 0.5)
    assert np.array_equal(half["G"], base["G"]) and np.array_equal(half["idx"], base["idx"])
    odd = oracle_lib.block_weighted(ft, 0.3 * w, 50, 0.5)
    assert np.array_equal(odd["idx"], base["idx"])
    assert np.max(np.abs(odd["G"] - base["G"])) <= 1e-9 * np.max(np.abs(base["G"]))


# ---------------------------------------------------------------- raster definition
@pytest.mark.parametrize("delta,B,L", [(0.5, 4, 6), (1.0, 4, 2), (0.5, 2, 3)])
def test_bruteforce_raster_definition(oracle_lib, delta, B, L):
    img, mask = tiny_case()
    got, lg, _ = oracle_lib.reconstruct_reuse(img, mask, 25, delta=delta, block_size=B,
                                              border=L, log=True)
    ref, lr = bruteforce_reuse(oracle_lib, img, mask, 25, delta, B, L, 0.7, 0.5)
    assert np.array_equal(got, ref)
    assert np.array_equal(lg, lr)


# ---------------------------------------------------------------- causality
@pytest.mark.parametrize("delta", [0.0, 0.5])
def test_changes_reach_later_blocks_only_through_reuse(oracle_lib, delta):
    B, L, H, W = 4, 6, 64, 64
    img, mask = synth.make_image(H, W, 31), synth.quarter_mask(H, W, 32)
    nbx = W // B
    jy, jx = 8, 8                                     # block j = (8, 8)
    img2 = img.copy()
    ys, xs = np.nonzero(mask[jy * B:(jy + 1) * B, jx * B:(jx + 1) * B])
    assert ys.size > 0
    img2[jy * B + ys, jx * B + xs] += 40.0
    a, _, _ = oracle_lib.reconstruct_reuse(img, mask, 30, delta=delta, block_size=B, border=L)
    b, _, _ = oracle_lib.reconstruct_reuse(img2, mask, 30, delta=delta, block_size=B, border=L)
    sees = np.zeros((H // B, nbx), bool)
    for by in range(H // B):
        for bx in range(nbx):
            sees[by, bx] = (by * B - L <= jy * B + B - 1 and jy * B <= by * B + B - 1 + L and
                            bx * B - L <= jx * B + B - 1 and jx * B <= bx * B + B - 1 + L)
    first = int(np.flatnonzero(sees.ravel())[0])      # first block in raster order that sees it
    reached = 0
    for by in range(H // B):
        for bx in range(nbx):
            t = (slice(by * B, by * B + B), slice(bx * B, bx * B + B))
            same = np.array_equal(a[t], b[t])
            if sees[by, bx]:
                continue
            if by * nbx + bx < first or delta == 0.0:
                assert same, (by, bx)
            elif not same:
                reached += 1
    if delta > 0.0:
        assert reached > 0


def test_reuse_keeps_known_pixels_and_fully_known_images(oracle_lib):
    img, mask = synth.workload("small64").inputs()
    out, _, _ = oracle_lib.reconstruct_reuse(img, mask, 30, delta=0.5)
    assert np.array_equal(out[mask != 0], img[mask != 0]) and np.all(np.isfinite(out))
    full, _, _ = oracle_lib.reconstruct_reuse(img, np.ones_like(mask), 20, delta=0.5)
    assert np.array_equal(full, img)


def exact_blocks(Hc, Wc, H, W, B, L):
    """Blocks of a top-left Hc x Wc crop that see exactly what they see in
    the H x W frame: support inside the crop (or cut by the frame's own
    edge) and every reused block exact too.  Returns a (nby, nbx) bool map."""
    nby, nbx = -(-Hc // B), -(-Wc // B)
    ok = np.zeros((nby, nbx), bool)
    for by in range(nby):
        for bx in range(nbx):
            clean = ((by * B + B + L <= Hc or Hc == H) and (bx * B + B + L <= Wc or Wc == W))
            if clean:
                for qy in range(max(0, (by * B - L) // B), by + 1):
                    for qx in range(max(0, (bx * B - L) // B), min(nbx, (bx * B + B + L - 1) // B + 1)):
                        if (qy, qx) < (by, bx) and not ok[qy, qx]:
                            clean = False
            ok[by, bx] = clean
    return ok


def test_crop_blocks_see_the_full_frame(oracle_lib):
    """The crop argument the GPU test relies on: the blocks exact_blocks
    selects come out bitwise the same from a crop as from the whole frame."""
    H, W, Hc, Wc, B, L = 64, 160, 40, 96, 4, 14
    img, mask = synth.make_image(H, W, 41), synth.quarter_mask(H, W, 42)
    full, _, _ = oracle_lib.reconstruct_reuse(img, mask, 30, delta=0.5, block_size=B, border=L)
    crop, _, _ = oracle_lib.reconstruct_reuse(img[:Hc, :Wc], mask[:Hc, :Wc], 30, delta=0.5,
                                              block_size=B, border=L)
    ok = exact_blocks(Hc, Wc, H, W, B, L)
    sel = np.kron(ok, np.ones((B, B), bool))[:Hc, :Wc]
    assert 20 < ok.sum() < ok.size
    assert np.array_equal(full[:Hc, :Wc][sel], crop[sel])
    # and the selection is not trivially small: the next blocks out differ
    assert not np.array_equal(full[:Hc, :Wc][~sel], crop[~sel])


# ---------------------------------------------------------------- each block given the reused frame
GIVEN_CASES = [
    (64, 64, "quarter", 4, 14, 100, 0.5),
    (22, 18, "quarter", 2, 3, 25, 1.0),
    (40, 52, "macroblock", 4, 6, 60, 0.25),
    (37, 9, "uniform:0.4", 4, 14, 40, 0.5),
]


@pytest.mark.parametrize("case", GIVEN_CASES)
def test_given_own_output_reproduces_the_sequential_scan(oracle_lib, case):
    """Each block of the scan reads its reused pixels from blocks that are
    final by then, so handing every block the scan's own finished frame gives
    each one the very inputs it had inside the scan: output and log bitwise
    equal, for square, wide and one-column frames and every mask kind."""
    H, W, mk, B, L, iters, delta = case
    img = synth.make_image(H, W, 3100 + H)
    mask = synth.make_mask(mk, H, W, 3200 + W)
    seq, ls, es = oracle_lib.reconstruct_reuse(img, mask, iters, delta=delta, block_size=B,
                                               border=L, log=True)
    got, lg, eg = oracle_lib.reconstruct_reuse_given(img, mask, seq, iters, delta=delta,
                                                     block_size=B, border=L, log=True)
    assert np.array_equal(got, seq) and np.array_equal(lg, ls) and eg == es


def test_given_delta_zero_is_the_block_independent_method(oracle_lib):
    img, mask = synth.workload("small64").inputs()
    junk = np.full(img.shape, 1.0e6)
    a, la, _ = oracle_lib.reconstruct(img, mask, 40, log=True)
    b, lb, _ = oracle_lib.reconstruct_reuse_given(img, mask, junk, 40, delta=0.0, log=True)
    assert np.array_equal(a, b) and np.array_equal(la, lb)


def test_given_frame_reaches_exactly_the_later_supports(oracle_lib):
    """A change of the given frame at a known pixel changes nothing (known
    pixels come from the input).  A change at a missing pixel p changes
    exactly the blocks that reuse p: those whose support holds p and that
    come after p's own block in raster order (Sec. II's original method
    reuses only what earlier blocks reconstructed)."""
    B, L, H, W = 4, 6, 48, 56
    img, mask = synth.make_image(H, W, 71), synth.quarter_mask(H, W, 72)
    base, _, _ = oracle_lib.reconstruct_reuse(img, mask, 30, delta=0.5, block_size=B, border=L)
    a, _, _ = oracle_lib.reconstruct_reuse_given(img, mask, base, 30, delta=0.5, block_size=B,
                                                 border=L)
    nby, nbx = H // B, W // B
    ky, kx = np.argwhere(mask[20:24, 24:28] != 0)[0] + (20, 24)
    moved = base.copy()
    moved[ky, kx] += 50.0
    b, _, _ = oracle_lib.reconstruct_reuse_given(img, mask, moved, 30, delta=0.5, block_size=B,
                                                 border=L)
    assert np.array_equal(a, b)
    py, px = np.argwhere(mask[20:24, 24:28] == 0)[0] + (20, 24)
    moved = base.copy()
    moved[py, px] += 50.0
    b, _, _ = oracle_lib.reconstruct_reuse_given(img, mask, moved, 30, delta=0.5, block_size=B,
                                                 border=L)
    own = (py // B) * nbx + px // B
    for by in range(nby):
        for bx in range(nbx):
            t = (slice(by * B, by * B + B), slice(bx * B, bx * B + B))
            inside = by * B - L <= py < by * B + B + L and bx * B - L <= px < bx * B + B + L
            reuses = inside and by * nbx + bx > own
            assert np.array_equal(a[t], b[t]) != reuses, (by, bx)


# ---------------------------------------------------------------- sensitivity
def perturbed_spread(o, img, mask, iters, delta, B, L, seeds=(0, 1, 2), sel=None, rel=1e-6):
    """How far the reuse variant moves when the known pixels change by a
    relative ``rel`` (1e-6 by default, below the resolution of a float32
    frame): the worst, over ``seeds``, of the share of reconstructed pixels
    within 1 code value, the argmax agreement and the PSNR gap, against the
    unperturbed result.  ``sel`` restricts the comparison to a pixel mask
    (and the argmax to the blocks it covers)."""
    from synth.metrics import parity_report
    H, W = img.shape
    a, la, _ = o.reconstruct_reuse(img, mask, iters, delta=delta, block_size=B, border=L, log=True)
    worst = {"frac_le_1": 1.0, "argmax_agree": 1.0, "psnr_gap": 0.0}
    for s in seeds:
        rng = np.random.default_rng(s)
        pert = img * (1.0 + rel * rng.standard_normal(img.shape))
        b, lb, _ = o.reconstruct_reuse(pert, mask, iters, delta=delta, block_size=B, border=L,
                                       log=True)
        if sel is None:
            rep = parity_report(img, mask, b, a, lb, la)
        else:
            blocks = np.kron(sel, np.ones((B, B), bool))[:H, :W]
            ids = np.flatnonzero(sel.ravel())
            rep = parity_report(img[blocks], mask[blocks], b[blocks], a[blocks], lb[ids], la[ids])
        for k in ("frac_le_1", "argmax_agree"):
            worst[k] = min(worst[k], rep[k])
        worst["psnr_gap"] = max(worst["psnr_gap"], rep["psnr_gap"])
    return a, la, worst


def test_reuse_amplifies_rounding_level_changes(oracle_lib):
    """The chain of reuse carries any change of a block's decisions into every
    later block that reuses it.  With the quarter mask at I = 100 a relative
    change of 1e-6 of the input, far below what a float32 frame resolves,
    flips a near-tied argmax somewhere and the flip spreads; the
    block-independent method moves in at most a block or two.  With fewer
    iterations, or masks whose late objectives are not crowded, the reuse
    variant does not move at all: those are the regimes where element-wise
    parity is meaningful."""
    img = synth.make_image(64, 64, 2164).astype(np.float32).astype(np.float64)
    mask = synth.make_mask("quarter", 64, 64, 2264)
    _, _, chaotic = perturbed_spread(oracle_lib, img, mask, 100, 0.5, 4, 14)
    assert chaotic["argmax_agree"] < 0.9 and chaotic["frac_le_1"] < 0.99
    assert chaotic["psnr_gap"] <= 0.05                 # the quality does not move
    rng = np.random.default_rng(0)
    pert = img * (1.0 + 1e-6 * rng.standard_normal(img.shape))
    _, la, _ = oracle_lib.reconstruct(img, mask, 100, log=True)
    _, lb, _ = oracle_lib.reconstruct(pert, mask, 100, log=True)
    assert (la != lb).any(axis=1).sum() <= 2
    for (H, W, mk, B, L, iters, delta) in STABLE_CASES:
        img = synth.make_image(H, W, 2100 + H).astype(np.float32).astype(np.float64)
        mask = synth.make_mask(mk, H, W, 2200 + W)
        _, _, w = perturbed_spread(oracle_lib, img, mask, iters, delta, B, L)
        assert w["frac_le_1"] == 1.0 and w["argmax_agree"] >= 0.99, (H, W, mk, B, L, iters)


# (H, W, mask, B, L, I, delta): cases in which the reuse variant does not move
# under a rounding-level change of its input (checked above)
STABLE_CASES = [
    (64, 64, "quarter", 4, 14, 50, 0.5),
    (64, 64, "quarter", 2, 15, 30, 0.5),
    (37, 9, "quarter", 4, 14, 60, 0.5),          # one block column: empty wavefront steps
    (70, 45, "uniform:0.3", 4, 14, 100, 1.0),
    (72, 80, "macroblock", 8, 12, 100, 0.25),
    (96, 96, "macroblock", 4, 14, 100, 0.5),
]


# ---------------------------------------------------------------- planted slips
MUTANTS = {
    "column_major_order": ("const int earlier = y < by * B || (y < (by + 1) * B && x < bx * B);",
                           "const int earlier = x < bx * B || (x < (bx + 1) * B && y < by * B);"),
    "reuses_current_block": ("const int earlier = y < by * B || (y < (by + 1) * B && x < bx * B);",
                             "const int earlier = y < by * B || (y < (by + 1) * B && x < (bx + 1) * B);"),
    "reused_value_from_input": ("reused ? src[(long)y * stride + x] : 0.0;",
                                "reused ? img[(long)y * stride + x] : 0.0;"),
    "given_frame_ignored": ("empty += reuse_block(img, mask, reused, out,",
                            "empty += reuse_block(img, mask, img, out,"),
    "given_blocks_shifted": ("tie_larger, (int)(b / nbx), (int)(b % nbx),",
                             "tie_larger, (int)(b % nbx), (int)(b / nbx),"),
    "reused_weight_without_delta": ("reused ? delta * rp[i] : 0.0;", "reused ? rp[i] : 0.0;"),
    "delta_on_known_pixels": ("w[i] = k ? rp[i] :", "w[i] = k ? delta * rp[i] :"),
}

PIN_CALLS = [
    test_delta_zero_is_the_block_independent_method,
    lambda o: test_first_block_has_nothing_to_reuse(o, 0.5),
    test_uniform_weight_scaling_is_invisible,
    lambda o: test_bruteforce_raster_definition(o, 0.5, 4, 6),
    lambda o: test_changes_reach_later_blocks_only_through_reuse(o, 0.5),
    test_reuse_keeps_known_pixels_and_fully_known_images,
    lambda o: test_given_own_output_reproduces_the_sequential_scan(o, GIVEN_CASES[1]),
    test_given_delta_zero_is_the_block_independent_method,
    test_given_frame_reaches_exactly_the_later_supports,
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_reuse_mutant(tmp_path, name):
    import oracle
    before, after = MUTANTS[name]
    src = open(os.path.join(os.path.dirname(oracle.__file__), "fsr_oracle.c")).read()
    assert src.count(before) == 1, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(before, after))
    lib = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-w", str(path), "-o", str(lib), "-lm"])
    saved = (oracle._LIB, oracle._lib)
    oracle._LIB, oracle._lib = str(lib), None
    try:
        caught = 0
        for call in PIN_CALLS:
            try:
                call(oracle)
            except AssertionError:
                caught += 1
    finally:
        oracle._LIB, oracle._lib = saved
    assert caught, f"no pin caught mutant {name}"
