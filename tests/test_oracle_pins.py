"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a textbook
library routine (numpy's FFT and least squares), a closed form, an invariant of
the method or a brute-force search.  Together they are chosen so that a
plausible slip anywhere in the oracle (a dropped term, a wrong sign or index,
a transposed operand, a wrong normalisation) fails at least one of them.
"""
import numpy as np
import pytest

import synth


def np_weight(known, rho):
    """Eq. 5 retyped independently for the checks: rho^dist on known pixels."""
    S = known.shape[0]
    c = (S - 1) / 2.0
    m = np.arange(S) - c
    d = np.sqrt(m[:, None] ** 2 + m[None, :] ** 2)
    return np.where(known != 0, rho ** d, 0.0)


def np_freq_weight(S):
    kt = S / 2.0 - np.abs(np.arange(S) - S / 2.0)
    return (1.0 - np.sqrt(2.0) * np.sqrt(kt[:, None] ** 2 / S ** 2 + kt[None, :] ** 2 / S ** 2)) ** 2


def random_support(S, seed, known_frac=None):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.0, 255.0, (S, S))
    if known_frac is None:
        known = synth.quarter_mask(S, S, seed + 7)
    else:
        known = (rng.random((S, S)) < known_frac).astype(np.uint8)
    known[S // 2, S // 2] = 1
    return np.where(known != 0, f, 0.0), known


def mirror(idx, S):
    k, l = divmod(int(idx), S)
    return ((S - k) % S) * S + (S - l) % S


# ---------------------------------------------------------------- P1: DFT convention
@pytest.mark.parametrize("S", [4, 6, 8, 16, 24, 32])
def test_dft_matches_numpy_fft2(oracle_lib, S):
    """O4 uses numpy's convention: unnormalised, exp(-j 2 pi (km + ln)/S), k along rows."""
    rng = np.random.default_rng(S)
    x = rng.normal(size=(S, S))
    x[0, 1] += 3.0  # make rows and columns distinguishable
    X = oracle_lib.dft2_real(x)
    ref = np.fft.fft2(x)
    assert np.max(np.abs(X - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_twiddle_table_exact_symmetry(oracle_lib):
    # reference in extended precision (x87 long double, 64-bit mantissa): a
    # double-precision exp(-2j pi q / S) carries its own angle rounding (up
    # to 1.5e-15 at q near S for S = 24).  The table itself is cos / sin of
    # the double-rounded angle 2 pi q / S (q <= S/2, mirrored above): the
    # angle's rounding (<= half an ulp of 2 pi, 4.4e-16) plus the libm
    # rounding bound each entry's error by about 2 ulp of 1 (4.4e-16).
    pi_l = np.longdouble("3.14159265358979323846264338327950288")
    for S in (8, 16, 24, 32):
        t = oracle_lib.twiddles(S)
        assert t[0] == 1.0
        assert t[S // 4] == -1j and t[S // 2] == -1.0 and t[3 * S // 4] == 1j
        for q in range(1, S):
            assert t[S - q] == np.conj(t[q])
        ang = 2 * pi_l * np.arange(S, dtype=np.longdouble) / np.longdouble(S)
        err_re = np.abs(t.real.astype(np.longdouble) - np.cos(ang))
        err_im = np.abs(t.imag.astype(np.longdouble) + np.sin(ang))
        assert float(max(err_re.max(), err_im.max())) <= 4.5e-16


# ---------------------------------------------------------------- weights
def test_weights_closed_form(oracle_lib):
    S = 32
    known = synth.quarter_mask(S, S, 3)
    w = oracle_lib.spatial_weight(known, 0.7)
    assert np.allclose(w, np_weight(known, 0.7), rtol=1e-14, atol=0)
    assert np.all(w[known == 0] == 0.0)
    # centre (S-1)/2 = 15.5: the four central pixels sit at distance sqrt(0.5)
    full = oracle_lib.spatial_weight(np.ones((S, S), np.uint8), 0.7)
    assert full[15, 15] == full[16, 16] == full[15, 16] == full[16, 15]
    assert abs(full[15, 15] - 0.7 ** np.sqrt(0.5)) < 1e-15
    assert np.array_equal(full, full[::-1, :]) and np.array_equal(full, full.T)
    wf = oracle_lib.freq_weight(S)
    assert np.allclose(wf, np_freq_weight(S), rtol=1e-14, atol=1e-30)
    assert wf[0, 0] == 1.0 and abs(wf[16, 16]) < 1e-30
    assert abs(wf[0, 1] - (1 - np.sqrt(2) / 32) ** 2) < 1e-15
    # symmetric under k -> S-k (needed for exact ties between mirror bins)
    for k in range(S):
        for l in range(S):
            assert wf[k, l] == wf[(S - k) % S, (S - l) % S]


# ---------------------------------------------------------------- P9: bitwise Hermitian
@pytest.mark.parametrize("S", [8, 16, 24, 32])
def test_spectra_bitwise_hermitian(oracle_lib, S):
    ft, known = random_support(S, 11)
    w = np_weight(known, 0.7)
    for x in (ft * w, w, ft):
        Xr, Xi = oracle_lib.dft2_real_parts(x)
        Xr_m = np.roll(Xr[::-1, ::-1], 1, axis=(0, 1))
        Xi_m = np.roll(Xi[::-1, ::-1], 1, axis=(0, 1))
        assert np.array_equal(Xr, Xr_m)
        assert np.array_equal(Xi, -Xi_m)
        h = S // 2
        for k, l in ((0, 0), (0, h), (h, 0), (h, h)):
            assert Xi[k, l] == 0.0


def test_residual_stays_hermitian_after_self_conjugate_picks(oracle_lib):
    ft, known = random_support(32, 12)
    res = oracle_lib.block(ft, known, 1, 0.7, 0.5)
    assert res["idx"][0] == 0  # DC dominates a [0,255] image
    Rr, Ri = res["Rr"], res["Ri"]
    assert np.array_equal(Rr, np.roll(Rr[::-1, ::-1], 1, axis=(0, 1)))
    assert np.array_equal(Ri, -np.roll(Ri[::-1, ::-1], 1, axis=(0, 1)))


# ---------------------------------------------------------------- P2: orthogonal case
def test_orthogonal_case_recovers_fft(oracle_lib):
    """All pixels known and rho = 1: w = 1, W = S^2 delta, so every pick copies
    one DFT coefficient of f into G and zeroes it in R (gamma = 1)."""
    S = 8
    rng = np.random.default_rng(5)
    f = rng.uniform(0, 255, (S, S))
    known = np.ones((S, S), np.uint8)
    F = np.fft.fft2(f)
    wf = np_freq_weight(S)
    n_pick = S * S - 1                      # bin (S/2, S/2) has w_f = 0
    res = oracle_lib.block(f, known, n_pick, 1.0, 1.0)
    picks = res["idx"].astype(int)
    assert sorted(picks) == sorted(set(range(S * S)) - {(S // 2) * S + S // 2})
    obj = (wf * np.abs(F) ** 2).ravel()[picks]
    assert np.all(np.diff(obj) <= 1e-9 * obj[0])
    # mirror bins tie exactly (Hermitian spectrum); the smaller index goes first
    pos = {int(b): i for i, b in enumerate(picks)}
    for b in picks:
        mb = mirror(b, S)
        if mb != b:
            assert (pos[b] < pos[mb]) == (b < mb)
    G = res["G"]
    mask = np.ones((S, S), bool)
    mask[S // 2, S // 2] = False
    assert np.max(np.abs(G[mask] - F[mask])) <= 1e-12 * np.max(np.abs(F))
    assert G[S // 2, S // 2] == 0
    # O7 against numpy's inverse FFT of the same G
    g = np.fft.ifft2(G).real
    for m in range(S):
        for n in range(S):
            assert abs(oracle_lib.model_pixel(G, m, n) - g[m, n]) < 1e-11


# ---------------------------------------------------------------- P3: energy descent
@pytest.mark.parametrize("gamma,S", [(0.3, 32), (0.5, 32), (1.0, 32), (0.5, 16), (0.5, 24)])
def test_energy_descent_closed_form(oracle_lib, gamma, S):
    """E(v+1) = E(v) - (2 gamma - gamma^2) |R(v)[u,v]|^2 / W[0,0], with E the
    weighted spatial residual energy (Eqs. 3-4) of the model built from the
    logged picks, evaluated independently with numpy."""
    I, rho = 60, 0.7
    ft, known = random_support(S, 21)
    res = oracle_lib.block(ft, known, I, rho, gamma)
    w = np_weight(known, rho)
    w00 = w.sum()
    G = np.zeros((S, S), complex)

    def energy(G):
        g = np.fft.ifft2(G)
        return np.sum(w * np.abs(ft - g) ** 2)

    E = [energy(G)]
    for it in range(I):
        u, v = divmod(int(res["idx"][it]), S)
        G[u, v] += gamma * res["p"][it] * S * S
        E.append(energy(G))
    E = np.array(E)
    drop = (2 * gamma - gamma ** 2) * np.abs(res["p"]) ** 2 * w00
    assert np.max(np.abs((E[:-1] - E[1:]) - drop)) <= 1e-10 * E[0]
    assert np.all(np.diff(E) <= 1e-10 * E[0])
    assert np.allclose(G, res["G"], rtol=0, atol=1e-9 * np.abs(G).max())


# ---------------------------------------------------------------- P4: residual consistency
@pytest.mark.parametrize("S", [16, 24, 32])
def test_residual_matches_definition(oracle_lib, S):
    """After I iterations R_w == DFT2((f~ - g) w) (Eqs. 4, 6, 7 and linearity)."""
    I, rho, gamma = 80, 0.7, 0.5
    ft, known = random_support(S, 31)
    res = oracle_lib.block(ft, known, I, rho, gamma)
    w = np_weight(known, rho)
    R0 = np.fft.fft2(ft * w)
    g = np.fft.ifft2(res["G"])
    R_def = np.fft.fft2((ft - g) * w)
    assert np.max(np.abs(res["R"] - R_def)) <= 1e-11 * np.max(np.abs(R0))


# ---------------------------------------------------------------- P5: brute-force first step
@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_first_step_matches_bruteforce_least_squares(oracle_lib, seed):
    """8x8 toy: for every atom phi_kl solve min_c sum w |f~ - c phi_kl|^2 with
    numpy.linalg.lstsq; the greedy step must pick argmax w_f * dE and p = c*."""
    S, rho, gamma = 8, 0.7, 0.5
    ft, known = random_support(S, 100 + seed)
    w = np_weight(known, rho)
    sw = np.sqrt(w).ravel()
    m = np.arange(S)
    E0 = np.sum(w * ft ** 2)
    wf = np_freq_weight(S)
    gain = np.empty((S, S))
    coef = np.empty((S, S), complex)
    for k in range(S):
        for l in range(S):
            phi = np.exp(2j * np.pi * (k * m[:, None] + l * m[None, :]) / S).ravel()
            c, *_ = np.linalg.lstsq((sw * phi)[:, None], (sw * ft.ravel()).astype(complex),
                                    rcond=None)
            coef[k, l] = c[0]
            gain[k, l] = E0 - np.sum(w.ravel() * np.abs(ft.ravel() - c[0] * phi) ** 2)
    score = (wf * gain).ravel()
    best = int(np.argmax(score))
    # the oracle breaks exact ties by the smaller index; brute force decides
    # near-ties only up to its own round-off
    near = np.flatnonzero(score >= score[best] * (1 - 1e-12))
    res = oracle_lib.block(ft, known, 1, rho, gamma)
    assert int(res["idx"][0]) == int(near.min())
    u, v = divmod(int(res["idx"][0]), S)
    assert abs(res["p"][0] - coef[u, v]) <= 1e-12 * abs(coef[u, v])
    # energy after the relaxed step
    phi = np.exp(2j * np.pi * (u * m[:, None] + v * m[None, :]) / S)
    E1 = np.sum(w * np.abs(ft - gamma * res["p"][0] * phi) ** 2)
    assert abs(E1 - (E0 - (2 * gamma - gamma ** 2) * gain[u, v])) <= 1e-12 * E0


# ---------------------------------------------------------------- P6: sinusoid recovery
@pytest.mark.parametrize("k0,l0", [(0, 1), (1, 2), (2, 1), (3, 5)])
@pytest.mark.parametrize("rho", [0.7, 0.9])
def test_grid_sinusoid_recovered(oracle_lib, k0, l0, rho):
    """A cosine on the 32-point DFT grid is exactly two atoms of every support
    block.  While the greedy loop only picks those two atoms it is coordinate
    descent on a two-unknown weighted least-squares problem whose unique
    solution is the cosine itself, so the block is recovered to round-off.
    With a broad spatial weight (rho = 0.9) every block stays on the atoms;
    with rho = 0.7 some blocks pick a third atom with a large coefficient,
    and are then not expected to be exact."""
    H = W = 64
    y = np.arange(H)[:, None]
    x = np.arange(W)[None, :]
    A = 50.0
    f = A * np.cos(2 * np.pi * (k0 * y + l0 * x) / 32 + 0.3)
    mask = synth.quarter_mask(H, W, 5)
    ids = np.arange(256)
    tg, lg, p, n_empty = oracle_lib.reconstruct_blocks(f, mask, ids, 200, rho=rho, gamma=0.5,
                                                       log=True, log_p=True)
    assert n_empty == 0
    atoms = {k0 * 32 + l0, mirror(k0 * 32 + l0, 32)}
    on_atoms = np.array([set(r[np.abs(pp) >= 1e-6 * A].tolist()) <= atoms
                         for r, pp in zip(lg, p)])
    ref = f.reshape(16, 4, 16, 4).transpose(0, 2, 1, 3).reshape(256, 4, 4)
    err = np.abs(tg - ref).reshape(256, 16).max(axis=1)
    assert np.all(err[on_atoms] <= 1e-9 * A)
    if rho == 0.9:
        assert on_atoms.all()
        # the first pick of every block is one of the two atoms of the cosine
        assert set(np.unique(lg[:, 0]).tolist()) <= atoms
    else:
        assert on_atoms.mean() > 0.4


# ---------------------------------------------------------------- P7: compose
def test_fully_known_image_unchanged(oracle_lib):
    img, _ = synth.workload("small64").inputs()
    out, _, _ = oracle_lib.reconstruct(img, np.ones_like(img, np.uint8), 20)
    assert np.array_equal(out, img)


def test_known_pixels_copied_bitwise(oracle_lib):
    img, mask = synth.workload("small64").inputs()
    out, _, _ = oracle_lib.reconstruct(img, mask, 30)
    assert np.array_equal(out[mask != 0], img[mask != 0])
    assert np.all(np.isfinite(out))


# ---------------------------------------------------------------- P8: tie rule
def test_tie_rule_only_mirrors_the_log(oracle_lib):
    """Exact ties occur between mirror bins of a Hermitian residual; either
    choice yields the conjugate model, whose real part is the same."""
    img, mask = synth.workload("small64").inputs()
    a, la, _ = oracle_lib.reconstruct(img, mask, 60, log=True)
    b, lb, _ = oracle_lib.reconstruct(img, mask, 60, log=True, tie_larger=True)
    assert np.max(np.abs(a - b)) <= 1e-9
    differ = 0
    for blk in range(la.shape[0]):
        d = np.flatnonzero(la[blk] != lb[blk])
        if d.size:
            differ += 1
            assert lb[blk, d[0]] == mirror(la[blk, d[0]], 32)
    assert differ > la.shape[0] // 2


# ---------------------------------------------------------------- P10: block independence
def test_translation_by_block_multiple(oracle_lib):
    img, mask = synth.make_image(64, 96, 77), synth.quarter_mask(64, 96, 78)
    out, _, _ = oracle_lib.reconstruct(img, mask, 40)
    sh = 8
    img2 = np.zeros((64, 96 + sh))
    mask2 = np.zeros((64, 96 + sh), np.uint8)
    img2[:, sh:] = img
    mask2[:, sh:] = mask
    out2, _, _ = oracle_lib.reconstruct(img2, mask2, 40)
    # blocks whose support sees only the copied content (or only unknown pixels
    # outside the image in both frames) are bitwise identical
    assert np.array_equal(out2[:, sh:], out)


def test_output_depends_only_on_support(oracle_lib):
    img, mask = synth.workload("small64").inputs()
    ids = np.array([0, 37, 255])
    a, la, _, _ = oracle_lib.reconstruct_blocks(img, mask, ids, 40, log=True)
    img2 = img.copy()
    mask2 = mask.copy()
    # block 37 = (by 2, bx 5): support rows -6..25, cols 6..37; change far away
    img2[40:, :] = 255.0 - img2[40:, :]
    mask2[50:, :] = 1
    b, lb, _, _ = oracle_lib.reconstruct_blocks(img2, mask2, ids[1:2], 40, log=True)
    assert np.array_equal(a[1], b[0]) and np.array_equal(la[1], lb[0])


# ---------------------------------------------------------------- P11: degenerate cases
def test_zero_iterations_gives_zero_model(oracle_lib):
    img, mask = synth.workload("small64").inputs()
    out, _, n_empty = oracle_lib.reconstruct(img, mask, 0)
    assert n_empty == 0
    assert np.all(out[mask == 0] == 0.0)
    assert np.array_equal(out[mask != 0], img[mask != 0])


def test_support_without_known_pixels(oracle_lib):
    H = W = 96
    img = synth.make_image(H, W, 9)
    mask = synth.quarter_mask(H, W, 10)
    mask[8:88, 8:88] = 0                  # hole larger than a 32x32 support
    out, lg, n_empty = oracle_lib.reconstruct(img, mask, 25, log=True)
    # count supports without known pixels independently
    B, L = 4, 14
    expect = 0
    empty_blocks = []
    for by in range(H // B):
        for bx in range(W // B):
            y0, x0 = by * B - L, bx * B - L
            sub = mask[max(y0, 0):y0 + 32, max(x0, 0):x0 + 32]
            if not sub.any():
                expect += 1
                empty_blocks.append(by * (W // B) + bx)
    assert expect > 0 and n_empty == expect
    for b in empty_blocks:
        by, bx = divmod(b, W // B)
        assert np.all(out[by * B:by * B + B, bx * B:bx * B + B] == 0.0)
        assert np.all(lg[b] == 0xFFFF)


def test_partial_blocks_at_ragged_border(oracle_lib):
    """Sizes that are not multiples of B: only in-image target pixels exist."""
    img = synth.make_image(37, 50, 4)
    mask = synth.quarter_mask(37, 50, 5)
    out, lg, _ = oracle_lib.reconstruct(img, mask, 30, log=True)
    assert lg.shape[0] == 10 * 13
    assert np.all(np.isfinite(out))
    assert np.array_equal(out[mask != 0], img[mask != 0])
    ids = np.arange(lg.shape[0])
    tg, lg2, _, _ = oracle_lib.reconstruct_blocks(img, mask, ids, 30, log=True)
    assert np.array_equal(lg2, lg)
    for b in ids:
        by, bx = divmod(int(b), 13)
        blk = out[by * 4:by * 4 + 4, bx * 4:bx * 4 + 4]
        t = tg[b][:blk.shape[0], :blk.shape[1]]
        assert np.array_equal(t, blk)
        assert np.all(np.isnan(tg[b][blk.shape[0]:, :])) and np.all(np.isnan(tg[b][:, blk.shape[1]:]))


def test_threads_do_not_change_results(oracle_lib):
    img, mask = synth.workload("small64").inputs()
    a, la, _ = oracle_lib.reconstruct(img, mask, 50, log=True, threads=1)
    b, lb, _ = oracle_lib.reconstruct(img, mask, 50, log=True, threads=4)
    assert np.array_equal(a, b) and np.array_equal(la, lb)


# ---------------------------------------------------------------- decision precision
def test_fp64_decision_resolves_sub_float32_differences(oracle_lib):
    """Eq. 8 is a plain argmax: the oracle must compare its FP64 objectives as
    they are.  All pixels known and rho = 1 make W = S^2 delta, so R0 =
    DFT2(f) and the objectives of f = A cos(2 pi n/S) + alpha A cos(2 pi m/S)
    at bins (0,1) and (1,0) differ by exactly the factor alpha^2 (closed
    form).  For alpha within a few 1e-8 of 1 the two objectives round to the
    same float32 value; the larger must still win: (1,0) (index 32) when
    alpha > 1, (0,1) (index 1) when alpha < 1, and with alpha = 1 they tie
    exactly and the smaller index 1 wins."""
    S, A = 32, 50.0
    m = np.arange(S)
    known = np.ones((S, S), np.uint8)
    wf = np_freq_weight(S)

    def objectives(alpha):
        f = A * np.cos(2 * np.pi * m[None, :] / S) + alpha * A * np.cos(2 * np.pi * m[:, None] / S)
        obj = wf * np.abs(np.fft.fft2(f)) ** 2
        return f, obj[0, 1], obj[1, 0]

    cases = [(1.0, 1)]
    for sign, expect in ((1.0, 32), (-1.0, 1)):
        for step in range(1, 200):
            alpha = 1.0 + sign * step * 5e-9
            f, a, b = objectives(alpha)
            if np.float32(a) == np.float32(b) and abs(b - a) > 1e-9 * a:
                cases.append((alpha, expect))
                break
    assert len(cases) == 3
    for alpha, expect in cases:
        f, _, _ = objectives(alpha)
        r = oracle_lib.block(f, known, 1, 1.0, 0.5)
        assert int(r["idx"][0]) == expect, (alpha, int(r["idx"][0]))


# ---------------------------------------------------------------- decision separations
def np_separation(obj, best, S):
    """Relative separation of the winner from the largest objective of any
    other bin, the winner's conjugate passed over when it ties exactly."""
    o = np.asarray(obj, np.float64).ravel().copy()
    k, l = divmod(int(best), S)
    conj = ((S - k) % S) * S + (S - l) % S
    top = o[best]
    o[best] = -1.0
    if conj != best and o[conj] == top:
        o[conj] = -1.0
    nxt = max(float(o.max()), 0.0)
    return (top - nxt) / top if top > 0 else 0.0


def test_separation_of_the_first_pick_closed_form(oracle_lib):
    """All pixels known and rho = 1: R(0) = DFT2(f) (numpy's FFT), so the first
    pick's objective w_f |F|^2 and its separation follow in closed form.  With
    the mean removed the winner is not DC; f is real, so the winner's
    conjugate ties it exactly and the separation is measured to the third
    largest objective, not 0."""
    S = 8
    rng = np.random.default_rng(15)
    f = rng.uniform(0, 255, (S, S))
    f -= f.mean()
    known = np.ones((S, S), np.uint8)
    obj = np_freq_weight(S) * np.abs(np.fft.fft2(f)) ** 2
    r = oracle_lib.block(f, known, 1, 1.0, 0.5)
    best = int(r["idx"][0])
    order = np.argsort(obj.ravel())[::-1]
    assert best == min(order[0], order[1]) and mirror(order[0], S) == order[1]
    third = obj.ravel()[order[2]]
    assert r["obj"][0] == pytest.approx(obj.ravel()[best], rel=1e-12)
    assert r["sep"][0] == pytest.approx((obj.ravel()[best] - third) / obj.ravel()[best], rel=1e-9)
    assert r["sep"][0] > 0.0


@pytest.mark.parametrize("S", [8, 16, 32])
def test_separation_log_matches_the_residual(oracle_lib, S):
    """At every iteration the logged objective and separation are those of the
    residual R(v) the iteration starts from (the oracle's own, pinned by the
    residual identity), recomputed with numpy."""
    I = 8
    ft, known = random_support(S, 31 + S)
    full = oracle_lib.block(ft, known, I, 0.7, 0.5)
    wf = np_freq_weight(S)
    for v in range(I):
        R = oracle_lib.block(ft, known, v, 0.7, 0.5)["R"] if v else None
        if R is None:
            x = ft * np_weight(known, 0.7)
            R = np.fft.fft2(x)
        obj = wf * np.abs(R) ** 2
        best = int(full["idx"][v])
        assert obj.ravel()[best] == pytest.approx(obj.max(), rel=1e-12)
        assert full["obj"][v] == pytest.approx(obj.ravel()[best], rel=1e-10)
        assert full["sep"][v] == pytest.approx(np_separation(obj, best, S), rel=1e-6, abs=1e-12)
