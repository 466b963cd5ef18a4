"""Seeded input generators: statistics the workloads promise."""
import numpy as np

import synth


def test_image_range_and_determinism():
    a = synth.make_image(120, 160, 5)
    b = synth.make_image(120, 160, 5)
    c = synth.make_image(120, 160, 6)
    assert a.dtype == np.float64 and a.shape == (120, 160)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0.0 and a.max() <= 255.0
    assert 20.0 < a.std() < 120.0            # content, not a flat frame


def test_quarter_mask_one_known_per_cell():
    m = synth.quarter_mask(64, 96, 3)
    cells = m.reshape(32, 2, 48, 2).sum(axis=(1, 3))
    assert np.all(cells == 1)
    pos = m.reshape(32, 2, 48, 2).transpose(0, 2, 1, 3).reshape(-1, 4).argmax(1)
    counts = np.bincount(pos, minlength=4)
    assert counts.min() > 0.2 * counts.sum()   # uniform choice within the cell
    assert np.array_equal(m, synth.quarter_mask(64, 96, 3))


def test_quarter_mask_odd_size_is_cropped():
    m = synth.quarter_mask(7, 9, 1)
    assert m.shape == (7, 9) and m.dtype == np.uint8
    assert np.all(m.reshape(-1) <= 1)


def test_macroblock_mask_drops_exact_quarter():
    H, W = 2160, 3840
    m = synth.macroblock_mask(H, W, 11)
    mb = m.reshape(H // 16, 16, W // 16, 16).max(axis=(1, 3))
    n_mb = (H // 16) * (W // 16)
    assert int((mb == 0).sum()) == round(0.25 * n_mb)
    inside = m.reshape(H // 16, 16, W // 16, 16).transpose(0, 2, 1, 3)[mb == 1]
    assert abs(1.0 - inside.mean() - 0.10) < 0.002


def test_uniform_loss_rate():
    m = synth.uniform_loss_mask(512, 512, 0.3, 2)
    assert abs(1.0 - m.mean() - 0.3) < 0.01


def test_workloads_and_block_counts():
    assert synth.workload("small64").n_blocks == 256
    assert synth.workload("fhd_quarter").n_blocks == 129600
    assert synth.workload("uhd_concealment").n_blocks == 518400
    assert synth.workload("fhd_quarter").support == 32


def test_batch_and_trace_are_seeded_and_mixed():
    a = synth.batch_items(64)
    assert [x.seed for x in a] == [x.seed for x in synth.batch_items(64)]
    assert {x.iterations for x in a} == {50, 100, 200}
    assert len({(x.height, x.width) for x in a}) == 4
    assert any(x.mask == "quarter" for x in a) and any(x.mask.startswith("uniform:") for x in a)
    tr = synth.serving_trace(2000)
    t = np.array([r.arrival_s for r in tr])
    assert np.all(np.diff(t) >= 0)
    rate = (len(t) - 1) / (t[-1] - t[0])
    assert 220 < rate < 260
    sizes = [r.item.height for r in tr]
    frac720 = sizes.count(720) / len(sizes)
    assert abs(frac720 - 5 / 9) < 0.05


def test_realtime_trace_interleaves_periodic_streams():
    tr = synth.realtime_trace(2.0, 30.0)
    assert len(tr) == 4 * 60
    t = np.array([r.arrival_s for r in tr])
    assert np.all(np.diff(t) > 0)                       # distinct phases: no two arrivals coincide
    for h in (480, 600, 1080, 2160):
        ts = np.array([r.arrival_s for r in tr if r.item.height == h])
        assert len(ts) == 60 and np.allclose(np.diff(ts), 1 / 30.0)
    assert {r.item.mask for r in tr} == {"quarter"}
    assert [r.item.seed for r in tr] == [r.item.seed for r in synth.realtime_trace(2.0, 30.0)]
