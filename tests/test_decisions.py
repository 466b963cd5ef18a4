"""Host logic of tests/decisions.py (which logged decisions FP32 can be held to)."""
import numpy as np

from tests.decisions import (OBJ_FLOOR, SEP_MIN, block_of_pixel, decision_report, parting_report,
                             resolvable_prefix)


def test_prefix_stops_at_the_first_unresolvable_decision():
    obj = np.array([[1.0, 0.5, 0.25, 0.1], [2.0, 1.0, 1.0, 1.0], [1.0, 1.0, 1.0, 1.0],
                    [0.0, 0.0, 0.0, 0.0]])
    sep = np.array([[0.5, 0.5, SEP_MIN / 2, 0.5],       # a near-tie at iteration 2
                    [0.5, 0.5, 0.5, 0.5],               # every decision resolvable
                    [SEP_MIN, 0.1, 0.1, 0.1],           # exactly at the threshold: resolvable
                    [0.5, 0.5, 0.5, 0.5]])              # empty support: objective 0
    obj[1, 3] = 2.0 * OBJ_FLOOR / 2                     # below the floor at iteration 3
    assert resolvable_prefix(obj, sep).tolist() == [2, 3, 4, 0]


def test_decision_report_counts_only_prefix_decisions():
    ol = np.array([[1, 2, 3, 4], [5, 6, 7, 8]])
    gl = np.array([[1, 2, 9, 9], [5, 9, 7, 8]])
    obj = np.ones((2, 4))
    sep = np.array([[0.5, 0.5, 0.0, 0.5], [0.5, 0.5, 0.5, 0.5]])
    rep = decision_report(gl, ol, obj, sep)
    assert rep["prefix_decisions"] == 2 + 4
    assert rep["prefix_agree"] == 5 / 6
    assert rep["blocks_parting_in_prefix"] == 1
    assert rep["strict_agree"] == 5 / 8 and rep["blocks_all_agree"] == 0.0


def test_block_map_and_parting_report():
    own = block_of_pixel(5, 7, 4)      # 2 x 2 blocks, ragged
    assert own[0, 0] == 0 and own[0, 6] == 1 and own[4, 0] == 2 and own[4, 6] == 3
    mask = np.zeros((5, 7), np.uint8)
    g = np.zeros((5, 7))
    o = np.zeros((5, 7))
    g[0, 6] = 5.0                      # block 1 parts and differs by 5
    g[4, 0] = 0.5                      # block 2 agrees and differs by 0.5
    ol = np.array([[0], [1], [2], [3]])
    gl = np.array([[0], [9], [2], [3]])
    rep = parting_report(mask, g, o, gl, ol, np.ones((4, 1)), np.ones((4, 1)), 4)
    assert rep["agreeing_blocks_unknown_px"] == 35 - 4 * 3
    assert rep["agreeing_blocks_max_abs"] == 0.5 and rep["agreeing_blocks_frac_le_1"] == 1.0
