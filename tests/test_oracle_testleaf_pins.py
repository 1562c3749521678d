"""Pins of the oracle's distillation-driven subdivision (Section 3.4: BuildKDTree with the
TestLeaf stopping rule), each against something other than the oracle's own statement:

* the tree of explicit split codes reproduces the best-first builder's tree when given its
  inner nodes, and rejects codes that are not splittable leaves;
* the rule's recursion and comparison on scores given by hand (the expected tree and test
  order worked out below);
* a distillation of zero steps is the PSNR of the initial parameters' render; one step is
  Adam's first step, whose closed form is p - lr g / (|g| + eps);
* a hand-built scene where the answer is known: a two-colour teacher split at x = 1/2 and
  students that can only be constant per leaf keep the root split and nothing else."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from oracle import testleaf
from testleaf_cases import two_halves


def test_codes_reproduce_the_best_first_tree():
    for cfg in (synth.C1,):
        g = synth.make_grid(cfg)
        t = oracle.build_tree(g, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
        inner = t.rows[t.rows[:, 8] >= 0][:, 0]
        for order in (inner, inner[::-1]):
            t2 = oracle.build_tree_codes(g, cfg.grid_n, order)
            assert np.array_equal(t.rows, t2.rows) and np.array_equal(t.mass, t2.mass)
    g = synth.make_grid(synth.C1)
    root = oracle.build_tree_codes(g, 32, [])
    assert root.rows.shape[0] == 1 and root.rows[0, 10] == 0 and root.mass[0] == oracle.build_tree(g, 32, 0, 1).mass[0]
    with pytest.raises(ValueError):
        oracle.build_tree_codes(g, 32, [2])          # the root is not split: 2 is no leaf
    with pytest.raises(ValueError):
        oracle.build_tree_codes(g, 32, [1, 1])       # 1 is no longer a leaf
    with pytest.raises(ValueError):
        oracle.build_tree_codes(np.ones((1, 1, 1), np.float32), 1, [1])   # one cell: unsplittable


def test_rule_on_given_scores():
    """Scores by leaf count: 20 dB x 1.05^(leaves - 1) up to 4 leaves, flat after.  With a
    1 % threshold the recursion keeps the root (2 leaves), then node 2 (3 leaves), then
    node 4 (4 leaves); node 8, 9, 5 and 3 give no gain and stay leaves."""
    g = np.ones((16, 16, 16), np.float32)

    def score(tree):
        return 20.0 * 1.05 ** (min(tree.n_leaves, 4) - 1)
    tree, log = testleaf.build_tree_distilled(g, 16, 6, 64, 0.01, score)
    assert [r[0] for r in log] == [1, 2, 4, 8, 9, 5, 3]
    assert [r[4] for r in log] == [True, True, True, False, False, False, False]
    assert [r[5] for r in log] == [2, 3, 4, 5, 5, 5, 5]
    inner = sorted(tree.rows[tree.rows[:, 8] >= 0][:, 0].tolist())
    assert inner == [1, 2, 4]
    assert np.array_equal(tree.rows, oracle.build_tree_codes(g, 16, [1, 2, 4]).rows)
    # the same scores under max_depth 1 and max_leaves 3
    assert [r[0] for r in testleaf.build_tree_distilled(g, 16, 1, 64, 0.01, score)[1]] == [1]
    t3, log3 = testleaf.build_tree_distilled(g, 16, 6, 3, 0.01, score)
    assert [r[0] for r in log3] == [1, 2] and t3.n_leaves == 3
    # a threshold no gain reaches: the root stays a leaf; a negative one keeps every split
    t0, log0 = testleaf.build_tree_distilled(g, 16, 6, 64, 0.06, score)
    assert t0.n_leaves == 1 and [r[4] for r in log0] == [False]
    tall, _ = testleaf.build_tree_distilled(g, 16, 2, 64, -1.0, score)
    assert tall.n_leaves == 4


def _targets(case, tree, W, cams):
    nh, hid = case.teacher_shape
    out = []
    for c in cams:
        o, d = synth.camera_rays(c)
        out.append((o, d, oracle.render(tree, W, nh, hid, o, d, case.s_max)[0]))
    return out


def test_distil_zero_and_one_step():
    case = two_halves(px=8)
    tt = oracle.build_tree_codes(case.grid, case.n, case.teacher_tree[1])
    W = case.teacher_weights(tt.leaf_boxes())
    batches = _targets(case, tt, W, case.cams)
    (eo, ed, et), = _targets(case, tt, W, [case.eval_cam])
    student = oracle.build_tree_codes(case.grid, case.n, [1])
    nh, hid = 4, 32
    init = synth.make_weights(1, nh, hid, 5)[0]
    w0, p0 = testleaf.distil(student, init, nh, hid, batches, (eo, ed), et, 0, 0.1, case.s_max)
    assert np.array_equal(w0, np.tile(init, (2, 1)))
    rgb = oracle.render(student, w0, nh, hid, eo, ed, case.s_max)[0]
    assert p0 == pytest.approx(10 * np.log10(1.0 / np.mean((rgb - et) ** 2)), rel=0, abs=1e-12)
    lr = 1e-3
    w1, _ = testleaf.distil(student, init, nh, hid, batches, (eo, ed), et, 1, lr, case.s_max)
    o, d, t = batches[0]
    rgb = oracle.render(student, w0, nh, hid, o, d, case.s_max)[0]
    gr = oracle.render_grad(student, w0, nh, hid, o, d, case.s_max, 2.0 * (rgb - t) / (3.0 * o.shape[1]))
    want = (w0.astype(np.float64) - lr * gr / (np.abs(gr) + 1e-8)).astype(np.float32)
    assert np.abs(gr).max() > 0
    assert np.array_equal(w1, want)


def test_two_halves_keep_only_the_root_split():
    case = two_halves()
    tt = oracle.build_tree_codes(case.grid, case.n, case.teacher_tree[1])
    assert tt.rows[0, 8] == 0 and tt.rows[0, 9] == case.n // 2      # split at x = 1/2
    W = case.teacher_weights(tt.leaf_boxes())
    batches = _targets(case, tt, W, case.cams)
    (eo, ed, et), = _targets(case, tt, W, [case.eval_cam])
    nh, hid = 4, 32

    def score(tree):
        return testleaf.distil(tree, case.init, nh, hid, batches, (eo, ed), et, case.n_max, case.lr, case.s_max)[1]
    tree, log = testleaf.build_tree_distilled(case.grid, case.n, case.max_depth, case.max_leaves,
                                              case.gain_thresh, score)
    assert np.array_equal(tree.rows, tt.rows)
    assert [r[0] for r in log] == [1, 2, 3] and [r[4] for r in log] == [True, False, False]
    gains = [(r[3] - r[2]) / r[2] for r in log]
    assert gains[0] > 5 * case.gain_thresh                     # far above the threshold
    assert max(abs(x) for x in gains[1:]) < case.gain_thresh / 2  # far below it
