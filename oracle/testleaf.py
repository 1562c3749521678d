"""Distillation-driven subdivision (Section 3.4: BuildKDTree with the TestLeaf stopping rule).

Test infrastructure only: a plain float64 statement of the rule that the library's
distilled tree build is checked against.

BuildKDTree recurses from the root, left subtree before right.  At each node the stopping
rule distils node MLPs of a fixed small shape from the teacher for a fixed number of
iterations and compares the average PSNR against that of the tree without the split; when
the PSNR difference is below a threshold (the paper's example: 1 %), the node stays a leaf.

Readings taken here (the paper leaves them open):
  * the difference is relative: the split is kept iff
    PSNR(tree with the node split) - PSNR(current tree) >= gain_thresh * PSNR(current tree);
  * "the original tree" is the tree built so far (every split kept before this test), and
    each trial tree is distilled from scratch: every leaf MLP starts from the same initial
    parameters, and step s (1-based) takes batch (s - 1) mod n_batches of teacher rays;
  * a distillation step is the training step of the renderer: render the batch with the
    float32 parameters, L = mean over rays and channels of (rgb - target)^2, gradient, one
    Adam step (float64 masters and moments here);
  * the PSNR is 10 log10(1 / mean squared error) over the colour channels of held-out
    evaluation rays against the teacher's colours;
  * a node is tested only when it is splittable (depth < max_depth, longest side >= 2
    cells) and the tree has fewer than max_leaves leaves; otherwise it is a leaf.
"""
from __future__ import annotations

import numpy as np

from . import adam, build_tree_codes, psnr, render, render_grad


def distil(tree, init, n_hidden, hidden, batches, eval_rays, eval_target, n_max, lr, s_max, eps=1e-4):
    """(float32 parameters [L][P], PSNR on the evaluation rays) after n_max distillation
    steps of one parameter set per leaf of `tree`, each starting from `init` [P].
    batches: list of (o[3][R], d[3][R], target[R][3]); eval_rays: (o, d)."""
    L = tree.n_leaves
    init = np.asarray(init, np.float32).reshape(-1)
    master = np.tile(init.astype(np.float64), (L, 1))
    m = np.zeros_like(master)
    v = np.zeros_like(master)
    for step in range(1, n_max + 1):
        o, d, target = batches[(step - 1) % len(batches)]
        w = master.astype(np.float32)
        rgb = render(tree, w, n_hidden, hidden, o, d, s_max, eps=eps, threads=1)[0]
        g = 2.0 * (rgb - np.asarray(target, np.float64)) / (3.0 * o.shape[1])
        grad = render_grad(tree, w, n_hidden, hidden, o, d, s_max, g, eps=eps)
        adam(master.reshape(-1), m.reshape(-1), v.reshape(-1), grad.reshape(-1), step, lr=lr)
    w = master.astype(np.float32)
    rgb = render(tree, w, n_hidden, hidden, eval_rays[0], eval_rays[1], s_max, eps=eps, threads=1)[0]
    return w, psnr(rgb, eval_target)


def build_tree_distilled(grid, n, max_depth, max_leaves, gain_thresh, score):
    """(tree, log) of BuildKDTree driven by the stopping rule.  score(tree) -> PSNR of a
    tree (distil(...)[1] for the method; any function for tests of the rule itself).
    log: one (code, depth, psnr_current, psnr_split, kept, leaves_of_trial) per test, in
    the order the recursion makes them."""
    split = []
    current = build_tree_codes(grid, n, split)
    psnr_cur = score(current)
    log = []

    def row_of(tree, code):
        return tree.rows[np.nonzero(tree.rows[:, 0] == code)[0][0]]

    def build(code):
        nonlocal current, psnr_cur
        r = row_of(current, code)
        depth = int(r[1])
        side = int((r[5:8] - r[2:5]).max())
        if depth >= max_depth or side < 2 or len(split) + 1 >= max_leaves:
            return
        trial = build_tree_codes(grid, n, split + [code])
        psnr_t = score(trial)
        kept = psnr_t - psnr_cur >= gain_thresh * psnr_cur
        log.append((code, depth, psnr_cur, psnr_t, bool(kept), trial.n_leaves))
        if not kept:
            return
        split.append(code)
        current, psnr_cur = trial, psnr_t
        build(2 * code)
        build(2 * code + 1)

    build(1)
    return current, log
