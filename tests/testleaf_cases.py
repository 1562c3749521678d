"""Seeded inputs of the distillation-driven subdivision tests (Section 3.4, TestLeaf): the
guidance grid, the teacher (a tree and its leaf parameters), the cameras of the distillation
batches and of the evaluation view, and the students' initial parameters.  Inputs only: each
side renders the teacher's colours itself."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import synth

STUDENT_HIDDEN, STUDENT_LAYERS = 32, 4     # the paper's node MLP: width 32, depth 4


@dataclass
class Case:
    grid: np.ndarray
    n: int
    teacher_tree: tuple          # ("codes", inner node codes) or ("best_first", max_depth, max_leaves)
    teacher_weights: object      # leaf boxes [L][6] of the teacher tree -> [L][P] float32
    teacher_shape: tuple         # (n_hidden, hidden)
    cams: list                   # distillation batches: one camera each
    eval_cam: object
    init: np.ndarray             # [P] float32, the students' initial parameters
    s_max: int
    n_max: int
    lr: float
    gain_thresh: float
    max_depth: int
    max_leaves: int


def const_leaf(n_hidden, hidden, sigma_bias, rgb_bias):
    """Parameters whose MLP is the constant (softplus(sigma_bias), sigmoid(rgb_bias)):
    every weight and every other bias zero."""
    w = np.zeros(synth.param_count(n_hidden, hidden), np.float32)
    o = synth.sigma_bias_offset(n_hidden, hidden)
    w[o] = sigma_bias
    w[o + 1:o + 4] = rgb_bias
    return w


def two_halves(px=12) -> Case:
    """A uniform grid (so the root's median plane is the middle plane x = 1/2) and a teacher
    of two leaves split there, each a constant field: red fog in x < 1/2, blue fog above.
    The students start from all-zero parameters, so they stay constant per leaf (every
    weight's gradient is multiplied by a zero weight or a zero activation): a one-leaf
    student cannot show both colours, the root split makes the teacher exactly
    representable, and no further split can add anything."""
    n = 16
    nh, hid = STUDENT_LAYERS, STUDENT_HIDDEN
    W = np.stack([const_leaf(nh, hid, 1.5, [3.0, -3.0, -3.0]), const_leaf(nh, hid, 1.5, [-3.0, -3.0, 3.0])])
    cams = synth.make_cameras(5, 99, px, px)
    return Case(grid=np.ones((n, n, n), np.float32), n=n, teacher_tree=("codes", [1]),
                teacher_weights=lambda boxes: W, teacher_shape=(nh, hid),
                cams=cams[:4], eval_cam=cams[4], init=np.zeros(synth.param_count(nh, hid), np.float32), s_max=32,
                n_max=40, lr=0.1, gain_thresh=0.1, max_depth=2, max_leaves=8)


def small_scene(px=16) -> Case:
    """The 32^3 blob scene of the smallest configuration as the teacher (its own 8-leaf tree
    and leaf MLPs), students of the paper's shape from a seeded He initialisation, the
    paper's 1 % threshold, depth <= 3."""
    cfg = synth.C1
    grid = synth.make_grid(cfg)
    cams = synth.make_cameras(5, 99, px, px)
    nh, hid = STUDENT_LAYERS, STUDENT_HIDDEN
    def weights(boxes):
        dens = synth.leaf_mean_density(grid, cfg.grid_n, boxes)
        return synth.make_weights(len(boxes), cfg.n_hidden, cfg.hidden, cfg.seed_weights, dens)
    return Case(grid=grid, n=cfg.grid_n, teacher_tree=("best_first", cfg.max_depth, cfg.max_leaves),
                teacher_weights=weights, teacher_shape=(cfg.n_hidden, cfg.hidden),
                cams=cams[:4], eval_cam=cams[4], init=synth.make_weights(1, nh, hid, 777)[0], s_max=32, n_max=20,
                lr=1e-2, gain_thresh=0.01, max_depth=3, max_leaves=8)
