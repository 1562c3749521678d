"""Scene set-up shared by the GPU tests: seeded inputs, the oracle's tree and the library.

Oracle inputs never come from the HIP path: the MLP parameters are generated from the
oracle's own tree (its leaf boxes set the sigma biases), and the library's tree is
checked bit-exact against the oracle's before those parameters are used with it.
"""
from __future__ import annotations

import numpy as np

import oracle
import synth


class Scene:
    """footprint > 0: renders use hierarchical sampling, so every node gets an MLP (indexed by
    its preorder node slot, its sigma bias from the mean density over its box)."""

    def __init__(self, cfg: synth.SceneConfig, grid=None, split=0, footprint=0.0):
        self.cfg = cfg
        self.split = split
        self.footprint = footprint
        self.grid = synth.make_grid(cfg) if grid is None else grid
        self.otree = oracle.build_tree(self.grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves, split)
        if footprint > 0:
            rows = self.otree.rows
            boxes = rows[np.argsort(rows[:, 11])][:, 2:8].copy()
        else:
            boxes = self.otree.leaf_boxes()
        self.n_sets = len(boxes)
        dens = synth.leaf_mean_density(self.grid, cfg.grid_n, boxes)
        self.W = synth.make_weights(self.n_sets, cfg.n_hidden, cfg.hidden, cfg.seed_weights, dens)

    def camera_rays(self, i=0, n=1, width=None, height=None):
        cams = synth.make_cameras(i + n, self.cfg.seed_cameras, width or self.cfg.width,
                                  height or self.cfg.height)[i:i + n]
        return synth.rays_for_cameras(cams)


def gpu_setup(scene: Scene, dtype, device="cuda:0"):
    """Library context, tree (checked bit-exact against the oracle) and packed MLP."""
    import torch
    import paper_2310_01881_amd as am
    ctx = am.Context(0)
    tree = am.Tree(ctx, scene.grid, scene.cfg.grid_n, scene.cfg.max_depth, scene.cfg.max_leaves, scene.split)
    assert np.array_equal(tree.rows, scene.otree.rows)
    assert np.array_equal(tree.mass, scene.otree.mass)
    master = torch.from_numpy(scene.W).to(device)
    mlp = am.Mlp(ctx, master, scene.cfg.n_hidden, scene.cfg.hidden, dtype, scene.n_sets)
    return ctx, tree, mlp


def to_dev(a, device="cuda:0"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)
