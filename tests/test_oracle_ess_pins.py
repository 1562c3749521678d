"""Pins of the oracle's occupancy grid and empty-space skipping (Section 4.1; reading in the
design notes): special cases of the grid, a hand-derived fixture, the two trivial grids, and
closed forms of the quadrature with samples dropped."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import c1_setup, constant_field


def test_occupancy_hand_derived():
    # 4^3 grid, block 2 -> 2^3 cells.  g(0,0,0) = 1 (q = 2^24), g(3,3,3) = 0.5 (q = 2^23),
    # g(2,0,1) = 0.001 (q = floor(16777.216 + 1/2) = 16777), everything else 0.
    g = np.zeros((4, 4, 4), np.float32)          # [k][j][i]
    g[0, 0, 0] = 1.0
    g[3, 3, 3] = 0.5
    g[1, 0, 2] = 0.001
    g = g.reshape(-1)

    def cells(thresh):
        return oracle.occupancy(g, 4, 2, thresh).reshape(2, 2, 2)    # [k][j][i]

    c = cells(0.0)                               # any positive density
    assert c[0, 0, 0] == 1 and c[1, 1, 1] == 1 and c[0, 0, 1] == 1 and c.sum() == 3
    assert cells(0.001).sum() == 3               # q_thr = 16777 <= 16777
    assert cells(0.0011).sum() == 2              # q_thr = 18455 > 16777
    assert cells(0.5).sum() == 2                 # 2^23 >= 2^23
    c = cells(0.50001)
    assert c.sum() == 1 and c[0, 0, 0] == 1      # only the maximum's block
    assert cells(1.0).sum() == 1
    # block 1 keeps the guidance resolution; block 4 a single cell
    assert oracle.occupancy(g, 4, 1, 0.0).sum() == 3
    assert oracle.occupancy(g, 4, 4, 0.9).tolist() == [1]


def test_occupancy_block_max_and_monotone():
    cfg = synth.C1
    g = synth.make_grid(cfg)
    n = cfg.grid_n
    prev = None
    for t in (0.0, 1e-3, 1e-2, 0.1, 0.5):
        c = oracle.occupancy(g, n, 2, t)
        if prev is not None:
            assert np.all(c <= prev)             # a higher threshold only empties cells
        prev = c
    # a coarser block is occupied iff one of its eight finer cells is
    fine = oracle.occupancy(g, n, 2, 1e-2).reshape(n // 2, n // 2, n // 2)
    coarse = oracle.occupancy(g, n, 4, 1e-2).reshape(n // 4, n // 4, n // 4)
    G = n // 4
    agg = fine.reshape(G, 2, G, 2, G, 2).max(axis=(1, 3, 5))
    assert np.array_equal(agg, coarse)


def test_all_occupied_is_the_plain_render_and_all_empty_is_black():
    cfg, g, tree, W = c1_setup()
    o, d = synth.camera_rays(synth.make_cameras(1, 301, 24, 24)[0])
    plain = oracle.render(tree, W, 2, 32, o, d, 64, eps=1e-4)
    full = oracle.render(tree, W, 2, 32, o, d, 64, eps=1e-4, occupancy=np.ones(16 ** 3, np.uint8))
    for a, b in zip(plain, full):
        assert np.array_equal(a, b)
    rgb, dep, op, ns, flags = oracle.render(tree, W, 2, 32, o, d, 64, eps=1e-4, occupancy=np.zeros(8 ** 3, np.uint8))
    assert not rgb.any() and not dep.any() and not op.any() and not ns.any()


@pytest.mark.parametrize("n", [8, 40, 64])
def test_half_space_closed_form(n):
    """Constant density, cells with x < 1/2 occupied, a ray along +x through one leaf: the
    kept samples are those at (j + 1/2)/n < 1/2, each of length 1/n."""
    g = np.ones(8 ** 3, np.float32)
    tree = oracle.build_tree(g, 8, 0, 1)
    W, sig = constant_field(1, 2, 32, 1.7, [0.2, 0.4, -0.3])
    s0 = float(sig[0])
    G = 8
    occ = np.zeros((G, G, G), np.uint8)         # [k][j][i]
    occ[:, :, :G // 2] = 1
    o = np.array([[-1.0], [0.3], [0.6]], np.float32)
    d = np.array([[1.0], [0.0], [0.0]], np.float32)
    rgb, depth, opac, ns, flags = oracle.render(tree, W, 2, 32, o, d, n, eps=0.0, occupancy=occ.reshape(-1))
    kept = sum(1 for j in range(n) if (j + 0.5) / n < 0.5)
    assert ns[0] == kept
    assert abs(opac[0] - (1 - math.exp(-s0 * kept / n))) < 1e-14
    # depth: the kept samples are the first ones, so the plain geometric series over them
    q = math.exp(-s0 / n)
    D = sum(q ** j * (1 - q) * (1.0 + (j + 0.5) / n) for j in range(kept))
    assert abs(depth[0] - D) < 1e-13
    assert flags[0] & oracle.FLAG_OCC_AMBIGUOUS == 0


def test_random_grid_against_per_sample_brute_force():
    """Piecewise-constant leaf densities and a random occupancy grid: the transmittance is that
    of the kept plain samples, found from the sample record and the grid by the test."""
    cfg, g, tree, W0 = c1_setup()
    sig_leaf = np.array([0.5, 1.0, 2.0, 0.1, 3.0, 0.25, 1.5, 0.75])
    W, sig = constant_field(8, 2, 32, 0.0, [0, 0, 0], sigma_per_leaf=sig_leaf)
    G = 16
    occ = (np.random.default_rng(3).random(G ** 3) < 0.6).astype(np.uint8)
    o, d = synth.random_rays(150, 17, inside_frac=0.3)
    s_max = 48
    rgb, depth, opac, ns, flags = oracle.render(tree, W, 2, 32, o, d, s_max, eps=0.0, occupancy=occ)
    checked = 0
    for r in range(o.shape[1]):
        rec = oracle.ray_samples(tree, W, 2, 32, o, d, r, s_max, eps=0.0)
        x = o[:, r].astype(np.float64)[None, :] + rec["t"][:, None] * d[:, r].astype(np.float64)[None, :]
        c = np.clip(np.floor(x * G), 0, G - 1).astype(int)
        keep = occ[c[:, 0] + G * (c[:, 1] + G * c[:, 2])] == 1
        assert ns[r] == keep.sum()
        tau = float((sig[rec["slot"]] * rec["delta"])[keep].sum())
        if flags[r] & oracle.FLAG_OCC_AMBIGUOUS:
            continue
        assert abs(opac[r] - (1 - math.exp(-tau))) < 1e-12
        checked += 1
    assert checked > 100


def test_boundary_samples_are_flagged_ambiguous():
    g = np.ones(8 ** 3, np.float32)
    tree = oracle.build_tree(g, 8, 0, 1)
    W, _ = constant_field(1, 2, 32, 1.0, [0, 0, 0])
    occ = np.zeros((4, 4, 4), np.uint8)
    occ[:, :, :2] = 1
    # 4 samples along x over [0, 1]: positions 1/8, 3/8, 5/8, 7/8; cell boundary at 1/2 is
    # far from all of them -> not ambiguous.  With 2 samples (1/4, 3/4) likewise.  A ray
    # along y at x = 1/2 (on the boundary) is ambiguous.
    o = np.array([[-1.0, 0.5], [0.3, -1.0], [0.6, 0.4]], np.float32)
    d = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]], np.float32)
    _, _, _, ns, flags = oracle.render(tree, W, 2, 32, o, d, 4, eps=0.0, occupancy=occ.reshape(-1))
    assert flags[0] & oracle.FLAG_OCC_AMBIGUOUS == 0 and ns[0] == 2
    assert flags[1] & oracle.FLAG_OCC_AMBIGUOUS
