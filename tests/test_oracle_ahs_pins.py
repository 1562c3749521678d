"""Pins of the oracle's hierarchical sampling (Section 3.5, HCheck; reading in the design
notes): node slots against the preorder definition, the two limits of the footprint, the
intervals against a brute-force grouping of leaf intervals by the first ancestor that the
test stops at, the sample-count rule, closed forms of the quadrature and finite differences
of the gradient."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import constant_field

N_HIDDEN, HIDDEN = 2, 32


def deep_tree(split=0):
    cfg = synth.scaled(synth.C2, grid_n=64, max_depth=8, max_leaves=64)
    g = synth.make_grid(cfg)
    return cfg, oracle.build_tree(g, cfg.grid_n, cfg.max_depth, cfg.max_leaves, split)


def by_code(tree):
    return {int(r[0]): r for r in tree.rows}


def subtree_size(codes, c):
    n = 0
    for x in codes:
        while x > c:
            x >>= 1
        n += x == c
    return n


@pytest.mark.parametrize("split", [0, 1])
def test_node_slots_are_left_first_preorder(split):
    cfg, tree = deep_tree(split)
    rows = tree.rows
    nodes = by_code(tree)
    codes = list(nodes)
    assert sorted(rows[:, 11].tolist()) == list(range(len(rows)))
    assert nodes[1][11] == 0
    for c, r in nodes.items():
        if r[8] < 0:
            continue
        assert nodes[2 * c][11] == r[11] + 1
        assert nodes[2 * c + 1][11] == r[11] + 1 + subtree_size(codes, 2 * c)
    leaves = rows[rows[:, 10] >= 0]
    assert np.array_equal(leaves[np.argsort(leaves[:, 11])][:, 10], np.arange(len(leaves)))


def leaf_to_node_slot(tree):
    m = np.full(tree.n_leaves, -1)
    lv = tree.rows[tree.rows[:, 10] >= 0]
    m[lv[:, 10]] = lv[:, 11]
    return m


def test_footprint_limits():
    cfg, tree = deep_tree()
    o, d = synth.random_rays(300, 11, inside_frac=0.0)            # all rays start outside
    t0, t1, slot, m = oracle.trace(tree, o, d)
    # a footprint so small that no node stops the descent: the leaf intervals, keyed by node slot
    a0, a1, aslot, am = oracle.trace(tree, o, d, footprint=1e-30)
    l2n = leaf_to_node_slot(tree)
    assert np.array_equal(am, m)
    for r in range(o.shape[1]):
        k = m[r]
        np.testing.assert_array_equal(a0[r, :k], t0[r, :k])
        np.testing.assert_array_equal(a1[r, :k], t1[r, :k])
        np.testing.assert_array_equal(aslot[r, :k], l2n[slot[r, :k]])
    # one so large that the root stops it for every ray entering at t > 0: one interval
    b0, b1, bslot, bm = oracle.trace(tree, o, d, footprint=1e30)
    hit = m > 0
    assert hit.sum() > 200
    assert np.all(bm[hit] == 1) and np.all(bm[~hit] == 0)
    for r in np.where(hit)[0]:
        assert bslot[r, 0] == 0
        assert b0[r, 0] == t0[r, 0] and b1[r, 0] == t1[r, m[r] - 1]
    # the root interval carries one leaf interval's share of samples
    W = synth.make_weights(tree.n_nodes, N_HIDDEN, HIDDEN, 3)
    for r in np.where(hit)[0][:40]:
        rec = oracle.ray_samples(tree, W, N_HIDDEN, HIDDEN, o, d, r, 64, eps=0.0, footprint=1e30)
        assert len(rec["t"]) == (64 // m[r] if m[r] <= 64 else 1)
        assert np.all(rec["slot"] == 0)


def entry_param(o, d, lo, hi):
    """The ray's entry parameter into the box [lo, hi] (t >= 0), by the slab test."""
    t = 0.0
    for a in range(3):
        ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        t = max(t, min(ta, tb))
    return t


def expected_intervals(tree, o, d, footprint, t0, t1, slot, m):
    """Groups a ray's leaf intervals by the node where the test stops: the first ancestor A
    (from the root) with float32(entry into A) > float32(side(A) / footprint)."""
    nodes = by_code(tree)
    n = tree.grid_n
    lv = tree.rows[tree.rows[:, 10] >= 0]
    leaf_code = np.zeros(tree.n_leaves, np.int64)
    leaf_code[lv[:, 10]] = lv[:, 0]
    f32 = np.float32(footprint)
    out = []
    for k in range(m):
        c = int(leaf_code[slot[k]])
        chain = [c >> s for s in range(c.bit_length() - 1, -1, -1)]      # root ... leaf
        stop = chain[-1]
        for a in chain[:-1]:
            r = nodes[a]
            lo, hi = r[2:5].astype(np.float64) / n, r[5:8].astype(np.float64) / n
            side = np.float32(np.float32((r[5:8] - r[2:5]).max()) / np.float32(n))
            t_stop = np.float32(side / f32)
            if np.float32(entry_param(o, d, lo, hi)) > t_stop:
                stop = a
                break
        ns = int(nodes[stop][11])
        if out and out[-1][2] == ns:
            out[-1][1] = t1[k]
        else:
            out.append([t0[k], t1[k], ns])
    return out


@pytest.mark.parametrize("footprint", [0.25, 0.5, 1.0])
def test_intervals_against_brute_force_grouping(footprint):
    cfg, tree = deep_tree()
    o, d = synth.random_rays(400, 12, inside_frac=0.3)
    t0, t1, slot, m = oracle.trace(tree, o, d)
    a0, a1, aslot, am = oracle.trace(tree, o, d, footprint=footprint)
    merged = 0
    for r in range(o.shape[1]):
        oo, dd = o[:, r].astype(np.float64), d[:, r].astype(np.float64)
        exp = expected_intervals(tree, oo, dd, footprint, t0[r], t1[r], slot[r], m[r])
        assert am[r] == len(exp), r
        for k, (e0, e1, es) in enumerate(exp):
            assert aslot[r, k] == es and a0[r, k] == e0 and a1[r, k] == e1, (r, k)
        merged += m[r] - am[r]
    assert merged > 50                       # the test does stop descents at this footprint


def test_sample_count_rule():
    cfg, tree = deep_tree()
    o, d = synth.random_rays(120, 13, inside_frac=0.3)
    f = 0.25
    _, _, _, m = oracle.trace(tree, o, d)
    a0, a1, aslot, am = oracle.trace(tree, o, d, footprint=f)
    W = synth.make_weights(tree.n_nodes, N_HIDDEN, HIDDEN, 4)
    for s_max in (1, 7, 64):
        for r in range(o.shape[1]):
            rec = oracle.ray_samples(tree, W, N_HIDDEN, HIDDEN, o, d, r, s_max, eps=0.0, footprint=f)
            if m[r] == 0:
                assert len(rec["t"]) == 0
                continue
            n = s_max // m[r] if m[r] <= s_max else 1
            keff = min(am[r], s_max)
            assert len(rec["t"]) == n * keff <= s_max
            for k in range(keff):
                seg = slice(k * n, (k + 1) * n)
                assert np.all(rec["slot"][seg] == aslot[r, k])
                assert abs(rec["delta"][seg].sum() - (a1[r, k] - a0[r, k])) < 1e-13
                exp_t = a0[r, k] + (np.arange(n) + 0.5) / n * (a1[r, k] - a0[r, k])
                np.testing.assert_allclose(rec["t"][seg], exp_t, rtol=0, atol=1e-13)


def test_piecewise_constant_node_densities():
    """Each node's MLP a constant density: transmittance from the brute-force grouping."""
    cfg, tree = deep_tree()
    o, d = synth.random_rays(200, 14, inside_frac=0.3)
    f = 0.25
    rng = np.random.default_rng(2)
    sig_node = rng.uniform(0.05, 3.0, tree.n_nodes)
    W, sig = constant_field(tree.n_nodes, N_HIDDEN, HIDDEN, 0.0, [0, 0, 0], sigma_per_leaf=sig_node)
    rgb, depth, opac, ns, flags = oracle.render(tree, W, N_HIDDEN, HIDDEN, o, d, 128, eps=0.0, footprint=f)
    t0, t1, slot, m = oracle.trace(tree, o, d)
    checked = 0
    for r in range(o.shape[1]):
        if m[r] == 0 or m[r] > 128:
            continue
        oo, dd = o[:, r].astype(np.float64), d[:, r].astype(np.float64)
        exp = expected_intervals(tree, oo, dd, f, t0[r], t1[r], slot[r], m[r])
        tau = sum(sig[s] * (e1 - e0) for e0, e1, s in exp)
        assert abs(opac[r] - (1 - math.exp(-tau))) < 1e-12
        checked += 1
    assert checked > 100


def test_gradient_matches_central_differences_with_hcheck():
    cfg, tree = deep_tree()
    o, d = synth.random_rays(60, 15, inside_frac=0.0)
    f = 0.25
    W = synth.make_weights(tree.n_nodes, N_HIDDEN, HIDDEN, 5,
                           np.full(tree.n_nodes, 2.0))
    rng = np.random.default_rng(6)
    g_rgb = rng.standard_normal((o.shape[1], 3))
    s_max = 16
    grad = oracle.render_grad(tree, W, N_HIDDEN, HIDDEN, o, d, s_max, g_rgb, eps=0.0, footprint=f)
    # inner-node MLPs receive gradient (they render the collapsed segments)
    inner = tree.rows[tree.rows[:, 8] >= 0][:, 11]
    assert np.abs(grad[inner]).sum() > 0

    def loss(Wp):
        rgb, _, _, _, _ = oracle.render(tree, Wp, N_HIDDEN, HIDDEN, o, d, s_max, eps=0.0, footprint=f)
        return (rgb * g_rgb).sum()

    sb = synth.sigma_bias_offset(N_HIDDEN, HIDDEN)
    used = np.where(np.abs(grad).sum(axis=1) > 0)[0]
    idx = [(int(s), sb) for s in used[:10]] + [(int(s), sb + 1) for s in used[:10]]
    for s, i in idx:
        base = float(W[s, i])
        h = 2.0 ** -14 * max(1.0, abs(base))
        Wp = W.copy(); Wp[s, i] = np.float32(base + h)
        Wm = W.copy(); Wm[s, i] = np.float32(base - h)
        fd = (loss(Wp) - loss(Wm)) / (float(Wp[s, i]) - float(Wm[s, i]))
        assert abs(grad[s, i] - fd) <= 1e-6 * max(1.0, abs(fd)), (s, i, grad[s, i], fd)


@pytest.mark.parametrize("footprint,expected", [
    (0.5, [(1.0, 1.25, 2), (1.25, 2.0, 5)]),     # t_stop = 2 for every inner node: leaves only
    (0.9, [(1.0, 1.25, 2), (1.25, 2.0, 4)]),     # t_stop = 1.111: node 3 (entered at 1.25) stops
    (1.5, [(1.0, 2.0, 0)]),                      # t_stop = 0.667: the root (entered at 1) stops
])
def test_hand_derived_4cube(footprint, expected):
    """The hand-derived 4-leaf tree of the golden fixture (root split at x = 1/4, node 2
    at y = 1/4, node 3 at y = 3/4; every inner node's longest side is 1, so t_stop = 1/f),
    preorder slots root 0, node 2 -> 1, node 4 -> 2, node 5 -> 3, node 3 -> 4, node 6 -> 5,
    node 7 -> 6, and a ray along +x at y = 0.1 entering at t = 1 and crossing x = 1/4 at
    t = 1.25.  It crosses two leaves (4 and 6), so S_max = 8 gives 4 samples per interval."""
    g = np.zeros((4, 4, 4), np.float32)
    g[0, 0, 0] = 1.0
    g[3, 3, 3] = 0.5
    tree = oracle.build_tree(g.reshape(-1), 4, 2, 4)
    assert {int(r[0]): int(r[11]) for r in tree.rows} == {1: 0, 2: 1, 4: 2, 5: 3, 3: 4, 6: 5, 7: 6}
    o = np.array([[-1.0], [0.1], [0.5]], np.float32)
    d = np.array([[1.0], [0.0], [0.0]], np.float32)
    t0, t1, slot, m = oracle.trace(tree, o, d, footprint=footprint)
    assert m[0] == len(expected)
    for k, (e0, e1, es) in enumerate(expected):
        assert (t0[0, k], t1[0, k], slot[0, k]) == (e0, e1, es)
    W = synth.make_weights(tree.n_nodes, N_HIDDEN, HIDDEN, 6)
    rec = oracle.ray_samples(tree, W, N_HIDDEN, HIDDEN, o, d, 0, 8, eps=0.0, footprint=footprint)
    exp_t = [e0 + (j + 0.5) / 4 * (e1 - e0) for e0, e1, _ in expected for j in range(4)]
    np.testing.assert_allclose(rec["t"], exp_t, rtol=0, atol=1e-15)
