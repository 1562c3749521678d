"""Pins of the FP64 oracle against facts other than itself.

Each test ties one oracle function to a closed form, an invariant, a brute-force
computation, a library routine or a hand-derived fixture, chosen so that a plausible
mistake (a dropped term, a wrong sign or index, a transposed operand) fails one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# helpers written from geometry, independent of the oracle's traversal
# ---------------------------------------------------------------------------
def chord_in_box(o, d, lo, hi):
    """Length of the ray parameter range (t >= 0) inside the box [lo, hi] (numpy, fp64).

    A ray parallel to an axis and lying in a face plane is counted by the half-open rule
    of the cells [lo, hi) (the upper face belongs to the next box, except the face at 1)."""
    o = np.asarray(o, np.float64); d = np.asarray(d, np.float64)
    tin, tout = 0.0, np.inf
    for a in range(3):
        if d[a] == 0.0:
            if o[a] < lo[a] or o[a] > hi[a] or (o[a] == hi[a] and hi[a] != 1.0):
                return 0.0
            continue
        ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        tin = max(tin, min(ta, tb)); tout = min(tout, max(ta, tb))
    return max(0.0, tout - tin)


def c1_setup():
    cfg = synth.C1
    g = synth.make_grid(cfg)
    tree = oracle.build_tree(g, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
    dens = synth.leaf_mean_density(g, cfg.grid_n, tree.leaf_boxes())
    W = synth.make_weights(tree.n_leaves, cfg.n_hidden, cfg.hidden, cfg.seed_weights, dens)
    return cfg, g, tree, W


# ---------------------------------------------------------------------------
# Tree (Section 3.4)
# ---------------------------------------------------------------------------
def load_golden_trees():
    out = {}
    for line in open(os.path.join(GOLDEN, "tree_4cube.txt")):
        if line.startswith("#") or not line.strip():
            continue
        head, row = line.split("|")
        md, ml = map(int, head.split())
        vals = list(map(int, row.split()))
        out.setdefault((md, ml), []).append(vals)
    return out


def test_tree_matches_hand_derived_golden():
    g = np.zeros((4, 4, 4), np.float32)       # [k][j][i]
    g[0, 0, 0] = 1.0
    g[3, 3, 3] = 0.5
    for (md, ml), rows in load_golden_trees().items():
        t = oracle.build_tree(g.reshape(-1), 4, md, ml)
        exp = np.array(rows, np.int64)
        assert t.n_nodes == len(exp)
        np.testing.assert_array_equal(t.rows[:, 0:11], exp[:, 0:11])
        np.testing.assert_array_equal(t.mass.astype(np.int64), exp[:, 11])


def test_tree_zero_mass_splits_at_midpoint():
    t = oracle.build_tree(np.zeros(8 ** 3, np.float32), 8, 4, 2)
    root = t.rows[0]
    assert root[8] == 0 and root[9] == 4


def quantised(g):
    g = g.astype(np.float64)
    gmax = g.max()
    return np.floor(np.ldexp(np.maximum(g, 0) / gmax, 24) + 0.5).astype(np.uint64)


@pytest.mark.parametrize("cfg_name,n,max_depth,max_leaves", [
    ("c1", 32, 3, 8), ("c1", 32, 6, 40), ("c2s", 64, 12, 200)])
def test_tree_partition_median_and_structure(cfg_name, n, max_depth, max_leaves):
    cfg = synth.C1 if cfg_name == "c1" else synth.scaled(synth.C2, grid_n=64)
    g = synth.make_grid(synth.scaled(cfg, grid_n=n))
    t = oracle.build_tree(g, n, max_depth, max_leaves)
    q = quantised(g).reshape(n, n, n)           # [k][j][i]
    rows = t.rows
    by_code = {int(r[0]): (r, int(m)) for r, m in zip(rows, t.mass)}
    # partition: every cell covered by exactly one leaf
    label = np.full((n, n, n), -1, np.int64)
    for r in rows[rows[:, 10] >= 0]:
        lx, ly, lz, hx, hy, hz = r[2:8]
        assert np.all(label[lz:hz, ly:hy, lx:hx] == -1)
        label[lz:hz, ly:hy, lx:hx] = r[10]
    assert np.all(label >= 0)
    assert t.n_leaves == max_leaves
    # masses are box sums of the quantised grid
    for r, m in zip(rows, t.mass):
        lx, ly, lz, hx, hy, hz = r[2:8]
        assert int(q[lz:hz, ly:hy, lx:hx].sum()) == int(m)
    # each split: longest axis (ties low), child boxes, weighted-median plane
    for r in rows[rows[:, 8] >= 0]:
        code, depth = int(r[0]), int(r[1])
        ext = r[5:8] - r[2:5]
        a, p = int(r[8]), int(r[9])
        assert a == int(np.argmax(ext)) and depth < max_depth
        left, lm = by_code[2 * code]
        right, rm = by_code[2 * code + 1]
        assert left[1] == depth + 1 and right[1] == depth + 1
        assert left[5 + a] == p and right[2 + a] == p
        total = lm + rm
        assert total == by_code[code][1]
        lo, hi = int(r[2 + a]), int(r[5 + a])
        assert lo < p < hi
        if total > 0:
            ax_sum = q[r[4]:r[7], r[3]:r[6], r[2]:r[5]].sum(axis=tuple(i for i in range(3) if i != 2 - a))
            pref = np.concatenate([[0], np.cumsum(ax_sum)])
            ok = [c for c in range(lo + 1, hi) if 2 * int(pref[c - lo]) >= total]
            assert p == (ok[0] if ok else hi - 1)
    # slots are the left-first depth-first order of the leaves
    leaves = rows[rows[:, 10] >= 0]
    D = int(rows[:, 1].max())
    key = [(int(r[0]) << (D - int(r[1]))) for r in leaves]
    np.testing.assert_array_equal(leaves[np.argsort(key)][:, 10], np.arange(len(leaves)))


def test_tree_best_first_mass_order():
    """Best-first: no remaining splittable leaf outweighs a node that was split after it existed.

    Leaves are split in decreasing mass order, so the lightest split node is at least as
    heavy as every splittable leaf left over when the leaf budget ran out."""
    cfg = synth.scaled(synth.C2, grid_n=64)
    g = synth.make_grid(cfg)
    t = oracle.build_tree(g, 64, 12, 100)
    rows, mass = t.rows, t.mass.astype(np.int64)
    inner = mass[rows[:, 8] >= 0]
    leaf = rows[:, 10] >= 0
    ext = rows[:, 5:8] - rows[:, 2:5]
    split_ok = leaf & (rows[:, 1] < 12) & (ext.max(axis=1) >= 2)
    assert mass[split_ok].max() <= inner.min()


def test_c1_tree_is_full_depth_three():
    cfg, g, tree, W = c1_setup()
    leaves = tree.rows[tree.rows[:, 10] >= 0]
    assert len(leaves) == 8 and np.all(leaves[:, 1] == 3)


# ---------------------------------------------------------------------------
# Traversal and sampling (Algorithm 1)
# ---------------------------------------------------------------------------
def rays_for_tests(n=400, seed=7):
    o1, d1 = synth.random_rays(n, seed)
    cam = synth.make_cameras(1, 301, 16, 16)[0]
    o2, d2 = synth.camera_rays(cam)
    o = np.concatenate([o1, o2], axis=1); d = np.concatenate([d1, d2], axis=1)
    # axis-aligned rays, including one lying in a split plane
    extra_o = np.array([[0.3, 0.5, 19 / 32], [0.5, -1.0, 0.25], [19 / 32, 0.2, 0.7]], np.float32).T
    extra_d = np.array([[0.0, 0.0, 1.0], [0.0, 1.0, 0.0], [0.0, 1.0, 0.0]], np.float32).T
    o = np.concatenate([o, extra_o], axis=1); d = np.concatenate([d, extra_d], axis=1)
    return np.ascontiguousarray(o), np.ascontiguousarray(d)


def test_traversal_brute_force_point_in_box_and_chords():
    cfg, g, tree, W = c1_setup()
    o, d = rays_for_tests()
    t0, t1, slot, m = oracle.trace(tree, o, d)
    boxes = tree.leaf_boxes().astype(np.float64) / cfg.grid_n
    n_hit = 0
    for r in range(o.shape[1]):
        oo, dd = o[:, r].astype(np.float64), d[:, r].astype(np.float64)
        chords = np.array([chord_in_box(oo, dd, b[:3], b[3:]) for b in boxes])
        root = chord_in_box(oo, dd, np.zeros(3), np.ones(3))
        k = m[r]
        if k == 0:
            assert root == 0.0
            continue
        n_hit += 1
        # front to back, contiguous, telescoping to the root chord
        assert np.all(t1[r, :k] > t0[r, :k])
        np.testing.assert_array_equal(t1[r, :k - 1], t0[r, 1:k])
        assert abs((t1[r, :k] - t0[r, :k]).sum() - root) <= 1e-12
        # the midpoint of every interval lies in exactly the leaf box named by its slot
        for j in range(k):
            x = oo + 0.5 * (t0[r, j] + t1[r, j]) * dd
            # half-open cells [lo, hi): a point on a split plane belongs to the upper box
            upper_ok = (x < boxes[:, 3:]) | ((x <= boxes[:, 3:]) & (boxes[:, 3:] == 1.0))
            inside = np.where(np.all((x >= boxes[:, :3]) & upper_ok, axis=1))[0]
            assert list(inside) == [slot[r, j]]
        # per-leaf chord lengths from independent box clipping
        per_leaf = np.zeros(len(boxes))
        np.add.at(per_leaf, slot[r, :k], t1[r, :k] - t0[r, :k])
        np.testing.assert_allclose(per_leaf, chords, atol=1e-12)
    assert n_hit > 100


def test_sampling_equal_counts_and_deltas():
    cfg, g, tree, W = c1_setup()
    o, d = rays_for_tests(60)
    t0, t1, slot, m = oracle.trace(tree, o, d)
    for s_max in (1, 5, 64):
        for r in range(o.shape[1]):
            rec = oracle.ray_samples(tree, W, cfg.n_hidden, cfg.hidden, o, d, r, s_max, eps=0.0)
            k = m[r]
            if k == 0:
                assert len(rec["t"]) == 0
                continue
            n = s_max // k if k <= s_max else 1
            keff = min(k, s_max)
            assert len(rec["t"]) == n * keff <= s_max
            for j in range(keff):
                seg = slice(j * n, (j + 1) * n)
                assert np.all(rec["slot"][seg] == slot[r, j])
                # equal count per interval whatever its length (normalised intervals)
                assert abs(rec["delta"][seg].sum() - (t1[r, j] - t0[r, j])) < 1e-13
                # midpoint stratification: t_i = t0 + (i + 1/2) * len / n
                exp_t = t0[r, j] + (np.arange(n) + 0.5) / n * (t1[r, j] - t0[r, j])
                np.testing.assert_allclose(rec["t"][seg], exp_t, rtol=0, atol=1e-13)


def test_jitter_generator_published_vector():
    # splitmix64 seeded with 0: first output 0xE220A8397B1DCDAF (Vigna's reference code)
    assert oracle.lib().orc_splitmix64(0) == 0xE220A8397B1DCDAF
    assert oracle.lib().orc_stratum_offset(1, 0, 0, 0) == 0xE220A8 / 2.0 ** 24
    assert oracle.lib().orc_stratum_offset(0, 5, 3, 2) == 0.5


# ---------------------------------------------------------------------------
# MLP (Section 3.1) against numpy matmuls
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_hidden,hidden", [(2, 32), (4, 64)])
def test_mlp_matches_numpy_matmul(n_hidden, hidden):
    rng = np.random.default_rng(3)
    W = synth.make_weights(1, n_hidden, hidden, 11)[0].astype(np.float64)
    W += rng.standard_normal(W.shape) * 0.1      # non-zero biases too
    W = W.astype(np.float32)
    x = rng.uniform(0, 1, (50, 3)); dirs = rng.standard_normal((50, 3))
    out, feat = oracle.mlp_eval(W, n_hidden, hidden, x, dirs, return_features=True)
    # positional encoding from its definition
    p = 2 * x - 1
    enc = [p]
    for k in range(4):
        enc += [np.sin(2 ** k * np.pi * p), np.cos(2 ** k * np.pi * p)]
    u = np.concatenate(enc + [dirs], axis=1)
    np.testing.assert_allclose(feat, u, rtol=0, atol=1e-15)
    a = u
    off = 0
    Wd = W.astype(np.float64)
    dims = synth.layer_dims(n_hidden, hidden)
    for li, (fi, fo) in enumerate(dims):
        Wl = Wd[off:off + fi * fo].reshape(fo, fi); off += fi * fo
        bl = Wd[off:off + fo]; off += fo
        z = a @ Wl.T + bl
        a = np.maximum(z, 0) if li < len(dims) - 1 else z
    ref = np.concatenate([np.logaddexp(0, a[:, :1]), 1 / (1 + np.exp(-a[:, 1:]))], axis=1)
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------------------
# Compositing: closed forms and invariants
# ---------------------------------------------------------------------------
def constant_field(n_leaves, n_hidden, hidden, sigma0, colour_bias, sigma_per_leaf=None):
    P = synth.param_count(n_hidden, hidden)
    W = np.zeros((n_leaves, P), np.float32)
    sb = synth.sigma_bias_offset(n_hidden, hidden)
    sig = np.full(n_leaves, sigma0) if sigma_per_leaf is None else np.asarray(sigma_per_leaf)
    W[:, sb] = synth.inverse_softplus(sig)
    W[:, sb + 1:sb + 4] = colour_bias
    return W, np.log1p(np.exp(W[:, sb].astype(np.float64)))


@pytest.mark.parametrize("s_max,jitter", [(2, False), (7, False), (64, False), (64, True)])
def test_constant_density_closed_form(s_max, jitter):
    g = np.ones(8 ** 3, np.float32)
    tree = oracle.build_tree(g, 8, 3, 8)
    W, sig = constant_field(8, 2, 32, 2.5, [0.3, -1.0, 2.0])
    sigma0 = float(sig[0])
    c = 1 / (1 + np.exp(-np.array([0.3, -1.0, 2.0], np.float32).astype(np.float64)))
    o = np.array([[0.37], [0.61], [-1.0]], np.float32)
    d = np.array([[0.0], [0.0], [1.0]], np.float32)          # chord length exactly 1
    rgb, depth, opac, ns, flags = oracle.render(tree, W, 2, 32, o, d, s_max, eps=0.0,
                                                jitter=jitter, seed=9)
    T_end = math.exp(-sigma0 * 1.0)
    assert abs(opac[0] - (1 - T_end)) < 1e-14
    np.testing.assert_allclose(rgb[0], c * (1 - T_end), rtol=0, atol=1e-14)


def test_clipped_ray_samples_only_first_intervals():
    """m > S_max: only the first S_max intervals carry one sample each."""
    g = np.ones(8 ** 3, np.float32)
    tree = oracle.build_tree(g, 8, 3, 8)                       # z split at plane 4
    W, sig = constant_field(8, 2, 32, 2.5, [0, 0, 0])
    o = np.array([[0.37], [0.61], [-1.0]], np.float32)
    d = np.array([[0.0], [0.0], [1.0]], np.float32)
    rgb, depth, opac, ns, flags = oracle.render(tree, W, 2, 32, o, d, 1, eps=0.0)
    assert ns[0] == 1 and flags[0] & oracle.FLAG_CLIPPED
    assert abs(opac[0] - (1 - math.exp(-float(sig[0]) * 0.5))) < 1e-14
    assert abs(depth[0] - opac[0] * 1.25) < 1e-14             # the one sample sits at t = 1.25


def test_constant_density_depth_geometric_series():
    g = np.ones(8 ** 3, np.float32)
    tree = oracle.build_tree(g, 8, 0, 1)                       # a single leaf
    W, sig = constant_field(1, 2, 32, 3.0, [0, 0, 0])
    s0 = float(sig[0])
    o = np.array([[0.5], [0.5], [-0.25]], np.float32)
    d = np.array([[0.0], [0.0], [1.0]], np.float32)
    n = 40
    rgb, depth, opac, ns, flags = oracle.render(tree, W, 2, 32, o, d, n, eps=0.0)
    delta = 1.0 / n
    q = math.exp(-s0 * delta)
    a = 1 - q
    t_in = 0.25
    # D = sum_j q^j a (t_in + (j + 1/2) delta)
    S0 = (1 - q ** n) / (1 - q)
    S1 = q * (1 - n * q ** (n - 1) + (n - 1) * q ** n) / (1 - q) ** 2
    D = a * ((t_in + 0.5 * delta) * S0 + delta * S1)
    assert abs(depth[0] - D) < 1e-13
    assert ns[0] == n


def test_piecewise_constant_transmittance_from_brute_force_chords():
    cfg, g, tree, W0 = c1_setup()
    sig_leaf = np.array([0.5, 1.0, 2.0, 0.1, 3.0, 0.25, 1.5, 0.75])
    W, sig = constant_field(8, 2, 32, 0.0, [0, 0, 0], sigma_per_leaf=sig_leaf)
    o, d = rays_for_tests(80)
    rgb, depth, opac, ns, flags = oracle.render(tree, W, 2, 32, o, d, 64, eps=0.0)
    boxes = tree.leaf_boxes().astype(np.float64) / cfg.grid_n
    for r in range(o.shape[1]):
        oo, dd = o[:, r].astype(np.float64), d[:, r].astype(np.float64)
        L = np.array([chord_in_box(oo, dd, b[:3], b[3:]) for b in boxes])
        if ns[r] == 0 or ns[r] < (L > 0).sum():
            continue
        T_end = math.exp(-(sig * L).sum())
        assert abs(opac[r] - (1 - T_end)) < 1e-12


def test_weight_sum_invariant_and_ert():
    cfg, g, tree, W = c1_setup()
    o, d = rays_for_tests(60)
    n_fired = 0
    for r in range(o.shape[1]):
        rec = oracle.ray_samples(tree, W, cfg.n_hidden, cfg.hidden, o, d, r, 64, eps=1e-4)
        if len(rec["t"]) == 0:
            continue
        J = rec["n_used"]
        tau = rec["sigma"][:J] * rec["delta"][:J]
        T_end = math.exp(-tau.sum())
        # sum of weights = 1 - final transmittance
        assert abs(rec["w"].sum() - (1 - T_end)) < 1e-14
        assert abs(rec["opacity"] - rec["w"].sum()) < 1e-14
        np.testing.assert_allclose(rec["ray_rgb"], (rec["w"][:, None] * rec["rgb"]).sum(0), atol=1e-14)
        if rec["flags"] & oracle.FLAG_ERT_FIRED:
            n_fired += 1
            assert T_end < 1e-4
            assert math.exp(-tau[:-1].sum()) >= 1e-4     # the sample before did not stop
            assert np.all(rec["w"][J:] == 0)
        else:
            assert J == len(rec["t"])
    assert n_fired > 0


# ---------------------------------------------------------------------------
# Gradient (training step) by central finite differences
# ---------------------------------------------------------------------------
def test_gradient_matches_central_differences():
    cfg, g, tree, W = c1_setup()
    o, d = synth.camera_rays(synth.make_cameras(1, 301, 12, 12)[0])
    rng = np.random.default_rng(5)
    sel = np.arange(o.shape[1])
    g_rgb = rng.standard_normal((len(sel), 3))
    g_dep = rng.standard_normal(len(sel)) * 0.1
    g_op = rng.standard_normal(len(sel)) * 0.1
    s_max = 16
    grad = oracle.render_grad(tree, W, 2, 32, o, d, s_max, g_rgb, g_dep, g_op, eps=0.0)

    def loss(Wp):
        rgb, dep, op, _, _ = oracle.render(tree, Wp, 2, 32, o, d, s_max, eps=0.0)
        return (rgb * g_rgb).sum() + (dep * g_dep).sum() + (op * g_op).sum()

    # oracle parameters are float32 in memory; perturb in float64 through a float64 copy
    # by scaling the loss function with exact float32 steps
    P = W.shape[1]
    idx = [(l, int(i)) for l in range(8) for i in rng.choice(P, 6, replace=False)]
    sb = synth.sigma_bias_offset(2, 32)
    idx += [(l, sb) for l in range(8)] + [(l, sb + 2) for l in range(8)]
    checked = 0
    for l, i in idx:
        base = float(W[l, i])
        h = 2.0 ** -16 * max(1.0, abs(base))
        Wp = W.copy(); Wp[l, i] = np.float32(base + h)
        Wm = W.copy(); Wm[l, i] = np.float32(base - h)
        hp = float(Wp[l, i]) - base; hm = base - float(Wm[l, i])
        fd = (loss(Wp) - loss(Wm)) / (hp + hm)
        Wp2 = W.copy(); Wp2[l, i] = np.float32(base + h / 4)
        Wm2 = W.copy(); Wm2[l, i] = np.float32(base - h / 4)
        fd2 = (loss(Wp2) - loss(Wm2)) / (float(Wp2[l, i]) - float(Wm2[l, i]))
        # skip parameters whose +-h window straddles a ReLU kink (the two step sizes disagree)
        if abs(fd - fd2) > 1e-6 * max(1.0, abs(fd)):
            continue
        assert abs(grad[l, i] - fd2) <= 1e-7 * max(1.0, abs(fd2)), (l, i, grad[l, i], fd2)
        checked += 1
    assert checked >= 0.8 * len(idx)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    p = rng.standard_normal(100)
    m = np.zeros(100); v = np.zeros(100)
    tp = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 11):
        g = rng.standard_normal(100)
        oracle.adam(p, m, v, g, step)
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=0, atol=1e-14)


# ---------------------------------------------------------------------------
# Buckets (sort by node id)
# ---------------------------------------------------------------------------
def test_buckets_are_contiguous_stable_and_counted():
    rng = np.random.default_rng(1)
    keys = rng.integers(0, 37, 5000)
    counts, offsets, perm = oracle.buckets(keys, 40)
    assert offsets[-1] == len(keys)
    for b in range(40):
        seg = perm[offsets[b]:offsets[b + 1]]
        assert len(seg) == counts[b] == (keys == b).sum()
        assert np.all(keys[seg] == b) and np.all(np.diff(seg.astype(np.int64)) > 0)


@pytest.mark.parametrize("n,max_depth,max_leaves", [(32, 6, 64), (32, 12, 40), (64, 12, 512)])
def test_middle_split_is_regular_subdivision(n, max_depth, max_leaves):
    """The regular subdivision of the ablation: breadth-first, middle planes, independent of
    the density; with 2^k leaves on a 2^m grid the leaves are equal boxes tiling the grid."""
    g1 = synth.make_grid(synth.scaled(synth.C1, grid_n=n))
    g2 = np.random.default_rng(3).uniform(0, 10, n ** 3).astype(np.float32)
    t1 = oracle.build_tree(g1, n, max_depth, max_leaves, split=1)
    t2 = oracle.build_tree(g2, n, max_depth, max_leaves, split=1)
    assert t1.n_leaves == max_leaves
    np.testing.assert_array_equal(t1.rows, t2.rows)          # the structure ignores the density
    rows = t1.rows
    q = quantised(g1).reshape(n, n, n)
    for r, m in zip(rows, t1.mass):
        lx, ly, lz, hx, hy, hz = r[2:8]
        assert int(q[lz:hz, ly:hy, lx:hx].sum()) == int(m)
    inner = rows[rows[:, 8] >= 0]
    for r in inner:
        a, p = int(r[8]), int(r[9])
        ext = r[5:8] - r[2:5]
        assert a == int(np.argmax(ext))
        assert p == (int(r[2 + a]) + int(r[5 + a])) // 2
    leaves = rows[rows[:, 10] >= 0]
    depths = leaves[:, 1]
    assert depths.max() - depths.min() <= 1                   # breadth-first
    # the leaves split at the deepest level are those of smallest code at the level above
    shallow = leaves[depths == depths.min()]
    deep_parents = sorted({int(c) >> 1 for c in leaves[depths == depths.max()][:, 0]})
    if depths.max() != depths.min():
        assert max(deep_parents) < shallow[:, 0].min()
    if max_leaves & (max_leaves - 1) == 0:
        k = max_leaves.bit_length() - 1
        side = n >> (k // 3)
        ext = leaves[:, 5:8] - leaves[:, 2:5]
        assert np.all(depths == k)
        assert np.all(ext.max(axis=1) <= side) and np.all(ext.min(axis=1) >= side // 2)
        assert np.all(np.prod(ext, axis=1) == n ** 3 // max_leaves)


def test_middle_split_hand_derived():
    """4^3 grid, regular subdivision: the root's sides tie, so x is cut at cell 2; then the
    depth-1 leaves in code order (2 before 3), each 2x4x4 cells, are cut along y at cell 2.
    Rows: code, depth, lo, hi, axis, plane, leaf slot, node slot."""
    g = np.random.default_rng(9).uniform(0, 1, 4 ** 3).astype(np.float32)   # ignored by the split
    rows4 = [
        (1, 0, 0, 0, 0, 4, 4, 4, 0, 2, -1, 0),
        (2, 1, 0, 0, 0, 2, 4, 4, 1, 2, -1, 1),
        (3, 1, 2, 0, 0, 4, 4, 4, 1, 2, -1, 4),
        (4, 2, 0, 0, 0, 2, 2, 4, -1, -1, 0, 2),
        (5, 2, 0, 2, 0, 2, 4, 4, -1, -1, 1, 3),
        (6, 2, 2, 0, 0, 4, 2, 4, -1, -1, 2, 5),
        (7, 2, 2, 2, 0, 4, 4, 4, -1, -1, 3, 6),
    ]
    t = oracle.build_tree(g, 4, 2, 4, split=1)
    np.testing.assert_array_equal(t.rows, np.array(rows4, np.int32))
    rows3 = [
        (1, 0, 0, 0, 0, 4, 4, 4, 0, 2, -1, 0),
        (2, 1, 0, 0, 0, 2, 4, 4, 1, 2, -1, 1),
        (3, 1, 2, 0, 0, 4, 4, 4, -1, -1, 2, 4),
        (4, 2, 0, 0, 0, 2, 2, 4, -1, -1, 0, 2),
        (5, 2, 0, 2, 0, 2, 4, 4, -1, -1, 1, 3),
    ]
    t = oracle.build_tree(g, 4, 2, 3, split=1)
    np.testing.assert_array_equal(t.rows, np.array(rows3, np.int32))
