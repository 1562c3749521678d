"""Pins of the oracle's learned-proposal functions (not in the paper; its reading is stated in
the oracle): features from the interval geometry, the network against numpy matmuls, the
analytic gradient against central differences, the slot masses' partition of the predicted
weight, the minimality of the selected slot set, and the all-fallback special case."""
import math

import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import constant_field


def scene():
    cfg = synth.C1
    g = synth.make_grid(cfg)
    tree = oracle.build_tree(g, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
    dens = synth.leaf_mean_density(g, cfg.grid_n, tree.leaf_boxes())
    W = synth.make_weights(tree.n_leaves, cfg.n_hidden, cfg.hidden, cfg.seed_weights, dens)
    prop = synth.make_prop_weights(cfg.seed_proposal)
    o, d = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras, 12, 12)[0])
    return cfg, tree, W, prop, o, d


def test_features_follow_interval_geometry():
    cfg, tree, W, prop, o, d = scene()
    feat, tau = oracle.prop_eval(tree, prop, o, d, cfg.s_max)
    t0, t1, slot, m = oracle.trace(tree, o, d)
    boxes = tree.leaf_boxes().astype(np.float64) / cfg.grid_n
    i = 0
    for r in range(o.shape[1]):
        for k in range(min(m[r], cfg.s_max)):
            f = feat[i]
            oo, dd = o[:, r].astype(np.float64), d[:, r].astype(np.float64)
            np.testing.assert_allclose(f[0:3], (oo - 0.5) / 2, atol=1e-15)
            np.testing.assert_allclose(f[3:6], dd, atol=1e-15)
            # sin^2 + cos^2 = 1 for every encoded pair
            for base in (6, 12, 18, 24):
                np.testing.assert_allclose(f[base:base + 3] ** 2 + f[base + 3:base + 6] ** 2, 1.0, atol=1e-14)
            assert f[30] == k / cfg.s_max
            lo, hi = boxes[slot[r, k], :3], boxes[slot[r, k], 3:]
            np.testing.assert_allclose(f[31:34], lo + hi - 1.0, atol=1e-15)
            np.testing.assert_allclose(f[34:37], hi - lo, atol=1e-15)
            entry = (f[37:40] + 1) / 2
            exit_ = (f[40:43] + 1) / 2
            np.testing.assert_allclose(entry, oo + t0[r, k] * dd, atol=1e-14)
            np.testing.assert_allclose(exit_, oo + t1[r, k] * dd, atol=1e-14)
            # entry and exit lie in the (closed) leaf box
            assert np.all(entry >= lo - 1e-12) and np.all(entry <= hi + 1e-12)
            assert np.all(exit_ >= lo - 1e-12) and np.all(exit_ <= hi + 1e-12)
            i += 1
    assert i == len(feat) > 50


def test_network_matches_numpy():
    cfg, tree, W, prop, o, d = scene()
    feat, tau = oracle.prop_eval(tree, prop, o, d, cfg.s_max)
    P = prop.astype(np.float64)
    a, off = feat, 0
    for li, (fi, fo) in enumerate(synth.PROP_DIMS):
        Wl = P[off:off + fi * fo].reshape(fo, fi); off += fi * fo
        bl = P[off:off + fo]; off += fo
        z = a @ Wl.T + bl
        a = np.maximum(z, 0) if li < 2 else z
    np.testing.assert_allclose(tau, np.logaddexp(0, a), rtol=1e-13, atol=1e-14)


def test_loss_gradient_matches_central_differences():
    cfg, tree, W, prop, o, d = scene()
    feat, _ = oracle.prop_eval(tree, prop, o, d, cfg.s_max)
    alpha = oracle.prop_targets(tree, W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max)
    assert alpha.shape == (len(feat), 32) and np.all((alpha >= 0) & (alpha <= 1))
    loss, grad = oracle.prop_loss_grad(prop, feat, alpha)
    rng = np.random.default_rng(0)
    idx = rng.choice(len(prop), 60, replace=False)
    checked = 0
    for i in idx:
        base = float(prop[i])
        vals = []
        for h in (2.0 ** -14, 2.0 ** -16):
            pp = prop.copy(); pp[i] = np.float32(base + h)
            pm = prop.copy(); pm[i] = np.float32(base - h)
            vals.append((oracle.prop_loss_grad(pp, feat, alpha)[0] - oracle.prop_loss_grad(pm, feat, alpha)[0])
                        / (float(pp[i]) - float(pm[i])))
        if abs(vals[0] - vals[1]) > 1e-6 * max(1e-3, abs(vals[1])):
            continue                     # a ReLU kink inside the step
        assert abs(grad[i] - vals[1]) <= 1e-6 * max(1e-3, abs(vals[1])), (i, grad[i], vals[1])
        checked += 1
    assert checked >= 45


def test_targets_reduce_to_closed_form_for_constant_density():
    """Constant sigma0 over a single leaf: every bin of an interval of length L has
    thickness sigma0 * L / 32."""
    g = np.ones(8 ** 3, np.float32)
    tree = oracle.build_tree(g, 8, 0, 1)
    P = synth.param_count(2, 32)
    W = np.zeros((1, P), np.float32)
    sb = synth.sigma_bias_offset(2, 32)
    W[0, sb] = synth.inverse_softplus(2.0)
    sigma0 = float(np.logaddexp(0, np.float64(W[0, sb])))
    o = np.array([[0.5], [0.5], [-1.0]], np.float32)
    d = np.array([[0.0], [0.0], [1.0]], np.float32)
    for s_max in (7, 32, 100):
        alpha = oracle.prop_targets(tree, W, 2, 32, o, d, s_max)
        np.testing.assert_allclose(alpha[0], -math.expm1(-sigma0 / 32), rtol=1e-13)


def plan_slot_masses(tau_ray, meff, n):
    """Slot masses of one ray from its predicted thicknesses: the bins composited front to
    back, each bin's weight spread over the slots it overlaps in proportion to the covered
    length (whole numbers of 1/(32 n) of the interval, so equal overlaps are equal)."""
    tt = tau_ray.reshape(-1)
    S = np.concatenate([[0.0], np.cumsum(tt)])
    wb = np.exp(-S[:-1]) * -np.expm1(-tt)
    p = np.zeros(meff * n)
    for k in range(meff):
        for b in range(32):
            for j in range(n):
                ov = min(32 * (j + 1), (b + 1) * n) - max(32 * j, b * n)
                if ov > 0:
                    p[k * n + j] += wb[k * 32 + b] * (ov / n)
    return p, -math.expm1(-S[-1])


@pytest.mark.parametrize("s_max", [64, 160])
def test_plan_invariants_and_all_fallback(s_max):
    cfg, tree, W, prop, o, d = scene()
    # an untrained proposal still yields valid plans; check the selection rule's invariants
    rgb, dep, op, ns, pn, psel, mass = oracle.render_proposal(tree, W, 2, 32, prop, o, d, s_max, eps=1e-4,
                                                              mass_thresh=0.5, cap=s_max)
    feat, tau = oracle.prop_eval(tree, prop, o, d, s_max)
    t0, t1, slot, m = oracle.trace(tree, o, d)
    i = 0
    n_planned = n_ties = 0
    for r in range(o.shape[1]):
        meff = min(m[r], s_max)
        if meff == 0:
            continue
        n = s_max // m[r] if m[r] <= s_max else 1
        p, M = plan_slot_masses(tau[i:i + meff], meff, n)
        i += meff
        assert abs(p.sum() - M) < 1e-12                    # slots partition the predicted weight
        assert abs(mass[r] - M) < 1e-12
        if M < 0.5:
            assert pn[r] == -1
            continue
        if pn[r] < 0:
            continue
        n_planned += 1
        sel = psel[r, :pn[r]]
        assert np.all(np.diff(sel) > 0)
        chosen = p[sel]
        assert chosen.sum() >= 0.5 * M - 1e-12
        assert chosen.sum() - chosen.min() < 0.5 * M + 1e-12   # none can be dropped
        others = np.delete(p, sel)
        assert others.size == 0 or others.max() <= chosen.min()
        # ties at the cut go to the earlier slots
        cut = chosen.min()
        tied = np.flatnonzero(p == cut)
        kept_tied = np.intersect1d(tied, sel)
        assert np.array_equal(kept_tied, tied[:kept_tied.size])
        n_ties += int(tied.size > kept_tied.size)
        assert ns[r] == pn[r]
    assert n_planned > 10
    if s_max == 160:
        assert n_ties > 0      # slots inside one bin tie, and some cut falls among them
    if s_max != 64:
        return
    # a threshold no predicted mass reaches: every ray falls back -> identical to plain
    rgb2, dep2, op2, ns2, pn2, _, _ = oracle.render_proposal(tree, W, 2, 32, prop, o, d, cfg.s_max, eps=1e-4,
                                                             mass_thresh=2.0, cap=48)
    rgb0, dep0, op0, ns0, _ = oracle.render(tree, W, 2, 32, o, d, cfg.s_max, eps=1e-4)
    assert np.all(pn2[ns0 > 0] == -1) and np.all(pn2[ns0 == 0] == 0)
    np.testing.assert_array_equal(rgb2, rgb0)
    np.testing.assert_array_equal(dep2, dep0)
    np.testing.assert_array_equal(ns2, ns0)


@pytest.mark.parametrize("sigma0,thresh", [(5.0, 0.9), (3.0, 0.95), (8.0, 0.99)])
def test_exact_histogram_selects_the_front_slots(sigma0, thresh):
    """A proposal that predicts the true bin thicknesses of a constant-density ray: one leaf,
    a ray along z with chord 1 and S_max = 32, so each of the 32 slots is one bin, bin b
    has thickness sigma0 / 32 and weight exp(-sigma0 b / 32) (1 - exp(-sigma0 / 32)),
    decreasing along the ray.  The plan keeps the first c slots, c the least count with
    1 - exp(-sigma0 c / 32) >= thresh (1 - exp(-sigma0)); the planned render is the plain
    quadrature over them, so its opacity is 1 - exp(-sigma0 c / 32) and it differs from the
    plain render by exactly the skipped weight."""
    g = np.ones(8 ** 3, np.float32)
    tree = oracle.build_tree(g, 8, 0, 1)
    W, sig = constant_field(1, 2, 32, sigma0, [0.4, -0.2, 1.0])
    s0 = float(sig[0])
    c0 = 1 / (1 + np.exp(-np.array([0.4, -0.2, 1.0], np.float32).astype(np.float64)))
    o = np.array([[0.37], [0.61], [-1.0]], np.float32)
    d = np.array([[0.0], [0.0], [1.0]], np.float32)
    tau = np.full((1, 32), s0 / 32)
    prop = np.zeros(oracle.prop_param_count(), np.float32)
    rgb, dep, op, ns, pn, psel, mass = oracle.render_proposal(tree, W, 2, 32, prop, o, d, 32, eps=0.0,
                                                              mass_thresh=thresh, cap=32, tau=tau)
    M = -math.expm1(-s0)
    assert abs(mass[0] - M) < 1e-14
    c = math.ceil(-32 / s0 * math.log(1 - thresh * M) - 1e-12)
    assert pn[0] == c and ns[0] == c
    assert list(psel[0, :c]) == list(range(c))
    op_c = -math.expm1(-s0 * c / 32)
    assert abs(op[0] - op_c) < 1e-14
    np.testing.assert_allclose(rgb[0], c0 * op_c, rtol=0, atol=1e-14)
    _, _, op_plain, _, _ = oracle.render(tree, W, 2, 32, o, d, 32, eps=0.0)
    assert abs((op_plain[0] - op[0]) - (math.exp(-s0 * c / 32) - math.exp(-s0))) < 1e-14
