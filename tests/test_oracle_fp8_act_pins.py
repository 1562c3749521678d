"""Pins of the oracle's float8-activation model (the float8 matrix-core variant of the leaf
MLPs): the C rounding of activations against the e4m3 table quantiser, the power-of-two
exponent rules on hand-worked values, the quantised forward on networks whose activations
are exactly representable (it must equal the plain forward) or hand-worked (closed forms),
the per-leaf exponent rows inside a render, and the calibration maxima against a numpy
forward over the oracle's own sample records."""
from __future__ import annotations

import numpy as np

import oracle
import synth
from oracle import fp8


def test_c_rounding_matches_the_table_quantiser():
    vals = fp8.decode(np.arange(127))
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(0, 500, 3000), np.abs(rng.standard_normal(3000)) * 0.02,
                        (vals[:-1] + vals[1:]) / 2, vals, [448.0, 460.0, 464.0, 1e4]])
    got = np.array([oracle.e4m3_round(v) for v in x])
    want = fp8.decode(fp8.encode(x))
    assert np.array_equal(got, want)


def test_c_bf16_rounding_matches_the_bit_rounding():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(3000) * np.exp(rng.uniform(-20, 20, 3000)),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, 3.0e38]])
    x = x.astype(np.float32)
    got = np.array([oracle.bf16_round(float(v)) for v in x])
    assert np.array_equal(got, fp8.bf16_round(x).astype(np.float64))


def test_exponent_rules_hand_worked():
    # activations: 1.25 m <= 256 * 2^k; 204.8 in float32 is just above 256 / 1.25 (and the
    # float32 below it just under), 1.25 * 0.8 (float32 0.8 is just above 0.8) is just above
    # 1 = 256 * 2^-8, and 1.25 * 0.375 = 0.46875 lies in (256 * 2^-10, 256 * 2^-9]
    assert fp8.act_exponents([204.79999, 204.8, 0.0, 0.8, 0.375, 1000.0]).tolist() == [0, 1, 0, -7, -9, 3]
    # weights: max |W| <= 448 * 2^e
    assert fp8.pow2_exponent([448.0, 448.5, 0.7, 0.0, 0.875], 448.0).tolist() == [0, 1, -9, 0, -9]


def _one_leaf(n_hidden, hidden, layers):
    """Master vector of one leaf from [(W[out][in], b[out]), ...]."""
    parts = []
    for W, b in layers:
        parts += [np.asarray(W, np.float64).reshape(-1), np.asarray(b, np.float64)]
    v = np.concatenate(parts).astype(np.float32)
    assert v.size == synth.param_count(n_hidden, hidden)
    return v


def test_representable_activations_leave_the_forward_unchanged():
    H = 8
    W0 = np.zeros((H, 30))
    b0 = [0.0, 1.0, 2.0, 3.0, 4.0, -1.0, 6.0, 8.0]          # ReLU outputs all e4m3 values
    W1 = np.eye(H)[::-1]                                     # a permutation: same values
    b1 = np.zeros(H)
    rng = np.random.default_rng(1)
    Wo = rng.standard_normal((4, H)) * 0.1
    bo = rng.standard_normal(4)
    p = _one_leaf(2, H, [(W0, b0), (W1, b1), (Wo, bo)])
    x = rng.uniform(0, 1, (50, 3)); dr = rng.standard_normal((50, 3))
    plain = oracle.mlp_eval(p, 2, H, x, dr)
    for k in ([0, 0], [-3, 2], [1, -1]):                    # 2^k steps keep these exact
        assert np.array_equal(oracle.mlp_eval_q8(p, 2, H, x, dr, k), plain), k


def test_rounding_and_saturation_closed_form():
    H = 2
    W0 = np.zeros((H, 30))
    b0 = [17.0, 1000.0]
    Wo = np.zeros((4, H))
    Wo[0] = [1.0 / 64, 0.0]
    Wo[1] = [0.0, 1.0 / 1024]
    Wo[2] = [-1.0 / 64, 1.0 / 1024]
    p = _one_leaf(1, H, [(W0, b0), (Wo, np.zeros(4))])
    x = np.full((1, 3), 0.3); dr = np.array([[0.0, 0.0, 1.0]])

    def heads(z):
        sp = np.log1p(np.exp(z[0]))
        return np.array([sp] + [1.0 / (1.0 + np.exp(-v)) for v in z[1:]])

    # k = 0: 17 is a tie between 16 and 18 -> 16 (even code); 1000 saturates at 256
    got = oracle.mlp_eval_q8(p, 1, H, x, dr, [0])[0]
    assert np.allclose(got, heads(np.array([16 / 64, 256 / 1024, -16 / 64 + 256 / 1024, 0.0])), rtol=1e-15)
    # k = 2: 17/4 = 4.25 -> 4 (tie, even) -> 16; 1000/4 = 250 -> 256 -> 1024
    got = oracle.mlp_eval_q8(p, 1, H, x, dr, [2])[0]
    assert np.allclose(got, heads(np.array([16 / 64, 1.0, -16 / 64 + 1.0, 0.0])), rtol=1e-15)
    # k = -12: 17 * 2^12 and 1000 * 2^12 saturate at 256 * 2^-12
    got = oracle.mlp_eval_q8(p, 1, H, x, dr, [-12])[0]
    s = 256 * 2.0 ** -12
    assert np.allclose(got, heads(np.array([s / 64, s / 1024, -s / 64 + s / 1024, 0.0])), rtol=1e-15)
    # negative pre-activations are zero before rounding; tiny ones underflow to zero
    p2 = _one_leaf(1, H, [(W0, [-3.0, 1e-4]), (Wo, np.zeros(4))])
    got = oracle.mlp_eval_q8(p2, 1, H, x, dr, [0])[0]
    assert np.allclose(got, heads(np.zeros(4)), rtol=1e-15)


def test_first_layer_inputs_are_bfloat16():
    """p_x = 2x - 1 just below an e4m3 midpoint (0.59375) rounds to the midpoint in bfloat16,
    which then goes to the even e4m3 neighbour 0.625; unrounded it would give 0.5625."""
    H = 2
    W0 = np.zeros((H, 30)); W0[0, 0] = 1.0
    Wo = np.zeros((4, H)); Wo[1, 0] = 1.0
    p = _one_leaf(1, H, [(W0, np.zeros(H)), (Wo, np.zeros(4))])
    px = 0.59375 - 2.0 ** -11
    x = np.array([[(px + 1.0) / 2.0, 0.5, 0.5]]); dr = np.array([[0.0, 0.0, 1.0]])
    assert 2.0 * x[0, 0] - 1.0 == px
    got = oracle.mlp_eval_q8(p, 1, H, x, dr, [0])[0, 1]
    assert got == 1.0 / (1.0 + np.exp(-0.625))
    assert oracle.mlp_eval(p, 1, H, x, dr)[0, 1] == 1.0 / (1.0 + np.exp(-px))


def _two_leaf_scene():
    cfg = synth.scaled(synth.C1, width=12, height=12)
    grid = synth.make_grid(cfg)
    tree = oracle.build_tree(grid, cfg.grid_n, 1, 2)
    assert tree.n_leaves == 2
    W = synth.make_weights(2, cfg.n_hidden, cfg.hidden, 11)
    cams = synth.make_cameras(1, cfg.seed_cameras, cfg.width, cfg.height)
    o, d = synth.rays_for_cameras(cams)
    return cfg, tree, W, o, d


def test_render_uses_each_leafs_exponent_row():
    """The q8 render of every ray equals the quadrature of the per-sample q8 outputs computed
    leaf by leaf with that leaf's own exponents (which differ between the two leaves)."""
    cfg, tree, W, o, d = _two_leaf_scene()
    k = np.array([[-2, 1], [3, -4]], np.int32)
    rgb, depth, opac = oracle.render_q8(tree, W, cfg.n_hidden, cfg.hidden, o, d, 32, k, eps=1e-4)
    plain, _, _, _, _ = oracle.render(tree, W, cfg.n_hidden, cfg.hidden, o, d, 32, eps=1e-4)
    assert not np.array_equal(rgb, plain)
    n_hit = 0
    for r in range(o.shape[1]):
        s = oracle.ray_samples(tree, W, cfg.n_hidden, cfg.hidden, o, d, r, 32, eps=1e-4)
        if len(s["t"]) == 0:
            assert not rgb[r].any()
            continue
        n_hit += 1
        x = o[:, r][None, :].astype(np.float64) + s["t"][:, None] * d[:, r][None, :].astype(np.float64)
        dr = np.repeat(d[:, r][None, :].astype(np.float64), len(x), 0)
        z = np.zeros((len(x), 4))
        for leaf in np.unique(s["slot"]):
            sel = s["slot"] == leaf
            out = oracle.mlp_eval_q8(W[leaf], cfg.n_hidden, cfg.hidden, x[sel], dr[sel], k[leaf])
            z[sel, 0] = np.log(np.expm1(out[:, 0]))                  # back to pre-activations
            z[sel, 1:] = np.log(out[:, 1:] / (1.0 - out[:, 1:]))
        res, _, _ = oracle.composite(z, s["t"], s["delta"], eps=1e-4)
        assert np.allclose(res[:3], rgb[r], rtol=0, atol=1e-12)
        assert np.allclose(res[3:], [depth[r], opac[r]], rtol=0, atol=1e-12)
    assert n_hit > 50


def test_calibration_maxima_against_numpy_forward():
    cfg, tree, W, o, d = _two_leaf_scene()
    got = oracle.act_max(tree, W, cfg.n_hidden, cfg.hidden, o, d, 32)
    want = np.zeros((2, cfg.n_hidden))
    sl = fp8.layer_slices(cfg.n_hidden, cfg.hidden)
    for r in range(o.shape[1]):
        s = oracle.ray_samples(tree, W, cfg.n_hidden, cfg.hidden, o, d, r, 32, eps=0.0)
        if len(s["t"]) == 0:
            continue
        x = o[:, r][None, :].astype(np.float64) + s["t"][:, None] * d[:, r][None, :].astype(np.float64)
        dr = np.repeat(d[:, r][None, :].astype(np.float64), len(x), 0)
        for leaf in np.unique(s["slot"]):
            sel = s["slot"] == leaf
            _, a = oracle.mlp_eval(W[leaf], cfg.n_hidden, cfg.hidden, x[sel], dr[sel], return_features=True)
            for li in range(cfg.n_hidden):
                ow, din, dout, ob = sl[li]
                Wl = W[leaf, ow:ow + din * dout].astype(np.float64).reshape(dout, din)
                a = np.maximum(a @ Wl.T + W[leaf, ob:ob + dout].astype(np.float64), 0.0)
                want[leaf, li] = max(want[leaf, li], a.max())
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    assert (want > 0).all()
