"""The float8 matrix-core leaf MLPs (AMNERF_FP8_ACT: e4m3 weights and activations) on the
GPU: the packed block's exponents and codes against the oracle's power-of-two quantisation,
the calibration maxima against the oracle's, per-sample outputs and renders against the
oracle's float8-activation model on the same exponents, and renders against the oracle on
the dequantised weights with float64 activations.

Rounding decisions are taken in different precisions on the two sides (float32 accumulation
on the matrix cores, float64 in the oracle), so an activation that lands next to an e4m3
rounding boundary can round the other way; the per-sample checks bound a high quantile and
the worst case instead of every value."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from oracle import fp8
from scene_util import Scene, gpu_setup, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2310_01881_amd as am  # noqa: E402

# Against the oracle's float8-activation model on the same exponents (measured values in
# the tests' output and the design notes).
PSNR_VS_Q8 = {"c1": 60.0, "c2": 68.0}      # measured 65.2 and 74.7 dB
# Against the oracle on the dequantised weights with float64 activations: the float8
# activations' own error.
PSNR_VS_DEQ = 46.0      # measured 50.7 (c1) and 50.5 dB (c2)


def block_regions(n_hidden):
    """(header, layer 0, float8 layers [(offset, bytes)], bias words, block bytes) as the
    packing call documents them."""
    off = 64 + 4096
    layers = []
    for _ in range(n_hidden - 1):
        layers.append((off, 4096))
        off += 4096
    layers.append((off, 2048))
    off += 2048
    bias = (off, n_hidden * 256 + 256)
    off += bias[1]
    return layers, bias, (off + 255) // 256 * 256


@pytest.mark.parametrize("n_hidden,n_leaves", [(1, 3), (2, 5), (3, 4), (4, 9)])
def test_packed_exponents_and_codes(n_hidden, n_leaves):
    print("fp8-act pack", n_hidden, n_leaves, flush=True)
    W = synth.make_weights(n_leaves, n_hidden, 64, 17)
    rng = np.random.default_rng(n_leaves)
    sl = fp8.layer_slices(n_hidden, 64)
    for ow, din, dout, ob in sl:
        W[:, ob:ob + dout] = rng.standard_normal((n_leaves, dout)).astype(np.float32)
    if n_hidden > 1:
        W[0, sl[1][0]:sl[1][0] + sl[1][1] * sl[1][2]] = 0.0           # an all-zero float8 layer
    W[1 % n_leaves, sl[-1][0]:sl[-1][0] + 64 * 4] *= 600.0              # an exponent above 0
    act_max = np.exp(rng.uniform(-6, 8, (n_leaves, n_hidden))).astype(np.float32)
    act_max[0, 0] = 0.0
    act_max[n_leaves - 1, -1] = np.float32(204.8)                       # just above 256 / 1.25
    ctx = am.Context(0)
    mlp = am.Mlp(ctx, to_dev(W), n_hidden, 64, am.AMNERF_FP8_ACT, n_leaves, act_max_dev=to_dev(act_max))
    torch.cuda.synchronize()
    blk = mlp.packed.cpu().numpy()
    layers, bias, per = block_regions(n_hidden)
    assert blk.size == per * n_leaves
    w_exp, k, _ = fp8.quantise_mma(W, n_hidden, 64, act_max)
    for leaf in range(n_leaves):
        b = blk[leaf * per:(leaf + 1) * per]
        hdr = b[:64].view(np.int32)
        assert np.array_equal(hdr[:n_hidden], k[leaf]), (leaf, hdr[:4], k[leaf])
        assert np.array_equal(hdr[4:4 + n_hidden], w_exp[leaf])
        k_out = np.concatenate([k[leaf, 1:] + 8, [0]])
        want_sc = np.clip(127 + w_exp[leaf] + k[leaf] - k_out, 0, 254)
        assert np.array_equal(hdr[8:8 + n_hidden], want_sc)
        assert not hdr[12:].any() and not hdr[n_hidden:4].any()
        for li, (off, n) in enumerate(layers):
            ow, din, dout, _ = sl[li + 1]
            w = W[leaf, ow:ow + din * dout].astype(np.float64) * 2.0 ** -w_exp[leaf, li]
            want = np.sort(np.concatenate([fp8.encode(w), np.zeros(n - w.size, np.uint8)]))
            got = np.sort(b[off:off + n])
            assert np.array_equal(got, want), (leaf, li, np.count_nonzero(got != want))
        assert not b[bias[0] + bias[1]:].any()


def calibrated(scene, cam=1, n_rays=3000, seed=0):
    """Calibration maxima from the oracle over a sample of another camera's rays."""
    cfg = scene.cfg
    oc, dc = scene.camera_rays(cam)
    pick = np.sort(np.random.default_rng(seed).choice(oc.shape[1], min(n_rays, oc.shape[1]), replace=False))
    return oracle.act_max(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, oc, dc, cfg.s_max, ray_idx=pick).astype(
        np.float32)


def test_calibration_maxima_against_oracle():
    cfg = synth.scaled(synth.C1, n_hidden=4, hidden=64)
    scene = Scene(cfg)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_BF16)
    o, d = scene.camera_rays()
    rob = np.where(oracle.robust(scene.otree, o, d))[0]
    o, d = np.ascontiguousarray(o[:, rob]), np.ascontiguousarray(d[:, rob])
    od, dd = to_dev(o), to_dev(d)
    am.render(ctx, tree, mlp, od, dd, cfg.s_max)
    got = torch.zeros((tree.n_leaves, cfg.n_hidden), dtype=torch.float32, device="cuda:0")
    am.amnerf_mlp_calibrate(ctx.h, cfg.n_hidden, tree.n_leaves, mlp.master, od, dd, got)
    torch.cuda.synchronize()
    g = got.cpu().numpy().astype(np.float64)
    want = oracle.act_max(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max)
    print("calibration maxima: max relative difference %.3e" % np.max(np.abs(g - want) / np.maximum(want, 1e-30)),
          flush=True)
    np.testing.assert_allclose(g, want, rtol=1e-4, atol=0)
    # the exponents agree wherever the maximum is not within 1e-4 of a rounding boundary
    kg, kw = fp8.act_exponents(g), fp8.act_exponents(want)
    frac = np.log2(1.25 * want / 448.0)
    safe = np.abs(frac - np.round(frac)) > 1e-4
    assert np.array_equal(kg[safe], kw[safe])
    # a second call over the same render accumulates to the same maxima
    am.amnerf_mlp_calibrate(ctx.h, cfg.n_hidden, tree.n_leaves, mlp.master, od, dd, got)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), g.astype(np.float32))
    # state errors: other rays, a render in rounds, a wrong parameter-set count
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_mlp_calibrate(ctx.h, cfg.n_hidden, tree.n_leaves, mlp.master, to_dev(o[:, :10]), to_dev(d[:, :10]),
                                got)
    assert e.value.code == am.AMNERF_ESTATE
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_mlp_calibrate(ctx.h, cfg.n_hidden, tree.n_leaves + 1, mlp.master, od, dd, got)
    assert e.value.code == am.AMNERF_EINVAL
    out = {"rgb": torch.empty((o.shape[1], 3), device="cuda:0")}
    am.amnerf_render(ctx.h, tree.h, mlp.desc, od, dd, cfg.s_max, out["rgb"], ert_rounds=True)
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_mlp_calibrate(ctx.h, cfg.n_hidden, tree.n_leaves, mlp.master, od, dd, got)
    assert e.value.code == am.AMNERF_ESTATE


def render_case(cfg, label, rays_sel=None):
    scene = Scene(cfg)
    amax = calibrated(scene)
    w_exp, k, deq = fp8.quantise_mma(scene.W, cfg.n_hidden, cfg.hidden, amax)
    ctx = am.Context(0)
    tree = am.Tree(ctx, scene.grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves, 0)
    assert np.array_equal(tree.rows, scene.otree.rows)
    mlp = am.Mlp(ctx, to_dev(scene.W), cfg.n_hidden, cfg.hidden, am.AMNERF_FP8_ACT, tree.n_leaves,
                 act_max_dev=to_dev(amax))
    o, d = scene.camera_rays()
    R = o.shape[1]
    print(label, "rays", R, flush=True)
    out = am.render(ctx, tree, mlp, to_dev(o), to_dev(d), cfg.s_max, ert_eps=cfg.ert_eps)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    assert st["n_nonfinite"] == 0 and st["n_unreached"] == 0
    rays = np.arange(R) if rays_sel is None else rays_sel(R)
    g = out["rgb"].cpu().numpy()[rays]
    q8, _, _ = oracle.render_q8(scene.otree, deq, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max, k, eps=cfg.ert_eps,
                                ray_idx=rays)
    rd, _, _, _, _ = oracle.render(scene.otree, deq, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max, eps=cfg.ert_eps,
                                   ray_idx=rays)
    rp, _, _, _, _ = oracle.render(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max,
                                   eps=cfg.ert_eps, ray_idx=rays)
    p_q8, p_deq, p_plain = oracle.psnr(g, q8), oracle.psnr(g, rd), oracle.psnr(g, rp)
    print("%s: psnr vs oracle float8 model %.2f dB (max abs %.3e), vs dequantised weights %.2f dB, vs float32 "
          "weights %.2f dB; oracle float8 model vs dequantised %.2f dB" % (
              label, p_q8, np.abs(g - q8).max(), p_deq, p_plain, oracle.psnr(q8, rd)), flush=True)
    return scene, ctx, tree, mlp, k, deq, p_q8, p_deq


def test_c1_render_against_oracle_models():
    cfg = synth.scaled(synth.C1, n_hidden=4, hidden=64)
    _, _, _, _, _, _, p_q8, p_deq = render_case(cfg, "c1-4x64 fp8-act")
    assert p_q8 > PSNR_VS_Q8["c1"]
    assert p_deq > PSNR_VS_DEQ


# (bar against the oracle's float8 model, bar against the dequantised weights) per budget;
# measured 76.4 / 44.3, 76.6 / 44.8 and 89.6 / 58.2 dB (the oracle's own float8 model sits
# 44.3, 44.8 and 58.2 dB from the dequantised weights: one sample per interval carries a
# whole interval's optical thickness, so activation rounding weighs more)
EXTREME_BARS = {1: (71.0, 40.0), 3: (71.0, 40.0), 255: (84.0, 53.0)}


@pytest.mark.parametrize("s_max", [1, 3, 255])
def test_sample_budget_extremes(s_max):
    """One sample per ray (rays crossing several leaves clipped to their first interval), a
    budget smaller than most rays' interval counts, and the largest budget: the render
    follows the oracle's float8-activation model on the same exponents."""
    cfg = synth.scaled(synth.C1, n_hidden=2, hidden=64, width=48, height=48, s_max=s_max)
    _, _, _, _, _, _, p_q8, p_deq = render_case(cfg, "c1-2x64 fp8-act s_max %d" % s_max)
    bar_q8, bar_deq = EXTREME_BARS[s_max]
    assert p_q8 > bar_q8
    assert p_deq > bar_deq


def test_c2_render_against_oracle_models():
    _, _, _, _, _, _, p_q8, p_deq = render_case(
        synth.C2, "c2 fp8-act", lambda R: np.sort(np.random.default_rng(4).choice(R, 2000, replace=False)))
    assert p_q8 > PSNR_VS_Q8["c2"]
    assert p_deq > PSNR_VS_DEQ


@pytest.mark.parametrize("n_hidden", [1, 2, 3, 4])
def test_per_sample_outputs_against_oracle_model(n_hidden):
    cfg = synth.scaled(synth.C1, n_hidden=n_hidden, hidden=64)
    scene = Scene(cfg)
    amax = calibrated(scene)
    _, k, deq = fp8.quantise_mma(scene.W, n_hidden, 64, amax)
    ctx = am.Context(0)
    tree = am.Tree(ctx, scene.grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves, 0)
    mlp = am.Mlp(ctx, to_dev(scene.W), n_hidden, 64, am.AMNERF_FP8_ACT, tree.n_leaves, act_max_dev=to_dev(amax))
    o, d = scene.camera_rays()
    R = o.shape[1]
    am.render(ctx, tree, mlp, to_dev(o), to_dev(d), cfg.s_max)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    ns = st["n_placed_samples"]
    so = torch.empty(R + 1, dtype=torch.int32, device="cuda:0")
    z = torch.empty((ns, 4), dtype=torch.float32, device="cuda:0")
    am.amnerf_render_inspect(ctx.h, ray_smp_off=so, sample_out=z)
    torch.cuda.synchronize()
    smp_off = so.cpu().numpy().astype(np.int64)
    z = z.cpu().numpy().astype(np.float64)
    rob = oracle.robust(scene.otree, o, d)
    rng = np.random.default_rng(n_hidden)
    errs = []
    for r in rng.choice(np.where(rob)[0], 150, replace=False):
        rec = oracle.ray_samples(scene.otree, deq, n_hidden, 64, o, d, int(r), cfg.s_max, eps=0.0)
        zr = z[smp_off[r]:smp_off[r + 1]]
        assert len(zr) == len(rec["t"])
        if len(zr) == 0:
            continue
        x = o[:, r][None, :].astype(np.float64) + rec["t"][:, None] * d[:, r][None, :].astype(np.float64)
        dr = np.repeat(d[:, r][None, :].astype(np.float64), len(x), 0)
        want = np.zeros((len(x), 4))
        for leaf in np.unique(rec["slot"]):
            sel = rec["slot"] == leaf
            want[sel] = oracle.mlp_eval_q8(deq[leaf], n_hidden, 64, x[sel], dr[sel], k[leaf])
        got = np.concatenate([np.logaddexp(0, zr[:, :1]), 1 / (1 + np.exp(-zr[:, 1:]))], axis=1)
        errs.append(np.abs(got - want).max(axis=1) / np.maximum(1.0, np.abs(want).max(axis=1)))
    e = np.concatenate(errs)
    q99, worst = np.quantile(e, 0.99), e.max()
    print("fp8-act %dx64 per-sample: %d samples, median %.2e, 99%% %.2e, max %.2e" % (
        n_hidden, e.size, np.median(e), q99, worst), flush=True)
    assert e.size > 1000
    assert q99 < 2e-3 and worst < 5e-2      # measured at most 6.2e-4 and 1.0e-2


def test_backward_rejects_fp8_act():
    cfg = synth.scaled(synth.C1, n_hidden=2, hidden=64)
    scene = Scene(cfg)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_FP8_ACT)
    o, d = scene.camera_rays()
    od, dd = to_dev(o), to_dev(d)
    am.render(ctx, tree, mlp, od, dd, cfg.s_max)
    g = torch.zeros((o.shape[1], 3), dtype=torch.float32, device="cuda:0")
    grad = torch.zeros_like(mlp.master)
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render_backward(ctx.h, tree.h, mlp.desc, od, dd, g, grad)
    assert e.value.code == am.AMNERF_EINVAL


def test_unsupported_shapes_rejected():
    for nh, hid in ((2, 32), (5, 64)):
        with pytest.raises(am.AmnerfError) as e:
            am.amnerf_mlp_packed_bytes(nh, hid, am.AMNERF_FP8_ACT, 4)
        assert e.value.code == am.AMNERF_EINVAL


@pytest.mark.parametrize("mode", ["plain", "hcheck", "ess"])
def test_multi_chunk_call_equals_chunk_by_chunk_calls(mode):
    """A three-pass call (odd passes on the context's second lane) with float8 activations,
    plain, with hierarchical sampling (node MLPs) or with empty space skipped: outputs and
    sample count bit-identical to three calls on the same slices."""
    cfg = synth.scaled(synth.C1, n_hidden=4, hidden=64)
    scene = Scene(cfg, footprint=0.5 if mode == "hcheck" else 0.0)
    ctx = am.Context(0)
    tree = am.Tree(ctx, scene.grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves, 0)
    amax = np.exp(np.random.default_rng(9).uniform(0, 3, (scene.n_sets, cfg.n_hidden))).astype(np.float32)
    mlp = am.Mlp(ctx, to_dev(scene.W), cfg.n_hidden, 64, am.AMNERF_FP8_ACT, scene.n_sets, act_max_dev=to_dev(amax))
    kw = {}
    if mode == "hcheck":
        kw = {"hcheck_footprint": scene.footprint}
    elif mode == "ess":
        kw = {"occupancy": am.Occupancy(ctx, scene.grid, cfg.grid_n, 2, 0.01)}
    o, d = scene.camera_rays()
    od = to_dev(o).repeat(1, 640).contiguous()
    dd = to_dev(d).repeat(1, 640).contiguous()
    R = od.shape[1]
    chunk = (1 << 28) // 255
    assert 2 * chunk < R < 3 * chunk
    print("fp8-act multi-chunk %s: rays %d" % (mode, R), flush=True)
    whole = am.render(ctx, tree, mlp, od, dd, 255, ert_eps=cfg.ert_eps, **kw)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    assert st["n_chunks"] == 3 and st["n_nonfinite"] == 0 and st["n_unreached"] == 0
    n_samples = 0
    for r0 in range(0, R, chunk):
        part = am.render(ctx, tree, mlp, od[:, r0:r0 + chunk].contiguous(), dd[:, r0:r0 + chunk].contiguous(), 255,
                         ert_eps=cfg.ert_eps, **kw)
        torch.cuda.synchronize()
        n_samples += am.amnerf_render_stats_get(ctx.h)["n_samples"]
        for k in ("rgb", "depth", "opacity"):
            assert torch.equal(whole[k][r0:r0 + chunk], part[k]), (k, r0)
    assert st["n_samples"] == n_samples
