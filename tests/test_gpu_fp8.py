"""The float8 leaf-MLP path on the GPU: the packed block against the oracle's e4m3
quantiser (bit-exact), and renders against the oracle run on the dequantised weights."""
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


def block_geometry(n_hidden, hidden):
    """Bytes of the bias area and code counts per layer of one float8 leaf block, as the
    packing call documents them."""
    bias_bytes = ((n_hidden * hidden + 16) * 4 + 15) // 16 * 16
    seg = [32 * hidden] + [hidden * hidden] * (n_hidden - 1) + [16 * hidden]
    return bias_bytes, seg


@pytest.mark.parametrize("n_hidden,hidden,n_leaves", [(1, 32, 3), (2, 32, 8), (4, 64, 37), (8, 64, 5)])
def test_packed_block_matches_quantiser(n_hidden, hidden, n_leaves):
    print("fp8 pack", n_hidden, hidden, n_leaves, flush=True)
    W = synth.make_weights(n_leaves, n_hidden, hidden, 7)
    rng = np.random.default_rng(n_leaves)
    sl = fp8.layer_slices(n_hidden, hidden)
    for ow, din, dout, ob in sl:                                 # non-zero biases too
        W[:, ob:ob + dout] = rng.standard_normal((n_leaves, dout)).astype(np.float32)
    W[0, sl[1][0]:sl[1][0] + sl[1][1] * sl[1][2]] = 0.0           # one all-zero layer
    ctx = am.Context(0)
    mlp = am.Mlp(ctx, to_dev(W), n_hidden, hidden, am.AMNERF_FP8, n_leaves)
    torch.cuda.synchronize()
    blk = mlp.packed.cpu().numpy()
    bias_bytes, seg = block_geometry(n_hidden, hidden)
    per = bias_bytes + 64 + sum(seg)
    assert blk.size == per * n_leaves
    scales, codes, _ = fp8.quantise(W, n_hidden, hidden)
    for leaf in range(n_leaves):
        b = blk[leaf * per:(leaf + 1) * per]
        bias = b[:bias_bytes].view(np.float32)
        want = np.concatenate([W[leaf, ob:ob + dout] for ow, din, dout, ob in sl])
        assert np.array_equal(bias[:want.size], want)
        assert not bias[want.size:].any()
        sc = b[bias_bytes:bias_bytes + 64].view(np.float32)[:len(sl)]
        assert np.array_equal(sc, scales[leaf]), (leaf, sc, scales[leaf])
        off = bias_bytes + 64
        for li, n in enumerate(seg):
            got = np.sort(b[off:off + n])
            exp = np.sort(np.concatenate([codes[li][leaf], np.zeros(n - codes[li][leaf].size, np.uint8)]))
            assert np.array_equal(got, exp), (leaf, li, np.count_nonzero(got != exp))
            off += n


def render_vs_oracle(scene, rays_sel, seed_label):
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_FP8)
    o, d = scene.camera_rays()
    R = o.shape[1]
    print(seed_label, "rays", R, flush=True)
    out = am.render(ctx, tree, mlp, to_dev(o), to_dev(d), cfg.s_max, ert_eps=cfg.ert_eps)
    torch.cuda.synchronize()
    am.amnerf_render_stats_get(ctx.h)
    _, _, deq = fp8.quantise(scene.W, cfg.n_hidden, cfg.hidden)
    rays = np.arange(R) if rays_sel is None else rays_sel(R)
    rgb8, dep8, op8, _, _ = oracle.render(scene.otree, deq.astype(np.float32), cfg.n_hidden, cfg.hidden, o, d,
                                          cfg.s_max, eps=cfg.ert_eps, ray_idx=rays)
    rgb, _, _, _, _ = oracle.render(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max,
                                    eps=cfg.ert_eps, ray_idx=rays)
    g = out["rgb"].cpu().numpy()[rays]
    p_q = oracle.psnr(g, rgb8)
    p_full = oracle.psnr(g, rgb)
    p_oracle_q = oracle.psnr(rgb8, rgb)
    print("%s: psnr vs oracle(dequantised) %.2f dB, vs oracle(float32 weights) %.2f dB; "
          "oracle dequantised vs float32 weights %.2f dB; max abs vs dequantised %.3e"
          % (seed_label, p_q, p_full, p_oracle_q, np.abs(g - rgb8).max()), flush=True)
    assert np.abs(g - rgb8).max() < 1e-2     # measured 2.0e-3 (small frame), 2.8e-3 (800x800)
    return p_q, p_full, p_oracle_q


def test_c1_fp8_full_frame():
    p_q, p_full, p_oq = render_vs_oracle(Scene(synth.C1), None, "c1 fp8")
    # against its own weights the float8 render carries only the bfloat16 rounding of weights
    # and activations; against the float32 weights its error is the quantisation's own (the
    # oracle with dequantised weights is as far off), plus no more than 1 dB
    assert p_q > 63.0   # measured 68.6 dB
    assert p_full > p_oq - 1.0


def test_c2_fp8_sampled():
    p_q, p_full, p_oq = render_vs_oracle(
        Scene(synth.C2), lambda R: np.sort(np.random.default_rng(4).choice(R, 1500, replace=False)), "c2 fp8")
    assert p_q > 60.0   # measured 65.0 dB
    assert p_full > p_oq - 1.0


def test_backward_rejects_fp8():
    scene = Scene(synth.C1)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_FP8)
    o, d = scene.camera_rays()
    od, dd = to_dev(o), to_dev(d)
    am.render(ctx, tree, mlp, od, dd, scene.cfg.s_max)
    g = torch.zeros((o.shape[1], 3), dtype=torch.float32, device="cuda:0")
    grad = torch.zeros_like(mlp.master)
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render_backward(ctx.h, tree.h, mlp.desc, od, dd, g, grad)
    assert e.value.code == am.AMNERF_EINVAL and "bfloat16" in am.amnerf_last_error()
