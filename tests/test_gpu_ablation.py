"""The regular-subdivision tree of the ablation without the adaptive split on the GPU: the
library's tree bit-exact against the oracle's, and renders through it (float32 and bf16 leaf
MLPs) against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from scene_util import Scene, gpu_setup

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2310_01881_amd as am  # noqa: E402
from test_gpu_render import check_intervals_and_sort, compare_render, fetch_inspect, render_all  # noqa: E402


def test_c1_middle_split_full_frame_fp32():
    scene = Scene(synth.C1, split=am.AMNERF_SPLIT_MIDDLE)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    ext = tree.rows[tree.rows[:, 10] >= 0][:, 5:8] - tree.rows[tree.rows[:, 10] >= 0][:, 2:5]
    assert tree.n_leaves == scene.cfg.max_leaves and np.unique(np.prod(ext, axis=1)).size == 1
    o, d = scene.camera_rays()
    R = o.shape[1]
    print("c1 middle split fp32: rays", R, flush=True)
    out = render_all(scene, ctx, tree, mlp, o, d, scene.cfg.s_max)
    st, ins = fetch_inspect(ctx, R, tree.n_leaves)
    assert st["n_nonfinite"] == 0
    rays = np.arange(R)
    robust = check_intervals_and_sort(scene, o, d, scene.cfg.s_max, ins, rays)
    e = compare_render(scene, out, o, d, scene.cfg.s_max, rays, robust)
    print("c1 middle split max err rgb/opacity/depth", e, flush=True)


def test_c2_middle_split_sampled_fp32():
    scene = Scene(synth.C2, split=am.AMNERF_SPLIT_MIDDLE)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    assert tree.n_leaves == 512
    o, d = scene.camera_rays()
    R = o.shape[1]
    print("c2 middle split fp32: rays", R, flush=True)
    out = render_all(scene, ctx, tree, mlp, o, d, scene.cfg.s_max)
    st, ins = fetch_inspect(ctx, R, tree.n_leaves)
    print("c2 middle split stats", st, flush=True)
    assert st["n_nonfinite"] == 0
    rays = np.sort(np.random.default_rng(12).choice(R, 1500, replace=False))
    robust = check_intervals_and_sort(scene, o, d, scene.cfg.s_max, ins, rays)
    e = compare_render(scene, out, o, d, scene.cfg.s_max, rays, robust)
    print("c2 middle split max err rgb/opacity/depth", e, flush=True)


def test_c2_middle_split_bf16_error_report():
    """The path the ablation times (bf16 leaf MLPs on the regular tree): 1 500 rays of the
    800x800 frame against the float64 oracle on the float32 weights, with the plain adaptive
    render's 35 dB bar."""
    import oracle
    scene = Scene(synth.C2, split=am.AMNERF_SPLIT_MIDDLE)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_BF16)
    o, d = scene.camera_rays()
    out = render_all(scene, ctx, tree, mlp, o, d, cfg.s_max)
    assert am.amnerf_render_stats_get(ctx.h)["n_nonfinite"] == 0
    rays = np.sort(np.random.default_rng(13).choice(o.shape[1], 1500, replace=False))
    rgb = oracle.render(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max, eps=cfg.ert_eps,
                        ray_idx=rays)[0]
    g = out["rgb"].cpu().numpy()[rays]
    psnr = oracle.psnr(g, rgb)
    print("c2 middle split bf16: psnr vs oracle %.2f dB, max abs %.3e" % (psnr, np.abs(g - rgb).max()), flush=True)
    assert psnr > 60.0 and np.abs(g - rgb).max() < 1e-2   # measured 65.7 dB, 2.6e-3


def test_split_mode_is_validated():
    ctx = am.Context(0)
    cfg = synth.C1
    grid = synth.make_grid(cfg)
    with pytest.raises(am.AmnerfError) as e:
        am.Tree(ctx, grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves, 2)
    assert e.value.code == am.AMNERF_EINVAL
