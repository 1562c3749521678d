"""Hierarchical sampling (Section 3.5, HCheck) on the GPU: intervals keyed by node slot,
samples, sort and renders against the oracle run with the same footprint; the two limits of
the footprint (the root stops every ray; no node stops any); the backward through node MLPs
against the oracle's gradient; argument checks."""
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
from test_gpu_render import check_intervals_and_sort, compare_render, fetch_inspect, render_all  # noqa: E402


def run_and_check(scene, rays_sel, label, s_max=None):
    cfg = scene.cfg
    s_max = s_max or cfg.s_max
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    assert mlp.n_leaves == tree.info.n_nodes
    o, d = scene.camera_rays()
    R = o.shape[1]
    print(label, "rays", R, "footprint", scene.footprint, flush=True)
    out = render_all(scene, ctx, tree, mlp, o, d, s_max)
    st, ins = fetch_inspect(ctx, R, scene.n_sets)
    assert st["n_nonfinite"] == 0
    rays = np.arange(R) if rays_sel is None else rays_sel(R)
    robust = check_intervals_and_sort(scene, o, d, s_max, ins, rays)
    e = compare_render(scene, out, o, d, s_max, rays, robust)
    # the same rays without hierarchical sampling: more intervals and samples
    leaf_iv = oracle.trace(scene.otree, o, d, ray_idx=rays)[3]
    hs_iv = np.diff(ins["ray_iv_off"].astype(np.int64))[rays]
    off = ins["ray_iv_off"].astype(np.int64)
    on_rays = np.concatenate([np.arange(off[r], off[r + 1]) for r in rays])
    inner = np.isin(ins["iv_slot"][on_rays], scene.otree.rows[scene.otree.rows[:, 8] >= 0][:, 11])
    print("%s: max err rgb/opacity/depth %s; intervals %d (leaves only %d), %d on inner nodes; samples %d"
          % (label, e, hs_iv.sum(), np.minimum(leaf_iv, s_max).sum(), inner.sum(), st["n_samples"]), flush=True)
    assert inner.sum() > 0 and hs_iv.sum() < np.minimum(leaf_iv, s_max).sum()
    return ctx, tree, mlp


def test_c1_hcheck_full_frame_fp32():
    run_and_check(Scene(synth.C1, footprint=0.5), None, "c1 hcheck")


def test_c1_hcheck_on_the_regular_tree_fp32():
    """Hierarchical sampling over the regular-subdivision tree: its node slots, stopping
    distances and node MLPs, small frame in full."""
    run_and_check(Scene(synth.C1, split=1, footprint=0.5), None, "c1 hcheck regular tree")


@pytest.mark.parametrize("footprint", [0.1, 0.25])
def test_c2_hcheck_sampled_fp32(footprint):
    run_and_check(Scene(synth.C2, footprint=footprint),
                  lambda R: np.sort(np.random.default_rng(21).choice(R, 1500, replace=False)),
                  "c2 hcheck %g" % footprint)


def test_hcheck_node_table_in_memory():
    """A tree of more than 2048 nodes: the node table and stopping distances are read from
    memory instead of LDS."""
    cfg = synth.scaled(synth.C2, grid_n=64, max_depth=12, max_leaves=2048, n_hidden=2, hidden=32,
                       width=64, height=64, s_max=96)
    scene = Scene(cfg, footprint=0.2)
    assert scene.otree.n_nodes > 2048
    run_and_check(scene, None, "2048-leaf hcheck")


def bf16_weights(W, n_hidden, hidden):
    """The weights (not the biases) rounded to bfloat16, nearest even, kept as float32."""
    Wb = np.array(W, np.float32, copy=True)
    for ow, din, dout, ob in fp8.layer_slices(n_hidden, hidden):
        u = Wb[:, ow:ow + din * dout].view(np.uint32)
        u[:] = (u + np.uint32(0x7FFF) + ((u >> 16) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return Wb


def test_hcheck_backward_matches_oracle_gradient():
    cfg = synth.scaled(synth.C2, grid_n=64, max_leaves=64, max_depth=12)
    scene = Scene(cfg, footprint=0.25)
    ctx = am.Context(0)
    tree = am.Tree(ctx, scene.grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
    assert np.array_equal(tree.rows, scene.otree.rows)
    tr = am.Trainer(ctx, tree, torch.from_numpy(scene.W).to("cuda:0"), cfg.n_hidden, cfg.hidden, n_sets=scene.n_sets)
    o, d = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras, 16, 16)[0])
    R = o.shape[1]
    rng = np.random.default_rng(8)
    g_rgb = (rng.standard_normal((R, 3)) / R).astype(np.float32)
    od, dd = to_dev(o), to_dev(d)
    rgb = torch.empty((R, 3), device="cuda:0")
    am.amnerf_render(ctx.h, tree.h, tr.mlp, od, dd, cfg.s_max, rgb, None, None, None, 1e-4,
                     hcheck_footprint=scene.footprint)
    grad = torch.empty_like(tr.master)
    am.amnerf_render_backward(ctx.h, tree.h, tr.mlp, od, dd, to_dev(g_rgb), grad)
    torch.cuda.synchronize()
    g_gpu = grad.cpu().numpy().astype(np.float64)
    # the kernel runs on the bfloat16 rounding of the weights (rounding them alone moves the
    # oracle's gradient by about 2e-2 relative on this scene), so the oracle is run on those
    # weights; what remains is the bfloat16 rounding of activations and gradients
    Wb = bf16_weights(scene.W, cfg.n_hidden, cfg.hidden)
    g_ref = oracle.render_grad(scene.otree, Wb, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max,
                               g_rgb.astype(np.float64), eps=1e-4, footprint=scene.footprint)
    g_f32 = oracle.render_grad(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max,
                               g_rgb.astype(np.float64), eps=1e-4, footprint=scene.footprint)
    e = float(np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref))
    e32 = float(np.linalg.norm(g_gpu - g_f32) / np.linalg.norm(g_f32))
    inner = scene.otree.rows[scene.otree.rows[:, 8] >= 0][:, 11]
    print("hcheck backward: relative L2 %.3e against the oracle on the bf16 weights, %.3e on the float32 "
          "weights; inner-node gradient norm %.3e" % (e, e32, np.linalg.norm(g_ref[inner])), flush=True)
    assert np.linalg.norm(g_ref[inner]) > 0
    assert np.isfinite(g_gpu).all() and e <= 2e-2
    hit = np.abs(g_ref).sum(axis=1) > 0
    assert np.all(g_gpu[~hit] == 0)


def test_hcheck_backward_f32_matches_oracle_gradient():
    """float32 node MLPs: the whole gradient, inner-node MLPs included, within 1e-4 relative
    L2 of the oracle's analytic gradient (pinned by central differences under hierarchical
    sampling with early termination on)."""
    cfg = synth.scaled(synth.C2, grid_n=64, max_leaves=64, max_depth=12)
    scene = Scene(cfg, footprint=0.25)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras, 16, 16)[0])
    R = o.shape[1]
    rng = np.random.default_rng(8)
    g_rgb = (rng.standard_normal((R, 3)) / R).astype(np.float32)
    od, dd = to_dev(o), to_dev(d)
    rgb = torch.empty((R, 3), device="cuda:0")
    am.amnerf_render(ctx.h, tree.h, mlp.desc, od, dd, cfg.s_max, rgb, None, None, None, 1e-4,
                     hcheck_footprint=scene.footprint)
    grad = torch.empty_like(mlp.master)
    am.amnerf_render_backward(ctx.h, tree.h, mlp.desc, od, dd, to_dev(g_rgb), grad)
    torch.cuda.synchronize()
    am.amnerf_render_stats_get(ctx.h)
    g_gpu = grad.cpu().numpy().astype(np.float64)
    g_ref = oracle.render_grad(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max,
                               g_rgb.astype(np.float64), eps=1e-4, footprint=scene.footprint)
    e = float(np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref))
    print("hcheck f32 backward: relative L2 %.3e" % e, flush=True)
    inner = scene.otree.rows[scene.otree.rows[:, 8] >= 0][:, 11]
    assert np.linalg.norm(g_ref[inner]) > 0
    assert np.isfinite(g_gpu).all() and e <= 1e-4


def test_hcheck_argument_checks():
    scene = Scene(synth.C1, footprint=0.5)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    od, dd = to_dev(o), to_dev(d)
    rgb = torch.empty((o.shape[1], 3), device="cuda:0")
    for f in (-1.0, float("inf"), float("nan")):
        with pytest.raises(am.AmnerfError) as e:
            am.amnerf_render(ctx.h, tree.h, mlp.desc, od, dd, 64, rgb, hcheck_footprint=f)
        assert e.value.code == am.AMNERF_EINVAL
    # a leaf-count MLP with hierarchical sampling, a node-count MLP without
    leaf = am.Mlp(ctx, torch.from_numpy(scene.W[:tree.n_leaves].copy()).to("cuda:0"), 2, 32, am.AMNERF_F32,
                  tree.n_leaves)
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render(ctx.h, tree.h, leaf.desc, od, dd, 64, rgb, hcheck_footprint=0.5)
    assert e.value.code == am.AMNERF_EINVAL and "per node" in am.amnerf_last_error()
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render(ctx.h, tree.h, mlp.desc, od, dd, 64, rgb)
    assert e.value.code == am.AMNERF_EINVAL
    # not combined with a proposal
    prop = am.Proposal(ctx, torch.from_numpy(synth.make_prop_weights(1)).to("cuda:0"))
    desc = prop.descriptor(am.AMNERF_F32, mass_thresh=0.99, cap=32)
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render(ctx.h, tree.h, mlp.desc, od, dd, 64, rgb, proposal=desc, hcheck_footprint=0.5)
    assert e.value.code == am.AMNERF_EINVAL and "proposal" in am.amnerf_last_error()


def test_hcheck_with_jitter():
    """Jittered strata under hierarchical sampling: the offset of interval k of a ray is the
    same counter-based hash, k counting the ray's HCheck intervals."""
    scene = Scene(synth.C1, footprint=0.5)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    R = o.shape[1]
    out = render_all(scene, ctx, tree, mlp, o, d, cfg.s_max, jitter=True, seed=1234)
    rays = np.arange(R)
    robust = oracle.robust(scene.otree, o, d, footprint=scene.footprint)
    e = compare_render(scene, out, o, d, cfg.s_max, rays, robust, jitter=True, seed=1234)
    print("c1 hcheck jitter: max err rgb/opacity/depth", e, flush=True)


def test_hcheck_node_count_capacity():
    """A 4096-leaf tree has 8191 nodes, more MLP sets than a render supports: ECAPACITY."""
    cfg = synth.scaled(synth.C2, grid_n=64, max_depth=12, max_leaves=4096, n_hidden=2, hidden=32,
                       width=8, height=8, s_max=32)
    g = synth.make_grid(cfg)
    ctx = am.Context(0)
    tree = am.Tree(ctx, g, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
    assert tree.info.n_nodes > 4096
    W = synth.make_weights(4096, 2, 32, 1)
    mlp = am.Mlp(ctx, torch.from_numpy(W).to("cuda:0"), 2, 32, am.AMNERF_F32, 4096)
    o, d = synth.camera_rays(synth.make_cameras(1, 3, 8, 8)[0])
    rgb = torch.empty((o.shape[1], 3), device="cuda:0")
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render(ctx.h, tree.h, mlp.desc, to_dev(o), to_dev(d), 32, rgb, hcheck_footprint=0.1)
    assert e.value.code == am.AMNERF_ECAPACITY


def test_hcheck_root_only_fp32():
    """A footprint so large that the root stops every ray (the cameras are outside the box, so
    every ray enters it at t > 0): one interval per hit ray, keyed by the root's slot 0, every
    sample in the root's bucket; renders against the oracle."""
    scene = Scene(synth.C1, footprint=1e30)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    R = o.shape[1]
    out = render_all(scene, ctx, tree, mlp, o, d, cfg.s_max)
    st, ins = fetch_inspect(ctx, R, scene.n_sets)
    assert st["n_nonfinite"] == 0
    m = np.diff(ins["ray_iv_off"].astype(np.int64))
    assert m.max() == 1 and st["n_intervals"] == np.count_nonzero(m) > 0
    assert np.all(ins["iv_slot"] == 0)
    assert ins["bucket_off"][1] == st["n_samples"] and np.all(ins["bucket_off"][1:] == st["n_samples"])
    rays = np.arange(R)
    robust = check_intervals_and_sort(scene, o, d, cfg.s_max, ins, rays)
    e = compare_render(scene, out, o, d, cfg.s_max, rays, robust)
    print("root only: %d intervals, %d samples, max err rgb/opacity/depth %s" % (
        st["n_intervals"], st["n_samples"], e), flush=True)


def test_hcheck_tiny_footprint_is_the_leaf_render():
    """A footprint so small that no node stops the descent: the intervals are the leaf
    intervals keyed by the leaves' node slots with the plain sample counts, so the render with
    node MLPs equals, bit for bit, the plain render whose leaf MLPs are those leaves' node
    MLPs."""
    scene = Scene(synth.C1, footprint=1e-30)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    od, dd = to_dev(o), to_dev(d)
    hs = am.render(ctx, tree, mlp, od, dd, cfg.s_max, ert_eps=cfg.ert_eps, hcheck_footprint=scene.footprint)
    torch.cuda.synchronize()
    n_hs = am.amnerf_render_stats_get(ctx.h)["n_samples"]
    rows = scene.otree.rows
    leaves = rows[rows[:, 10] >= 0]
    l2n = np.empty(tree.n_leaves, np.int64)
    l2n[leaves[:, 10]] = leaves[:, 11]
    leaf_w = torch.from_numpy(np.ascontiguousarray(scene.W[l2n])).to("cuda:0")
    leaf_mlp = am.Mlp(ctx, leaf_w, cfg.n_hidden, cfg.hidden, am.AMNERF_F32, tree.n_leaves)
    plain = am.render(ctx, tree, leaf_mlp, od, dd, cfg.s_max, ert_eps=cfg.ert_eps)
    torch.cuda.synchronize()
    assert am.amnerf_render_stats_get(ctx.h)["n_samples"] == n_hs > 0
    for k in ("rgb", "depth", "opacity"):
        assert torch.equal(hs[k], plain[k]), k


@pytest.mark.parametrize("dtype", [am.AMNERF_BF16, am.AMNERF_FP8])
def test_c2_hcheck_reduced_precision_error_report(dtype):
    """Node MLPs packed in bf16 or e4m3 under HCheck (f = 0.25, the 800x800 frame), 1 500 rays,
    with the plain leaf render's bars: bf16 above 35 dB against the float64 oracle on the
    float32 node weights; e4m3 above 45 dB against the oracle on the dequantised weights, and
    within 1 dB of that oracle's own distance to the float32-weight render."""
    scene = Scene(synth.C2, footprint=0.25)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, dtype)
    o, d = scene.camera_rays()
    out = render_all(scene, ctx, tree, mlp, o, d, cfg.s_max)
    assert am.amnerf_render_stats_get(ctx.h)["n_nonfinite"] == 0
    rays = np.sort(np.random.default_rng(4).choice(o.shape[1], 1500, replace=False))

    def ref(W):
        return oracle.render(scene.otree, W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max, eps=cfg.ert_eps,
                             ray_idx=rays, footprint=scene.footprint)[0]

    g = out["rgb"].cpu().numpy()[rays]
    rgb = ref(scene.W)
    p_full = oracle.psnr(g, rgb)
    if dtype == am.AMNERF_BF16:
        print("c2 hcheck bf16: psnr vs oracle %.2f dB, max abs %.3e" % (p_full, np.abs(g - rgb).max()), flush=True)
        assert p_full > 59.0 and np.abs(g - rgb).max() < 1e-2   # measured 64.1 dB, 3.7e-3
    else:
        rgb8 = ref(fp8.quantise(scene.W, cfg.n_hidden, cfg.hidden)[2].astype(np.float32))
        p_q, p_oq = oracle.psnr(g, rgb8), oracle.psnr(rgb8, rgb)
        print("c2 hcheck e4m3: psnr vs oracle(dequantised) %.2f dB, vs oracle(float32) %.2f dB; oracle "
              "dequantised vs float32 %.2f dB" % (p_q, p_full, p_oq), flush=True)
        assert p_q > 59.0 and np.abs(g - rgb8).max() < 1e-2 and p_full > p_oq - 1.0   # measured 64.7 dB
