"""Empty-space skipping on the GPU: the occupancy grid bit-exact against the oracle's, per-ray
kept-sample counts exact and renders within the float32 bars against the oracle run with the
same grid, an all-occupied grid bit-identical to the plain render, an all-empty one black,
and argument checks."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from scene_util import Scene, gpu_setup, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2310_01881_amd as am  # noqa: E402
from test_gpu_render import TOL_DEPTH, TOL_RGB  # noqa: E402


@pytest.mark.parametrize("cfg,block,thresh", [(synth.C1, 1, 0.0), (synth.C1, 2, 0.01), (synth.C2, 4, 0.03),
                                              (synth.C3, 2, 0.01)])
def test_occupancy_grid_matches_oracle(cfg, block, thresh):
    g = synth.make_grid(cfg)
    ctx = am.Context(0)
    occ = am.Occupancy(ctx, g, cfg.grid_n, block, thresh)
    ref = oracle.occupancy(g, cfg.grid_n, block, thresh)
    assert occ.g == cfg.grid_n // block
    assert np.array_equal(occ.cells(), ref) and occ.n_occupied == int(ref.sum())
    print("%s block %d thresh %g: %d of %d cells occupied" % (cfg.name, block, thresh, ref.sum(), ref.size))


def ess_check(scene, occ_cells, occ, o, d, rays, s_max, label):
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    R = o.shape[1]
    out = am.render(ctx, tree, mlp, to_dev(o), to_dev(d), s_max, ert_eps=cfg.ert_eps,
                    occupancy=am.Occupancy(ctx, scene.grid, cfg.grid_n, *occ), hcheck_footprint=scene.footprint)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    assert st["n_nonfinite"] == 0 and st["n_chunks"] == 1
    smp_off = torch.empty(R + 1, dtype=torch.int32, device="cuda:0")
    am.amnerf_render_inspect(ctx.h, ray_smp_off=smp_off)
    torch.cuda.synchronize()
    kept = np.diff(smp_off.cpu().numpy().astype(np.int64))[rays]
    rgb, dep, op, ns, flags = oracle.render(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, s_max,
                                            eps=cfg.ert_eps, ray_idx=rays, occupancy=occ_cells,
                                            footprint=scene.footprint)
    robust = oracle.robust(scene.otree, o, d, ray_idx=rays, footprint=scene.footprint)
    amb = (flags & (oracle.FLAG_OCC_AMBIGUOUS | oracle.FLAG_ERT_AMBIGUOUS)) != 0
    ok = robust & ~amb
    assert ok.mean() > 0.95, ok.mean()
    np.testing.assert_array_equal(kept[ok], ns[ok])
    g_rgb = out["rgb"].cpu().numpy()[rays]
    g_op = out["opacity"].cpu().numpy()[rays]
    g_dep = out["depth"].cpu().numpy()[rays]
    e = (np.abs(g_rgb - rgb)[ok].max(), np.abs(g_op - op)[ok].max(), np.abs(g_dep - dep)[ok].max())
    print("%s: kept %d of %d plain samples; %d of %d rays compared; max err rgb/opacity/depth %s" % (
        label, st["n_samples"], st["n_plain_samples"], ok.sum(), len(rays), e), flush=True)
    assert e[0] <= TOL_RGB and e[1] <= TOL_RGB and e[2] <= TOL_DEPTH
    assert st["n_samples"] < st["n_plain_samples"]
    return ctx, tree, mlp


@pytest.mark.parametrize("footprint", [0.0, 0.5])
def test_c1_full_frame_fp32(footprint):
    """The small frame in full, without and with hierarchical sampling."""
    scene = Scene(synth.C1, footprint=footprint)
    cfg = scene.cfg
    occ_cells = oracle.occupancy(scene.grid, cfg.grid_n, 2, 0.01)
    o, d = scene.camera_rays()
    ess_check(scene, occ_cells, (2, 0.01), o, d, np.arange(o.shape[1]), cfg.s_max, "c1 ess f=%g" % footprint)


def test_c1_regular_tree_fp32():
    """Empty-space skipping under the regular-subdivision tree, small frame in full."""
    scene = Scene(synth.C1, split=1)
    cfg = scene.cfg
    occ_cells = oracle.occupancy(scene.grid, cfg.grid_n, 2, 0.01)
    o, d = scene.camera_rays()
    ess_check(scene, occ_cells, (2, 0.01), o, d, np.arange(o.shape[1]), cfg.s_max, "c1 ess regular tree")


def test_c3_subset_fp32():
    """200 000 random pixels of the large scene's camera 0 (S_max 192), occupancy at half the
    guidance resolution, 1 % threshold; 1 500 rays compared."""
    scene = Scene(synth.C3)
    cfg = scene.cfg
    occ_cells = oracle.occupancy(scene.grid, cfg.grid_n, 2, 0.01)
    o, d = scene.camera_rays()
    pick = np.sort(np.random.default_rng(31).choice(o.shape[1], 200_000, replace=False))
    o, d = np.ascontiguousarray(o[:, pick]), np.ascontiguousarray(d[:, pick])
    rays = np.sort(np.random.default_rng(32).choice(o.shape[1], 1500, replace=False))
    ess_check(scene, occ_cells, (2, 0.01), o, d, rays, cfg.s_max, "c3 ess")


def test_all_occupied_is_bit_identical_to_plain():
    scene = Scene(synth.C1)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    od, dd = to_dev(o), to_dev(d)
    plain = am.render(ctx, tree, mlp, od, dd, cfg.s_max, ert_eps=cfg.ert_eps)
    full = am.Occupancy(ctx, np.ones(cfg.grid_n ** 3, np.float32), cfg.grid_n, 4, 0.5)
    assert full.n_occupied == full.g ** 3
    ess = am.render(ctx, tree, mlp, od, dd, cfg.s_max, ert_eps=cfg.ert_eps, occupancy=full)
    torch.cuda.synchronize()
    for k in ("rgb", "depth", "opacity"):
        assert torch.equal(plain[k], ess[k]), k


def test_all_empty_renders_black():
    """An occupancy grid with no occupied cell (a zero guidance grid) drops every sample: the
    plain intervals are still traversed, nothing reaches the MLP and every output is 0."""
    scene = Scene(synth.C1)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    empty = am.Occupancy(ctx, np.zeros(cfg.grid_n ** 3, np.float32), cfg.grid_n, 2, 0.0)
    assert empty.n_occupied == 0
    o, d = scene.camera_rays()
    out = am.render(ctx, tree, mlp, to_dev(o), to_dev(d), cfg.s_max, ert_eps=cfg.ert_eps, occupancy=empty)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    assert st["n_samples"] == 0 and st["n_plain_samples"] > 0 and st["n_nonfinite"] == 0
    for k in ("rgb", "depth", "opacity"):
        assert torch.count_nonzero(out[k]) == 0, k


def test_argument_checks():
    scene = Scene(synth.C1)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    occ = am.Occupancy(ctx, scene.grid, cfg.grid_n, 2, 0.01)
    o, d = scene.camera_rays()
    od, dd = to_dev(o), to_dev(d)
    rgb = torch.empty((o.shape[1], 3), device="cuda:0")
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render(ctx.h, tree.h, mlp.desc, od, dd, 64, rgb, jitter=True, occupancy=occ)
    assert e.value.code == am.AMNERF_EINVAL and "jitter" in am.amnerf_last_error()
    prop = am.Proposal(ctx, torch.from_numpy(synth.make_prop_weights(1)).to("cuda:0"))
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render(ctx.h, tree.h, mlp.desc, od, dd, 64, rgb, occupancy=occ,
                         proposal=prop.descriptor(am.AMNERF_F32, 0.99, 32))
    assert e.value.code == am.AMNERF_EINVAL and "proposal" in am.amnerf_last_error()
    for args in ((3, 0.01), (2, -0.1), (2, 1.5), (64, 0.01)):
        with pytest.raises(am.AmnerfError):
            am.Occupancy(ctx, scene.grid, cfg.grid_n, *args)


def test_c3_camera_in_two_passes_fp32():
    """Camera 0 of the large scene whole (2 073 600 rays, two passes at S_max 192) with empty
    space skipped; 1 500 rays of both passes against the oracle."""
    scene = Scene(synth.C3)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    occ_cells = oracle.occupancy(scene.grid, cfg.grid_n, 2, 0.01)
    o, d = scene.camera_rays()
    R = o.shape[1]
    out = am.render(ctx, tree, mlp, to_dev(o), to_dev(d), cfg.s_max, ert_eps=cfg.ert_eps,
                    occupancy=am.Occupancy(ctx, scene.grid, cfg.grid_n, 2, 0.01))
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    assert st["n_chunks"] == 2 and st["n_nonfinite"] == 0
    rays = np.sort(np.random.default_rng(33).choice(R, 1500, replace=False))
    chunk = (1 << 28) // cfg.s_max
    assert rays.min() < chunk <= rays.max()
    rgb, dep, op, ns, flags = oracle.render(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max,
                                            eps=cfg.ert_eps, ray_idx=rays, occupancy=occ_cells)
    robust = oracle.robust(scene.otree, o, d, ray_idx=rays)
    ok = robust & ((flags & (oracle.FLAG_OCC_AMBIGUOUS | oracle.FLAG_ERT_AMBIGUOUS)) == 0)
    assert ok.mean() > 0.95
    e = np.abs(out["rgb"].cpu().numpy()[rays] - rgb)[ok].max()
    print("c3 ess two passes: kept %d of %d samples; max rgb err %.3e on %d rays" % (
        st["n_samples"], st["n_plain_samples"], e, ok.sum()), flush=True)
    assert e <= TOL_RGB


def test_backward_after_skipping_is_rejected():
    scene = Scene(synth.C1)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_BF16)
    occ = am.Occupancy(ctx, scene.grid, cfg.grid_n, 2, 0.01)
    o, d = scene.camera_rays()
    od, dd = to_dev(o), to_dev(d)
    am.render(ctx, tree, mlp, od, dd, cfg.s_max, occupancy=occ)
    g = torch.zeros((o.shape[1], 3), dtype=torch.float32, device="cuda:0")
    grad = torch.zeros_like(mlp.master)
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render_backward(ctx.h, tree.h, mlp.desc, od, dd, g, grad)
    assert e.value.code == am.AMNERF_ESTATE and "empty space" in am.amnerf_last_error()
    # a plain render on the same context is differentiable again
    am.render(ctx, tree, mlp, od, dd, cfg.s_max)
    am.amnerf_render_backward(ctx.h, tree.h, mlp.desc, od, dd, g, grad)
    torch.cuda.synchronize()
    assert torch.count_nonzero(grad) == 0          # zero upstream gradient


@pytest.mark.parametrize("dtype", [am.AMNERF_BF16, am.AMNERF_FP8])
def test_c2_reduced_precision_error_report(dtype):
    """Leaf MLPs packed in bf16 or e4m3 with empty space skipped (the 800x800 frame, occupancy
    at half the guidance resolution, 1 % threshold), 1 500 rays against the oracle run with the
    same grid, with the plain render's bars: bf16 above 35 dB against the float32 weights;
    e4m3 above 45 dB against the dequantised weights, and within 1 dB of that oracle's own
    distance to the float32-weight render."""
    from oracle import fp8
    scene = Scene(synth.C2)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, dtype)
    occ_cells = oracle.occupancy(scene.grid, cfg.grid_n, 2, 0.01)
    o, d = scene.camera_rays()
    out = am.render(ctx, tree, mlp, to_dev(o), to_dev(d), cfg.s_max, ert_eps=cfg.ert_eps,
                    occupancy=am.Occupancy(ctx, scene.grid, cfg.grid_n, 2, 0.01))
    torch.cuda.synchronize()
    assert am.amnerf_render_stats_get(ctx.h)["n_nonfinite"] == 0
    rays = np.sort(np.random.default_rng(5).choice(o.shape[1], 1500, replace=False))

    def ref(W):
        return oracle.render(scene.otree, W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max, eps=cfg.ert_eps,
                             ray_idx=rays, occupancy=occ_cells)[0]

    g = out["rgb"].cpu().numpy()[rays]
    rgb = ref(scene.W)
    p_full = oracle.psnr(g, rgb)
    if dtype == am.AMNERF_BF16:
        print("c2 ess bf16: psnr vs oracle %.2f dB, max abs %.3e" % (p_full, np.abs(g - rgb).max()), flush=True)
        assert p_full > 59.0 and np.abs(g - rgb).max() < 1e-2   # measured 64.7 dB, 3.9e-3
    else:
        rgb8 = ref(fp8.quantise(scene.W, cfg.n_hidden, cfg.hidden)[2].astype(np.float32))
        p_q, p_oq = oracle.psnr(g, rgb8), oracle.psnr(rgb8, rgb)
        print("c2 ess e4m3: psnr vs oracle(dequantised) %.2f dB, vs oracle(float32) %.2f dB; oracle "
              "dequantised vs float32 %.2f dB" % (p_q, p_full, p_oq), flush=True)
        assert p_q > 60.0 and np.abs(g - rgb8).max() < 1e-2 and p_full > p_oq - 1.0   # measured 65.2 dB
