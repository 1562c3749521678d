"""The large uneven scene on the GPU: 256^3 grid with a 100:1 blob-density skew, 4096-leaf
tree, 4x64 leaf MLPs, S_max 192, 1920x1080 cameras -- parity on sampled rays."""
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
from test_gpu_render import check_intervals_and_sort, compare_render, fetch_inspect  # noqa: E402

S_MAX = synth.C3.s_max
# float8 activations on the 30-camera launch, against the oracle's float8 model and against
# the dequantised weights (measured 82.1 and 54.5 dB)
PSNR_FP8ACT_VS_Q8 = 76.0
PSNR_FP8ACT_VS_DEQ = 49.0
# the proposal launch against the oracle's planned render on the dequantised weights
# (measured 79.6 dB)
PSNR_PROP_LAUNCH = 74.0


@pytest.fixture(scope="module")
def scene():
    print("c3 scene set-up", flush=True)
    return Scene(synth.C3)


def test_c3_fp32_one_pass_subset(scene):
    """200 000 random pixels of camera 0 in one pass: node ids and intervals on robust rays,
    bucket offsets and the permutation bit-exact, float32 render within the float32 bar."""
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    assert tree.n_leaves == 4096
    o, d = scene.camera_rays()
    pick = np.sort(np.random.default_rng(5).choice(o.shape[1], 200_000, replace=False))
    o, d = np.ascontiguousarray(o[:, pick]), np.ascontiguousarray(d[:, pick])
    R = o.shape[1]
    print("c3 fp32 subset: rays", R, flush=True)
    out = am.render(ctx, tree, mlp, to_dev(o), to_dev(d), S_MAX, ert_eps=scene.cfg.ert_eps)
    torch.cuda.synchronize()
    st, ins = fetch_inspect(ctx, R, tree.n_leaves)
    print("c3 stats", st, flush=True)
    assert st["n_chunks"] == 1 and st["n_nonfinite"] == 0
    rays = np.sort(np.random.default_rng(6).choice(R, 1500, replace=False))
    robust = check_intervals_and_sort(scene, o, d, S_MAX, ins, rays)
    e = compare_render(scene, out, o, d, S_MAX, rays, robust)
    print("c3 fp32 max err rgb/opacity/depth", e, flush=True)
    sizes = np.diff(ins["bucket_off"].astype(np.int64))
    nz = sizes[sizes > 0]
    print("c3 bucket sizes: %d non-empty of %d, min %d, median %d, max %d" % (
        nz.size, sizes.size, nz.min(), np.median(nz), nz.max()), flush=True)
    # the skewed scene gives buckets over at least two orders of magnitude
    assert nz.max() >= 100 * nz.min()


def test_c3_fp8_full_camera_in_two_passes(scene):
    """Camera 0 whole (2 073 600 rays, two passes at S_max 192) with float8 weights, checked
    on sampled rays of both passes against the oracle on the dequantised weights."""
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_FP8)
    o, d = scene.camera_rays()
    R = o.shape[1]
    print("c3 fp8: rays", R, flush=True)
    out = am.render(ctx, tree, mlp, to_dev(o), to_dev(d), S_MAX, ert_eps=cfg.ert_eps)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    print("c3 fp8 stats", st, flush=True)
    assert st["n_chunks"] == 2 and st["n_nonfinite"] == 0
    rays = np.sort(np.random.default_rng(7).choice(R, 1500, replace=False))
    chunk = (1 << 28) // S_MAX
    assert rays.min() < chunk <= rays.max()
    _, _, deq = fp8.quantise(scene.W, cfg.n_hidden, cfg.hidden)
    rgb_q, _, _, _, _ = oracle.render(scene.otree, deq.astype(np.float32), cfg.n_hidden, cfg.hidden, o, d, S_MAX,
                                      eps=cfg.ert_eps, ray_idx=rays)
    rgb, _, _, _, _ = oracle.render(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, S_MAX,
                                    eps=cfg.ert_eps, ray_idx=rays)
    g = out["rgb"].cpu().numpy()[rays]
    p_q, p_full, p_oq = oracle.psnr(g, rgb_q), oracle.psnr(g, rgb), oracle.psnr(rgb_q, rgb)
    print("c3 fp8: psnr vs oracle(dequantised) %.2f dB, vs oracle(float32 weights) %.2f dB, "
          "quantisation alone %.2f dB" % (p_q, p_full, p_oq), flush=True)
    assert p_q > 63.0 and np.abs(g - rgb_q).max() < 1e-2   # measured 68.7 dB
    assert p_full > p_oq - 1.0


def test_c3_thirty_cameras_in_one_call(scene):
    """The benchmark's launch: 30 cameras (62.2 M rays) in one call with float8 weights, 45
    passes of at most 2^28 / S_max rays; 1 500 rays sampled across all cameras and passes
    against the oracle on the dequantised weights."""
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_FP8)
    cams = synth.make_cameras(cfg.n_cameras, cfg.seed_cameras, cfg.width, cfg.height)
    R1 = cfg.width * cfg.height
    R = R1 * len(cams)
    o_all = torch.empty((3, R), dtype=torch.float32, device="cuda:0")
    d_all = torch.empty((3, R), dtype=torch.float32, device="cuda:0")
    rng = np.random.default_rng(8)
    pick = np.sort(rng.choice(R, 1500, replace=False))
    o_pick = np.zeros((3, pick.size), np.float32)
    d_pick = np.zeros((3, pick.size), np.float32)
    for i, c in enumerate(cams):
        o, d = synth.camera_rays(c)
        o_all[:, i * R1:(i + 1) * R1] = torch.from_numpy(o).to("cuda:0")
        d_all[:, i * R1:(i + 1) * R1] = torch.from_numpy(d).to("cuda:0")
        sel = (pick >= i * R1) & (pick < (i + 1) * R1)
        o_pick[:, sel] = o[:, pick[sel] - i * R1]
        d_pick[:, sel] = d[:, pick[sel] - i * R1]
    print("c3 30 cameras: rays", R, flush=True)
    out = am.render(ctx, tree, mlp, o_all, d_all, S_MAX, ert_eps=cfg.ert_eps)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    print("c3 30 cameras stats", st, flush=True)
    assert st["n_chunks"] == -(-R // ((1 << 28) // S_MAX)) and st["n_nonfinite"] == 0
    g = out["rgb"][torch.from_numpy(pick).to("cuda:0")].cpu().numpy()
    _, _, deq = fp8.quantise(scene.W, cfg.n_hidden, cfg.hidden)
    rgb_q, _, _, _, _ = oracle.render(scene.otree, deq.astype(np.float32), cfg.n_hidden, cfg.hidden, o_pick, d_pick,
                                      S_MAX, eps=cfg.ert_eps)
    p_q = oracle.psnr(g, rgb_q)
    print("c3 30 cameras fp8: psnr vs oracle(dequantised) %.2f dB on %d rays of %d cameras" % (
        p_q, pick.size, len(np.unique(pick // R1))), flush=True)
    assert p_q > 65.0 and np.abs(g - rgb_q).max() < 1e-2   # measured 70.3 dB


def test_c3_thirty_cameras_fp8act_in_one_call(scene):
    """The benchmark's float8-activation launch: 30 cameras in one call with e4m3 weights and
    activations on the float8 matrix cores, activation exponents from the oracle's
    calibration maxima over 3 000 rays of another camera; 1 500 rays sampled across all
    cameras and passes against the oracle's float8-activation model on the same exponents,
    and against the oracle on the dequantised weights with float64 activations."""
    cfg = scene.cfg
    oc, dc = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras + 7777, cfg.width, cfg.height)[0])
    cal = np.sort(np.random.default_rng(2).choice(oc.shape[1], 3000, replace=False))
    amax = oracle.act_max(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, oc, dc, S_MAX, ray_idx=cal).astype(np.float32)
    _, k, deq = fp8.quantise_mma(scene.W, cfg.n_hidden, cfg.hidden, amax)
    ctx = am.Context(0)
    tree = am.Tree(ctx, scene.grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
    mlp = am.Mlp(ctx, to_dev(scene.W), cfg.n_hidden, cfg.hidden, am.AMNERF_FP8_ACT, tree.n_leaves,
                 act_max_dev=to_dev(amax))
    cams = synth.make_cameras(cfg.n_cameras, cfg.seed_cameras, cfg.width, cfg.height)
    R1 = cfg.width * cfg.height
    R = R1 * len(cams)
    o_all = torch.empty((3, R), dtype=torch.float32, device="cuda:0")
    d_all = torch.empty((3, R), dtype=torch.float32, device="cuda:0")
    pick = np.sort(np.random.default_rng(18).choice(R, 1500, replace=False))
    o_pick = np.zeros((3, pick.size), np.float32)
    d_pick = np.zeros((3, pick.size), np.float32)
    for i, c in enumerate(cams):
        o, d = synth.camera_rays(c)
        o_all[:, i * R1:(i + 1) * R1] = torch.from_numpy(o).to("cuda:0")
        d_all[:, i * R1:(i + 1) * R1] = torch.from_numpy(d).to("cuda:0")
        sel = (pick >= i * R1) & (pick < (i + 1) * R1)
        o_pick[:, sel] = o[:, pick[sel] - i * R1]
        d_pick[:, sel] = d[:, pick[sel] - i * R1]
    print("c3 30 cameras fp8act: rays", R, flush=True)
    out = am.render(ctx, tree, mlp, o_all, d_all, S_MAX, ert_eps=cfg.ert_eps)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    assert st["n_chunks"] == -(-R // ((1 << 28) // S_MAX)) and st["n_nonfinite"] == 0 and st["n_unreached"] == 0
    g = out["rgb"][torch.from_numpy(pick).to("cuda:0")].cpu().numpy()
    q8, _, _ = oracle.render_q8(scene.otree, deq, cfg.n_hidden, cfg.hidden, o_pick, d_pick, S_MAX, k, eps=cfg.ert_eps)
    rd, _, _, _, _ = oracle.render(scene.otree, deq, cfg.n_hidden, cfg.hidden, o_pick, d_pick, S_MAX, eps=cfg.ert_eps)
    p_q8, p_deq = oracle.psnr(g, q8), oracle.psnr(g, rd)
    print("c3 30 cameras fp8act: psnr vs oracle float8 model %.2f dB (max abs %.3e), vs dequantised weights "
          "%.2f dB on %d rays of %d cameras" % (p_q8, np.abs(g - q8).max(), p_deq, pick.size,
                                                len(np.unique(pick // R1))), flush=True)
    assert p_q8 > PSNR_FP8ACT_VS_Q8 and p_deq > PSNR_FP8ACT_VS_DEQ


def test_c3_fifty_cameras_with_proposal_in_one_call(scene):
    """The proposal workload's launch: 50 cameras (103.7 M rays) in one call with e4m3 leaf
    weights and a proposal planning most rays (untrained, mass threshold 0.5, at most 48
    samples; float32 inference so that plans are comparable with the oracle's float64 ones);
    1 500 rays sampled across all cameras and passes against the oracle's planned render on
    the dequantised weights."""
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_FP8)
    prop_w = synth.make_prop_weights(cfg.seed_proposal)
    prop = am.Proposal(ctx, torch.from_numpy(prop_w).to("cuda:0"))
    desc = prop.descriptor(am.AMNERF_F32, mass_thresh=0.5, cap=48)
    cams = synth.make_cameras(50, cfg.seed_cameras, cfg.width, cfg.height)
    R1 = cfg.width * cfg.height
    R = R1 * len(cams)
    o_all = torch.empty((3, R), dtype=torch.float32, device="cuda:0")
    d_all = torch.empty((3, R), dtype=torch.float32, device="cuda:0")
    pick = np.sort(np.random.default_rng(28).choice(R, 1500, replace=False))
    o_pick = np.zeros((3, pick.size), np.float32)
    d_pick = np.zeros((3, pick.size), np.float32)
    for i, c in enumerate(cams):
        o, d = synth.camera_rays(c)
        o_all[:, i * R1:(i + 1) * R1] = torch.from_numpy(o).to("cuda:0")
        d_all[:, i * R1:(i + 1) * R1] = torch.from_numpy(d).to("cuda:0")
        sel = (pick >= i * R1) & (pick < (i + 1) * R1)
        o_pick[:, sel] = o[:, pick[sel] - i * R1]
        d_pick[:, sel] = d[:, pick[sel] - i * R1]
    print("c3 50 cameras with proposal: rays", R, flush=True)
    rgb = torch.empty((R, 3), device="cuda:0")
    am.amnerf_render(ctx.h, tree.h, mlp.desc, o_all, d_all, S_MAX, rgb, None, None, None, cfg.ert_eps,
                     proposal=desc)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    print("c3 50 cameras with proposal stats", st, flush=True)
    assert st["n_nonfinite"] == 0 and st["n_unreached"] == 0 and st["n_chunks"] > 1
    assert st["n_samples"] < 0.8 * st["n_plain_samples"]
    g = rgb[torch.from_numpy(pick).to("cuda:0")].cpu().numpy()
    _, _, deq = fp8.quantise(scene.W, cfg.n_hidden, cfg.hidden)
    orgb, _, _, ons, opn, _, omass = oracle.render_proposal(scene.otree, deq.astype(np.float32), cfg.n_hidden,
                                                            cfg.hidden, prop_w, o_pick, d_pick, S_MAX,
                                                            eps=cfg.ert_eps, mass_thresh=0.5, cap=48)
    near = np.abs(omass - 0.5) < 1e-4          # a plan decided within float32 rounding of the cut
    p = oracle.psnr(g[~near], orgb[~near])
    print("c3 50 cameras with proposal: %d of %d sampled rays planned, psnr vs oracle(dequantised) %.2f dB "
          "(max abs %.3e)" % ((opn > 0).sum(), pick.size, p, np.abs(g[~near] - orgb[~near]).max()), flush=True)
    assert (opn > 0).sum() > 0.3 * pick.size
    assert p > PSNR_PROP_LAUNCH
