"""Parity of the HIP rendering path (through the C ABI) with the FP64 oracle."""
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

# Tolerances (float32 path vs float64 oracle): rgb, opacity and depth 1e-5 absolute (depth
# sums w t with t up to ~3.5; measured errors are below 1e-6).
TOL_RGB = 1e-5
TOL_DEPTH = 1e-5


def inspect(ctx, R):
    st = am.amnerf_render_stats_get(ctx.h)
    niv, ns = st["n_intervals"], st["n_placed_samples"]
    L = None
    dev = "cuda:0"
    b = {
        "ray_iv_off": torch.empty(R + 1, dtype=torch.int32, device=dev),
        "ray_smp_off": torch.empty(R + 1, dtype=torch.int32, device=dev),
        "iv_t0": torch.empty(max(niv, 1), dtype=torch.float32, device=dev),
        "iv_dt": torch.empty(max(niv, 1), dtype=torch.float32, device=dev),
        "iv_slot": torch.empty(max(niv, 1), dtype=torch.int32, device=dev),
        "iv_n": torch.empty(max(niv, 1), dtype=torch.int32, device=dev),
        "perm": torch.empty(max(ns, 1), dtype=torch.int32, device=dev),
        "sample_out": torch.empty((max(ns, 1), 4), dtype=torch.float32, device=dev),
        "ray_used": torch.empty(max(R, 1), dtype=torch.int32, device=dev),
    }
    return st, b


def fetch_inspect(ctx, R, n_leaves):
    st, b = inspect(ctx, R)
    b["bucket_off"] = torch.empty(n_leaves + 1, dtype=torch.int32, device="cuda:0")
    am.amnerf_render_inspect(ctx.h, **b)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in b.items()}
    niv, ns = st["n_intervals"], st["n_placed_samples"]
    for k in ("iv_t0", "iv_dt", "iv_slot", "iv_n"):
        out[k] = out[k][:niv]
    out["perm"] = out["perm"][:ns].view(np.uint32)
    out["sample_out"] = out["sample_out"][:ns]
    out["ray_used"] = out["ray_used"][:R]
    return st, out


def check_intervals_and_sort(scene, o, d, s_max, ins, rays_to_check, max_nonrobust=0.01):
    """Node ids bit-exact on robust rays; perm and bucket offsets bit-exact everywhere."""
    R = o.shape[1]
    f = getattr(scene, "footprint", 0.0)
    t0, t1, slot, m = oracle.trace(scene.otree, o, d, ray_idx=rays_to_check, footprint=f)
    m_leaf = oracle.trace(scene.otree, o, d, ray_idx=rays_to_check)[3] if f > 0 else m
    robust = oracle.robust(scene.otree, o, d, ray_idx=rays_to_check, footprint=f)
    off = ins["ray_iv_off"].astype(np.int64)
    n_nonrobust = 0
    for q, r in enumerate(rays_to_check):
        a, b = off[r], off[r + 1]
        meff = min(m[q], s_max)
        if not robust[q]:
            n_nonrobust += 1
            continue
        assert b - a == meff, (r, b - a, meff)
        np.testing.assert_array_equal(ins["iv_slot"][a:b], slot[q, :meff])
        np.testing.assert_allclose(ins["iv_t0"][a:b], t0[q, :meff], rtol=0, atol=2e-6)
        np.testing.assert_allclose(ins["iv_dt"][a:b], (t1 - t0)[q, :meff], rtol=1e-6, atol=1e-7)
        if meff:
            n = s_max // m_leaf[q] if m_leaf[q] <= s_max else 1
            assert np.all(ins["iv_n"][a:b] == n)
    assert n_nonrobust <= max(2, max_nonrobust * len(rays_to_check))
    # the sort: ray-major sample keys expanded from intervals, stably sorted
    keys = np.repeat(ins["iv_slot"], ins["iv_n"])
    counts, offsets, perm = oracle.buckets(keys, scene.n_sets)
    np.testing.assert_array_equal(ins["bucket_off"].view(np.uint32), offsets)
    np.testing.assert_array_equal(ins["perm"], perm)
    smp_off = ins["ray_smp_off"].astype(np.int64)
    assert smp_off[R] == len(keys)
    return robust


def compare_render(scene, out, o, d, s_max, rays_to_check, robust, tol_rgb=TOL_RGB, tol_depth=TOL_DEPTH,
                   jitter=False, seed=0, min_ok=0.98):
    cfg = scene.cfg
    rgb, dep, op, ns, flags = oracle.render(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, s_max,
                                            eps=cfg.ert_eps, ray_idx=rays_to_check, jitter=jitter, seed=seed,
                                            footprint=getattr(scene, "footprint", 0.0))
    g_rgb = out["rgb"].cpu().numpy()[rays_to_check]
    g_dep = out["depth"].cpu().numpy()[rays_to_check]
    g_op = out["opacity"].cpu().numpy()[rays_to_check]
    ok = robust & ((flags & oracle.FLAG_ERT_AMBIGUOUS) == 0)
    assert ok.mean() > min_ok
    e_rgb = np.abs(g_rgb - rgb)[ok].max()
    e_op = np.abs(g_op - op)[ok].max()
    e_dep = np.abs(g_dep - dep)[ok].max()
    assert e_rgb <= tol_rgb, e_rgb
    assert e_op <= tol_rgb, e_op
    assert e_dep <= tol_depth, e_dep
    return e_rgb, e_op, e_dep


def render_all(scene, ctx, tree, mlp, o, d, s_max, **kw):
    od, dd = to_dev(o), to_dev(d)
    out = am.render(ctx, tree, mlp, od, dd, s_max, ert_eps=scene.cfg.ert_eps,
                    hcheck_footprint=getattr(scene, "footprint", 0.0), **kw)
    torch.cuda.synchronize()
    am.amnerf_render_stats_get(ctx.h)    # checks that no interval entry was left unreached
    return out


def test_c1_fp32_parity_full_frame():
    scene = Scene(synth.C1)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    R = o.shape[1]
    print("c1 fp32: rays", R, flush=True)
    out = render_all(scene, ctx, tree, mlp, o, d, scene.cfg.s_max)
    st, ins = fetch_inspect(ctx, R, tree.n_leaves)
    assert st["n_nonfinite"] == 0
    rays = np.arange(R)
    robust = check_intervals_and_sort(scene, o, d, scene.cfg.s_max, ins, rays)
    e = compare_render(scene, out, o, d, scene.cfg.s_max, rays, robust)
    print("c1 fp32 max err rgb/opacity/depth", e)


def test_c1_per_sample_mlp_outputs():
    """sigma and rgb of every sample (ray-major) against the oracle's per-sample record."""
    scene = Scene(synth.C1)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    R = o.shape[1]
    render_all(scene, ctx, tree, mlp, o, d, scene.cfg.s_max)
    st, ins = fetch_inspect(ctx, R, tree.n_leaves)
    smp_off = ins["ray_smp_off"].astype(np.int64)
    rng = np.random.default_rng(0)
    for r in rng.choice(R, 200, replace=False):
        rec = oracle.ray_samples(scene.otree, scene.W, 2, 32, o, d, r, scene.cfg.s_max, eps=0.0)
        z = ins["sample_out"][smp_off[r]:smp_off[r + 1]].astype(np.float64)
        g = np.concatenate([np.logaddexp(0, z[:, :1]), 1 / (1 + np.exp(-z[:, 1:]))], axis=1)
        assert len(g) == len(rec["t"])
        if len(g) == 0:
            continue
        # float32 sample positions are within ~1 ulp(t) ~ 2.4e-7 of the oracle's; the highest
        # encoding frequency (8 pi on p = 2x - 1) turns that into ~1e-5 on pre-activations
        np.testing.assert_allclose(g[:, 0], rec["sigma"], rtol=2e-5, atol=2e-5)
        np.testing.assert_allclose(g[:, 1:], rec["rgb"], rtol=0, atol=1e-5)


def test_determinism_bit_identical():
    scene = Scene(synth.C1)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    a = render_all(scene, ctx, tree, mlp, o, d, 64)
    b = render_all(scene, ctx, tree, mlp, o, d, 64)
    for k in ("rgb", "depth", "opacity"):
        assert torch.equal(a[k], b[k])


@pytest.mark.parametrize("s_max", [1, 3, 17, 255])
def test_sample_budgets_and_clipping(s_max):
    scene = Scene(synth.scaled(synth.C1, max_depth=6, max_leaves=40))
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = synth.random_rays(3000, 11)
    R = o.shape[1]
    out = render_all(scene, ctx, tree, mlp, o, d, s_max)
    st, ins = fetch_inspect(ctx, R, tree.n_leaves)
    rays = np.arange(R)
    robust = check_intervals_and_sort(scene, o, d, s_max, ins, rays)
    compare_render(scene, out, o, d, s_max, rays, robust)


def test_jittered_strata_match_oracle():
    scene = Scene(synth.C1)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    R = o.shape[1]
    out = render_all(scene, ctx, tree, mlp, o, d, 64, jitter=True, seed=1234567)
    st, ins = fetch_inspect(ctx, R, tree.n_leaves)
    robust = oracle.robust(scene.otree, o, d)
    compare_render(scene, out, o, d, 64, np.arange(R), robust, jitter=True, seed=1234567)


def test_empty_and_missing_rays():
    scene = Scene(synth.C1)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    # zero rays
    o = np.zeros((3, 0), np.float32)
    out = render_all(scene, ctx, tree, mlp, o, o, 64)
    assert out["rgb"].shape == (0, 3)
    # rays that all miss the box: zero samples, zero outputs
    o = np.tile(np.array([[3.0], [3.0], [3.0]], np.float32), (1, 300))
    d = np.tile(np.array([[1.0], [0.0], [0.0]], np.float32), (1, 300))
    out = render_all(scene, ctx, tree, mlp, o, d, 64)
    assert am.amnerf_render_stats_get(ctx.h)["n_samples"] == 0
    assert torch.count_nonzero(out["rgb"]) == 0 and torch.count_nonzero(out["opacity"]) == 0


def test_single_leaf_and_max_leaves_trees():
    for cfg in (synth.scaled(synth.C1, max_depth=0, max_leaves=1),
                synth.scaled(synth.C2, grid_n=64, max_depth=12, max_leaves=4096, n_hidden=2, hidden=32,
                             width=48, height=48, s_max=96)):
        scene = Scene(cfg)
        ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
        assert tree.n_leaves == cfg.max_leaves
        o, d = scene.camera_rays()
        R = o.shape[1]
        out = render_all(scene, ctx, tree, mlp, o, d, cfg.s_max)
        st, ins = fetch_inspect(ctx, R, tree.n_leaves)
        rays = np.arange(R)
        robust = check_intervals_and_sort(scene, o, d, cfg.s_max, ins, rays)
        compare_render(scene, out, o, d, cfg.s_max, rays, robust)


def test_c2_full_size_sampled_parity_fp32():
    """800x800, 512 leaves, 4x64 MLPs, S_max 128: the bench workload, checked on sampled rays."""
    scene = Scene(synth.C2)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    R = o.shape[1]
    print("c2 fp32: rays", R, flush=True)
    out = render_all(scene, ctx, tree, mlp, o, d, 128)
    st, ins = fetch_inspect(ctx, R, tree.n_leaves)
    print("c2 stats", st, flush=True)
    assert st["n_nonfinite"] == 0
    rng = np.random.default_rng(2)
    rays = np.sort(rng.choice(R, 1500, replace=False))
    robust = check_intervals_and_sort(scene, o, d, 128, ins, rays)
    e = compare_render(scene, out, o, d, 128, rays, robust)
    print("c2 fp32 max err rgb/opacity/depth", e)


def test_c2_bf16_error_report():
    scene = Scene(synth.C2)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_BF16)
    o, d = scene.camera_rays()
    R = o.shape[1]
    out = render_all(scene, ctx, tree, mlp, o, d, 128)
    rng = np.random.default_rng(3)
    rays = np.sort(rng.choice(R, 1500, replace=False))
    rgb, dep, op, ns, flags = oracle.render(scene.otree, scene.W, 4, 64, o, d, 128, eps=1e-4, ray_idx=rays)
    g = out["rgb"].cpu().numpy()[rays]
    psnr = oracle.psnr(g, rgb)
    print("c2 bf16 psnr vs oracle %.2f dB, max abs %.3e" % (psnr, np.abs(g - rgb).max()))
    assert psnr > 59.0 and np.abs(g - rgb).max() < 1e-2   # measured 64.4 dB, 4.6e-3


@pytest.mark.parametrize("n_hidden,hidden", [(1, 32), (3, 64), (5, 32), (8, 64)])
def test_mlp_shapes(n_hidden, hidden):
    """Every hidden-layer count the kernels unroll differently (none, odd, even, the maximum):
    float32 per-sample outputs against the oracle's per-sample record, and the bf16 and e4m3
    renders against the oracle (the latter on its dequantised weights)."""
    from oracle import fp8
    cfg = synth.scaled(synth.C1, n_hidden=n_hidden, hidden=hidden)
    scene = Scene(cfg)
    o, d = scene.camera_rays()
    R = o.shape[1]
    print("mlp shape %dx%d" % (n_hidden, hidden), flush=True)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    render_all(scene, ctx, tree, mlp, o, d, cfg.s_max)
    st, ins = fetch_inspect(ctx, R, tree.n_leaves)
    smp_off = ins["ray_smp_off"].astype(np.int64)
    rng = np.random.default_rng(n_hidden)
    for r in rng.choice(R, 60, replace=False):
        rec = oracle.ray_samples(scene.otree, scene.W, n_hidden, hidden, o, d, r, cfg.s_max, eps=0.0)
        z = ins["sample_out"][smp_off[r]:smp_off[r + 1]].astype(np.float64)
        assert len(z) == len(rec["t"])
        if len(z) == 0:
            continue
        g = np.concatenate([np.logaddexp(0, z[:, :1]), 1 / (1 + np.exp(-z[:, 1:]))], axis=1)
        np.testing.assert_allclose(g[:, 0], rec["sigma"], rtol=2e-5, atol=2e-5)
        np.testing.assert_allclose(g[:, 1:], rec["rgb"], rtol=0, atol=1e-5)
    rays = np.sort(rng.choice(R, 800, replace=False))
    ref, _, _, _, _ = oracle.render(scene.otree, scene.W, n_hidden, hidden, o, d, cfg.s_max, eps=1e-4, ray_idx=rays)
    _, _, deq = fp8.quantise(scene.W, n_hidden, hidden)
    ref8, _, _, _, _ = oracle.render(scene.otree, deq.astype(np.float32), n_hidden, hidden, o, d, cfg.s_max,
                                     eps=1e-4, ray_idx=rays)
    for dtype, want in ((am.AMNERF_BF16, ref), (am.AMNERF_FP8, ref8)):
        m2 = am.Mlp(ctx, mlp.master, n_hidden, hidden, dtype, tree.n_leaves)
        out = render_all(scene, ctx, tree, m2, o, d, cfg.s_max)
        psnr = oracle.psnr(out["rgb"].cpu().numpy()[rays], want)
        print("  dtype %d: psnr %.2f dB" % (dtype, psnr), flush=True)
        assert psnr > 57.0   # measured 62.6-68.7 dB


def test_axis_parallel_and_inside_rays():
    """Rays along the axes (zero direction components), from outside and from inside the box,
    some on cell planes: intervals, sort and float32 render against the oracle."""
    scene = Scene(synth.scaled(synth.C1, max_depth=6, max_leaves=40))
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    rng = np.random.default_rng(21)
    os_, ds_ = [], []
    for a in range(3):
        for sgn in (1.0, -1.0):
            for inside in (False, True):
                n = 200
                o = rng.uniform(0.02, 0.98, (3, n))
                if not inside:
                    o[a] = -0.5 if sgn > 0 else 1.5
                if inside:
                    o[:, :20] = np.round(o[:, :20] * 32) / 32      # on cell planes
                d = np.zeros((3, n))
                d[a] = sgn
                os_.append(o)
                ds_.append(d)
    o = np.ascontiguousarray(np.concatenate(os_, axis=1).astype(np.float32))
    d = np.ascontiguousarray(np.concatenate(ds_, axis=1).astype(np.float32))
    R = o.shape[1]
    out = render_all(scene, ctx, tree, mlp, o, d, 64)
    st, ins = fetch_inspect(ctx, R, tree.n_leaves)
    rays = np.arange(R)
    # a tenth of the rays start on cell planes, so a few percent graze a split
    robust = check_intervals_and_sort(scene, o, d, 64, ins, rays, max_nonrobust=0.05)
    print("axis-parallel rays: %d, robust %d, samples %d" % (R, robust.sum(), st["n_samples"]))
    assert st["n_samples"] > 0
    compare_render(scene, out, o, d, 64, rays, robust, min_ok=0.9)


def test_multi_chunk_call_equals_chunk_by_chunk_calls():
    """A call over 2.6 M rays at S_max 255 runs in three passes (odd passes on the second
    lane); its outputs and sample count are bit-identical to three calls on the same slices."""
    scene = Scene(synth.C1)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    reps = 640
    od = to_dev(o).repeat(1, reps).contiguous()
    dd = to_dev(d).repeat(1, reps).contiguous()
    R = od.shape[1]
    chunk = (1 << 28) // 255
    assert 2 * chunk < R < 3 * chunk
    print("multi-chunk: rays", R, flush=True)
    whole = am.render(ctx, tree, mlp, od, dd, 255, ert_eps=scene.cfg.ert_eps)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    assert st["n_chunks"] == 3 and st["n_nonfinite"] == 0
    n_samples = 0
    for r0 in range(0, R, chunk):
        part = am.render(ctx, tree, mlp, od[:, r0:r0 + chunk].contiguous(), dd[:, r0:r0 + chunk].contiguous(), 255,
                         ert_eps=scene.cfg.ert_eps)
        torch.cuda.synchronize()
        n_samples += am.amnerf_render_stats_get(ctx.h)["n_samples"]
        for k in ("rgb", "depth", "opacity"):
            assert torch.equal(whole[k][r0:r0 + chunk], part[k]), (k, r0)
    assert st["n_samples"] == n_samples


@pytest.mark.parametrize("mode", ["hcheck", "ess"])
def test_multi_chunk_call_with_options_equals_chunk_by_chunk_calls(mode):
    """The same three-pass call with hierarchical sampling (f = 0.5, node MLPs) or with empty
    space skipped (occupancy at half the guidance resolution, 1 % threshold): outputs and
    sample count bit-identical to three calls on the same slices."""
    scene = Scene(synth.C1, footprint=0.5 if mode == "hcheck" else 0.0)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    if mode == "hcheck":
        kw = {"hcheck_footprint": scene.footprint}
    else:
        kw = {"occupancy": am.Occupancy(ctx, scene.grid, cfg.grid_n, 2, 0.01)}
    o, d = scene.camera_rays()
    od = to_dev(o).repeat(1, 640).contiguous()
    dd = to_dev(d).repeat(1, 640).contiguous()
    R = od.shape[1]
    chunk = (1 << 28) // 255
    assert 2 * chunk < R < 3 * chunk
    print("multi-chunk %s: rays %d" % (mode, R), flush=True)
    whole = am.render(ctx, tree, mlp, od, dd, 255, ert_eps=cfg.ert_eps, **kw)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    assert st["n_chunks"] == 3 and st["n_nonfinite"] == 0
    n_samples = 0
    for r0 in range(0, R, chunk):
        part = am.render(ctx, tree, mlp, od[:, r0:r0 + chunk].contiguous(), dd[:, r0:r0 + chunk].contiguous(), 255,
                         ert_eps=cfg.ert_eps, **kw)
        torch.cuda.synchronize()
        n_samples += am.amnerf_render_stats_get(ctx.h)["n_samples"]
        for k in ("rgb", "depth", "opacity"):
            assert torch.equal(whole[k][r0:r0 + chunk], part[k]), (k, r0)
    assert st["n_samples"] == n_samples
