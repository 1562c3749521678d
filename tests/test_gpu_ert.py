"""Early termination in rounds (Section 4.1): the leaf MLPs evaluate each ray's samples in
windows of 64, and a ray that terminated in an earlier window has no later samples
evaluated.  The render is the same quadrature, so its outputs, weights and stop indices
must be bit-identical to the single-pass render; only the evaluated-sample count drops, to
exactly the windows up to and including each ray's stop (checked against the oracle's stop
index on rays whose stop is not ambiguous)."""
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


def render(ctx, tree, mlp, o, d, s_max, flags, weights=False, eps=1e-4, seed=0, footprint=0.0, proposal=None,
           occupancy=None, static=False):
    R = o.shape[1]
    dev = "cuda:0"
    out = [torch.full((R, 3), -1.0, device=dev), torch.full((R,), -1.0, device=dev),
           torch.full((R,), -1.0, device=dev), torch.full((R * s_max,), -1.0, device=dev) if weights else None]
    rays = am.amnerf_rays(o.data_ptr(), d.data_ptr(), R)
    prm = am.amnerf_render_params(s_max, eps, flags, seed, am.C.pointer(proposal) if proposal is not None else None,
                                  footprint, am._handle(occupancy))
    ro = am.amnerf_render_out(*[None if t is None else t.data_ptr() for t in out])
    fn = am.lib().amnerf_render_static if static else am.lib().amnerf_render
    am._check(fn(ctx.h, tree.h, am.C.byref(mlp.desc), am.C.byref(rays), am.C.byref(prm), am.C.byref(ro),
                 am._stream(None)))
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    used = smp_off = None
    if st["n_chunks"] == 1 and not static:
        u = torch.empty(R, dtype=torch.int32, device=dev)
        so = torch.empty(R + 1, dtype=torch.int32, device=dev)
        am.amnerf_render_inspect(ctx.h, ray_used=u, ray_smp_off=so)
        torch.cuda.synchronize()
        used, smp_off = u.cpu().numpy().astype(np.int64), so.cpu().numpy().astype(np.int64)
    return out, st, used, smp_off


def expected_evaluated(used, smp_off):
    """Samples of the windows up to and including each ray's stop window."""
    ns = np.diff(smp_off)
    win = np.where(used > 0, (used + 63) // 64 * 64, 0)
    return int(np.minimum(ns, win).sum())


def compare(a, b, what):
    for name, x, y in zip(("rgb", "depth", "opacity", "weights"), a, b):
        if x is not None:
            assert torch.equal(x, y), (what, name)


CASES = {
    "small_f32_s128": dict(cfg=synth.C1, dtype=am.AMNERF_F32, s_max=128, weights=True),
    "small_f32_s255_jitter": dict(cfg=synth.C1, dtype=am.AMNERF_F32, s_max=255, jitter=True),
    "small_bf16_hcheck": dict(cfg=synth.C1, dtype=am.AMNERF_BF16, s_max=128, footprint=0.5),
    "small_bf16_occupancy": dict(cfg=synth.C1, dtype=am.AMNERF_BF16, s_max=128, occupancy=True),
    "small_f32_proposal": dict(cfg=synth.C1, dtype=am.AMNERF_F32, s_max=160, proposal=True, saves=False),
    "c2_bf16_s128": dict(cfg=synth.C2, dtype=am.AMNERF_BF16, s_max=128, rays=120_000),
    "small_fp8act_s192": dict(cfg=synth.scaled(synth.C1, n_hidden=4, hidden=64), dtype=am.AMNERF_FP8_ACT, s_max=192),
}


@pytest.mark.parametrize("case", list(CASES))
def test_rounds_are_bit_identical_to_a_single_pass(case):
    c = CASES[case]
    cfg = c["cfg"]
    print("ert rounds case", case, flush=True)
    scene = Scene(cfg, footprint=c.get("footprint", 0.0))
    ctx, tree, mlp = gpu_setup(scene, c["dtype"])
    ctx2 = am.Context(0)
    o, d = scene.camera_rays()
    if "rays" in c:
        pick = np.sort(np.random.default_rng(5).choice(o.shape[1], c["rays"], replace=False))
        o, d = np.ascontiguousarray(o[:, pick]), np.ascontiguousarray(d[:, pick])
    od, dd = to_dev(o), to_dev(d)
    kw = dict(weights=c.get("weights", False), footprint=c.get("footprint", 0.0))
    flags = am.AMNERF_JITTER if c.get("jitter") else 0
    if c.get("jitter"):
        kw["seed"] = 77
    if c.get("occupancy"):
        kw["occupancy"] = am.Occupancy(ctx, scene.grid, cfg.grid_n, 2, 0.01)
    if c.get("proposal"):
        prop = am.Proposal(ctx, torch.from_numpy(synth.make_prop_weights(3)).to("cuda:0"))
        kw["proposal"] = prop.descriptor(am.AMNERF_F32, mass_thresh=0.6, cap=48)
    one, st1, used1, off1 = render(ctx, tree, mlp, od, dd, c["s_max"], flags, **kw)
    rnd, st2, used2, off2 = render(ctx2, tree, mlp, od, dd, c["s_max"], flags | am.AMNERF_ERT_ROUNDS, **kw)
    compare(rnd, one, case)
    assert np.array_equal(used1, used2) and np.array_equal(off1, off2)
    assert st2["n_composited"] == st1["n_composited"]
    assert st2["n_placed_samples"] == st1["n_placed_samples"] == st1["n_samples"]
    assert st2["n_samples"] == expected_evaluated(used2, off2)
    print("%s: evaluated %d of %d samples in rounds (composited %d)" % (
        case, st2["n_samples"], st1["n_samples"], st2["n_composited"]), flush=True)
    if c.get("saves", True):
        assert st2["n_samples"] < st1["n_samples"]
    else:
        assert st2["n_samples"] <= st1["n_samples"]


def test_rounds_evaluated_count_against_the_oracle():
    """Per ray, the windows evaluated are those up to the oracle's stop sample (float32 plain
    path, rays whose stop is not within the ambiguity band of the threshold)."""
    scene = Scene(synth.C1)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = scene.camera_rays()
    _, st, used, off = render(ctx, tree, mlp, to_dev(o), to_dev(d), 128, am.AMNERF_ERT_ROUNDS)
    rgb, _, _, ns, flags = oracle.render(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, 128, eps=1e-4)
    robust = oracle.robust(scene.otree, o, d)
    ok = robust & ((flags & oracle.FLAG_ERT_AMBIGUOUS) == 0)
    n_used = np.zeros(o.shape[1], np.int64)
    rng = np.random.default_rng(2)
    check = np.sort(rng.choice(np.where(ok & (ns > 64))[0], 300, replace=False))
    for r in check:
        n_used[r] = oracle.ray_samples(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, int(r), 128,
                                       eps=1e-4)["n_used"]
    assert np.array_equal(used[check], n_used[check])
    want = np.minimum(ns[check], (n_used[check] + 63) // 64 * 64)
    got = np.minimum(np.diff(off)[check], (used[check] + 63) // 64 * 64)
    assert np.array_equal(got, want)
    assert (n_used[check] <= 64).sum() > 0      # some rays stop in the first window


def test_rounds_multi_chunk_and_static():
    """A call of several passes (odd passes on the second lane) and the allocation-free render,
    each in rounds, equal to the single-pass render."""
    scene = Scene(synth.C1)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_BF16)
    o, d = scene.camera_rays()
    reps = 260          # 1 064 960 rays at s_max 255: two passes of at most 1 052 689 rays
    od, dd = to_dev(np.tile(o, reps)), to_dev(np.tile(d, reps))
    one, st1, _, _ = render(ctx, tree, mlp, od, dd, 255, 0)
    rnd, st2, _, _ = render(am.Context(0), tree, mlp, od, dd, 255, am.AMNERF_ERT_ROUNDS)
    assert st1["n_chunks"] == st2["n_chunks"] == 2
    compare(rnd, one, "multi-chunk")
    assert st2["n_composited"] == st1["n_composited"] and st2["n_samples"] < st1["n_samples"]
    os_, ds_ = to_dev(o[:, :3000]), to_dev(d[:, :3000])
    ref, sr, _, _ = render(ctx, tree, mlp, os_, ds_, 128, 0)
    sta, ss, _, _ = render(ctx, tree, mlp, os_, ds_, 128, am.AMNERF_ERT_ROUNDS, static=True)
    compare(sta, ref, "static")
    assert ss["n_samples"] < sr["n_samples"]


@pytest.mark.parametrize("dtype", [am.AMNERF_F32, am.AMNERF_BF16])
def test_backward_after_rounds_equals_backward_after_single_pass(dtype):
    scene = Scene(synth.C1)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, dtype)
    o, d = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras, 24, 24)[0])
    od, dd = to_dev(o), to_dev(d)
    R = o.shape[1]
    g = to_dev(np.random.default_rng(1).standard_normal((R, 3)).astype(np.float32))
    grads = []
    for flags in (0, am.AMNERF_ERT_ROUNDS):
        render(ctx, tree, mlp, od, dd, 128, flags)
        gr = torch.empty_like(mlp.master)
        am.amnerf_render_backward(ctx.h, tree.h, mlp.desc, od, dd, g, gr)
        torch.cuda.synchronize()
        grads.append(gr)
    assert torch.equal(grads[0], grads[1])
