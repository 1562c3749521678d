"""The learned proposal on the GPU (inference, planned render, training step) against the oracle."""
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


def setup(cfg, dtype=am.AMNERF_F32, prop_seed=None):
    scene = Scene(cfg)
    ctx = am.Context(0)
    tree = am.Tree(ctx, scene.grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
    assert np.array_equal(tree.rows, scene.otree.rows)
    mlp = am.Mlp(ctx, torch.from_numpy(scene.W).to("cuda:0"), cfg.n_hidden, cfg.hidden, dtype, tree.n_leaves)
    prop_w = synth.make_prop_weights(cfg.seed_proposal if prop_seed is None else prop_seed)
    prop = am.Proposal(ctx, torch.from_numpy(prop_w).to("cuda:0"))
    return scene, ctx, tree, mlp, prop, prop_w


def render(ctx, tree, mlp, o, d, s_max, proposal=None, eps=1e-4):
    od, dd = to_dev(o), to_dev(d)
    R = o.shape[1]
    rgb = torch.empty((R, 3), device="cuda:0")
    dep = torch.empty(R, device="cuda:0")
    op = torch.empty(R, device="cuda:0")
    am.amnerf_render(ctx.h, tree.h, mlp.desc, od, dd, s_max, rgb, dep, op, None, eps, proposal=proposal)
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    return rgb.cpu().numpy(), dep.cpu().numpy(), op.cpu().numpy(), st


def ray_sample_counts(ctx, R):
    b = torch.empty(R + 1, dtype=torch.int32, device="cuda:0")
    am.amnerf_render_inspect(ctx.h, ray_smp_off=b)
    torch.cuda.synchronize()
    return np.diff(b.cpu().numpy().astype(np.int64))


@pytest.mark.parametrize("dtype,tol", [(am.AMNERF_F32, 2e-5), (am.AMNERF_BF16, 0.08)])
def test_inference_matches_oracle(dtype, tol):
    cfg = synth.C1
    scene, ctx, tree, mlp, prop, prop_w = setup(cfg)
    o, d = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras, 16, 16)[0])
    tau = prop.infer(tree, mlp.desc, to_dev(o), to_dev(d), cfg.s_max, dtype=dtype).cpu().numpy()
    feat, tau_ref = oracle.prop_eval(scene.otree, prop_w, o, d, cfg.s_max)
    assert tau.shape == tau_ref.shape
    err = np.abs(tau - tau_ref).max() / max(1.0, np.abs(tau_ref).max())
    print("proposal inference dtype %d: max rel err %.3e" % (dtype, err))
    assert err <= tol


def test_all_fallback_is_bit_identical_to_plain():
    cfg = synth.C1
    scene, ctx, tree, mlp, prop, prop_w = setup(cfg)
    o, d = scene.camera_rays()
    plain = render(ctx, tree, mlp, o, d, cfg.s_max)
    desc = prop.descriptor(am.AMNERF_F32, mass_thresh=2.0, cap=cfg.s_max)
    fb = render(ctx, tree, mlp, o, d, cfg.s_max, proposal=desc)
    for a, b in zip(plain[:3], fb[:3]):
        assert np.array_equal(a, b)
    assert fb[3]["n_samples"] == plain[3]["n_samples"]
    assert fb[3]["n_fallback"] == int((ray_sample_counts(ctx, o.shape[1]) > 0).sum())


@pytest.mark.parametrize("case", ["small_s64", "small_s160", "small_s255", "large_subset"])
def test_planned_render_matches_oracle(case):
    """An untrained proposal with a low mass threshold plans for many rays: compare per-ray
    sample counts with the oracle's plans and the rendered colours where the plans agree.
    S_max 160 and 255 give rays of up to 192 and 256 slots (three and four registers of the
    selection's sort); the large scene is checked on 20 000 random pixels of one camera."""
    if case == "large_subset":
        cfg, s_max, thresh, cap = synth.C3, synth.C3.s_max, 0.5, 48
    else:
        cfg, s_max = synth.C1, int(case.split("_s")[1])
        thresh, cap = (0.5, 40) if s_max == 64 else (0.6, 48)
    print("planned render case", case, flush=True)
    scene, ctx, tree, mlp, prop, prop_w = setup(cfg)
    o, d = scene.camera_rays()
    if case == "large_subset":
        pick = np.sort(np.random.default_rng(11).choice(o.shape[1], 20_000, replace=False))
        o, d = np.ascontiguousarray(o[:, pick]), np.ascontiguousarray(d[:, pick])
    R = o.shape[1]
    desc = prop.descriptor(am.AMNERF_F32, mass_thresh=thresh, cap=cap)
    rgb, dep, op, st = render(ctx, tree, mlp, o, d, s_max, proposal=desc)
    counts = ray_sample_counts(ctx, R)
    orgb, odep, oop, ons, opn, opsel, omass = oracle.render_proposal(scene.otree, scene.W, cfg.n_hidden, cfg.hidden,
                                                                     prop_w, o, d, s_max, eps=1e-4,
                                                                     mass_thresh=thresh, cap=cap)
    mask = torch.empty((R, 4), dtype=torch.int64, device="cuda:0")
    am.amnerf_render_inspect(ctx.h, slot_mask=mask)
    torch.cuda.synchronize()
    bits = np.unpackbits(mask.cpu().numpy().view(np.uint8).reshape(R, 32), axis=1, bitorder="little")
    same = counts == ons
    planned = opn > 0
    print("plans: %d planned rays, %d fallback (gpu %d), counts agree on %.4f of rays, max plan %d slots" % (
        planned.sum(), (opn < 0).sum(), st["n_fallback"], same.mean(), opn.max()))
    assert planned.sum() > 0.2 * R
    assert same.mean() >= 0.995
    ok = same & ~np.isin(np.arange(R), np.where(np.abs(omass - thresh) < 1e-4)[0])
    err = np.abs(rgb[ok] - orgb[ok]).max()
    # the kept slots themselves: on rays whose counts agree, the GPU's kept-slot set equals
    # the oracle's plan (all slots for a ray that fell back)
    n_set = n_eq = 0
    for r in np.where(ok & (ons > 0))[0]:
        kept = np.nonzero(bits[r])[0]
        if opn[r] < 0:
            want = np.arange(counts[r])
            kept = kept[kept < counts[r]]
        else:
            want = np.sort(opsel[r, :opn[r]])
        n_set += 1
        n_eq += np.array_equal(kept, want)
    print("planned render: max |rgb - oracle| on agreeing rays %.3e; kept-slot sets equal on %d of %d rays"
          % (err, n_eq, n_set))
    assert n_set > 0 and n_eq >= 0.995 * n_set
    assert err <= 1e-5
    assert st["n_samples"] < st["n_plain_samples"]
    if s_max > 128:
        # some planned rays chose from more than 128 slots (the sort's wider forms ran)
        m = oracle.trace(scene.otree, o, d, cap=s_max + 1)[3]
        slots = np.where(m > 0, np.minimum(m, s_max) * np.maximum(s_max // np.maximum(m, 1), 1), 0)
        print("planned rays with more than 128 slots: %d" % int((planned & (slots > 128)).sum()))
        assert (planned & (slots > 128)).sum() > 0


def test_training_step_gradient_matches_oracle():
    cfg = synth.C1
    scene, ctx, tree, mlp, prop, prop_w = setup(cfg)
    o, d = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras, 16, 16)[0])
    loss = prop.train_step(tree, mlp.desc, to_dev(o), to_dev(d), cfg.s_max, lr=0.0).item()
    g = prop.grad.cpu().numpy().astype(np.float64)
    feat, _ = oracle.prop_eval(scene.otree, prop_w, o, d, cfg.s_max)
    alpha = oracle.prop_targets(scene.otree, scene.W, 2, 32, o, d, cfg.s_max)
    loss_ref, g_ref = oracle.prop_loss_grad(prop_w, feat, alpha)
    e = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print("proposal training: loss %.6e vs %.6e, gradient rel L2 %.3e" % (loss, loss_ref, e))
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    assert e <= 1e-3


def test_training_reduces_samples_and_keeps_quality():
    """Train on a few cameras, test on a held-out one: fewer samples than plain sampling, and
    the proposal render stays close to the plain render."""
    cfg = synth.scaled(synth.C2, grid_n=64, max_leaves=64, max_depth=12, width=64, height=64)
    scene, ctx, tree, mlp, prop, prop_w = setup(cfg, am.AMNERF_F32)
    cams = synth.make_cameras(9, cfg.seed_cameras, 64, 64)
    o_tr, d_tr = synth.rays_for_cameras(cams[:8])
    o_te, d_te = synth.rays_for_cameras(cams[8:])
    otr, dtr = to_dev(o_tr), to_dev(d_tr)
    gen = torch.Generator(device="cuda:0").manual_seed(cfg.seed_batches)
    losses = []
    for it in range(300):
        idx = torch.randint(0, otr.shape[1], (4096,), device="cuda:0", generator=gen)
        losses.append(prop.train_step(tree, mlp.desc, otr[:, idx].contiguous(), dtr[:, idx].contiguous(), 128,
                                      lr=3e-3).item())
    prop.repack()
    plain = render(ctx, tree, mlp, o_te, d_te, 128)
    desc = prop.descriptor(am.AMNERF_F32, mass_thresh=0.99, cap=48)
    pr = render(ctx, tree, mlp, o_te, d_te, 128, proposal=desc)
    psnr = oracle.psnr(pr[0], plain[0])
    spr = pr[3]["n_samples"] / max(1, (ray_sample_counts(ctx, o_te.shape[1]) > 0).sum())
    print("proposal training loss %.4e -> %.4e; held-out: %d -> %d samples, fallback %d rays, psnr vs plain %.2f dB"
          % (losses[0], losses[-1], plain[3]["n_samples"], pr[3]["n_samples"], pr[3]["n_fallback"], psnr))
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:10])
    assert pr[3]["n_samples"] < 0.8 * plain[3]["n_samples"]
    assert psnr >= 40.0   # measured 44.2 dB


def test_failed_call_after_freed_workspace_leaves_no_inspectable_render():
    """A proposal render keeps its plan in the context's third workspace.  A later call that
    regrows that workspace and then fails (here: amnerf_propose whose scene MLP has the wrong
    number of leaves) must leave no render to inspect or differentiate: AMNERF_ESTATE, not a
    copy out of freed memory.  A call that fails its argument checks first changes nothing."""
    scene = Scene(synth.C1)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    prop = am.Proposal(ctx, torch.from_numpy(synth.make_prop_weights(1)).to("cuda:0"))
    o, d = (to_dev(a) for a in scene.camera_rays(0))
    R = o.shape[1]
    am.render(ctx, tree, mlp, o, d, cfg.s_max, proposal=prop.descriptor(am.AMNERF_F32, 0.5, 48))
    used = torch.empty(R, dtype=torch.int32, device="cuda:0")
    mask = torch.empty((R, 4), dtype=torch.int64, device="cuda:0")
    am.amnerf_render_inspect(ctx.h, ray_used=used, slot_mask=mask)
    torch.cuda.synchronize()
    # bad s_max: rejected before any workspace is touched; the render stays inspectable
    with pytest.raises(am.AmnerfError) as e:
        prop.infer(tree, mlp.desc, o, d, 0)
    assert e.value.code == am.AMNERF_EINVAL
    am.amnerf_render_inspect(ctx.h, ray_used=used)
    # many rays regrow the third workspace, then the scene MLP is refused
    big = [to_dev(a) for a in scene.camera_rays(1, width=400, height=400)]
    wrong = am.Mlp(ctx, torch.from_numpy(synth.make_weights(1, cfg.n_hidden, cfg.hidden, 1)).to("cuda:0"),
                   cfg.n_hidden, cfg.hidden, am.AMNERF_F32, 1)
    with pytest.raises(am.AmnerfError) as e:
        prop.infer(tree, wrong.desc, big[0], big[1], cfg.s_max)
    assert e.value.code == am.AMNERF_EINVAL
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render_inspect(ctx.h, ray_used=used)
    assert e.value.code == am.AMNERF_ESTATE
    grad = torch.empty_like(mlp.master)
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render_backward(ctx.h, tree.h, mlp.desc, o, d, torch.zeros((R, 3), device="cuda:0"), grad)
    assert e.value.code == am.AMNERF_ESTATE
