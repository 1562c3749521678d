"""The hand-written backward (compositing + grouped MLP), Adam and the training step on the GPU,
against the FP64 oracle's analytic gradient (itself pinned by central differences on the CPU)."""
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

# float32 operands against the float64 oracle: relative L2 error of the whole gradient
# vector (sample positions, features and sums carry float32 rounding, ~1e-6 relative).
TOL_F32_REL_L2 = 1e-4
# bfloat16 operands against the oracle run on the same bf16-rounded weights.  What remains
# is the bf16 rounding of the activations (and of the gradients at the MFMA inputs), which
# moves a few ReLU pre-activations across zero: each such sample switches a unit's whole
# backward contribution, so with random-sign upstream gradients (the gradient itself a
# random-sign sum over samples) the relative L2 error grows like the square root of the
# switched fraction: about 2% here (see the design notes).  Upstream gradients of a
# squared-error loss against a teacher sum coherently, and there the bar is 1e-2.
TOL_BF16_RANDOM = 3e-2
TOL_BF16_MSE = 1e-2
# per-sample compositing backward (float32) against the oracle's, per ray and column:
# |gpu - ref| <= 1e-5 * max over the ray's samples of |ref|.  dL/dsigma^_j = delta_j
# logistic(sigma^_j) dL/dtau_j sums O(1) terms (T_{j+1} c_j against the suffix sums, each
# weighted by the upstream gradient), so its float32 rounding is a few ulps of
# G = sum_c |g_c| + |g_depth| t_j + |g_opacity| times delta_j, whatever the result's size:
# that column also gets 1e-6 delta_j G (about 16 float32 ulps).
TOL_COMP = 1e-5
TOL_COMP_TAU_ULPS = 1e-6


def setup(scene):
    """Context, tree and a bf16 trainer over the scene's weights."""
    ctx = am.Context(0)
    tree = am.Tree(ctx, scene.grid, scene.cfg.grid_n, scene.cfg.max_depth, scene.cfg.max_leaves)
    assert np.array_equal(tree.rows, scene.otree.rows)
    master = torch.from_numpy(scene.W).to("cuda:0")
    tr = am.Trainer(ctx, tree, master, scene.cfg.n_hidden, scene.cfg.hidden)
    return ctx, tree, tr


def gpu_grad(scene, ctx, tree, mlp, master, o, d, s_max, eps, g_rgb, g_dep, g_op, sample_grad=False):
    od, dd = to_dev(o), to_dev(d)
    R = o.shape[1]
    rgb = torch.empty((R, 3), device="cuda:0")
    am.amnerf_render(ctx.h, tree.h, mlp, od, dd, s_max, rgb, None, None, None, eps)
    grad = torch.empty_like(master)
    am.amnerf_render_backward(ctx.h, tree.h, mlp, od, dd, to_dev(g_rgb.astype(np.float32)), grad,
                              to_dev(g_dep.astype(np.float32)), to_dev(g_op.astype(np.float32)))
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    g = grad.cpu().numpy().astype(np.float64)
    if not sample_grad:
        return g
    ns = st["n_placed_samples"]
    gs = torch.empty((max(ns, 1), 4), device="cuda:0")
    smp_off = torch.empty(R + 1, dtype=torch.int32, device="cuda:0")
    used = torch.empty(R, dtype=torch.int32, device="cuda:0")
    am.amnerf_render_backward_inspect(ctx.h, gs)
    am.amnerf_render_inspect(ctx.h, ray_smp_off=smp_off, ray_used=used)
    torch.cuda.synchronize()
    return g, gs.cpu().numpy()[:ns].astype(np.float64), smp_off.cpu().numpy().astype(np.int64), used.cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def bf16_round(W):
    return torch.from_numpy(W).to(torch.bfloat16).to(torch.float32).numpy()


C2_SMALL = synth.scaled(synth.C2, grid_n=64, max_leaves=64, max_depth=12)


def random_upstream(R, seed=7):
    """dL/d(rgb, depth, opacity) per ray with random signs."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((R, 3)) / R, rng.standard_normal(R) * 0.1 / R, rng.standard_normal(R) * 0.1 / R


def mse_upstream(scene, W, o, d, s_max, eps):
    """dL/drgb = 2 (rgb - target) / (3 R) of a squared-error loss, with rgb the oracle's render
    with weights W and a target 0.05 brighter in red and 0.05 darker in blue: the residuals'
    signs agree over the image, as they do in training."""
    cfg = scene.cfg
    rgb, _, _, _, _ = oracle.render(scene.otree, W, cfg.n_hidden, cfg.hidden, o, d, s_max, eps=eps)
    R = o.shape[1]
    target = rgb + np.array([0.05, 0.0, -0.05])
    return 2.0 * (rgb - target) / (3 * R), np.zeros(R), np.zeros(R)


@pytest.mark.parametrize("cfg,eps", [
    (synth.C1, 0.0),
    (synth.C1, 1e-4),
    (C2_SMALL, 1e-4),
])
def test_backward_f32_matches_oracle_gradient(cfg, eps):
    """float32 forward and backward: the whole gradient within 1e-4 relative L2 of the
    oracle's analytic gradient (itself pinned by central differences, with early termination
    on and off).  256 rays (a 16x16 camera) through an 8-leaf (2x32) or 64-leaf (4x64) scene."""
    scene = Scene(cfg)
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras, 16, 16)[0])
    R = o.shape[1]
    g_rgb, g_dep, g_op = random_upstream(R)
    g_gpu = gpu_grad(scene, ctx, tree, mlp.desc, mlp.master, o, d, cfg.s_max, eps, g_rgb, g_dep, g_op)
    f64 = lambda a: a.astype(np.float32).astype(np.float64)
    g_ref = oracle.render_grad(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max,
                               f64(g_rgb), f64(g_dep), f64(g_op), eps=eps)
    e = rel_l2(g_gpu, g_ref)
    print("f32 backward %s eps=%g: relative L2 error %.3e, |g| %.3e" % (cfg.name, eps, e, np.linalg.norm(g_ref)))
    assert np.isfinite(g_gpu).all()
    assert e <= TOL_F32_REL_L2
    hit = np.abs(g_ref).sum(axis=1) > 0
    assert np.all(g_gpu[~hit] == 0)


@pytest.mark.parametrize("cfg,eps,kind", [
    (synth.C1, 0.0, "random"),
    (synth.C1, 1e-4, "random"),
    (C2_SMALL, 1e-4, "random"),
    (synth.C1, 1e-4, "mse"),
    (C2_SMALL, 1e-4, "mse"),
])
def test_backward_bf16_matches_oracle_on_bf16_weights(cfg, eps, kind):
    """bfloat16 forward and backward against the oracle run on the bf16-rounded weights."""
    scene = Scene(cfg)
    ctx, tree, tr = setup(scene)
    o, d = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras, 16, 16)[0])
    R = o.shape[1]
    Wb = bf16_round(scene.W)
    if kind == "random":
        g_rgb, g_dep, g_op = random_upstream(R)
    else:
        g_rgb, g_dep, g_op = mse_upstream(scene, Wb, o, d, cfg.s_max, eps)
    g_gpu = gpu_grad(scene, ctx, tree, tr.mlp, tr.master, o, d, cfg.s_max, eps, g_rgb, g_dep, g_op)
    f64 = lambda a: a.astype(np.float32).astype(np.float64)
    g_ref = oracle.render_grad(scene.otree, Wb, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max, f64(g_rgb), f64(g_dep),
                               f64(g_op), eps=eps)
    e = rel_l2(g_gpu, g_ref)
    print("bf16 backward %s eps=%g %s: relative L2 error %.3e against the oracle on bf16 weights"
          % (cfg.name, eps, kind, e))
    assert np.isfinite(g_gpu).all()
    assert e <= (TOL_BF16_RANDOM if kind == "random" else TOL_BF16_MSE)
    hit = np.abs(g_ref).sum(axis=1) > 0
    assert np.all(g_gpu[~hit] == 0)


def test_full_batch_backward_on_sampled_rays():
    """The backward at the training step's full size: a 262 144-ray batch of the 800x800
    scene (512 leaves, one chunk, the training batches' recipe) with upstream gradients on
    a seeded subset of its rays only.  The gradient is linear in the upstream gradients and
    every other ray contributes exact zeros, so it must equal the oracle's over the subset
    alone: on 4 096 rays (about 8 per leaf) at the squared-error bar against the oracle on the
    bf16-rounded weights, and, on 256 rays, exactly zero for every leaf none of them crosses.
    (With about one ray per leaf, 256 rays leave the bf16 rounding of a few ReLU inputs
    unaveraged: measured 2.3e-2 there.)  Subset rays are robust ones (no split edge within
    the traversal's rounding), so both sides trace the same leaves."""
    cfg = synth.C2
    scene = Scene(cfg)
    ctx, tree, tr = setup(scene)
    B = 262144
    tcams = synth.make_cameras(100, cfg.seed_batches + 3, cfg.width, cfg.height)
    o, d = synth.random_pixel_rays(tcams, B, cfg.seed_batches + 4)
    Wb = bf16_round(scene.W)
    f64 = lambda a: a.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(9)
    for n_sub in (4096, 256):
        cand = np.sort(rng.choice(B, n_sub + 64, replace=False))
        sub = cand[oracle.robust(scene.otree, o[:, cand], d[:, cand])][:n_sub]
        assert len(sub) == n_sub
        # a squared-error residual of one sign over the image (red too dark, blue too bright)
        g_sub = np.tile(2.0 * np.array([-0.05, 0.0, 0.05]) / (3 * n_sub), (n_sub, 1))
        g_rgb = np.zeros((B, 3))
        g_rgb[sub] = g_sub
        print("full-batch backward: %d rays, upstream gradients on %d" % (B, n_sub), flush=True)
        g_gpu = gpu_grad(scene, ctx, tree, tr.mlp, tr.master, o, d, cfg.s_max, cfg.ert_eps, g_rgb, np.zeros(B),
                         np.zeros(B))
        st = am.amnerf_render_stats_get(ctx.h)
        assert st["n_chunks"] == 1 and st["n_rays"] == B and st["n_unreached"] == 0
        assert np.isfinite(g_gpu).all()
        g_ref = oracle.render_grad(scene.otree, Wb, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max, f64(g_sub),
                                   np.zeros(n_sub), np.zeros(n_sub), eps=cfg.ert_eps, ray_idx=sub)
        e = rel_l2(g_gpu, g_ref)
        _, _, slot, m = oracle.trace(scene.otree, o, d, ray_idx=sub)
        crossed = np.zeros(g_ref.shape[0], bool)
        for k in range(n_sub):
            crossed[slot[k, :m[k]]] = True
        print("full-batch backward, %d rays: relative L2 error %.3e against the oracle on bf16 weights; "
              "%d of %d leaves crossed" % (n_sub, e, crossed.sum(), len(crossed)), flush=True)
        if n_sub == 4096:
            assert e <= TOL_BF16_MSE
        else:
            assert e <= TOL_BF16_RANDOM
            assert crossed.sum() > 100 and (~crossed).sum() > 10
            assert np.all(g_gpu[~crossed] == 0)


def inv_softplus(s):
    return np.where(s > 30, s, np.log(np.expm1(np.maximum(s, 1e-300))))


def logit(c):
    return np.log(c) - np.log1p(-c)


@pytest.mark.parametrize("cfg,eps,dtype", [
    (synth.C1, 1e-4, am.AMNERF_F32),
    (synth.C1, 0.0, am.AMNERF_F32),
    (C2_SMALL, 1e-4, am.AMNERF_F32),
    (C2_SMALL, 1e-4, am.AMNERF_BF16),
])
def test_composite_backward_per_sample_matches_oracle(cfg, eps, dtype):
    """The compositing backward sample by sample: the GPU's dL/d(sigma^, r^, g^, b^) against
    the oracle's per-ray compositing gradient, evaluated on the oracle's own per-sample record
    (positions, segment lengths and MLP outputs from the seeded inputs).  The float32 leaf
    MLPs agree with the oracle's to ~1e-6, so each element agrees to 1e-5 of the ray's
    largest; the forward's stop index (recorded per ray) equals the oracle's on every ray
    whose stop is not within 1e-4 of the threshold.  With bf16 leaf MLPs the outputs move by
    ~1e-2, so only the stop index and the zero gradient after it are compared."""
    scene = Scene(cfg)
    ctx, tree, mlp = gpu_setup(scene, dtype)
    o, d = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras, 24, 24)[0])
    R = o.shape[1]
    rng = np.random.default_rng(3)
    g_rgb, g_dep, g_op = rng.standard_normal((R, 3)), rng.standard_normal(R) * 0.1, rng.standard_normal(R) * 0.1
    g, gs, smp_off, used = gpu_grad(scene, ctx, tree, mlp.desc, mlp.master, o, d, cfg.s_max, eps,
                                    g_rgb, g_dep, g_op, sample_grad=True)
    robust = oracle.robust(scene.otree, o, d)
    n_cmp = n_stop = worst = 0
    for r in range(R):
        rec = oracle.ray_samples(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, r, cfg.s_max, eps=eps)
        a, b = smp_off[r], smp_off[r + 1]
        ns = len(rec["t"])
        assert np.all(gs[a + used[r]:b] == 0)       # nothing after the forward's stop
        n_stop += used[r] < b - a
        if dtype != am.AMNERF_F32 or not robust[r] or rec["flags"] & oracle.FLAG_ERT_AMBIGUOUS:
            continue
        assert b - a == ns, (r, b - a, ns)
        assert used[r] == rec["n_used"], (r, used[r], rec["n_used"])
        J = rec["n_used"]
        if ns == 0:
            continue
        z = np.zeros((ns, 4))
        z[:J] = np.column_stack([inv_softplus(rec["sigma"][:J]), logit(rec["rgb"][:J])])
        gv = np.array([*g_rgb[r], g_dep[r], g_op[r]], np.float32).astype(np.float64)
        ref, Jr = oracle.composite_grad(z, rec["t"], rec["delta"], gv, eps=eps)
        assert Jr == J
        scale = np.abs(ref).max(axis=0)
        G = np.abs(gv[:3]).sum() + abs(gv[3]) * rec["t"] + abs(gv[4])
        bar = np.repeat((TOL_COMP * scale)[None, :], ns, axis=0)
        bar[:, 0] += TOL_COMP_TAU_ULPS * rec["delta"] * G
        err = np.abs(gs[a:b] - ref)
        assert np.all(err <= bar + 1e-12), (r, (err / bar).max())
        worst = max(worst, float((err / bar).max()))
        n_cmp += 1
    print("per-sample compositing backward %s eps=%g dtype %d: %d rays compared, %d stopped early, worst "
          "error / bar %.2e"
          % (cfg.name, eps, dtype, n_cmp, n_stop, worst))
    if eps > 0:
        assert n_stop > 0
    if dtype == am.AMNERF_F32:
        assert n_cmp > 0.9 * (smp_off[1:] > smp_off[:-1]).sum()


def test_backward_is_deterministic():
    scene = Scene(synth.C1)
    ctx, tree, tr = setup(scene)
    o, d = synth.camera_rays(synth.make_cameras(1, 301, 32, 32)[0])
    R = o.shape[1]
    g = np.full((R, 3), 1.0 / R)
    z = np.zeros(R)
    a = gpu_grad(scene, ctx, tree, tr.mlp, tr.master, o, d, 64, 1e-4, g, z, z)
    b = gpu_grad(scene, ctx, tree, tr.mlp, tr.master, o, d, 64, 1e-4, g, z, z)
    assert np.array_equal(a, b)


def test_adam_matches_oracle():
    ctx = am.Context(0)
    rng = np.random.default_rng(3)
    n = 10000
    p = rng.standard_normal(n).astype(np.float32)
    pt, mt, vt = to_dev(p), torch.zeros(n, device="cuda:0"), torch.zeros(n, device="cuda:0")
    p64, m64, v64 = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32)
        am.amnerf_adam_step(ctx.h, pt, mt, vt, to_dev(g), step, lr=1e-2)
        oracle.adam(p64, m64, v64, g.astype(np.float64), step, lr=1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(pt.cpu().numpy(), p64, rtol=0, atol=1e-5)


def test_train_step_gradient_equals_backward_of_mse_and_autograd():
    scene = Scene(synth.C1)
    ctx, tree, tr = setup(scene)
    o, d = synth.camera_rays(synth.make_cameras(1, 301, 24, 24)[0])
    od, dd = to_dev(o), to_dev(d)
    R = o.shape[1]
    target = to_dev(np.random.default_rng(1).uniform(0, 1, (R, 3)).astype(np.float32))
    loss = tr.step(od, dd, target, 64, grad_only=True).item()
    g_step = tr.grad.clone()
    # same gradient through the autograd wrapper
    master = tr.master.clone().requires_grad_(True)
    rgb, dep, op = am.RenderFn.apply(master, ctx, tree, od, dd, 64, 1e-4, 2, 32)
    l2 = ((rgb - target) ** 2).mean()
    l2.backward()
    torch.cuda.synchronize()
    assert abs(l2.item() - loss) <= 1e-6 * max(1.0, loss)
    np.testing.assert_allclose(master.grad.cpu().numpy(), g_step.cpu().numpy(), rtol=1e-4, atol=1e-9)


def test_training_reduces_loss_teacher_student():
    """A re-seeded student fitted to a teacher's renders by the library's own training step."""
    cfg = synth.scaled(synth.C2, grid_n=64, max_leaves=64, max_depth=12)
    teacher = Scene(cfg)
    ctx, tree, tr_t = setup(teacher)
    cams = synth.make_cameras(8, cfg.seed_cameras, 64, 64)
    o, d = synth.rays_for_cameras(cams)
    od, dd = to_dev(o), to_dev(d)
    R = o.shape[1]
    target = torch.empty((R, 3), device="cuda:0")
    mlp_t = am.Mlp(ctx, torch.from_numpy(teacher.W).to("cuda:0"), cfg.n_hidden, cfg.hidden, am.AMNERF_F32,
                   tree.n_leaves)
    am.amnerf_render(ctx.h, tree.h, mlp_t.desc, od, dd, 128, target, None, None, None, 1e-4)
    dens = synth.leaf_mean_density(teacher.grid, cfg.grid_n, teacher.otree.leaf_boxes())
    W_s = synth.make_weights(tree.n_leaves, cfg.n_hidden, cfg.hidden, cfg.seed_student, dens)
    tr = am.Trainer(ctx, tree, torch.from_numpy(W_s).to("cuda:0"), cfg.n_hidden, cfg.hidden)
    gen = torch.Generator(device="cuda:0").manual_seed(cfg.seed_batches)
    losses = []
    for it in range(60):
        idx = torch.randint(0, R, (4096,), device="cuda:0", generator=gen)
        ob, db_, tb = od[:, idx].contiguous(), dd[:, idx].contiguous(), target[idx].contiguous()
        losses.append(tr.step(ob, db_, tb, 128, lr=3e-3).item())
    print("teacher-student loss: first %.4e, last %.4e" % (losses[0], losses[-1]))
    assert np.isfinite(losses).all()
    assert np.mean(losses[-5:]) < 0.5 * np.mean(losses[:5])


def test_backward_stage_timing():
    """With timing on, every backward pass records its stages: a training step all four (the
    Adam stage includes the repack), a backward pass alone no Adam; the forward stages of
    the step's render are timed as usual."""
    scene = Scene(synth.C1)
    ctx, tree, tr = setup(scene)
    o, d = synth.camera_rays(synth.make_cameras(1, 301, 24, 24)[0])
    od, dd = to_dev(o), to_dev(d)
    R = o.shape[1]
    target = to_dev(np.random.default_rng(1).uniform(0, 1, (R, 3)).astype(np.float32))
    am.amnerf_ctx_set_timing(ctx.h, True)
    am.amnerf_timing_collect(ctx.h)
    am.amnerf_timing_collect_backward(ctx.h)
    for _ in range(3):
        tr.step(od, dd, target, 64, lr=1e-3)
    torch.cuda.synchronize()
    bwd, nb = am.amnerf_timing_collect_backward(ctx.h)
    fwd, nf = am.amnerf_timing_collect(ctx.h)
    assert nb == 3 and nf == 3
    assert all(v > 0 for v in bwd.values()), bwd
    assert fwd["mlp"] > 0 and fwd["composite"] > 0
    # a backward pass alone: no Adam stage
    am.amnerf_render(ctx.h, tree.h, tr.mlp, od, dd, 64, torch.empty((R, 3), device="cuda:0"), None, None, None, 1e-4)
    grad = torch.empty_like(tr.master)
    am.amnerf_render_backward(ctx.h, tree.h, tr.mlp, od, dd, to_dev(np.full((R, 3), 1.0, np.float32)), grad)
    torch.cuda.synchronize()
    bwd, nb = am.amnerf_timing_collect_backward(ctx.h)
    assert nb == 1 and bwd["adam"] == 0.0 and bwd["mlp_bwd"] > 0 and bwd["comp_bwd"] > 0
    am.amnerf_ctx_set_timing(ctx.h, False)
    tr.step(od, dd, target, 64, lr=1e-3)
    torch.cuda.synchronize()
    assert am.amnerf_timing_collect_backward(ctx.h)[1] == 0
