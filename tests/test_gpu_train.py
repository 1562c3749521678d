"""The hand-written backward (compositing + grouped MLP), Adam and the training step on the GPU,
against the FP64 oracle's analytic gradient (itself pinned by central differences on the CPU)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from scene_util import Scene, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2310_01881_amd as am  # noqa: E402

# bfloat16 operands (weights, activations, gradients at the MFMA inputs) against a float64
# reference: relative L2 error of the whole gradient vector.
TOL_REL_L2 = 2e-2


def setup(scene):
    ctx = am.Context(0)
    tree = am.Tree(ctx, scene.grid, scene.cfg.grid_n, scene.cfg.max_depth, scene.cfg.max_leaves)
    assert np.array_equal(tree.rows, scene.otree.rows)
    master = torch.from_numpy(scene.W).to("cuda:0")
    tr = am.Trainer(ctx, tree, master, scene.cfg.n_hidden, scene.cfg.hidden)
    return ctx, tree, tr


def gpu_grad(scene, ctx, tree, tr, o, d, s_max, eps, g_rgb, g_dep, g_op):
    od, dd = to_dev(o), to_dev(d)
    R = o.shape[1]
    rgb = torch.empty((R, 3), device="cuda:0")
    am.amnerf_render(ctx.h, tree.h, tr.mlp, od, dd, s_max, rgb, None, None, None, eps)
    grad = torch.empty_like(tr.master)
    am.amnerf_render_backward(ctx.h, tree.h, tr.mlp, od, dd, to_dev(g_rgb.astype(np.float32)), grad,
                              to_dev(g_dep.astype(np.float32)), to_dev(g_op.astype(np.float32)))
    torch.cuda.synchronize()
    return grad.cpu().numpy().astype(np.float64)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("cfg,eps", [
    (synth.C1, 0.0),
    (synth.C1, 1e-4),
    (synth.scaled(synth.C2, grid_n=64, max_leaves=64, max_depth=12), 1e-4),
])
def test_backward_matches_oracle_gradient(cfg, eps):
    """256 rays (a 16x16 camera) through an 8-leaf (2x32) or 64-leaf (4x64) scene."""
    scene = Scene(cfg)
    ctx, tree, tr = setup(scene)
    o, d = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras, 16, 16)[0])
    R = o.shape[1]
    rng = np.random.default_rng(7)
    g_rgb = rng.standard_normal((R, 3)) / R
    g_dep = rng.standard_normal(R) * 0.1 / R
    g_op = rng.standard_normal(R) * 0.1 / R
    s_max = cfg.s_max
    g_gpu = gpu_grad(scene, ctx, tree, tr, o, d, s_max, eps, g_rgb, g_dep, g_op)
    g_ref = oracle.render_grad(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, s_max,
                               g_rgb.astype(np.float32).astype(np.float64),
                               g_dep.astype(np.float32).astype(np.float64),
                               g_op.astype(np.float32).astype(np.float64), eps=eps)
    e = rel_l2(g_gpu, g_ref)
    print("backward %s eps=%g: relative L2 error %.3e, |g| %.3e" % (cfg.name, eps, e, np.linalg.norm(g_ref)))
    assert np.isfinite(g_gpu).all()
    assert e <= TOL_REL_L2
    # leaves that no sample reached have exactly zero gradient
    hit = np.abs(g_ref).sum(axis=1) > 0
    assert np.all(g_gpu[~hit] == 0)


def test_backward_is_deterministic():
    scene = Scene(synth.C1)
    ctx, tree, tr = setup(scene)
    o, d = synth.camera_rays(synth.make_cameras(1, 301, 32, 32)[0])
    R = o.shape[1]
    g = np.full((R, 3), 1.0 / R)
    z = np.zeros(R)
    a = gpu_grad(scene, ctx, tree, tr, o, d, 64, 1e-4, g, z, z)
    b = gpu_grad(scene, ctx, tree, tr, o, d, 64, 1e-4, g, z, z)
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
