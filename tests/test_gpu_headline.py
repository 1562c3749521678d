"""The headline path on the 800x800 workload (128^3 guidance grid, 512-leaf tree, 4x64 leaf
MLPs, S_max 128): bf16 leaf MLPs plus the learned proposal, trained here by the library's
own training step with the benchmark's recipe (200 training cameras, a pool of 2 000 000
random pixel rays, 1500 steps of 32 768 rays, lr 3e-3 then 1e-3), keeps >= 45 dB PSNR against
the FP64 oracle's plain render on a seeded subset of held-out camera 0, with far fewer
samples than the plain sampler."""
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

PSNR_TARGET_DB = 45.0


def test_bf16_plus_trained_proposal_reaches_45db_against_the_oracle():
    cfg = synth.C2
    scene = Scene(cfg)
    ctx, tree, mlp32 = gpu_setup(scene, am.AMNERF_F32)
    mlp16 = am.Mlp(ctx, mlp32.master, cfg.n_hidden, cfg.hidden, am.AMNERF_BF16, tree.n_leaves)
    dev = "cuda:0"
    prop = am.Proposal(ctx, torch.from_numpy(synth.make_prop_weights(cfg.seed_proposal)).to(dev))
    train_cams = synth.make_cameras(200, cfg.seed_batches, cfg.width, cfg.height)
    pool_o, pool_d = synth.random_pixel_rays(train_cams, 2_000_000, cfg.seed_batches + 1)
    pool_o, pool_d = to_dev(pool_o), to_dev(pool_d)
    gen = torch.Generator(device=dev).manual_seed(cfg.seed_batches + 2)
    steps, batch = 1500, 32768
    first = last = None
    for it in range(steps):
        lr = 3e-3 if it < 0.7 * steps else 1e-3
        idx = torch.randint(0, pool_o.shape[1], (batch,), device=dev, generator=gen)
        loss = prop.train_step(tree, mlp32.desc, pool_o[:, idx].contiguous(), pool_d[:, idx].contiguous(),
                               cfg.s_max, lr=lr)
        if it == 0:
            first = float(loss.item())
        if it % 500 == 0:
            print("proposal step %d loss %.3e" % (it, float(loss.item())), flush=True)
    last = float(loss.item())
    prop.repack()
    # held-out camera 0 of the benchmark's 8 (seed of the scene's cameras), whole frame on the GPU
    o, d = synth.camera_rays(synth.make_cameras(1, cfg.seed_cameras, cfg.width, cfg.height)[0])
    R = o.shape[1]
    od, dd = to_dev(o), to_dev(d)
    rgb = torch.empty((R, 3), device=dev)
    am.amnerf_render(ctx.h, tree.h, mlp16.desc, od, dd, cfg.s_max, rgb, None, None, None, cfg.ert_eps,
                     proposal=prop.descriptor(am.AMNERF_BF16, mass_thresh=0.99, cap=48))
    torch.cuda.synchronize()
    st = am.amnerf_render_stats_get(ctx.h)
    pick = np.sort(np.random.default_rng(2024).choice(R, 6000, replace=False))
    ref, _, _, _, _ = oracle.render(scene.otree, scene.W, cfg.n_hidden, cfg.hidden, o, d, cfg.s_max,
                                    eps=cfg.ert_eps, ray_idx=pick)
    got = rgb.cpu().numpy().astype(np.float64)[pick]
    psnr = oracle.psnr(got, ref)
    print("headline bf16 + proposal: loss %.3e -> %.3e; %d samples (plain %d), %d fallback rays; "
          "PSNR %.2f dB against the oracle on %d rays, max |rgb - oracle| %.3e"
          % (first, last, st["n_samples"], st["n_plain_samples"], st["n_fallback"], psnr, len(pick),
             np.abs(got - ref).max()), flush=True)
    assert last < 0.5 * first
    assert st["n_samples"] < 0.5 * st["n_plain_samples"]
    assert psnr >= PSNR_TARGET_DB
