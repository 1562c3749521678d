"""The allocation-free render (amnerf_render_static, for callers that cannot allocate device
memory) against amnerf_render: bit-identical outputs and statistics on two calls in a row,
the second smaller; oversize calls and proposal renders rejected before any work; no device
memory allocated by the call."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from scene_util import Scene, gpu_setup, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2310_01881_amd as am  # noqa: E402


def outputs(R, s_max=None):
    dev = "cuda:0"
    out = [torch.full((R, 3), -1.0, device=dev), torch.full((R,), -1.0, device=dev),
           torch.full((R,), -1.0, device=dev)]
    out.append(None if s_max is None else torch.full((R * s_max,), -1.0, device=dev))
    return out


C2_SMALL = synth.scaled(synth.C2, grid_n=64, max_leaves=64, max_depth=12)


@pytest.mark.parametrize("cfg,dtype,sizes,weights", [
    (synth.C1, am.AMNERF_F32, (4096, 1000), True),
    (C2_SMALL, am.AMNERF_BF16, (6000, 2500), False),
    (C2_SMALL, am.AMNERF_FP8_ACT, (6000, 2500), False),
])
def test_static_render_equals_render(cfg, dtype, sizes, weights):
    scene = Scene(cfg)
    ctx, tree, mlp = gpu_setup(scene, dtype)
    ctx_ref = am.Context(0)
    o_all, d_all = synth.rays_for_cameras(synth.make_cameras(2, cfg.seed_cameras, 80, 80))
    for n in sizes:
        print("static render: %s, %d rays" % (cfg.name, n), flush=True)
        o, d = to_dev(o_all[:, :n]), to_dev(d_all[:, :n])
        ref = outputs(n, cfg.s_max if weights else None)
        got = outputs(n, cfg.s_max if weights else None)
        am.amnerf_render(ctx_ref.h, tree.h, mlp.desc, o, d, cfg.s_max, *ref, cfg.ert_eps)
        am.amnerf_render_static(ctx.h, tree.h, mlp.desc, o, d, cfg.s_max, *got, cfg.ert_eps)
        torch.cuda.synchronize()
        for name, a, b in zip(("rgb", "depth", "opacity", "weights"), got, ref):
            if b is not None:
                assert torch.equal(a, b), (n, name)
        st, st_ref = am.amnerf_render_stats_get(ctx.h), am.amnerf_render_stats_get(ctx_ref.h)
        for k in ("n_rays", "n_intervals", "n_samples", "n_chunks", "n_composited", "n_nonfinite"):
            assert st[k] == st_ref[k], (n, k)
        assert st["n_samples"] > 0
    # the static render's arrays live in the shared workspace: no inspection or backward
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render_inspect(ctx.h, ray_smp_off=torch.empty(sizes[-1] + 1, dtype=torch.int32, device="cuda:0"))
    assert e.value.code == am.AMNERF_ESTATE


def test_static_render_rejects_oversize_and_proposal():
    scene = Scene(C2_SMALL)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_BF16)
    cap = am.amnerf_render_static_capacity()
    assert cap == 64 << 20
    # about 20 + 40 min(s_max, L) + 28 s_max bytes per ray: 30 000 rays need > 64 MiB
    R = 30000
    o = torch.zeros((3, R), device="cuda:0")
    d = torch.zeros((3, R), device="cuda:0")
    d[2] = 1.0
    got = outputs(R)
    with pytest.raises(am.AmnerfError) as e:
        am.amnerf_render_static(ctx.h, tree.h, mlp.desc, o, d, cfg.s_max, *got, cfg.ert_eps)
    assert e.value.code == am.AMNERF_ECAPACITY and "needs" in am.amnerf_last_error()
    torch.cuda.synchronize()
    assert torch.all(got[0] == -1.0)             # nothing was enqueued
    prop = am.Proposal(ctx, torch.from_numpy(synth.make_prop_weights(1)).to("cuda:0"))
    rays = am.amnerf_rays(o.data_ptr(), d.data_ptr(), 16)
    prm = am.amnerf_render_params(cfg.s_max, cfg.ert_eps, 0, 0, am.C.pointer(prop.descriptor()), 0.0, None)
    out = am.amnerf_render_out(got[0].data_ptr(), None, None, None)
    rc = am.lib().amnerf_render_static(ctx.h, tree.h, am.C.byref(mlp.desc), am.C.byref(rays), am.C.byref(prm),
                                       am.C.byref(out), None)
    assert rc == am.AMNERF_EINVAL


def test_static_render_allocates_no_device_memory():
    scene = Scene(synth.C1)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    o, d = (to_dev(a) for a in scene.camera_rays())
    R = o.shape[1]
    got = outputs(R)
    am.amnerf_render_static(ctx.h, tree.h, mlp.desc, o, d, cfg.s_max, *got, cfg.ert_eps)   # warm-up
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        am.amnerf_render_static(ctx.h, tree.h, mlp.desc, o, d, cfg.s_max, *got, cfg.ert_eps)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    print("device memory free before / after three static renders: %d / %d" % (free0, free1), flush=True)
    assert free1 == free0
