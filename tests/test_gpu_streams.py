"""Frames in flight: two library contexts, each on its own stream (default priority), render
camera frames back to back with no host synchronisation between them; every output is
bit-identical to the same camera rendered alone.  Plain, with hierarchical sampling, with
empty space skipped and with a (untrained) proposal (the tree, the MLP, the occupancy grid and
the proposal are shared, read only)."""
from __future__ import annotations

import pytest

import synth
from scene_util import Scene, gpu_setup, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2310_01881_amd as am  # noqa: E402


@pytest.mark.parametrize("mode", ["plain", "hcheck", "ess", "proposal"])
def test_two_contexts_on_two_streams(mode):
    scene = Scene(synth.C1, footprint=0.5 if mode == "hcheck" else 0.0)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_BF16)
    ctx2 = am.Context(0)
    kw = {}
    if mode == "hcheck":
        kw["hcheck_footprint"] = scene.footprint
    elif mode == "ess":
        kw["occupancy"] = am.Occupancy(ctx, scene.grid, cfg.grid_n, 2, 0.01)
    elif mode == "proposal":
        prop = am.Proposal(ctx, torch.from_numpy(synth.make_prop_weights(1)).to("cuda:0"))
        kw["proposal"] = prop.descriptor(am.AMNERF_BF16, 0.99, 48)
    n_cams = 4
    rays = [tuple(to_dev(a) for a in scene.camera_rays(i)) for i in range(n_cams)]
    alone = [am.render(ctx, tree, mlp, o, d, cfg.s_max, ert_eps=cfg.ert_eps, **kw) for o, d in rays]
    torch.cuda.synchronize()
    streams = [torch.cuda.current_stream(), torch.cuda.Stream()]
    streams[1].wait_stream(streams[0])
    ctxs = [ctx, ctx2]
    frames = []
    for k in range(4 * n_cams):
        q = k % 2
        o, d = rays[k % n_cams]
        frames.append(am.render(ctxs[q], tree, mlp, o, d, cfg.s_max, ert_eps=cfg.ert_eps, stream=streams[q], **kw))
    torch.cuda.synchronize()
    for c in ctxs:
        am.amnerf_render_stats_get(c.h)
    for k, out in enumerate(frames):
        for name in ("rgb", "depth", "opacity"):
            assert torch.equal(out[name], alone[k % n_cams][name]), (mode, k, name)
    print("%s: %d frames on two streams bit-identical to the frames alone" % (mode, len(frames)), flush=True)


def test_weights_on_a_side_stream():
    """render() on a stream other than the current one: the per-sample weights are cleared
    on that stream before the render writes them, so every frame's weights equal the weights
    of the same frame rendered on the current stream."""
    scene = Scene(synth.C1)
    cfg = scene.cfg
    ctx, tree, mlp = gpu_setup(scene, am.AMNERF_F32)
    rays = [tuple(to_dev(a) for a in scene.camera_rays(i)) for i in range(3)]
    alone = [am.render(ctx, tree, mlp, o, d, cfg.s_max, ert_eps=cfg.ert_eps, weights=True) for o, d in rays]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    ctx2 = am.Context(0)
    outs = [am.render(ctx2, tree, mlp, o, d, cfg.s_max, ert_eps=cfg.ert_eps, weights=True, stream=side)
            for o, d in rays for _ in range(2)]
    torch.cuda.synchronize()
    for k, out in enumerate(outs):
        for name in ("rgb", "depth", "opacity", "weights"):
            assert torch.equal(out[name], alone[k // 2][name]), (k, name)
