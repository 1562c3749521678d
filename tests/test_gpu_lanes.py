"""Render lanes: a call of five passes gives bit-identical outputs and statistics whatever
the number of passes in flight (1 to 4 lanes), plain and with empty space skipped (whose
passes wait on the host for their interval counts); out-of-range lane counts are rejected."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from scene_util import Scene, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2310_01881_amd as am  # noqa: E402


@pytest.mark.parametrize("mode", ["plain", "ess"])
def test_outputs_do_not_depend_on_the_lane_count(mode):
    cfg = synth.scaled(synth.C1, n_hidden=4, hidden=64)
    scene = Scene(cfg)
    ctx = am.Context(0)
    tree = am.Tree(ctx, scene.grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves, 0)
    mlp = am.Mlp(ctx, to_dev(scene.W), cfg.n_hidden, 64, am.AMNERF_BF16, scene.n_sets)
    kw = {"occupancy": am.Occupancy(ctx, scene.grid, cfg.grid_n, 2, 0.01)} if mode == "ess" else {}
    o, d = scene.camera_rays()
    od = to_dev(o).repeat(1, 1100).contiguous()
    dd = to_dev(d).repeat(1, 1100).contiguous()
    R = od.shape[1]
    chunk = (1 << 28) // 255
    assert 4 * chunk < R < 5 * chunk
    ref = st_ref = None
    for lanes in (4, 1, 2, 3):
        print("lanes %d, %s: rays %d" % (lanes, mode, R), flush=True)
        am.amnerf_ctx_set_render_lanes(ctx.h, lanes)
        out = am.render(ctx, tree, mlp, od, dd, 255, ert_eps=cfg.ert_eps, **kw)
        torch.cuda.synchronize()
        st = am.amnerf_render_stats_get(ctx.h)
        assert st["n_chunks"] == 5 and st["n_nonfinite"] == 0 and st["n_unreached"] == 0
        if ref is None:
            ref, st_ref = out, st
            continue
        for k in ("rgb", "depth", "opacity"):
            assert torch.equal(out[k], ref[k]), (lanes, k)
        for k in ("n_intervals", "n_samples", "n_composited", "n_placed_samples"):
            assert st[k] == st_ref[k], (lanes, k)
    assert float(ref["opacity"].max()) > 0.5
    for bad in (0, am.AMNERF_MAX_RENDER_LANES + 1):
        with pytest.raises(am.AmnerfError) as e:
            am.amnerf_ctx_set_render_lanes(ctx.h, bad)
        assert e.value.code == am.AMNERF_EINVAL
