#!/usr/bin/env python3
"""Rendering throughput of the adaptive multi-NeRF hot path on one MI355X.

One step renders one 800x800 frame (640 000 rays) of the seeded 128^3-grid scene with a
512-leaf KD tree and 4x64 per-leaf MLPs, at most 128 samples per ray, through the whole
path: traversal -> (learned proposal) -> per-leaf samples -> sort by leaf -> grouped MLP
-> compositing.  Rays of 8 held-out cameras are resident in HBM before the timed region;
step k renders camera k mod 8.  Seven paths are timed: plain float32, plain bfloat16,
bfloat16 with the learned proposal (bfloat16 inference, <= 48 samples per ray, fallback
below 0.99 predicted mass), float8 (e4m3) leaf weights without and with the proposal, and
plain float32 and bfloat16 with early termination in 64-sample rounds (terminated rays
drop out before the leaf MLPs).  The proposal is first trained (untimed) by the library's
own kernels on plain-render targets from 200 seeded training cameras.  Each path is timed
one frame at a time (an event after every frame; the median frame is reported, with
per-stage event timing), then with --inflight frames in flight (one library context per
stream, frame k on stream k mod N; --windows windows of --steps frames, the median window
reported; every frame is still rendered in full, and the last frame of each stream is
checked bit-identical to the same camera rendered alone).  `value` is the proposal path's
samples/s (samples evaluated by the leaf MLPs) with frames in flight, and `ms_per_step`
its ms/frame.  The oracle (float64, CPU, on every host core the process is given)
renders a bounded random subset of camera 0's rays: that gives the CPU baseline and the
PSNR of each GPU path against the oracle.  The same scene is also rendered with a
regular-subdivision tree (the ablation without the adaptive split) and with hierarchical
sampling at three footprints, and a training step is timed (median step, per-stage
events, the MLP backward's roofline, and the oracle's training step as its CPU baseline).

A second, larger workload follows in the same run and is reported under `large_scene`
(skip it with --no-large): 1920x1080 frames of a 256^3-grid scene with a 100:1 blob-density
skew, a 4096-leaf tree, float8 (and bfloat16) leaf weights and S_max 192; one call renders
30 held-out cameras without a proposal (and with empty space skipped by an occupancy
grid), and one call renders 50 held-out cameras (the same first 30, then 20 more) with a
proposal trained on 200 other cameras (--large-paths picks a subset of these paths).  The
`fp8act` paths run float8 weights and activations on the float8 matrix cores, with
activation exponents from a calibration render of 2^20 pixels of 20 other cameras; they
are priced at the float8 peak and judged against the oracle's float8 model and against the
oracle on their own dequantised weights.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_SAMPLE_4x64 = 2 * (30 * 64 + 3 * 64 * 64 + 64 * 4)   # 28 928, unpadded
# backward per sample: the forward again (activations are recomputed, not stored), the input
# gradients of layers 1..4 (layer 0's input needs none) and every weight gradient
FLOP_PER_SAMPLE_BWD_4x64 = FLOP_PER_SAMPLE_4x64 + 2 * (3 * 64 * 64 + 64 * 4) + FLOP_PER_SAMPLE_4x64   # 82 944
PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0, "f32": 157.3}


HEADLINE_PSNR_DB = 45.0   # the headline path's quality bar against the oracle
PROPOSAL_TEST_CAMERAS = 50   # held-out cameras of the large scene's proposal renders


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def host_cpus():
    """Host cores this process may run on (what nproc prints)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_threads():
    """Threads for the oracle: every host core of the process, unless OMP_NUM_THREADS gives the
    process a smaller CPU share (then that share)."""
    n = host_cpus()
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def median(xs):
    xs = sorted(xs)
    k = len(xs)
    return 0.5 * (xs[(k - 1) // 2] + xs[k // 2])


LARGE_PATHS = ("fp8", "fp8_prop", "bf16", "bf16_prop", "fp8_untrained_prop", "fp8_ess", "fp8act", "fp8act_prop")


def large_scene(args, am, torch, np, synth, ctx):
    """The 1920x1080 scene: 256^3 grid with a 100:1 blob-density skew, 4096-leaf tree,
    4x64 leaf MLPs with float8 weights, S_max 192.  30 held-out cameras are rendered by one
    call (62.2 M rays, processed in chunks of at most 2^28 / S_max rays); a proposal is
    trained on 200 other cameras.  Accuracy against the oracle on a seeded 1/64 pixel
    subset of camera 0; the proposal's error against the plain float8 render on every pixel
    of the 30 cameras (the plain renderer judges it)."""
    cfg = synth.C3
    dev = "cuda:0"
    am.amnerf_ctx_set_render_lanes(ctx.h, args.lanes)
    t0 = time.perf_counter()
    grid = synth.make_grid(cfg)
    tree = am.Tree(ctx, grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
    L = tree.n_leaves
    dens = synth.leaf_mean_density(grid, cfg.grid_n, tree.leaf_boxes())
    W = synth.make_weights(L, cfg.n_hidden, cfg.hidden, cfg.seed_weights, dens)
    master = torch.from_numpy(W).to(dev)
    mlps = {k: am.Mlp(ctx, master, cfg.n_hidden, cfg.hidden, dt, L)
            for k, dt in (("fp8", am.AMNERF_FP8), ("bf16", am.AMNERF_BF16), ("f32", am.AMNERF_F32))}
    wanted = [k for k in LARGE_PATHS if k in args.large_paths.split(",")]
    calibration = None
    act_max = None
    if any(k.startswith("fp8act") for k in wanted):
        # float8 activations on the matrix cores: activation exponents from the calibration
        # maxima of a bfloat16 render of 2^20 random pixels of 20 other cameras (untimed)
        t0 = time.perf_counter()
        cal_cams = synth.make_cameras(20, cfg.seed_batches + 3, cfg.width, cfg.height)
        co, cd = synth.random_pixel_rays(cal_cams, 1 << 20, cfg.seed_batches + 4)
        co, cd = torch.from_numpy(co).to(dev), torch.from_numpy(cd).to(dev)
        cal_rgb = torch.empty((co.shape[1], 3), dtype=torch.float32, device=dev)
        am.amnerf_render(ctx.h, tree.h, mlps["bf16"].desc, co, cd, cfg.s_max, cal_rgb, None, None, None, cfg.ert_eps)
        act_max = torch.zeros((L, cfg.n_hidden), dtype=torch.float32, device=dev)
        am.amnerf_mlp_calibrate(ctx.h, cfg.n_hidden, L, master, co, cd, act_max)
        mlps["fp8act"] = am.Mlp(ctx, master, cfg.n_hidden, cfg.hidden, am.AMNERF_FP8_ACT, L, act_max_dev=act_max)
        torch.cuda.synchronize()
        unseen = int((act_max.max(dim=1).values == 0).sum())
        del co, cd, cal_rgb
        calibration = {"rays": 1 << 20, "cameras": 20, "seconds": time.perf_counter() - t0,
                       "leaves_without_samples": unseen}
        log("large calibration: %s" % calibration)
    # 50 held-out cameras: the proposal paths render all of them in one call; the paths
    # without a proposal render the first 30 (the same seeds) in one call
    n_cams = cfg.n_cameras
    n_prop_cams = PROPOSAL_TEST_CAMERAS
    cams = synth.make_cameras(n_prop_cams, cfg.seed_cameras, cfg.width, cfg.height)
    R1 = cfg.width * cfg.height
    R = R1 * n_cams
    R50 = R1 * n_prop_cams
    o50 = torch.empty((3, R50), dtype=torch.float32, device=dev)
    d50 = torch.empty((3, R50), dtype=torch.float32, device=dev)
    for i, c in enumerate(cams):
        o, d = synth.camera_rays(c)
        o50[:, i * R1:(i + 1) * R1] = torch.from_numpy(o).to(dev)
        d50[:, i * R1:(i + 1) * R1] = torch.from_numpy(d).to(dev)
    o_all, d_all = o50[:, :R].contiguous(), d50[:, :R].contiguous()
    log("large scene %s: %d leaves, %d rays per call (%d with a proposal), set-up %.1f s" % (
        cfg.name, L, R, R50, time.perf_counter() - t0))

    prop_training = None
    prop = desc = desc_untrained = None
    if any(k.endswith("_prop") for k in wanted):
        # proposal trained on 200 other cameras (untimed)
        t0 = time.perf_counter()
        prop = am.Proposal(ctx, torch.from_numpy(synth.make_prop_weights(cfg.seed_proposal)).to(dev))
        untrained = am.Proposal(ctx, torch.from_numpy(synth.make_prop_weights(cfg.seed_proposal)).to(dev))
        untrained.repack()
        train_cams = synth.make_cameras(200, cfg.seed_batches, cfg.width, cfg.height)
        pool_o, pool_d = synth.random_pixel_rays(train_cams, 2_000_000, cfg.seed_batches + 1)
        pool_o, pool_d = torch.from_numpy(pool_o).to(dev), torch.from_numpy(pool_d).to(dev)
        gen = torch.Generator(device=dev).manual_seed(cfg.seed_batches + 2)
        losses = []
        for it in range(args.large_prop_steps):
            lr = 3e-3 if it < 0.7 * args.large_prop_steps else 1e-3
            idx = torch.randint(0, pool_o.shape[1], (args.prop_batch,), device=dev, generator=gen)
            loss = prop.train_step(tree, mlps["f32"].desc, pool_o[:, idx].contiguous(),
                                   pool_d[:, idx].contiguous(), cfg.s_max, lr=lr)
            if it % 1000 == 0 or it == args.large_prop_steps - 1:
                losses.append(float(loss.item()))
        prop.repack()
        torch.cuda.synchronize()
        t_prop = time.perf_counter() - t0
        del pool_o, pool_d
        log("large proposal: %d steps in %.1f s, loss %s" % (args.large_prop_steps, t_prop,
                                                              ["%.2e" % v for v in losses]))
        desc = prop.descriptor(am.AMNERF_BF16, mass_thresh=0.99, cap=48)
        desc_untrained = untrained.descriptor(am.AMNERF_BF16, mass_thresh=0.99, cap=48)
        prop_training = {"steps": args.large_prop_steps, "rays_per_step": args.prop_batch, "cameras": 200,
                         "seconds": t_prop, "loss_first_last": [losses[0], losses[-1]] if losses else None}

    # empty-space skipping: occupancy at half the guidance resolution, 1 % of the peak density
    occ = am.Occupancy(ctx, grid, cfg.grid_n, 2, 0.01)
    paths = {"fp8": ("fp8", None, None), "fp8_prop": ("fp8", desc, None), "bf16": ("bf16", None, None),
             "bf16_prop": ("bf16", desc, None), "fp8_untrained_prop": ("fp8", desc_untrained, None),
             "fp8_ess": ("fp8", None, occ), "fp8act": ("fp8act", None, None), "fp8act_prop": ("fp8act", desc, None)}
    paths = {k: paths[k] for k in wanted}

    def cams_of(kind):
        return n_prop_cams if kind.endswith("_prop") else n_cams
    outs = {k: torch.empty((R1 * cams_of(k), 3), dtype=torch.float32, device=dev) for k in paths}

    def render(kind, rgb, n_c=None):
        mk, pd, oc = paths[kind]
        o, d = (o50, d50) if (n_c or cams_of(kind)) == n_prop_cams else (o_all, d_all)
        am.amnerf_render(ctx.h, tree.h, mlps[mk].desc, o, d, cfg.s_max, rgb, None, None, None, cfg.ert_eps,
                         proposal=pd, occupancy=oc)

    res = {}
    am.amnerf_ctx_set_timing(ctx.h, True)
    for kind in paths:
        rgb = outs[kind]
        nc = cams_of(kind)
        render(kind, rgb)                                    # warm-up, and the sample counts
        st = am.amnerf_render_stats_get(ctx.h)
        am.amnerf_timing_collect(ctx.h)
        calls = args.large_calls if kind != "fp8_untrained_prop" else 1
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(calls + 1)]
        evs[0].record()
        for c in range(calls):
            render(kind, rgb)
            evs[c + 1].record()
        torch.cuda.synchronize()
        dt = 1e-3 * median([evs[c].elapsed_time(evs[c + 1]) for c in range(calls)])
        stage_ms, npass = am.amnerf_timing_collect(ctx.h)
        mlp_ms = stage_ms["mlp"] / calls
        Rk = R1 * nc
        tf = FLOP_PER_SAMPLE_4x64 * st["n_samples"] / (mlp_ms * 1e-3) / 1e12
        act8 = paths[kind][0] == "fp8act"
        peak = PEAK_TFLOPS["fp8" if act8 else "bf16"]
        kname = ("k_mlp8<4> (e4m3 weights and activations; first layer bf16)" if act8 else "k_mlp<64,bf16>"
                 + (" (e4m3 weights widened on chip)" if paths[kind][0] == "fp8" else ""))
        res[kind] = {"ms_per_frame": 1e3 * dt / nc, "ms_per_call": 1e3 * dt, "cameras_per_call": nc,
                     "samples_per_s": st["n_samples"] / dt, "samples_per_frame": st["n_samples"] / nc,
                     "composited_samples_per_frame": st["n_composited"] / nc,
                     "samples_per_ray": st["n_samples"] / Rk, "fallback_fraction": st["n_fallback"] / Rk,
                     "chunks_per_call": st["n_chunks"],
                     "stage_ms_per_frame": {k: v / calls / nc for k, v in stage_ms.items()},
                     "mlp_tflops": tf,
                     "roofline": {"bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s",
                                  "frac": tf / peak, "traffic": None, "kernel": kname, "kernel_ms_per_call": mlp_ms}}
        log("large %s: %.3f ms/frame (%d cameras per call, median of %d calls), %.3e samples/s, %.1f samples/ray, "
            "fallback %.3f, MLP %.3f of peak, stages %s" % (
                kind, res[kind]["ms_per_frame"], nc, calls, res[kind]["samples_per_s"], res[kind]["samples_per_ray"],
                res[kind]["fallback_fraction"], tf / peak,
                {k: round(v, 4) for k, v in res[kind]["stage_ms_per_frame"].items()}))
    am.amnerf_ctx_set_timing(ctx.h, False)

    # each proposal render judged by the plain render with the same leaf weights, every pixel
    # of its cameras (the outputs of the last timed call; the plain render of the 50 cameras
    # is made for this, untimed)
    psnr_prop_vs_plain = {}
    plain50 = {}
    for kind, ref in (("fp8_prop", "fp8"), ("bf16_prop", "bf16"), ("fp8_untrained_prop", "fp8"), ("fp8_ess", "fp8"),
                      ("fp8act_prop", "fp8act")):
        if kind not in outs or ref not in paths:
            continue
        if cams_of(kind) == n_prop_cams:
            if ref not in plain50:
                plain50[ref] = torch.empty((R50, 3), dtype=torch.float32, device=dev)
                render(ref, plain50[ref], n_prop_cams)
            ref_rgb = plain50[ref]
        else:
            ref_rgb = outs[ref]
        rep = am.amnerf_error_stats(ctx.h, outs[kind].view(-1), ref_rgb.view(-1).double())
        psnr_prop_vs_plain[kind] = rep["psnr"]
    del plain50
    log("large proposal psnr vs plain: %s" % {k: round(v, 2) for k, v in psnr_prop_vs_plain.items()})

    # bucket sizes of one single-chunk pass (plain e4m3): the first 2^20 rays of camera 0
    spread = None
    if "fp8" in outs:
        n_sub = 1 << 20
        o_sub, d_sub = o_all[:, :n_sub].contiguous(), d_all[:, :n_sub].contiguous()
        sub_rgb = torch.empty((n_sub, 3), dtype=torch.float32, device=dev)
        am.amnerf_render(ctx.h, tree.h, mlps["fp8"].desc, o_sub, d_sub, cfg.s_max, sub_rgb, None, None, None,
                         cfg.ert_eps)
        st = am.amnerf_render_stats_get(ctx.h)
        ns = st["n_samples"]
        bo = torch.empty(L + 1, dtype=torch.int32, device=dev)
        am.amnerf_render_inspect(ctx.h, bucket_off=bo)
        sizes = np.diff(bo.cpu().numpy().astype(np.int64))
        nz = sizes[sizes > 0]
        spread = {"rays": n_sub, "samples": int(ns), "leaves_nonempty": int(nz.size),
                  "min": int(nz.min()), "p1": float(np.percentile(nz, 1)), "median": float(np.median(nz)),
                  "p99": float(np.percentile(nz, 99)), "max": int(nz.max()),
                  "max_over_min_nonempty": float(nz.max() / nz.min()),
                  "p99_over_p1": float(np.percentile(nz, 99) / max(np.percentile(nz, 1), 1))}
        log("large bucket sizes: %s" % spread)

    acc = None
    acc_kinds = [k for k in ("fp8", "fp8_prop", "fp8_ess", "fp8act", "fp8act_prop") if k in outs]
    if not args.no_cpu and acc_kinds:
        import oracle
        from oracle import fp8 as ofp8
        otree = oracle.build_tree(grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
        assert np.array_equal(otree.rows, tree.rows)
        o0, d0 = synth.camera_rays(cams[0])
        sel = np.sort(np.random.default_rng(64).choice(R1, R1 // 64, replace=False))
        threads = cpu_threads()
        t0 = time.perf_counter()
        rgb_o, _, _, ns_o, _ = oracle.render(otree, W, cfg.n_hidden, cfg.hidden, o0, d0, cfg.s_max, eps=cfg.ert_eps,
                                             ray_idx=sel, threads=threads)
        t_o = time.perf_counter() - t0
        cpu_plain = {"value": float(ns_o.sum()) / t_o, "unit": "samples/s", "cores": threads, "kind": "oracle",
                     "host_cpus": host_cpus(),
                     "sample": "seeded 1/64 pixel subset of camera 0 (%d rays, %d samples), float64 plain render, "
                               "%.1f s" % (sel.size, int(ns_o.sum()), t_o)}
        _, _, deq = ofp8.quantise(W, cfg.n_hidden, cfg.hidden)
        rgb_q, _, _, _, _ = oracle.render(otree, deq.astype(np.float32), cfg.n_hidden, cfg.hidden, o0, d0, cfg.s_max,
                                          eps=cfg.ert_eps, ray_idx=sel, threads=threads)
        rgb_qa = rgb_q8 = None
        if act_max is not None:
            # the float8 matrix-core model: its own (power-of-two) weight quantisation, with
            # float64 activations, and with float8 activations on the same exponents
            _, k_act, deq_a = ofp8.quantise_mma(W, cfg.n_hidden, cfg.hidden, act_max.cpu().numpy())
            rgb_qa, _, _, _, _ = oracle.render(otree, deq_a, cfg.n_hidden, cfg.hidden, o0, d0, cfg.s_max,
                                               eps=cfg.ert_eps, ray_idx=sel, threads=threads)
            rgb_q8, _, _ = oracle.render_q8(otree, deq_a, cfg.n_hidden, cfg.hidden, o0, d0, cfg.s_max, k_act,
                                            eps=cfg.ert_eps, ray_idx=sel, threads=threads)
        sel_dev = torch.from_numpy(sel).to(dev)
        acc = {"rays": int(sel.size), "sample": "seeded 1/64 pixel subset of camera 0"}

        def psnr_vs(x, ref):
            return am.amnerf_error_stats(ctx.h, x, torch.from_numpy(np.ascontiguousarray(ref)).to(dev).view(-1))["psnr"]
        for kind in acc_kinds:
            x = outs[kind][:R1][sel_dev].contiguous().view(-1)
            acc["psnr_%s_vs_oracle_db" % kind] = psnr_vs(x, rgb_o)
            if kind.startswith("fp8act"):
                acc["psnr_%s_vs_oracle_fp8_weights_db" % kind] = psnr_vs(x, rgb_qa)
                acc["psnr_%s_vs_oracle_fp8_model_db" % kind] = psnr_vs(x, rgb_q8)
            else:
                acc["psnr_%s_vs_oracle_fp8_weights_db" % kind] = psnr_vs(x, rgb_q)
        log("large accuracy: %s" % acc)
        if "fp8" in res:
            res["fp8"]["cpu_baseline"] = cpu_plain
        if "fp8_prop" in res:
            # the proposal render on the oracle (float64 proposal network, selection and leaf
            # MLPs), over a bounded random subset of camera 0
            pm = prop.master.cpu().numpy()
            prng = np.random.default_rng(6464)

            def oracle_prop(idx):
                return oracle.render_proposal(otree, W, cfg.n_hidden, cfg.hidden, pm, o0, d0, cfg.s_max,
                                              eps=cfg.ert_eps, mass_thresh=0.99, cap=48, ray_idx=idx,
                                              threads=threads)[3]
            idx = np.sort(prng.choice(R1, 4000, replace=False))
            t0 = time.perf_counter()
            oracle_prop(idx)
            per_ray = (time.perf_counter() - t0) / idx.size
            n_p = int(min(R1, max(4000, 0.5 * args.cpu_seconds / max(per_ray, 1e-9))))
            idx = np.sort(prng.choice(R1, n_p, replace=False))
            t0 = time.perf_counter()
            ns_p = oracle_prop(idx)
            t_p = time.perf_counter() - t0
            res["fp8_prop"]["cpu_baseline"] = {
                "value": float(ns_p.sum()) / t_p, "unit": "samples/s", "cores": threads, "kind": "oracle",
                "host_cpus": host_cpus(),
                "sample": "%d random rays of held-out camera 0 (%d samples), float64 proposal render (float32 "
                          "leaf weights), %.1f s" % (n_p, int(ns_p.sum()), t_p)}
            log("large oracle: plain %.3e, proposal %.3e samples/s on %d threads" % (
                cpu_plain["value"], res["fp8_prop"]["cpu_baseline"]["value"], threads))

    return {"workload": "1920x1080 frames, 256^3 guidance grid (2000 anisotropic blobs, 100:1 density skew), "
                        "%d-leaf KD tree (max depth 12), 4x64 leaf MLPs, <=192 samples/ray, ERT at T<1e-4; "
                        "%d held-out cameras rendered by one call (%d with the proposal)" % (L, n_cams, n_prop_cams),
            "n_leaves": L, "rays_per_call": R, "cameras_per_call": n_cams, "render_lanes": args.lanes,
            "proposal_rays_per_call": R50, "proposal_cameras_per_call": n_prop_cams, "paths": res,
            "occupancy": {"cells": occ.g ** 3, "occupied": occ.n_occupied, "block": 2, "thresh": 0.01},
            "psnr_vs_plain_db": psnr_prop_vs_plain, "bucket_sizes": spread, "accuracy": acc,
            "proposal_training": prop_training, "fp8act_calibration": calibration}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prop-steps", type=int, default=1500, help="proposal training steps (untimed)")
    ap.add_argument("--prop-batch", type=int, default=32768)
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target oracle time")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--train-steps", type=int, default=20, help="timed training steps (0: skip)")
    ap.add_argument("--paths", default="f32,bf16,bf16_prop,fp8,fp8_prop,f32_rounds,bf16_rounds",
                    help="comma-separated render paths to time (the headline bf16_prop is always timed)")
    ap.add_argument("--train-batch", type=int, default=262144)
    ap.add_argument("--no-large", action="store_true", help="skip the 1920x1080 4096-leaf scene")
    ap.add_argument("--large-calls", type=int, default=3, help="timed 30-camera calls of the large scene")
    ap.add_argument("--lanes", type=int, default=4,
                    help="render lanes of the large scene's multi-chunk calls (chunks in flight at once)")
    ap.add_argument("--large-prop-steps", type=int, default=6000, help="proposal training steps, large scene")
    ap.add_argument("--large-paths", default=",".join(LARGE_PATHS),
                    help="comma-separated render paths of the large scene (each PSNR comparison needs its "
                         "plain reference path too)")
    ap.add_argument("--ablation-steps", type=int, default=400,
                    help="training steps per student of the ablation's quality comparison (0: skip)")
    ap.add_argument("--inflight", type=int, default=3,
                    help="frames in flight for the throughput line: contexts on streams of their own")
    ap.add_argument("--windows", type=int, default=5,
                    help="timed windows of --steps frames with frames in flight (the median is reported)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (rays would shard "
              "across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)
    bad = set(args.large_paths.split(",")) - set(LARGE_PATHS)
    if bad:
        ap.error("unknown --large-paths entries %s (known: %s)" % (sorted(bad), ",".join(LARGE_PATHS)))

    import numpy as np
    import torch

    import paper_2310_01881_amd as am
    import synth

    cfg = synth.C2
    dev = "cuda:0"
    log("scene %s" % cfg.name)
    grid = synth.make_grid(cfg)
    ctx = am.Context(0)
    tree = am.Tree(ctx, grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
    L = tree.n_leaves
    dens = synth.leaf_mean_density(grid, cfg.grid_n, tree.leaf_boxes())
    W = synth.make_weights(L, cfg.n_hidden, cfg.hidden, cfg.seed_weights, dens)
    master = torch.from_numpy(W).to(dev)
    mlps = {"f32": am.Mlp(ctx, master, cfg.n_hidden, cfg.hidden, am.AMNERF_F32, L),
            "bf16": am.Mlp(ctx, master, cfg.n_hidden, cfg.hidden, am.AMNERF_BF16, L),
            "fp8": am.Mlp(ctx, master, cfg.n_hidden, cfg.hidden, am.AMNERF_FP8, L)}
    n_cams = 8
    cams = synth.make_cameras(n_cams, cfg.seed_cameras, cfg.width, cfg.height)
    rays = []
    for c in cams:
        o, d = synth.camera_rays(c)
        rays.append((torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)))
    R = cfg.width * cfg.height

    # ---- learned proposal, trained by the library (untimed) ----
    t0 = time.perf_counter()
    prop = am.Proposal(ctx, torch.from_numpy(synth.make_prop_weights(cfg.seed_proposal)).to(dev))
    train_cams = synth.make_cameras(200, cfg.seed_batches, cfg.width, cfg.height)
    pool_o, pool_d = synth.random_pixel_rays(train_cams, 2_000_000, cfg.seed_batches + 1)
    pool_o, pool_d = torch.from_numpy(pool_o).to(dev), torch.from_numpy(pool_d).to(dev)
    gen = torch.Generator(device=dev).manual_seed(cfg.seed_batches + 2)
    losses = []
    for it in range(args.prop_steps):
        lr = 3e-3 if it < 0.7 * args.prop_steps else 1e-3
        idx = torch.randint(0, pool_o.shape[1], (args.prop_batch,), device=dev, generator=gen)
        loss = prop.train_step(tree, mlps["f32"].desc, pool_o[:, idx].contiguous(), pool_d[:, idx].contiguous(),
                               cfg.s_max, lr=lr)
        if it % 100 == 0 or it == args.prop_steps - 1:
            losses.append(float(loss.item()))
    prop.repack()
    torch.cuda.synchronize()
    t_prop = time.perf_counter() - t0
    log("proposal: %d steps of %d rays in %.1f s, loss %s" % (args.prop_steps, args.prop_batch, t_prop,
                                                             ["%.2e" % v for v in losses]))
    desc = prop.descriptor(am.AMNERF_BF16, mass_thresh=0.99, cap=48)

    # (leaf weights, proposal, early termination in 64-sample rounds)
    all_paths = {"f32": ("f32", None, False), "bf16": ("bf16", None, False), "bf16_prop": ("bf16", desc, False),
                 "fp8": ("fp8", None, False), "fp8_prop": ("fp8", desc, False),
                 "f32_rounds": ("f32", None, True), "bf16_rounds": ("bf16", None, True)}
    wanted = set(args.paths.split(",")) | {"bf16_prop"}
    paths = {k: v for k, v in all_paths.items() if k in wanted}
    outs = {k: {"rgb": torch.empty((R, 3), device=dev), "depth": torch.empty(R, device=dev),
                "opacity": torch.empty(R, device=dev)} for k in paths}

    def render(kind, cam):
        o, d = rays[cam]
        ob = outs[kind]
        mk, pd, rounds = paths[kind]
        am.amnerf_render(ctx.h, tree.h, mlps[mk].desc, o, d, cfg.s_max, ob["rgb"], ob["depth"], ob["opacity"],
                         None, cfg.ert_eps, proposal=pd, ert_rounds=rounds)

    # samples per camera (untimed): evaluated by the leaf MLPs, and composited (in front of
    # each ray's termination)
    samples = {k: [] for k in paths}
    composited = {k: [] for k in paths}
    fallback, plain = [], []
    for kind in paths:
        for cam in range(n_cams):
            render(kind, cam)
            st = am.amnerf_render_stats_get(ctx.h)
            samples[kind].append(st["n_samples"])
            composited[kind].append(st["n_composited"])
            if kind == "bf16_prop":
                fallback.append(st["n_fallback"])
                plain.append(st["n_plain_samples"])
    torch.cuda.synchronize()
    log("samples per frame: plain %s, proposal %s, fallback rays %s" % (plain, samples["bf16_prop"], fallback))

    # one frame at a time: an event after every frame on the render stream, the median frame
    # (GPU time between consecutive events) reported
    results = {}
    am.amnerf_ctx_set_timing(ctx.h, True)
    for kind in paths:
        for w in range(args.warmup):
            render(kind, w % n_cams)
        torch.cuda.synchronize()
        am.amnerf_timing_collect(ctx.h)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t0 = time.perf_counter()
        evs[0].record()
        for k in range(args.steps):
            render(kind, k % n_cams)
            evs[k + 1].record()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        frame_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
        stage_ms, npass = am.amnerf_timing_collect(ctx.h)
        n_s = sum(samples[kind][k % n_cams] for k in range(args.steps)) / args.steps
        n_c = sum(composited[kind][k % n_cams] for k in range(args.steps)) / args.steps
        mlp_ms = stage_ms["mlp"] / max(npass, 1)
        med = median(frame_ms)
        results[kind] = {
            "ms_per_frame": med,
            "ms_per_frame_mean": 1e3 * dt / args.steps,
            "ms_per_frame_min_max": [min(frame_ms), max(frame_ms)],
            "samples_per_s": n_s / (med * 1e-3),
            "samples_per_frame": n_s,
            "composited_samples_per_frame": n_c,
            "stage_ms_per_frame": {k: v / max(npass, 1) for k, v in stage_ms.items()},
            "mlp_ms": mlp_ms,
            "mlp_tflops": FLOP_PER_SAMPLE_4x64 * n_s / (mlp_ms * 1e-3) / 1e12,
        }
        log("%s: %.3f ms/frame (median of %d), %.3e samples/s, %.0f evaluated / %.0f composited samples, "
            "stages %s" % (kind, med, args.steps, results[kind]["samples_per_s"], n_s, n_c,
                           {k: round(v, 4) for k, v in results[kind]["stage_ms_per_frame"].items()}))
    am.amnerf_ctx_set_timing(ctx.h, False)

    # ---- frames in flight: one context per stream (the contexts share the tree and the
    #      weights, each has its own workspace), frame k on stream k mod N, so the host
    #      enqueues the next frame while the current one runs and one frame's latency-bound
    #      stages overlap another's matrix-core stage.  Every frame is rendered in full. ----
    inflight = None
    if args.inflight > 1:
        N = args.inflight
        ctxs = [ctx] + [am.Context(0) for _ in range(N - 1)]
        streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(N - 1)]
        iouts = [{"rgb": torch.empty((R, 3), device=dev), "depth": torch.empty(R, device=dev),
                  "opacity": torch.empty(R, device=dev)} for _ in range(N)]

        def prender(kind, cam, q):
            o, d = rays[cam]
            ob = iouts[q]
            mk, pd, rounds = paths[kind]
            am.amnerf_render(ctxs[q].h, tree.h, mlps[mk].desc, o, d, cfg.s_max, ob["rgb"], ob["depth"],
                             ob["opacity"], None, cfg.ert_eps, proposal=pd, stream=streams[q], ert_rounds=rounds)
        inflight = {"frames_in_flight": N, "windows": args.windows, "paths": {}}
        for kind in paths:
            for w in range(args.warmup):
                prender(kind, w % n_cams, w % N)
            torch.cuda.synchronize()
            # --windows timed windows of --steps frames each; the median window is reported
            wins = []
            for _ in range(args.windows):
                t0 = time.perf_counter()
                for k in range(args.steps):
                    prender(kind, k % n_cams, k % N)
                torch.cuda.synchronize()
                wins.append(time.perf_counter() - t0)
            dt = median(wins)
            n_s = sum(samples[kind][k % n_cams] for k in range(args.steps))
            # the last frame of each stream equals the same camera rendered alone
            same = True
            for q in range(N):
                k = args.steps - 1 - ((args.steps - 1 - q) % N)
                render(kind, k % n_cams)
                torch.cuda.synchronize()
                same = same and all(torch.equal(iouts[q][c], outs[kind][c]) for c in ("rgb", "depth", "opacity"))
            inflight["paths"][kind] = {"ms_per_frame": 1e3 * dt / args.steps, "samples_per_s": n_s / dt,
                                       "window_ms_per_frame": [1e3 * x / args.steps for x in wins],
                                       "identical_to_single_stream": bool(same)}
            log("%s, %d frames in flight: %.3f ms/frame, %.3e samples/s, outputs identical: %s" % (
                kind, N, 1e3 * dt / args.steps, n_s / dt, same))
            if not same:
                raise SystemExit("frames in flight changed a render")
        del ctxs[1:]

    # ---- ablation without the adaptive subdivision: the same grid under a regular tree of as
    #      many leaves (middle planes, breadth-first), plain bf16 render, same cameras ----
    ablation = None
    if "bf16" in paths:
        rtree = am.Tree(ctx, grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves, am.AMNERF_SPLIT_MIDDLE)
        rdens = synth.leaf_mean_density(grid, cfg.grid_n, rtree.leaf_boxes())
        rW = synth.make_weights(rtree.n_leaves, cfg.n_hidden, cfg.hidden, cfg.seed_weights, rdens)
        rmlp = am.Mlp(ctx, torch.from_numpy(rW).to(dev), cfg.n_hidden, cfg.hidden, am.AMNERF_BF16, rtree.n_leaves)
        ob = outs["bf16"]

        def rrender(cam):
            o, d = rays[cam]
            am.amnerf_render(ctx.h, rtree.h, rmlp.desc, o, d, cfg.s_max, ob["rgb"], ob["depth"], ob["opacity"],
                             None, cfg.ert_eps)
        rs = []
        for cam in range(n_cams):
            rrender(cam)
            rs.append(am.amnerf_render_stats_get(ctx.h)["n_samples"])
        for w in range(args.warmup):
            rrender(w % n_cams)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            rrender(k % n_cams)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0

        def mass_spread(t):
            lv = t.mass[t.rows[:, 10] >= 0].astype(np.float64)
            return float(lv.max() / max(np.median(lv), 1.0))
        ablation = {"tree": "regular subdivision, %d leaves" % rtree.n_leaves, "path": "bf16, no proposal",
                    "ms_per_frame": 1e3 * dt / args.steps,
                    "samples_per_frame": float(np.mean(rs)),
                    "adaptive_ms_per_frame": results["bf16"]["ms_per_frame"],
                    "adaptive_samples_per_frame": results["bf16"]["samples_per_frame"],
                    "leaf_mass_max_over_median": mass_spread(rtree),
                    "adaptive_leaf_mass_max_over_median": mass_spread(tree)}
        log("ablation (regular tree): %.3f ms/frame, %.3e samples/frame; adaptive %.3f ms, %.3e samples" % (
            ablation["ms_per_frame"], ablation["samples_per_frame"], ablation["adaptive_ms_per_frame"],
            ablation["adaptive_samples_per_frame"]))
        rtree.close()
        del rmlp

    # ---- the ablation's quality side: a finer field (a 4096-leaf adaptive tree on the same
    #      grid, random 4x64 leaf MLPs following the density) is the teacher; 64-leaf students
    #      on the adaptive and on the regular tree are fitted to its renders by the library's
    #      training step (same rays, seeds, steps and learning rate), then rendered on a
    #      held-out camera against the teacher ----
    if ablation is not None and args.ablation_steps > 0:
        t0 = time.perf_counter()
        ttree = am.Tree(ctx, grid, cfg.grid_n, cfg.max_depth, 4096)
        tdens = synth.leaf_mean_density(grid, cfg.grid_n, ttree.leaf_boxes())
        tW = synth.make_weights(ttree.n_leaves, cfg.n_hidden, cfg.hidden, cfg.seed_weights + 50, tdens)
        tmlp = am.Mlp(ctx, torch.from_numpy(tW).to(dev), cfg.n_hidden, cfg.hidden, am.AMNERF_F32, ttree.n_leaves)
        B = 65536
        tcams = synth.make_cameras(100, cfg.seed_batches + 7, cfg.width, cfg.height)
        po, pd = synth.random_pixel_rays(tcams, 8 * B, cfg.seed_batches + 8)
        po, pd = torch.from_numpy(po).to(dev), torch.from_numpy(pd).to(dev)
        ptgt = torch.empty((8 * B, 3), device=dev)
        am.amnerf_render(ctx.h, ttree.h, tmlp.desc, po, pd, cfg.s_max, ptgt, None, None, None, cfg.ert_eps)
        o0, d0 = rays[0]
        ref = torch.empty((R, 3), device=dev)
        am.amnerf_render(ctx.h, ttree.h, tmlp.desc, o0, d0, cfg.s_max, ref, None, None, None, cfg.ert_eps)
        batches = [(po[:, i * B:(i + 1) * B].contiguous(), pd[:, i * B:(i + 1) * B].contiguous(),
                    ptgt[i * B:(i + 1) * B].contiguous()) for i in range(8)]
        quality = {"teacher": "4096-leaf adaptive tree, random 4x64 leaf MLPs (density-following sigma biases)",
                   "students": "64 leaves, 4x64 bf16 leaf MLPs, %d Adam steps of %d rays (lr 1e-3) on teacher renders "
                               "from 100 cameras; PSNR of camera 0 against the teacher" % (args.ablation_steps, B)}
        for name, split in (("adaptive", am.AMNERF_SPLIT_MEDIAN), ("regular", am.AMNERF_SPLIT_MIDDLE)):
            stree = am.Tree(ctx, grid, cfg.grid_n, cfg.max_depth, 64, split)
            sdens = synth.leaf_mean_density(grid, cfg.grid_n, stree.leaf_boxes())
            sW = synth.make_weights(stree.n_leaves, cfg.n_hidden, cfg.hidden, cfg.seed_student, sdens)
            tr = am.Trainer(ctx, stree, torch.from_numpy(sW).to(dev), cfg.n_hidden, cfg.hidden)
            first = float(tr.step(*batches[0], cfg.s_max, lr=1e-3).item())
            for it in range(1, args.ablation_steps):
                tr.step(*batches[it % 8], cfg.s_max, lr=1e-3)
            last = float(tr.loss.item())
            img = torch.empty((R, 3), device=dev)
            am.amnerf_render(ctx.h, stree.h, tr.mlp, o0, d0, cfg.s_max, img, None, None, None, cfg.ert_eps)
            ns = am.amnerf_render_stats_get(ctx.h)["n_samples"]
            rep = am.amnerf_error_stats(ctx.h, img.view(-1), ref.view(-1).double())
            quality[name] = {"psnr_vs_teacher_db": rep["psnr"], "loss_first_last": [first, last],
                             "samples_per_frame": ns}
            log("ablation quality, %s tree: %.2f dB against the teacher after %d steps (loss %.3e -> %.3e)" % (
                name, rep["psnr"], args.ablation_steps, first, last))
            del tr
            stree.close()
        quality["seconds"] = time.perf_counter() - t0
        ablation["quality"] = quality
        del tmlp, batches, po, pd, ptgt
        ttree.close()

    # ---- hierarchical sampling (HCheck): every node gets an MLP, plain bf16 render, same
    #      cameras; the footprint (sample spacing per unit distance) is a free parameter ----
    hier = None
    if "bf16" in paths:
        rows = tree.rows
        nboxes = rows[np.argsort(rows[:, 11])][:, 2:8].copy()
        ndens = synth.leaf_mean_density(grid, cfg.grid_n, nboxes)
        nW = synth.make_weights(len(nboxes), cfg.n_hidden, cfg.hidden, cfg.seed_weights, ndens)
        nmlp = am.Mlp(ctx, torch.from_numpy(nW).to(dev), cfg.n_hidden, cfg.hidden, am.AMNERF_BF16, len(nboxes))
        ob = outs["bf16"]
        hier = {"path": "bf16, no proposal, %d node MLPs" % len(nboxes),
                "adaptive_leaves_ms_per_frame": results["bf16"]["ms_per_frame"],
                "adaptive_leaves_samples_per_frame": results["bf16"]["samples_per_frame"], "footprints": {}}
        for fp in (0.05, 0.1, 0.25):
            def hrender(cam):
                o, d = rays[cam]
                am.amnerf_render(ctx.h, tree.h, nmlp.desc, o, d, cfg.s_max, ob["rgb"], ob["depth"], ob["opacity"],
                                 None, cfg.ert_eps, hcheck_footprint=fp)
            hs, hiv = [], []
            for cam in range(n_cams):
                hrender(cam)
                st = am.amnerf_render_stats_get(ctx.h)
                hs.append(st["n_samples"])
                hiv.append(st["n_intervals"])
            for w in range(args.warmup):
                hrender(w % n_cams)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(args.steps):
                hrender(k % n_cams)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            hier["footprints"][str(fp)] = {"ms_per_frame": 1e3 * dt / args.steps,
                                           "samples_per_frame": float(np.mean(hs)),
                                           "intervals_per_frame": float(np.mean(hiv))}
            log("hierarchical sampling, footprint %g: %.3f ms/frame, %.3e samples/frame, %.3e intervals/frame" % (
                fp, 1e3 * dt / args.steps, np.mean(hs), np.mean(hiv)))
        del nmlp

    # ---- training step on the same scene (teacher-student, bf16 forward, float32 gradients,
    #      Adam), timed apart from the frame ----
    train = train_host = None
    if args.train_steps > 0:
        B = args.train_batch
        tcams = synth.make_cameras(100, cfg.seed_batches + 3, cfg.width, cfg.height)
        po, pd = synth.random_pixel_rays(tcams, 4 * B, cfg.seed_batches + 4)
        po, pd = torch.from_numpy(po).to(dev), torch.from_numpy(pd).to(dev)
        ptarget = torch.empty((4 * B, 3), device=dev)
        am.amnerf_render(ctx.h, tree.h, mlps["f32"].desc, po, pd, cfg.s_max, ptarget, None, None, None, cfg.ert_eps)
        batches = [(po[:, i * B:(i + 1) * B].contiguous(), pd[:, i * B:(i + 1) * B].contiguous(),
                    ptarget[i * B:(i + 1) * B].contiguous()) for i in range(4)]
        W_s = synth.make_weights(L, cfg.n_hidden, cfg.hidden, cfg.seed_student, dens)
        trainer = am.Trainer(ctx, tree, torch.from_numpy(W_s).to(dev), cfg.n_hidden, cfg.hidden)
        tlosses, tsamples = [], 0
        for it in range(2):
            ob, db_, tb = batches[it % 4]
            tlosses.append(float(trainer.step(ob, db_, tb, cfg.s_max, lr=1e-3).item()))
        torch.cuda.synchronize()
        am.amnerf_ctx_set_timing(ctx.h, True)
        am.amnerf_timing_collect(ctx.h)
        am.amnerf_timing_collect_backward(ctx.h)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.train_steps + 1)]
        evs[0].record()
        for it in range(args.train_steps):
            ob, db_, tb = batches[it % 4]
            trainer.step(ob, db_, tb, cfg.s_max, lr=1e-3)
            evs[it + 1].record()
        torch.cuda.synchronize()
        step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.train_steps)]
        fwd_ms, nf = am.amnerf_timing_collect(ctx.h)
        bwd_ms, nb = am.amnerf_timing_collect_backward(ctx.h)
        am.amnerf_ctx_set_timing(ctx.h, False)
        t_ms = median(step_ms)
        for it in range(4):
            ob, db_, tb = batches[it]
            tlosses.append(float(trainer.step(ob, db_, tb, cfg.s_max, lr=1e-3).item()))
            tsamples += am.amnerf_render_stats_get(ctx.h)["n_samples"]
        spp = tsamples / 4
        stages = {"forward_" + k: v / max(nf, 1) for k, v in fwd_ms.items()}
        stages.update({k: v / max(nb, 1) for k, v in bwd_ms.items()})
        bwd_tf = FLOP_PER_SAMPLE_BWD_4x64 * spp / (stages["mlp_bwd"] * 1e-3) / 1e12
        train = {"ms_per_step": t_ms, "ms_per_step_mean": sum(step_ms) / len(step_ms),
                 "rays_per_step": B, "samples_per_step": spp,
                 "samples_per_s": spp / (t_ms * 1e-3), "steps": args.train_steps,
                 "loss_first_last": [tlosses[0], tlosses[-1]],
                 "stage_ms_per_step": stages,
                 "tflops_per_step": (FLOP_PER_SAMPLE_4x64 + FLOP_PER_SAMPLE_BWD_4x64) * spp / (t_ms * 1e-3) / 1e12,
                 "roofline": {"bound": "mfma", "achieved": bwd_tf, "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                              "frac": bwd_tf / PEAK_TFLOPS["bf16"], "traffic": None,
                              "kernel": "k_mlp_bwd<64, 4>", "kernel_ms": stages["mlp_bwd"],
                              "flop_per_sample": FLOP_PER_SAMPLE_BWD_4x64},
                 "workload": "teacher = the scene's leaf MLPs (float32 renders as targets), student re-seeded; "
                             "%d-ray batches drawn from 100 cameras at 800x800" % B}
        log("train: %.3f ms/step (median of %d), %.3e samples/s, loss %.3e -> %.3e, stages %s" % (
            t_ms, args.train_steps, train["samples_per_s"], tlosses[0], tlosses[-1],
            {k: round(v, 4) for k, v in stages.items()}))
        train_host = (trainer.master.cpu().numpy(), batches[0][0].cpu().numpy(), batches[0][1].cpu().numpy(),
                      batches[0][2].cpu().numpy())

    # outputs of camera 0 for the accuracy report
    imgs = {}
    for kind in paths:
        render(kind, 0)
        torch.cuda.synchronize()
        imgs[kind] = outs[kind]["rgb"].clone()

    cpu = None
    psnr = {k: None for k in paths}
    max_abs = {k: None for k in paths}
    if not args.no_cpu:
        import oracle
        otree = oracle.build_tree(grid, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
        assert np.array_equal(otree.rows, tree.rows)
        o0, d0 = synth.camera_rays(cams[0])
        threads = cpu_threads()
        rng = np.random.default_rng(12345)
        probe = np.sort(rng.choice(R, 4000, replace=False))
        oracle.render(otree, W, cfg.n_hidden, cfg.hidden, o0, d0, cfg.s_max, eps=cfg.ert_eps, ray_idx=probe,
                      threads=threads)
        t0 = time.perf_counter()
        oracle.render(otree, W, cfg.n_hidden, cfg.hidden, o0, d0, cfg.s_max, eps=cfg.ert_eps, ray_idx=probe,
                      threads=threads)
        per_ray = (time.perf_counter() - t0) / len(probe)
        n_sample = int(min(R, max(4000, args.cpu_seconds / max(per_ray, 1e-9))))
        sel = np.sort(rng.choice(R, n_sample, replace=False))
        t0 = time.perf_counter()
        rgb, dep, op, ns, flags = oracle.render(otree, W, cfg.n_hidden, cfg.hidden, o0, d0, cfg.s_max,
                                                eps=cfg.ert_eps, ray_idx=sel, threads=threads)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": float(ns.sum()) / t_cpu, "unit": "samples/s", "cores": threads, "kind": "oracle",
               "sample": "%d random rays of held-out camera 0 (%.1f%% of one 800x800 frame, %d samples), "
                         "float64 plain render, %.1f s" % (n_sample, 100.0 * n_sample / R, int(ns.sum()), t_cpu)}
        # the same oracle on one host thread, over every sixteenth ray of that sample
        sel1 = sel[::16]
        t0 = time.perf_counter()
        ns1 = oracle.render(otree, W, cfg.n_hidden, cfg.hidden, o0, d0, cfg.s_max, eps=cfg.ert_eps, ray_idx=sel1,
                            threads=1)[3]
        t1c = time.perf_counter() - t0
        cpu["one_thread"] = {"value": float(ns1.sum()) / t1c, "rays": int(sel1.size), "seconds": t1c}
        # float64 error report on the GPU over the sampled rays
        sel_dev = torch.from_numpy(sel).to(dev)
        ref_dev = torch.from_numpy(np.ascontiguousarray(rgb, dtype=np.float64)).to(dev).view(-1)
        for kind in paths:
            rep = am.amnerf_error_stats(ctx.h, imgs[kind][sel_dev].contiguous().view(-1), ref_dev)
            psnr[kind] = rep["psnr"]
            max_abs[kind] = rep["max_abs"]
        cpu["host_cpus"] = host_cpus()
        log("oracle: %.3e samples/s on %d threads (%d host cores); psnr %s; max |rgb - oracle| %s" % (
            cpu["value"], threads, cpu["host_cpus"], {k: round(v, 2) for k, v in psnr.items()},
            {k: float("%.3g" % v) for k, v in max_abs.items()}))
        if train_host is not None:
            # the training step on the oracle: float64 forward render, the MSE gradient of its
            # colours, and the float64 parameter gradient (one host thread: the oracle's
            # gradient is single-threaded), over a bounded random subset of the first batch
            Ws_h, tob, tdb, ttb = train_host
            trng = np.random.default_rng(4321)

            def oracle_step(idx):
                rgb_s, _, _, ns_s, _ = oracle.render(otree, Ws_h, cfg.n_hidden, cfg.hidden, tob, tdb, cfg.s_max,
                                                     eps=cfg.ert_eps, ray_idx=idx, threads=1)
                g = 2.0 * (rgb_s - ttb[idx]) / (3.0 * tob.shape[1])
                oracle.render_grad(otree, Ws_h, cfg.n_hidden, cfg.hidden, tob, tdb, cfg.s_max, g,
                                   eps=cfg.ert_eps, ray_idx=idx)
                return int(ns_s.sum())
            idx = np.sort(trng.choice(tob.shape[1], 128, replace=False))
            t0 = time.perf_counter()
            oracle_step(idx)
            per_ray = (time.perf_counter() - t0) / idx.size
            n_t = int(min(tob.shape[1], max(128, 0.5 * args.cpu_seconds / max(per_ray, 1e-9))))
            idx = np.sort(trng.choice(tob.shape[1], n_t, replace=False))
            t0 = time.perf_counter()
            ns_t = oracle_step(idx)
            t_t = time.perf_counter() - t0
            train["cpu_baseline"] = {
                "value": ns_t / t_t, "unit": "samples/s", "cores": 1, "kind": "oracle", "host_cpus": host_cpus(),
                "sample": "%d random rays of the first %d-ray training batch (%d samples): float64 forward "
                          "render, MSE gradient, float64 parameter gradient; %.1f s" % (n_t, tob.shape[1], ns_t, t_t)}
            log("oracle training step: %.3e samples/s on one thread" % (ns_t / t_t))

    large = None
    if not args.no_large:
        del mlps, outs, imgs
        if args.train_steps > 0:
            del trainer, batches, po, pd, ptarget
        torch.cuda.empty_cache()
        large = large_scene(args, am, torch, np, synth, ctx)

    head = results["bf16_prop"]
    achieved = head["mlp_tflops"]
    traffic = None
    prof = os.path.join(ROOT, "profiles", "mlp_bf16_c2_traffic.json")
    if os.path.exists(prof):
        rec = json.load(open(prof))
        src = open(os.path.join(ROOT, "paper_2310_01881_amd", "csrc", "mlp.hip"), "rb").read()
        if rec.get("mlp_source_sha256") == hashlib.sha256(src).hexdigest():
            traffic = rec.get("hbm_bytes_per_launch")
    # the throughput line: frames in flight when measured, else one frame at a time
    tput = inflight["paths"] if inflight else results
    line = {
        "metric": "samples/s + ms/frame 800x800: BF16+proposal vs plain FP32 at PSNR>=45 dB vs oracle",
        "value": tput["bf16_prop"]["samples_per_s"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tput["bf16_prop"]["ms_per_frame"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "800x800 frame, 128^3 guidance grid (200 anisotropic blobs + ground slab), "
                               "512-leaf KD tree (max depth 12), 4x64 per-leaf MLPs, <=128 samples/ray, "
                               "ERT at T<1e-4; 8 held-out cameras",
                   "rays_per_step": R, "n_leaves": L, "path": "bf16 leaf MLPs + learned proposal (bf16 inference, "
                   "<=48 samples/ray, fallback below 0.99 predicted mass)",
                   "frames_in_flight": inflight["frames_in_flight"] if inflight else 1,
                   "one_frame_at_a_time": {"ms_per_frame": head["ms_per_frame"], "samples_per_s": head["samples_per_s"]},
                   "plain_samples_per_step": sum(plain) / n_cams,
                   "proposal_samples_per_step": sum(samples["bf16_prop"]) / n_cams,
                   "fallback_rays_per_step": sum(fallback) / n_cams,
                   "proposal_training": {"steps": args.prop_steps, "rays_per_step": args.prop_batch,
                                         "cameras": 200, "seconds": t_prop, "loss_first_last": [losses[0], losses[-1]]}},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["bf16"], "traffic": traffic,
                     "kernel": "k_mlp<64,bf16>", "kernel_ms": head["mlp_ms"]},
        "cpu_baseline": cpu,
        "psnr_vs_oracle_db": psnr,
        "max_abs_rgb_vs_oracle": max_abs,
        "speedup_vs_plain_fp32": tput["f32"]["ms_per_frame"] / tput["bf16_prop"]["ms_per_frame"] if "f32" in tput else None,
        "speedup_vs_plain_fp32_in_rounds": (tput["f32_rounds"]["ms_per_frame"] / tput["bf16_prop"]["ms_per_frame"]
                                            if "f32_rounds" in tput else None),
        "training": train,
        "paths": results,
        "frames_in_flight": inflight,
        "large_scene": large,
        "ablation_regular_tree": ablation,
        "hierarchical_sampling": hier,
    }
    print(json.dumps(line), flush=True)
    head_psnr = psnr.get("bf16_prop")
    if head_psnr is not None and not head_psnr >= HEADLINE_PSNR_DB:
        print("bench.py: the headline path is at %.2f dB against the oracle, below the %.0f dB it is quoted at"
              % (head_psnr, HEADLINE_PSNR_DB), file=sys.stderr, flush=True)
        sys.exit(1)


if __name__ == "__main__":
    main()
