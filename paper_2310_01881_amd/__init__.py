"""Python binding of libamnerf (adaptive multi-NeRF rendering on AMD MI355X).

Every function here only marshals arguments for the C ABI in ``include/amnerf.h``; all
steps of the rendering path run in the library's HIP kernels.  torch is used for device
memory and streams: tensors are passed by ``data_ptr()``, streams by their handle.
The library must have been built (``python paper_2310_01881_amd/build.py``); importing
this module fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamnerf.so")

AMNERF_OK = 0
AMNERF_EINVAL = -1
AMNERF_ENOMEM = -2
AMNERF_EDEVICE = -3
AMNERF_ECAPACITY = -4
AMNERF_ESTATE = -5
AMNERF_F32 = 0
AMNERF_BF16 = 1
AMNERF_FP8 = 2
AMNERF_FP8_ACT = 3
AMNERF_SPLIT_MEDIAN = 0
AMNERF_SPLIT_MIDDLE = 1
AMNERF_JITTER = 1
AMNERF_TRAIN_F32 = 2
AMNERF_TESTLEAF_F32 = 1
AMNERF_ERT_ROUNDS = 2
AMNERF_MAX_GRID = 512
AMNERF_MAX_DEPTH = 16
AMNERF_MAX_LEAVES = 4096
AMNERF_MAX_SAMPLES = 255
AMNERF_MAX_RENDER_LANES = 4

# symbols declared in include/amnerf.h
EXPORTS = [
    "amnerf_last_error", "amnerf_version", "amnerf_ctx_create", "amnerf_ctx_destroy",
    "amnerf_build_tree", "amnerf_tree_info_get", "amnerf_tree_export", "amnerf_tree_destroy",
    "amnerf_build_occupancy", "amnerf_occupancy_info_get", "amnerf_occupancy_export", "amnerf_occupancy_destroy",
    "amnerf_mlp_param_count", "amnerf_mlp_packed_bytes", "amnerf_mlp_pack", "amnerf_render",
    "amnerf_render_stats_get", "amnerf_render_inspect", "amnerf_ctx_set_timing", "amnerf_ctx_set_render_lanes",
    "amnerf_timing_collect", "amnerf_timing_collect_backward", "amnerf_render_backward",
    "amnerf_build_tree_codes", "amnerf_build_tree_distilled", "amnerf_adam_step", "amnerf_train_step",
    "amnerf_prop_param_count", "amnerf_prop_packed_bytes", "amnerf_prop_pack", "amnerf_propose",
    "amnerf_error_stats", "amnerf_render_backward_inspect", "amnerf_render_static",
    "amnerf_render_static_capacity", "amnerf_mlp_pack_fp8_act", "amnerf_mlp_calibrate",
]
AMNERF_PROPOSE_INFER = 0
AMNERF_PROPOSE_TRAIN = 1
AMNERF_GRAD_ONLY = 1
STAGES = ["traverse", "proposal", "sort", "expand", "mlp", "composite"]
BWD_STAGES = ["comp_bwd", "mlp_bwd", "grad_reduce", "adam"]


class AmnerfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("amnerf error %d: %s" % (code, msg))
        self.code = code


class amnerf_tree_params(C.Structure):
    _fields_ = [("max_depth", C.c_int32), ("max_leaves", C.c_int32), ("split", C.c_int32)]


class amnerf_tree_info(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_leaves", C.c_int32), ("depth", C.c_int32),
                ("grid_n", C.c_int32)]


class amnerf_mlp_shape(C.Structure):
    _fields_ = [("n_hidden", C.c_int32), ("hidden", C.c_int32)]


class amnerf_mlp(C.Structure):
    _fields_ = [("shape", amnerf_mlp_shape), ("dtype", C.c_int32), ("n_leaves", C.c_int32),
                ("packed_dev", C.c_void_p)]


class amnerf_rays(C.Structure):
    _fields_ = [("o_dev", C.c_void_p), ("d_dev", C.c_void_p), ("n_rays", C.c_int64)]


class amnerf_proposal(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("packed_dev", C.c_void_p), ("mass_thresh", C.c_float), ("cap", C.c_int32)]


class amnerf_render_params(C.Structure):
    _fields_ = [("s_max", C.c_int32), ("ert_eps", C.c_float), ("flags", C.c_uint32),
                ("jitter_seed", C.c_uint64), ("proposal", C.POINTER(amnerf_proposal)),
                ("hcheck_footprint", C.c_float), ("occupancy", C.c_void_p)]


class amnerf_render_out(C.Structure):
    _fields_ = [("rgb_dev", C.c_void_p), ("depth_dev", C.c_void_p), ("opacity_dev", C.c_void_p),
                ("weights_dev", C.c_void_p)]


class amnerf_render_stats(C.Structure):
    _fields_ = [("n_rays", C.c_int64), ("n_intervals", C.c_int64), ("n_samples", C.c_int64),
                ("n_tiles", C.c_int64), ("n_chunks", C.c_int64), ("n_nonfinite", C.c_int64),
                ("n_fallback", C.c_int64), ("n_plain_samples", C.c_int64), ("n_unreached", C.c_int64),
                ("n_composited", C.c_int64), ("n_placed_samples", C.c_int64)]


class amnerf_inspect(C.Structure):
    _fields_ = [("ray_iv_off", C.c_void_p), ("ray_smp_off", C.c_void_p), ("iv_t0", C.c_void_p),
                ("iv_dt", C.c_void_p), ("iv_slot", C.c_void_p), ("iv_n", C.c_void_p),
                ("bucket_off", C.c_void_p), ("perm", C.c_void_p), ("sample_out", C.c_void_p),
                ("ray_used", C.c_void_p), ("slot_mask", C.c_void_p)]


class amnerf_adam_params(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int32)]


class amnerf_mlp_train(C.Structure):
    _fields_ = [("shape", amnerf_mlp_shape), ("n_leaves", C.c_int32), ("master_dev", C.c_void_p),
                ("grad_dev", C.c_void_p), ("m_dev", C.c_void_p), ("v_dev", C.c_void_p),
                ("packed_dev", C.c_void_p)]


class amnerf_train_params(C.Structure):
    _fields_ = [("render", amnerf_render_params), ("adam", amnerf_adam_params), ("flags", C.c_uint32)]


class amnerf_testleaf_params(C.Structure):
    _fields_ = [("student", amnerf_mlp_shape), ("init_dev", C.c_void_p), ("n_max", C.c_int32),
                ("gain_thresh", C.c_float), ("lr", C.c_float), ("n_batches", C.c_int32),
                ("batches", C.POINTER(amnerf_rays)), ("targets", C.POINTER(C.c_void_p)), ("eval", amnerf_rays),
                ("eval_target_dev", C.c_void_p), ("render", amnerf_render_params), ("flags", C.c_uint32)]


class amnerf_testleaf_record(C.Structure):
    _fields_ = [("code", C.c_uint32), ("depth", C.c_int32), ("leaves_of_trial", C.c_int32), ("kept", C.c_int32),
                ("psnr_current", C.c_double), ("psnr_split", C.c_double)]


class amnerf_propose_params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("s_max", C.c_int32), ("infer_dtype", C.c_int32),
                ("infer_packed_dev", C.c_void_p), ("tau_dev", C.c_void_p), ("tau_cap", C.c_int64),
                ("master_dev", C.c_void_p), ("grad_dev", C.c_void_p), ("m_dev", C.c_void_p), ("v_dev", C.c_void_p),
                ("packed_dev", C.c_void_p), ("adam", amnerf_adam_params), ("loss_dev", C.c_void_p)]


def _load():
    # torch bundles its own HIP runtime under the soname libamdhip64.so.7.  Loading torch
    # first makes this library's dependency resolve to that same runtime, so one process
    # never holds two HIP/HSA runtimes (device pointers and streams come from torch).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libamnerf.so is not built: run `python paper_2310_01881_amd/build.py` "
                          "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.amnerf_last_error.restype = C.c_char_p
    lib.amnerf_version.restype = C.c_int
    lib.amnerf_ctx_create.argtypes = [C.c_int, C.c_size_t, C.POINTER(P)]
    lib.amnerf_ctx_destroy.argtypes = [P]
    lib.amnerf_build_tree.argtypes = [P, P, C.c_int32, C.POINTER(amnerf_tree_params), C.POINTER(P)]
    lib.amnerf_build_tree_codes.argtypes = [P, P, C.c_int32, P, C.c_int32, C.POINTER(P)]
    lib.amnerf_build_tree_distilled.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32,
                                                C.POINTER(amnerf_testleaf_params), C.POINTER(P),
                                                C.POINTER(amnerf_testleaf_record), C.c_int32,
                                                C.POINTER(C.c_int32)]
    lib.amnerf_tree_info_get.argtypes = [P, C.POINTER(amnerf_tree_info)]
    lib.amnerf_tree_export.argtypes = [P, P, P]
    lib.amnerf_tree_destroy.argtypes = [P]
    lib.amnerf_build_occupancy.argtypes = [P, P, C.c_int32, C.c_int32, C.c_float, C.POINTER(P)]
    lib.amnerf_occupancy_info_get.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
    lib.amnerf_occupancy_export.argtypes = [P, P]
    lib.amnerf_occupancy_destroy.argtypes = [P]
    lib.amnerf_mlp_param_count.argtypes = [C.POINTER(amnerf_mlp_shape)]
    lib.amnerf_mlp_param_count.restype = C.c_int64
    lib.amnerf_mlp_packed_bytes.argtypes = [C.POINTER(amnerf_mlp_shape), C.c_int32, C.c_int32,
                                            C.POINTER(C.c_size_t)]
    lib.amnerf_mlp_pack.argtypes = [P, C.POINTER(amnerf_mlp_shape), C.c_int32, C.c_int32, P, P, P]
    lib.amnerf_mlp_pack_fp8_act.argtypes = [P, C.POINTER(amnerf_mlp_shape), C.c_int32, P, P, P, P]
    lib.amnerf_mlp_calibrate.argtypes = [P, C.POINTER(amnerf_mlp_shape), C.c_int32, P, C.POINTER(amnerf_rays), P, P]
    lib.amnerf_render.argtypes = [P, P, C.POINTER(amnerf_mlp), C.POINTER(amnerf_rays),
                                  C.POINTER(amnerf_render_params), C.POINTER(amnerf_render_out), P]
    lib.amnerf_render_static.argtypes = lib.amnerf_render.argtypes
    lib.amnerf_render_static_capacity.restype = C.c_size_t
    lib.amnerf_render_stats_get.argtypes = [P, C.POINTER(amnerf_render_stats)]
    lib.amnerf_render_inspect.argtypes = [P, C.POINTER(amnerf_inspect), P]
    lib.amnerf_ctx_set_timing.argtypes = [P, C.c_int]
    lib.amnerf_ctx_set_render_lanes.argtypes = [P, C.c_int]
    lib.amnerf_timing_collect.argtypes = [P, P, C.POINTER(C.c_int64)]
    lib.amnerf_timing_collect_backward.argtypes = [P, P, C.POINTER(C.c_int64)]
    lib.amnerf_render_backward.argtypes = [P, P, C.POINTER(amnerf_mlp), C.POINTER(amnerf_rays), P, P, P, P, P]
    lib.amnerf_render_backward_inspect.argtypes = [P, P, P]
    lib.amnerf_adam_step.argtypes = [P, C.c_int64, P, P, P, P, C.POINTER(amnerf_adam_params), P]
    lib.amnerf_error_stats.argtypes = [P, P, P, P, C.c_int64, C.POINTER(C.c_double * 4), P]
    lib.amnerf_train_step.argtypes = [P, P, C.POINTER(amnerf_mlp_train), C.POINTER(amnerf_rays), P,
                                      C.POINTER(amnerf_train_params), P, P]
    lib.amnerf_prop_param_count.restype = C.c_int64
    lib.amnerf_prop_packed_bytes.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
    lib.amnerf_prop_pack.argtypes = [P, C.c_int32, P, P, P]
    lib.amnerf_propose.argtypes = [P, P, C.POINTER(amnerf_mlp), C.POINTER(amnerf_rays),
                                   C.POINTER(amnerf_propose_params), C.POINTER(C.c_int64), P]
    return lib


_lib = _load()


def lib():
    return _lib


def _check(rc):
    if rc != AMNERF_OK:
        raise AmnerfError(rc, _lib.amnerf_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------------------
# C-ABI mirrors (same names, argument marshalling only)
# ---------------------------------------------------------------------------------------
def amnerf_last_error() -> str:
    return _lib.amnerf_last_error().decode()


def amnerf_version() -> int:
    return _lib.amnerf_version()


def amnerf_ctx_create(device: int = 0, workspace_cap: int = 0):
    h = C.c_void_p()
    _check(_lib.amnerf_ctx_create(device, workspace_cap, C.byref(h)))
    return h


def amnerf_ctx_destroy(ctx):
    _check(_lib.amnerf_ctx_destroy(ctx))


def amnerf_build_tree(ctx, grid: np.ndarray, n: int, max_depth: int, max_leaves: int, split: int = 0):
    g = np.ascontiguousarray(grid, dtype=np.float32)
    if g.size != n ** 3:
        raise ValueError("grid has %d cells, expected %d" % (g.size, n ** 3))
    h = C.c_void_p()
    prm = amnerf_tree_params(max_depth, max_leaves, split)
    _check(_lib.amnerf_build_tree(ctx, g.ctypes.data_as(C.c_void_p), n, C.byref(prm), C.byref(h)))
    return h


def amnerf_build_tree_codes(ctx, grid: np.ndarray, n: int, codes):
    g = np.ascontiguousarray(grid, dtype=np.float32)
    if g.size != n ** 3:
        raise ValueError("grid has %d cells, expected %d" % (g.size, n ** 3))
    c = np.ascontiguousarray(np.asarray(codes, np.uint32).reshape(-1))
    h = C.c_void_p()
    _check(_lib.amnerf_build_tree_codes(ctx, g.ctypes.data_as(C.c_void_p), n,
                                        c.ctypes.data_as(C.c_void_p) if c.size else None, int(c.size), C.byref(h)))
    return h


def amnerf_build_tree_distilled(ctx, grid: np.ndarray, n: int, max_depth: int, max_leaves: int, n_hidden: int,
                                hidden: int, init_dev, n_max: int, gain_thresh: float, lr: float, batches,
                                eval_rays, eval_target_dev, s_max: int, ert_eps: float = 1e-4, f32: bool = False,
                                log_cap: int = 4096):
    """(tree handle, list of test records as dicts).  batches: [(o_dev, d_dev, target_dev)];
    eval_rays: (o_dev, d_dev); eval_target_dev: float64 [rays][3]."""
    g = np.ascontiguousarray(grid, dtype=np.float32)
    if g.size != n ** 3:
        raise ValueError("grid has %d cells, expected %d" % (g.size, n ** 3))
    nb = len(batches)
    rays = (amnerf_rays * max(nb, 1))(*[amnerf_rays(_ptr(o), _ptr(d), int(o.shape[1])) for o, d, _ in batches])
    tgts = (C.c_void_p * max(nb, 1))(*[_ptr(t) for _, _, t in batches])
    eo, ed = eval_rays
    prm = amnerf_testleaf_params(amnerf_mlp_shape(n_hidden, hidden), _ptr(init_dev), n_max, gain_thresh, lr, nb,
                                 rays, tgts, amnerf_rays(_ptr(eo), _ptr(ed), int(eo.shape[1])), _ptr(eval_target_dev),
                                 amnerf_render_params(s_max, ert_eps, 0, 0, None, 0.0, None),
                                 AMNERF_TESTLEAF_F32 if f32 else 0)
    log = (amnerf_testleaf_record * log_cap)()
    nlog = C.c_int32()
    h = C.c_void_p()
    _check(_lib.amnerf_build_tree_distilled(ctx, g.ctypes.data_as(C.c_void_p), n, max_depth, max_leaves,
                                            C.byref(prm), C.byref(h), log, log_cap, C.byref(nlog)))
    recs = [{k: getattr(log[i], k) for k, _ in amnerf_testleaf_record._fields_} for i in range(min(nlog.value, log_cap))]
    return h, recs


def amnerf_tree_info_get(tree) -> amnerf_tree_info:
    info = amnerf_tree_info()
    _check(_lib.amnerf_tree_info_get(tree, C.byref(info)))
    return info


def amnerf_tree_export(tree):
    info = amnerf_tree_info_get(tree)
    rows = np.zeros((info.n_nodes, 12), np.int32)
    mass = np.zeros(info.n_nodes, np.uint64)
    _check(_lib.amnerf_tree_export(tree, rows.ctypes.data_as(C.c_void_p), mass.ctypes.data_as(C.c_void_p)))
    return rows, mass


def amnerf_tree_destroy(tree):
    _check(_lib.amnerf_tree_destroy(tree))


def amnerf_build_occupancy(ctx, grid: np.ndarray, n: int, block: int, thresh: float):
    g = np.ascontiguousarray(grid, dtype=np.float32)
    if g.size != n ** 3:
        raise ValueError("grid has %d cells, expected %d" % (g.size, n ** 3))
    h = C.c_void_p()
    _check(_lib.amnerf_build_occupancy(ctx, g.ctypes.data_as(C.c_void_p), n, block, thresh, C.byref(h)))
    return h


def amnerf_occupancy_info_get(occ):
    g, n = C.c_int32(), C.c_int64()
    _check(_lib.amnerf_occupancy_info_get(occ, C.byref(g), C.byref(n)))
    return int(g.value), int(n.value)


def amnerf_occupancy_export(occ) -> np.ndarray:
    g, _ = amnerf_occupancy_info_get(occ)
    cells = np.zeros(g ** 3, np.uint8)
    _check(_lib.amnerf_occupancy_export(occ, cells.ctypes.data_as(C.c_void_p)))
    return cells


def amnerf_occupancy_destroy(occ):
    _check(_lib.amnerf_occupancy_destroy(occ))


def amnerf_mlp_param_count(n_hidden: int, hidden: int) -> int:
    s = amnerf_mlp_shape(n_hidden, hidden)
    return int(_lib.amnerf_mlp_param_count(C.byref(s)))


def amnerf_mlp_packed_bytes(n_hidden: int, hidden: int, dtype: int, n_leaves: int) -> int:
    s = amnerf_mlp_shape(n_hidden, hidden)
    out = C.c_size_t()
    _check(_lib.amnerf_mlp_packed_bytes(C.byref(s), dtype, n_leaves, C.byref(out)))
    return int(out.value)


def amnerf_mlp_pack(ctx, n_hidden: int, hidden: int, dtype: int, n_leaves: int, master_dev, packed_dev,
                    stream=None):
    s = amnerf_mlp_shape(n_hidden, hidden)
    _check(_lib.amnerf_mlp_pack(ctx, C.byref(s), dtype, n_leaves, _ptr(master_dev), _ptr(packed_dev),
                                _stream(stream)))


def amnerf_mlp_pack_fp8_act(ctx, n_hidden: int, n_leaves: int, master_dev, act_max_dev, packed_dev, stream=None):
    s = amnerf_mlp_shape(n_hidden, 64)
    _check(_lib.amnerf_mlp_pack_fp8_act(ctx, C.byref(s), n_leaves, _ptr(master_dev), _ptr(act_max_dev),
                                        _ptr(packed_dev), _stream(stream)))


def amnerf_mlp_calibrate(ctx, n_hidden: int, n_leaves: int, master_dev, o_dev, d_dev, act_max_dev, stream=None):
    s = amnerf_mlp_shape(n_hidden, 64)
    rays = amnerf_rays(_ptr(o_dev), _ptr(d_dev), int(o_dev.shape[1]))
    _check(_lib.amnerf_mlp_calibrate(ctx, C.byref(s), n_leaves, _ptr(master_dev), C.byref(rays), _ptr(act_max_dev),
                                     _stream(stream)))


def amnerf_render(ctx, tree, mlp: amnerf_mlp, o_dev, d_dev, s_max: int, rgb_dev, depth_dev=None,
                  opacity_dev=None, weights_dev=None, ert_eps: float = 1e-4, jitter: bool = False,
                  seed: int = 0, stream=None, proposal: "amnerf_proposal" = None, hcheck_footprint: float = 0.0,
                  occupancy=None, ert_rounds: bool = False):
    rays = amnerf_rays(_ptr(o_dev), _ptr(d_dev), int(o_dev.shape[1]) if o_dev is not None else 0)
    flags = (AMNERF_JITTER if jitter else 0) | (AMNERF_ERT_ROUNDS if ert_rounds else 0)
    prm = amnerf_render_params(s_max, ert_eps, flags, seed,
                               C.pointer(proposal) if proposal is not None else None, hcheck_footprint,
                               _handle(occupancy))
    out = amnerf_render_out(_ptr(rgb_dev), _ptr(depth_dev), _ptr(opacity_dev), _ptr(weights_dev))
    _check(_lib.amnerf_render(ctx, tree, C.byref(mlp), C.byref(rays), C.byref(prm), C.byref(out),
                              _stream(stream)))


def amnerf_render_static(ctx, tree, mlp: amnerf_mlp, o_dev, d_dev, s_max: int, rgb_dev, depth_dev=None,
                         opacity_dev=None, weights_dev=None, ert_eps: float = 1e-4, jitter: bool = False,
                         seed: int = 0, stream=None, hcheck_footprint: float = 0.0, ert_rounds: bool = False):
    rays = amnerf_rays(_ptr(o_dev), _ptr(d_dev), int(o_dev.shape[1]) if o_dev is not None else 0)
    flags = (AMNERF_JITTER if jitter else 0) | (AMNERF_ERT_ROUNDS if ert_rounds else 0)
    prm = amnerf_render_params(s_max, ert_eps, flags, seed, None, hcheck_footprint, None)
    out = amnerf_render_out(_ptr(rgb_dev), _ptr(depth_dev), _ptr(opacity_dev), _ptr(weights_dev))
    _check(_lib.amnerf_render_static(ctx, tree, C.byref(mlp), C.byref(rays), C.byref(prm), C.byref(out),
                                     _stream(stream)))


def amnerf_render_static_capacity() -> int:
    return int(_lib.amnerf_render_static_capacity())


def amnerf_render_stats_get(ctx) -> dict:
    st = amnerf_render_stats()
    _check(_lib.amnerf_render_stats_get(ctx, C.byref(st)))
    return {k: getattr(st, k) for k, _ in st._fields_}


def amnerf_render_inspect(ctx, stream=None, **bufs):
    ins = amnerf_inspect(*[_ptr(bufs.get(k)) for k, _ in amnerf_inspect._fields_])
    _check(_lib.amnerf_render_inspect(ctx, C.byref(ins), _stream(stream)))


def amnerf_ctx_set_timing(ctx, enable: bool):
    _check(_lib.amnerf_ctx_set_timing(ctx, 1 if enable else 0))


def amnerf_ctx_set_render_lanes(ctx, n_lanes: int):
    """Chunks in flight at once in a multi-chunk render (1 .. AMNERF_MAX_RENDER_LANES)."""
    _check(_lib.amnerf_ctx_set_render_lanes(ctx, int(n_lanes)))


def amnerf_timing_collect(ctx):
    """(dict stage -> summed ms, number of timed passes)."""
    ms = np.zeros(len(STAGES), np.float64)
    n = C.c_int64()
    _check(_lib.amnerf_timing_collect(ctx, ms.ctypes.data_as(C.c_void_p), C.byref(n)))
    return dict(zip(STAGES, ms.tolist())), int(n.value)


def amnerf_timing_collect_backward(ctx):
    """(dict backward stage -> summed ms, number of timed backward passes)."""
    ms = np.zeros(len(BWD_STAGES), np.float64)
    n = C.c_int64()
    _check(_lib.amnerf_timing_collect_backward(ctx, ms.ctypes.data_as(C.c_void_p), C.byref(n)))
    return dict(zip(BWD_STAGES, ms.tolist())), int(n.value)


def amnerf_render_backward(ctx, tree, mlp: amnerf_mlp, o_dev, d_dev, g_rgb_dev, grad_dev, g_depth_dev=None,
                           g_opacity_dev=None, stream=None):
    rays = amnerf_rays(_ptr(o_dev), _ptr(d_dev), int(o_dev.shape[1]))
    _check(_lib.amnerf_render_backward(ctx, tree, C.byref(mlp), C.byref(rays), _ptr(g_rgb_dev),
                                       _ptr(g_depth_dev), _ptr(g_opacity_dev), _ptr(grad_dev),
                                       _stream(stream)))


def amnerf_render_backward_inspect(ctx, sample_grad_dev, stream=None):
    _check(_lib.amnerf_render_backward_inspect(ctx, _ptr(sample_grad_dev), _stream(stream)))


def amnerf_adam_step(ctx, param_dev, m_dev, v_dev, grad_dev, step, lr=1e-3, beta1=0.9, beta2=0.999,
                     eps=1e-8, stream=None):
    prm = amnerf_adam_params(lr, beta1, beta2, eps, step)
    _check(_lib.amnerf_adam_step(ctx, param_dev.numel(), _ptr(param_dev), _ptr(m_dev), _ptr(v_dev),
                                 _ptr(grad_dev), C.byref(prm), _stream(stream)))


def amnerf_error_stats(ctx, x_dev, ref_dev, sel_dev=None, stream=None):
    """float64 error report of a float32 device tensor against float64 device reference values
    (same number of elements; sel_dev an optional uint8 mask): dict with max_abs, sum_sq, count,
    sum_abs, and psnr (peak 1) and mse derived from them."""
    n = x_dev.numel()
    if ref_dev.numel() != n or (sel_dev is not None and sel_dev.numel() != n):
        raise ValueError("amnerf_error_stats: size mismatch")
    out = (C.c_double * 4)()
    _check(_lib.amnerf_error_stats(ctx, _ptr(x_dev), _ptr(ref_dev), _ptr(sel_dev), n, C.byref(out), _stream(stream)))
    mx, sq, cnt, ab = out[0], out[1], out[2], out[3]
    mse = sq / cnt if cnt > 0 else 0.0
    psnr = float("inf") if mse == 0.0 else 10.0 * math.log10(1.0 / mse)
    return {"max_abs": mx, "sum_sq": sq, "count": int(cnt), "sum_abs": ab, "mse": mse, "psnr": psnr}


def amnerf_train_step(ctx, tree, train: amnerf_mlp_train, o_dev, d_dev, target_dev, loss_dev, s_max, step,
                      lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, ert_eps=1e-4, jitter=False, seed=0,
                      grad_only=False, stream=None, hcheck_footprint=0.0, f32=False):
    rays = amnerf_rays(_ptr(o_dev), _ptr(d_dev), int(o_dev.shape[1]))
    prm = amnerf_train_params(amnerf_render_params(s_max, ert_eps, AMNERF_JITTER if jitter else 0, seed, None,
                                                   hcheck_footprint),
                              amnerf_adam_params(lr, beta1, beta2, eps, step),
                              (AMNERF_GRAD_ONLY if grad_only else 0) | (AMNERF_TRAIN_F32 if f32 else 0))
    _check(_lib.amnerf_train_step(ctx, tree, C.byref(train), C.byref(rays), _ptr(target_dev), C.byref(prm),
                                  _ptr(loss_dev), _stream(stream)))


def amnerf_prop_param_count() -> int:
    return int(_lib.amnerf_prop_param_count())


def amnerf_prop_packed_bytes(dtype: int) -> int:
    out = C.c_size_t()
    _check(_lib.amnerf_prop_packed_bytes(dtype, C.byref(out)))
    return int(out.value)


def amnerf_prop_pack(ctx, dtype, master_dev, packed_dev, stream=None):
    _check(_lib.amnerf_prop_pack(ctx, dtype, _ptr(master_dev), _ptr(packed_dev), _stream(stream)))


def amnerf_propose(ctx, tree, scene_mlp: amnerf_mlp, o_dev, d_dev, params: "amnerf_propose_params", stream=None):
    rays = amnerf_rays(_ptr(o_dev), _ptr(d_dev), int(o_dev.shape[1]))
    n = C.c_int64()
    _check(_lib.amnerf_propose(ctx, tree, C.byref(scene_mlp), C.byref(rays), C.byref(params), C.byref(n),
                               _stream(stream)))
    return int(n.value)


# ---------------------------------------------------------------------------------------
# Convenience objects (still marshalling only)
# ---------------------------------------------------------------------------------------
class Context:
    """Owns an amnerf_ctx; closes it on ``close()`` or garbage collection."""

    def __init__(self, device: int = 0, workspace_cap: int = 0):
        self.device = device
        self.h = amnerf_ctx_create(device, workspace_cap)

    def close(self):
        if self.h is not None:
            amnerf_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Occupancy:
    """Occupancy bit grid for empty-space skipping (G = n / block cells per side)."""

    def __init__(self, ctx: Context, grid, n, block, thresh):
        self.ctx = ctx
        self.h = amnerf_build_occupancy(ctx.h, grid, n, block, thresh)
        self.g, self.n_occupied = amnerf_occupancy_info_get(self.h)

    def cells(self):
        return amnerf_occupancy_export(self.h)

    def close(self):
        if self.h is not None:
            amnerf_occupancy_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _handle(x):
    """A raw handle, or the handle of a wrapper object (Occupancy), or None."""
    if x is None:
        return None
    return x.h if hasattr(x, "h") else x


class Tree:
    def __init__(self, ctx: Context, grid, n, max_depth, max_leaves, split=0, handle=None):
        self.ctx = ctx
        self.h = handle if handle is not None else amnerf_build_tree(ctx.h, grid, n, max_depth, max_leaves, split)
        self.info = amnerf_tree_info_get(self.h)
        self.rows, self.mass = amnerf_tree_export(self.h)

    @classmethod
    def from_codes(cls, ctx: Context, grid, n, codes):
        """The tree whose inner nodes are exactly the given node codes."""
        return cls(ctx, None, n, 0, 0, handle=amnerf_build_tree_codes(ctx.h, grid, n, codes))

    @property
    def n_leaves(self):
        return self.info.n_leaves

    def leaf_boxes(self):
        lv = self.rows[self.rows[:, 10] >= 0]
        return lv[np.argsort(lv[:, 10])][:, 2:8].copy()

    def close(self):
        if self.h is not None:
            amnerf_tree_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """Packed per-leaf parameters on the device (kept alive with the descriptor)."""

    def __init__(self, ctx: Context, master_dev, n_hidden, hidden, dtype, n_leaves, stream=None, act_max_dev=None):
        """act_max_dev: calibration maxima for AMNERF_FP8_ACT (amnerf_mlp_calibrate), else None."""
        import torch
        nbytes = amnerf_mlp_packed_bytes(n_hidden, hidden, dtype, n_leaves)
        self.packed = torch.empty(nbytes, dtype=torch.uint8, device=master_dev.device)
        self.master = master_dev
        if act_max_dev is not None:
            if dtype != AMNERF_FP8_ACT or hidden != 64:
                raise ValueError("calibration maxima are for AMNERF_FP8_ACT (hidden 64) only")
            amnerf_mlp_pack_fp8_act(ctx.h, n_hidden, n_leaves, master_dev, act_max_dev, self.packed, stream)
        else:
            amnerf_mlp_pack(ctx.h, n_hidden, hidden, dtype, n_leaves, master_dev, self.packed, stream)
        self.desc = amnerf_mlp(amnerf_mlp_shape(n_hidden, hidden), dtype, n_leaves,
                               C.c_void_p(self.packed.data_ptr()))
        self.n_hidden, self.hidden, self.dtype, self.n_leaves = n_hidden, hidden, dtype, n_leaves


def render(ctx: Context, tree: Tree, mlp: Mlp, o_dev, d_dev, s_max, ert_eps=1e-4, jitter=False, seed=0,
           weights=False, stream=None, hcheck_footprint=0.0, occupancy=None, proposal=None):
    """Allocates the outputs and renders on `stream` (default: the current stream); returns
    dict of device tensors.  The outputs are allocated and cleared on `stream` itself, which
    first waits for the current stream (where the inputs were produced), and they are
    recorded as used by it, so the caching allocator never hands their memory to other work
    while the render may still write them."""
    import torch
    R = int(o_dev.shape[1])
    dev = o_dev.device
    cur = torch.cuda.current_stream(dev)
    st = cur if stream is None else stream
    if st != cur:
        st.wait_stream(cur)
    with torch.cuda.stream(st):
        out = {"rgb": torch.empty((R, 3), dtype=torch.float32, device=dev),
               "depth": torch.empty(R, dtype=torch.float32, device=dev),
               "opacity": torch.empty(R, dtype=torch.float32, device=dev)}
        if weights:
            out["weights"] = torch.zeros(R * s_max, dtype=torch.float32, device=dev)
    amnerf_render(ctx.h, tree.h, mlp.desc, o_dev, d_dev, s_max, out["rgb"], out["depth"], out["opacity"],
                  out.get("weights"), ert_eps, jitter, seed, st, proposal=proposal,
                  hcheck_footprint=hcheck_footprint, occupancy=occupancy)
    if st != cur:
        for t in out.values():
            t.record_stream(st)
        for t in (o_dev, d_dev):
            t.record_stream(st)
    return out


class Trainer:
    """Float32 masters, gradient and Adam moments of a leaf-MLP set, plus its bf16 packed block."""

    def __init__(self, ctx: Context, tree: Tree, master_dev, n_hidden, hidden, n_sets=None, f32=False):
        import torch
        self.ctx, self.tree = ctx, tree
        self.f32 = f32
        dt = AMNERF_F32 if f32 else AMNERF_BF16
        self.master = master_dev.contiguous()
        self.grad = torch.zeros_like(self.master)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        L = tree.n_leaves if n_sets is None else n_sets   # n_nodes for hierarchical sampling
        nbytes = amnerf_mlp_packed_bytes(n_hidden, hidden, dt, L)
        self.packed = torch.empty(nbytes, dtype=torch.uint8, device=self.master.device)
        amnerf_mlp_pack(ctx.h, n_hidden, hidden, dt, L, self.master, self.packed)
        self.desc = amnerf_mlp_train(amnerf_mlp_shape(n_hidden, hidden), L, C.c_void_p(self.master.data_ptr()),
                                     C.c_void_p(self.grad.data_ptr()), C.c_void_p(self.m.data_ptr()),
                                     C.c_void_p(self.v.data_ptr()), C.c_void_p(self.packed.data_ptr()))
        self.mlp = amnerf_mlp(amnerf_mlp_shape(n_hidden, hidden), dt, L, C.c_void_p(self.packed.data_ptr()))
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.master.device)
        self.step_no = 0

    def step(self, o_dev, d_dev, target_dev, s_max, lr=1e-3, grad_only=False, **kw):
        if not grad_only:
            self.step_no += 1
        amnerf_train_step(self.ctx.h, self.tree.h, self.desc, o_dev, d_dev, target_dev, self.loss, s_max,
                          max(self.step_no, 1), lr=lr, grad_only=grad_only, f32=self.f32, **kw)
        return self.loss


def _render_fn():
    import torch

    class RenderFn(torch.autograd.Function):
        """rgb, depth, opacity = RenderFn.apply(master, ctx, tree, o, d, s_max, ert_eps, n_hidden, hidden
        [, dtype]).

        Forward packs the float32 master parameters (to bfloat16 by default, or float32 with
        dtype=AMNERF_F32) and renders; backward returns dL/dmaster from the library's
        hand-written backward pass.  The library differentiates the last render of its
        context; if another render ran on the context in between, backward renders the same
        inputs again first (the per-sample activations are recomputed anyway)."""

        @staticmethod
        def forward(fctx, master, ctx, tree, o_dev, d_dev, s_max, ert_eps, n_hidden, hidden, dtype=AMNERF_BF16):
            L = tree.n_leaves
            nbytes = amnerf_mlp_packed_bytes(n_hidden, hidden, dtype, L)
            packed = torch.empty(nbytes, dtype=torch.uint8, device=master.device)
            master_c = master.detach().contiguous()
            amnerf_mlp_pack(ctx.h, n_hidden, hidden, dtype, L, master_c, packed)
            desc = amnerf_mlp(amnerf_mlp_shape(n_hidden, hidden), dtype, L, C.c_void_p(packed.data_ptr()))
            R = int(o_dev.shape[1])
            rgb = torch.empty((R, 3), dtype=torch.float32, device=master.device)
            depth = torch.empty(R, dtype=torch.float32, device=master.device)
            opac = torch.empty(R, dtype=torch.float32, device=master.device)
            amnerf_render(ctx.h, tree.h, desc, o_dev, d_dev, s_max, rgb, depth, opac, None, ert_eps)
            fctx.keep = (ctx, tree, desc, packed, o_dev, d_dev, master_c, s_max, ert_eps)
            return rgb, depth, opac

        @staticmethod
        def backward(fctx, g_rgb, g_depth, g_opac):
            ctx, tree, desc, packed, o_dev, d_dev, master_c, s_max, ert_eps = fctx.keep
            grad = torch.empty_like(master_c)
            args = (g_rgb.contiguous(), grad, None if g_depth is None else g_depth.contiguous(),
                    None if g_opac is None else g_opac.contiguous())
            try:
                amnerf_render_backward(ctx.h, tree.h, desc, o_dev, d_dev, *args)
            except AmnerfError as e:
                if e.code != AMNERF_ESTATE:
                    raise
                R = int(o_dev.shape[1])
                scratch = torch.empty((R, 3), dtype=torch.float32, device=master_c.device)
                amnerf_render(ctx.h, tree.h, desc, o_dev, d_dev, s_max, scratch, None, None, None, ert_eps)
                amnerf_render_backward(ctx.h, tree.h, desc, o_dev, d_dev, *args)
            return grad, None, None, None, None, None, None, None, None, None

    return RenderFn


class _LazyRenderFn:
    _fn = None

    def __getattr__(self, name):
        if _LazyRenderFn._fn is None:
            _LazyRenderFn._fn = _render_fn()
        return getattr(_LazyRenderFn._fn, name)


RenderFn = _LazyRenderFn()


class Proposal:
    """Float32 proposal parameters with Adam state, float32 (training) and bf16 packed blocks."""

    def __init__(self, ctx: Context, master_dev):
        import torch
        self.ctx = ctx
        self.master = master_dev.contiguous()
        self.grad = torch.zeros_like(self.master)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        dev = self.master.device
        self.packed = {AMNERF_F32: torch.empty(amnerf_prop_packed_bytes(AMNERF_F32), dtype=torch.uint8, device=dev),
                       AMNERF_BF16: torch.empty(amnerf_prop_packed_bytes(AMNERF_BF16), dtype=torch.uint8, device=dev)}
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.step_no = 0
        self.repack()

    def repack(self):
        for dt, buf in self.packed.items():
            amnerf_prop_pack(self.ctx.h, dt, self.master, buf)

    def descriptor(self, dtype=AMNERF_BF16, mass_thresh=0.99, cap=48):
        self._desc = amnerf_proposal(dtype, C.c_void_p(self.packed[dtype].data_ptr()), mass_thresh, cap)
        return self._desc

    def train_step(self, tree: "Tree", scene_mlp: amnerf_mlp, o_dev, d_dev, s_max, lr=1e-3):
        self.step_no += 1
        prm = amnerf_propose_params(AMNERF_PROPOSE_TRAIN, s_max, 0, None, None, 0,
                                    C.c_void_p(self.master.data_ptr()), C.c_void_p(self.grad.data_ptr()),
                                    C.c_void_p(self.m.data_ptr()), C.c_void_p(self.v.data_ptr()),
                                    C.c_void_p(self.packed[AMNERF_F32].data_ptr()),
                                    amnerf_adam_params(lr, 0.9, 0.999, 1e-8, self.step_no),
                                    C.c_void_p(self.loss.data_ptr()))
        amnerf_propose(self.ctx.h, tree.h, scene_mlp, o_dev, d_dev, prm)
        return self.loss

    def infer(self, tree: "Tree", scene_mlp: amnerf_mlp, o_dev, d_dev, s_max, dtype=AMNERF_F32, cap=1 << 22):
        import torch
        tau = torch.empty((cap, 32), dtype=torch.float32, device=self.master.device)
        prm = amnerf_propose_params(AMNERF_PROPOSE_INFER, s_max, dtype, C.c_void_p(self.packed[dtype].data_ptr()),
                                    C.c_void_p(tau.data_ptr()), cap, None, None, None, None, None,
                                    amnerf_adam_params(0, 0, 0, 0, 1), None)
        n = amnerf_propose(self.ctx.h, tree.h, scene_mlp, o_dev, d_dev, prm)
        return tau[:n]
