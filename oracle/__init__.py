"""FP64 CPU oracle for the adaptive multi-NeRF rendering path -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product (``paper_2310_01881_amd``) never imports it and shares no
code with it.  ``orc.c`` holds the arithmetic (plain loops in double precision); this
module only loads the shared object and marshals numpy arrays.

``fp8.py`` (numpy) states the float8 e4m3 weight storage of the quantised leaf MLPs;
the float8 checks render with its dequantised weights.

Two steps use library routines as permitted building blocks:
``buckets`` (the stable sort of sample indices by leaf slot is ``numpy.argsort`` with
``kind="stable"``) and ``psnr``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
NODE_COLS = 12
FLAG_ERT_AMBIGUOUS = 1
FLAG_ERT_FIRED = 2
FLAG_CLIPPED = 4
FLAG_OCC_AMBIGUOUS = 8


def build(force: bool = False) -> str:
    """Compile orc.c with gcc (double precision, no FP contraction, OpenMP)."""
    src = os.path.join(_HERE, "orc.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-std=c11", "-D_DEFAULT_SOURCE", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_SO)
        P = C.c_void_p
        i32, i64, dbl, u64, f32 = C.c_int32, C.c_int64, C.c_double, C.c_uint64, C.c_float
        _lib.orc_build_tree.argtypes = [P, i32, i32, i32, i32, i32, P, P, P, P]
        _lib.orc_build_tree_codes.argtypes = [P, i32, i32, P, i32, P, P, P, P]
        _lib.orc_trace_rays.argtypes = [P, i32, i32, P, P, i64, P, i64, i32, P, P, P, P, f32]
        _lib.orc_robust.argtypes = [P, i32, i32, P, P, i64, P, i64, dbl, dbl, P, f32]
        _lib.orc_mlp_eval.argtypes = [P, i32, i32, P, P, i64, P, P]
        _lib.orc_mlp_eval_q8.argtypes = [P, i32, i32, P, P, i64, P, P]
        _lib.orc_render_q8.argtypes = [P, i32, i32, P, i32, i32, i32, P, P, i64, P, i64, i32, dbl, P,
                                       P, P, P, i32]
        _lib.orc_act_max.argtypes = [P, i32, i32, P, i32, i32, i32, P, P, i64, P, i64, i32, P, i32]
        _lib.orc_e4m3_round.argtypes = [dbl]
        _lib.orc_e4m3_round.restype = dbl
        _lib.orc_bf16_round.argtypes = [dbl]
        _lib.orc_bf16_round.restype = dbl
        _lib.orc_render.argtypes = [P, i32, i32, P, i32, i32, i32, P, P, i64, P, i64, i32, dbl,
                                    i32, u64, P, P, P, P, P, i32, f32, P, i32]
        _lib.orc_occupancy.argtypes = [P, i32, i32, dbl, P]
        _lib.orc_ray_samples.argtypes = [P, i32, i32, P, i32, i32, i32, P, P, i64, i64, i32, dbl,
                                         i32, u64, i32, P, P, P, P, P, P, P, f32]
        _lib.orc_ray_samples.restype = i32
        _lib.orc_render_grad.argtypes = [P, i32, i32, P, i32, i32, i32, P, P, i64, P, i64, i32,
                                         dbl, i32, u64, P, P, P, P, f32]
        _lib.orc_adam.argtypes = [P, P, P, P, i64, i32, dbl, dbl, dbl, dbl]
        _lib.orc_adam.restype = None
        _lib.orc_splitmix64.argtypes = [u64]
        _lib.orc_splitmix64.restype = u64
        _lib.orc_stratum_offset.argtypes = [i32, u64, i64, i32]
        _lib.orc_stratum_offset.restype = dbl
        _lib.orc_render_proposal.argtypes = [P, i32, i32, P, i32, i32, i32, P, P, P, i64, P, i64, i32, dbl,
                                             dbl, i32, P, P, P, P, P, P, P, i32, P]
        _lib.orc_prop_eval.argtypes = [P, i32, i32, P, P, P, i64, P, i64, i32, i64, P, P]
        _lib.orc_prop_eval.restype = i64
        _lib.orc_prop_targets.argtypes = [P, i32, i32, P, i32, i32, i32, P, P, i64, P, i64, i32, i64, P]
        _lib.orc_prop_targets.restype = i64
        _lib.orc_prop_loss_grad.argtypes = [P, P, P, i64, P]
        _lib.orc_prop_loss_grad.restype = dbl
        _lib.orc_prop_param_count.restype = i32
        _lib.orc_composite.argtypes = [i32, P, P, P, dbl, P, P]
        _lib.orc_composite.restype = i32
        _lib.orc_composite_grad.argtypes = [i32, P, P, P, dbl, P, P]
        _lib.orc_composite_grad.restype = i32
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Tree:
    """An exported node table: rows of (code, depth, lo[3], hi[3], axis, plane, leaf slot,
    node slot)."""

    def __init__(self, rows, mass, grid_n):
        self.rows = rows
        self.mass = mass
        self.grid_n = grid_n

    @property
    def n_nodes(self):
        return len(self.rows)

    @property
    def n_leaves(self):
        return int((self.rows[:, 10] >= 0).sum())

    def leaf_boxes(self):
        lv = self.rows[self.rows[:, 10] >= 0]
        return lv[np.argsort(lv[:, 10])][:, 2:8].copy()


def build_tree(grid, n, max_depth, max_leaves, split=0) -> Tree:
    """KD tree of the guidance grid: split 0 = density-median subdivision (best-first by
    mass), 1 = regular subdivision (breadth-first, middle planes)."""
    grid = _c(grid, np.float32)
    cap = 2 * max_leaves
    rows = np.zeros((cap, NODE_COLS), np.int32)
    mass = np.zeros(cap, np.uint64)
    nn = np.zeros(1, np.int32)
    nl = np.zeros(1, np.int32)
    rc = lib().orc_build_tree(_p(grid), n, max_depth, max_leaves, int(split), cap, _p(rows), _p(mass), _p(nn), _p(nl))
    if rc != 0:
        raise ValueError("orc_build_tree failed")
    k = int(nn[0])
    return Tree(rows[:k].copy(), mass[:k].copy(), n)


def build_tree_codes(grid, n, codes) -> Tree:
    """The tree whose inner nodes are exactly `codes` (binary node codes, root 1, children 2c
    and 2c + 1), each split at its density median; a code must name a splittable leaf of the
    tree its smaller codes give."""
    grid = _c(grid, np.float32)
    codes = np.ascontiguousarray(np.asarray(codes, np.uint32).reshape(-1))
    cap = 2 * codes.size + 1
    rows = np.zeros((cap, NODE_COLS), np.int32)
    mass = np.zeros(cap, np.uint64)
    nn = np.zeros(1, np.int32)
    nl = np.zeros(1, np.int32)
    rc = lib().orc_build_tree_codes(_p(grid), n, codes.size, _p(codes) if codes.size else None, cap, _p(rows),
                                    _p(mass), _p(nn), _p(nl))
    if rc != 0:
        raise ValueError("orc_build_tree_codes failed (a code is not a splittable leaf)")
    return Tree(rows[:int(nn[0])].copy(), mass[:int(nn[0])].copy(), n)


def _sel(ray_idx, R):
    if ray_idx is None:
        return None, R
    ri = _c(ray_idx, np.int64)
    return ri, len(ri)


def trace(tree: Tree, o, d, ray_idx=None, cap=None, footprint=0.0):
    """Leaf intervals per ray: (t0[n][cap], t1[n][cap], slot[n][cap], m[n]); with footprint > 0
    the intervals of hierarchical sampling, keyed by node slot."""
    o = _c(o, np.float32); d = _c(d, np.float32)
    R = o.shape[1]
    ri, n = _sel(ray_idx, R)
    cap = cap or tree.n_leaves + 1
    t0 = np.zeros((n, cap)); t1 = np.zeros((n, cap))
    slot = np.full((n, cap), -1, np.int32); m = np.zeros(n, np.int32)
    rc = lib().orc_trace_rays(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(o), _p(d), R, _p(ri), n,
                              cap, _p(t0), _p(t1), _p(slot), _p(m), float(footprint))
    if rc != 0:
        raise ValueError("orc_trace_rays failed")
    return t0, t1, slot, m


def robust(tree: Tree, o, d, ray_idx=None, min_len=1e-5, eps=1e-6, footprint=0.0):
    o = _c(o, np.float32); d = _c(d, np.float32)
    R = o.shape[1]
    ri, n = _sel(ray_idx, R)
    out = np.zeros(n, np.int32)
    lib().orc_robust(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(o), _p(d), R, _p(ri), n,
                     min_len, eps, _p(out), float(footprint))
    return out.astype(bool)


def mlp_eval(params_leaf, n_hidden, hidden, x, dirs, return_features=False):
    p = _c(params_leaf, np.float32)
    x = _c(x, np.float64); dirs = _c(dirs, np.float64)
    n = len(x)
    out = np.zeros((n, 4)); feat = np.zeros((n, 30)) if return_features else None
    if lib().orc_mlp_eval(_p(p), n_hidden, hidden, _p(x), _p(dirs), n, _p(out), _p(feat)) != 0:
        raise ValueError("orc_mlp_eval failed")
    return (out, feat) if return_features else out


def mlp_eval_q8(params_leaf, n_hidden, hidden, x, dirs, act_exp):
    """mlp_eval in the float8 model: bfloat16 input features, float8 hidden activations with
    the leaf's exponents act_exp[n_hidden]."""
    p = _c(params_leaf, np.float32)
    x = _c(x, np.float64); dirs = _c(dirs, np.float64)
    k = _c(act_exp, np.int32)
    assert k.shape == (n_hidden,)
    out = np.zeros((len(x), 4))
    if lib().orc_mlp_eval_q8(_p(p), n_hidden, hidden, _p(x), _p(dirs), len(x), _p(k), _p(out)) != 0:
        raise ValueError("orc_mlp_eval_q8 failed")
    return out


def e4m3_round(x):
    """Nearest e4m3 value of x in [0, 448] (448 for x >= 448), ties to even."""
    return lib().orc_e4m3_round(float(x))


def bf16_round(x):
    """Nearest bfloat16 value of x, ties to even."""
    return lib().orc_bf16_round(float(x))


def occupancy(grid, n, block, thresh):
    """Occupancy cells uint8[G^3] (G = n / block) for empty-space skipping."""
    grid = _c(grid, np.float32)
    G = n // block
    out = np.zeros(G ** 3, np.uint8)
    if lib().orc_occupancy(_p(grid), n, block, float(thresh), _p(out)) != G:
        raise ValueError("orc_occupancy failed")
    return out


def render(tree: Tree, params, n_hidden, hidden, o, d, s_max, eps=1e-4, ray_idx=None,
           jitter=False, seed=0, threads=None, footprint=0.0, occupancy=None):
    """Per-ray (rgb[n][3], depth[n], opacity[n], n_samples[n], flags[n]) in float64.  With
    footprint > 0: hierarchical sampling, params holding one set per node (by node slot).  With
    occupancy cells (uint8[G^3]): samples in empty cells are dropped, and n_samples counts the
    kept ones."""
    params = _c(params, np.float32)
    o = _c(o, np.float32); d = _c(d, np.float32)
    R = o.shape[1]
    ri, n = _sel(ray_idx, R)
    rgb = np.zeros((n, 3)); depth = np.zeros(n); opac = np.zeros(n)
    ns = np.zeros(n, np.int32); flags = np.zeros(n, np.int32)
    threads = threads or min(16, os.cpu_count() or 1)
    occ, occ_g = None, 0
    if occupancy is not None:
        occ = _c(occupancy, np.uint8)
        occ_g = round(occ.size ** (1 / 3))
        if occ_g ** 3 != occ.size:
            raise ValueError("occupancy must hold G^3 cells")
    rc = lib().orc_render(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(params), params.shape[0],
                          n_hidden, hidden, _p(o), _p(d), R, _p(ri), n, s_max, eps, int(jitter),
                          seed, _p(rgb), _p(depth), _p(opac), _p(ns), _p(flags), threads, float(footprint),
                          _p(occ), occ_g)
    if rc != 0:
        raise ValueError("orc_render failed")
    return rgb, depth, opac, ns, flags


def render_q8(tree: Tree, params, n_hidden, hidden, o, d, s_max, act_exp, eps=1e-4, ray_idx=None,
              threads=None):
    """render() of leaf samples with float8 hidden activations (exponents act_exp[L][n_hidden]):
    (rgb[n][3], depth[n], opacity[n])."""
    params = _c(params, np.float32)
    o = _c(o, np.float32); d = _c(d, np.float32)
    k = _c(act_exp, np.int32)
    assert k.shape == (params.shape[0], n_hidden)
    R = o.shape[1]
    ri, n = _sel(ray_idx, R)
    rgb = np.zeros((n, 3)); depth = np.zeros(n); opac = np.zeros(n)
    threads = threads or min(16, os.cpu_count() or 1)
    if lib().orc_render_q8(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(params), params.shape[0], n_hidden,
                           hidden, _p(o), _p(d), R, _p(ri), n, s_max, eps, _p(k), _p(rgb), _p(depth), _p(opac),
                           threads) != 0:
        raise ValueError("orc_render_q8 failed")
    return rgb, depth, opac


def act_max(tree: Tree, params, n_hidden, hidden, o, d, s_max, ray_idx=None, threads=None):
    """Calibration maxima [L][n_hidden]: the largest ReLU output of each leaf's hidden layers
    over every sample placed on the selected rays (float64, no early termination)."""
    params = _c(params, np.float32)
    o = _c(o, np.float32); d = _c(d, np.float32)
    R = o.shape[1]
    ri, n = _sel(ray_idx, R)
    out = np.zeros((params.shape[0], n_hidden))
    threads = threads or min(16, os.cpu_count() or 1)
    if lib().orc_act_max(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(params), params.shape[0], n_hidden, hidden,
                         _p(o), _p(d), R, _p(ri), n, s_max, _p(out), threads) != 0:
        raise ValueError("orc_act_max failed")
    return out


def ray_samples(tree: Tree, params, n_hidden, hidden, o, d, r, s_max, eps=1e-4, jitter=False, seed=0,
                footprint=0.0):
    """Front-to-back per-sample record of ray r as a dict of arrays."""
    params = _c(params, np.float32)
    o = _c(o, np.float32); d = _c(d, np.float32)
    cap = s_max + 1
    slot = np.zeros(cap, np.int32); t = np.zeros(cap); de = np.zeros(cap); sg = np.zeros(cap)
    rgb = np.zeros((cap, 3)); w = np.zeros(cap); ray = np.zeros(7)
    ns = lib().orc_ray_samples(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(params), params.shape[0],
                               n_hidden, hidden, _p(o), _p(d), o.shape[1], int(r), s_max, eps,
                               int(jitter), seed, cap, _p(slot), _p(t), _p(de), _p(sg), _p(rgb),
                               _p(w), _p(ray), float(footprint))
    if ns < 0:
        raise ValueError("orc_ray_samples failed")
    return dict(slot=slot[:ns], t=t[:ns], delta=de[:ns], sigma=sg[:ns], rgb=rgb[:ns], w=w[:ns],
                ray_rgb=ray[:3].copy(), depth=ray[3], opacity=ray[4], flags=int(ray[5]),
                n_used=int(ray[6]))


def render_grad(tree: Tree, params, n_hidden, hidden, o, d, s_max, g_rgb, g_depth=None,
                g_opac=None, eps=1e-4, ray_idx=None, jitter=False, seed=0, footprint=0.0):
    """dL/dparams [L][P] (float64) for upstream gradients of the rendered outputs."""
    params = _c(params, np.float32)
    o = _c(o, np.float32); d = _c(d, np.float32)
    R = o.shape[1]
    ri, n = _sel(ray_idx, R)
    g_rgb = _c(g_rgb, np.float64)
    gd = None if g_depth is None else _c(g_depth, np.float64)
    ga = None if g_opac is None else _c(g_opac, np.float64)
    grad = np.zeros(params.shape, np.float64)
    rc = lib().orc_render_grad(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(params), params.shape[0],
                               n_hidden, hidden, _p(o), _p(d), R, _p(ri), n, s_max, eps, int(jitter),
                               seed, _p(g_rgb), _p(gd), _p(ga), _p(grad), float(footprint))
    if rc != 0:
        raise ValueError("orc_render_grad failed")
    return grad


def composite(z, t, delta, eps=1e-4):
    """One ray's quadrature from its samples' output pre-activations z[ns][4]
    (sigma^, r^, g^, b^), positions t[ns] and segment lengths delta[ns]:
    ((rgb[3], depth, opacity), weights[ns], samples composited)."""
    z = _c(z, np.float64).reshape(-1, 4)
    ns = len(z)
    t = _c(t, np.float64); delta = _c(delta, np.float64)
    assert t.shape == (ns,) and delta.shape == (ns,)
    out = np.zeros(5); w = np.zeros(max(ns, 1))
    used = lib().orc_composite(ns, _p(z), _p(t), _p(delta), float(eps), _p(out), _p(w))
    return out, w[:ns], int(used)


def composite_grad(z, t, delta, g, eps=1e-4):
    """dL/dz[ns][4] for L = g . (rgb[3], depth, opacity) of composite(); (dz, samples
    composited)."""
    z = _c(z, np.float64).reshape(-1, 4)
    ns = len(z)
    t = _c(t, np.float64); delta = _c(delta, np.float64)
    g = _c(g, np.float64)
    assert g.shape == (5,)
    dz = np.zeros((max(ns, 1), 4))
    J = lib().orc_composite_grad(ns, _p(z), _p(t), _p(delta), float(eps), _p(g), _p(dz))
    return dz[:ns], int(J)


def adam(p, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays (step is 1-based)."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(g, np.float64)
    lib().orc_adam(_p(p), _p(m), _p(v), _p(g), p.size, step, lr, b1, b2, eps)


def buckets(keys, n_buckets):
    """Counts, exclusive offsets and the stable sort permutation of keys (the definition)."""
    keys = np.asarray(keys)
    counts = np.bincount(keys, minlength=n_buckets).astype(np.uint32)
    offsets = np.zeros(n_buckets + 1, np.uint32)
    offsets[1:] = np.cumsum(counts)
    perm = np.argsort(keys, kind="stable").astype(np.uint32)
    return counts, offsets, perm


def psnr(a, b, peak=1.0):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(peak * peak / mse)


# ---------------------------------------------------------------------------------------
# learned proposal
# ---------------------------------------------------------------------------------------
PROP_IN, PROP_H, PROP_BINS = 43, 64, 32


def prop_param_count():
    return int(lib().orc_prop_param_count())


def render_proposal(tree: Tree, params, n_hidden, hidden, prop, o, d, s_max, eps=1e-4, mass_thresh=0.99,
                    cap=48, ray_idx=None, threads=None, tau=None):
    """Per ray: rgb, depth, opacity, samples used, plan size (-1 = fallback), plan slots [n][cap], M^.
    tau: for a single ray, given bin thicknesses [intervals][32] in place of the network's."""
    params = _c(params, np.float32)
    prop = _c(prop, np.float32)
    o = _c(o, np.float32); d = _c(d, np.float32)
    R = o.shape[1]
    ri, n = _sel(ray_idx, R)
    rgb = np.zeros((n, 3)); depth = np.zeros(n); opac = np.zeros(n)
    ns = np.zeros(n, np.int32); pn = np.zeros(n, np.int32); psel = np.zeros((n, cap), np.int32)
    mass = np.zeros(n)
    threads = threads or min(16, os.cpu_count() or 1)
    rc = lib().orc_render_proposal(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(params), params.shape[0],
                                   n_hidden, hidden, _p(prop), _p(o), _p(d), R, _p(ri), n, s_max, eps,
                                   mass_thresh, cap, _p(rgb), _p(depth), _p(opac), _p(ns), _p(pn), _p(psel),
                                   _p(mass), threads, _p(None if tau is None else _c(tau, np.float64)))
    if rc != 0:
        raise ValueError("orc_render_proposal failed")
    return rgb, depth, opac, ns, pn, psel, mass


def prop_eval(tree: Tree, prop, o, d, s_max, ray_idx=None, cap=1 << 22):
    """Features [N][43] and predicted bin thicknesses [N][32] of every sampled interval."""
    prop = _c(prop, np.float32)
    o = _c(o, np.float32); d = _c(d, np.float32)
    R = o.shape[1]
    ri, n = _sel(ray_idx, R)
    N = int(lib().orc_prop_eval(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(prop), _p(o), _p(d), R, _p(ri), n,
                                s_max, 0, None, None))
    feat = np.zeros((N, PROP_IN)); tau = np.zeros((N, PROP_BINS))
    lib().orc_prop_eval(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(prop), _p(o), _p(d), R, _p(ri), n, s_max,
                        N, _p(feat), _p(tau))
    return feat, tau


def prop_targets(tree: Tree, params, n_hidden, hidden, o, d, s_max, ray_idx=None):
    """Bin opacities 1 - exp(-tau_b) of the plain quadrature, [N][32], intervals ray by ray."""
    params = _c(params, np.float32)
    o = _c(o, np.float32); d = _c(d, np.float32)
    R = o.shape[1]
    ri, n = _sel(ray_idx, R)
    N = int(lib().orc_prop_targets(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(params), params.shape[0],
                                   n_hidden, hidden, _p(o), _p(d), R, _p(ri), n, s_max, 0, None))
    alpha = np.zeros((N, PROP_BINS))
    lib().orc_prop_targets(_p(tree.rows), tree.n_nodes, tree.grid_n, _p(params), params.shape[0], n_hidden,
                           hidden, _p(o), _p(d), R, _p(ri), n, s_max, N, _p(alpha))
    return alpha


def prop_loss_grad(prop, feat, alpha):
    """(loss, gradient[P]) of mean((1 - exp(-tau^) - alpha)^2) over items and bins."""
    prop = _c(prop, np.float32)
    feat = _c(feat, np.float64); alpha = _c(alpha, np.float64)
    grad = np.zeros(prop_param_count())
    loss = lib().orc_prop_loss_grad(_p(prop), _p(feat), _p(alpha), len(feat), _p(grad))
    return float(loss), grad
