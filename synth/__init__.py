"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the bench.

This module only *makes inputs*: guidance density grids, pinhole-camera rays and
per-leaf MLP parameter sets.  It holds none of the method's arithmetic (no tree
construction, traversal, sampling, inference or compositing), so the CPU oracle
and the HIP path can both consume its arrays without sharing any code.

The paper's scenes (NeRF synthetic/real scenes, Ueno, Dragon, Material, House1/2;
Section 4.1) are not available; the seeded scenes below stand in for them with the
shape of the paper's workloads: an axis-aligned scene box, density concentrated in
blobs and a ground slab, a few hundred to a few thousand KD-tree leaves
(Section 4.1 caps the tree near 1k nodes), and 64-192 samples per ray, which
brackets the 24-145 average samples per ray of the comparison table (Section 4.3).

Conventions
-----------
* Grid: float32[N^3], index ``i + N*(j + N*k)`` (x fastest); cell (i,j,k) is the
  value at the cell centre ((i+1/2)/N, (j+1/2)/N, (k+1/2)/N); scene box [0,1]^3.
* Rays: SoA float32 ``o[3][R]``, ``d[3][R]``; computed in float64 then rounded.
* MLP parameters: float32 ``[L][P]``; per linear layer ``W[out][in]`` row-major
  followed by ``b[out]``.  Input width 30 (27 positional-encoding features of the
  sample position followed by the 3 view-direction components), output width 4
  (sigma pre-activation, then r, g, b pre-activations).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

IN_DIM = 30
OUT_DIM = 4


# ----------------------------------------------------------------------------
# Configurations of the five synthetic workloads
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class SceneConfig:
    name: str
    k: int                      # workload number; seeds are base + k
    grid_n: int
    n_blobs: int
    anisotropic: bool
    s_range: tuple
    amp_range: tuple
    ground_cells: int = 0       # cells with z index < ground_cells get ground_amp added
    ground_amp: float = 0.0
    skew: float = 1.0           # blob count per unit volume in [0,1/2)^3 vs elsewhere
    max_depth: int = 3
    max_leaves: int = 8
    n_hidden: int = 2
    hidden: int = 32
    width: int = 64
    height: int = 64
    s_max: int = 64
    ert_eps: float = 1e-4
    n_cameras: int = 1

    @property
    def seed_scene(self): return 100 + self.k

    @property
    def seed_weights(self): return 200 + self.k

    @property
    def seed_cameras(self): return 300 + self.k

    @property
    def seed_student(self): return 400 + self.k

    @property
    def seed_proposal(self): return 500 + self.k

    @property
    def seed_batches(self): return 600 + self.k


C1 = SceneConfig(name="c1_64px_8leaf_2x32", k=1, grid_n=32, n_blobs=20, anisotropic=False,
                 s_range=(0.05, 0.2), amp_range=(5.0, 50.0), max_depth=3, max_leaves=8,
                 n_hidden=2, hidden=32, width=64, height=64, s_max=64)
C2 = SceneConfig(name="c2_800px_512leaf_4x64", k=2, grid_n=128, n_blobs=200, anisotropic=True,
                 s_range=(0.02, 0.15), amp_range=(5.0, 50.0), ground_cells=10, ground_amp=100.0,
                 max_depth=12, max_leaves=512, n_hidden=4, hidden=64, width=800, height=800,
                 s_max=128)
C3 = SceneConfig(name="c3_1080p_4096leaf_4x64", k=3, grid_n=256, n_blobs=2000, anisotropic=True,
                 s_range=(0.01, 0.08), amp_range=(5.0, 50.0), skew=100.0, max_depth=12,
                 max_leaves=4096, n_hidden=4, hidden=64, width=1920, height=1080, s_max=192,
                 n_cameras=30)
CONFIGS = {"c1": C1, "c2": C2, "c3": C3}


def scaled(cfg: SceneConfig, **kw) -> SceneConfig:
    """A copy of ``cfg`` with some fields replaced (small test variants)."""
    d = dict(cfg.__dict__)
    d.update(kw)
    return SceneConfig(**d)


# ----------------------------------------------------------------------------
# Guidance density grid
# ----------------------------------------------------------------------------
def _random_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def make_grid(cfg: SceneConfig) -> np.ndarray:
    """Sum of truncated Gaussian blobs (plus an optional ground slab) at cell centres.

    Each blob is ``A * exp(-0.5 * m^2)`` with ``m`` its Mahalanobis distance; terms with
    ``m > 4`` are dropped (the blob is evaluated on the bounding box of that ellipsoid).
    """
    n = cfg.grid_n
    rng = np.random.Generator(np.random.PCG64(cfg.seed_scene))
    g = np.zeros((n, n, n), dtype=np.float64)          # indexed [k][j][i]
    centres = (np.arange(n, dtype=np.float64) + 0.5) / n
    if cfg.skew != 1.0:
        # blob count per unit volume in the octant [0,1/2)^3 is `skew` times the rest
        n_rest = int(round(cfg.n_blobs / (1.0 + cfg.skew / 7.0)))
        n_oct = cfg.n_blobs - n_rest
        regions = [0] * n_oct + [1] * n_rest
    else:
        regions = [2] * cfg.n_blobs
    # blob parameters are drawn in order; the boxes are evaluated on a thread pool (numpy
    # releases the interpreter lock inside its array kernels) and summed in blob order
    blobs = []
    for reg in regions:
        if reg == 0:
            mu = rng.uniform(0.0, 0.5, 3)
        elif reg == 1:
            while True:
                mu = rng.uniform(0.0, 1.0, 3)
                if not np.all(mu < 0.5):
                    break
        else:
            mu = rng.uniform(0.1, 0.9, 3)
        amp = rng.uniform(*cfg.amp_range)
        if cfg.anisotropic:
            s = rng.uniform(*cfg.s_range, 3)
            rot = _random_rotation(rng)
            cov = rot @ np.diag(s * s) @ rot.T
        else:
            s1 = rng.uniform(*cfg.s_range)
            cov = np.eye(3) * s1 * s1
        blobs.append((mu, amp, cov))

    def box(blob):
        mu, amp, cov = blob
        prec = np.linalg.inv(cov)
        half = 4.0 * np.sqrt(np.diag(cov))
        lo = np.clip(np.floor((mu - half) * n).astype(int), 0, n)
        hi = np.clip(np.ceil((mu + half) * n).astype(int) + 1, 0, n)
        if np.any(hi <= lo):
            return None
        xs = centres[lo[0]:hi[0]] - mu[0]
        ys = centres[lo[1]:hi[1]] - mu[1]
        zs = centres[lo[2]:hi[2]] - mu[2]
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        m2 = (prec[0, 0] * X * X + prec[1, 1] * Y * Y + prec[2, 2] * Z * Z
              + 2.0 * (prec[0, 1] * X * Y + prec[0, 2] * X * Z + prec[1, 2] * Y * Z))
        val = amp * np.exp(-0.5 * m2)
        val[m2 > 16.0] = 0.0
        return lo, hi, val

    workers = max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as pool:
        window = 2 * workers
        futs = [pool.submit(box, b) for b in blobs[:window]]
        for i in range(len(blobs)):
            r = futs[i].result()
            futs[i] = None
            if i + window < len(blobs):
                futs.append(pool.submit(box, blobs[i + window]))
            if r is not None:
                lo, hi, val = r
                g[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += val
    if cfg.ground_cells > 0:
        g[:cfg.ground_cells, :, :] += cfg.ground_amp
    return np.ascontiguousarray(g.astype(np.float32).reshape(-1))


# ----------------------------------------------------------------------------
# Cameras and rays
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Camera:
    position: tuple
    width: int
    height: int
    fov_y_deg: float = 40.0


def make_cameras(n: int, seed: int, width: int, height: int, radius: float = 2.0,
                 fov_y_deg: float = 40.0) -> list:
    """Pinhole cameras on a sphere of ``radius`` around the scene centre, looking at it.

    Directions are uniform on the sphere, redrawn while |u_z| > 0.95 so that the
    +z up vector is never (nearly) parallel to the view direction.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cams = []
    while len(cams) < n:
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        if abs(u[2]) > 0.95:
            continue
        pos = np.array([0.5, 0.5, 0.5]) + radius * u
        cams.append(Camera(tuple(float(v) for v in pos), width, height, fov_y_deg))
    return cams


def camera_rays(cam: Camera) -> tuple:
    """Rays through the pixel centres of ``cam``: float32 SoA ``o[3][R]``, ``d[3][R]``.

    Pixel (i, j) is row-major with j the row from the top; R = width*height.
    """
    W, H = cam.width, cam.height
    pos = np.array(cam.position, dtype=np.float64)
    centre = np.array([0.5, 0.5, 0.5])
    f = centre - pos
    f /= np.linalg.norm(f)
    up = np.array([0.0, 0.0, 1.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(math.radians(cam.fov_y_deg) / 2.0)
    aspect = W / H
    xs = ((np.arange(W, dtype=np.float64) + 0.5) / W * 2.0 - 1.0) * th * aspect
    ys = (1.0 - (np.arange(H, dtype=np.float64) + 0.5) / H * 2.0) * th
    Y, X = np.meshgrid(ys, xs, indexing="ij")
    d = f[:, None] + X.reshape(1, -1) * r[:, None] + Y.reshape(1, -1) * u[:, None]
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    o = np.broadcast_to(pos[:, None], d.shape)
    return (np.ascontiguousarray(o.astype(np.float32)),
            np.ascontiguousarray(d.astype(np.float32)))


def random_pixel_rays(cams: list, n: int, seed: int) -> tuple:
    """Rays through n seeded random pixel centres of random cameras (all cameras share W, H)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ci = rng.integers(0, len(cams), n)
    W, H = cams[0].width, cams[0].height
    px = rng.integers(0, W * H, n)
    o = np.empty((3, n), np.float64)
    d = np.empty((3, n), np.float64)
    up = np.array([0.0, 0.0, 1.0])
    centre = np.array([0.5, 0.5, 0.5])
    for c in np.unique(ci):
        sel = np.where(ci == c)[0]
        cam = cams[c]
        pos = np.array(cam.position, dtype=np.float64)
        f = centre - pos
        f /= np.linalg.norm(f)
        r = np.cross(f, up)
        r /= np.linalg.norm(r)
        u = np.cross(r, f)
        th = math.tan(math.radians(cam.fov_y_deg) / 2.0)
        i = px[sel] % W
        j = px[sel] // W
        x = ((i + 0.5) / W * 2.0 - 1.0) * th * (W / H)
        y = (1.0 - (j + 0.5) / H * 2.0) * th
        dd = f[:, None] + x[None, :] * r[:, None] + y[None, :] * u[:, None]
        dd /= np.linalg.norm(dd, axis=0, keepdims=True)
        d[:, sel] = dd
        o[:, sel] = pos[:, None]
    return np.ascontiguousarray(o.astype(np.float32)), np.ascontiguousarray(d.astype(np.float32))


def rays_for_cameras(cams: list) -> tuple:
    """Concatenated rays of several cameras (camera-major)."""
    os_, ds_ = zip(*(camera_rays(c) for c in cams))
    return np.ascontiguousarray(np.concatenate(os_, axis=1)), np.ascontiguousarray(np.concatenate(ds_, axis=1))


def random_rays(n: int, seed: int, inside_frac: float = 0.5) -> tuple:
    """Rays with random origins (some inside the box, some outside) and random directions."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_in = int(n * inside_frac)
    o_in = rng.uniform(0.0, 1.0, (3, n_in))
    u = rng.standard_normal((3, n - n_in))
    u /= np.linalg.norm(u, axis=0, keepdims=True)
    o_out = 0.5 + 2.0 * u
    o = np.concatenate([o_in, o_out], axis=1)
    tgt = rng.uniform(0.1, 0.9, (3, n))
    d = tgt - o
    d[:, :n_in] = rng.standard_normal((3, n_in))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    return np.ascontiguousarray(o.astype(np.float32)), np.ascontiguousarray(d.astype(np.float32))


# ----------------------------------------------------------------------------
# Per-leaf MLP parameters
# ----------------------------------------------------------------------------
def layer_dims(n_hidden: int, hidden: int) -> list:
    """(in, out) of each linear layer: 30 -> H, (n_hidden-1) x H -> H, H -> 4."""
    dims = [(IN_DIM, hidden)] + [(hidden, hidden)] * (n_hidden - 1) + [(hidden, OUT_DIM)]
    return dims


def param_count(n_hidden: int, hidden: int) -> int:
    return sum(i * o + o for i, o in layer_dims(n_hidden, hidden))


def sigma_bias_offset(n_hidden: int, hidden: int) -> int:
    """Offset of the sigma-output bias inside one leaf's parameter block."""
    off = 0
    dims = layer_dims(n_hidden, hidden)
    for i, o in dims[:-1]:
        off += i * o + o
    i, o = dims[-1]
    return off + i * o


def leaf_mean_density(grid: np.ndarray, n: int, leaf_boxes: np.ndarray) -> np.ndarray:
    """Mean guidance density over the cells of each integer leaf box [lo, hi)^3."""
    g = grid.reshape(n, n, n).astype(np.float64)
    out = np.empty(len(leaf_boxes))
    for s, (lx, ly, lz, hx, hy, hz) in enumerate(leaf_boxes):
        out[s] = g[lz:hz, ly:hy, lx:hx].mean()
    return out


def inverse_softplus(y: np.ndarray) -> np.ndarray:
    y = np.maximum(np.asarray(y, dtype=np.float64), 1e-4)
    return np.where(y > 30.0, y, np.log(np.expm1(np.minimum(y, 30.0))))


def make_weights(n_leaves: int, n_hidden: int, hidden: int, seed: int,
                 leaf_density: np.ndarray | None = None) -> np.ndarray:
    """He-normal float32 parameters ``[L][P]``; biases zero except the sigma bias.

    The sigma-output bias of leaf ``s`` is softplus^-1 of its mean guidance density,
    so that the random field's density follows the guidance grid leaf by leaf.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    P = param_count(n_hidden, hidden)
    out = np.zeros((n_leaves, P), dtype=np.float64)
    for s in range(n_leaves):
        off = 0
        for fi, fo in layer_dims(n_hidden, hidden):
            w = rng.standard_normal((fo, fi)) * math.sqrt(2.0 / fi)
            out[s, off:off + fi * fo] = w.reshape(-1)
            off += fi * fo + fo
    if leaf_density is not None:
        out[:, sigma_bias_offset(n_hidden, hidden)] = inverse_softplus(leaf_density)
    return np.ascontiguousarray(out.astype(np.float32))


def leaf_boxes_from_nodes(nodes: np.ndarray) -> np.ndarray:
    """Leaf boxes [L][6] in slot order from an exported node table ([n][12] int32)."""
    leaves = nodes[nodes[:, 10] >= 0]
    leaves = leaves[np.argsort(leaves[:, 10])]
    return np.ascontiguousarray(leaves[:, 2:8])


# ----------------------------------------------------------------------------
# Proposal network parameters
# ----------------------------------------------------------------------------
PROP_DIMS = [(43, 64), (64, 64), (64, 32)]


def make_prop_weights(seed: int) -> np.ndarray:
    """He-normal float32 parameters of the 43 -> 64 -> 64 -> 32 proposal MLP, biases 0.

    Layout as the leaf MLPs: per layer W[out][in] row-major, then b[out]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fi, fo in PROP_DIMS:
        parts.append((rng.standard_normal((fo, fi)) * math.sqrt(2.0 / fi)).reshape(-1))
        parts.append(np.zeros(fo))
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))
