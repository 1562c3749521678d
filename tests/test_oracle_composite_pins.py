"""Pins of the oracle's per-ray compositing (the quadrature of Section 3.1 with the early
termination of Section 4.1) and of its gradient, and of the full rendering gradient with
early termination switched on.

`oracle.composite` / `oracle.composite_grad` take one ray's per-sample output
pre-activations; the GPU's compositing backward is compared with them sample by sample.
Pins: closed forms of a constant-density ray, agreement with the full renderer on the
rays of the small scene, central differences (early termination off and on, on rays whose
stop index cannot move under the perturbation), and torch float64 autograd of the same
quadrature written with torch operations.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def inv_softplus(s):
    return np.log(np.expm1(s))


def logit(c):
    return np.log(c / (1.0 - c))


def c1_setup():
    cfg = synth.C1
    g = synth.make_grid(cfg)
    tree = oracle.build_tree(g, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
    dens = synth.leaf_mean_density(g, cfg.grid_n, tree.leaf_boxes())
    W = synth.make_weights(tree.n_leaves, cfg.n_hidden, cfg.hidden, cfg.seed_weights, dens)
    return cfg, tree, W


def ray_records(eps, n_rays=144, s_max=64):
    """Per-sample records of the small scene's rays: (z[ns][4], t, delta, record)."""
    cfg, tree, W = c1_setup()
    o, d = synth.camera_rays(synth.make_cameras(1, 301, 12, 12)[0])
    out = []
    for r in range(min(n_rays, o.shape[1])):
        rec = oracle.ray_samples(tree, W, cfg.n_hidden, cfg.hidden, o, d, r, s_max, eps=eps)
        if len(rec["t"]) == 0:
            continue
        J = rec["n_used"]
        z = np.zeros((len(rec["t"]), 4))    # samples after the stop are never read
        z[:J] = np.column_stack([inv_softplus(rec["sigma"][:J]), logit(rec["rgb"][:J])])
        out.append((z, rec["t"], rec["delta"], rec))
    return out


def stop_margin(sigma, delta, eps, J):
    """Log-distance from eps of the transmittances that decide the stop: the stop index
    cannot move while every T_{j+1}, j < J - 1, stays above eps and T_J (after the stop
    sample, or at the end of the ray) stays on its side."""
    T = np.exp(-np.cumsum(sigma * delta))
    m = np.inf
    for j in range(J):
        m = min(m, abs(math.log(T[j] / eps)))
    return m


# ---------------------------------------------------------------------------
# forward
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 7, 40])
def test_constant_density_closed_forms(n):
    """Equal samples of a constant density: opacity 1 - e^{-sigma L}, colour c times it,
    depth the geometric series of the centred strata."""
    sigma0, L, t_in = 2.7, 1.3, 0.4
    delta = L / n
    t = t_in + (np.arange(n) + 0.5) * delta
    cz = np.array([0.3, -1.1, 2.0])
    z = np.column_stack([np.full(n, inv_softplus(sigma0)), np.tile(cz, (n, 1))])
    out, w, used = oracle.composite(z, t, np.full(n, delta), eps=0.0)
    c = 1 / (1 + np.exp(-cz))
    assert used == n
    assert abs(out[4] - (1 - math.exp(-sigma0 * L))) < 1e-14
    np.testing.assert_allclose(out[:3], c * (1 - math.exp(-sigma0 * L)), rtol=0, atol=1e-14)
    q = math.exp(-sigma0 * delta)
    S0 = (1 - q ** n) / (1 - q)
    S1 = q * (1 - n * q ** (n - 1) + (n - 1) * q ** n) / (1 - q) ** 2
    D = (1 - q) * ((t_in + 0.5 * delta) * S0 + delta * S1)
    assert abs(out[3] - D) < 1e-13
    assert abs(w.sum() - (1 - math.exp(-sigma0 * L))) < 1e-14


def test_constant_density_stop_index():
    """T_{j+1} = e^{-sigma delta (j+1)}: the first j with T_{j+1} < eps is
    ceil(ln(1/eps) / (sigma delta)) - 1; later samples get weight 0."""
    sigma0, delta, n, eps = 5.0, 0.1, 64, 1e-4
    z = np.column_stack([np.full(n, inv_softplus(sigma0)), np.zeros((n, 3))])
    t = (np.arange(n) + 0.5) * delta
    out, w, used = oracle.composite(z, t, np.full(n, delta), eps=eps)
    j_stop = math.ceil(math.log(1 / eps) / (sigma0 * delta)) - 1
    assert used == j_stop + 1
    assert np.all(w[used:] == 0)
    assert abs(out[4] - (1 - math.exp(-sigma0 * delta * used))) < 1e-14


@pytest.mark.parametrize("eps", [0.0, 1e-4])
def test_composite_equals_full_renderer(eps):
    """From the per-sample record of the full renderer, the ray outputs, the weights and the
    number of samples composited are reproduced (to the rounding of the inverted heads)."""
    recs = ray_records(eps)
    n_stop = 0
    for z, t, delta, rec in recs:
        out, w, used = oracle.composite(z, t, delta, eps=eps)
        assert used == rec["n_used"]
        np.testing.assert_allclose(out[:3], rec["ray_rgb"], rtol=0, atol=1e-12)
        assert abs(out[3] - rec["depth"]) < 1e-12 and abs(out[4] - rec["opacity"]) < 1e-12
        np.testing.assert_allclose(w, rec["w"], rtol=0, atol=1e-12)
        n_stop += used < len(t)
    assert len(recs) > 50
    if eps > 0:
        assert n_stop > 0


# ---------------------------------------------------------------------------
# gradient
# ---------------------------------------------------------------------------
def fd_grad(z, t, delta, g, eps, h=1e-6):
    G = np.zeros_like(z)
    for j in range(z.shape[0]):
        for k in range(4):
            zp = z.copy(); zp[j, k] += h
            zm = z.copy(); zm[j, k] -= h
            fp = oracle.composite(zp, t, delta, eps)[0] @ g
            fm = oracle.composite(zm, t, delta, eps)[0] @ g
            G[j, k] = (fp - fm) / (2 * h)
    return G


@pytest.mark.parametrize("eps", [0.0, 1e-4])
def test_composite_grad_matches_central_differences(eps):
    rng = np.random.default_rng(11)
    recs = ray_records(eps)
    checked = stops = 0
    for z, t, delta, rec in recs[::3]:
        J = rec["n_used"]
        if eps > 0 and stop_margin(rec["sigma"], delta, eps, J) < 0.1:
            continue            # the stop index could move under the perturbation
        g = rng.standard_normal(5)
        dz, Jg = oracle.composite_grad(z, t, delta, g, eps=eps)
        assert Jg == J
        fd = fd_grad(z, t, delta, g, eps)
        # central differences with h = 1e-6 on an O(1) loss carry ~1e-10 of rounding
        scale = np.abs(fd).max()
        assert np.abs(dz - fd).max() <= 2e-9 + 1e-7 * scale, (np.abs(dz - fd).max(), scale)
        assert np.all(dz[J:] == 0)
        checked += 1
        stops += J < len(t)
    assert checked >= 15
    if eps > 0:
        assert stops >= 3


def test_composite_grad_matches_torch_autograd():
    """The same truncated quadrature written with torch float64 operations and
    differentiated by autograd (stop index taken from the oracle's forward)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    recs = ray_records(1e-4)
    for z, t, delta, rec in recs[::5]:
        J = rec["n_used"]
        g = rng.standard_normal(5)
        dz, _ = oracle.composite_grad(z, t, delta, g, eps=1e-4)
        zt = torch.tensor(z[:J], dtype=torch.float64, requires_grad=True)
        tt = torch.tensor(t[:J], dtype=torch.float64)
        dt = torch.tensor(delta[:J], dtype=torch.float64)
        tau = torch.nn.functional.softplus(zt[:, 0]) * dt
        S_excl = torch.cumsum(tau, 0) - tau
        w = torch.exp(-S_excl) * (-torch.expm1(-tau))
        c = torch.sigmoid(zt[:, 1:])
        L = (g[0] * (w * c[:, 0]).sum() + g[1] * (w * c[:, 1]).sum() + g[2] * (w * c[:, 2]).sum()
             + g[3] * (w * tt).sum() + g[4] * w.sum())
        L.backward()
        np.testing.assert_allclose(dz[:J], zt.grad.numpy(), rtol=0, atol=1e-11 * max(1.0, np.abs(dz).max()))


def test_empty_ray():
    out, w, used = oracle.composite(np.zeros((0, 4)), np.zeros(0), np.zeros(0))
    assert used == 0 and np.all(out == 0)
    dz, J = oracle.composite_grad(np.zeros((0, 4)), np.zeros(0), np.zeros(0), np.ones(5))
    assert J == 0 and dz.shape == (0, 4)


# ---------------------------------------------------------------------------
# full rendering gradient with early termination on
# ---------------------------------------------------------------------------
def stable_rays(tree, W, cfg, o, d, s_max, eps, margin=0.1, footprint=0.0):
    """Rays whose stop index cannot move under a small parameter perturbation."""
    keep = []
    for r in range(o.shape[1]):
        rec = oracle.ray_samples(tree, W, cfg.n_hidden, cfg.hidden, o, d, r, s_max, eps=eps, footprint=footprint)
        ns = len(rec["t"])
        if ns == 0:
            continue
        if stop_margin(rec["sigma"], rec["delta"], eps, rec["n_used"]) >= margin:
            keep.append(r)
    return np.array(keep, np.int64)


def fd_check(tree, W, cfg, o, d, sel, s_max, eps, rng, footprint=0.0):
    g_rgb = rng.standard_normal((len(sel), 3))
    g_dep = rng.standard_normal(len(sel)) * 0.1
    g_op = rng.standard_normal(len(sel)) * 0.1
    grad = oracle.render_grad(tree, W, cfg.n_hidden, cfg.hidden, o, d, s_max, g_rgb, g_dep, g_op, eps=eps,
                              ray_idx=sel, footprint=footprint)

    def loss(Wp):
        rgb, dep, op, _, _ = oracle.render(tree, Wp, cfg.n_hidden, cfg.hidden, o, d, s_max, eps=eps, ray_idx=sel,
                                           footprint=footprint)
        return (rgb * g_rgb).sum() + (dep * g_dep).sum() + (op * g_op).sum()

    n_sets, P = W.shape
    sb = synth.sigma_bias_offset(cfg.n_hidden, cfg.hidden)
    idx = [(l, int(i)) for l in range(n_sets) for i in rng.choice(P, 4, replace=False)]
    idx += [(l, sb) for l in range(n_sets)] + [(l, sb + 1) for l in range(n_sets)]
    checked = 0
    for l, i in idx:
        base = float(W[l, i])
        h = 2.0 ** -16 * max(1.0, abs(base))
        fds = []
        for hh in (h, h / 4):
            Wp = W.copy(); Wp[l, i] = np.float32(base + hh)
            Wm = W.copy(); Wm[l, i] = np.float32(base - hh)
            fds.append((loss(Wp) - loss(Wm)) / (float(Wp[l, i]) - float(Wm[l, i])))
        if abs(fds[0] - fds[1]) > 1e-6 * max(1.0, abs(fds[0])):
            continue            # the window straddles a ReLU kink
        assert abs(grad[l, i] - fds[1]) <= 1e-7 * max(1.0, abs(fds[1])), (l, i, grad[l, i], fds[1])
        checked += 1
    return checked, len(idx)


def test_render_gradient_with_early_termination_matches_central_differences():
    cfg, tree, W = c1_setup()
    o, d = synth.camera_rays(synth.make_cameras(1, 301, 16, 16)[0])
    eps, s_max = 1e-4, 64
    sel = stable_rays(tree, W, cfg, o, d, s_max, eps)
    # the subset must contain rays that stop early
    _, _, _, ns, flags = oracle.render(tree, W, cfg.n_hidden, cfg.hidden, o, d, s_max, eps=eps, ray_idx=sel)
    n_fired = int(((flags & oracle.FLAG_ERT_FIRED) != 0).sum())
    assert n_fired >= 10, n_fired
    checked, total = fd_check(tree, W, cfg, o, d, sel, s_max, eps, np.random.default_rng(5))
    assert checked >= 0.8 * total


def test_render_gradient_with_early_termination_under_hierarchical_sampling():
    cfg = synth.C1
    g = synth.make_grid(cfg)
    tree = oracle.build_tree(g, cfg.grid_n, cfg.max_depth, cfg.max_leaves)
    rows = tree.rows
    boxes = rows[np.argsort(rows[:, 11])][:, 2:8].copy()
    dens = synth.leaf_mean_density(g, cfg.grid_n, boxes)
    W = synth.make_weights(len(boxes), cfg.n_hidden, cfg.hidden, cfg.seed_weights, dens)
    o, d = synth.camera_rays(synth.make_cameras(1, 301, 16, 16)[0])
    eps, s_max, f = 1e-4, 64, 0.5
    sel = stable_rays(tree, W, cfg, o, d, s_max, eps, footprint=f)
    _, _, _, ns, flags = oracle.render(tree, W, cfg.n_hidden, cfg.hidden, o, d, s_max, eps=eps, ray_idx=sel,
                                       footprint=f)
    assert int(((flags & oracle.FLAG_ERT_FIRED) != 0).sum()) >= 10
    checked, total = fd_check(tree, W, cfg, o, d, sel, s_max, eps, np.random.default_rng(6), footprint=f)
    assert checked >= 0.8 * total
