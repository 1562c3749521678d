"""The float64 error report on the GPU against numpy float64 on the same seeded data."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2310_01881_amd as am  # noqa: E402


def _report(ctx, x, ref, sel=None):
    xd = torch.from_numpy(x).to("cuda:0")
    rd = torch.from_numpy(ref).to("cuda:0")
    sd = None if sel is None else torch.from_numpy(sel.astype(np.uint8)).to("cuda:0")
    return am.amnerf_error_stats(ctx.h, xd, rd, sd)


@pytest.mark.parametrize("n", [0, 1, 1000, 1_000_003, 3 * 640_000])
def test_matches_numpy(n):
    rng = np.random.default_rng(7 + n)
    ref = rng.random(n)
    x = (ref + rng.normal(0.0, 1e-3, n)).astype(np.float32)
    sel = rng.random(n) < 0.9
    ctx = am.Context(0)
    for mask in (None, sel):
        r = _report(ctx, x, ref, mask)
        m = np.ones(n, bool) if mask is None else mask
        e = x.astype(np.float64)[m] - ref[m]
        assert r["count"] == int(m.sum())
        if r["count"] == 0:
            assert r["max_abs"] == 0.0 and r["sum_sq"] == 0.0
            continue
        assert r["max_abs"] == np.abs(e).max()          # same float64 differences, max is exact
        assert abs(r["sum_sq"] - np.sum(e * e)) <= 1e-12 * np.sum(e * e)
        assert abs(r["sum_abs"] - np.sum(np.abs(e))) <= 1e-12 * np.sum(np.abs(e))
        assert abs(r["psnr"] - 10 * np.log10(1.0 / np.mean(e * e))) <= 1e-9


def test_deterministic_and_nan():
    rng = np.random.default_rng(3)
    ref = rng.random(500_000)
    x = ref.astype(np.float32)
    ctx = am.Context(0)
    a = _report(ctx, x, ref)
    b = _report(ctx, x, ref)
    assert a == b
    x[1234] = np.nan
    c = _report(ctx, x, ref)
    assert c["max_abs"] == float("inf")
