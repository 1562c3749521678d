"""Pins of the oracle's float8 e4m3 quantiser against the OCP E4M3 definition."""
from __future__ import annotations

import numpy as np

from oracle import fp8


def test_spec_table_values():
    # values the OCP 8-bit floating-point specification lists for E4M3
    cases = {
        0x7E: 448.0,             # largest normal  S.1111.110
        0x08: 2.0 ** -6,         # smallest normal S.0001.000
        0x07: 0.875 * 2 ** -6,   # largest subnormal S.0000.111
        0x01: 2.0 ** -9,         # smallest subnormal S.0000.001
        0x38: 1.0,               # exponent field 7 = bias
        0x00: 0.0,
    }
    for code, v in cases.items():
        assert fp8.decode(code) == v
        assert fp8.encode(v) == code
        assert fp8.encode(-v) == (code | 0x80 if v else 0)
    assert np.isnan(fp8.decode(0x7F)) and np.isnan(fp8.decode(0xFF))


def test_every_finite_code_round_trips():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F and c != 0x80])
    assert np.array_equal(fp8.encode(fp8.decode(codes)), codes.astype(np.uint8))


def test_nearest_with_ties_to_even_against_brute_force():
    vals = fp8.decode(np.arange(127))
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-500, 500, 4000),
                        rng.standard_normal(4000) * 0.05,
                        (vals[:-1] + vals[1:]) / 2,           # exact midpoints
                        -(vals[:-1] + vals[1:]) / 2])
    got = fp8.decode(fp8.encode(x))
    a = np.minimum(np.abs(x), 448.0)
    dist = np.abs(a[:, None] - vals[None, :])
    best = dist.min(axis=1)
    assert not np.isnan(got).any()
    assert np.allclose(np.abs(np.abs(got) - a), best, rtol=0, atol=0)
    mids = np.concatenate([(vals[:-1] + vals[1:]) / 2])
    mc = fp8.encode(mids).astype(int)
    assert np.all(mc % 2 == 0)                       # ties go to the even code
    assert np.all(np.sign(got[x != 0]) * np.sign(x[x != 0]) >= 0)


def test_saturation_and_monotone():
    assert np.all(fp8.encode([449.0, 463.9, 464.0, 1e6, 1e30]) == 0x7E)
    assert np.all(fp8.encode([-449.0, -1e6]) == 0xFE)
    x = np.linspace(0, 500, 20001)
    v = fp8.decode(fp8.encode(x))
    assert np.all(np.diff(v) >= 0)


def test_quantise_scales_codes_and_exact_grid():
    n_hidden, hidden = 2, 32
    sl = fp8.layer_slices(n_hidden, hidden)
    P = sl[-1][3] + 4
    rng = np.random.default_rng(1)
    W = rng.standard_normal((3, P)).astype(np.float32)
    W[2, sl[1][0]:sl[1][0] + hidden * hidden] = 0.0         # an all-zero layer: scale 1
    scales, codes, deq = fp8.quantise(W, n_hidden, hidden)
    for li, (ow, din, dout, ob) in enumerate(sl):
        w = W[:, ow:ow + din * dout]
        for leaf in range(3):
            mx = np.abs(w[leaf]).max()
            if mx == 0:
                assert scales[leaf, li] == 1.0 and not codes[li][leaf].any()
                continue
            assert scales[leaf, li] == np.float32(mx) / np.float32(448)
            # the largest weight lands on the largest code
            assert (codes[li][leaf][np.argmax(np.abs(w[leaf]))] & 0x7F) == 0x7E
            # relative error of a normal-range weight is at most half a mantissa step, 1/16
            big = np.abs(w[leaf]) / scales[leaf, li] >= 2.0 ** -6
            err = np.abs(deq[leaf, ow:ow + din * dout] - w[leaf])
            assert np.all(err[big] <= np.abs(w[leaf][big]) / 16 * (1 + 1e-6))
        # biases pass through unchanged
        assert np.array_equal(deq[:, ob:ob + dout], W[:, ob:ob + dout].astype(np.float64))
    # weights already on the scaled e4m3 grid are reproduced exactly
    grid = fp8.decode(rng.integers(0, 126, size=(2, P))) * 0.25
    for ow, din, dout, ob in sl:
        grid[:, ow] = 448 * 0.25                            # every layer's max: scale 0.25
    g32 = grid.astype(np.float32)
    _, _, deq2 = fp8.quantise(g32, n_hidden, hidden)
    for ow, din, dout, ob in sl:
        assert np.array_equal(deq2[:, ow:ow + din * dout], g32[:, ow:ow + din * dout].astype(np.float64))
