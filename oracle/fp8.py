"""Float8 e4m3 weight quantisation for the oracle -- TEST INFRASTRUCTURE.

The paper computes in full precision; the float8 variant of the leaf MLPs stores each
linear layer's weights as e4m3 codes with one float32 scale per leaf and layer.  This
module states that storage from its definitions, independently of the HIP path:

* e4m3 is the OCP 8-bit floating-point format E4M3: a sign bit, 4 exponent bits with bias
  7 and 3 mantissa bits; exponent field 0 holds the subnormals m/8 * 2^-6; there are no
  infinities, the all-ones pattern S.1111.111 is NaN, so the largest finite value is
  S.1111.110 = 448.  Conversion rounds to the nearest value, ties to the even code, and
  saturates at 448.
* The scale of a layer is max |W| / 448 in float32 (1 for an all-zero layer); the codes
  are e4m3(W / scale) with the division in float32.

The encoder looks the value up in the table of all finite codes (``decode`` of 0..126)
rather than by exponent arithmetic, so it shares no steps with the device encoder.

The float8 matrix-core variant (``quantise_mma``) also rounds the hidden activations, so
both operands of every hidden and output layer are e4m3, and all its scales are powers of
two (an exact rescaling, applied by the matrix instruction's block scales):

* a weight layer l >= 1 gets the exponent e = the smallest integer with max |W| <= 448 * 2^e
  (0 for an all-zero layer) and the codes e4m3(W / 2^e); the first layer's weights are
  bfloat16 (round to nearest even), its inputs being the bfloat16 positional encoding;
  biases stay float32;
* hidden layer j's ReLU outputs a get the exponent k = the smallest integer with
  1.25 * m <= 256 * 2^k, m the calibration maximum of that leaf and layer (0 when m = 0),
  and are held as 2^k * e4m3(min(a / 2^k, 256)) (the oracle's C forward applies this):
  saturation at 256, the largest power of two e4m3 holds, lets the kernel apply ReLU and
  saturation as one clamp to [0, 1] before a conversion that scales by 2^8.
"""
from __future__ import annotations

import numpy as np

MAX = 448.0


def decode(codes) -> np.ndarray:
    """Value of each e4m3 code (float64); NaN for the two NaN codes."""
    c = np.asarray(codes, dtype=np.int64) & 0xFF
    e = (c >> 3) & 15
    m = c & 7
    mag = np.where(e == 0, m / 8.0 * 2.0 ** -6, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    mag = np.where((c & 0x7F) == 0x7F, np.nan, mag)
    return np.where(c & 0x80, -mag, mag)


_TABLE = decode(np.arange(127))          # the 127 non-negative finite values, increasing


def encode(x) -> np.ndarray:
    """e4m3 codes (uint8) of x: nearest value, ties to the even code, saturating at 448.

    The sign bit is set for x < 0 (so -0.0 encodes as +0)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), MAX)
    hi = np.clip(np.searchsorted(_TABLE, a, side="left"), 1, 126)   # _TABLE[hi-1] < a <= _TABLE[hi]
    lo = hi - 1
    dlo = a - _TABLE[lo]
    dhi = _TABLE[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    code = np.where(a == 0.0, 0, code)
    return (code | np.where(x < 0, 0x80, 0)).astype(np.uint8)


def layer_slices(n_hidden: int, hidden: int):
    """(w_offset, din, dout, b_offset) of every linear layer of one leaf's master vector."""
    dims = [(30, hidden)] + [(hidden, hidden)] * (n_hidden - 1) + [(hidden, 4)]
    out, off = [], 0
    for din, dout in dims:
        out.append((off, din, dout, off + din * dout))
        off += din * dout + dout
    return out


def quantise(W: np.ndarray, n_hidden: int, hidden: int):
    """Per leaf and layer: (scales float32[L][n_layers], codes list per layer [L][dout*din]
    uint8, dequantised float64 parameters [L][P] with the biases unchanged)."""
    W = np.asarray(W, dtype=np.float32)
    L = W.shape[0]
    sl = layer_slices(n_hidden, hidden)
    scales = np.zeros((L, len(sl)), np.float32)
    codes = []
    deq = W.astype(np.float64).copy()
    for li, (ow, din, dout, _) in enumerate(sl):
        w = W[:, ow:ow + din * dout]
        mx = np.abs(w).max(axis=1)
        s = np.where(mx > 0, mx / np.float32(MAX), np.float32(1.0)).astype(np.float32)
        q = encode((w / s[:, None]).astype(np.float32))
        scales[:, li] = s
        codes.append(q)
        deq[:, ow:ow + din * dout] = decode(q) * s[:, None].astype(np.float64)
    return scales, codes, deq


def bf16_round(x) -> np.ndarray:
    """float32 values rounded to the nearest bfloat16 (ties to even), as float32; finite inputs."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def pow2_exponent(m, limit: float) -> np.ndarray:
    """Smallest integer e with m <= limit * 2^e, elementwise for m > 0; 0 where m == 0."""
    m = np.asarray(m, dtype=np.float64)
    out = np.zeros(m.shape, np.int32)
    for idx in zip(*np.nonzero(m > 0)):
        v = float(m[idx])
        e = int(np.ceil(np.log2(v / limit)))
        while v > limit * 2.0 ** e:          # exact comparisons settle the logarithm's rounding
            e += 1
        while v <= limit * 2.0 ** (e - 1):
            e -= 1
        out[idx] = e
    return out


ACT_SAT = 256.0   # float8 activations saturate at ACT_SAT * 2^k


def act_exponents(act_max) -> np.ndarray:
    """Activation exponents [L][n_hidden] from float32 calibration maxima: 1.25 m <= 256 * 2^k."""
    m = np.asarray(act_max, dtype=np.float32).astype(np.float64)
    return pow2_exponent(1.25 * m, ACT_SAT)


def quantise_mma(W: np.ndarray, n_hidden: int, hidden: int, act_max):
    """The float8 matrix-core model of the leaf MLPs: (weight exponents int32[L][n_hidden] of
    layers 1..n_hidden, activation exponents int32[L][n_hidden], dequantised parameters
    float32[L][P] -- every value exact in float32 -- for the oracle's forward with float8
    activations)."""
    W = np.asarray(W, dtype=np.float32)
    L = W.shape[0]
    sl = layer_slices(n_hidden, hidden)
    deq = W.copy()
    ow, din, dout, _ = sl[0]
    deq[:, ow:ow + din * dout] = bf16_round(W[:, ow:ow + din * dout])
    w_exp = np.zeros((L, n_hidden), np.int32)
    for li in range(1, n_hidden + 1):
        ow, din, dout, _ = sl[li]
        w = W[:, ow:ow + din * dout].astype(np.float64)
        e = pow2_exponent(np.abs(w).max(axis=1), MAX)
        w_exp[:, li - 1] = e
        scaled = w * np.exp2(-e.astype(np.float64))[:, None]          # exact
        deq[:, ow:ow + din * dout] = (decode(encode(scaled)) * np.exp2(e.astype(np.float64))[:, None]).astype(np.float32)
    return w_exp, act_exponents(act_max), deq
