"""The FP8 E4M3 input encoding: torch's codes and values against the
format's definition (all 256 codes), and the per-column quantiser's bounds."""
import math

import numpy as np
import torch

import abg_synth as synth


def test_e4m3_code_table():
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8).view(torch.float8_e4m3fn)
    got = codes.to(torch.float64).numpy()
    for b in range(256):
        want = synth.e4m3_value(b)
        if math.isnan(want):
            assert math.isnan(got[b]), b
        else:
            assert got[b] == want, (b, got[b], want)
    assert synth.e4m3_value(0x7E) == 448.0 and synth.e4m3_value(0x01) == 2.0 ** -9


def test_quantiser_bounds():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal((500, 37)) * rng.uniform(0.01, 100.0, 37)).astype(np.float32)
    x[:, 5] = 0.0
    codes, scale, values = synth.quantize_e4m3(x)
    assert codes.dtype == np.uint8 and codes.shape == x.shape and scale.dtype == np.float32
    assert scale[5] == 1.0 and np.all(values[:, 5] == 0.0)
    table = np.array([synth.e4m3_value(b) for b in range(256)])
    dec = table[codes] * scale.astype(np.float64)[None, :]
    assert np.array_equal(dec, values)  # the values are the codes' definition times the scales
    assert np.all(np.isfinite(values))
    # round to nearest: within half a unit of E4M3's 3-bit mantissa (relative
    # 2^-4) for normal codes, within half the subnormal step below
    y = x.astype(np.float64) / scale.astype(np.float64)[None, :]
    q = values / scale.astype(np.float64)[None, :]
    err = np.abs(q - y)
    assert np.all(err <= np.maximum(np.abs(y) * 2.0 ** -4, 2.0 ** -10) * (1 + 1e-6))
    assert np.max(np.abs(q)) <= 448.0
