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


def test_library_e4m3_encoder_matches_round_to_nearest_even():
    """The encoder the sparse-attribute form stages codes with
    (tpo_e4m3_encode, host side of the same function the staging kernel
    runs): every code's value maps to that code, every midpoint between
    neighbouring codes goes to the even one, values beyond 448 saturate, and
    random values of all magnitudes agree with torch's E4M3 conversion."""
    import paper_2405_11922_amd as tpo

    tpo.load_library()
    enc = tpo.tpo_e4m3_encode
    table = [synth.e4m3_value(b) for b in range(256)]
    for b in range(256):
        v = table[b]
        if math.isnan(v):
            continue
        got = enc(v)
        assert table[got] == v and (got & 0x80) == (b & 0x80), (b, got, v)
    pos = sorted({table[b] for b in range(0x7F) if not math.isnan(table[b])})
    for lo, hi in zip(pos[:-1], pos[1:]):
        mid = 0.5 * (lo + hi)  # exact in binary32 for E4M3 neighbours
        got = enc(mid)
        b_lo, b_hi = table.index(lo), table.index(hi)
        assert got == (b_lo if b_lo % 2 == 0 else b_hi), (lo, hi, got)
        assert enc(-mid) == (got | 0x80)
    assert enc(448.0) == 0x7E and enc(1e6) == 0x7E and enc(-1e6) == 0xFE and enc(float("nan")) == 0x7F
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-4, 2.6, 20000)).astype(np.float32)
    x = np.clip(x, -448.0, 448.0)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = np.array([enc(float(v)) for v in x], dtype=np.uint8)
    assert np.array_equal(got, want)
