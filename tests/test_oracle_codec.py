"""Pins for the reference FP8 (E4M3FN) and BF16 codecs."""
import numpy as np
import torch

from oracle import codec


def test_e4m3_anchor_codes():
    tab = codec.e4m3_table()
    assert tab[0x7E] == 448.0                 # largest finite
    assert np.isnan(tab[0x7F]) and np.isnan(tab[0xFF])
    assert tab[0x01] == 2.0 ** -9             # smallest subnormal
    assert tab[0x08] == 2.0 ** -6             # smallest normal
    assert tab[0x38] == 1.0
    assert tab[0xB8] == -1.0
    finite = tab[~np.isnan(tab)]
    assert len(np.unique(finite)) == 253      # +0 and -0 compare equal
    assert np.all(np.diff(tab[:0x7F]) > 0)


def test_e4m3_matches_torch_in_range():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 30, rng.uniform(-448, 448, 20000),
                        rng.standard_normal(5000) * 1e-3, codec.e4m3_table()[:0x7F]])
    x = x.astype(np.float32)
    ours = codec.e4m3_encode(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)
    # midpoints between neighbours go to the even code
    pos = codec.e4m3_table()[:0x7F]
    mid = ((pos[:-1] + pos[1:]) / 2).astype(np.float32)
    c = codec.e4m3_encode(mid)
    assert np.all(c % 2 == 0)


def test_e4m3_saturates():
    c = codec.e4m3_encode(np.array([449.0, 1e6, -1e30, 464.0, 480.0]))
    assert list(c) == [0x7E, 0x7E, 0xFE, 0x7E, 0x7E]


def test_bf16_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(50000), rng.standard_normal(1000) * 1e-30,
                        rng.standard_normal(1000) * 1e30]).astype(np.float32)
    # exact ties: low 16 bits 0x8000
    ties = (rng.integers(0, 2 ** 31, 1000).astype(np.uint32) & 0xFFFF0000) | 0x8000
    x = np.concatenate([x, ties.view(np.float32)])
    x = x[np.isfinite(x)]
    ours = codec.bf16_encode(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_quantize_roundtrip_bound():
    rng = np.random.default_rng(2)
    k = (rng.standard_normal((300, 166)) / (1 + np.arange(166) % 31)).astype(np.float32)
    k[5] = 0.0
    for kind, rel in [("bf16", 2.0 ** -8), ("fp8", 2.0 ** -4)]:  # unit roundoff 2^-p
        codes, s = codec.quantize(k, kind)
        assert s[5] == 1.0
        back = codec.dequantize(codes, s, kind)
        err = np.abs(back - k)
        # half an ulp of the scaled value (8 and 4 significant bits), plus the fp8 subnormal floor
        floor = s[:, None] * (2.0 ** -10 if kind == "fp8" else 0.0)
        bound = rel * np.abs(k) * (1 + 1e-6) + floor + 1e-7 * np.abs(k)
        assert np.all(err <= bound)
