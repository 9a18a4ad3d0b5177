"""Pins of the oracle's reduced-precision codecs against the format definitions
and against PyTorch's CPU conversions (an independent library routine)."""
import numpy as np
import pytest
import torch


def test_bf16_decode_exhaustive(orc):
    codes = np.arange(65536, dtype=np.uint32)
    ref = torch.from_numpy(codes.astype(np.uint16).view(np.int16)).view(torch.bfloat16).float().numpy()
    ours = np.array([orc.bf16_decode(int(c)) for c in codes], dtype=np.float32)
    same = (ours.view(np.uint32) == ref.view(np.uint32)) | (np.isnan(ours) & np.isnan(ref))
    assert same.all()


def test_bf16_encode_matches_library_rne(orc):
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32),
        (rng.standard_normal(2000) * 1e-38).astype(np.float32),  # subnormal range
        np.array([0.0, -0.0, 1.0, -1.0, 3.3895314e38, 1e-45], dtype=np.float32),
    ])
    # exact ties: low 16 bits == 0x8000, both parities of the kept bit
    base = rng.integers(0x3F000000, 0x40000000, 2000, dtype=np.uint32) & 0xFFFF0000
    ties = (base | 0x8000).view(np.float32)
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    ours = np.array([orc.bf16_encode(float(v)) for v in x], dtype=np.uint16)
    assert np.array_equal(ours, ref)


def test_e4m3_decode_exhaustive(orc):
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).double().numpy()
    ours = np.array([orc.e4m3_decode(int(c)) for c in codes])
    same = (ours == ref) | (np.isnan(ours) & np.isnan(ref))
    assert same.all()
    assert np.nanmax(ours) == 448.0 and np.isnan(ours[0x7F]) and np.isnan(ours[0xFF])
    assert ours[1] == 2.0 ** -9  # smallest subnormal


def test_e4m3_encode_matches_library_in_range(orc):
    rng = np.random.default_rng(1)
    x = np.concatenate([
        (rng.standard_normal(20000) * 50).astype(np.float32),
        (rng.standard_normal(2000) * 0.01).astype(np.float32),
        np.array([0.0, -0.0, 448.0, -448.0, 2.0 ** -10, 3 * 2.0 ** -11], dtype=np.float32),
    ])
    # midpoints between neighbouring codes (exact ties)
    vals = np.array([orc.e4m3_decode(c) for c in range(0, 0x7E)])
    mids = ((vals[:-1] + vals[1:]) / 2).astype(np.float32)
    x = np.concatenate([x, mids, -mids])
    x = x[np.abs(x) <= 448.0]
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    ours = np.array([orc.e4m3_encode(float(v)) for v in x], dtype=np.uint8)
    assert np.array_equal(ours, ref)


def test_e4m3_saturates(orc):
    assert orc.e4m3_encode(449.0) == 0x7E
    assert orc.e4m3_encode(1e30) == 0x7E
    assert orc.e4m3_encode(-1e30) == 0xFE
    assert orc.e4m3_encode(float("nan")) == 0x7F


@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
def test_quantize_scales_and_roundtrip(orc, fmt):
    rng = np.random.default_rng(2)
    X = (rng.standard_normal((37, 5)) * np.array([1.0, 1e-3, 0.0, 250.0, 7.0])).astype(np.float32)
    codes, scale = orc.quantize(X, fmt)
    qmax = np.float32(448.0 if fmt == "e4m3" else 1.0)
    amax = np.abs(X).max(axis=0)
    expect = np.where(amax > 0, amax / qmax, np.float32(1.0)).astype(np.float32)
    assert np.array_equal(scale, expect)
    Xt = orc.dequantize(codes, scale, fmt)
    rel = 2.0 ** -8 if fmt == "bf16" else 2.0 ** -3  # half an ulp of the fraction width
    err = np.abs(Xt - X) / np.maximum(amax, 1e-30)
    assert np.all(err[:, amax > 0] <= rel)
    assert np.all(Xt[:, 2] == 0.0)
    # each code is the correctly rounded x / s
    q = X / scale
    if fmt == "bf16":
        ref = torch.from_numpy(np.ascontiguousarray(q)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    else:
        ref = torch.from_numpy(np.ascontiguousarray(q)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(np.ascontiguousarray(codes), ref)


def test_e4m3_encode_dense_sweep(orc):
    """Every binary32 value in [-480, 480] whose low 13 bits are zero (about
    half a million values, several per E4M3 interval, including every code
    and every midpoint) encodes as the library conversion does (saturating
    above 448, where the library's conversion is not defined)."""
    bits = np.arange(0, 0x43F00000 >> 13, dtype=np.uint32) << 13   # 0 .. 480.0
    x = bits.view(np.float32)
    x = np.concatenate([x, -x])
    inr = np.abs(x) <= 448.0
    ref = torch.from_numpy(x[inr]).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    ours = np.array([orc.e4m3_encode(float(v)) for v in x], dtype=np.uint8)
    assert np.array_equal(ours[inr], ref)
    sat = np.where(x[~inr] > 0, 0x7E, 0xFE).astype(np.uint8)
    assert np.array_equal(ours[~inr], sat)
    # the matrix quantiser (one column whose largest magnitude is 448: scale 1)
    codes, scale = orc.quantize(np.asfortranarray(x[inr][:, None]), "e4m3")
    assert scale[0] == 1.0
    assert np.array_equal(np.asarray(codes).ravel(), ref)
