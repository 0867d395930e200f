"""Pins of the oracle's number formats and latent generator against library
routines and published values (not against the oracle itself)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O


def test_e4m3_decode_exhaustive_vs_torch():
    # torch.float8_e4m3fn implements the OCP FP8 E4M3 format (bias 7, no inf)
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    mine = np.array([O.lib().orc_e4m3_to_f64(int(c)) for c in codes])
    nan = np.isnan(ref)
    assert (np.isnan(mine) == nan).all()
    assert nan.sum() == 2 and nan[0x7F] and nan[0xFF]  # S.1111.111 only
    np.testing.assert_array_equal(mine[~nan], ref[~nan])


def test_e4m3_landmarks():
    dec = O.lib().orc_e4m3_to_f64
    assert dec(0x7E) == 448.0  # largest finite, OCP spec
    assert dec(0x01) == 2.0 ** -9  # smallest subnormal
    assert dec(0x08) == 2.0 ** -6  # smallest normal
    assert dec(0x38) == 1.0
    assert O.round_fmt(1e6, "e4m3") == 448.0  # saturating conversion
    assert O.round_fmt(-470.0, "e4m3") == -448.0


def test_e4m3_rounding_vs_torch():
    g = np.random.default_rng(0)
    x = np.concatenate([g.uniform(-448, 448, 4000), g.uniform(-1, 1, 4000), g.uniform(-0.05, 0.05, 4000),
                        np.array([0.0, 2.0 ** -10, 3 * 2.0 ** -11, 1.0625, 1.1875, 240.0, 232.0, 440.0])])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    mine = np.array([O.round_fmt(float(v), "e4m3") for v in x32])
    np.testing.assert_array_equal(mine, ref)


def test_bf16_rounding_vs_torch():
    g = np.random.default_rng(1)
    bits = g.integers(0, 2 ** 32, 20000, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    x = x[np.isfinite(x) & (np.abs(x) < 3e38)]
    # add exact ties: values halfway between two bf16 numbers
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, -ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    mine = np.array([O.round_fmt(float(v), "bf16") for v in x])
    np.testing.assert_array_equal(mine, ref)


def test_f16_rounding_and_decode_vs_numpy():
    g = np.random.default_rng(2)
    x = np.concatenate([g.standard_normal(5000) * 1e-4, g.standard_normal(5000), g.uniform(-7e4, 7e4, 2000),
                        g.uniform(-1e-7, 1e-7, 2000)])
    ref = x.astype(np.float16).astype(np.float64)  # numpy rounds binary64 -> binary16 directly
    mine = np.array([O.round_fmt(float(v), "f16") for v in x])
    np.testing.assert_array_equal(mine, ref)
    allbits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    ref = allbits.view(np.float16).astype(np.float64)
    mine = np.array([O.lib().orc_f16_to_f64(int(b)) for b in allbits])
    fin = np.isfinite(ref)
    np.testing.assert_array_equal(mine[fin], ref[fin])
    assert (np.isnan(mine) == np.isnan(ref)).all()
    enc = np.array([O.lib().orc_f64_to_f16_bits(float(v)) for v in ref[fin]], np.uint16)
    np.testing.assert_array_equal(enc.view(np.float16).astype(np.float64), ref[fin])


def test_bf16_decode_vs_torch():
    b = np.arange(0, 65536, 7, dtype=np.int64).astype(np.int16)
    ref = torch.from_numpy(b).view(torch.bfloat16).to(torch.float64).numpy()
    mine = np.array([O.lib().orc_bf16_to_f64(int(v) & 0xFFFF) for v in b])
    fin = np.isfinite(ref)
    np.testing.assert_array_equal(mine[fin], ref[fin])


def test_philox_published_vector():
    # Random123 known-answer vector for philox4x64-10, counter 0, key 0
    out = O.philox4x64_10([0, 0, 0, 0], [0, 0])
    assert [int(v) for v in out] == [0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B,
                                      0x7E68B68AEC7BA23B]


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((123, 7), (5, 0, 0, 0)),
                                     ((2 ** 64 - 1, 3), (2 ** 64 - 1, 9, 0, 0))])
def test_philox_vs_numpy(key, ctr):
    # numpy's Philox is philox4x64-10; it increments the 256-bit counter before each block
    bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
    raw = bg.random_raw(4)
    c = list(ctr)
    for i in range(4):
        c[i] = (c[i] + 1) % 2 ** 64
        if c[i]:
            break
    assert [int(v) for v in O.philox4x64_10(c, key)] == [int(v) for v in raw]


def test_init_values_uniform():
    v = O.init_grid(seed=5, obj=3, amp=1e-4, grid_dtype="f32", count=200000).astype(np.float64)
    assert v.min() >= -1e-4 and v.max() < 1e-4
    # uniform on [-1e-4, 1e-4): mean 0, variance amp^2 / 3
    assert abs(v.mean()) < 5 * 1e-4 / np.sqrt(3 * 200000)
    assert abs(v.var() / (1e-8 / 3) - 1) < 0.02
    h = O.init_grid(seed=5, obj=3, amp=1e-4, grid_dtype="f16", count=1000)
    np.testing.assert_array_equal(h.view(np.float16).astype(np.float32), v[:1000].astype(np.float32).astype(np.float16))
    # a window equals the same slice of the whole
    w = O.init_grid(seed=5, obj=3, amp=1e-4, grid_dtype="f32", count=77, begin=1001)
    np.testing.assert_array_equal(w, v[1001:1078].astype(np.float32))
    # subnormal half latents are kept (|v| < 6.1e-5 is subnormal in binary16)
    hv = h.view(np.float16).astype(np.float64)
    assert ((np.abs(hv) < 6.1e-5) & (hv != 0)).sum() > 100
