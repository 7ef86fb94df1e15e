"""The 2-byte scene format's host-side converters (input preparation, not
method arithmetic): BF16 and FP16 rounding to nearest, ties to even."""
import numpy as np

from paper_2606_09074_amd import synth


def _bf16_nearest_brute(x: np.ndarray) -> np.ndarray:
    """Nearest BF16 by comparing the two truncation neighbours in FP64 (ties
    to the even mantissa): an independent route to the same rounding."""
    u = x.view(np.uint32)
    lo = (u >> 16).astype(np.uint32)
    hi = lo + 1
    vlo = (lo << 16).view(np.float32).astype(np.float64)
    vhi = (hi << 16).view(np.float32).astype(np.float64)
    xd = x.astype(np.float64)
    dlo, dhi = np.abs(xd - vlo), np.abs(vhi - xd)
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ((lo & 1) == 1))
    return np.where(pick_hi, hi, lo).astype(np.uint16)


def test_bf16_round_to_nearest_even():
    rng = np.random.default_rng(11)
    x = (rng.standard_normal(200_000) * np.exp(rng.uniform(-30, 30, 200_000))).astype(np.float32)
    np.testing.assert_array_equal(synth.f32_to_bf16_bits(x), _bf16_nearest_brute(x))


def test_bf16_ties_and_specials():
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 3.4e38, -3.4e38, np.inf, -np.inf,
                  0.0, -0.0], dtype=np.float32)
    got = synth.f32_to_bf16_bits(x)
    assert [hex(v) for v in got] == ["0x3f80", "0x3f80", "0x3f82", "0xbf80", "0x7f80", "0xff80", "0x7f80",
                                     "0xff80", "0x0", "0x8000"]
    nan = synth.f32_to_bf16_bits(np.array([np.nan, -np.nan], dtype=np.float32))
    assert np.all(np.isnan(synth.bf16_bits_to_f32(nan)))


def test_mixed_round_trip_and_plane_split():
    spec = synth.SMALL.with_n(3000)
    planes = synth.make_planes(spec)
    q = synth.quantize_bf16_f16(planes)
    assert q.dtype == np.int16 and q.shape == planes.shape
    d = synth.dequantize_bf16_f16(q)
    # geometry and opacity planes are BF16 (8 significant bits), SH planes IEEE half
    np.testing.assert_array_equal(synth.f32_to_bf16_bits(planes[:11]), q[:11].view(np.uint16))
    np.testing.assert_array_equal(planes[11:].astype(np.float16), q[11:].view(np.float16))
    rel = np.abs(d[:11] - planes[:11]) / np.abs(planes[:11])
    assert rel.max() <= 2.0 ** -8       # unit roundoff of an 8-bit significand
    # already representable values survive a second conversion unchanged
    np.testing.assert_array_equal(synth.quantize_bf16_f16(d), q)


def test_half_format_round_trip():
    """The half 2-byte format: every plane IEEE half (numpy's conversion,
    checked against the two neighbouring halves in FP64), within half a unit
    of an 11-bit significand of the FP32 value for the scene's normal-range
    values."""
    spec = synth.SMALL.with_n(3000)
    planes = synth.make_planes(spec)
    h = synth.quantize_f16(planes)
    assert h.dtype == np.float16 and h.shape == planes.shape
    d = synth.dequantize_f16(h)
    x = planes.astype(np.float64)
    lo = np.nextafter(h, np.float16(-np.inf)).astype(np.float64)
    hi = np.nextafter(h, np.float16(np.inf)).astype(np.float64)
    err = np.abs(d.astype(np.float64) - x)
    assert np.all(err <= np.abs(lo - x)) and np.all(err <= np.abs(hi - x))   # nearest half
    normal = np.abs(x) >= 2.0 ** -14
    assert np.all(err[normal] <= 2.0 ** -11 * np.abs(x[normal]))
    np.testing.assert_array_equal(synth.quantize_f16(d), h)
