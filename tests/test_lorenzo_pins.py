"""Pins of the quantizing front end's oracle (oracle/lorenzo.py) to facts
that do not come from the oracle itself.

- Prequantization: values that are exact multiples of 2 eb (a power-of-two
  bound, so every product is exact) give their multiple; exact half-way
  values round to the even neighbour; huge finite values clamp to +-2^24;
  a field holding a NaN or an infinity is refused (no error bound covers a
  non-finite value).
- A 2x2x2 field whose codes are derived by hand below.
- Residual: summing it back along the three axes (the predictor's inverse,
  a 3D prefix sum) recovers the prequantized integers; on tiny grids it
  equals the eight-neighbour inclusion-exclusion sum evaluated point by
  point; on one axis it is numpy's first difference; it annihilates any
  field that is a sum of terms each independent of one axis.
- Codes: the outlier rule at its edges for several radii.
- Slabs: the partition tiles [0, n) with block-aligned starts.
- A plausible mistake planted in a copy of the residual (a dropped axis, a
  wrong sign, a transposed axis) fails the inverse pin.
"""
import itertools

import numpy as np
import pytest

from oracle import lorenzo as lz


def _inverse(e):
    """The predictor's inverse: prefix sums along every axis."""
    d = np.asarray(e, dtype=np.int64)
    for axis in range(d.ndim):
        d = np.cumsum(d, axis=axis)
    return d


# -- prequantization ---------------------------------------------------------

def test_prequantize_exact_multiples():
    inv = 512.0  # eb = 2^-10, 2 eb = 2^-9
    k = np.arange(-5000, 5001, dtype=np.int64)
    x = (k.astype(np.float64) / 512.0).astype(np.float32)
    assert np.array_equal(lz.prequantize(x, inv), k)


def test_prequantize_ties_to_even():
    inv = 512.0
    k = np.arange(-300, 300, dtype=np.int64)
    x = ((k.astype(np.float64) + 0.5) / 512.0).astype(np.float32)  # exactly half-way
    d = lz.prequantize(x, inv)
    even = np.where(k % 2 == 0, k, k + 1)  # k + 0.5 rounds to whichever of k, k + 1 is even
    assert np.array_equal(d, even)
    assert np.array_equal(lz.prequantize(np.float32([0.5, 1.5, 2.5, -0.5, -1.5, -2.5]), 1.0),
                          [0, 2, 2, 0, -2, -2])


def test_prequantize_rounding_error_at_most_half():
    rng = np.random.default_rng(3)
    x = rng.normal(0, 100, 100_000).astype(np.float32)
    inv = 1.0 / (2 * 0.01)
    d = lz.prequantize(x, inv)
    exact = x.astype(np.float64) * np.float64(np.float32(inv))
    # the float32 product is within half an ulp of the exact one (< 2^-24 relative)
    assert np.all(np.abs(exact - d) <= 0.5 + np.abs(exact) * 2.0 ** -24)


def test_prequantize_huge_values_clamp():
    x = np.float32([1e30, -1e30, 16777216.0 * 4, -16777216.0 * 4, 3e38, -0.0])
    # 3e38 * 4 overflows the float32 product to +inf, which clamps like any huge value
    assert list(lz.prequantize(x, 4.0)) == [1 << 24, -(1 << 24), 1 << 24, -(1 << 24), 1 << 24, 0]


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_non_finite_values_are_rejected(bad):
    x = np.zeros((2, 3, 4), dtype=np.float32)
    x[1, 2, 3] = bad
    with pytest.raises(lz.NonFiniteInput):
        lz.prequantize(x, 1.0)
    with pytest.raises(lz.NonFiniteInput):
        lz.lorenzo_codes(x, 1.0, 8)


def test_hand_derived_2x2x2():
    # x[i, j, k] with 2 eb = 1 (r = 1): rint gives d = 1 4 / 2 8 / 3 5 / 7 20
    # (2.5 -> 2, 7.5 -> 8 and 19.5 -> 20 are ties to even).  Residual
    # e = sum over (a, b, c) in {0, 1}^3 of (-1)^(a + b + c) d[i - a, j - b, k - c]:
    #   e000 = 1                          e001 = 4 - 1 = 3
    #   e010 = 2 - 1 = 1                  e011 = 8 - 2 - 4 + 1 = 3
    #   e100 = 3 - 1 = 2                  e101 = 5 - 3 - 4 + 1 = -1
    #   e110 = 7 - 3 - 2 + 1 = 3          e111 = 20 - 7 - 5 - 8 + 3 + 2 + 4 - 1 = 8
    # radius 4: code = e + 4 inside [1, 7], else 0; e111 + 4 = 12 is an outlier.
    x = np.float32([[[0.6, 4.4], [2.5, 7.5]], [[2.75, 5.0], [7.25, 19.5]]])
    assert np.array_equal(lz.prequantize(x, 1.0).reshape(-1), [1, 4, 2, 8, 3, 5, 7, 20])
    assert np.array_equal(lz.lorenzo_residual(lz.prequantize(x, 1.0)).reshape(-1), [1, 3, 1, 3, 2, -1, 3, 8])
    assert np.array_equal(lz.lorenzo_codes(x, 1.0, 4), [5, 7, 5, 7, 6, 3, 7, 0])
    # one NaN anywhere refuses the whole field
    y = x.copy()
    y[0, 1, 0] = np.nan
    with pytest.raises(lz.NonFiniteInput):
        lz.lorenzo_codes(y, 1.0, 4)


# -- residual ----------------------------------------------------------------

@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 9), (1, 7, 5), (4, 1, 6), (3, 4, 5), (6, 2, 3), (5, 5, 1)])
def test_residual_inverse_recovers_input(shape):
    rng = np.random.default_rng(sum(shape))
    d = rng.integers(-(1 << 24), (1 << 24) + 1, size=shape)
    assert np.array_equal(_inverse(lz.lorenzo_residual(d)), d)


def test_residual_is_eight_neighbour_sum():
    rng = np.random.default_rng(11)
    d = rng.integers(-1000, 1000, size=(3, 4, 5))
    e = lz.lorenzo_residual(d)

    def at(i, j, k):
        return int(d[i, j, k]) if i >= 0 and j >= 0 and k >= 0 else 0

    for i, j, k in itertools.product(range(3), range(4), range(5)):
        want = 0
        for a, b, c in itertools.product((0, 1), repeat=3):
            want += (-1) ** (a + b + c) * at(i - a, j - b, k - c)
        assert e[i, j, k] == want, (i, j, k)


def test_residual_one_axis_is_first_difference():
    rng = np.random.default_rng(5)
    d = rng.integers(-50, 50, size=(1, 1, 40))
    assert np.array_equal(lz.lorenzo_residual(d).reshape(-1), np.diff(d.reshape(-1), prepend=0))


def test_residual_annihilates_axis_free_terms():
    rng = np.random.default_rng(8)
    nz, ny, nx = 6, 7, 8
    f = rng.integers(-100, 100, size=(1, ny, nx))
    g = rng.integers(-100, 100, size=(nz, 1, nx))
    h = rng.integers(-100, 100, size=(nz, ny, 1))
    d = f + g + h
    e = lz.lorenzo_residual(d)
    assert not e[1:, 1:, 1:].any()
    c = lz.lorenzo_residual(np.full((3, 3, 3), 17))
    assert c[0, 0, 0] == 17 and np.count_nonzero(c) == 1


# -- codes -------------------------------------------------------------------

@pytest.mark.parametrize("radius", [1, 2, 4, 512, 8192])
def test_codes_outlier_rule(radius):
    e = np.arange(-radius - 3, radius + 4, dtype=np.int64)
    q = lz.residual_codes(e, radius)
    for ei, qi in zip(e, q):
        if -radius < ei < radius:
            assert qi == ei + radius
        else:
            assert qi == 0


def test_codes_end_to_end_constant_and_ramp():
    # constant field: only the origin is predicted from zeros
    x = np.full((4, 4, 4), 3.0, dtype=np.float32)
    q = lz.lorenzo_codes(x, 1.0, 8).reshape(4, 4, 4)
    assert q[0, 0, 0] == 3 + 8 and np.all(q.reshape(-1)[1:] == 8)
    # a ramp along the fastest axis: residual 1 on the first row, 0 elsewhere
    x = np.broadcast_to(np.arange(6, dtype=np.float32), (3, 4, 6))
    q = lz.lorenzo_codes(x, 1.0, 8).reshape(3, 4, 6)
    assert np.all(q[0, 0, 1:] == 9) and q[0, 0, 0] == 8
    rest = q.copy()
    rest[0, 0, :] = 8
    assert np.all(rest == 8)


# -- slabs -------------------------------------------------------------------

@pytest.mark.parametrize("n,s", [(1, 1), (4096, 1), (10000, 2), (10000, 3), (1 << 20, 7), (123457, 30)])
def test_slab_bounds_tile_the_stream(n, s):
    b = lz.slab_bounds(n, s)
    assert b[0][0] == 0 and b[-1][1] == n
    for (lo, hi), (lo2, _) in zip(b, b[1:]):
        assert hi == lo2 and lo % 4096 == 0
    assert lz.slab_bounds(10000, 2) == [(0, 4096), (4096, 10000)]


def test_slab_histograms_sum_to_histogram():
    rng = np.random.default_rng(2)
    codes = rng.integers(0, 64, size=50_000).astype(np.uint16)
    rows = lz.slab_histograms(codes, 64, 5)
    assert rows.shape == (5, 64)
    assert np.array_equal(rows.sum(axis=0), np.bincount(codes, minlength=64))


# -- planted mistakes --------------------------------------------------------

def _drop_axis(d):
    e = np.array(d, dtype=np.int64)
    for axis in (0, 2):
        e = np.diff(e, axis=axis, prepend=0)
    return e


def _wrong_sign(d):
    e = np.array(d, dtype=np.int64)
    for axis in range(3):
        e = np.diff(e, axis=axis, prepend=0)
    e[1:, 1:, 1:] += 2 * d[:-1, :-1, :-1]  # flips the sign of the far corner
    return e


def _shifted_axis(d):
    e = np.array(d, dtype=np.int64)
    for axis in range(3):
        e = np.diff(e, axis=axis, prepend=0)
    return np.roll(e, 1, axis=2)


@pytest.mark.parametrize("wrong", [_drop_axis, _wrong_sign, _shifted_axis])
def test_inverse_pin_catches_planted_mistakes(wrong):
    rng = np.random.default_rng(4)
    d = rng.integers(-100, 100, size=(3, 4, 5))
    assert not np.array_equal(_inverse(wrong(d)), d)
    assert np.array_equal(_inverse(lz.lorenzo_residual(d)), d)


def test_agrees_with_float64_division_almost_everywhere():
    """The generator of the Huffman workloads divides in float64; the front
    end multiplies by a float32 reciprocal.  The two readings of the
    prequantization may differ only where x / (2 eb) is within rounding of a
    half-integer, a tiny fraction of a smooth field."""
    import torch

    from paper_2010_10039_amd import workloads

    x, eb = workloads.lorenzo_field(dim=48, seed=3)
    q = lz.lorenzo_codes(x, float(np.float32(1.0 / (2.0 * eb))), 512)
    d64 = torch.round(torch.from_numpy(x).to(torch.float64) / (2.0 * eb)).to(torch.int64).numpy()
    q64 = lz.residual_codes(lz.lorenzo_residual(d64), 512).reshape(-1)
    assert np.mean(q != q64) < 1e-3
