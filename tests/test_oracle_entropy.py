"""Pins of the best-view oracle (Eq. 2) against closed forms and brute force."""
import math

import numpy as np

from oracle import entropy as E


def _frame(vals):
    """A 1 x len(vals) frame whose pixels are grey (r = g = b = v)."""
    v = np.asarray(vals, dtype=np.float32)
    f = np.zeros((1, 1, len(v), 4), dtype=np.float32)
    f[..., 0] = f[..., 1] = f[..., 2] = v
    f[..., 3] = 1.0
    return f


def test_constant_image_has_zero_entropy():
    assert E.entropy(E.histograms(_frame([0.3] * 50))[0]) == 0.0


def test_two_equal_halves_is_one_bit():
    assert E.entropy(E.histograms(_frame([0.0] * 8 + [1.0] * 8))[0]) == 1.0


def test_uniform_over_all_codes_is_eight_bits():
    vals = np.arange(256) / 255.0
    h = E.histograms(_frame(vals))[0]
    assert (h == 1).all()
    assert abs(E.entropy(h) - 8.0) < 1e-12


def test_entropy_closed_form_for_k_equal_bins():
    for k in (3, 5, 7, 100):
        assert abs(E.entropy(np.ones(k)) - math.log2(k)) < 1e-12


def test_entropy_brute_force_and_permutation():
    rng = np.random.default_rng(1)
    c = rng.integers(0, 50, size=256)
    n = c.sum()
    ref = 0.0
    for x in c:
        if x:
            ref -= (x / n) * math.log2(x / n)
    assert abs(E.entropy(c) - ref) < 1e-12
    assert abs(E.entropy(rng.permutation(c)) - ref) < 1e-12


def test_channel_codes_round_half_up_and_clamp():
    c = np.array([-1.0, 0.0, 0.5 / 255, 1.5 / 255, 0.5, 1.0, 2.0, np.float32(254.5 / 255)], dtype=np.float32)
    q = E.channel_codes(c)
    assert q[0] == 0 and q[1] == 0 and q[5] == 255 and q[6] == 255
    assert q[4] == 128                      # 127.5 + 0.5 -> 128
    assert q[2] in (0, 1) and q[3] in (1, 2)
    assert (q >= 0).all() and (q <= 255).all()


def test_grey_weights_sum_to_one():
    # equal channels map to themselves: (256 q + 128) >> 8 = q
    q = np.arange(256, dtype=np.float32) / 255.0
    f = np.stack([q, q, q, np.ones_like(q)], axis=-1)[None, None]
    assert (E.grey_codes(f)[0, 0] == np.arange(256)).all()
    # pure primaries
    f = np.zeros((1, 1, 3, 4), dtype=np.float32)
    f[0, 0, 0, 0] = f[0, 0, 1, 1] = f[0, 0, 2, 2] = 1.0
    assert E.grey_codes(f)[0, 0].tolist() == [(77 * 255 + 128) >> 8, (150 * 255 + 128) >> 8, (29 * 255 + 128) >> 8]


def test_best_view_is_first_maximum():
    a = _frame([0.0] * 16)
    b = _frame([0.0] * 8 + [1.0] * 8)
    c = _frame([0.0] * 4 + [0.4] * 4 + [0.7] * 4 + [1.0] * 4)
    frames = np.concatenate([a, b, c, c, b])
    best, H = E.best_view(frames)
    assert best == 2
    assert np.allclose(H, [0.0, 1.0, 2.0, 2.0, 1.0])


def _round_f32(x):
    """x (a non-negative Fraction) rounded to the nearest FP32 value, ties to even:
    the rounding of one FP32 operation, written out in exact rational arithmetic."""
    from fractions import Fraction
    if x == 0:
        return Fraction(0)
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1                                       # 2^e <= x < 2^(e+1)
    ulp = Fraction(2) ** (e - 23)
    m = x / ulp
    f = m.numerator // m.denominator
    r = m - f
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and f % 2 == 1):
        f += 1
    return f * ulp


def test_channel_codes_at_every_rounding_boundary():
    """Around each boundary (k - 1/2)/255 of the 8-bit code, 64 FP32 values on
    either side: the oracle's code equals floor(round32(round32(255 c) + 1/2)),
    each FP32 operation written out as an exact rational rounding, and it equals
    the exact floor(255 c + 1/2) except for values whose exact 255 c + 1/2 lies
    within 2^-15 of the integer k (there the FP32 sum rounds onto k)."""
    import math
    from fractions import Fraction
    flips = 0
    for k in range(1, 256):
        b = np.float32((k - 0.5) / 255.0)
        vals = [b]
        lo = hi = b
        for _ in range(64):
            lo = np.nextafter(lo, np.float32(0.0))
            hi = np.nextafter(hi, np.float32(1.0))
            vals += [lo, hi]
        vals = np.array(vals, dtype=np.float32)
        got = E.channel_codes(vals)
        for c, q in zip(vals.tolist(), got.tolist()):
            cf = Fraction(c)
            fp32 = math.floor(_round_f32(_round_f32(255 * cf) + Fraction(1, 2)))
            assert q == fp32, (k, c, q, fp32)
            exact = math.floor(255 * cf + Fraction(1, 2))
            if q != exact:
                flips += 1
                assert abs(255 * cf + Fraction(1, 2) - k) < Fraction(1, 2 ** 15), (k, c)
        assert got.min() == k - 1 and got.max() == k          # both codes occur around it
    assert flips < 255 * 8                                     # a few values per boundary at most
